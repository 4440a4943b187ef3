// FP64 dense products on the gfx950 matrix cores (v_mfma_f64_16x16x4f64), used for the
// dense part of the preconditioner (Sec. 2.1): Newton-Schulz re-orthogonalisation of the
// FP32 eigenvector matrix, the contraction Q^T A Q, and the final polish of V.
//
// C = alpha * op(A) * B + beta * Cin for square row-major n x n operands.  A block computes
// a 64 x 64 tile of C with four waves (2 x 2 of 32 x 32), stepping K by 16 through LDS.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace je {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GB = 64;   // tile of C
constexpr int GK = 32;   // K step

// One 64 x 64 tile of C.  K advances in steps of GK; the operands of the next step are
// loaded into registers while the matrix cores work on the current one (with a single
// workgroup per CU at n = 1024 nothing else would hide the global-load latency).
template <int TRANSA>
__device__ __forceinline__ void dgemm_tile(int n, double alpha, const double* __restrict__ A,
                                           int lda, const double* __restrict__ B, int ldb,
                                           double beta, const double* Cin, int ldcin, double* C,
                                           int ldc, int tile_i, int tile_j) {
  __shared__ double sA[GK][GB + 2];  // sA[k][i] = op(A)[i0 + i][k0 + k]
  __shared__ double sB[GK][GB + 2];  // sB[k][j] = B[k0 + k][j0 + j]
  constexpr int PER = GB * GK / 256;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = tile_i * GB, j0 = tile_j * GB;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  double ra[PER], rb[PER];
  // element e of a K step: A part (i, k) with the contiguous index fastest, B part (k, j)
  auto a_idx = [&](int e, int& i, int& k) {
    if (TRANSA) { i = e % GB; k = e / GB; }   // A[k][i]: contiguous in i
    else { k = e % GK; i = e / GK; }          // A[i][k]: contiguous in k
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * 256;
      int i, k;
      a_idx(e, i, k);
      const int gi = i0 + i, gk = k0 + k;
      ra[t] = (gi < n && gk < n) ? (TRANSA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk])
                                 : 0.0;
      const int j = e % GB, kb = e / GB;
      const int gkb = k0 + kb, gj = j0 + j;
      rb[t] = (gkb < n && gj < n) ? B[(size_t)gkb * ldb + gj] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += GK) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * 256;
      int i, k;
      a_idx(e, i, k);
      sA[k][i] = ra[t];
      sB[e / GB][e % GB] = rb[t];
    }
    __syncthreads();
    if (k0 + GK < n) fetch(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = sA[kk + lk][wi + t * 16 + lr];
        bv[t] = sB[kk + lk][wj + t * 16 + lr];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 16 x 16 tile sits in lane j + 16 * (i % 4), register i / 4
  // (A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k).
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + wi + a * 16 + 4 * r + lk;
        int j = j0 + wj + b * 16 + lr;
        if (i < n && j < n) {
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * Cin[(size_t)i * ldcin + j];
          C[(size_t)i * ldc + j] = v;
        }
      }
}

template <int TRANSA>
__global__ __launch_bounds__(256) void k_dgemm(int n, double alpha, const double* __restrict__ A,
                                               int lda, const double* __restrict__ B, int ldb,
                                               double beta, const double* Cin, int ldcin,
                                               double* C, int ldc) {
  dgemm_tile<TRANSA>(n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc, blockIdx.y, blockIdx.x);
}

__device__ __forceinline__ double* bm_ptr(BMat& b, size_t off) {
  return *reinterpret_cast<double**>(reinterpret_cast<char*>(&b) + off);
}

// One product per matrix of a batch, operands chosen by BMat field offsets (leading
// dimension b.ld for all of them); tiles past the matrix's n exit.  Workgroups are handed
// to the 8 XCDs round-robin by linear index, so the 1-D grid is ordered to put every tile
// of matrix z on XCD z mod 8: the tiles of a product then share the operand panels in one
// L2 instead of fetching them into several.
constexpr int kXcds = 8;

template <int TRANSA>
__global__ __launch_bounds__(256) void k_dgemm_b(BMat* __restrict__ mats, int count, int nb,
                                                 double alpha, size_t offA, size_t offB,
                                                 double beta, size_t offCin, size_t offC,
                                                 int ns_mask) {
  const int L = blockIdx.x, xcd = L % kXcds, slot = L / kXcds, T = nb * nb;
  const int z = xcd + kXcds * (slot / T), t = slot % T;
  if (z >= count) return;
  BMat& b = mats[z];
  const int n = b.n;
  const int by = t / nb, bx = t % nb;
  if (by * GB >= n || bx * GB >= n) return;
  if (ns_mask && b.ns_done) {  // converged member: C = 0 (its update then leaves X as is)
    double* C = bm_ptr(b, offC);
    for (int e = threadIdx.x; e < GB * GB; e += 256) {
      const int i = by * GB + e / GB, j = bx * GB + e % GB;
      if (i < n && j < n) C[(size_t)i * b.ld + j] = 0.0;
    }
    return;
  }
  dgemm_tile<TRANSA>(n, alpha, bm_ptr(b, offA), b.ld, bm_ptr(b, offB), b.ld, beta,
                     beta != 0.0 ? bm_ptr(b, offCin) : nullptr, b.ld, bm_ptr(b, offC), b.ld,
                     by, bx);
}

hipError_t launch_dgemm_b(BMat* m, int count, int nmax, int transA, double alpha, size_t offA,
                          size_t offB, double beta, size_t offCin, size_t offC, hipStream_t s,
                          int ns_mask) {
  const int nb = (nmax + GB - 1) / GB;
  const long long blocks = (long long)kXcds * ((count + kXcds - 1) / kXcds) * nb * nb;
  dim3 g((unsigned)blocks), bl(256);
  if (transA)
    hipLaunchKernelGGL(k_dgemm_b<1>, g, bl, 0, s, m, count, nb, alpha, offA, offB, beta, offCin,
                       offC, ns_mask);
  else
    hipLaunchKernelGGL(k_dgemm_b<0>, g, bl, 0, s, m, count, nb, alpha, offA, offB, beta, offCin,
                       offC, ns_mask);
  return hipGetLastError();
}

__global__ void k_add_identity_b(BMat* __restrict__ mats, size_t off, double scale,
                                 int ns_mask) {
  BMat& b = mats[blockIdx.y];
  if (ns_mask && b.ns_done) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < b.n) bm_ptr(b, off)[(size_t)i * b.ld + i] += scale;
}

hipError_t launch_add_identity_b(BMat* m, int count, int nmax, size_t off, double scale,
                                 hipStream_t s, int ns_mask) {
  hipLaunchKernelGGL(k_add_identity_b, dim3((nmax + 255) / 256, count), dim3(256), 0, s, m, off,
                     scale, ns_mask);
  return hipGetLastError();
}

__global__ void k_ns_reset_b(BMat* __restrict__ mats, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) mats[i].ns_done = 0;
}

// Convergence rule of a Newton-Schulz step that started from residual r (the same rule as
// a single problem's): r <= 4 n u, or r^2 <= n u / 2 (the step left about (3/4) r^2).
__global__ void k_ns_flag_b(BMat* __restrict__ mats, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  BMat& b = mats[i];
  const double r = b.scal[1], nu = b.n * 0x1p-53;
  if (r <= 4.0 * nu || r * r <= 0.5 * nu) b.ns_done = 1;
}

hipError_t launch_ns_reset_b(BMat* m, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_reset_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count);
  return hipGetLastError();
}

hipError_t launch_ns_flag_b(BMat* m, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_flag_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count);
  return hipGetLastError();
}

hipError_t launch_dgemm(int n, int transA, double alpha, const double* A, int lda, const double* B,
                        int ldb, double beta, const double* Cin, int ldcin, double* C, int ldc,
                        hipStream_t s) {
  int nb = (n + GB - 1) / GB;
  dim3 g(nb, nb), b(256);
  if (transA)
    hipLaunchKernelGGL(k_dgemm<1>, g, b, 0, s, n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc);
  else
    hipLaunchKernelGGL(k_dgemm<0>, g, b, 0, s, n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc);
  return hipGetLastError();
}

// ------------------------------------------------------------------ split-precision product
// C = op(A) * B on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16).  Every FP64 operand
// is split into three BF16 slices, v ~ s0 + s1 + s2 (each the BF16 rounding of the FP64
// residual left by the previous ones: about 24 significant bits), and the six slice
// products s_a * s_b with a + b <= 2 are accumulated in FP32, smallest first.  FP32
// accumulators are added into FP64 every kSplitFlush K steps, so FP32 rounding
// accumulates over 128 terms rather than n (compensated accumulation).  The result carries
// FP32-level error (~2^-24 |A| |B|): the precision variant of the Q^T A Q contraction.
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int SK = 16;          // K step (one bf16 MFMA)
constexpr int kSplitFlush = 8;  // K steps per FP32 accumulation chunk

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ double bf16_value(unsigned short h) {
  return (double)__uint_as_float((unsigned)h << 16);
}

__device__ __forceinline__ void split3(double v, unsigned short& s0, unsigned short& s1,
                                       unsigned short& s2) {
  s0 = bf16_bits((float)v);
  const double r1 = v - bf16_value(s0);
  s1 = bf16_bits((float)r1);
  const double r2 = r1 - bf16_value(s1);
  s2 = bf16_bits((float)r2);
}

template <int TRANSA>
__global__ __launch_bounds__(256) void k_gemm_split(int n, const double* __restrict__ A, int lda,
                                                    const double* __restrict__ B, int ldb,
                                                    double* __restrict__ C, int ldc) {
  // sA[s][i][k]: slice s of op(A)[i0 + i][k0 + k]; sB[s][j][k]: slice s of B[k0 + k][j0 + j]
  __shared__ __align__(8) unsigned short sA[3][GB][SK + 4];
  __shared__ __align__(8) unsigned short sB[3][GB][SK + 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = blockIdx.y * GB, j0 = blockIdx.x * GB;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  const int lr = lane & 15, lq = lane >> 4;
  f4 acc[2][2];
  double acc64[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
    }
  int chunk = 0;
  for (int k0 = 0; k0 < n; k0 += SK) {
#pragma unroll
    for (int t = 0; t < GB * SK / 256; ++t) {
      const int e = tid + t * 256;
      int i, k;
      if (TRANSA) { i = e % GB; k = e / GB; }   // A[k][i]: contiguous in i
      else { k = e % SK; i = e / SK; }          // A[i][k]: contiguous in k
      const int gi = i0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < n && gk < n) v = TRANSA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      split3(v, sA[0][i][k], sA[1][i][k], sA[2][i][k]);
      const int j = e % GB, kb = e / GB;
      const int gkb = k0 + kb, gj = j0 + j;
      const double u = (gkb < n && gj < n) ? B[(size_t)gkb * ldb + gj] : 0.0;
      split3(u, sB[0][j][kb], sB[1][j][kb], sB[2][j][kb]);
    }
    __syncthreads();
    bf4 af[3][2], bfr[3][2];
#pragma unroll
    for (int sl = 0; sl < 3; ++sl)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[sl][t] = *reinterpret_cast<const bf4*>(&sA[sl][wi + t * 16 + lr][4 * lq]);
        bfr[sl][t] = *reinterpret_cast<const bf4*>(&sB[sl][wj + t * 16 + lr][4 * lq]);
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        f4 c = acc[a][b];
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[2][a], bfr[0][b], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[1][a], bfr[1][b], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[0][a], bfr[2][b], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[1][a], bfr[0][b], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[0][a], bfr[1][b], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[0][a], bfr[0][b], c, 0, 0, 0);
        acc[a][b] = c;
      }
    __syncthreads();
    if (++chunk == kSplitFlush) {
      chunk = 0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[a][b][r] += (double)acc[a][b][r];
          acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
  // D[i][j] of a 16 x 16 tile sits in lane j + 16 * (i / 4), register i % 4
  // (A[i][k] in lane i + 16 (k / 4), element k % 4; B[k][j] in lane j + 16 (k / 4)).
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wi + a * 16 + 4 * lq + r;
        const int j = j0 + wj + b * 16 + lr;
        if (i < n && j < n) C[(size_t)i * ldc + j] = acc64[a][b][r] + (double)acc[a][b][r];
      }
}

hipError_t launch_gemm_split(int n, int transA, const double* A, int lda, const double* B,
                             int ldb, double* C, int ldc, hipStream_t s) {
  int nb = (n + GB - 1) / GB;
  dim3 g(nb, nb), b(256);
  if (transA) hipLaunchKernelGGL(k_gemm_split<1>, g, b, 0, s, n, A, lda, B, ldb, C, ldc);
  else hipLaunchKernelGGL(k_gemm_split<0>, g, b, 0, s, n, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

__global__ void k_add_identity(double* C, int n, int ldc, double scale) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) C[(size_t)i * ldc + i] += scale;
}

hipError_t launch_add_identity(double* C, int n, int ldc, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_add_identity, dim3((n + 255) / 256), dim3(256), 0, s, C, n, ldc, scale);
  return hipGetLastError();
}

// A <- (A + A^T) / 2, both halves from the same sum so that A is exactly symmetric.
__device__ __forceinline__ void symmetrize_tile(double* A, int n, int ld, int bi, int bj) {
  if (bi > bj) return;
  __shared__ double t1[32][33], t2[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int i0 = bi * 32, j0 = bj * 32;
  for (int r = ty; r < 32; r += 8) {
    int i = i0 + r, j = j0 + tx;
    t1[r][tx] = (i < n && j < n) ? A[(size_t)i * ld + j] : 0.0;  // t1[i][j] = A(i0+i, j0+j)
    int i2 = j0 + r, j2 = i0 + tx;
    t2[r][tx] = (i2 < n && j2 < n) ? A[(size_t)i2 * ld + j2] : 0.0;  // t2[j][i] = A(j0+j, i0+i)
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    int i = i0 + r, j = j0 + tx;
    if (i < n && j < n) A[(size_t)i * ld + j] = 0.5 * (t1[r][tx] + t2[tx][r]);
    int i2 = j0 + r, j2 = i0 + tx;
    if (i2 < n && j2 < n) A[(size_t)i2 * ld + j2] = 0.5 * (t1[tx][r] + t2[r][tx]);
  }
}

__global__ __launch_bounds__(256) void k_symmetrize(double* A, int n, int ld) {
  symmetrize_tile(A, n, ld, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_symmetrize_b(BMat* __restrict__ mats, size_t off) {
  BMat& b = mats[blockIdx.z];
  if ((int)blockIdx.y * 32 >= b.n || (int)blockIdx.x * 32 >= b.n) return;
  symmetrize_tile(bm_ptr(b, off), b.n, b.ld, blockIdx.y, blockIdx.x);
}

hipError_t launch_symmetrize_b(BMat* m, int count, int nmax, size_t off, hipStream_t s) {
  int nb = (nmax + 31) / 32;
  hipLaunchKernelGGL(k_symmetrize_b, dim3(nb, nb, count), dim3(256), 0, s, m, off);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* A, int n, int ld, hipStream_t s) {
  int nb = (n + 31) / 32;
  hipLaunchKernelGGL(k_symmetrize, dim3(nb, nb), dim3(256), 0, s, A, n, ld);
  return hipGetLastError();
}

}  // namespace je
