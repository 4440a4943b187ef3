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
                                           int ldc) {
  __shared__ double sA[GK][GB + 2];  // sA[k][i] = op(A)[i0 + i][k0 + k]
  __shared__ double sB[GK][GB + 2];  // sB[k][j] = B[k0 + k][j0 + j]
  constexpr int PER = GB * GK / 256;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = blockIdx.y * GB, j0 = blockIdx.x * GB;
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
  dgemm_tile<TRANSA>(n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc);
}

__device__ __forceinline__ double* bm_ptr(BMat& b, size_t off) {
  return *reinterpret_cast<double**>(reinterpret_cast<char*>(&b) + off);
}

// One product per matrix of a batch, operands chosen by BMat field offsets (leading
// dimension b.ld for all of them); tiles past the matrix's n exit.
template <int TRANSA>
__global__ __launch_bounds__(256) void k_dgemm_b(BMat* __restrict__ mats, double alpha,
                                                 size_t offA, size_t offB, double beta,
                                                 size_t offCin, size_t offC) {
  BMat& b = mats[blockIdx.z];
  const int n = b.n;
  if ((int)blockIdx.y * GB >= n || (int)blockIdx.x * GB >= n) return;
  dgemm_tile<TRANSA>(n, alpha, bm_ptr(b, offA), b.ld, bm_ptr(b, offB), b.ld, beta,
                     beta != 0.0 ? bm_ptr(b, offCin) : nullptr, b.ld, bm_ptr(b, offC), b.ld);
}

hipError_t launch_dgemm_b(BMat* m, int count, int nmax, int transA, double alpha, size_t offA,
                          size_t offB, double beta, size_t offCin, size_t offC, hipStream_t s) {
  int nb = (nmax + GB - 1) / GB;
  dim3 g(nb, nb, count), bl(256);
  if (transA)
    hipLaunchKernelGGL(k_dgemm_b<1>, g, bl, 0, s, m, alpha, offA, offB, beta, offCin, offC);
  else
    hipLaunchKernelGGL(k_dgemm_b<0>, g, bl, 0, s, m, alpha, offA, offB, beta, offCin, offC);
  return hipGetLastError();
}

__global__ void k_add_identity_b(BMat* __restrict__ mats, size_t off, double scale) {
  BMat& b = mats[blockIdx.y];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < b.n) bm_ptr(b, off)[(size_t)i * b.ld + i] += scale;
}

hipError_t launch_add_identity_b(BMat* m, int count, int nmax, size_t off, double scale,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_add_identity_b, dim3((nmax + 255) / 256, count), dim3(256), 0, s, m, off,
                     scale);
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
