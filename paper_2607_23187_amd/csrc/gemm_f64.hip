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
// Products up to n = kNarrowMaxN use 64 x 32 tiles: twice the workgroups of the 64 x 64
// tiling (at n = 1024, 512 instead of 256: two per CU), so that the K-loop latency of one
// workgroup is hidden by the other's matrix-core work.
constexpr int kNarrowMaxN = 1024;

// One 64 x BN tile of C (BN = 64, or 32 for the narrow tiles of small products).  K
// advances in steps of GK; the operands of the next step are loaded into registers while
// the matrix cores work on the current one (with few workgroups per CU nothing else would
// hide the global-load latency).  Four waves split the tile 2 x 2 (32 x BN/2 each).
// KS = 2 (narrow tiles): eight waves, the second four taking the second half of every K
// step into accumulators of their own, added to the first four's at the end (first half +
// second half, a fixed order): twice the waves per CU to hide the matrix-core latency.
// SYM: the product is symmetric (X^T X, or Q^T (A Q) for symmetric A); only tiles on or
// above the diagonal are computed, and each entry C[i][j], i <= j, is also stored at
// C[j][i], so the result is exactly symmetric (beta must be 0).
template <int TRANSA, bool SYM = false, int BN = GB, int KS = 1>
__device__ __forceinline__ void dgemm_tile(int n, double alpha, const double* __restrict__ A,
                                           int lda, const double* __restrict__ B, int ldb,
                                           double beta, const double* Cin, int ldcin, double* C,
                                           int ldc, int tile_i, int tile_j) {
  static_assert(BN == 64 || BN == 32, "64 x 64 or 64 x 32 tiles");
  static_assert(KS == 1 || (KS == 2 && BN == 32), "K split only for the narrow tiles");
  constexpr int NB = BN / 32;             // 16-column MFMA tiles per wave
  constexpr int NT = 256 * KS;
  __shared__ double sA[GK][GB + 2];  // sA[k][i] = op(A)[i0 + i][k0 + k]
  __shared__ double sB[GK][BN + 2];  // sB[k][j] = B[k0 + k][j0 + j]
  constexpr int PER = GB * GK / NT, PERB = BN * GK / NT;
  const int tid = threadIdx.x, lane = tid & 63, w = (tid >> 6) & 3, kh = tid >> 8;
  const int i0 = tile_i * GB, j0 = tile_j * BN;
  const int wi = (w >> 1) * 32, wj = (w & 1) * (BN / 2);
  const int lr = lane & 15, lk = lane >> 4;
  d4 acc[2][NB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  double ra[PER], rb[PERB];
  // element e of a K step: A part (i, k) with the contiguous index fastest, B part (k, j)
  auto a_idx = [&](int e, int& i, int& k) {
    if (TRANSA) { i = e % GB; k = e / GB; }   // A[k][i]: contiguous in i
    else { k = e % GK; i = e / GK; }          // A[i][k]: contiguous in k
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      int i, k;
      a_idx(e, i, k);
      const int gi = i0 + i, gk = k0 + k;
      ra[t] = (gi < n && gk < n) ? (TRANSA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk])
                                 : 0.0;
    }
#pragma unroll
    for (int t = 0; t < PERB; ++t) {
      const int e = tid + t * NT;
      const int j = e % BN, kb = e / BN;
      const int gkb = k0 + kb, gj = j0 + j;
      rb[t] = (gkb < n && gj < n) ? B[(size_t)gkb * ldb + gj] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += GK) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      int i, k;
      a_idx(e, i, k);
      sA[k][i] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < PERB; ++t) {
      const int e = tid + t * NT;
      sB[e / BN][e % BN] = rb[t];
    }
    __syncthreads();
    if (k0 + GK < n) fetch(k0 + GK);
#pragma unroll
    for (int kk = kh * (GK / KS); kk < (kh + 1) * (GK / KS); kk += 4) {
      double av[2], bv[NB];
#pragma unroll
      for (int t = 0; t < 2; ++t) av[t] = sA[kk + lk][wi + t * 16 + lr];
#pragma unroll
      for (int t = 0; t < NB; ++t) bv[t] = sB[kk + lk][wj + t * 16 + lr];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  if constexpr (KS == 2) {
    // the second half's accumulators through LDS (sA is free after the last step)
    double* part = &sA[0][0];
    if (kh == 1) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[((w * 2 + a) * 4 + r) * 64 + lane] = acc[a][0][r];
    }
    __syncthreads();
    if (kh == 1) return;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][0][r] += part[((w * 2 + a) * 4 + r) * 64 + lane];
  }
  // D[i][j] of a 16 x 16 tile sits in lane j + 16 * (i % 4), register i / 4
  // (A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k).
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int i = i0 + wi + a * 16 + 4 * r + lk;
        int j = j0 + wj + b * 16 + lr;
        if (SYM) {
          if (i <= j && j < n) {
            const double v = alpha * acc[a][b][r];
            C[(size_t)i * ldc + j] = v;
            if (i < j) C[(size_t)j * ldc + i] = v;
          }
        } else if (i < n && j < n) {
          double v = alpha * acc[a][b][r];
          if (beta != 0.0) v += beta * Cin[(size_t)i * ldcin + j];
          C[(size_t)i * ldc + j] = v;
        }
      }
}

// K split (eight waves) for the narrow tiles
template <int BN>
constexpr int ks_of() { return BN == 32 ? 2 : 1; }

template <int TRANSA, int BN = GB>
__global__ __launch_bounds__(256 * ks_of<BN>()) void k_dgemm(
    int n, double alpha, const double* __restrict__ A, int lda, const double* __restrict__ B,
    int ldb, double beta, const double* Cin, int ldcin, double* C, int ldc) {
  dgemm_tile<TRANSA, false, BN, ks_of<BN>()>(n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C,
                                             ldc, blockIdx.y, blockIdx.x);
}

// Tile t of the tiles holding entries on or above the diagonal, row by row, for row tiles
// of 64 and column tiles of 64 / r (r = 1 or 2): (by, bx) with bx >= r by, bx < nbc.
__device__ __forceinline__ void upper_tile(int t, int nbc, int r, int& by, int& bx) {
  by = 0;
  while (t >= nbc - r * by) { t -= nbc - r * by; ++by; }
  bx = r * by + t;
}

// Tiles of upper_tile for n: row tiles of 64, column tiles of BN.
static int upper_tiles(int n, int BN) {
  const int nbr = (n + GB - 1) / GB, nbc = (n + BN - 1) / BN, r = GB / BN;
  int t = 0;
  for (int by = 0; by < nbr; ++by) t += nbc - r * by;
  return t;
}

// C = alpha A^T B, symmetric: one workgroup per tile holding entries on or above the
// diagonal.
template <int BN>
__global__ __launch_bounds__(256 * ks_of<BN>()) void k_dgemm_sym(
    int n, int nbc, double alpha, const double* __restrict__ A, int lda,
    const double* __restrict__ B, int ldb, double* C, int ldc) {
  int by, bx;
  upper_tile(blockIdx.x, nbc, GB / BN, by, bx);
  dgemm_tile<1, true, BN, ks_of<BN>()>(n, alpha, A, lda, B, ldb, 0.0, nullptr, 0, C, ldc, by,
                                       bx);
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

template <int TRANSA, bool SYM = false>
__global__ __launch_bounds__(256) void k_dgemm_b(BMat* __restrict__ mats, int count, int nb,
                                                 double alpha, size_t offA, size_t offB,
                                                 double beta, size_t offCin, size_t offC,
                                                 int ns_mask) {
  const int T = SYM ? nb * (nb + 1) / 2 : nb * nb;
  const int L = blockIdx.x, xcd = L % kXcds, slot = L / kXcds;
  const int z = xcd + kXcds * (slot / T), t = slot % T;
  if (z >= count) return;
  BMat& b = mats[z];
  const int n = b.n;
  int by, bx;
  if (SYM) upper_tile(t, nb, 1, by, bx);
  else { by = t / nb; bx = t % nb; }
  if (by * GB >= n || bx * GB >= n) return;
  if (ns_mask && b.ns_done) {  // converged member: C = 0 (its update then leaves X as is)
    double* C = bm_ptr(b, offC);
    for (int e = threadIdx.x; e < GB * GB; e += 256) {
      const int i = by * GB + e / GB, j = bx * GB + e % GB;
      if (i < n && j < n) {
        C[(size_t)i * b.ld + j] = 0.0;
        if (SYM) C[(size_t)j * b.ld + i] = 0.0;  // and the mirrored tile
      }
    }
    return;
  }
  dgemm_tile<TRANSA, SYM>(n, alpha, bm_ptr(b, offA), b.ld, bm_ptr(b, offB), b.ld, beta,
                          beta != 0.0 ? bm_ptr(b, offCin) : nullptr, b.ld, bm_ptr(b, offC),
                          b.ld, by, bx);
}

hipError_t launch_dgemm_sym_b(BMat* m, int count, int nmax, double alpha, size_t offA,
                              size_t offB, size_t offC, hipStream_t s, int ns_mask) {
  const int nb = (nmax + GB - 1) / GB;
  const long long blocks = (long long)kXcds * ((count + kXcds - 1) / kXcds) * (nb * (nb + 1) / 2);
  hipLaunchKernelGGL((k_dgemm_b<1, true>), dim3((unsigned)blocks), dim3(256), 0, s, m, count, nb,
                     alpha, offA, offB, 0.0, (size_t)0, offC, ns_mask);
  return hipGetLastError();
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

hipError_t launch_dgemm_sym(int n, double alpha, const double* A, int lda, const double* B,
                            int ldb, double* C, int ldc, hipStream_t s) {
  if (n <= kNarrowMaxN) {
    hipLaunchKernelGGL(k_dgemm_sym<32>, dim3(upper_tiles(n, 32)), dim3(256 * ks_of<32>()), 0, s, n,
                       (n + 31) / 32, alpha, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_dgemm_sym<GB>, dim3(upper_tiles(n, GB)), dim3(256), 0, s, n,
                     (n + GB - 1) / GB, alpha, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}


hipError_t launch_dgemm(int n, int transA, double alpha, const double* A, int lda, const double* B,
                        int ldb, double beta, const double* Cin, int ldcin, double* C, int ldc,
                        hipStream_t s) {
  const int nb = (n + GB - 1) / GB;
  if (n <= kNarrowMaxN) {
    const dim3 g((n + 31) / 32, nb), b(256 * ks_of<32>());
    if (transA)
      hipLaunchKernelGGL((k_dgemm<1, 32>), g, b, 0, s, n, alpha, A, lda, B, ldb, beta, Cin, ldcin,
                         C, ldc);
    else
      hipLaunchKernelGGL((k_dgemm<0, 32>), g, b, 0, s, n, alpha, A, lda, B, ldb, beta, Cin, ldcin,
                         C, ldc);
    return hipGetLastError();
  }
  dim3 g(nb, nb), b(256);
  if (transA)
    hipLaunchKernelGGL(k_dgemm<1>, g, b, 0, s, n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc);
  else
    hipLaunchKernelGGL(k_dgemm<0>, g, b, 0, s, n, alpha, A, lda, B, ldb, beta, Cin, ldcin, C, ldc);
  return hipGetLastError();
}

// ------------------------------------------------------------------ split-precision product
// C = op(A) * B on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16) with FP64 accuracy, by
// error-free slicing:
//   * every row i of op(A) is scaled by 2^-ea_i and every column j of B by 2^-eb_j (exact),
//     the powers of two that bring the row's / column's largest entry below 1;
//   * a scaled entry x (|x| < 1) is cut into kSlices integer slices of 8 bits,
//     x = sum_s 2^(-8 (s + 1)) alpha_s, alpha_s = rint(256 r_s), r_(s+1) = 256 r_s - alpha_s
//     (|alpha_0| <= 256, |alpha_s| <= 128 after it): every slice is an integer that BF16
//     holds exactly, and the cut is exact in FP64 (the residual after 7 slices is below
//     2^-57 of the row's or column's largest entry);
//   * products of slices are integers below 2^16, exact in FP32.  For every K block of
//     kSplitKb = 32 terms, the slice products of one level d = s + t (all of them scaled
//     by 2^(-8 (d + 2))) are accumulated in FP32: every partial sum is an integer below
//     2^24 (at most 7 pairs x 32 terms x 2^16), so the FP32 accumulation is exact whatever
//     the order inside the matrix core;
//   * each level's exact block sum is added into an FP64 accumulator with its weight
//     2^(-8 (d + 2)), levels d = 0 .. kSlices - 1 (slice pairs with s + t >= kSlices are
//     below 2^-64 of |op(A)| |B| and dropped), and the row and column scales are applied
//     at the end.
// The FP64 accumulation over n / 32 blocks rounds like an FP64 product does; everything
// before it is exact, so the result carries FP64-level error (the accuracy the FP64 phase
// needs from Q^T A Q, Sec. 2.1), from 28 BF16 slice products per block.
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kSlices = 7;     // 8-bit slices per operand entry
constexpr int kSplitKb = 32;   // K block accumulated exactly in FP32
constexpr int SPL = kSplitKb + 4;  // LDS row of one slice tile (bf16), 8-byte aligned

// bf16 bits of an integer |v| <= 256 (exact)
__device__ __forceinline__ unsigned short bf16_int(double v) {
  return (unsigned short)(__float_as_uint((float)v) >> 16);
}

// Exponent e with max |x| < 2^e over the row (trans = 0: row r of M, contiguous) or the
// column (trans = 1: column r of M); 0 for a zero row.  One wave per row / column.
__global__ __launch_bounds__(256) void k_split_exp(const double* __restrict__ M, int n, int ld,
                                                   int trans, int* __restrict__ ex) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  double m = 0.0;
  for (int k = lane; k < n; k += 64)
    m = fmax(m, fabs(trans ? M[(size_t)k * ld + r] : M[(size_t)r * ld + k]));
  m = wave_max_d(m);
  if (lane == 0) {
    int e = 0;
    if (m > 0.0) {
      (void)frexp(m, &e);  // m = f 2^e, f in [1/2, 1): m < 2^e
    }
    ex[r] = e;
  }
}

// Slice planes P[s][r][k] (r < np rows of op(M) or columns of M, k < kp, zero padded) of
// the scaled entries: trans = 0: entry M[r][k]; trans = 1: entry M[k][r].  32 x 32 tiles
// through LDS so that both the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void k_split_slices(const double* __restrict__ M, int n, int ld,
                                                      int trans, const int* __restrict__ ex,
                                                      unsigned short* __restrict__ P, int np,
                                                      int kp) {
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int r0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  // t[rr][kk] = entry (r0 + rr, k0 + kk) of op(M)
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + (trans ? tx : i), k = k0 + (trans ? i : tx);
    double v = 0.0;
    if (r < n && k < n) v = trans ? M[(size_t)k * ld + r] : M[(size_t)r * ld + k];
    if (trans) t[tx][i] = v;
    else t[i][tx] = v;
  }
  __syncthreads();
  const size_t plane = (size_t)np * kp;
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, k = k0 + tx;
    if (r >= np || k >= kp) continue;
    double x = (r < n) ? ldexp(t[i][tx], -ex[r]) : 0.0;
#pragma unroll
    for (int sl = 0; sl < kSlices; ++sl) {
      const double y = x * 256.0;
      const double a = rint(y);
      x = y - a;
      P[sl * plane + (size_t)r * kp + k] = bf16_int(a);
    }
  }
}

// One 64 x 64 tile of C from the slice planes of op(A) (PA, rows i) and B (PB, columns j).
__global__ __launch_bounds__(256) void k_gemm_split(int n, const unsigned short* __restrict__ PA,
                                                    const unsigned short* __restrict__ PB,
                                                    int kp, const int* __restrict__ ea,
                                                    const int* __restrict__ eb,
                                                    double* __restrict__ C, int ldc, int np) {
  __shared__ __align__(16) unsigned short sA[kSlices][GB][SPL];
  __shared__ __align__(16) unsigned short sB[kSlices][GB][SPL];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = blockIdx.y * GB, j0 = blockIdx.x * GB;
  const int wi = (w >> 1) * 32, wj = (w & 1) * 32;
  const int lr = lane & 15, lq = lane >> 4;
  const size_t plane = (size_t)np * kp;
  double acc64[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][b][r] = 0.0;
  for (int k0 = 0; k0 < kp; k0 += kSplitKb) {
    // 7 slices x 64 rows x 32 k of each operand: 8-byte pieces (4 bf16), 7 per thread each
    for (int e = tid; e < kSlices * GB * (kSplitKb / 4); e += 256) {
      const int sl = e / (GB * (kSplitKb / 4));
      const int rem = e - sl * (GB * (kSplitKb / 4));
      const int r = rem / (kSplitKb / 4), c4 = (rem % (kSplitKb / 4)) * 4;
      *reinterpret_cast<bf4*>(&sA[sl][r][c4]) =
          *reinterpret_cast<const bf4*>(PA + sl * plane + (size_t)(i0 + r) * kp + k0 + c4);
      *reinterpret_cast<bf4*>(&sB[sl][r][c4]) =
          *reinterpret_cast<const bf4*>(PB + sl * plane + (size_t)(j0 + r) * kp + k0 + c4);
    }
    __syncthreads();
    // level d: all slice pairs s + t = d, exact FP32 sums over the block
#pragma unroll
    for (int d = kSlices - 1; d >= 0; --d) {
      f4 acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int sa = 0; sa <= d; ++sa) {
        const int sb = d - sa;
#pragma unroll
        for (int kk = 0; kk < kSplitKb; kk += 16) {
          bf4 af[2], bfr[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            af[t] = *reinterpret_cast<const bf4*>(&sA[sa][wi + t * 16 + lr][kk + 4 * lq]);
            bfr[t] = *reinterpret_cast<const bf4*>(&sB[sb][wj + t * 16 + lr][kk + 4 * lq]);
          }
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], acc[a][b], 0,
                                                                     0, 0);
        }
      }
      const double wd = ldexp(1.0, -8 * (d + 2));
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[a][b][r] += wd * (double)acc[a][b][r];
    }
    __syncthreads();
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
        if (i < n && j < n) C[(size_t)i * ldc + j] = ldexp(acc64[a][b][r], ea[i] + eb[j]);
      }
}

static int split_np(int n) { return (n + GB - 1) / GB * GB; }

size_t gemm_split_bytes(int n) {
  const size_t np = split_np(n);
  return 2 * (size_t)kSlices * np * np * 2 + 2 * ((np * 4 + 255) & ~(size_t)255);
}

hipError_t launch_gemm_split(int n, int transA, const double* A, int lda, const double* B,
                             int ldb, double* C, int ldc, void* work, hipStream_t s) {
  const int np = split_np(n), kp = np;  // GB is a multiple of the K block
  const size_t plane = (size_t)np * kp;
  unsigned short* PA = (unsigned short*)work;
  unsigned short* PB = PA + kSlices * plane;
  int* ea = (int*)(PB + kSlices * plane);
  int* eb = ea + ((np * 4 + 255) & ~255) / 4;
  const int nt = (np + 31) / 32;
  // op(A): rows of A, or columns of A when transposed; B: its columns
  hipLaunchKernelGGL(k_split_exp, dim3((n + 3) / 4), dim3(256), 0, s, A, n, lda, transA, ea);
  hipLaunchKernelGGL(k_split_exp, dim3((n + 3) / 4), dim3(256), 0, s, B, n, ldb, 1, eb);
  hipLaunchKernelGGL(k_split_slices, dim3(nt, nt), dim3(256), 0, s, A, n, lda, transA, ea, PA, np,
                     kp);
  hipLaunchKernelGGL(k_split_slices, dim3(nt, nt), dim3(256), 0, s, B, n, ldb, 1, eb, PB, np, kp);
  const int nb = np / GB;
  hipLaunchKernelGGL(k_gemm_split, dim3(nb, nb), dim3(256), 0, s, n, PA, PB, kp, ea, eb, C, ldc,
                     np);
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
