// Low-precision spectral decomposition of the preconditioner (Sec. 2.1): a parallel
// cyclic two-sided Jacobi in FP32 followed (in the host driver) by FP64 Newton-Schulz
// re-orthogonalisation of the eigenvector matrix.
//
// Ordering: round-robin (circle method).  The matrix is kept in "pair order": in every
// round the pairs are the storage positions (2a, 2a+1), a = 0..m-1, m = n2/2 (n2 = n
// rounded up to even; an odd n gets one zero dummy index whose rotations are the
// identity).  One kernel per round applies all m disjoint rotations,
// A <- J^T A J and V <- V J, and writes the result permuted for the next round: position
// 0 stays, the top positions (even) move one pair to the right, the bottom positions (odd)
// one pair to the left, with the circle closing at both ends.  After n2 - 1 rounds every
// pair of indices has met once (one sweep).  Every 2x2 block is read and written as two
// float2 values, so all traffic is coalesced.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace je {

// New storage position of the index at position x after one round (m pairs).
__device__ __host__ __forceinline__ int rr_next(int x, int m) {
  if (m == 1) return x;
  if (x == 0) return 0;
  if (x & 1) {
    int a = (x - 1) >> 1;
    return a == 0 ? 2 : x - 2;
  }
  int a = x >> 1;
  return a == m - 1 ? 2 * m - 1 : x + 2;
}

struct PairRot {
  float c, s, t, app, aqq, apq;
};

__device__ __forceinline__ PairRot pair_rot(const float* __restrict__ A, int ld, int a) {
  PairRot r;
  const float2 d0 = *reinterpret_cast<const float2*>(A + (size_t)(2 * a) * ld + 2 * a);
  const float2 d1 = *reinterpret_cast<const float2*>(A + (size_t)(2 * a + 1) * ld + 2 * a);
  r.app = d0.x;
  r.apq = d0.y;
  r.aqq = d1.y;
  if (r.apq == 0.0f) {
    r.c = 1.0f; r.s = 0.0f; r.t = 0.0f;
  } else {
    rot_params<float>(r.app, r.aqq, r.apq, r.t, r.c, r.s);
  }
  return r;
}

// Blocks [0, nbA) update 16 x 16 pair-blocks of A; blocks [nbA, ...) update V.
__global__ __launch_bounds__(256) void k_rr_round(const float* __restrict__ Ain,
                                                  float* __restrict__ Aout, int ld,
                                                  const float* __restrict__ Vin,
                                                  float* __restrict__ Vout, int ldv, int nrows,
                                                  int m, int nbA1, int nbA) {
  __shared__ PairRot rr[16], rc[16];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  int bid = blockIdx.x;
  if (bid < nbA) {
    const int ba = bid / nbA1, bb = bid - ba * nbA1;
    if (threadIdx.x < 16) {
      int a = ba * 16 + threadIdx.x;
      if (a < m) rr[threadIdx.x] = pair_rot(Ain, ld, a);
    } else if (threadIdx.x < 32) {
      int b = bb * 16 + threadIdx.x - 16;
      if (b < m) rc[threadIdx.x - 16] = pair_rot(Ain, ld, b);
    }
    __syncthreads();
    const int a = ba * 16 + ty, b = bb * 16 + tx;
    if (a >= m || b >= m) return;
    const PairRot& R = rr[ty];
    const PairRot& Cc = rc[tx];
    float o00, o01, o10, o11;
    if (a == b) {
      o00 = R.app + R.t * R.apq;
      o11 = R.aqq - R.t * R.apq;
      o01 = 0.0f;
      o10 = 0.0f;
    } else {
      const float2 m0 = *reinterpret_cast<const float2*>(Ain + (size_t)(2 * a) * ld + 2 * b);
      const float2 m1 = *reinterpret_cast<const float2*>(Ain + (size_t)(2 * a + 1) * ld + 2 * b);
      // rows: G_a^T M
      const float r00 = R.c * m0.x + R.s * m1.x, r01 = R.c * m0.y + R.s * m1.y;
      const float r10 = R.c * m1.x - R.s * m0.x, r11 = R.c * m1.y - R.s * m0.y;
      // columns: (G_a^T M) G_b
      o00 = Cc.c * r00 + Cc.s * r01;
      o01 = Cc.c * r01 - Cc.s * r00;
      o10 = Cc.c * r10 + Cc.s * r11;
      o11 = Cc.c * r11 - Cc.s * r10;
    }
    const int ra = rr_next(2 * a, m), rb = rr_next(2 * a + 1, m);
    const int ca = rr_next(2 * b, m), cb = rr_next(2 * b + 1, m);
    Aout[(size_t)ra * ld + ca] = o00;
    Aout[(size_t)ra * ld + cb] = o01;
    Aout[(size_t)rb * ld + ca] = o10;
    Aout[(size_t)rb * ld + cb] = o11;
    return;
  }
  // V part: block covers 16 rows x 16 column pairs
  bid -= nbA;
  const int nbc = (m + 15) / 16;
  const int bi = bid / nbc, bb = bid - bi * nbc;
  if (threadIdx.x < 16) {
    int b = bb * 16 + threadIdx.x;
    if (b < m) rc[threadIdx.x] = pair_rot(Ain, ld, b);
  }
  __syncthreads();
  const int i = bi * 16 + ty, b = bb * 16 + tx;
  if (i >= nrows || b >= m) return;
  const PairRot& Cc = rc[tx];
  const float2 v = *reinterpret_cast<const float2*>(Vin + (size_t)i * ldv + 2 * b);
  Vout[(size_t)i * ldv + rr_next(2 * b, m)] = Cc.c * v.x + Cc.s * v.y;
  Vout[(size_t)i * ldv + rr_next(2 * b + 1, m)] = Cc.c * v.y - Cc.s * v.x;
}

// A32 (n2 x n2, zero padded) <- fl32(A)
__global__ void k_to_f32_pad(const double* __restrict__ A, int n, int lda, float* __restrict__ B,
                             int n2) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n2 * n2) return;
  int i = (int)(idx / n2), j = (int)(idx - (size_t)i * n2);
  B[idx] = (i < n && j < n) ? (float)A[(size_t)i * lda + j] : 0.0f;
}

__global__ void k_identity_f32(float* V, int nrows, int ldv) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrows * ldv) return;
  int i = (int)(idx / ldv), j = (int)(idx - (size_t)i * ldv);
  V[idx] = (i == j) ? 1.0f : 0.0f;
}

// off(A)^2 and ||A||_F^2 of an n2 x n2 FP32 matrix (double accumulation, fixed order).
__global__ __launch_bounds__(256) void k_off_norm_f32(const float* __restrict__ A, int n2,
                                                      double* __restrict__ partial) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n2) return;
  double so = 0.0, sd = 0.0;
  for (int l = lane; l < n2; l += 64) {
    double v = A[(size_t)row * n2 + l];
    if (l == row) sd += v * v;
    else so += v * v;
  }
  so = wave_sum_d(so);
  sd = wave_sum_d(sd);
  if (lane == 0) { partial[2 * row] = so; partial[2 * row + 1] = sd; }
}

__global__ __launch_bounds__(256) void k_off_norm_sum(const double* __restrict__ partial, int n2,
                                                      double* out) {
  __shared__ double w[2][4];
  double so = 0.0, sd = 0.0;
  for (int k = threadIdx.x; k < n2; k += 256) { so += partial[2 * k]; sd += partial[2 * k + 1]; }
  so = wave_sum_d(so);
  sd = wave_sum_d(sd);
  if ((threadIdx.x & 63) == 0) { w[0][threadIdx.x >> 6] = so; w[1][threadIdx.x >> 6] = sd; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = ((w[0][0] + w[0][1]) + w[0][2]) + w[0][3];
    double d = ((w[1][0] + w[1][1]) + w[1][2]) + w[1][3];
    out[0] = sqrt(o);
    out[1] = sqrt(o + d);
  }
}

// Q (n x n, FP64, row-major) <- columns of V32 at positions colmap[0..n)
__global__ void k_gather_q(const float* __restrict__ V, int n, int ldv, const int* __restrict__ colmap,
                           double* __restrict__ Q, int ldq) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
  Q[(size_t)i * ldq + j] = (double)V[(size_t)i * ldv + colmap[j]];
}

size_t precond_f32_bytes(int n) {
  size_t n2 = (size_t)(n + (n & 1));
  size_t b = 2 * n2 * n2 * 4 + 2 * (size_t)n * n2 * 4;  // A32 x2, V32 x2
  b += 2 * n2 * 8 + 64;                                  // partial sums + result
  b += (size_t)n * 4 + 256;                              // column map
  return (b + 255) & ~(size_t)255;
}

hipError_t run_precond_f32(const double* Asym, int n, int ld, double* Q, int ldq, void* scratch,
                           int max_sweeps, int* sweeps, hipStream_t s) {
  const int n2 = n + (n & 1), m = n2 / 2;
  char* p = (char*)scratch;
  float* A0 = (float*)p; p += (size_t)n2 * n2 * 4;
  float* A1 = (float*)p; p += (size_t)n2 * n2 * 4;
  float* V0 = (float*)p; p += (size_t)n * n2 * 4;
  float* V1 = (float*)p; p += (size_t)n * n2 * 4;
  double* part = (double*)p; p += 2 * (size_t)n2 * 8;
  double* res = (double*)p; p += 64;
  int* colmap = (int*)p;
  hipError_t e;
  {
    size_t tot = (size_t)n2 * n2;
    hipLaunchKernelGGL(k_to_f32_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Asym,
                       n, ld, A0, n2);
    size_t totv = (size_t)n * n2;
    hipLaunchKernelGGL(k_identity_f32, dim3((unsigned)((totv + 255) / 256)), dim3(256), 0, s, V0,
                       n, n2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // position -> index bookkeeping on the host (to find the dummy column for odd n)
  int* pos_idx = new int[n2];
  int* tmp = new int[n2];
  for (int x = 0; x < n2; ++x) pos_idx[x] = x;
  const int nb1 = (m + 15) / 16;
  const int nbA = nb1 * nb1;
  const int nbV = ((n + 15) / 16) * nb1;
  double h[2];
  hipLaunchKernelGGL(k_off_norm_f32, dim3((n2 + 3) / 4), dim3(256), 0, s, A0, n2, part);
  hipLaunchKernelGGL(k_off_norm_sum, dim3(1), dim3(256), 0, s, part, n2, res);
  if ((e = hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, s)) != hipSuccess) goto out;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) goto out;
  {
    double off = h[0], nrm = h[1];
    const double tol = 0x1p-22;
    int sw = 0;
    while (sw < max_sweeps && off > tol * nrm) {
      for (int r = 0; r < n2 - 1; ++r) {
        hipLaunchKernelGGL(k_rr_round, dim3(nbA + nbV), dim3(256), 0, s, A0, A1, n2, V0, V1, n2, n,
                           m, nb1, nbA);
        float* t = A0; A0 = A1; A1 = t;
        t = V0; V0 = V1; V1 = t;
        for (int x = 0; x < n2; ++x) tmp[rr_next(x, m)] = pos_idx[x];
        for (int x = 0; x < n2; ++x) pos_idx[x] = tmp[x];
      }
      if ((e = hipGetLastError()) != hipSuccess) goto out;
      ++sw;
      hipLaunchKernelGGL(k_off_norm_f32, dim3((n2 + 3) / 4), dim3(256), 0, s, A0, n2, part);
      hipLaunchKernelGGL(k_off_norm_sum, dim3(1), dim3(256), 0, s, part, n2, res);
      if ((e = hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, s)) != hipSuccess) goto out;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) goto out;
      double prev = off;
      off = h[0];
      nrm = h[1];
      if (off >= prev) break;
    }
    *sweeps = sw;
  }
  {
    int* cm = new int[n];
    int j = 0;
    for (int x = 0; x < n2; ++x)
      if (pos_idx[x] < n) cm[j++] = x;
    e = hipMemcpyAsync(colmap, cm, (size_t)n * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    delete[] cm;
    if (e != hipSuccess) goto out;
    size_t tot = (size_t)n * n;
    hipLaunchKernelGGL(k_gather_q, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V0, n, n2,
                       colmap, Q, ldq);
    e = hipGetLastError();
  }
out:
  delete[] pos_idx;
  delete[] tmp;
  return e;
}

}  // namespace je
