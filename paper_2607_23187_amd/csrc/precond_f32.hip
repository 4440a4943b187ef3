// Low-precision spectral decomposition of the preconditioner (Sec. 2.1): a blocked
// two-sided Jacobi in FP32 (the eigenvector matrix is re-orthogonalised in FP64 by the host
// driver afterwards).
//
// The matrix (padded with zero rows/columns to np = a multiple of 64) is split into
// 32-row blocks.  A sweep visits every pair of blocks once in round-robin (circle method)
// order: nb - 1 rounds of nb/2 disjoint block pairs.  For each pair (I, J) of a round one
// workgroup applies scalar FP32 Jacobi rotations (parallel round-robin inside the block)
// to the 64 x 64 subproblem [[A_II, A_IJ], [A_JI, A_JJ]] in LDS, accumulating its
// orthogonal factor U_IJ; then every other 64 x 64 block of A is replaced by
// U_P^T A_PR U_R and the columns of V by V U_R.  Each round reads and writes A and V once,
// so a sweep costs nb - 1 passes over memory instead of np - 1.  For n <= 64 the single
// block pair is the whole matrix and the subproblem solve is the whole decomposition.
#include <hip/hip_runtime.h>

#include <vector>

#include "device_common.h"
#include "kernels.h"

namespace je {

constexpr int PB = 32;          // block rows
constexpr int PM = 64;          // subproblem size (two blocks)
constexpr int PL = PM + 4;      // LDS row stride (floats), rows stay 16-byte aligned

// Index pair k of round r of the circle method on 64 indices (index 63 fixed).
__device__ __forceinline__ void circle64(int r, int k, int& p, int& q) {
  int x, y;
  if (k == 0) { x = 63; y = r; }
  else { x = (r + k) % 63; y = (r - k + 63) % 63; }
  p = min(x, y);
  q = max(x, y);
}

__device__ __forceinline__ int blk_row(int I, int J, int i) {
  return i < PB ? I * PB + i : J * PB + (i - PB);
}

// One workgroup per block pair: Jacobi on the 64 x 64 subproblem in LDS.  The solved block
// goes back into A (upper triangle, mirrored, so A stays exactly symmetric) and its
// orthogonal factor U = product of the rotations into U.  Every rotation ends like the
// scalar method's: the pivot entry becomes exactly 0 and the diagonal app + t apq,
// aqq - t apq, so the diagonal blocks keep the entry-wise accuracy of scalar Jacobi.
//
// With full != 0 an inner sweep visits all 2016 pairs of the subproblem (63 rounds of the
// circle method); otherwise only the 1024 pairs that couple the two blocks (32 rounds,
// round r pairing local index a with 32 + (a + r) mod 32).  The first round of every outer
// sweep is full: its block pairs cover each block once, so every pair inside a block is
// rotated there, and the later rounds need only the cross pairs: one outer sweep then
// rotates each index pair once, like a scalar cyclic sweep.
//
// A rotation is skipped when both a_pq and a_pp - a_qq are at the rounding level of the
// diagonal (|.| <= 2^-22 (|a_pp| + |a_qq|)): FP32 cannot tell such eigenvalues apart, its
// rotation angle would be set by rounding noise, and the large noise-driven rotations
// inside a cluster would keep re-mixing the cluster's couplings to the rest of the matrix,
// so that they only decay linearly.  Those entries are left for the FP64 phase.
constexpr int SNT = 512;
constexpr float kNoise = 0x1p-22f;

__device__ __forceinline__ bool f32_noise_pair(float app, float aqq, float apq) {
  const float nz = kNoise * (fabsf(app) + fabsf(aqq));
  return fabsf(app - aqq) <= nz && fabsf(apq) <= nz;
}

// Rotation of the FP32 stage: the same formula as the FP64 phase (t = 2a / (|d| +
// sqrt(d^2 + 4a^2)), sign of d; c = 1/sqrt(1+t^2); s = t c) evaluated with the hardware
// square root, reciprocal and reciprocal square root (about 1 ulp each).  The stage's
// result is re-orthogonalised in FP64, so the angle only needs FP32 working accuracy, and
// these few instructions replace the correctly rounded sequences that made every inner
// round issue-bound.
__device__ __forceinline__ void rot_fast(float app, float aqq, float apq, float& t, float& c,
                                         float& s) {
  float d = app - aqq, a = apq;
  const float m = fmaxf(fabsf(d), fabsf(a));
  if (m < 0x1p-50f || m > 0x1p50f) {
    int e;
    (void)frexpf(m, &e);
    d = ldexpf(d, -e);
    a = ldexpf(a, -e);
  }
  const float den = fabsf(d) + __builtin_amdgcn_sqrtf(d * d + 4.0f * (a * a));
  float tt = (2.0f * a) * __builtin_amdgcn_rcpf(den);
  if (d < 0.0f) tt = -tt;
  c = __builtin_amdgcn_rsqf(1.0f + tt * tt);
  s = tt * c;
  t = tt;
}

__device__ __forceinline__ void inner_pair(int full, int r, int k, int& p, int& q) {
  if (full) {
    circle64(r, k, p, q);
  } else {
    p = k;
    q = PB + ((k + r) & (PB - 1));
  }
}

__device__ __forceinline__ void solve_body(float (*S)[PL], float (*Ut)[PL], float* __restrict__ A,
                                           int np, int2 pr, float* __restrict__ Uo,
                                           int inner_max, int full, float tol2, float rho2) {
  __shared__ float cs_c[32], cs_s[32], cs_dp[32], cs_dq[32], cs_z[32];
  __shared__ float red[2][SNT / 64];
  const int tid = threadIdx.x;
  for (int e = tid; e < PM * PM; e += SNT) {
    int i = e / PM, j = e % PM;
    S[i][j] = A[(size_t)blk_row(pr.x, pr.y, i) * np + blk_row(pr.x, pr.y, j)];
    Ut[i][j] = (i == j) ? 1.0f : 0.0f;
  }
  __syncthreads();
  // row phase: pair kb, columns jb .. jb+3 (the 16 lanes of a pair share one wave);
  // column phase: pair kc, rows ic .. ic+3
  const int kb = tid >> 4, jb = (tid & 15) * 4;
  const int kc = tid & 31, ic = (tid >> 5) * 4;
  const int nr = full ? PM - 1 : PB;
  float prev_off = 3.4e38f;
  for (int sw = 0; sw < inner_max; ++sw) {
    for (int r = 0; r < nr; ++r) {
      {
        int p, q;
        inner_pair(full, r, kb, p, q);
        // every lane of the pair reads the 2x2 block before any lane of it stores
        float app = S[p][p], aqq = S[q][q];
        const float apq = S[p][q];
        const float4 x = *reinterpret_cast<const float4*>(&S[p][jb]);
        const float4 y = *reinterpret_cast<const float4*>(&S[q][jb]);
        float c = 1.0f, s = 0.0f;
        const bool skip = apq == 0.0f || f32_noise_pair(app, aqq, apq);
        if (!skip) {
          float t;
          rot_fast(app, aqq, apq, t, c, s);
          app = app + t * apq;
          aqq = aqq - t * apq;
        }
        float4 xo, yo;
        xo.x = c * x.x + s * y.x; yo.x = c * y.x - s * x.x;
        xo.y = c * x.y + s * y.y; yo.y = c * y.y - s * x.y;
        xo.z = c * x.z + s * y.z; yo.z = c * y.z - s * x.z;
        xo.w = c * x.w + s * y.w; yo.w = c * y.w - s * x.w;
        *reinterpret_cast<float4*>(&S[p][jb]) = xo;
        *reinterpret_cast<float4*>(&S[q][jb]) = yo;
        if ((tid & 15) == 0) {
          cs_c[kb] = c; cs_s[kb] = s;
          cs_dp[kb] = app; cs_dq[kb] = aqq;
          cs_z[kb] = skip ? apq : 0.0f;
        }
      }
      __syncthreads();
      {
        int p, q;
        inner_pair(full, r, kc, p, q);
        const float c = cs_c[kc], s = cs_s[kc];
        float sx[4], sy[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) { sx[k] = S[ic + k][p]; sy[k] = S[ic + k][q]; }
        const float4 up = *reinterpret_cast<const float4*>(&Ut[p][ic]);
        const float4 uq = *reinterpret_cast<const float4*>(&Ut[q][ic]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int i = ic + k;
          float op = c * sx[k] + s * sy[k], oq = c * sy[k] - s * sx[k];
          if (i == p) { op = cs_dp[kc]; oq = cs_z[kc]; }
          if (i == q) { op = cs_z[kc]; oq = cs_dq[kc]; }
          S[i][p] = op;
          S[i][q] = oq;
        }
        float4 po, qo;
        po.x = c * up.x + s * uq.x; qo.x = c * uq.x - s * up.x;
        po.y = c * up.y + s * uq.y; qo.y = c * uq.y - s * up.y;
        po.z = c * up.z + s * uq.z; qo.z = c * uq.z - s * up.z;
        po.w = c * up.w + s * uq.w; qo.w = c * uq.w - s * up.w;
        *reinterpret_cast<float4*>(&Ut[p][ic]) = po;
        *reinterpret_cast<float4*>(&Ut[q][ic]) = qo;
      }
      __syncthreads();
    }
    if (sw + 1 < inner_max) {
      // off(S) and ||S||_F decide whether another inner sweep pays
      float so = 0.0f, sd = 0.0f;
      for (int e = tid; e < PM * PM; e += SNT) {
        int i = e / PM, j = e % PM;
        float v = S[i][j] * S[i][j];
        if (i == j) sd += v; else so += v;
      }
      for (int o = 32; o > 0; o >>= 1) { so += __shfl_xor(so, o); sd += __shfl_xor(sd, o); }
      if ((tid & 63) == 0) { red[0][tid >> 6] = so; red[1][tid >> 6] = sd; }
      __syncthreads();
      float off = 0.0f, dg = 0.0f;
      for (int w = 0; w < SNT / 64; ++w) { off += red[0][w]; dg += red[1][w]; }
      __syncthreads();
      if (off <= tol2 * (off + dg) || off >= rho2 * prev_off) break;
      prev_off = off;
    }
  }
  for (int e = tid; e < PM * PM; e += SNT) {
    int i = e / PM, j = e % PM;
    Uo[e] = Ut[j][i];
    float v = (i <= j) ? S[i][j] : S[j][i];
    A[(size_t)blk_row(pr.x, pr.y, i) * np + blk_row(pr.x, pr.y, j)] = v;
  }
}

// Block update of A for block pairs P < R: A_PR <- U_P^T A_PR U_R, mirrored to A_RP (so A
// stays exactly symmetric).  The diagonal pair blocks were written by the subproblem solve.
__global__ __launch_bounds__(256) void k_block_apply_a(float* __restrict__ A, int np,
                                                       const int2* __restrict__ pairs,
                                                       const float* __restrict__ U, int nb2) {
  __shared__ __align__(16) float Up[PM][PL], Ur[PM][PL], Ab[PM][PL];
  const int tid = threadIdx.x;
  // blockIdx.x enumerates P < R
  int b = blockIdx.x, P = 0;
  while (b >= nb2 - 1 - P) { b -= nb2 - 1 - P; ++P; }
  const int R = P + 1 + b;
  const int2 pp = pairs[P], pr = pairs[R];
  const float* Ug = U + (size_t)P * PM * PM;
  const float* Uh = U + (size_t)R * PM * PM;
  for (int e = tid; e < PM * PM; e += 256) {
    int i = e / PM, j = e % PM;
    Up[i][j] = Ug[e];
    Ur[i][j] = Uh[e];
    Ab[i][j] = A[(size_t)blk_row(pp.x, pp.y, i) * np + blk_row(pr.x, pr.y, j)];
  }
  __syncthreads();
  const int ti = (tid >> 4) * 4, tj = (tid & 15) * 4;
  float acc[4][4];
  // T = U_P^T A_PR
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = 0.0f;
  for (int k = 0; k < PM; ++k) {
    float4 u = *reinterpret_cast<const float4*>(&Up[k][ti]);
    float4 x = *reinterpret_cast<const float4*>(&Ab[k][tj]);
    float uu[4] = {u.x, u.y, u.z, u.w}, xx[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(uu[a], xx[c], acc[a][c]);
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) Ab[ti + a][tj + c] = acc[a][c];
  __syncthreads();
  // out = T U_R
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = 0.0f;
  for (int k = 0; k < PM; ++k) {
    float4 u = *reinterpret_cast<const float4*>(&Ur[k][tj]);
    float uu[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      float t = Ab[ti + a][k];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(t, uu[c], acc[a][c]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int gi = blk_row(pp.x, pp.y, ti + a), gj = blk_row(pr.x, pr.y, tj + c);
      A[(size_t)gi * np + gj] = acc[a][c];
      A[(size_t)gj * np + gi] = acc[a][c];
    }
}

// V <- V U_R on the columns of block pair R, for the tile of 64 rows from r0.
__device__ __forceinline__ void vtile_body(float (*Ur)[PL], float (*Vb)[PL], float* __restrict__ V,
                                           int nrows, int np, int r0, int2 pr,
                                           const float* __restrict__ Uh) {
  const int tid = threadIdx.x;
  for (int e = tid; e < PM * PM; e += SNT) {
    int i = e / PM, j = e % PM;
    Ur[i][j] = Uh[e];
    Vb[i][j] = (r0 + i < nrows) ? V[(size_t)(r0 + i) * np + blk_row(pr.x, pr.y, j)] : 0.0f;
  }
  __syncthreads();
  const int ti = (tid >> 4) * 2, tj = (tid & 15) * 4;
  float acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[a][c] = 0.0f;
#pragma unroll 4
  for (int k = 0; k < PM; ++k) {
    float4 u = *reinterpret_cast<const float4*>(&Ur[k][tj]);
    float uu[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      float t = Vb[ti + a][k];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(t, uu[c], acc[a][c]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (r0 + ti + a < nrows)
        V[(size_t)(r0 + ti + a) * np + blk_row(pr.x, pr.y, tj + c)] = acc[a][c];
}

// One launch per round: blocks [0, nsolve) solve the round's block pairs (writing U of this
// round); the remaining blocks apply the previous round's factors to V, which no solve reads,
// so the V update runs beside the next round's subproblem solves.
__global__ __launch_bounds__(SNT) void k_block_round(float* __restrict__ A, int np,
                                                     const int2* __restrict__ pairs,
                                                     float* __restrict__ U, int nsolve,
                                                     int inner_max, int full, float tol2,
                                                     float rho2, float* __restrict__ V, int nrows,
                                                     const int2* __restrict__ vpairs,
                                                     const float* __restrict__ vU, int nvt) {
  __shared__ __align__(16) float lds[2][PM][PL];
  if ((int)blockIdx.x < nsolve) {
    solve_body(lds[0], lds[1], A, np, pairs[blockIdx.x], U + (size_t)blockIdx.x * PM * PM,
               inner_max, full, tol2, rho2);
  } else {
    const int b = blockIdx.x - nsolve, R = b / nvt, rt = b - R * nvt;
    vtile_body(lds[0], lds[1], V, nrows, np, rt * PM, vpairs[R], vU + (size_t)R * PM * PM);
  }
}

// A32 (np x np, zero padded) <- fl32(A)
__global__ void k_to_f32_pad(const double* __restrict__ A, int n, int lda, float* __restrict__ B,
                             int np) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)np * np) return;
  int i = (int)(idx / np), j = (int)(idx - (size_t)i * np);
  B[idx] = (i < n && j < n) ? (float)A[(size_t)i * lda + j] : 0.0f;
}

__global__ void k_identity_f32(float* V, int nrows, int ldv) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nrows * ldv) return;
  int i = (int)(idx / ldv), j = (int)(idx - (size_t)i * ldv);
  V[idx] = (i == j) ? 1.0f : 0.0f;
}

// off(A)^2 and ||A||_F^2 of an np x np FP32 matrix (double accumulation, fixed order).
__global__ __launch_bounds__(256) void k_off_norm_f32(const float* __restrict__ A, int np,
                                                      double* __restrict__ partial) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= np) return;
  double so = 0.0, sd = 0.0;
  for (int l = lane; l < np; l += 64) {
    double v = A[(size_t)row * np + l];
    if (l == row) sd += v * v;
    else so += v * v;
  }
  so = wave_sum_fast(so);
  sd = wave_sum_fast(sd);
  if (lane == 0) { partial[2 * row] = so; partial[2 * row + 1] = sd; }
}

__global__ __launch_bounds__(256) void k_off_norm_sum(const double* __restrict__ partial, int np,
                                                      double* out) {
  __shared__ double w[2][4];
  double so = 0.0, sd = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) { so += partial[2 * k]; sd += partial[2 * k + 1]; }
  so = wave_sum_fast(so);
  sd = wave_sum_fast(sd);
  if ((threadIdx.x & 63) == 0) { w[0][threadIdx.x >> 6] = so; w[1][threadIdx.x >> 6] = sd; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = ((w[0][0] + w[0][1]) + w[0][2]) + w[0][3];
    double d = ((w[1][0] + w[1][1]) + w[1][2]) + w[1][3];
    out[0] = sqrt(o);
    out[1] = sqrt(o + d);
  }
}

// Q (n x n, FP64, row-major) <- the first n columns of V32
__global__ void k_gather_q(const float* __restrict__ V, int n, int ldv, double* __restrict__ Q,
                           int ldq) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
  Q[(size_t)i * ldq + j] = (double)V[(size_t)i * ldv + j];
}

static int padded(int n) { return (n + PM - 1) / PM * PM; }

size_t precond_f32_bytes(int n) {
  size_t np = (size_t)padded(n), nb = np / PB;
  size_t b = np * np * 4 + (size_t)n * np * 4;   // A32, V32
  b += 2 * (nb / 2) * PM * PM * 4;                // U of every block pair of two rounds
  b += (nb - 1 > 0 ? nb - 1 : 1) * (nb / 2) * 8;  // pair table of all rounds
  b += 2 * np * 8 + 256;                          // partial sums + result
  return (b + 4095) & ~(size_t)4095;
}

hipError_t run_precond_f32(const double* Asym, int n, int ld, double* Q, int ldq, void* scratch,
                           int max_sweeps, double tol, double rho, int* sweeps, hipStream_t s) {
  const int np = padded(n), nb = np / PB, nb2 = nb / 2, rounds = nb - 1;
  char* p = (char*)scratch;
  float* A32 = (float*)p; p += (size_t)np * np * 4;
  float* V32 = (float*)p; p += (size_t)n * np * 4;
  float* U = (float*)p; p += 2 * (size_t)nb2 * PM * PM * 4;
  int2* pairs = (int2*)p; p += (size_t)rounds * nb2 * 8;
  double* part = (double*)p; p += 2 * (size_t)np * 8;
  double* res = (double*)p;
  hipError_t e;
  // circle-method block pairs of every round (block nb - 1 fixed)
  std::vector<int2> tab((size_t)rounds * nb2);
  for (int r = 0; r < rounds; ++r)
    for (int k = 0; k < nb2; ++k) {
      int x, y;
      if (k == 0) { x = nb - 1; y = r; }
      else { x = (r + k) % (nb - 1); y = (r - k + (nb - 1)) % (nb - 1); }
      tab[(size_t)r * nb2 + k] = int2{x < y ? x : y, x < y ? y : x};
    }
  if ((e = hipMemcpyAsync(pairs, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return e;
  {
    size_t tot = (size_t)np * np;
    hipLaunchKernelGGL(k_to_f32_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Asym,
                       n, ld, A32, np);
    size_t totv = (size_t)n * np;
    hipLaunchKernelGGL(k_identity_f32, dim3((unsigned)((totv + 255) / 256)), dim3(256), 0, s, V32,
                       n, np);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  double h[2];
  auto off_norm = [&]() -> hipError_t {
    hipLaunchKernelGGL(k_off_norm_f32, dim3((np + 3) / 4), dim3(256), 0, s, A32, np, part);
    hipLaunchKernelGGL(k_off_norm_sum, dim3(1), dim3(256), 0, s, part, np, res);
    hipError_t r = hipMemcpyAsync(h, res, 16, hipMemcpyDeviceToHost, s);
    if (r == hipSuccess) r = hipStreamSynchronize(s);
    return r;
  };
  if ((e = off_norm()) != hipSuccess) return e;
  double off = h[0], nrm = h[1];
  // a single block pair is the whole matrix: its subproblem solve converges it
  const int inner = (nb == 2) ? max_sweeps : 1;
  const int nvt = (n + PM - 1) / PM;
  // U of consecutive rounds alternates between two buffers; the V update of a round runs
  // in the next round's launch (or in a launch of its own after the last round)
  long long g = 0;
  int vround = -1;
  auto ubuf = [&](long long k) { return U + (size_t)(k & 1) * nb2 * PM * PM; };
  auto vlaunch_args = [&](int nsolve, const int2* pr, float* Uw, int full) {
    const int nv = vround >= 0 ? nvt * nb2 : 0;
    const int2* vp = vround >= 0 ? pairs + (size_t)vround * nb2 : pairs;
    hipLaunchKernelGGL(k_block_round, dim3(nsolve + nv), dim3(SNT), 0, s, A32, np, pr, Uw,
                       nsolve, inner, full, (float)(tol * tol), (float)(rho * rho), V32, n, vp,
                       ubuf(g - 1), nvt);
  };
  int sw = 0;
  while (sw < max_sweeps && off > tol * nrm) {
    for (int r = 0; r < rounds; ++r, ++g) {
      const int2* pr = pairs + (size_t)r * nb2;
      vlaunch_args(nb2, pr, ubuf(g), r == 0 ? 1 : 0);
      if (nb2 > 1)
        hipLaunchKernelGGL(k_block_apply_a, dim3(nb2 * (nb2 - 1) / 2), dim3(256), 0, s, A32, np,
                           pr, ubuf(g), nb2);
      vround = r;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ++sw;
    double prev = off;
    if ((e = off_norm()) != hipSuccess) return e;
    off = h[0];
    nrm = h[1];
    if (nb == 2 || off >= rho * prev) break;
  }
  if (vround >= 0) {
    vlaunch_args(0, pairs, nullptr, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  *sweeps = sw;
  size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(k_gather_q, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V32, n, np,
                     Q, ldq);
  return hipGetLastError();
}

}  // namespace je
