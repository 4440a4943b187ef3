// Low-precision spectral decomposition of the preconditioner (Sec. 2.1): a blocked
// two-sided Jacobi in FP32 (the eigenvector matrix is re-orthogonalised in FP64 by the host
// driver afterwards).
//
// The matrix (padded with zero rows/columns to np = a multiple of 2 PB) is split into
// blocks of PB rows (PB = 16 or 32).  A sweep visits every pair of blocks once in
// round-robin (circle method) order: nb - 1 rounds of nb/2 disjoint block pairs.  For each
// pair (I, J) of a round one workgroup applies scalar FP32 Jacobi rotations (parallel
// round-robin inside the block) to the PM x PM subproblem [[A_II, A_IJ], [A_JI, A_JJ]]
// (PM = 2 PB) in LDS, accumulating its orthogonal factor U_IJ; then every other PM x PM
// block of A is replaced by U_P^T A_PR U_R and the columns of V by V U_R.  Each round reads
// and writes A and V once, so a sweep costs nb - 1 passes over memory instead of np - 1.
// For n <= PM the single block pair is the whole matrix and the subproblem solve is the
// whole decomposition.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "device_common.h"
#include "kernels.h"

namespace je {

// The FP32 stage's rotations may fuse multiply-adds (the library is built without
// contraction so that the FP64 pivot sequence is a function of the input bits alone; the
// FP32 stage only has to reach FP32 working accuracy, and its result is re-orthogonalised
// in FP64): one fused operation instead of a product and a sum in every rotated entry.
#define FP32_CONTRACT _Pragma("clang fp contract(fast)")

// Block geometry: PB rows per block, PM = 2 PB per subproblem, LDS rows padded by 4 floats
// (16-byte aligned), NT threads per workgroup so that both phases of an inner round give
// every thread four entries of S.
template <int PB>
struct Blk {
  static_assert(PB % 4 == 0, "tiles move four consecutive floats per lane");
  static constexpr int PM = 2 * PB;
  static constexpr int PL = PM + 4;
  static constexpr int NT = PB * PM / 4;
};

// Index pair k of round r of the circle method on M indices (index M - 1 fixed).
template <int M>
__device__ __forceinline__ void circle(int r, int k, int& p, int& q) {
  int x, y;
  if (k == 0) { x = M - 1; y = r; }
  else { x = (r + k) % (M - 1); y = (r - k + M - 1) % (M - 1); }
  p = min(x, y);
  q = max(x, y);
}

template <int PB>
__device__ __forceinline__ int blk_row(int I, int J, int i) {
  return i < PB ? I * PB + i : J * PB + (i - PB);
}

// LDS staging of PM x PM operands, four consecutive columns per lane (16-byte accesses;
// PB is a multiple of 4, so the four never straddle two blocks).  Block (rows of pair rp,
// columns of pair cp) of a padded np x np matrix:
template <int PB>
__device__ __forceinline__ void load_pair_block(float (*T)[Blk<PB>::PL],
                                                const float* __restrict__ A, int np, int2 rp,
                                                int2 cp) {
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT;
  for (int e = threadIdx.x; e < PM * PM / 4; e += NT) {
    const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
    *reinterpret_cast<float4*>(&T[i][j]) = *reinterpret_cast<const float4*>(
        A + (size_t)blk_row<PB>(rp.x, rp.y, i) * np + blk_row<PB>(cp.x, cp.y, j));
  }
}

// a row-major PM x PM factor:
template <int PB>
__device__ __forceinline__ void load_factor(float (*T)[Blk<PB>::PL],
                                            const float* __restrict__ U) {
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT;
  for (int e = threadIdx.x; e < PM * PM / 4; e += NT) {
    const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
    *reinterpret_cast<float4*>(&T[i][j]) = *reinterpret_cast<const float4*>(U + i * PM + j);
  }
}

// the identity:
template <int PB>
__device__ __forceinline__ void set_identity(float (*T)[Blk<PB>::PL]) {
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT;
  for (int e = threadIdx.x; e < PM * PM / 4; e += NT) {
    const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
    *reinterpret_cast<float4*>(&T[i][j]) =
        make_float4(i == j ? 1.0f : 0.0f, i == j + 1 ? 1.0f : 0.0f, i == j + 2 ? 1.0f : 0.0f,
                    i == j + 3 ? 1.0f : 0.0f);
  }
}

// Write-back of a solved subproblem: U (row-major PM x PM) = Ut^T, and the block pair of
// A from the upper triangle of S, mirrored.
template <int PB>
__device__ __forceinline__ void store_solved(const float (*S)[Blk<PB>::PL],
                                             const float (*Ut)[Blk<PB>::PL],
                                             float* __restrict__ Uo, float* __restrict__ Aout,
                                             int np, int2 pr) {
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT;
  for (int e = threadIdx.x; e < PM * PM / 4; e += NT) {
    const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
    const float4 u = make_float4(Ut[j][i], Ut[j + 1][i], Ut[j + 2][i], Ut[j + 3][i]);
    const float4 v =
        make_float4(i <= j ? S[i][j] : S[j][i], i <= j + 1 ? S[i][j + 1] : S[j + 1][i],
                    i <= j + 2 ? S[i][j + 2] : S[j + 2][i], i <= j + 3 ? S[i][j + 3] : S[j + 3][i]);
    *reinterpret_cast<float4*>(Uo + i * PM + j) = u;
    *reinterpret_cast<float4*>(Aout + (size_t)blk_row<PB>(pr.x, pr.y, i) * np +
                               blk_row<PB>(pr.x, pr.y, j)) = v;
  }
}

// One workgroup per block pair: Jacobi on the PM x PM subproblem in LDS.  The solved block
// goes back into A (upper triangle, mirrored, so A stays exactly symmetric) and its
// orthogonal factor U = product of the rotations into U.  Every rotation ends like the
// scalar method's: the pivot entry becomes exactly 0 and the diagonal app + t apq,
// aqq - t apq, so the diagonal blocks keep the entry-wise accuracy of scalar Jacobi.
//
// With full != 0 an inner sweep visits all pairs of the subproblem (PM - 1 rounds of the
// circle method); otherwise only the PB^2 pairs that couple the two blocks (PB rounds,
// round r pairing local index a with PB + (a + r) mod PB).  The first round of every outer
// sweep is full: its block pairs cover each block once, so every pair inside a block is
// rotated there, and the later rounds need only the cross pairs: one outer sweep then
// rotates each index pair once, like a scalar cyclic sweep.
//
// A rotation is skipped when both a_pq and a_pp - a_qq are at the rounding level of the
// diagonal (|.| <= 2^-22 (|a_pp| + |a_qq|)): FP32 cannot tell such eigenvalues apart, its
// rotation angle would be set by rounding noise, and the large noise-driven rotations
// inside a cluster would keep re-mixing the cluster's couplings to the rest of the matrix,
// so that they only decay linearly.  Those entries are left for the FP64 phase.
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
  FP32_CONTRACT
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

template <int PB>
__device__ __forceinline__ void inner_pair(int full, int r, int k, int& p, int& q) {
  if (full) {
    circle<2 * PB>(r, k, p, q);
  } else {
    p = k;
    q = PB + ((k + r) & (PB - 1));
  }
}

// Two-phase inner round (the form used for 16-row blocks).  Both phases read rows only.  With J the product of the round's disjoint
// rotations, the row phase forms M = J^T S and stores it transposed, W = M^T; the second
// phase forms J^T W = (S J ... )^T, i.e. the rotated matrix J^T S J read by rows (it is
// symmetric up to rounding; its upper triangle is the one used).  A lane keeps the same
// pair and columns in both phases, so its c, s stay in registers.
template <int PB>
__device__ __forceinline__ void solve_body_rows(float (*S)[Blk<PB>::PL], float (*W)[Blk<PB>::PL],
                                           float (*Ut)[Blk<PB>::PL], const float* Ain,
                                           float* Aout, int np, int2 pr, float* __restrict__ Uo,
                                           int inner_max, int full, float tol2, float rho2,
                                           bool preloaded) {
  FP32_CONTRACT
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT, LB = PM / 4;
  __shared__ float red[2][NT / 64];
  const int tid = threadIdx.x;
  if (!preloaded) {
    load_pair_block<PB>(S, Ain, np, pr, pr);
    set_identity<PB>(Ut);
    __syncthreads();
  }
  // pair kb, columns jb .. jb+3 (the LB lanes of a pair share one wave)
  const int kb = tid / LB, jb = (tid % LB) * 4;
  const int nr = full ? PM - 1 : PB;
  float prev_off = 3.4e38f;
  for (int sw = 0; sw < inner_max; ++sw) {
    for (int r = 0; r < nr; ++r) {
      int p, q;
      inner_pair<PB>(full, r, kb, p, q);
      // every lane of the pair reads the 2x2 block before any lane of it stores
      float app = S[p][p], aqq = S[q][q];
      const float apq = S[p][q];
      const float4 x = *reinterpret_cast<const float4*>(&S[p][jb]);
      const float4 y = *reinterpret_cast<const float4*>(&S[q][jb]);
      // rows p, q of U^T belong to this pair's lanes alone in this round: rotated here,
      // beside the first phase, off the second phase's dependency chain
      const float4 up = *reinterpret_cast<const float4*>(&Ut[p][jb]);
      const float4 uq = *reinterpret_cast<const float4*>(&Ut[q][jb]);
      float c = 1.0f, s = 0.0f;
      const bool skip = apq == 0.0f || f32_noise_pair(app, aqq, apq);
      if (!skip) {
        float t;
        rot_fast(app, aqq, apq, t, c, s);
        app = app + t * apq;
        aqq = aqq - t * apq;
      }
      const float z = skip ? apq : 0.0f;
      W[jb + 0][p] = c * x.x + s * y.x; W[jb + 0][q] = c * y.x - s * x.x;
      W[jb + 1][p] = c * x.y + s * y.y; W[jb + 1][q] = c * y.y - s * x.y;
      W[jb + 2][p] = c * x.z + s * y.z; W[jb + 2][q] = c * y.z - s * x.z;
      W[jb + 3][p] = c * x.w + s * y.w; W[jb + 3][q] = c * y.w - s * x.w;
      {
        float4 po, qo;
        po.x = c * up.x + s * uq.x; qo.x = c * uq.x - s * up.x;
        po.y = c * up.y + s * uq.y; qo.y = c * uq.y - s * up.y;
        po.z = c * up.z + s * uq.z; qo.z = c * uq.z - s * up.z;
        po.w = c * up.w + s * uq.w; qo.w = c * uq.w - s * up.w;
        *reinterpret_cast<float4*>(&Ut[p][jb]) = po;
        *reinterpret_cast<float4*>(&Ut[q][jb]) = qo;
      }
      __syncthreads();
      {
        const float4 wx = *reinterpret_cast<const float4*>(&W[p][jb]);
        const float4 wy = *reinterpret_cast<const float4*>(&W[q][jb]);
        float xo[4] = {c * wx.x + s * wy.x, c * wx.y + s * wy.y, c * wx.z + s * wy.z,
                       c * wx.w + s * wy.w};
        float yo[4] = {c * wy.x - s * wx.x, c * wy.y - s * wx.y, c * wy.z - s * wx.z,
                       c * wy.w - s * wx.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (jb + v == p) { xo[v] = app; yo[v] = z; }
          if (jb + v == q) { xo[v] = z; yo[v] = aqq; }
        }
        *reinterpret_cast<float4*>(&S[p][jb]) = make_float4(xo[0], xo[1], xo[2], xo[3]);
        *reinterpret_cast<float4*>(&S[q][jb]) = make_float4(yo[0], yo[1], yo[2], yo[3]);
      }
      __syncthreads();
    }
    if (sw + 1 < inner_max) {
      // off(S) and ||S||_F decide whether another inner sweep pays
      float so = 0.0f, sd = 0.0f;
      for (int e = tid; e < PM * PM; e += NT) {
        int i = e / PM, j = e % PM;
        float v = S[i][j] * S[i][j];
        if (i == j) sd += v; else so += v;
      }
      for (int o = 32; o > 0; o >>= 1) { so += __shfl_xor(so, o); sd += __shfl_xor(sd, o); }
      if ((tid & 63) == 0) { red[0][tid >> 6] = so; red[1][tid >> 6] = sd; }
      __syncthreads();
      float off = 0.0f, dg = 0.0f;
      for (int w = 0; w < NT / 64; ++w) { off += red[0][w]; dg += red[1][w]; }
      __syncthreads();
      if (off <= tol2 * (off + dg) || off >= rho2 * prev_off) break;
      prev_off = off;
    }
  }
  store_solved<PB>(S, Ut, Uo, Aout, np, pr);
}

// Rotation of one pair of an inner round, from the current subproblem: cosine, sine, the
// new diagonal entries and the new pivot entry (0, or a_pq itself when the pair is
// skipped, see f32_noise_pair).
struct RotF {
  float c, s, napp, naqq, z;
};

template <int PL>
__device__ __forceinline__ RotF pair_rot(const float (*S)[PL], int p, int q) {
  FP32_CONTRACT
  const float app = S[p][p], aqq = S[q][q], apq = S[p][q];
  RotF r{1.0f, 0.0f, app, aqq, apq};
  if (!(apq == 0.0f || f32_noise_pair(app, aqq, apq))) {
    float t;
    rot_fast(app, aqq, apq, t, r.c, r.s);
    r.napp = app + t * apq;
    r.naqq = aqq - t * apq;
    r.z = 0.0f;
  }
  return r;
}

// 2 x 2 block X = S[{pb, qb}][{pc, qc}] of the rotated subproblem J^T S J: rows by pair b,
// then columns by pair c; the diagonal block of a pair (b == c) gets its new diagonal and
// pivot entries exactly.
__device__ __forceinline__ void rot_block(const RotF& rb, const RotF& rc, bool diag, float& x,
                                          float& y, float& z, float& w) {
  FP32_CONTRACT
  const float x1 = rb.c * x + rb.s * z, y1 = rb.c * y + rb.s * w;
  const float z1 = rb.c * z - rb.s * x, w1 = rb.c * w - rb.s * y;
  x = diag ? rb.napp : rc.c * x1 + rc.s * y1;
  y = diag ? rb.z : rc.c * y1 - rc.s * x1;
  z = diag ? rb.z : rc.c * z1 + rc.s * w1;
  w = diag ? rb.naqq : rc.c * w1 - rc.s * z1;
}

// The rotation evaluated by lane `src` of this wave (cross-lane read, ds_bpermute).
__device__ __forceinline__ RotF fetch_rot(const RotF& x, int src) {
  RotF r;
  r.c = __shfl(x.c, src);
  r.s = __shfl(x.s, src);
  r.napp = __shfl(x.napp, src);
  r.naqq = __shfl(x.naqq, src);
  r.z = __shfl(x.z, src);
  return r;
}

// An inner round is one phase: the pairs of the round are disjoint, so J^T S J is, block by
// block, X_bc -> J_b^T X_bc J_c over the 2 x 2 blocks of pair b's rows and pair c's columns.
// Lane l of wave w owns column pair c = l mod 32 and row pairs kb = 2 w + l / 32 and
// kb + PM / 4: the blocks (kb, c), (kb + PM / 4, c), and columns 4 (c mod 16) .. + 3 of rows
// p, q of U^T for one of the two row pairs.  The 32 lanes of a half wave share a row pair,
// so their reads and writes of S fall on 32 consecutive columns (32 banks) in the rounds
// that pair the two blocks (with the former layout, two column pairs per lane, they met
// two-way bank conflicts: batched solve 66 -> 62 ms).  A lane evaluates its column pair's rotation itself and reads the row pairs'
// from the lanes that evaluated them (the same instructions on the same values in every
// lane, so all lanes agree).  S is double-buffered: a round reads one buffer and writes the
// other, and a single barrier separates rounds.  S stays symmetric up to rounding; its upper
// triangle is the one used.  (Used for 32-row blocks: measured against the two-phase form,
// n = 4096 FP32 stage 243 -> 236 ms, batches 272 -> 261 ms; for 16-row blocks, two waves per
// subproblem, the two-phase form is faster, n = 1024 27.8 vs 34.7 ms.)
template <int PB>
__device__ __forceinline__ void solve_body_blocks(float (*S)[Blk<PB>::PL], float (*W)[Blk<PB>::PL],
                                           float (*Ut)[Blk<PB>::PL], const float* Ain,
                                           float* Aout, int np, int2 pr, float* __restrict__ Uo,
                                           int inner_max, int full, float tol2, float rho2,
                                           bool preloaded) {
  FP32_CONTRACT
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT, PL = Blk<PB>::PL;
  static_assert(PM == 64 && NT == 512, "32-row blocks: 8 waves, 32 column pairs");
  __shared__ float red[2][NT / 64];
  const int tid = threadIdx.x;
  if (!preloaded) {
    load_pair_block<PB>(S, Ain, np, pr, pr);
    set_identity<PB>(Ut);
    __syncthreads();
  }
  const int lane = tid & 63, c = lane & 31;
  const int kb0 = 2 * (tid >> 6) + (lane >> 5);
  const int nr = full ? PM - 1 : PB;
  float(*Sc)[PL] = S;
  float(*Sn)[PL] = W;
  float prev_off = 3.4e38f;
  for (int sw = 0; sw < inner_max; ++sw) {
    for (int r = 0; r < nr; ++r) {
      int pc, qc;
      inner_pair<PB>(full, r, c, pc, qc);
      const RotF rc = pair_rot<PL>(Sc, pc, qc);
      int pb[2], qb[2];
      RotF rb[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kb = kb0 + h * (PM / 4);
        inner_pair<PB>(full, r, kb, pb[h], qb[h]);
        float x = Sc[pb[h]][pc], y = Sc[pb[h]][qc], z = Sc[qb[h]][pc], w = Sc[qb[h]][qc];
        rb[h] = fetch_rot(rc, kb);
        rot_block(rb[h], rc, kb == c, x, y, z, w);
        Sn[pb[h]][pc] = x; Sn[pb[h]][qc] = y; Sn[qb[h]][pc] = z; Sn[qb[h]][qc] = w;
      }
      {
        // rows p, q of U^T: lane c < 16 takes columns 4c .. 4c + 3 of the first row pair,
        // lane c >= 16 those of the second
        const int h = c >> 4, jb = 4 * (c & 15);
        const RotF& ru = h ? rb[1] : rb[0];
        const int pu = h ? pb[1] : pb[0], qu = h ? qb[1] : qb[0];
        const float4 up = *reinterpret_cast<const float4*>(&Ut[pu][jb]);
        const float4 uq = *reinterpret_cast<const float4*>(&Ut[qu][jb]);
        float4 po, qo;
        po.x = ru.c * up.x + ru.s * uq.x; qo.x = ru.c * uq.x - ru.s * up.x;
        po.y = ru.c * up.y + ru.s * uq.y; qo.y = ru.c * uq.y - ru.s * up.y;
        po.z = ru.c * up.z + ru.s * uq.z; qo.z = ru.c * uq.z - ru.s * up.z;
        po.w = ru.c * up.w + ru.s * uq.w; qo.w = ru.c * uq.w - ru.s * up.w;
        *reinterpret_cast<float4*>(&Ut[pu][jb]) = po;
        *reinterpret_cast<float4*>(&Ut[qu][jb]) = qo;
      }
      __syncthreads();
      float(*t)[PL] = Sc;
      Sc = Sn;
      Sn = t;
    }
    if (sw + 1 < inner_max) {
      // off(S) and ||S||_F decide whether another inner sweep pays
      float so = 0.0f, sd = 0.0f;
      for (int e = tid; e < PM * PM; e += NT) {
        int i = e / PM, j = e % PM;
        float v = Sc[i][j] * Sc[i][j];
        if (i == j) sd += v; else so += v;
      }
      for (int o = 32; o > 0; o >>= 1) { so += __shfl_xor(so, o); sd += __shfl_xor(sd, o); }
      if ((tid & 63) == 0) { red[0][tid >> 6] = so; red[1][tid >> 6] = sd; }
      __syncthreads();
      float off = 0.0f, dg = 0.0f;
      for (int w = 0; w < NT / 64; ++w) { off += red[0][w]; dg += red[1][w]; }
      __syncthreads();
      if (off <= tol2 * (off + dg) || off >= rho2 * prev_off) break;
      prev_off = off;
    }
  }
  if (Sc != S) {  // the result ends in S (callers read it there)
    for (int e = tid; e < PM * PM; e += NT) {
      int i = e / PM, j = e % PM;
      S[i][j] = Sc[i][j];
    }
    __syncthreads();
  }
  store_solved<PB>(S, Ut, Uo, Aout, np, pr);
}

template <int PB>
__device__ __forceinline__ void solve_body(float (*S)[Blk<PB>::PL], float (*W)[Blk<PB>::PL],
                                           float (*Ut)[Blk<PB>::PL], const float* Ain,
                                           float* Aout, int np, int2 pr, float* __restrict__ Uo,
                                           int inner_max, int full, float tol2, float rho2,
                                           bool preloaded = false) {
  if constexpr (PB == 16)
    solve_body_rows<PB>(S, W, Ut, Ain, Aout, np, pr, Uo, inner_max, full, tol2, rho2, preloaded);
  else
    solve_body_blocks<PB>(S, W, Ut, Ain, Aout, np, pr, Uo, inner_max, full, tol2, rho2,
                          preloaded);
}

// out (PM x PM) = X^T Y if TA, else X Y; X, Y in LDS.  On the matrix cores
// (v_mfma_f32_16x16x4f32): the output is split into 16 x 16 tiles, two per wave (wave w
// owns tiles 2w and 2w + 1, row-major over the (PM/16)^2 tiles), K advances by 4 per
// instruction.  Operand layout: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k; result
// D[i][j] in lane j + 16 (i / 4), register i % 4 (checked by an in-bounds probe).
typedef float f4 __attribute__((ext_vector_type(4)));

template <int PB, bool TA>
__device__ __forceinline__ void tile_mfma(float (*X)[Blk<PB>::PL], float (*Y)[Blk<PB>::PL],
                                          f4 (&acc)[2]) {
  constexpr int PM = Blk<PB>::PM, TT = PM / 16;
  static_assert(Blk<PB>::NT / 64 * 2 == TT * TT, "two 16 x 16 tiles per wave");
  const int l = threadIdx.x & 63, t0 = (threadIdx.x >> 6) * 2;
  const int li = l & 15, lk = l >> 4;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int ti = (t0 + u) / TT, tj = (t0 + u) % TT;
    f4 c = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < PM; k0 += 4) {
      const float a = TA ? X[k0 + lk][16 * ti + li] : X[16 * ti + li][k0 + lk];
      const float b = Y[k0 + lk][16 * tj + li];
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    acc[u] = c;
  }
}

// Row and column (within the PM x PM output) of register v of tile u of this lane.
template <int PB>
__device__ __forceinline__ void tile_rc(int u, int v, int& i, int& j) {
  constexpr int TT = Blk<PB>::PM / 16;
  const int l = threadIdx.x & 63, t = (threadIdx.x >> 6) * 2 + u;
  i = 16 * (t / TT) + 4 * (l >> 4) + v;
  j = 16 * (t % TT) + (l & 15);
}

template <int PB>
__device__ __forceinline__ void tile_store_lds(float (*T)[Blk<PB>::PL], const f4 (&acc)[2]) {
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i, j;
      tile_rc<PB>(u, v, i, j);
      T[i][j] = acc[u][v];
    }
}

// Block update of A for block pairs P < R: A_PR <- U_P^T A_PR U_R, mirrored to A_RP (so A
// stays exactly symmetric).  The diagonal pair blocks were written by the subproblem solve.
template <int PB>
__global__ __launch_bounds__(Blk<PB>::NT) void k_block_apply_a(float* __restrict__ A, int np,
                                                               const int2* __restrict__ pairs,
                                                               const float* __restrict__ U,
                                                               int nb2) {
  constexpr int PM = Blk<PB>::PM, PL = Blk<PB>::PL, NT = Blk<PB>::NT;
  __shared__ __align__(16) float Up[PM][PL], Ur[PM][PL], Ab[PM][PL];
  const int tid = threadIdx.x;
  // blockIdx.x enumerates P < R
  int b = blockIdx.x, P = 0;
  while (b >= nb2 - 1 - P) { b -= nb2 - 1 - P; ++P; }
  const int R = P + 1 + b;
  const int2 pp = pairs[P], pr = pairs[R];
  const float* Ug = U + (size_t)P * PM * PM;
  const float* Uh = U + (size_t)R * PM * PM;
  for (int e = tid; e < PM * PM; e += NT) {
    int i = e / PM, j = e % PM;
    Up[i][j] = Ug[e];
    Ur[i][j] = Uh[e];
    Ab[i][j] = A[(size_t)blk_row<PB>(pp.x, pp.y, i) * np + blk_row<PB>(pr.x, pr.y, j)];
  }
  __syncthreads();
  f4 acc[2];
  tile_mfma<PB, true>(Up, Ab, acc);  // T = U_P^T A_PR
  __syncthreads();
  tile_store_lds<PB>(Ab, acc);
  __syncthreads();
  tile_mfma<PB, false>(Ab, Ur, acc);  // T U_R
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i, j;
      tile_rc<PB>(u, v, i, j);
      const int gi = blk_row<PB>(pp.x, pp.y, i), gj = blk_row<PB>(pr.x, pr.y, j);
      A[(size_t)gi * np + gj] = acc[u][v];
      A[(size_t)gj * np + gi] = acc[u][v];
    }
}

// V <- V U_R on the columns of block pair R, for the tile of PM rows from r0 (RT threads,
// two 16 x 16 output tiles per wave on the matrix cores).
template <int PB, bool STAGED = false>
__device__ __forceinline__ void vtile_body(float (*Ur)[Blk<PB>::PL], float (*Vb)[Blk<PB>::PL],
                                           float* __restrict__ V, int nrows, int np, int r0,
                                           int2 pr, const float* __restrict__ Uh) {
  constexpr int PM = Blk<PB>::PM, RT = Blk<PB>::NT;
  const int tid = threadIdx.x;
  // four consecutive columns per lane (they lie in one block: PB is a multiple of 4)
  for (int e = tid; e < PM * PM / 4; e += RT) {
    const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
    *reinterpret_cast<float4*>(&Ur[i][j]) = *reinterpret_cast<const float4*>(Uh + i * PM + j);
    *reinterpret_cast<float4*>(&Vb[i][j]) =
        (r0 + i < nrows) ? *reinterpret_cast<const float4*>(
                               V + (size_t)(r0 + i) * np + blk_row<PB>(pr.x, pr.y, j))
                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  __syncthreads();
  f4 acc[2];
  tile_mfma<PB, false>(Vb, Ur, acc);
  if constexpr (STAGED) {
    // through LDS, so that rows are stored four consecutive columns per lane (measured
    // faster for the batched steps, 165 -> 152 us, and not for the fused rounds, where the
    // two extra barriers cost more)
    __syncthreads();
    tile_store_lds<PB>(Vb, acc);
    __syncthreads();
    for (int e = tid; e < PM * PM / 4; e += RT) {
      const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
      if (r0 + i < nrows)
        *reinterpret_cast<float4*>(V + (size_t)(r0 + i) * np + blk_row<PB>(pr.x, pr.y, j)) =
            *reinterpret_cast<const float4*>(&Vb[i][j]);
    }
  } else {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i, j;
        tile_rc<PB>(u, v, i, j);
        if (r0 + i < nrows) V[(size_t)(r0 + i) * np + blk_row<PB>(pr.x, pr.y, j)] = acc[u][v];
      }
  }
}

// One launch per round: blocks [0, nsolve) solve the round's block pairs (writing U of this
// round); the remaining blocks apply the previous round's factors to V, which no solve reads,
// so the V update runs beside the next round's subproblem solves.
template <int PB>
__global__ __launch_bounds__(Blk<PB>::NT) void k_block_round(
    float* __restrict__ A, int np, const int2* __restrict__ pairs, float* __restrict__ U,
    int nsolve, int inner_max, int full, float tol2, float rho2, float* __restrict__ V,
    int nrows, const int2* __restrict__ vpairs, const float* __restrict__ vU, int nvt) {
  constexpr int PM = Blk<PB>::PM, PL = Blk<PB>::PL;
  __shared__ __align__(16) float lds[3][PM][PL];
  if ((int)blockIdx.x < nsolve) {
    solve_body<PB>(lds[0], lds[1], lds[2], A, A, np, pairs[blockIdx.x],
                   U + (size_t)blockIdx.x * PM * PM, inner_max, full, tol2, rho2);
  } else {
    const int b = blockIdx.x - nsolve, R = b / nvt, rt = b - R * nvt;
    vtile_body<PB>(lds[0], lds[1], V, nrows, np, rt * PM, vpairs[R], vU + (size_t)R * PM * PM);
  }
}

// 16 x 16 tile (ti, tj) of op(X) Y on the matrix cores, K a multiple of 4; X, Y in LDS,
// op(X)[i][k] = X[k][xc + i] if TA else X[i][xc + k], Y[k][j] = Y[k][yc + j].
template <int PL, bool TA>
__device__ __forceinline__ f4 mfma_tile(const float (*X)[PL], int xc, const float (*Y)[PL], int yc,
                                        int K, int ti, int tj) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  f4 c = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const float a = TA ? X[k0 + lk][xc + 16 * ti + li] : X[16 * ti + li][xc + k0 + lk];
    const float b = Y[k0 + lk][yc + 16 * tj + li];
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  return c;
}

// Fused round r >= 2 of a sweep.  The block update of round r - 1 is not launched on its
// own: one launch runs
//   blocks [0, nb2)             the subproblem solves of round r,
//   [nb2, nb2 + na)             the A update of round r - 1 (pair blocks P < R),
//   [nb2 + na, nb2 + na + nb2)  the copy of round r - 1's within-pair blocks,
//   [.., + nvt nb2)             the V update of round r - 1,
// reading Acur and writing Anxt, so that no workgroup reads what another one writes.  Acur
// holds round r - 1's pair blocks after its solves and every other block before round
// r - 1's update.  A solve of round r pairs blocks I, J that round r - 1 had in different
// pairs P (I in half hI) and R (J in half hJ), so it forms its cross block itself as
// U_P(:, hI)^T A_PR U_R(:, hJ) and reads its diagonal blocks as they are; the A update
// leaves the blocks paired in round r to those solves.  apply_only (the last round of a
// sweep): only the A update of round r - 1, for every block, and the copy of its whole
// pair blocks.  pos[X] = 2 * (index of the pair holding block X) + (X is its second block).
template <int PB>
__global__ __launch_bounds__(Blk<PB>::NT) void k_block_fused(
    const float* __restrict__ Acur, float* __restrict__ Anxt, int np, int nb2,
    const int2* __restrict__ pairs_r, const int* __restrict__ pos_r,
    const int2* __restrict__ pairs_p, const int* __restrict__ pos_p,
    const float* __restrict__ Uprev, float* __restrict__ Ucur, int apply_only,
    float* __restrict__ V, int nrows, int nvt) {
  constexpr int PM = Blk<PB>::PM, PL = Blk<PB>::PL, NT = Blk<PB>::NT, TB = PB / 16;
  __shared__ __align__(16) float lds[3][PM][PL];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int ns = apply_only ? 0 : nb2, na = nb2 * (nb2 - 1) / 2;
  int b = blockIdx.x;
  if (b < ns) {
    // ---- solve of round r, pair b = (I, J)
    float(*S)[PL] = lds[0];
    float(*W)[PL] = lds[1];
    float(*Ut)[PL] = lds[2];
    const int2 pr = pairs_r[b];
    const int pi = pos_p[pr.x], pj = pos_p[pr.y];
    const int P = pi >> 1, hI = pi & 1, R = pj >> 1, hJ = pj & 1;
    const int2 PP = pairs_p[P], RR = pairs_p[R];
    const float* UP = Uprev + (size_t)P * PM * PM;
    const float* UR = Uprev + (size_t)R * PM * PM;
    load_pair_block<PB>(W, Acur, np, PP, RR);
    load_factor<PB>(Ut, UR);
    __syncthreads();
    // T = A_PR U_R(:, hJ): PM x PB, one 16 x 16 tile per wave
    const f4 t = mfma_tile<PL, false>(W, 0, Ut, hJ * PB, PM, w / TB, w % TB);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) S[16 * (w / TB) + 4 * (l >> 4) + v][16 * (w % TB) + (l & 15)] = t[v];
    load_factor<PB>(W, UP);
    __syncthreads();
    // X = U_P(:, hI)^T T: PB x PB, tiles on the first TB^2 waves
    f4 x = {0.0f, 0.0f, 0.0f, 0.0f};
    if (w < TB * TB) x = mfma_tile<PL, true>(W, hI * PB, S, 0, PM, w / TB, w % TB);
    __syncthreads();
    if (w < TB * TB) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (w / TB) + 4 * (l >> 4) + v, j = 16 * (w % TB) + (l & 15);
        S[i][PB + j] = x[v];
        S[PB + j][i] = x[v];
      }
    }
    for (int e = tid; e < PB * PB / 4; e += NT) {
      const int i = e / (PB / 4), j = (e % (PB / 4)) * 4;
      *reinterpret_cast<float4*>(&S[i][j]) =
          *reinterpret_cast<const float4*>(Acur + (size_t)(pr.x * PB + i) * np + pr.x * PB + j);
      *reinterpret_cast<float4*>(&S[PB + i][PB + j]) =
          *reinterpret_cast<const float4*>(Acur + (size_t)(pr.y * PB + i) * np + pr.y * PB + j);
    }
    set_identity<PB>(Ut);
    __syncthreads();
    solve_body<PB>(S, W, Ut, Acur, Anxt, np, pr, Ucur + (size_t)b * PM * PM, 1, 0, 0.0f, 0.0f,
                   true);
    return;
  }
  b -= ns;
  if (b < na) {
    // ---- A update of round r - 1 for pair blocks P < R
    float(*Up)[PL] = lds[0];
    float(*Ur)[PL] = lds[1];
    float(*Ab)[PL] = lds[2];
    int P = 0;
    while (b >= nb2 - 1 - P) { b -= nb2 - 1 - P; ++P; }
    const int R = P + 1 + b;
    const int2 PP = pairs_p[P], RR = pairs_p[R];
    load_factor<PB>(Up, Uprev + (size_t)P * PM * PM);
    load_factor<PB>(Ur, Uprev + (size_t)R * PM * PM);
    load_pair_block<PB>(Ab, Acur, np, PP, RR);
    __syncthreads();
    f4 acc[2];
    tile_mfma<PB, true>(Up, Ab, acc);
    __syncthreads();
    tile_store_lds<PB>(Ab, acc);
    __syncthreads();
    tile_mfma<PB, false>(Ab, Ur, acc);
    __syncthreads();
    // the new block by rows in Up and transposed in Ab: both orientations are stored four
    // consecutive columns per lane
    tile_store_lds<PB>(Up, acc);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i, j;
        tile_rc<PB>(u, v, i, j);
        Ab[j][i] = acc[u][v];
      }
    __syncthreads();
    for (int e = tid; e < PM * PM / 4; e += NT) {
      const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
      const int X = i < PB ? PP.x : PP.y, Y = j < PB ? RR.x : RR.y;
      if (!apply_only && (pos_r[X] >> 1) == (pos_r[Y] >> 1)) continue;  // paired in round r
      *reinterpret_cast<float4*>(Anxt + (size_t)blk_row<PB>(PP.x, PP.y, i) * np +
                                 blk_row<PB>(RR.x, RR.y, j)) =
          *reinterpret_cast<const float4*>(&Up[i][j]);
    }
    for (int e = tid; e < PM * PM / 4; e += NT) {
      const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;  // row i of A_RP, columns j..j+3
      const int X = j < PB ? PP.x : PP.y, Y = i < PB ? RR.x : RR.y;
      if (!apply_only && (pos_r[X] >> 1) == (pos_r[Y] >> 1)) continue;
      *reinterpret_cast<float4*>(Anxt + (size_t)blk_row<PB>(RR.x, RR.y, i) * np +
                                 blk_row<PB>(PP.x, PP.y, j)) =
          *reinterpret_cast<const float4*>(&Ab[i][j]);
    }
    return;
  }
  b -= na;
  if (b < nb2) {
    // ---- copy of round r - 1's pair block b: its off-diagonal blocks, or all of it
    const int2 PP = pairs_p[b];
    for (int e = tid; e < PM * PM / 4; e += NT) {
      const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
      if (!apply_only && ((i < PB) == (j < PB))) continue;  // diagonal blocks: the solves'
      const size_t g = (size_t)blk_row<PB>(PP.x, PP.y, i) * np + blk_row<PB>(PP.x, PP.y, j);
      *reinterpret_cast<float4*>(Anxt + g) = *reinterpret_cast<const float4*>(Acur + g);
    }
    return;
  }
  b -= nb2;
  {
    const int R = b / nvt, rt = b - R * nvt;
    vtile_body<PB>(lds[0], lds[1], V, nrows, np, rt * PM, pairs_p[R], Uprev + (size_t)R * PM * PM);
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

// Block rows of the FP32 stage.  32 when one 64 x 64 subproblem is the whole matrix
// (n <= 64) and above n = 2048, where the per-round passes over A and V dominate and fewer
// rounds pay; 16 in between, where the subproblem solves dominate and a 32 x 32 inner round
// is cheaper (measured at n = 1024: 32.8 vs 36.4 ms; at n = 4096: 423 vs 297 ms).
// `request` 16 or 32 overrides the choice (0: automatic).
static int block_rows(int n, int request) {
  if (request == 16 || request == 32) return request;
  return (n <= 64 || n > 2048) ? 32 : 16;
}

template <int PB>
static size_t blocked_bytes(int n) {
  constexpr int PM = Blk<PB>::PM;
  size_t np = (size_t)((n + PM - 1) / PM * PM), nb = np / PB;
  size_t b = np * np * 4 + (size_t)n * np * 4;   // A32, V32
  b += 2 * (nb / 2) * PM * PM * 4;                // U of every block pair of two rounds
  b += (nb - 1 > 0 ? nb - 1 : 1) * (nb / 2) * 8;  // pair table of all rounds
  b += 2 * np * 8 + 256;                          // partial sums + result
  b += np * np * 4 + (nb - 1 > 0 ? nb - 1 : 1) * nb * 4 + 256;  // second A32, block positions
  return (b + 4095) & ~(size_t)4095;
}

size_t precond_f32_bytes(int n) {
  return std::max(blocked_bytes<16>(n), blocked_bytes<32>(n));
}

// Graph replay of the sweeps (`graph` argument) is off by default: on MI355X it measures the
// same as direct launches (n = 1024: 31.9 vs 31.0 ms for the FP32 stage; n = 4096: 274 vs
// 273 ms) -- the cost between dependent launches is on the device, not in the host calls.

template <int PB>
static hipError_t run_blocked(const double* Asym, int n, int ld, double* Q, int ldq,
                              void* scratch, int max_sweeps, double tol, double rho, int* sweeps,
                              bool graphs, hipStream_t s) {
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT;
  const int np = (n + PM - 1) / PM * PM, nb = np / PB, nb2 = nb / 2, rounds = nb - 1;
  char* p = (char*)scratch;
  float* A32 = (float*)p; p += (size_t)np * np * 4;
  float* V32 = (float*)p; p += (size_t)n * np * 4;
  float* U = (float*)p; p += 2 * (size_t)nb2 * PM * PM * 4;
  int2* pairs = (int2*)p; p += (size_t)rounds * nb2 * 8;
  double* part = (double*)p; p += 2 * (size_t)np * 8;
  double* res = (double*)p; p += 256;
  float* A32b = (float*)p; p += (size_t)np * np * 4;
  int* pos = (int*)p;
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
  // pos[r nb + X] = 2 * (pair of round r holding block X) + (X is its second block)
  std::vector<int> ptab((size_t)rounds * nb);
  for (int r = 0; r < rounds; ++r)
    for (int k = 0; k < nb2; ++k) {
      const int2 q = tab[(size_t)r * nb2 + k];
      ptab[(size_t)r * nb + q.x] = 2 * k;
      ptab[(size_t)r * nb + q.y] = 2 * k + 1;
    }
  if ((e = hipMemcpyAsync(pos, ptab.data(), ptab.size() * 4, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return e;
  // the table is host memory read by an asynchronous copy: it must outlive the copy
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  {
    size_t tot = (size_t)np * np;
    hipLaunchKernelGGL(k_to_f32_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Asym,
                       n, ld, A32, np);
    size_t totv = (size_t)n * np;
    hipLaunchKernelGGL(k_identity_f32, dim3((unsigned)((totv + 255) / 256)), dim3(256), 0, s, V32,
                       n, np);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // Acur holds the current A32; fused rounds write the other buffer and swap
  float* Acur = A32;
  float* Anxt = A32b;
  double h[2];
  auto off_norm = [&]() -> hipError_t {
    hipLaunchKernelGGL(k_off_norm_f32, dim3((np + 3) / 4), dim3(256), 0, s, Acur, np, part);
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
  auto round_launch = [&](int nsolve, const int2* pr, float* Uw, int full) {
    const int nv = vround >= 0 ? nvt * nb2 : 0;
    const int2* vp = vround >= 0 ? pairs + (size_t)vround * nb2 : pairs;
    hipLaunchKernelGGL(k_block_round<PB>, dim3(nsolve + nv), dim3(NT), 0, s, Acur, np, pr, Uw,
                       nsolve, inner, full, (float)(tol * tol), (float)(rho * rho), V32, n, vp,
                       ubuf(g - 1), nvt);
  };
  // Rounds 0 and 1 of a sweep are launched as solves + V update, then the A update (round
  // 1's update is deferred); from round 2 on, each round is one fused launch that also
  // carries the previous round's A update, and the sweep ends with that update for its
  // last round.  A sweep swaps the buffers nb - 2 times (even), so every sweep starts from
  // the same buffer.
  const bool fused = nb >= 4;
  const int na = nb2 * (nb2 - 1) / 2;
  auto sweep_launches = [&](hipStream_t st) {
    for (int r = 0; r < rounds; ++r, ++g) {
      const int2* pr = pairs + (size_t)r * nb2;
      const int nv = vround >= 0 ? nvt * nb2 : 0;
      const int2* vp = vround >= 0 ? pairs + (size_t)vround * nb2 : pairs;
      if (!fused || r < 2) {
        hipLaunchKernelGGL(k_block_round<PB>, dim3(nb2 + nv), dim3(NT), 0, st, Acur, np, pr,
                           ubuf(g), nb2, inner, r == 0 ? 1 : 0, (float)(tol * tol),
                           (float)(rho * rho), V32, n, vp, ubuf(g - 1), nvt);
        if (nb2 > 1 && !(fused && r == 1))
          hipLaunchKernelGGL(k_block_apply_a<PB>, dim3(na), dim3(NT), 0, st, Acur, np, pr,
                             ubuf(g), nb2);
      } else {
        hipLaunchKernelGGL(k_block_fused<PB>, dim3(nb2 + na + nb2 + nv), dim3(NT), 0, st, Acur,
                           Anxt, np, nb2, pr, pos + (size_t)r * nb, pairs + (size_t)(r - 1) * nb2,
                           pos + (size_t)(r - 1) * nb, ubuf(g - 1), ubuf(g), 0, V32, n, nvt);
        std::swap(Acur, Anxt);
      }
      vround = r;
    }
    if (fused) {
      // the A update of the sweep's last round (its factors are ubuf(g - 1))
      hipLaunchKernelGGL(k_block_fused<PB>, dim3(na + nb2), dim3(NT), 0, st, Acur, Anxt, np, nb2,
                         pairs, pos, pairs + (size_t)(rounds - 1) * nb2,
                         pos + (size_t)(rounds - 1) * nb, ubuf(g - 1), ubuf(g), 1, V32, n, nvt);
      std::swap(Acur, Anxt);
    }
  };
  // From the second sweep on, a sweep's launches depend only on the parity of its first
  // round (rounds per sweep is odd): each parity's sequence is captured once into a graph
  // (on a private stream) and replayed when graphs are enabled.
  const bool use_graph = graphs && nb2 > 1;
  hipStream_t cs = nullptr;
  hipGraphExec_t ex[2] = {nullptr, nullptr};
  auto cleanup = [&]() {
    for (auto& x : ex) if (x) { (void)hipGraphExecDestroy(x); x = nullptr; }
    if (cs) { (void)hipStreamDestroy(cs); cs = nullptr; }
  };
  int sw = 0;
  while (sw < max_sweeps && off > tol * nrm) {
    if (!use_graph || vround < 0) {
      sweep_launches(s);
    } else {
      const int par = (int)(g & 1);
      if (!ex[par]) {
        if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
          cleanup();
          return e;
        }
        const long long g_save = g;
        const int v_save = vround;
        float* const a_save = Acur;
        float* const b_save = Anxt;
        hipGraph_t gr = nullptr;
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
          cleanup();
          return e;
        }
        sweep_launches(cs);
        e = hipStreamEndCapture(cs, &gr);
        if (e == hipSuccess) e = hipGraphInstantiate(&ex[par], gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (e != hipSuccess) { cleanup(); return e; }
        g = g_save;
        vround = v_save;
        Acur = a_save;
        Anxt = b_save;
      }
      if ((e = hipGraphLaunch(ex[par], s)) != hipSuccess) { cleanup(); return e; }
      g += rounds;
      vround = rounds - 1;
    }
    if ((e = hipGetLastError()) != hipSuccess) { cleanup(); return e; }
    ++sw;
    double prev = off;
    if ((e = off_norm()) != hipSuccess) { cleanup(); return e; }
    off = h[0];
    nrm = h[1];
    if (nb == 2 || off >= rho * prev) break;
  }
  cleanup();
  if (vround >= 0) {
    round_launch(0, pairs, nullptr, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  *sweeps = sw;
  size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(k_gather_q, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V32, n, np,
                     Q, ldq);
  return hipGetLastError();
}

// ------------------------------------------------------------------ batches
// Every matrix of a batch runs the same blocked FP32 Jacobi (blocks of PB = 16 or 32 rows,
// one size per batch) at its own pace: a step performs the next round of every matrix not
// yet done (subproblem solves, then the A and V block updates), and a control kernel
// closes a sweep when a matrix's round counter wraps (off-norm, stop rule).  Blocks of a
// launch are spread over the matrices by prefix sums of their per-matrix block counts.
// 32 by default: a batch is throughput-bound, and 16-row blocks need more sweeps (2048
// matrices, n in [32, 512]: 9.6 against 8.1 sweeps on average, 280-285 against 256-265 ms
// per batch on MI355X).
int precond_f32_block_b(int nmax, int request) {
  if (request == 16 || request == 32) return request;
  (void)nmax;
  return 32;
}

// Workgroup index in the order that keeps consecutive indices on one XCD: the hardware
// hands workgroups to the 8 XCDs round-robin (id mod 8), so XCD x gets the contiguous range
// of indices [x q + min(x, r), + q + (x < r)) of the G = 8 q + r workgroups.  The block
// updates of a step read each subproblem factor from several consecutive workgroups; on one
// XCD they share its L2 instead of fetching the factor once per XCD.
constexpr int kF32Xcds = 8;

__device__ __forceinline__ int xcd_order(int bid, int G) {
  const int x = bid % kF32Xcds, i = bid / kF32Xcds, q = G / kF32Xcds, r = G % kF32Xcds;
  return x * q + min(x, r) + i;
}

__device__ __forceinline__ int find_mat(const int* __restrict__ prefix, int count, int blk) {
  int lo = 0, hi = count - 1;  // largest m with prefix[m] <= blk
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int2 block_pair(int nb, int r, int k) {
  int x, y;
  if (k == 0) { x = nb - 1; y = r; }
  else { x = (r + k) % (nb - 1); y = (r - k + (nb - 1)) % (nb - 1); }
  return int2{min(x, y), max(x, y)};
}

template <int PB>
__device__ __forceinline__ float* ubuf_b(const BMat& b, int par) {
  constexpr int PM = Blk<PB>::PM;
  return b.U + (size_t)par * (b.nb / 2) * PM * PM;
}

// Sums of squares of a PM x PM LDS tile by one workgroup of NT threads (FP64, fixed
// order): the off-diagonal part (weighted) and the diagonal part (diag != 0 only).
template <int PB>
__device__ __forceinline__ void tile_sq(float (*T)[Blk<PB>::PL], bool diag, double w,
                                        double* __restrict__ out) {
  constexpr int PM = Blk<PB>::PM, NT = Blk<PB>::NT;
  __shared__ double red[2][NT / 64];
  double so = 0.0, sd = 0.0;
  for (int e = threadIdx.x; e < PM * PM; e += NT) {
    const int i = e / PM, j = e % PM;
    const double v = T[i][j];
    if (diag && i == j) sd += v * v; else so += v * v;
  }
  so = wave_sum_fast(so);
  sd = wave_sum_fast(sd);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = so; red[1][threadIdx.x >> 6] = sd; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = 0.0, d = 0.0;
    for (int k = 0; k < NT / 64; ++k) { o += red[0][k]; d += red[1][k]; }
    out[0] = w * o;
    out[1] = d;
  }
}

template <int PB>
__global__ __launch_bounds__(Blk<PB>::NT) void k_round_solve_b(
    BMat* __restrict__ mats, const int* __restrict__ act, const int* __restrict__ prefix,
    int count, int max_inner, float tol2, float rho2) {
  constexpr int PM = Blk<PB>::PM, PL = Blk<PB>::PL;
  __shared__ __align__(16) float lds[3][PM][PL];
  const int j = find_mat(prefix, count, blockIdx.x);
  BMat& b = mats[act[j]];
  const int k = blockIdx.x - prefix[j];
  if (b.f_done || k >= b.nb / 2) return;
  const int r = b.f_round;
  const int2 pr = block_pair(b.nb, r, k);
  const int par = (b.f_sweeps * (b.nb - 1) + r) & 1;
  solve_body<PB>(lds[0], lds[1], lds[2], b.A32, b.A32, b.np, pr, ubuf_b<PB>(b, par) + (size_t)k * PM * PM,
                  b.nb == 2 ? max_inner : 1, r == 0 ? 1 : 0, tol2, rho2);
  // the solved block as written back: its upper triangle, mirrored
  for (int e = threadIdx.x; e < PM * PM; e += Blk<PB>::NT) {
    const int i = e / PM, j = e % PM;
    if (i > j) lds[1][i][j] = lds[0][j][i];
    else lds[1][i][j] = lds[0][i][j];
  }
  __syncthreads();
  tile_sq<PB>(lds[1], true, 1.0, b.part + 2 * k);
}

template <int PB>
__global__ __launch_bounds__(Blk<PB>::NT) void k_round_apply_a_b(
    BMat* __restrict__ mats, const int* __restrict__ act, const int* __restrict__ prefix,
    int count) {
  constexpr int PM = Blk<PB>::PM, PL = Blk<PB>::PL, NT = Blk<PB>::NT;
  static_assert(2 * NT * 4 == PM * PM, "two four-float groups of a tile per thread");
  // two LDS tiles (four workgroups per CU): U_R waits in registers until U_P is consumed
  __shared__ __align__(16) float X[PM][PL], Y[PM][PL];
  const int L = xcd_order(blockIdx.x, gridDim.x);
  const int j = find_mat(prefix, count, L);
  BMat& bm = mats[act[j]];
  const int nb2 = bm.nb / 2;
  int bl = L - prefix[j];
  if (bm.f_done || bl >= nb2 * (nb2 - 1) / 2) return;
  int P = 0;
  while (bl >= nb2 - 1 - P) { bl -= nb2 - 1 - P; ++P; }
  const int R = P + 1 + bl;
  const int r = bm.f_round;
  const int2 pp = block_pair(bm.nb, r, P), pr = block_pair(bm.nb, r, R);
  const int par = (bm.f_sweeps * (bm.nb - 1) + r) & 1;
  const float* Ug = ubuf_b<PB>(bm, par) + (size_t)P * PM * PM;
  const float* Uh = ubuf_b<PB>(bm, par) + (size_t)R * PM * PM;
  float* A = bm.A32;
  const int np = bm.np, tid = threadIdx.x;
  // four consecutive columns per lane (they lie in one block: PB is a multiple of 4):
  // X = U_P, Y = A_PR, registers = U_R
  const int i0 = tid / (PM / 4), j0 = (tid % (PM / 4)) * 4, i1 = i0 + NT / (PM / 4);
  const float4 ur0 = *reinterpret_cast<const float4*>(Uh + i0 * PM + j0);
  const float4 ur1 = *reinterpret_cast<const float4*>(Uh + i1 * PM + j0);
  *reinterpret_cast<float4*>(&X[i0][j0]) = *reinterpret_cast<const float4*>(Ug + i0 * PM + j0);
  *reinterpret_cast<float4*>(&X[i1][j0]) = *reinterpret_cast<const float4*>(Ug + i1 * PM + j0);
  *reinterpret_cast<float4*>(&Y[i0][j0]) = *reinterpret_cast<const float4*>(
      A + (size_t)blk_row<PB>(pp.x, pp.y, i0) * np + blk_row<PB>(pr.x, pr.y, j0));
  *reinterpret_cast<float4*>(&Y[i1][j0]) = *reinterpret_cast<const float4*>(
      A + (size_t)blk_row<PB>(pp.x, pp.y, i1) * np + blk_row<PB>(pr.x, pr.y, j0));
  __syncthreads();
  f4 acc[2];
  tile_mfma<PB, true>(X, Y, acc);  // T = U_P^T A_PR
  __syncthreads();
  tile_store_lds<PB>(Y, acc);
  *reinterpret_cast<float4*>(&X[i0][j0]) = ur0;
  *reinterpret_cast<float4*>(&X[i1][j0]) = ur1;
  __syncthreads();
  tile_mfma<PB, false>(Y, X, acc);  // T U_R
  __syncthreads();
  // the new block A_PR by rows in X and transposed (A_RP by rows) in Y, so that both are
  // stored four consecutive columns per lane
  tile_store_lds<PB>(X, acc);
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i, j;
      tile_rc<PB>(u, v, i, j);
      Y[j][i] = acc[u][v];
    }
  __syncthreads();
  for (int e = tid; e < PM * PM / 4; e += NT) {
    const int i = e / (PM / 4), j = (e % (PM / 4)) * 4;
    *reinterpret_cast<float4*>(A + (size_t)blk_row<PB>(pp.x, pp.y, i) * np +
                               blk_row<PB>(pr.x, pr.y, j)) =
        *reinterpret_cast<const float4*>(&X[i][j]);
    *reinterpret_cast<float4*>(A + (size_t)blk_row<PB>(pr.x, pr.y, i) * np +
                               blk_row<PB>(pp.x, pp.y, j)) =
        *reinterpret_cast<const float4*>(&Y[i][j]);
  }
  tile_sq<PB>(X, false, 2.0, bm.part + 2 * (nb2 + L - prefix[j]));
}

template <int PB>
__global__ __launch_bounds__(Blk<PB>::NT) void k_round_apply_v_b(
    BMat* __restrict__ mats, const int* __restrict__ act, const int* __restrict__ prefix,
    int count) {
  constexpr int PM = Blk<PB>::PM, PL = Blk<PB>::PL;
  __shared__ __align__(16) float lds[2][PM][PL];
  const int L = xcd_order(blockIdx.x, gridDim.x);
  const int j = find_mat(prefix, count, L);
  BMat& b = mats[act[j]];
  const int nvt = (b.n + PM - 1) / PM, nb2 = b.nb / 2;
  const int bl = L - prefix[j];
  if (b.f_done || bl >= nvt * nb2) return;
  const int R = bl / nvt, rt = bl - R * nvt;
  const int r = b.f_round;
  const int par = (b.f_sweeps * (b.nb - 1) + r) & 1;
  vtile_body<PB, true>(lds[0], lds[1], b.V32, b.n, b.np, rt * PM, block_pair(b.nb, r, R),
                  ubuf_b<PB>(b, par) + (size_t)R * PM * PM);
}

// off(A32) and ||A32||_F of one matrix by one workgroup (FP64 sums, fixed order).
__device__ __forceinline__ void off_norm_wg(const float* __restrict__ A, int np, double& off,
                                            double& nrm) {
  __shared__ double w[2][4];
  double so = 0.0, sd = 0.0;
  // entries e = threadIdx.x + 256 k in increasing order; (i, j) advanced without division
  // (np <= 8192, so e fits an int)
  int i = (int)threadIdx.x / np, j = (int)threadIdx.x - i * np;
  for (int e = threadIdx.x; e < np * np; e += 256) {
    double v = A[e];
    if (i == j) sd += v * v; else so += v * v;
    j += 256;
    while (j >= np) { j -= np; ++i; }
  }
  so = wave_sum_fast(so);
  sd = wave_sum_fast(sd);
  if ((threadIdx.x & 63) == 0) { w[0][threadIdx.x >> 6] = so; w[1][threadIdx.x >> 6] = sd; }
  __syncthreads();
  const double o = ((w[0][0] + w[0][1]) + w[0][2]) + w[0][3];
  const double d = ((w[1][0] + w[1][1]) + w[1][2]) + w[1][3];
  off = sqrt(o);
  nrm = sqrt(o + d);
}

// Start of a pass: A32 <- fl32(matrix at off) padded, V32 <- I, off-norm, done flags.
__global__ __launch_bounds__(256) void k_f32_start_b(BMat* __restrict__ mats, size_t off,
                                                     double tol) {
  BMat& b = mats[blockIdx.x];
  const double* S = *reinterpret_cast<double* const*>(reinterpret_cast<const char*>(&b) + off);
  const int n = b.n, np = b.np;
  // rows by waves, columns by lanes (np is a multiple of 64)
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int i = wv; i < np; i += 4)
    for (int j = ln; j < np; j += 64)
      b.A32[(size_t)i * np + j] = (i < n && j < n) ? (float)S[(size_t)i * b.ld + j] : 0.0f;
  for (int i = wv; i < n; i += 4)
    for (int j = ln; j < np; j += 64) b.V32[(size_t)i * np + j] = (i == j) ? 1.0f : 0.0f;
  __syncthreads();
  double o, nr;
  off_norm_wg(b.A32, np, o, nr);
  if (threadIdx.x == 0) {
    b.f_round = 0;
    b.f_sweeps = 0;
    b.f_off = o;
    b.f_nrm = nr;
    b.f_done = (o <= tol * nr) ? 1 : 0;
  }
}

// End of a step: advance the round; at the end of a sweep apply the stop rule.
__global__ void k_f32_control_b(BMat* __restrict__ mats, const int* __restrict__ act, int count,
                                int max_sweeps, double tol, double rho) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  BMat& b = mats[act[t]];
  if (b.f_done) return;
  if (b.f_round + 1 < b.nb - 1) {
    b.f_round = b.f_round + 1;
    return;
  }
  // off(A32)^2 and ||A32||_F^2 after the sweep's last round: every block of A was written
  // by that round (diagonal pair blocks by the solves, the others by the A update), each
  // with its sums of squares in a fixed slot, added here in slot order
  const int nb2 = b.nb / 2, np2 = nb2 + nb2 * (nb2 - 1) / 2;
  double so = 0.0, sd = 0.0;
  for (int k = 0; k < np2; ++k) { so += b.part[2 * k]; sd += b.part[2 * k + 1]; }
  const double o = sqrt(so), nr = sqrt(so + sd);
  const double prev = b.f_off;
  b.f_sweeps = b.f_sweeps + 1;
  b.f_pass_sweeps = b.f_pass_sweeps + 1;
  b.f_round = 0;
  b.f_off = o;
  b.f_nrm = nr;
  if (b.nb == 2 || o <= tol * nr || o >= rho * prev || b.f_sweeps >= max_sweeps) b.f_done = 1;
}

__global__ void k_f32_done_b(const BMat* __restrict__ mats, int count, int* __restrict__ done) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) done[i] = mats[i].f_done;
}

__global__ void k_f32_gather_b(BMat* __restrict__ mats, size_t qoff) {
  BMat& b = mats[blockIdx.y];
  double* Q = *reinterpret_cast<double**>(reinterpret_cast<char*>(&b) + qoff);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // n <= 8192: fits an int
  if (idx >= b.n * b.n) return;
  const int i = idx / b.n, j = idx - i * b.n;
  Q[(size_t)i * b.ld + j] = (double)b.V32[(size_t)i * b.np + j];
}

// Bytes of the FP32 stage of one matrix of a batch with blocks of pb rows; its layout:
// A32 (np x np), V32 (n x np), two rounds of subproblem factors, per-block sums.
size_t precond_f32_part_b(int n, int pb) {
  const size_t PM = 2 * (size_t)pb;
  size_t np = ((size_t)n + PM - 1) / PM * PM, nb = np / pb, nb2 = nb / 2;
  size_t b = np * np * 4 + (size_t)n * np * 4 + 2 * nb2 * PM * PM * 4;
  return (b + 255) & ~(size_t)255;
}

size_t precond_f32_bytes_b(int n, int pb) {
  const size_t PM = 2 * (size_t)pb;
  size_t np = ((size_t)n + PM - 1) / PM * PM, nb = np / pb, nb2 = nb / 2;
  size_t b = precond_f32_part_b(n, pb);
  b += (nb2 + nb2 * (nb2 - 1) / 2) * 16;  // per-block sums of squares of a round
  return (b + 255) & ~(size_t)255;
}

hipError_t F32Batch::rebuild() {
  const int PM = 2 * pb;
  int* d_act = dwork + count;
  int* d_ps = dwork + 2 * count;
  int* d_pa = dwork + 3 * count;
  int* d_pv = dwork + 4 * count;
  act.clear(); ps.clear(); pa.clear(); pv.clear();
  tps = tpa = tpv = 0;
  max_rounds = 1;
  for (int i = 0; i < count; ++i) {
    if (done[i]) continue;
    const int np = (nvec[i] + PM - 1) / PM * PM, nb = np / pb, nb2 = nb / 2;
    const int nvt = (nvec[i] + PM - 1) / PM;
    act.push_back(i); ps.push_back(tps); pa.push_back(tpa); pv.push_back(tpv);
    tps += nb2; tpa += nb2 * (nb2 - 1) / 2; tpv += nvt * nb2;
    max_rounds = std::max(max_rounds, nb - 1);
  }
  na = (int)act.size();
  if (na == 0) return hipSuccess;
  hipError_t r;
  if ((r = hipMemcpyAsync(d_act, act.data(), na * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return r;
  if ((r = hipMemcpyAsync(d_ps, ps.data(), na * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return r;
  if ((r = hipMemcpyAsync(d_pa, pa.data(), na * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return r;
  if ((r = hipMemcpyAsync(d_pv, pv.data(), na * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return r;
  return hipStreamSynchronize(s);  // the host vectors are reused by the next rebuild
}

hipError_t F32Batch::poll() {
  hipLaunchKernelGGL(k_f32_done_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count, dwork);
  hipError_t r = hipMemcpyAsync(done.data(), dwork, count * 4, hipMemcpyDeviceToHost, s);
  if (r == hipSuccess) r = hipStreamSynchronize(s);
  return r;
}

void F32Batch::release() {
  if (gx) (void)hipGraphExecDestroy(gx);
  gx = nullptr;
}

hipError_t F32Batch::begin(BMat* m_, const int* nvec_, int count_, int nmax_, int* dwork_,
                           size_t off, size_t qoff_, int max_sweeps_, double tol_, double rho_,
                           hipStream_t s_, bool graph_, hipStream_t cap_, int pb_) {
  release();
  pb = pb_ == 16 ? 16 : 32;
  m = m_; nvec = nvec_; count = count_; nmax = nmax_; dwork = dwork_; qoff = qoff_;
  max_sweeps = max_sweeps_; tol = tol_; rho = rho_; s = s_; graph = graph_ && cap_; cap = cap_;
  step = 0;
  finished = false;
  done.assign(count, 0);
  hipLaunchKernelGGL(k_f32_start_b, dim3(count), dim3(256), 0, s, m, off, tol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = poll()) != hipSuccess) return e;
  if ((e = rebuild()) != hipSuccess) return e;
  live = na;
  // every matrix ends within max_sweeps sweeps of at most max_rounds rounds
  max_steps = (long long)max_sweeps * max_rounds;
  return hipSuccess;
}

// k steps of every listed matrix: subproblem solves, A and V block updates, round control.
template <int PB>
static void round_launches(const F32Batch& f) {
  constexpr int NT = Blk<PB>::NT;
  const int c = f.count;
  hipLaunchKernelGGL(k_round_solve_b<PB>, dim3(f.tps), dim3(NT), 0, f.s, f.m, f.dwork + c,
                     f.dwork + 2 * c, f.na, f.max_sweeps, (float)(f.tol * f.tol),
                     (float)(f.rho * f.rho));
  if (f.tpa > 0)
    hipLaunchKernelGGL(k_round_apply_a_b<PB>, dim3(f.tpa), dim3(NT), 0, f.s, f.m, f.dwork + c,
                       f.dwork + 3 * c, f.na);
  hipLaunchKernelGGL(k_round_apply_v_b<PB>, dim3(f.tpv), dim3(NT), 0, f.s, f.m, f.dwork + c,
                     f.dwork + 4 * c, f.na);
}

hipError_t F32Batch::launch_steps(int k) {
  for (int j = 0; j < k; ++j) {
    if (pb == 16) round_launches<16>(*this);
    else round_launches<32>(*this);
    hipLaunchKernelGGL(k_f32_control_b, dim3((na + 63) / 64), dim3(64), 0, s, m, dwork + count,
                       na, max_sweeps, tol, rho);
  }
  return hipGetLastError();
}

hipError_t F32Batch::advance(int steps) {
  const int poll_every = 8;
  hipError_t e;
  if (graph) {
    // the same steps and polls as below; every matrix is done by max_steps (its sweep
    // limit), so the steps a last replay runs past it change nothing
    for (int k = 0; k < steps && step < max_steps && live > 0; k += poll_every) {
      if (!gx) {
        hipGraph_t g = nullptr;
        if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return e;
        hipStream_t run = s;
        s = cap;
        hipError_t ec = launch_steps(poll_every);
        if (ec == hipSuccess) {
          hipLaunchKernelGGL(k_f32_done_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count,
                             dwork);
          ec = hipGetLastError();
        }
        s = run;
        const hipError_t ee = hipStreamEndCapture(cap, &g);
        if (ec == hipSuccess) ec = ee;
        if (ec == hipSuccess) ec = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (ec != hipSuccess) { gx = nullptr; return ec; }
      }
      if ((e = hipGraphLaunch(gx, s)) != hipSuccess) return e;
      step += poll_every;
      if ((e = hipMemcpyAsync(done.data(), dwork, count * 4, hipMemcpyDeviceToHost, s)) !=
          hipSuccess)
        return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      live = 0;
      for (int i = 0; i < count; ++i) live += done[i] ? 0 : 1;
      // once a quarter of the listed matrices are done, the lists are rebuilt and the
      // graph captured again: blocks of finished matrices would otherwise fill every launch
      if (live > 0 && live * 4 <= na * 3) {
        if ((e = rebuild()) != hipSuccess) return e;
        release();
      }
    }
  } else {
    for (int k = 0; k < steps && step < max_steps && na > 0; ++k, ++step) {
      if ((e = launch_steps(1)) != hipSuccess) return e;
      if ((step + 1) % poll_every == 0) {
        if ((e = poll()) != hipSuccess) return e;
        if ((e = rebuild()) != hipSuccess) return e;
      }
    }
  }
  if (step >= max_steps || (graph ? live : na) == 0) {
    size_t tot = (size_t)nmax * nmax;
    hipLaunchKernelGGL(k_f32_gather_b, dim3((unsigned)((tot + 255) / 256), count), dim3(256), 0,
                       s, m, qoff);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    finished = true;
    release();
  }
  return hipSuccess;
}

hipError_t run_precond_f32_b(BMat* m, const int* nvec, int count, int nmax, int* dwork,
                             size_t off, size_t qoff, int max_sweeps, double tol, double rho,
                             hipStream_t s) {
  F32Batch f;
  hipError_t e = f.begin(m, nvec, count, nmax, dwork, off, qoff, max_sweeps, tol, rho, s);
  while (e == hipSuccess && !f.finished) e = f.advance(1 << 30);
  return e;
}

hipError_t run_precond_f32(const double* Asym, int n, int ld, double* Q, int ldq, void* scratch,
                           int max_sweeps, double tol, double rho, int* sweeps, int block,
                           bool graphs, hipStream_t s) {
  if (block_rows(n, block) == 16)
    return run_blocked<16>(Asym, n, ld, Q, ldq, scratch, max_sweeps, tol, rho, sweeps, graphs,
                           s);
  return run_blocked<32>(Asym, n, ld, Q, ldq, scratch, max_sweeps, tol, rho, sweeps, graphs, s);
}

}  // namespace je
