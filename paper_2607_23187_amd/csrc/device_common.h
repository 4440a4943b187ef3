// Device-side building blocks of the gfx950 Jacobi eigensolver: the pivot scores, the
// rotation parameters and wave64 reductions.  Compiled with -ffp-contract=off: every
// floating-point expression below is evaluated as written, one IEEE operation at a time
// (double sqrt and division are correctly rounded on gfx950), so the pivot sequence is
// a function of the input bits alone.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace je {

constexpr int kWave = 64;

// Gap-aware pivot score, eq. (1):
//   L_ij = 2 a_ij^2 / (|a_ii - a_jj| + sqrt(|a_ii - a_jj|^2 + 4 a_ij^2)).
// It equals the shift of the eigenvalues of the 2x2 block [[a_ii, a_ij], [a_ij, a_jj]]
// away from its diagonal (the Li-Li bound, tight for 2x2, Sec. 3).  Defined as 0 when
// a_ij^2 is 0 in FP64 (the formula is 0/0 when also a_ii == a_jj).
__device__ __forceinline__ double gap_score(double aii, double ajj, double aij) {
  double a2 = aij * aij;
  if (a2 == 0.0) return 0.0;
  double d = fabs(aii - ajj);
  return (2.0 * a2) / (d + sqrt(d * d + 4.0 * a2));
}

// Selection score: greedy (classical) uses |a_ij|, gap uses eq. (1).
template <bool GAP>
__device__ __forceinline__ double sel_score(double aii, double ajj, double aij) {
  if constexpr (GAP) return gap_score(aii, ajj, aij);
  else return fabs(aij);
}

// Rotation G = [[c, -s], [s, c]] with G^T [[app, apq], [apq, aqq]] G diagonal (Sec. 2):
// t = tan of the rotation angle is the root of t^2 + 2 theta t - 1 = 0 of modulus <= 1,
// theta = (app - aqq) / (2 apq), sgn(0) = +1; t = 1/(2 theta) once |theta| > 2^500.
// Afterwards app' = app + t apq and aqq' = aqq - t apq.
template <typename T>
__device__ __forceinline__ void rot_params(T app, T aqq, T apq, T& t, T& c, T& s);

template <>
__device__ __forceinline__ void rot_params<double>(double app, double aqq, double apq, double& t,
                                                   double& c, double& s) {
  double theta = (app - aqq) / (2.0 * apq);
  double tt;
  if (fabs(theta) > 0x1p500) {
    tt = 1.0 / (2.0 * theta);
  } else {
    tt = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
    if (theta < 0.0) tt = -tt;
  }
  c = 1.0 / sqrt(1.0 + tt * tt);
  s = tt * c;
  t = tt;
}

template <>
__device__ __forceinline__ void rot_params<float>(float app, float aqq, float apq, float& t,
                                                  float& c, float& s) {
  float theta = (app - aqq) / (2.0f * apq);
  float tt;
  if (fabsf(theta) > 0x1p60f) {
    tt = 1.0f / (2.0f * theta);
  } else {
    tt = 1.0f / (fabsf(theta) + sqrtf(1.0f + theta * theta));
    if (theta < 0.0f) tt = -tt;
  }
  c = 1.0f / sqrtf(1.0f + tt * tt);
  s = tt * c;
  t = tt;
}

// ------------------------------------------------------------------ wave64 helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int readlane_i(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// DPP move of a double (two 32-bit halves) within rows of 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wave-uniform maximum: butterfly inside each row of 16 lanes on the DPP network
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror), then the
// four row results through v_readlane.
__device__ __forceinline__ double wave_max_fast(double m) {
  m = fmax(m, dpp_d<0xB1>(m));
  m = fmax(m, dpp_d<0x4E>(m));
  m = fmax(m, dpp_d<0x141>(m));
  m = fmax(m, dpp_d<0x140>(m));
  double r0 = readlane_d(m, 0), r1 = readlane_d(m, 16), r2 = readlane_d(m, 32),
         r3 = readlane_d(m, 48);
  return fmax(fmax(r0, r1), fmax(r2, r3));
}

// Lane holding the largest score, the smallest key among equal scores.  Keys of lanes
// holding a candidate are distinct; lanes with nothing to offer pass a negative score.
// The result is wave-uniform; -1 when no lane has a candidate.
__device__ __forceinline__ int wave_argmax_lane(double score, int key) {
  double m = wave_max_fast(score);
  if (m < 0.0) return -1;
  unsigned long long b = __ballot(score == m);
  if (__popcll(b) == 1) return __ffsll((long long)b) - 1;
  int k = wave_min_i(score == m ? key : 0x7fffffff);
  b = __ballot(score == m && key == k);
  return __ffsll((long long)b) - 1;
}

}  // namespace je
