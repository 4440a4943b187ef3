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
// t = s / c is the root of modulus <= 1 of t^2 + 2 theta t - 1 = 0 with
// theta = (app - aqq) / (2 apq), evaluated as
//   t = sgn(delta) 2 apq / (|delta| + sqrt(delta^2 + 4 apq^2)),  delta = app - aqq,
// sgn(0) = +1 (one division fewer than going through theta).  t depends only on the ratio
// delta : apq, so when both are tiny or huge they are scaled by the same power of two
// first (exact).  c = 1/sqrt(1 + t^2), s = t c; the new diagonal entries are app + t apq
// and aqq - t apq.
template <typename T>
__device__ __forceinline__ void rot_params(T app, T aqq, T apq, T& t, T& c, T& s);

template <>
__device__ __forceinline__ void rot_params<double>(double app, double aqq, double apq, double& t,
                                                   double& c, double& s) {
  double d = app - aqq, a = apq;
  double m = fmax(fabs(d), fabs(a));
  if (m < 0x1p-400 || m > 0x1p400) {
    int e;
    (void)frexp(m, &e);
    d = ldexp(d, -e);
    a = ldexp(a, -e);
  }
  double den = fabs(d) + sqrt(d * d + 4.0 * (a * a));
  double tt = (2.0 * a) / den;
  if (d < 0.0) tt = -tt;
  c = 1.0 / sqrt(1.0 + tt * tt);
  s = tt * c;
  t = tt;
}

template <>
__device__ __forceinline__ void rot_params<float>(float app, float aqq, float apq, float& t,
                                                  float& c, float& s) {
  float d = app - aqq, a = apq;
  float m = fmaxf(fabsf(d), fabsf(a));
  if (m < 0x1p-50f || m > 0x1p50f) {
    int e;
    (void)frexpf(m, &e);
    d = ldexpf(d, -e);
    a = ldexpf(a, -e);
  }
  float den = fabsf(d) + sqrtf(d * d + 4.0f * (a * a));
  float tt = (2.0f * a) / den;
  if (d < 0.0f) tt = -tt;
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

// (bound_ctrl set: the patterns used here never leave the row, and in this form the move
// folds into the consuming VALU instruction as a DPP operand)
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}

// Monotone 32-bit key of a score: the bits of its float rounding (non-decreasing in the
// score for scores >= 0), -1 for "no candidate".
__device__ __forceinline__ int key32(double s) { return s >= 0.0 ? __float_as_int((float)s) : -1; }

// Wave-uniform maximum of 32-bit keys: butterfly inside each row of 16 lanes on the DPP
// network (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror; each a
// single v_max_i32 with a DPP operand), then the four row results on the scalar unit.
__device__ __forceinline__ int wave_max_i(int m) {
  m = max(m, dpp_i<0xB1>(m));
  m = max(m, dpp_i<0x4E>(m));
  m = max(m, dpp_i<0x141>(m));
  m = max(m, dpp_i<0x140>(m));
  int r0 = __builtin_amdgcn_readlane(m, 0), r1 = __builtin_amdgcn_readlane(m, 16);
  int r2 = __builtin_amdgcn_readlane(m, 32), r3 = __builtin_amdgcn_readlane(m, 48);
  return max(max(r0, r1), max(r2, r3));
}

// Lane holding the largest score, the smallest key among equal scores (keys of lanes with
// a candidate are distinct); -1 when no lane has a candidate (negative scores).  The float
// keys find the lanes that can hold the maximum; equal float keys are settled exactly in
// FP64 on the scalar path.  The result is wave-uniform.
__device__ __forceinline__ int wave_argmax_lane(double score, int key) {
  const int k32 = key32(score);
  const int m = wave_max_i(k32);
  if (m < 0) return -1;
  unsigned long long b = __ballot(k32 == m);
  int w = __ffsll((long long)b) - 1;
  b &= b - 1;
  if (b) {
    double bs = readlane_d(score, w);
    int bk = __builtin_amdgcn_readlane(key, w);
    while (b) {
      int l = __ffsll((long long)b) - 1;
      b &= b - 1;
      double x = readlane_d(score, l);
      int kx = __builtin_amdgcn_readlane(key, l);
      if (x > bs || (x == bs && kx < bk)) { bs = x; bk = kx; w = l; }
    }
  }
  return w;
}

// Upper bound of every score whose key32 is <= m: the next float above the float key (the
// conversion rounds to nearest, so the float is within half an ulp of the score, in the
// normal and the subnormal range alike); +inf stays +inf; -1 when m is "no candidate".
__device__ __forceinline__ double key_ub(int m) {
  if (m < 0) return -1.0;
  return m >= 0x7f800000 ? (double)__int_as_float(0x7f800000) : (double)__int_as_float(m + 1);
}

// Wave-uniform upper bound of max(v); -1 when every lane passes a negative value.
__device__ __forceinline__ double wave_max_ub(double v) {
  return key_ub(wave_max_i(key32(v)));
}

// Wave-uniform maximum of doubles (exact).
__device__ __forceinline__ double wave_max_fast(double m) {
  m = fmax(m, dpp_d<0xB1>(m));
  m = fmax(m, dpp_d<0x4E>(m));
  m = fmax(m, dpp_d<0x141>(m));
  m = fmax(m, dpp_d<0x140>(m));
  double r0 = readlane_d(m, 0), r1 = readlane_d(m, 16), r2 = readlane_d(m, 32),
         r3 = readlane_d(m, 48);
  return fmax(fmax(r0, r1), fmax(r2, r3));
}

// Wave-uniform sum of doubles (butterfly in rows, then the four row sums in order).
__device__ __forceinline__ double wave_sum_fast(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  double r0 = readlane_d(v, 0), r1 = readlane_d(v, 16), r2 = readlane_d(v, 32),
         r3 = readlane_d(v, 48);
  return ((r0 + r1) + r2) + r3;
}

}  // namespace je
