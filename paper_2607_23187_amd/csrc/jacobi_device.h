// Wave-level building blocks of the pivoted Jacobi kernels (one workgroup per matrix and
// the multi-workgroup form): candidates of the argmax, their wave reductions, and the
// per-row cache refresh of Sec. 3.2.  Included by the kernel files only.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace je {

struct Cand {
  double s;  // score (negative: no candidate)
  double a;  // matrix entry at (row, column)
  double u;  // bound of the row's other scores (row-p/q candidates)
  int i;     // row
  int c;     // column
  int f;     // stale flag
  int pad;
};

__device__ __forceinline__ Cand empty_cand() {
  return Cand{-1.0, 0.0, -1.0, 0x7fffffff, 0x7fffffff, 0, 0};
}

__device__ __forceinline__ bool better(double s1, int k1, double s2, int k2) {
  return s1 > s2 || (s1 == s2 && k1 < k2);
}

// Payload of lane w, wave-uniform.  Row and column (< 2^13) and the stale flag travel as
// one packed 32-bit value.
__device__ __forceinline__ Cand read_cand(const Cand& x, int w, bool with_u) {
  if (w < 0) return empty_cand();
  Cand r;
  r.s = readlane_d(x.s, w);
  r.a = readlane_d(x.a, w);
  r.u = with_u ? readlane_d(x.u, w) : -1.0;
  const int pk = readlane_i((x.i & 0x1fff) | ((x.c & 0x1fff) << 13) | (x.f << 26), w);
  r.i = pk & 0x1fff;
  r.c = (pk >> 13) & 0x1fff;
  r.f = pk >> 26;
  r.pad = 0;
  return r;
}

// Wave-uniform argmax of three candidates at once (independent chains interleave).  For b
// and c the result's u bounds every value but the winner's: the winning lane offers its
// second value, the others their best.
// Winner lane of one argmax given its key maximum m (the second half of wave_argmax_lane).
__device__ __forceinline__ int argmax_finish(double score, int key, int k32, int m) {
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

// Three wave_argmax_lane at once: the three key butterflies are interleaved so that the
// DPP wait states of one chain are filled by the others.
__device__ __forceinline__ void wave_argmax_lane3(double sa, int ka, double sb, int kb, double sc,
                                                  int kc, int& la, int& lb, int& lc) {
  const int a = key32(sa), b = key32(sb), c = key32(sc);
  int ma = a, mb = b, mc = c;
  ma = max(ma, dpp_i<0xB1>(ma)); mb = max(mb, dpp_i<0xB1>(mb)); mc = max(mc, dpp_i<0xB1>(mc));
  ma = max(ma, dpp_i<0x4E>(ma)); mb = max(mb, dpp_i<0x4E>(mb)); mc = max(mc, dpp_i<0x4E>(mc));
  ma = max(ma, dpp_i<0x141>(ma)); mb = max(mb, dpp_i<0x141>(mb)); mc = max(mc, dpp_i<0x141>(mc));
  ma = max(ma, dpp_i<0x140>(ma)); mb = max(mb, dpp_i<0x140>(mb)); mc = max(mc, dpp_i<0x140>(mc));
  auto rows = [](int m) {
    const int r0 = __builtin_amdgcn_readlane(m, 0), r1 = __builtin_amdgcn_readlane(m, 16);
    const int r2 = __builtin_amdgcn_readlane(m, 32), r3 = __builtin_amdgcn_readlane(m, 48);
    return max(max(r0, r1), max(r2, r3));
  };
  const int Ma = rows(ma), Mb = rows(mb), Mc = rows(mc);
  la = argmax_finish(sa, ka, a, Ma);
  lb = argmax_finish(sb, kb, b, Mb);
  lc = argmax_finish(sc, kc, c, Mc);
}

__device__ __forceinline__ void wave_best3(Cand& a, int ka, Cand& b, int kb, Cand& c, int kc) {
  int la, lb, lc;
  wave_argmax_lane3(a.s, ka, b.s, kb, c.s, kc, la, lb, lc);
  const int lane = lane_id();
  // bounds of b and c (wave_max_ub of each, the two butterflies interleaved)
  int mb = key32(lane == lb ? b.u : b.s), mc = key32(lane == lc ? c.u : c.s);
  mb = max(mb, dpp_i<0xB1>(mb)); mc = max(mc, dpp_i<0xB1>(mc));
  mb = max(mb, dpp_i<0x4E>(mb)); mc = max(mc, dpp_i<0x4E>(mc));
  mb = max(mb, dpp_i<0x141>(mb)); mc = max(mc, dpp_i<0x141>(mc));
  mb = max(mb, dpp_i<0x140>(mb)); mc = max(mc, dpp_i<0x140>(mc));
  auto ub_of = [](int m) {
    const int r = max(max(__builtin_amdgcn_readlane(m, 0), __builtin_amdgcn_readlane(m, 16)),
                      max(__builtin_amdgcn_readlane(m, 32), __builtin_amdgcn_readlane(m, 48)));
    return key_ub(r);
  };
  const double ub = ub_of(mb), uc = ub_of(mc);
  a = read_cand(a, la, false);
  b = read_cand(b, lb, false);
  c = read_cand(c, lc, false);
  b.u = ub;
  c.u = uc;
}

// Refresh of one row's cache after rotation (p, q) changed its entries at columns p and q
// to scores sp, sq (matrix values xp, xq).  Fresh row: bs/ba/bv is its exact best and bu
// bounds its other scores.  Stale row: bs bounds all its scores.  Straight-line code: all
// cases are evaluated and selected.
__device__ __forceinline__ void refresh_entry(double& bs, int& ba, double& bv, double& bu,
                                              int& bst, int p, int q, double sp, double xp,
                                              double sq, double xq) {
  const bool hit = (ba == p) || (ba == q);
  if (__builtin_expect(bst || hit, 0)) {
    // stale row (bs bounds all its scores) or fresh row whose best column moved (bu bounds
    // the others): exact again when the larger new score is strictly above that bound
    const bool qb = sq > sp;
    const double v = qb ? sq : sp, a = qb ? xq : xp, o = qb ? sp : sq;
    const int col = qb ? q : p;
    const double bound = bst ? bs : bu;
    const bool up = v > bound;
    bs = up ? v : bound;
    bv = up ? a : bv;
    bu = up ? fmax(bound, o) : bu;
    ba = up ? col : ba;
    bst = up ? 0 : 1;
  } else {
    // fresh row, best column untouched: insert (sp, p) then (sq, q)
    const bool b1 = better(sp, p, bs, ba);
    const double bs1 = b1 ? sp : bs, bv1 = b1 ? xp : bv, bu1 = fmax(bu, b1 ? bs : sp);
    const int ba1 = b1 ? p : ba;
    const bool b2 = better(sq, q, bs1, ba1);
    bs = b2 ? sq : bs1;
    bv = b2 ? xq : bv1;
    bu = fmax(bu1, b2 ? bs1 : sq);
    ba = b2 ? q : ba1;
  }
}

// Per-thread top two of the new row p (or q): best (score, column, value), second value.
__device__ __forceinline__ void cand_top2(Cand& x, double v, int col, double a) {
  if (better(v, col, x.s, x.c)) { x.u = fmax(x.u, x.s); x.s = v; x.c = col; x.a = a; }
  else x.u = fmax(x.u, v);
}

}  // namespace je
