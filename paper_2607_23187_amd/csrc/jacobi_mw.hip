// FP64 pivoted Jacobi phase (Algorithm 1, greedy or gap-aware pivots of eq. (1)) of one
// large matrix on several workgroups at once.
//
// The arithmetic, the pivot rule, the per-row caches of Sec. 3.2 and the mirrored storage
// of A are those of the one-workgroup kernel (jacobi_kernels.hip); only the reductions are
// spread out.  G workgroups of one wave each own the rows k = T + i G 64 (T = 64 g + lane,
// i < RM).  Every rotation:
//   1. each wave reduces its own candidates (best cached pivot over its rows, best entries
//      of the new rows p and q of the last rotation) and publishes them in a slot of a
//      double-buffered exchange area;
//   2. it arrives at a counter barrier, and when all G have arrived it reads all G slots
//      and reduces them the same way, so every workgroup holds the same winner;
//   3. each workgroup applies the rotation to its own rows (rows p, q of A at its columns,
//      and the mirrored columns p, q of its rows), refreshes its caches and computes its
//      candidates for the next round.
// A full rescan of a stale row is one more exchange round.
//
// Placement and memory ordering: workgroups are dispatched to the XCDs round-robin, so the
// grid is 8 G and only workgroups with blockIdx % 8 == 0 work; they share XCD 0 and its
// L2.  Loads of A and of the exchange area are relaxed agent-scope atomics (they miss the
// per-CU cache and read L2), stores are workgroup-scope (acknowledged by that L2), and a
// wave waits for its stores to be acknowledged before it arrives at a barrier.  A start barrier checks every workgroup's
// XCC id: if they do not share one XCD (or a start wait runs out) the kernel returns
// without touching the state and the host runs the one-workgroup kernel instead.  Every
// wait is bounded; a wait that runs out sets an abort flag that ends all workgroups.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "jacobi_device.h"
#include "kernels.h"

namespace je {

constexpr int kMwStride = 8;            // XCDs: workgroup i runs on XCD i % 8
constexpr int kMwSpinLimit = 1 << 22;   // polls of one wait before it gives up
constexpr int kMwWords = 28;            // words of one workgroup's slot: 6 candidates x 4 + 3 sums

__device__ __forceinline__ double ld_ag(const double* p) {
  const unsigned long long v = __hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}

// Stores need only reach the L2 that every workgroup of the launch shares (they all run on
// one XCD, checked at the start): workgroup-scope stores are acknowledged there, without
// the write-through of device-scope ones (measured 0.81 against 1.08 us per exchange round
// for 16 workgroups).  Readers use agent-scope loads, which miss their own CU's cache.
__device__ __forceinline__ void st_ag(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int ld_ag_i(int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_ag_i(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrival of this workgroup at exchange round `round` (1-based) and the wait for all G.
// False when the wait ran out or another workgroup gave up (the abort flag is then set).
__device__ __forceinline__ bool mw_sync(MwCtl* mc, int G, int round) {
  int ok = 1;
  // this wave's stores (its slot and its part of A) have been acknowledged by L2; the
  // compiler fences keep every memory access of the round on its side of the barrier
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(&mc->counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int target = G * round;
    int spins = 0;
    while (ld_ag_i(&mc->counter) < target) {
      if (++spins > kMwSpinLimit || ld_ag_i(&mc->abort)) {
        st_ag_i(&mc->abort, 1);
        ok = 0;
        break;
      }
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return __builtin_amdgcn_readfirstlane(ok) != 0;
}

// A candidate as four words of a slot: score, value, bound, and (row | flag << 31,
// column) as two 32-bit halves (row and column are non-negative ints).
__device__ __forceinline__ void put_cand(double* w, const Cand& x) {
  st_ag(w + 0, x.s);
  st_ag(w + 1, x.a);
  st_ag(w + 2, x.u);
  const unsigned lo = (unsigned)x.i | ((unsigned)(x.f & 1) << 31);
  const long long pk = (long long)lo | ((long long)(unsigned)x.c << 32);
  st_ag(w + 3, __longlong_as_double(pk));
}

__device__ __forceinline__ Cand get_cand(const double* w) {
  Cand x;
  x.s = ld_ag(w + 0);
  x.a = ld_ag(w + 1);
  x.u = ld_ag(w + 2);
  const unsigned long long pk = (unsigned long long)__double_as_longlong(ld_ag(w + 3));
  const unsigned lo = (unsigned)(pk & 0xffffffffull);
  x.i = (int)(lo & 0x7fffffffu);
  x.f = (int)(lo >> 31);
  x.c = (int)(unsigned)(pk >> 32);
  x.pad = 0;
  return x;
}

template <int RM, bool GAP>
__global__ __launch_bounds__(64) void k_jacobi_mw(JDesc d, long long log_base, MwCtl* mc,
                                                  double* xb, int G) {
  if (blockIdx.x % kMwStride) return;
  const int g = blockIdx.x / kMwStride;
  if (g >= G) return;
  extern __shared__ double s_diag[];
  const int lane = threadIdx.x;
  const int T = g * kWave + lane, GT = G * kWave;
  const int n = d.n;
  const bool use_cert = !GAP && d.stop == STOP_CERT;
  const bool use_off = d.stop == STOP_OFF;
  const int ld = d.ld;
  double* gA = d.A;
  auto ld_a = [&](int r, int c) -> double { return ld_ag(gA + (size_t)r * ld + c); };
  auto st_a = [&](int r, int c, double v) { st_ag(gA + (size_t)r * ld + c, v); };

  // ---- start: every workgroup on one XCD, all of them resident
  int round = 1;
  if (lane == 0) st_ag_i(&mc->xcc[g], __builtin_amdgcn_s_getreg(20 | (3 << 11)) & 0xf);
  if (!mw_sync(mc, G, round)) {
    // not all resident: nothing touched yet, the host falls back
    if (lane == 0) st_ag_i(&mc->misplaced, 1);
    return;
  }
  {
    const int x0 = ld_ag_i(&mc->xcc[0]);
    const int xi = lane < G ? ld_ag_i(&mc->xcc[lane]) : x0;
    if (__ballot(xi != x0)) {
      if (g == 0 && lane == 0) st_ag_i(&mc->misplaced, 1);
      return;
    }
  }

  // ---- per-thread rows k = T + i GT; the whole diagonal in LDS
  double dk[RM], bs[RM], bv[RM], bu[RM], cb[RM], cu[RM], of2[RM];
  int ba[RM], bst[RM], ca[RM], cst[RM], tk[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    int k = T + i * GT;
    if (k < n) {
      dk[i] = d.diag[k]; bs[i] = d.bs[k]; ba[i] = d.ba[k]; bv[i] = d.bv[k]; bst[i] = d.bst[k];
      bu[i] = d.bu[k]; of2[i] = d.off2[k]; tk[i] = d.ts[k];
      if (use_cert) { cb[i] = d.cb[k]; ca[i] = d.ca[k]; cst[i] = d.cst[k]; cu[i] = d.cu[k]; }
      else { cb[i] = -1.0; ca[i] = -1; cst[i] = 0; cu[i] = -1.0; }
    } else {
      dk[i] = 0.0; bs[i] = -1.0; ba[i] = -1; bv[i] = 0.0; bst[i] = 0; bu[i] = -1.0; of2[i] = 0.0;
      tk[i] = 0; cb[i] = -1.0; ca[i] = -1; cst[i] = 0; cu[i] = -1.0;
    }
  }
  for (int l = lane; l < n; l += kWave) s_diag[l] = d.diag[l];
  __syncthreads();

  long long rot = d.ctl->rotations;
  long long rescans = 0;
  int status = ST_OK, done = 0, failed = 0;
  const double thr = d.thr;
  int lp = -1, lq = -1, lrot = 0;
  double lapp = 0.0, laqq = 0.0;
  bool pend = false;
  Cand rp = empty_cand(), rq = rp, cp = rp, cq = rp;
  double op = 0.0, oq = 0.0;
  Cand W = empty_cand(), C = empty_cand();
  double off_tot = 0.0;

  auto diag_of = [&](int x) -> double { return x == lp ? lapp : (x == lq ? laqq : s_diag[x]); };
  auto slot = [&](int b, int wg) -> double* { return xb + (size_t)(b * G + wg) * kMwWords; };
  // optional phase timers of workgroup 0 (10 ns ticks): local reductions, publishing and
  // the store acknowledgements, the barrier wait, reading and reducing the slots, the
  // rotation parameters with the row loads, the update
  const bool prof = d.prof != nullptr && g == 0;
  long long tph[6] = {0, 0, 0, 0, 0, 0}, tmark = 0;
  auto tick = [&]() -> long long { return prof ? (long long)wall_clock64() : 0; };
  auto lap = [&](int k) {
    if (prof) { const long long t = tick(); tph[k] += t - tmark; tmark = t; }
  };

  // Full rescan of row r's selection (which == 0) or certificate (which == 1) cache: each
  // workgroup scans its columns, one exchange round combines them.
  auto rescan = [&](int r, int which) -> bool {
    const double arr = diag_of(r);
    double vals[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int l = T + i * GT;
      vals[i] = (l < n && l != r) ? ld_a(r, l) : 0.0;
    }
    Cand x = empty_cand();
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int l = T + i * GT;
      if (l >= n || l == r) continue;
      double v = vals[i];
      double sc = which == 0 ? sel_score<GAP>(arr, dk[i], v) : gap_score(arr, dk[i], v);
      cand_top2(x, sc, l, v);
    }
    Cand e1 = empty_cand(), e2 = empty_cand();
    wave_best3(e1, 0, x, x.c, e2, 0);
    ++round;
    const int b = round & 1;
    if (lane == 0) put_cand(slot(b, g), x);
    if (!mw_sync(mc, G, round)) return false;
    Cand y = lane < G ? get_cand(slot(b, lane)) : empty_cand();
    Cand f1 = empty_cand(), f2 = empty_cand();
    wave_best3(f1, 0, y, y.c, f2, 0);
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      if (T + i * GT == r) {
        if (which == 0) { bs[i] = y.s; ba[i] = y.c; bv[i] = y.a; bu[i] = y.u; bst[i] = 0; }
        else { cb[i] = y.s; ca[i] = y.c; cu[i] = y.u; cst[i] = 0; }
      }
    }
    ++rescans;
    return true;
  };

  for (;;) {
    tmark = tick();
    // ---- per-thread candidates over own rows
    Cand x1 = empty_cand(), x4 = empty_cand();
    double o7 = 0.0;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int k = T + i * GT;
      if (k >= n) continue;
      if (pend && (k == lp || k == lq)) continue;
      if (bs[i] > x1.s) { x1.s = bs[i]; x1.i = k; x1.c = ba[i]; x1.a = bv[i]; x1.f = bst[i]; }
      if (use_cert && cb[i] > x4.s) { x4.s = cb[i]; x4.i = k; x4.c = ca[i]; x4.f = cst[i]; }
      if (use_off) o7 += of2[i];
    }
    // ---- wave reductions (rp, rq, cp, cq are empty unless a rotation is pending)
    Cand w1 = x1, w2 = rp, w3 = rq, w4 = x4, w5 = cp, w6 = cq;
    wave_best3(w1, x1.i, w2, rp.c, w3, rq.c);
    if (use_cert) wave_best3(w4, x4.i, w5, cp.c, w6, cq.c);
    double s7 = 0.0, s8 = 0.0, s9 = 0.0;
    if (use_off) { s7 = wave_sum_fast(o7); s8 = wave_sum_fast(op); s9 = wave_sum_fast(oq); }
    lap(0);
    // ---- exchange: publish, wait for all, read all
    ++round;
    const int b = round & 1;
    {
      double* my = slot(b, g);
      if (lane == 0) put_cand(my, w1);
      if (lane == 1) put_cand(my + 4, w2);
      if (lane == 2) put_cand(my + 8, w3);
      if (use_cert) {
        if (lane == 3) put_cand(my + 12, w4);
        if (lane == 4) put_cand(my + 16, w5);
        if (lane == 5) put_cand(my + 20, w6);
      }
      if (use_off && lane == 6) { st_ag(my + 24, s7); st_ag(my + 25, s8); st_ag(my + 26, s9); }
    }
    if (prof) { __builtin_amdgcn_s_waitcnt(0); lap(1); }
    if (!mw_sync(mc, G, round)) { failed = 1; break; }
    lap(2);
    {
      const double* sl = slot(b, lane < G ? lane : 0);
      Cand y1 = empty_cand(), y2 = y1, y3 = y1;
      if (lane < G) { y1 = get_cand(sl); y2 = get_cand(sl + 4); y3 = get_cand(sl + 8); }
      wave_best3(y1, y1.i, y2, y2.c, y3, y3.c);
      w1 = y1; w2 = y2; w3 = y3;
      if (use_cert) {
        Cand y4 = empty_cand(), y5 = y4, y6 = y4;
        if (lane < G) { y4 = get_cand(sl + 12); y5 = get_cand(sl + 16); y6 = get_cand(sl + 20); }
        wave_best3(y4, y4.i, y5, y5.c, y6, y6.c);
        w4 = y4; w5 = y5; w6 = y6;
      }
      if (use_off) {
        // fixed order over the workgroups: the same sums in every workgroup
        double a7 = 0.0, a8 = 0.0, a9 = 0.0;
        for (int x = 0; x < G; ++x) {
          const double* sx = slot(b, x);
          a7 += ld_ag(sx + 24); a8 += ld_ag(sx + 25); a9 += ld_ag(sx + 26);
        }
        s7 = a7; s8 = a8; s9 = a9;
      }
    }
    lap(3);
    // ---- fold in the rows of the last rotation
    W = w1;
    C = w4;
    off_tot = s7;
    if (pend) {
      if (better(w2.s, lp, W.s, W.i)) W = Cand{w2.s, w2.a, w2.u, lp, w2.c, 0, 0};
      if (better(w3.s, lq, W.s, W.i)) W = Cand{w3.s, w3.a, w3.u, lq, w3.c, 0, 0};
      if (use_cert) {
        if (better(w5.s, lp, C.s, C.i)) C = Cand{w5.s, 0.0, w5.u, lp, w5.c, 0, 0};
        if (better(w6.s, lq, C.s, C.i)) C = Cand{w6.s, 0.0, w6.u, lq, w6.c, 0, 0};
      }
      off_tot = (s7 + s8) + s9;
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        int k = T + i * GT;
        if (k == lp) {
          bs[i] = w2.s; ba[i] = w2.c; bv[i] = w2.a; bu[i] = w2.u; bst[i] = 0; of2[i] = s8;
          if (use_cert) { cb[i] = w5.s; ca[i] = w5.c; cu[i] = w5.u; cst[i] = 0; }
        } else if (k == lq) {
          bs[i] = w3.s; ba[i] = w3.c; bv[i] = w3.a; bu[i] = w3.u; bst[i] = 0; of2[i] = s9;
          if (use_cert) { cb[i] = w6.s; ca[i] = w6.c; cu[i] = w6.u; cst[i] = 0; }
        }
      }
      if (lane == 0) { s_diag[lp] = lapp; s_diag[lq] = laqq; }
      pend = false;
      rp = empty_cand(); rq = rp; cp = rp; cq = rp;
      op = 0.0; oq = 0.0;
    }
    if (n < 2) { done = 1; break; }
    // ---- the winner must be exact
    if (W.f) {
      if (!rescan(W.i, 0)) { failed = 1; break; }
      continue;
    }
    // ---- stop rules (checked before every rotation)
    if (d.stop == STOP_CERT) {
      if (GAP) {
        if (W.s <= thr) { done = 1; break; }
      } else {
        if (C.s <= thr) { done = 1; break; }
        if (C.f) {
          if (!rescan(C.i, 1)) { failed = 1; break; }
          continue;
        }
      }
    } else if (d.stop == STOP_OFF) {
      if (sqrt(off_tot) <= thr) { done = 1; break; }
    } else {
      if (W.s <= thr) { done = 1; break; }
    }
    if (rot >= d.maxrot) { status = ST_MAXROT; done = 1; break; }
    if (W.a == 0.0) { status = ST_STALL; done = 1; break; }
    if (rot - log_base >= d.log_cap) break;  // log full: drain and resume

    // ---- rotation (p, q): issue the row loads first, the parameters overlap them
    const int p = min(W.i, W.c), q = max(W.i, W.c);
    double xv[RM], yv[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int k = T + i * GT;
      xv[i] = 0.0; yv[i] = 0.0;
      if (k >= n || k == p || k == q) continue;
      xv[i] = ld_a(p, k);
      yv[i] = ld_a(q, k);
    }
    const double apq = W.a;
    const double app = diag_of(p), aqq = diag_of(q);
    double t, c, s;
    rot_params<double>(app, aqq, apq, t, c, s);
    const double napp = app + t * apq;
    const double naqq = aqq - t * apq;
    const int nts = (int)(rot + 1);
    if (prof) { __builtin_amdgcn_s_waitcnt(0); lap(4); }
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int k = T + i * GT;
      if (k >= n) continue;
      if (k == p) {
        st_a(q, p, 0.0);
        st_a(p, q, 0.0);
        dk[i] = napp; tk[i] = nts;
        cand_top2(rq, 0.0, p, 0.0);
        if (use_cert) cand_top2(cq, 0.0, p, 0.0);
        continue;
      }
      if (k == q) {
        dk[i] = naqq; tk[i] = nts;
        cand_top2(rp, 0.0, q, 0.0);
        if (use_cert) cand_top2(cp, 0.0, q, 0.0);
        continue;
      }
      const double x = xv[i], y = yv[i];
      const double xn = c * x + s * y;
      const double yn = c * y - s * x;
      st_a(p, k, xn);
      st_a(q, k, yn);
      st_a(k, p, xn);
      st_a(k, q, yn);
      const double sp = sel_score<GAP>(dk[i], napp, xn);
      const double sq = sel_score<GAP>(dk[i], naqq, yn);
      refresh_entry(bs[i], ba[i], bv[i], bu[i], bst[i], p, q, sp, xn, sq, yn);
      cand_top2(rp, sp, k, xn);
      cand_top2(rq, sq, k, yn);
      if (use_cert) {
        const double lpv = gap_score(dk[i], napp, xn);
        const double lqv = gap_score(dk[i], naqq, yn);
        double dummy = 0.0;
        refresh_entry(cb[i], ca[i], dummy, cu[i], cst[i], p, q, lpv, 0.0, lqv, 0.0);
        cand_top2(cp, lpv, k, 0.0);
        cand_top2(cq, lqv, k, 0.0);
      }
      if (use_off) { op += xn * xn; oq += yn * yn; }
    }
    if (g == 0 && lane == 0) d.log[rot - log_base] = RotEntry{p, q, c, s};
    lap(5);
    lp = p; lq = q; lapp = napp; laqq = naqq; lrot = nts;
    pend = true;
    ++rot;
  }
  if (failed) return;  // the host reports a device error; the state is not resumable

  // ---- write the state back (a later launch may resume from it)
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    int k = T + i * GT;
    if (k < n) {
      d.diag[k] = dk[i]; d.bs[k] = bs[i]; d.ba[k] = ba[i]; d.bv[k] = bv[i]; d.bst[k] = bst[i];
      d.bu[k] = bu[i]; d.off2[k] = of2[i]; d.ts[k] = tk[i];
      if (use_cert) { d.cb[k] = cb[i]; d.ca[k] = ca[i]; d.cst[k] = cst[i]; d.cu[k] = cu[i]; }
    }
  }
  if (prof && lane == 0)
    for (int k = 0; k < 6; ++k) d.prof[k] += tph[k];
  if (g == 0 && lane == 0) {
    JCtl* ctl = d.ctl;
    ctl->rotations = rot;
    ctl->rescans += rescans;
    ctl->status = status;
    ctl->done = done;
    ctl->final_sel = W.s;
    ctl->final_cert = GAP ? W.s : C.s;
    ctl->final_off = sqrt(off_tot);
  }
}

// Workgroups and rows per thread for n: G = min(32, ceil(n / 64)) one-wave workgroups, RM
// rows per thread (1, 2 or 4).
void mw_shape(int n, int* G, int* RM) {
  int g = (n + kWave - 1) / kWave;
  if (g > kMwMaxGroups) g = kMwMaxGroups;
  int rm = (n + g * kWave - 1) / (g * kWave);
  if (rm == 3) rm = 4;
  *G = g;
  *RM = rm;
}

size_t mw_bytes(int n) {
  int G, RM;
  mw_shape(n, &G, &RM);
  return sizeof(MwCtl) + (size_t)2 * G * kMwWords * sizeof(double);
}

template <int RM, bool GAP>
static hipError_t launch_mw_t(const JDesc& d, long long log_base, int G, MwCtl* mc, double* xb,
                              hipStream_t s) {
  const size_t sh = (size_t)d.n * sizeof(double);
  auto fn = k_jacobi_mw<RM, GAP>;
  if (sh > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_zero_words(mc, (int)(sizeof(MwCtl) / 4), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(G * kMwStride), dim3(kWave), sh, s, d, log_base, mc, xb, G);
  return hipGetLastError();
}

hipError_t launch_jacobi_mw(const JDesc& d, long long log_base, void* buf, hipStream_t s) {
  int G, RM;
  mw_shape(d.n, &G, &RM);
  // every row needs an owner thread
  if ((long long)G * kWave * RM < d.n || G > kMwMaxGroups) return hipErrorInvalidValue;
  MwCtl* mc = (MwCtl*)buf;
  double* xb = (double*)((char*)buf + sizeof(MwCtl));
  if (d.pivot == 1) {
    if (RM == 1) return launch_mw_t<1, true>(d, log_base, G, mc, xb, s);
    if (RM == 2) return launch_mw_t<2, true>(d, log_base, G, mc, xb, s);
    return launch_mw_t<4, true>(d, log_base, G, mc, xb, s);
  }
  if (RM == 1) return launch_mw_t<1, false>(d, log_base, G, mc, xb, s);
  if (RM == 2) return launch_mw_t<2, false>(d, log_base, G, mc, xb, s);
  return launch_mw_t<4, false>(d, log_base, G, mc, xb, s);
}

}  // namespace je
