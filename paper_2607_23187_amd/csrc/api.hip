// Host side of the C ABI declared in include/jacobi.h: argument checking, the per-device
// workspace pool and the order of the phases of one solve:
//   1. symmetric FP64 copy of the upper triangle, finiteness check, ||A||_F
//   2. (FP32 preconditioner) blocked parallel FP32 Jacobi -> V_l, FP64 Newton-Schulz -> Q;
//      a refinement pass repeats this on fl32(Q^T A Q); A_hat = Q^T (A Q) on the matrix
//      cores, symmetrised                                                       (Sec. 2.1)
//   3. initial per-row scores, persistent pivoted Jacobi (greedy or eq. (1)), stop rule of
//      Theorem 1 (or off-norm / raw score); the rotation log is drained into V = Q G_1 G_2...
//   4. one Newton-Schulz polish of V, eigenvalues sorted ascending, V permuted to match.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/jacobi.h"
#include "kernels.h"

using namespace je;

namespace {

std::mutex g_mu;

struct Pool {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::vector<Pool> g_pools;

void* pool_get(size_t bytes, int* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { *err = JE_ERR_DEVICE; return nullptr; }
  if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1);
  Pool& p = g_pools[dev];
  if (p.bytes < bytes) {
    if (p.ptr) { (void)hipDeviceSynchronize(); (void)hipFree(p.ptr); p.ptr = nullptr; p.bytes = 0; }
    if (hipMalloc(&p.ptr, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *err = JE_ERR_NOMEM;
      return nullptr;
    }
    p.bytes = bytes;
  }
  return p.ptr;
}

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
inline int ld_of(int n) { return (n + 7) & ~7; }

long long log_cap_for(int n, long long maxrot) {
  long long cap = 1ll << 22;
  return std::max<long long>(1, std::min(cap, maxrot));
}

long long default_maxrot(int n) { return 40ll * n * n + 64; }

// FP32 sweep stop rules.  The first pass works on fl32(A), whose rounding puts a floor of
// about u_32 ||A||_F under off(A32): stop at 2^-22 ||A||_F or when a sweep stops helping.
// A refinement pass works on a nearly diagonal fl32(Q^T A Q) whose off-diagonal entries FP32
// holds with full relative precision; it sweeps until a sweep no longer halves off(A32).
constexpr double kF32Tol1 = 0x1p-22, kF32Rho1 = 1.0;
constexpr double kF32Tol1Refined = 0x1p-18;
// Stop tolerance of the first FP32 pass: its FP32 floor when it is the only pass; looser
// when a refinement pass follows, which starts from fl32(Q^T A Q) (off ~ u_32 ||A|| however
// far the first pass went), so the first pass's last sweeps below that level buy nothing.
static double f32_tol1(int passes) { return passes <= 1 ? kF32Tol1 : kF32Tol1Refined; }
constexpr double kF32Rho2 = 0.5;
// Refinement pass: sweeps until a sweep fails to halve off, or off <= 2^-30 ||A||_F (below
// that the remaining off-diagonal mass is the FP32-level coupling inside clusters that the
// pass skips, and the sweep that would show the stall is saved).
constexpr double kF32Tol2 = 0x1p-30;

// Smallest n whose FP64 Jacobi phase runs on several workgroups by default (MI355X, per
// rotation, one workgroup against several: n = 512 3.77 / 4.10 us, 1024 5.02 / 4.29,
// 2048 7.23 / 4.77, 4096 11.52 / 5.37; the two cross near n = 670).
constexpr int kMultiWgMinN = 768;

// Range of the entries solved as given: outside it the input is scaled by a power of two
// (exact) so that squares in FP64 and the FP32 copy of the preconditioner stay in range.
constexpr double kRangeLo = 0x1p-60, kRangeHi = 0x1p60;

// Exponent e with 2^e maxabs in [1/2, 1) when maxabs is outside the range, else 0.
int range_exp(double maxabs) {
  if (!(maxabs > 0.0) || (maxabs >= kRangeLo && maxabs <= kRangeHi)) return 0;
  int e = 0;
  (void)std::frexp(maxabs, &e);
  return -e;
}

// Workspace carving for one problem of size n.
struct WS {
  double *Asym, *A, *Q, *X, *T, *R, *Vw;
  double *diag, *bs, *bv, *cb, *off2, *rowsq, *scal, *bu, *cu;
  int *ba, *bst, *ca, *cst, *ts, *rank, *flag;
  long long* prof;
  JCtl* ctl;
  RotEntry* log;
  void* f32;
  void* mw;       // control block and exchange area of the multi-workgroup Jacobi kernel
  void* split;    // slice planes of the split-precision contraction (opts.split_gemm)
  long long log_cap;
};

size_t ws_bytes(int n, int precond, long long log_cap, int split = 0) {
  size_t ld = ld_of(n);
  size_t mat = al((size_t)n * ld * 8);
  size_t b = 0;
  b += mat;                       // Asym (also the Jacobi matrix without preconditioner)
  b += mat;                       // Vw
  if (precond) b += 5 * mat;      // A, Q, X, T, R
  else b += 2 * mat;              // X, R (polish)
  b += 8 * al((size_t)n * 8);     // diag bs bv cb off2 rowsq bu cu
  b += al(64);                    // scalars
  b += 7 * al((size_t)n * 4);     // ba bst ca cst ts rank flag
  b += al(sizeof(JCtl));
  b += al(64);                    // phase timers
  b += al((size_t)log_cap * sizeof(RotEntry));
  if (precond) b += al(precond_f32_bytes(n));
  b += al(mw_bytes(n));
  if (precond && split) b += al(gemm_split_bytes(n));
  return b;
}

WS ws_carve(void* base, int n, int precond, long long log_cap, int split = 0) {
  WS w{};
  char* p = (char*)base;
  size_t ld = ld_of(n);
  size_t mat = al((size_t)n * ld * 8);
  auto take = [&](size_t b) { char* r = p; p += al(b); return (void*)r; };
  w.Asym = (double*)take(mat);
  w.Vw = (double*)take(mat);
  if (precond) {
    w.A = (double*)take(mat);
    w.Q = (double*)take(mat);
    w.X = (double*)take(mat);
    w.T = (double*)take(mat);
    w.R = (double*)take(mat);
  } else {
    w.A = w.Asym;
    w.Q = nullptr;
    w.X = (double*)take(mat);
    w.R = (double*)take(mat);
    w.T = nullptr;
  }
  w.diag = (double*)take((size_t)n * 8);
  w.bs = (double*)take((size_t)n * 8);
  w.bv = (double*)take((size_t)n * 8);
  w.cb = (double*)take((size_t)n * 8);
  w.off2 = (double*)take((size_t)n * 8);
  w.rowsq = (double*)take((size_t)n * 8);
  w.bu = (double*)take((size_t)n * 8);
  w.cu = (double*)take((size_t)n * 8);
  w.scal = (double*)take(64);
  w.ba = (int*)take((size_t)n * 4);
  w.bst = (int*)take((size_t)n * 4);
  w.ca = (int*)take((size_t)n * 4);
  w.cst = (int*)take((size_t)n * 4);
  w.ts = (int*)take((size_t)n * 4);
  w.rank = (int*)take((size_t)n * 4);
  w.flag = (int*)take((size_t)n * 4);
  w.ctl = (JCtl*)take(sizeof(JCtl));
  w.prof = (long long*)take(64);
  w.log = (RotEntry*)take((size_t)log_cap * sizeof(RotEntry));
  w.f32 = precond ? take(precond_f32_bytes(n)) : nullptr;
  w.mw = take(mw_bytes(n));
  w.split = (precond && split) ? take(gemm_split_bytes(n)) : nullptr;
  w.log_cap = log_cap;
  return w;
}

#define HIPCHK(x)                       \
  do {                                  \
    if ((x) != hipSuccess) {            \
      (void)hipGetLastError();          \
      return JE_ERR_DEVICE;             \
    }                                   \
  } while (0)

// Elapsed time on a stream between construction and stop() (HIP events).  Timers are
// switched off per thread for the entry point that must not create runtime objects.
thread_local bool t_timers_off = false;

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  bool ok;
  explicit Timer(hipStream_t st) : s(st) {
    ok = !t_timers_off && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    if (ok) (void)hipEventRecord(a, s);
  }
  float stop() {
    float ms = 0.f;
    if (!ok) return 0.f;
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
  }
  ~Timer() {
    if (ok) { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  }
};

// One Newton-Schulz step toward the nearest orthogonal matrix, as a small correction:
// R = I - X^T X, X <- X + X R / 2.  Returns ||R||_F (before the step) through `rnorm`.
int ns_step(double*& X, double*& Xalt, double* R, int n, int ld, double* part, double* scal,
            double* rnorm, hipStream_t s) {
  HIPCHK(launch_dgemm_sym(n, -1.0, X, ld, X, ld, R, ld, s));
  HIPCHK(launch_add_identity(R, n, ld, 1.0, s));
  if (rnorm) {
    HIPCHK(launch_fro2(R, n, ld, part, scal, s));
    HIPCHK(hipMemcpyAsync(rnorm, scal, 8, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(launch_dgemm(n, 0, 0.5, X, ld, R, ld, 1.0, X, ld, Xalt, ld, s));
  std::swap(X, Xalt);
  return JE_OK;
}

// Newton-Schulz is done once a step starts from ||I - X^T X||_F <= 4 n u, or from a
// residual r whose square is below n u / 2: a step leaves about (3/4) r^2 plus rounding, so
// the step that would only confirm convergence is skipped.
bool ns_converged(double rn, int n) {
  const double nu = n * 0x1p-53;
  return rn <= 4.0 * nu || rn * rn <= 0.5 * nu;
}

// Newton-Schulz steps on X until converged (at most 6); X may be swapped with Xalt.
int orthonormalize(double*& X, double*& Xalt, double* R, int n, int ld, double* part,
                   double* scal, hipStream_t s) {
  for (int itn = 0; itn < 6; ++itn) {
    double rn = 0.0;
    int r = ns_step(X, Xalt, R, n, ld, part, scal, &rn, s);
    if (r) return r;
    HIPCHK(hipStreamSynchronize(s));
    if (ns_converged(rn, n)) break;
  }
  return JE_OK;
}

// The preconditioner of Sec. 2.1 for the symmetric Asym (row-major, ld): an FP32 spectral
// decomposition of fl32(Asym) re-orthogonalised by Newton-Schulz into X; with
// o.fp32_passes = 2 the FP32 Jacobi runs again on fl32(X^T Asym X) and X <- X V_2,
// re-orthogonalised.  X and Xo may be swapped; R, T, A are n x ld temporaries.
int precond_q(const double* Asym, int n, int ld, double*& X, double*& Xo, double* R, double* T,
              double* A, void* f32, const je_opts& o, double* part, double* scal, int* sweeps,
              hipStream_t s, bool refine_floor = true) {
  int sw = 0;
  *sweeps = 0;
  HIPCHK(run_precond_f32(Asym, n, ld, X, ld, f32, o.fp32_max_sweeps, f32_tol1(o.fp32_passes),
                         kF32Rho1, &sw, o.fp32_block, o.graph != 0, s));
  *sweeps += sw;
  int r = orthonormalize(X, Xo, R, n, ld, part, scal, s);
  if (r) return r;
  for (int pass = 1; pass < o.fp32_passes; ++pass) {
    HIPCHK(launch_dgemm(n, 0, 1.0, Asym, ld, X, ld, 0.0, nullptr, 0, T, ld, s));
    HIPCHK(launch_dgemm_sym(n, 1.0, X, ld, T, ld, A, ld, s));
    HIPCHK(run_precond_f32(A, n, ld, T, ld, f32, o.fp32_max_sweeps,
                           refine_floor ? kF32Tol2 : 0.0, kF32Rho2, &sw, o.fp32_block,
                           o.graph != 0, s));
    *sweeps += sw;
    HIPCHK(launch_dgemm(n, 0, 1.0, X, ld, T, ld, 0.0, nullptr, 0, Xo, ld, s));
    std::swap(X, Xo);
    r = orthonormalize(X, Xo, R, n, ld, part, scal, s);
    if (r) return r;
  }
  return JE_OK;
}

// One solve in the workspace at `base` (ws_bytes(n, precond, cap) bytes, device memory).
int solve_one(const double* Au, int n, int lda, double* W, double* V, int ldv, double tol,
              int pivot, int precond, const je_opts& o, je_stats* st, hipStream_t s,
              void* base, long long cap) {
  const long long maxrot = o.max_rotations > 0 ? o.max_rotations : default_maxrot(n);
  WS w = ws_carve(base, n, precond, cap, o.split_gemm);
  const int ld = ld_of(n);
  je_stats S{};

  // ---- 1. symmetric copy, finiteness, range, ||A||_F
  Timer tp(s);
  HIPCHK(launch_zero_words(w.flag, 1, s));
  HIPCHK(launch_symcopy(Au, n, lda, w.Asym, ld, w.diag, nullptr, w.flag, s));
  HIPCHK(launch_maxabs(w.Asym, n, ld, w.rowsq, w.scal + 4, s));
  int flag = 0;
  double maxabs = 0.0;
  HIPCHK(hipMemcpyAsync(&flag, w.flag, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&maxabs, w.scal + 4, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (flag) return JE_ERR_NONFINITE;
  // out-of-range input: solved as 2^e A (exact), eigenvalues scaled back
  const int e_scale = range_exp(maxabs);
  if (e_scale) HIPCHK(launch_scale(w.Asym, n, ld, w.diag, e_scale, s));
  S.scale_exp = e_scale;
  double normF = 0.0;
  HIPCHK(launch_fro2(w.Asym, n, ld, w.rowsq, w.scal, s));
  HIPCHK(hipMemcpyAsync(&normF, w.scal, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!std::isfinite(normF)) return JE_ERR_NONFINITE;
  // thresholds and reported norms refer to the caller's A; the solve runs on 2^e A
  const double unscale = std::ldexp(1.0, -e_scale);
  S.normF = normF * unscale;
  double thr;
  if (o.abs_thr > 0.0) thr = std::ldexp(o.abs_thr, e_scale);
  else if (o.stop == JE_STOP_CERT) thr = tol * normF / (2.0 * n * (double)(n - 1));
  else thr = tol * normF;
  S.thr = thr * unscale;

  // ---- 2. preconditioner
  double* Ajac = w.Asym;
  double* Vw = w.Vw;
  if (precond) {
    double* X = w.Q;
    double* Xo = w.X;
    int r = precond_q(w.Asym, n, ld, X, Xo, w.R, w.T, w.A, w.f32, o, w.rowsq, w.scal,
                      &S.sweeps32, s);
    if (r) return r;
    S.ms_precond = tp.stop();
    Timer tg(s);
    // A_hat = X^T (A X): T = A X, A_hat = X^T T, exactly symmetric (the FP64 product forms
    // the upper half and mirrors it; the split product forms all of it, then symmetrised)
    if (o.split_gemm) {
      HIPCHK(launch_gemm_split(n, 0, w.Asym, ld, X, ld, w.T, ld, w.split, s));
      HIPCHK(launch_gemm_split(n, 1, X, ld, w.T, ld, w.A, ld, w.split, s));
      HIPCHK(launch_symmetrize(w.A, n, ld, s));
    } else {
      HIPCHK(launch_dgemm(n, 0, 1.0, w.Asym, ld, X, ld, 0.0, nullptr, 0, w.T, ld, s));
      HIPCHK(launch_dgemm_sym(n, 1.0, X, ld, w.T, ld, w.A, ld, s));
    }
    HIPCHK(hipMemcpyAsync(Vw, X, (size_t)n * ld * 8, hipMemcpyDeviceToDevice, s));
    Ajac = w.A;
    S.ms_gemm = tg.stop();
    HIPCHK(launch_offnorm(w.A, n, ld, w.rowsq, w.scal + 2, s));
    HIPCHK(hipMemcpyAsync(&S.a_hat_off, w.scal + 2, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!std::isfinite(S.a_hat_off)) return JE_ERR_NONFINITE;
    S.a_hat_off *= unscale;
  } else {
    HIPCHK(launch_set_identity(Vw, n, ld, s));
    S.ms_precond = tp.stop();
  }

  // ---- 3. pivoted Jacobi
  Timer tj(s);
  JDesc d{};
  d.A = Ajac; d.n = n; d.ld = ld;
  d.diag = w.diag; d.bs = w.bs; d.ba = w.ba; d.bv = w.bv; d.bst = w.bst;
  d.cb = w.cb; d.ca = w.ca; d.cst = w.cst; d.off2 = w.off2; d.ts = w.ts;
  d.bu = w.bu; d.cu = w.cu;
  d.log = w.log; d.log_cap = cap; d.ctl = w.ctl;
  d.thr = thr; d.maxrot = maxrot; d.pivot = pivot; d.stop = o.stop;
  if (precond) HIPCHK(launch_get_diag(Ajac, n, ld, w.diag, s));
  HIPCHK(launch_zero_words(w.ctl, sizeof(JCtl) / 4, s));
  // opts.profile: per-phase timers of the Jacobi kernel
  const bool profile = o.profile != 0;
  if (profile) {
    HIPCHK(launch_zero_words(w.prof, 16, s));
    d.prof = w.prof;
  }
  HIPCHK(launch_init_rows(d, s));
  const bool lds = jacobi_fits_lds(n);
  const bool mirror = o.update_mode != 2;  // one problem: mirror mode unless asked otherwise
  // several workgroups for large HBM-resident problems (mirror mode, no phase timers)
  bool multi = !lds && mirror &&
               (o.jacobi_wgs == 2 || (o.jacobi_wgs == 0 && n >= kMultiWgMinN));
  long long base_rot = 0;
  JCtl hc{};
  float ms_apply = 0.f;
  float ms_kernel = 0.f;
  for (;;) {
    Timer tk(s);
    if (multi) HIPCHK(launch_jacobi_mw(d, base_rot, w.mw, s));
    else HIPCHK(launch_jacobi(d, base_rot, lds, mirror, s));
    ms_kernel += tk.stop();
    HIPCHK(hipMemcpyAsync(&hc, w.ctl, sizeof(JCtl), hipMemcpyDeviceToHost, s));
    MwCtl mc{};
    if (multi) HIPCHK(hipMemcpyAsync(&mc, w.mw, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (multi && mc.misplaced) {
      // the workgroups were not all resident on one XCD: the state is untouched, the
      // one-workgroup kernel takes over
      multi = false;
      continue;
    }
    if (multi && mc.abort) return JE_ERR_DEVICE;
    long long m = hc.rotations - base_rot;
    if (o.pivot_log && base_rot < o.pivot_log_cap) {
      long long mm = std::min(m, o.pivot_log_cap - base_rot);
      HIPCHK(launch_copy_pivots(w.log, mm, o.pivot_log + 2 * base_rot, s));
    }
    Timer ta(s);
    HIPCHK(launch_apply_log(Vw, n, ld, w.log, m, s));
    ms_apply += ta.stop();
    base_rot = hc.rotations;
    if (hc.done) break;
  }
  S.ms_jacobi = tj.stop() - ms_apply;
  if (profile) {
    // the timers tick at 100 MHz (10 ns)
    long long pr[8];
    HIPCHK(hipMemcpy(pr, w.prof, 64, hipMemcpyDeviceToHost));
    const double r = (double)std::max<long long>(1, hc.rotations);
    for (int k = 0; k < 6; ++k) S.prof_ns[k] = pr[k] * 10.0 / r;
  }
  S.ms_jacobi_kernel = ms_kernel;
  S.ms_apply_log = ms_apply;
  int rows_per_thread = 0;
  if (multi) mw_shape(n, &S.jacobi_wgs, &rows_per_thread);
  else S.jacobi_wgs = 1;
  S.rotations = hc.rotations;
  S.rescans = hc.rescans;
  S.final_max_score = hc.final_cert * unscale;
  S.final_off = hc.final_off * unscale;
  S.status = hc.status == ST_MAXROT ? JE_WARN_MAXROT : (hc.status == ST_STALL ? JE_WARN_STALL : JE_OK);

  // ---- 4. polish, sort, output
  Timer tf(s);
  if (V && o.polish_v) {
    double* X = Vw;
    double* Xalt = w.X;
    int r = ns_step(X, Xalt, w.R, n, ld, w.rowsq, w.scal, nullptr, s);
    if (r) return r;
    Vw = X;
  }
  HIPCHK(launch_sort_output(w.diag, n, Vw, ld, W, V, ldv, w.rank, o.sort, -e_scale, s));
  HIPCHK(hipStreamSynchronize(s));
  S.ms_finalize = tf.stop() + ms_apply;
  if (st) *st = S;
  return S.status;
}

// ------------------------------------------------------------------ batches
// All problems of a batch (n >= 2) go through the same sequence of launches; every launch
// covers the whole batch (grids sized for the largest n, blocks past a matrix's n exit).
// The FP32 stage runs each matrix at its own pace; the FP64 Jacobi phase is one persistent
// launch per workgroup shape (LDS-resident n <= 64, HBM-resident above), each workgroup
// taking the next matrix, largest first, from a device counter.  Logs are drained for all
// matrices between launches; unfinished matrices are relaunched.
constexpr long long kBatchLogCap = 1ll << 16;

// Tuned workgroup shapes of the batched Jacobi phase, per (class, pivot, size bucket).
// opts.tune = 0 keeps the default shapes (one wave LDS-resident, 512 threads otherwise).
std::mutex g_tune_mu;
std::map<int, int> g_tune;

struct BatchLayout {
  size_t bytes = 0;
  std::vector<size_t> off;  // per member: offset of its workspace
};

// ------------------------------------------------------------------ one-sided SVD
// Stop threshold: greedy and gap scores, Theorem 1 on A = B^T B; relative score, the same
// form with ||A||_F replaced by 1 (the score is scale-free).
double svd_thr(int pivot, double tol, int n, double normF) {
  if (n < 2) return 0.0;
  const double den = 2.0 * n * (double)(n - 1);
  return pivot == JE_PIVOT_RELATIVE ? tol / den : tol * normF / den;
}

int svd_one(const double* B, int m, int n, int ldb, double* S, double* U, int ldu, double* V,
            int ldv, double tol, int pivot, int precond, const je_opts& o, je_stats* st,
            hipStream_t s) {
  const long long maxrot = o.max_rotations > 0 ? o.max_rotations : default_maxrot(n);
  const size_t ld = ld_of(n);  // row stride of B (row-major), G, V^T and the preconditioner
  const bool pre = precond && n > 1;
  const size_t ym = al((size_t)m * ld * 8), mat = al((size_t)n * ld * 8);
  size_t bytes = 2 * ym + 2 * mat + 5 * al((size_t)n * 8) + 3 * al((size_t)n * 4) + al(64) +
                 al(sizeof(JCtl));
  if (pre) bytes += 5 * mat + al(precond_f32_bytes(n));
  int err = JE_OK;
  char* p = (char*)pool_get(bytes, &err);
  if (!p) return err;
  auto take = [&](size_t b) { char* r = p; p += al(b); return (void*)r; };
  double* Y = (double*)take(ym);
  double* Y2 = (double*)take(ym);
  double* G = (double*)take(mat);
  double* Vt = (double*)take(mat);
  double* best = (double*)take((size_t)n * 8);
  double* part = (double*)take((size_t)n * 8);
  double* diag = (double*)take((size_t)n * 8);
  double* rowp = (double*)take((size_t)n * 8);
  double* rowq = (double*)take((size_t)n * 8);
  int* arg = (int*)take((size_t)n * 4);
  int* rank = (int*)take((size_t)n * 4);
  int* flag = (int*)take((size_t)n * 4);
  double* scal = (double*)take(64);
  JCtl* ctl = (JCtl*)take(sizeof(JCtl));
  double *Q = nullptr, *Qo = nullptr, *R = nullptr, *T = nullptr, *A = nullptr;
  void* f32 = nullptr;
  if (pre) {
    Q = (double*)take(mat);
    Qo = (double*)take(mat);
    R = (double*)take(mat);
    T = (double*)take(mat);
    A = (double*)take(mat);
    f32 = take(precond_f32_bytes(n));
  }
  je_stats Sx{};

  // ---- 1. B row-major, finiteness, A = B^T B, ||A||_F
  Timer tp(s);
  HIPCHK(hipMemsetAsync(flag, 0, 4, s));
  HIPCHK(launch_svd_load(B, m, n, ldb, Y, (int)ld, flag, s));
  HIPCHK(launch_svd_gram(Y, (int)ld, m, n, G, (int)ld, s));
  HIPCHK(launch_fro2(G, n, (int)ld, part, scal, s));
  int hflag = 0;
  double normF = 0.0;
  HIPCHK(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&normF, scal, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hflag || !std::isfinite(normF)) return JE_ERR_NONFINITE;
  Sx.normF = normF;
  const double thr = o.abs_thr > 0.0 ? o.abs_thr : svd_thr(pivot, tol, n, normF);
  Sx.thr = thr;

  // ---- 2. preconditioner: right singular vectors of B from the FP32 decomposition of
  // fl32(B^T B), re-orthogonalised -> Q; the one-sided method runs on B Q
  double* Vr = V ? Vt : nullptr;
  if (pre) {
    // no off-norm floor in the refinement: the Gram matrix of a graded B has eigenvalues
    // far below 2^-30 ||B^T B||, whose vectors the longer refinement resolves (1024 x 512,
    // singular values over 4 decades: 3456 vs 7973 one-sided rotations)
    int r = precond_q(G, n, (int)ld, Q, Qo, R, T, A, f32, o, part, scal, &Sx.sweeps32, s, false);
    if (r) return r;
    Sx.ms_precond = tp.stop();
    Timer tg(s);
    HIPCHK(launch_svd_rowmix(Y, (int)ld, Q, (int)ld, m, n, Y2, (int)ld, s));
    std::swap(Y, Y2);
    if (Vr) HIPCHK(launch_svd_transpose(Q, (int)ld, n, Vr, (int)ld, s));
    HIPCHK(launch_svd_gram(Y, (int)ld, m, n, G, (int)ld, s));
    HIPCHK(launch_offnorm(G, n, (int)ld, part, scal + 2, s));
    HIPCHK(hipMemcpyAsync(&Sx.a_hat_off, scal + 2, 8, hipMemcpyDeviceToHost, s));
    Sx.ms_gemm = tg.stop();
  } else {
    if (Vr) HIPCHK(launch_set_identity(Vr, n, (int)ld, s));
    Sx.ms_precond = tp.stop();
  }

  // ---- 3. one-sided pivoted Jacobi
  Timer tj(s);
  SDesc d{};
  d.Y = Y; d.m = m; d.ldy = (int)ld;
  d.Vt = Vr; d.ldv = (int)ld;
  d.G = G; d.n = n; d.ldg = (int)ld;
  d.best = best; d.arg = arg; d.diag = diag; d.rowp = rowp; d.rowq = rowq;
  d.thr = thr; d.maxrot = maxrot; d.pivot = pivot;
  d.plog = o.pivot_log; d.logcap = o.pivot_log ? o.pivot_log_cap : 0;
  d.ctl = ctl;
  HIPCHK(hipMemsetAsync(ctl, 0, sizeof(JCtl), s));
  HIPCHK(launch_svd_jacobi(d, s));
  JCtl hc{};
  HIPCHK(hipMemcpyAsync(&hc, ctl, sizeof(JCtl), hipMemcpyDeviceToHost, s));
  Sx.ms_jacobi = tj.stop();
  Sx.ms_jacobi_kernel = Sx.ms_jacobi;
  Sx.rotations = hc.rotations;
  Sx.rescans = hc.rescans;
  Sx.final_max_score = hc.final_sel;
  Sx.status = hc.status == ST_MAXROT ? JE_WARN_MAXROT : (hc.status == ST_STALL ? JE_WARN_STALL : JE_OK);

  // ---- 4. singular values (descending), vectors
  Timer tf(s);
  HIPCHK(launch_offnorm(G, n, (int)ld, part, scal + 3, s));
  HIPCHK(hipMemcpyAsync(&Sx.final_off, scal + 3, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(launch_svd_out(Y, (int)ld, m, G, (int)ld, Vr, (int)ld, n, rank, S, U, ldu, V, ldv, s));
  HIPCHK(hipStreamSynchronize(s));
  Sx.ms_finalize = tf.stop();
  if (st) *st = Sx;
  return Sx.status;
}

int check_svd_args(const double* B, int m, int n, int ldb, const double* S, const double* U,
                   int ldu, const double* V, int ldv, double tol, int pivot, int precond,
                   const je_opts& o) {
  if (!B && n > 0) return -1;
  if (m < 0 || m < n) return -2;
  if (n < 0) return -3;
  if (ldb < std::max(1, m)) return -4;
  if (!S && n > 0) return -5;
  if (U && ldu < std::max(1, m)) return -7;
  if (V && ldv < std::max(1, n)) return -9;
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    if (!(o.abs_thr > 0.0)) return -10;
  }
  if (pivot != JE_PIVOT_GREEDY && pivot != JE_PIVOT_GAP && pivot != JE_PIVOT_RELATIVE)
    return -11;
  if (precond != JE_PRECOND_NONE && precond != JE_PRECOND_FP32) return -12;
  if (o.fp32_max_sweeps < 0 || o.fp32_passes < 1 || o.fp32_passes > 2) return -13;
  if (o.pivot_log && o.pivot_log_cap < 0) return -13;
  return 0;
}


size_t bws_bytes(int n, int precond, long long cap) {
  size_t ld = ld_of(n);
  size_t mat = al((size_t)n * ld * 8);
  size_t b = 7 * mat + 8 * al((size_t)n * 8) + al(64) + 7 * al((size_t)n * 4) +
             al(sizeof(JCtl)) + al((size_t)cap * sizeof(RotEntry));
  // the FP32 stage's state for either block size (a cohort picks one for all members)
  if (precond) b += al(std::max(precond_f32_bytes_b(n, 16), precond_f32_bytes_b(n, 32)));
  return b;
}

void bws_carve(char* p, BMat& b, int n, int precond, long long cap, int pb) {
  const size_t ld = ld_of(n);
  const size_t mat = al((size_t)n * ld * 8);
  auto take = [&](size_t bytes) { char* r = p; p += al(bytes); return (void*)r; };
  b.ld = (int)ld;
  b.Asym = (double*)take(mat); b.A = (double*)take(mat); b.Vw = (double*)take(mat);
  b.X = (double*)take(mat); b.Xb = (double*)take(mat); b.T = (double*)take(mat);
  b.R = (double*)take(mat);
  b.diag = (double*)take((size_t)n * 8); b.rowsq = (double*)take((size_t)n * 8);
  JDesc& d = b.jd;
  d.bs = (double*)take((size_t)n * 8); d.bv = (double*)take((size_t)n * 8);
  d.cb = (double*)take((size_t)n * 8); d.off2 = (double*)take((size_t)n * 8);
  d.bu = (double*)take((size_t)n * 8); d.cu = (double*)take((size_t)n * 8);
  b.scal = (double*)take(64);
  d.ba = (int*)take((size_t)n * 4); d.bst = (int*)take((size_t)n * 4);
  d.ca = (int*)take((size_t)n * 4); d.cst = (int*)take((size_t)n * 4);
  d.ts = (int*)take((size_t)n * 4);
  b.rank = (int*)take((size_t)n * 4); b.flag = (int*)take((size_t)n * 4);
  d.ctl = (JCtl*)take(sizeof(JCtl));
  d.log = (RotEntry*)take((size_t)cap * sizeof(RotEntry));
  d.log_cap = cap;
  if (precond) {
    const int PM = 2 * pb;
    const int np = (n + PM - 1) / PM * PM;
    char* f = (char*)take(std::max(precond_f32_bytes_b(n, 16), precond_f32_bytes_b(n, 32)));
    b.np = np;
    b.nb = np / pb;
    b.A32 = (float*)f;
    b.V32 = b.A32 + (size_t)np * np;
    b.U = b.V32 + (size_t)n * np;
    b.part = (double*)(f + precond_f32_part_b(n, pb));
  }
}

#define BF(f) BM_FIELD(f)

// Device bytes of a cohort's tables for `cnt` members (beside the members' workspaces).
size_t cohort_meta_bytes(int cnt) {
  return 2 * al((size_t)cnt * sizeof(BMat)) + 8 * al((size_t)cnt * 4 + 4) + al(64) +
         al((size_t)cnt * sizeof(BInfo));
}

// Device bytes a batch of these sizes needs (workspaces + tables).
size_t batch_bytes(const std::vector<int>& sizes, int precond) {
  size_t tot = 0;
  for (int nn : sizes) tot += bws_bytes(nn, precond, kBatchLogCap);
  return tot + cohort_meta_bytes((int)sizes.size());
}

// The launches `body` makes on stream s, captured into an executable graph (no memset or
// copy nodes: buffers are cleared by kernels).
template <class F>
hipError_t capture_graph(hipStream_t s, hipGraphExec_t* gx, F body) {
  hipGraph_t g = nullptr;
  *gx = nullptr;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t ec = body();
  const hipError_t ee = hipStreamEndCapture(s, &g);
  if (ec == hipSuccess) ec = ee;
  if (ec == hipSuccess) ec = hipGraphInstantiate(gx, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (ec != hipSuccess) *gx = nullptr;
  return ec;
}

inline void drop_graph(hipGraphExec_t& gx) {
  if (gx) (void)hipGraphExecDestroy(gx);
  gx = nullptr;
}

// Members whose FP64 Jacobi phase runs LDS-resident in a batch.  A single problem keeps A in
// LDS up to n = 128 (jacobi_fits_lds); a batch only up to n = 64: an LDS-resident launch
// sizes its LDS for its largest member, and at n = 128 (134 KB) one workgroup per CU is
// resident, so the class (64, 128] runs faster HBM-resident with several workgroups per CU
// (2048 matrices, n in [32, 512]: persistent launches 45 against 50 ms per batch).
constexpr int kBatchLdsMaxN = 64;
inline bool batch_lds(int n) { return n <= kBatchLdsMaxN && jacobi_fits_lds(n); }

// Workgroups of a persistent batched launch: one per member up to 2048 one-wave (LDS) or
// 128-thread workgroups, up to 1024 larger ones (four per CU).
inline int queue_grid(bool lds, int threads, size_t members) {
  return (int)std::min<size_t>(members, (lds || threads <= 128) ? 2048 : 1024);
}

// One problem of a cohort: the caller's arrays, its workspace, and the caller's index.
struct Member {
  const double* A;
  int n, lda;
  double* W;
  double* V;
  int ldv;
  char* ws;     // bws_bytes(n, precond, kBatchLogCap) bytes of device memory
  int idx;      // index of the problem in the caller's arrays (or request slot)
};

// A set of problems solved together in bounded steps (the batched method of the library):
// begin() checks and scales the inputs, every step() advances the whole cohort by one
// bounded piece of work (a few FP32 rounds, one Newton-Schulz step, one persistent FP64
// Jacobi launch of at most `step_rot` rotations per member, ...).  Members whose FP64 phase
// has ended are finalised (polish, sort, output) at the end of the step that ended it and
// leave the cohort; their results are appended to `left`.  Every member gives the same
// bits whatever its cohort: all launches act on each member independently, in the same
// order of operations.
struct Cohort {
  enum Phase { SETUP, F32A, NS1, REFINE, F32B, NS2, CONTRACT, JACOBI, DONE };
  struct Left {
    int idx;         // Member::idx
    int status;
    je_stats st;
  };

  // configuration
  double tol = 0.0;
  int pivot = 1, precond = 1;
  je_opts o{};
  hipStream_t s = nullptr;
  long long step_rot = kBatchLogCap;
  // members (arrays compacted when members leave)
  std::vector<Member> mem;
  std::vector<BMat> hm;
  std::vector<BInfo> hi;
  std::vector<double> nrm;
  std::vector<int> nv;
  int cnt = 0, nmax = 0;
  // device tables
  char* meta = nullptr;
  BMat *dm = nullptr, *dfin = nullptr;
  int *d_idx_lds = nullptr, *d_idx_hbm = nullptr, *d_work = nullptr, *d_cnt = nullptr;
  BInfo* d_info = nullptr;
  // progress
  Phase phase = SETUP;
  int ns_iter = 0, pass = 0;
  size_t offX = BF(X), offXb = BF(Xb);
  F32Batch f32;
  int f32_pb = 32;  // block rows of the FP32 stage (one size for the cohort)
  bool mirror = false;
  int shape_lds = 64, shape_hbm = 512;
  je_stats S{};
  float ms_kernel = 0.f, ms_apply = 0.f;
  std::vector<Left> left;
  // graph replay (opts.graph): a Newton-Schulz step (one graph per buffer parity), the
  // persistent FP64 launches and the log drain of a step, captured for the current
  // membership (gen counts the changes of membership) and replayed until it changes
  int gen = 0, graph_gen = -1;
  hipGraphExec_t g_ns[2] = {nullptr, nullptr}, g_jq = nullptr, g_ja = nullptr;
  // graphs are captured on a stream of their own (the caller's may be the null stream,
  // which cannot be captured) and launched on the caller's
  hipStream_t cap = nullptr;

  Cohort() = default;
  Cohort(const Cohort&) = delete;
  Cohort& operator=(const Cohort&) = delete;
  ~Cohort() {
    drop_graphs();
    f32.release();
    if (cap) (void)hipStreamDestroy(cap);
  }
  int capture_stream() {
    if (!cap) HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    return JE_OK;
  }
  // the launches `body` makes (on the member stream s) captured into *gx
  template <class F>
  int capture(hipGraphExec_t* gx, F body) {
    if (int r = capture_stream()) return r;
    hipStream_t run = s;
    s = cap;
    const hipError_t e = capture_graph(cap, gx, body);
    s = run;
    HIPCHK(e);
    return JE_OK;
  }
  void drop_graphs() {
    drop_graph(g_ns[0]); drop_graph(g_ns[1]); drop_graph(g_jq); drop_graph(g_ja);
  }
  // graphs of an older membership are dropped
  void graphs_current() {
    if (graph_gen != gen) { drop_graphs(); graph_gen = gen; }
  }

  int collect() {
    HIPCHK(launch_collect_b(dm, cnt, d_info, s));
    HIPCHK(hipMemcpyAsync(hi.data(), d_info, (size_t)cnt * sizeof(BInfo), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    return JE_OK;
  }
  int upload() {
    HIPCHK(hipMemcpyAsync(dm, hm.data(), (size_t)cnt * sizeof(BMat), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return JE_OK;
  }
  int download() {
    HIPCHK(hipMemcpyAsync(hm.data(), dm, (size_t)cnt * sizeof(BMat), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return JE_OK;
  }
  void refresh_sizes() {
    nmax = 0;
    nv.resize(cnt);
    for (int i = 0; i < cnt; ++i) {
      nv[i] = hm[i].n;
      nmax = std::max(nmax, hm[i].n);
    }
  }
  // Keep the members with keep[i] != 0 (device state downloaded first, tables re-uploaded).
  int compact(const std::vector<char>& keep) {
    if (int r = download()) return r;
    std::vector<Member> m2;
    std::vector<BMat> h2;
    std::vector<BInfo> i2;
    std::vector<double> n2;
    for (int i = 0; i < cnt; ++i)
      if (keep[i]) {
        m2.push_back(mem[i]); h2.push_back(hm[i]); i2.push_back(hi[i]);
        n2.push_back(nrm.empty() ? 0.0 : nrm[i]);
      }
    mem.swap(m2); hm.swap(h2); hi.swap(i2);
    if (!nrm.empty()) nrm.swap(n2);
    cnt = (int)mem.size();
    ++gen;
    refresh_sizes();
    if (cnt == 0) { phase = DONE; return JE_OK; }
    return upload();
  }
  void leave(int i, int status, const je_stats* st) {
    Left l;
    l.idx = mem[i].idx;
    l.status = status;
    if (st) l.st = *st;
    else { std::memset(&l.st, 0, sizeof(l.st)); l.st.status = status; }
    left.push_back(l);
  }

  // members: workspaces already assigned; meta: cohort_meta_bytes(members.size()) bytes
  int begin(std::vector<Member> members, char* meta_, double tol_, int pivot_, int precond_,
            const je_opts& o_, hipStream_t s_, long long step_rot_) {
    mem = std::move(members);
    cnt = (int)mem.size();
    tol = tol_; pivot = pivot_; precond = precond_; o = o_; s = s_; step_rot = step_rot_;
    meta = meta_;
    char* mp = meta;
    dm = (BMat*)mp; mp += al((size_t)cnt * sizeof(BMat));
    dfin = (BMat*)mp; mp += al((size_t)cnt * sizeof(BMat));
    d_idx_lds = (int*)mp; mp += al((size_t)cnt * 4 + 4);
    d_idx_hbm = (int*)mp; mp += al((size_t)cnt * 4 + 4);
    d_work = (int*)mp; mp += 5 * al((size_t)cnt * 4 + 4);  // FP32 stage launch lists
    d_cnt = (int*)mp; mp += al(64);                        // queue counters
    d_info = (BInfo*)mp;
    hi.assign(cnt, BInfo{});
    hm.assign(cnt, BMat{});
    int nbig = 0;
    for (const Member& m : mem) nbig = std::max(nbig, m.n);
    f32_pb = precond_f32_block_b(nbig, o.fp32_block);
    for (int i = 0; i < cnt; ++i) {
      BMat& x = hm[i];
      std::memset(&x, 0, sizeof(x));
      x.Au = mem[i].A; x.n = mem[i].n; x.lda = mem[i].lda;
      x.Wout = mem[i].W; x.Vout = mem[i].V; x.ldv = mem[i].ldv;
      bws_carve(mem[i].ws, x, mem[i].n, precond, kBatchLogCap, f32_pb);
    }
    refresh_sizes();
    if (int r = upload()) return r;
    Timer tp(s);
    // ---- symmetric copies, finiteness, range, ||A||_F
    HIPCHK(launch_reset_b(dm, cnt, s));
    HIPCHK(launch_symcopy_b(dm, cnt, nmax, s));
    HIPCHK(launch_maxabs_b(dm, cnt, nmax, BF(Asym), 4, s));
    if (int r = collect()) return r;
    // out-of-range members are solved as 2^e A (exact), their eigenvalues scaled back
    {
      bool any = false;
      for (int i = 0; i < cnt; ++i) {
        hm[i].a_exp = hi[i].nonfinite ? 0 : range_exp(hi[i].maxabs);
        any = any || hm[i].a_exp != 0;
      }
      if (any) {
        if (int r = upload()) return r;
        HIPCHK(launch_scale_b(dm, cnt, nmax, BF(Asym), s));
      }
    }
    HIPCHK(launch_fro2_b(dm, cnt, nmax, BF(Asym), 0, s));
    if (int r = collect()) return r;
    // members with a non-finite entry leave here (outputs untouched, as for one problem)
    {
      std::vector<char> keep(cnt, 1);
      bool drop = false;
      for (int i = 0; i < cnt; ++i)
        if (hi[i].nonfinite || !std::isfinite(hi[i].normF)) {
          leave(i, JE_ERR_NONFINITE, nullptr);
          keep[i] = 0;
          drop = true;
        }
      if (drop) {
        if (int r = compact(keep)) return r;
        if (cnt == 0) return JE_OK;
      }
    }
    nrm.resize(cnt);
    for (int i = 0; i < cnt; ++i) nrm[i] = hi[i].normF;
    for (int i = 0; i < cnt; ++i) {
      BMat& x = hm[i];
      const int nn = x.n;
      JDesc& d = x.jd;
      double thr;
      if (o.abs_thr > 0.0) thr = std::ldexp(o.abs_thr, x.a_exp);
      else if (o.stop == JE_STOP_CERT) thr = tol * nrm[i] / (2.0 * nn * (double)(nn - 1));
      else thr = tol * nrm[i];
      d.A = precond ? x.A : x.Asym;
      d.n = nn; d.ld = x.ld; d.diag = x.diag;
      d.thr = thr;
      d.maxrot = o.max_rotations > 0 ? o.max_rotations : default_maxrot(nn);
      d.pivot = pivot; d.stop = o.stop;
      d.prof = nullptr;
      // a persistent launch stops a member after step_rot rotations (log drained between)
      d.log_cap = std::min<long long>(d.log_cap, step_rot);
      x.log_base = 0;
      x.f_pass_sweeps = 0;
    }
    if (int r = upload()) return r;
    // a batch keeps rows only (timestamp mode) unless asked otherwise: with hundreds of
    // matrices in flight the mirrored column stores, each dirtying a cache line for 8
    // bytes, make HBM writes the larger cost
    mirror = o.update_mode == 1;
    if (precond) {
      if (o.graph)
        if (int r = capture_stream()) return r;
      HIPCHK(f32.begin(dm, nv.data(), cnt, nmax, d_work, BF(Asym), offX, o.fp32_max_sweeps,
                       f32_tol1(o.fp32_passes), kF32Rho1, s, o.graph != 0, cap, f32_pb));
      phase = F32A;
    } else {
      HIPCHK(launch_set_identity_b(dm, cnt, nmax, BF(Vw), s));
      phase = CONTRACT;
    }
    S.ms_precond += tp.stop();
    return JE_OK;
  }

  // One Newton-Schulz step on every member not yet converged; *converged when all are.
  hipError_t ns_launches() {
    hipError_t e;
    if ((e = launch_dgemm_sym_b(dm, cnt, nmax, -1.0, offX, offX, BF(R), s, 1))) return e;
    if ((e = launch_add_identity_b(dm, cnt, nmax, BF(R), 1.0, s, 1))) return e;
    if ((e = launch_fro2_b(dm, cnt, nmax, BF(R), 1, s))) return e;
    if ((e = launch_dgemm_b(dm, cnt, nmax, 0, 0.5, offX, BF(R), 1.0, offX, offXb, s))) return e;
    if ((e = launch_ns_flag_b(dm, cnt, s))) return e;
    return launch_collect_b(dm, cnt, d_info, s);
  }
  int ns_step(bool* converged) {
    if (ns_iter == 0) HIPCHK(launch_ns_reset_b(dm, cnt, s));
    if (o.graph) {
      graphs_current();
      hipGraphExec_t& g = g_ns[offX == BF(X) ? 0 : 1];
      if (!g)
        if (int r = capture(&g, [&] { return ns_launches(); })) return r;
      HIPCHK(hipGraphLaunch(g, s));
    } else {
      HIPCHK(ns_launches());
    }
    std::swap(offX, offXb);
    HIPCHK(hipMemcpyAsync(hi.data(), d_info, (size_t)cnt * sizeof(BInfo), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    bool all = true;
    for (int i = 0; i < cnt; ++i) all = all && ns_converged(hi[i].rnorm, hm[i].n);
    ++ns_iter;
    *converged = all || ns_iter >= 6;
    if (*converged) ns_iter = 0;
    return JE_OK;
  }

  // Workgroup shape of each class: tuned once per (class, pivot, size bucket) and cached.
  int tune_shapes() {
    std::vector<int> ord(cnt), il, ih;
    for (int i = 0; i < cnt; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return hm[a].n > hm[b].n; });
    int nl = 0, nh = 0;
    for (int i : ord) {
      if (batch_lds(hm[i].n)) { il.push_back(i); nl = std::max(nl, hm[i].n); }
      else { ih.push_back(i); nh = std::max(nh, hm[i].n); }
    }
    const int use_cert = (pivot == 0 && o.stop == JE_STOP_CERT) ? 1 : 0;
    auto tuned = [&](bool lds, const std::vector<int>& lst, int nmx, int* shape) -> int {
      if (lst.empty()) return JE_OK;
      // the default shape first; another replaces it only if it is 5% faster (the fastest
      // such)
      const int a = lds ? 64 : 512;
      const std::vector<int> shapes = lds ? std::vector<int>{64, 128}
                                          : std::vector<int>{512, 256, 128};
      if ((lds && nmx > 128) || (!lds && nmx > 512)) return JE_OK;  // one shape only
      const int key = (lds ? 1 : 2) * 1000 + pivot * 100 + (int)std::ceil(std::log2((double)nmx));
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) { *shape = it->second; return JE_OK; }
      }
      if (!o.tune) return JE_OK;
      // the trial runs on the class itself (up to 1024 matrices, spread over its sizes):
      // a small sample leaves the device half idle and favours the wrong shape
      std::vector<int> smp;
      const size_t want = std::min<size_t>(lst.size(), 1024);
      for (size_t t = 0; t < want; ++t) smp.push_back(lst[t * lst.size() / want]);
      HIPCHK(hipMemcpyAsync(d_idx_lds, smp.data(), smp.size() * 4, hipMemcpyHostToDevice, s));
      const size_t offJ = precond ? BF(A) : BF(Asym);
      // the FP64 matrices of the whole batch are saved in T and restored after each trial
      HIPCHK(launch_copy_mat_b(dm, cnt, nmax, BF(T), offJ, s));
      float t_default = 0.f, t_best = 0.f;
      for (int shp : shapes) {
        HIPCHK(launch_zero_words(d_cnt, 2, s));
        Timer tt(s);
        HIPCHK(launch_jacobi_queue(dm, d_idx_lds, (int)smp.size(), nmx, pivot, lds, mirror,
                                   shp, d_cnt, queue_grid(lds, shp, smp.size()), s));
        const float ms = tt.stop();
        if (shp == a) { t_default = ms; t_best = ms; *shape = a; }
        else if (ms < 0.95f * t_default && ms < t_best) { t_best = ms; *shape = shp; }
        HIPCHK(launch_copy_mat_b(dm, cnt, nmax, offJ, BF(T), s));
        HIPCHK(launch_get_diag_b(dm, cnt, nmax, offJ, s));
        HIPCHK(launch_reset_b(dm, cnt, s));
        HIPCHK(launch_init_rows_b(dm, cnt, nmax, pivot, use_cert, s));
      }
      HIPCHK(hipStreamSynchronize(s));
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = *shape;
      return JE_OK;
    };
    if (int r = tuned(true, il, nl, &shape_lds)) return r;
    // a requested shape of the HBM-resident class (128 and 256 threads cover n <= 512)
    if (o.batch_threads == 512 || (o.batch_threads > 0 && nh <= 512)) {
      shape_hbm = o.batch_threads;
      return JE_OK;
    }
    if (int r = tuned(false, ih, nh, &shape_hbm)) return r;
    return JE_OK;
  }

  // Members whose FP64 phase ended: polish, sort, output (on a table of just them), report,
  // and leave the cohort.
  int finalize(const std::vector<char>& fin) {
    std::vector<BMat> hf;
    for (int i = 0; i < cnt; ++i)
      if (fin[i]) hf.push_back(hm[i]);
    const int nf = (int)hf.size();
    if (nf == 0) return JE_OK;
    int nfmax = 0;
    for (const BMat& x : hf) nfmax = std::max(nfmax, x.n);
    Timer tf(s);
    HIPCHK(hipMemcpyAsync(dfin, hf.data(), (size_t)nf * sizeof(BMat), hipMemcpyHostToDevice, s));
    bool anyv = false;
    for (const BMat& x : hf) anyv = anyv || x.Vout != nullptr;
    if (anyv && o.polish_v) {
      HIPCHK(launch_dgemm_sym_b(dfin, nf, nfmax, -1.0, BF(Vw), BF(Vw), BF(R), s));
      HIPCHK(launch_add_identity_b(dfin, nf, nfmax, BF(R), 1.0, s));
      HIPCHK(launch_dgemm_b(dfin, nf, nfmax, 0, 0.5, BF(Vw), BF(R), 1.0, BF(Vw), BF(X), s));
      HIPCHK(launch_copy_mat_b(dfin, nf, nfmax, BF(Vw), BF(X), s));
    }
    HIPCHK(launch_sort_output_b(dfin, nf, nfmax, o.sort, s));
    HIPCHK(hipStreamSynchronize(s));
    const float ms_fin = tf.stop();
    std::vector<char> keep(cnt, 1);
    for (int i = 0; i < cnt; ++i) {
      if (!fin[i]) continue;
      keep[i] = 0;
      const JCtl& c = hi[i].ctl;
      const int st = c.status == ST_MAXROT ? JE_WARN_MAXROT
                     : (c.status == ST_STALL ? JE_WARN_STALL : JE_OK);
      je_stats x = S;
      const double unscale = std::ldexp(1.0, -hm[i].a_exp);
      x.ms_jacobi_kernel = ms_kernel;
      x.ms_apply_log = ms_apply;
      x.ms_finalize = ms_fin;
      x.rotations = c.rotations;
      x.rescans = c.rescans;
      x.final_max_score = c.final_cert * unscale;
      x.final_off = c.final_off * unscale;
      x.normF = nrm[i] * unscale;
      x.thr = hm[i].jd.thr * unscale;
      x.sweeps32 = hi[i].sweeps32;
      x.scale_exp = hm[i].a_exp;
      x.jacobi_wgs = 1;
      x.status = st;
      leave(i, st, &x);
    }
    return compact(keep);
  }

  // One bounded piece of work.
  int step() {
    switch (phase) {
      case F32A:
      case F32B: {
        Timer tp(s);
        HIPCHK(f32.advance(8));
        if (f32.finished) {
          if (phase == F32A) {
            phase = NS1;
          } else {
            HIPCHK(launch_dgemm_b(dm, cnt, nmax, 0, 1.0, offX, BF(T), 0.0, 0, offXb, s));
            std::swap(offX, offXb);
            phase = NS2;
          }
        }
        S.ms_precond += tp.stop();
        return JE_OK;
      }
      case NS1:
      case NS2: {
        Timer tp(s);
        bool conv = false;
        if (int r = ns_step(&conv)) return r;
        if (conv) {
          if (phase == NS1 && pass + 1 < o.fp32_passes) phase = REFINE;
          else phase = CONTRACT;
          if (phase == REFINE) ++pass;
        }
        if (phase == CONTRACT) {
          // the contraction below is timed as ms_gemm
          S.ms_precond += tp.stop();
          return JE_OK;
        }
        S.ms_precond += tp.stop();
        return JE_OK;
      }
      case REFINE: {
        Timer tp(s);
        HIPCHK(launch_dgemm_b(dm, cnt, nmax, 0, 1.0, BF(Asym), offX, 0.0, 0, BF(T), s));
        HIPCHK(launch_dgemm_sym_b(dm, cnt, nmax, 1.0, offX, BF(T), BF(A), s));
        HIPCHK(f32.begin(dm, nv.data(), cnt, nmax, d_work, BF(A), BF(T), o.fp32_max_sweeps,
                         kF32Tol2, kF32Rho2, s, o.graph != 0, cap, f32_pb));
        phase = F32B;
        S.ms_precond += tp.stop();
        return JE_OK;
      }
      case CONTRACT: {
        if (precond) {
          Timer tg(s);
          HIPCHK(launch_dgemm_b(dm, cnt, nmax, 0, 1.0, BF(Asym), offX, 0.0, 0, BF(T), s));
          HIPCHK(launch_dgemm_sym_b(dm, cnt, nmax, 1.0, offX, BF(T), BF(A), s));
          HIPCHK(launch_copy_mat_b(dm, cnt, nmax, BF(Vw), offX, s));
          HIPCHK(launch_get_diag_b(dm, cnt, nmax, BF(A), s));
          S.ms_gemm += tg.stop();
        }
        Timer tj(s);
        HIPCHK(launch_reset_b(dm, cnt, s));
        const int use_cert = (pivot == 0 && o.stop == JE_STOP_CERT) ? 1 : 0;
        HIPCHK(launch_init_rows_b(dm, cnt, nmax, pivot, use_cert, s));
        if (int r = tune_shapes()) return r;
        phase = JACOBI;
        S.ms_jacobi += tj.stop();
        return JE_OK;
      }
      case JACOBI: {
        Timer tj(s);
        if (o.graph) graphs_current();
        if (!o.graph || !g_jq) {
          std::vector<int> ord(cnt);
          for (int i = 0; i < cnt; ++i) ord[i] = i;
          // largest first: the order of the FP64 work queue
          std::stable_sort(ord.begin(), ord.end(),
                           [&](int a, int b) { return hm[a].n > hm[b].n; });
          std::vector<int> il, ih;
          int nl = 0, nh = 0;
          for (int i : ord) {
            if (batch_lds(hm[i].n)) { il.push_back(i); nl = std::max(nl, hm[i].n); }
            else { ih.push_back(i); nh = std::max(nh, hm[i].n); }
          }
          if (!il.empty())
            HIPCHK(hipMemcpyAsync(d_idx_lds, il.data(), il.size() * 4, hipMemcpyHostToDevice, s));
          if (!ih.empty())
            HIPCHK(hipMemcpyAsync(d_idx_hbm, ih.data(), ih.size() * 4, hipMemcpyHostToDevice, s));
          HIPCHK(hipStreamSynchronize(s));  // the index vectors are host memory
          const int gl = queue_grid(true, shape_lds, il.size());
          const int gh = queue_grid(false, shape_hbm, ih.size());
          auto queue = [&]() -> hipError_t {
            hipError_t e = launch_zero_words(d_cnt, 2, s);
            if (e == hipSuccess && !il.empty())
              e = launch_jacobi_queue(dm, d_idx_lds, (int)il.size(), nl, pivot, true, mirror,
                                      shape_lds, d_cnt, gl, s);
            if (e == hipSuccess && !ih.empty())
              e = launch_jacobi_queue(dm, d_idx_hbm, (int)ih.size(), nh, pivot, false, mirror,
                                      shape_hbm, d_cnt + 1, gh, s);
            return e;
          };
          if (!o.graph) {
            Timer tk(s);
            HIPCHK(queue());
            ms_kernel += tk.stop();
          } else {
            // kernel attributes (the LDS size) are set outside the capture: grid 0 only
            // prepares the launch
            if (!il.empty())
              HIPCHK(launch_jacobi_queue(dm, d_idx_lds, (int)il.size(), nl, pivot, true, mirror,
                                         shape_lds, d_cnt, 0, s));
            if (!ih.empty())
              HIPCHK(launch_jacobi_queue(dm, d_idx_hbm, (int)ih.size(), nh, pivot, false,
                                         mirror, shape_hbm, d_cnt + 1, 0, s));
            if (int r = capture(&g_jq, queue)) return r;
            if (int r = capture(&g_ja, [&]() -> hipError_t {
                  hipError_t e = launch_apply_log_b(dm, cnt, nmax, s);
                  return e == hipSuccess ? launch_collect_b(dm, cnt, d_info, s) : e;
                }))
              return r;
          }
        }
        if (o.graph) {
          Timer tk(s);
          HIPCHK(hipGraphLaunch(g_jq, s));
          ms_kernel += tk.stop();
          Timer ta(s);
          HIPCHK(hipGraphLaunch(g_ja, s));
          ms_apply += ta.stop();
          HIPCHK(hipMemcpyAsync(hi.data(), d_info, (size_t)cnt * sizeof(BInfo),
                                hipMemcpyDeviceToHost, s));
          HIPCHK(hipStreamSynchronize(s));
        } else {
          Timer ta(s);
          HIPCHK(launch_apply_log_b(dm, cnt, nmax, s));
          ms_apply += ta.stop();
          if (int r = collect()) return r;
        }
        S.ms_jacobi += tj.stop();
        std::vector<char> fin(cnt, 0);
        bool any = false;
        for (int i = 0; i < cnt; ++i) {
          fin[i] = hi[i].ctl.done ? 1 : 0;
          any = any || fin[i];
        }
        if (any) return finalize(fin);
        return JE_OK;
      }
      default:
        return JE_OK;
    }
  }
};

// All problems of a batch (n >= 2) go through one cohort: every launch covers the whole
// batch (grids sized for the largest n, blocks past a matrix's n exit).  The FP32 stage
// runs each matrix at its own pace; the FP64 Jacobi phase is one persistent launch per
// workgroup shape (LDS-resident n <= 64, HBM-resident above), each workgroup taking the
// next matrix, largest first, from a device counter.  Logs are drained for all matrices
// between launches; unfinished matrices are relaunched.
int solve_batched(std::vector<int> idx, const double* const* Ain, const int* n,
                  const int* lda, double* const* W, double* const* V, const int* ldv, double tol,
                  int pivot, int precond, const je_opts& o, int* info, je_stats* stats,
                  hipStream_t s) {
  const int cnt = (int)idx.size();
  if (cnt == 0) return JE_OK;
  std::vector<Member> mem(cnt);
  size_t tot = 0;
  std::vector<size_t> woff(cnt);
  for (int i = 0; i < cnt; ++i) {
    woff[i] = tot;
    tot += bws_bytes(n[idx[i]], precond, kBatchLogCap);
  }
  int err = JE_OK;
  char* base = (char*)pool_get(tot + cohort_meta_bytes(cnt), &err);
  if (!base) return err;
  for (int i = 0; i < cnt; ++i) {
    const int b = idx[i];
    mem[i] = Member{Ain[b], n[b], lda[b], W[b], V ? V[b] : nullptr, ldv ? ldv[b] : n[b],
                    base + woff[i], b};
  }
  Cohort c;
  int r = c.begin(mem, base + tot, tol, pivot, precond, o, s, kBatchLogCap);
  while (r == JE_OK && c.phase != Cohort::DONE) r = c.step();
  if (r != JE_OK) return r;
  int worst = JE_OK;
  for (const Cohort::Left& l : c.left) {
    info[l.idx] = l.status;
    worst = std::max(worst, l.status);
    if (stats) stats[l.idx] = l.st;
  }
  return worst;
}

// ------------------------------------------------------------------ serving
// Continuous batching of a request stream.  One device buffer of hbm_budget bytes (the
// arena) holds the workspaces of every request in flight; `lanes` host threads, each with
// its own stream, run cohorts (Cohort above) in bounded steps.  At every step boundary a
// lane admits queued requests: the oldest one of the size classes it serves (n <= 128,
// <= 512, <= 1024, larger; see lane_serves) and the queued requests of that class, in
// arrival order, as far as their workspaces fit in the arena, form a new cohort that runs
// beside the lane's other cohorts (at most kLaneCohorts at once).  A request whose
// workspace does not fit stays queued until memory is freed.  Members whose solve has
// ended leave their cohort at the end of that step: their completion record is posted and
// their workspace returned to the arena.  Cohorts of different lanes run concurrently on
// the device; the cohorts of one lane interleave step by step.
constexpr long long kServeStepRot = 4096;  // FP64 rotations per member per step
// Cohorts a lane runs at once: a request that arrives while its lane is at this limit
// waits and joins the next cohort, so cohorts grow with the load (a cohort of k large
// matrices costs about as long as one of a single large matrix).
constexpr int kLaneCohorts = 2;

struct SrvReq {
  const double* A;
  int n, lda;
  double* W;
  double* V;
  int ldv;
  long long tag;
  double t_submit;
};

// First-fit allocator over the arena (offsets in 256-byte units), adjacent free blocks
// merged on release.
struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void init(char* b, size_t n) {
    base = b;
    bytes = n & ~(size_t)255;
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  char* get(size_t n) {
    n = al(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > n) free_[off + n] = sz - n;
      return base + off;
    }
    return nullptr;
  }
  void put(char* p, size_t n) {
    n = al(n);
    size_t off = (size_t)(p - base);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
};

struct Server {
  int device = 0;
  double tol = 0.0;
  int pivot = 1, precond = 1;
  je_opts o{};
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SrvReq> queue;
  std::deque<je_done> done;
  long long in_flight = 0;
  bool stop = false;
  int error = 0;
  void* buffer = nullptr;
  Arena arena;
  long long mem_gen = 0;  // incremented whenever memory returns to the arena
  int lanes_n = 1;
  std::vector<std::thread> lanes;
  std::chrono::steady_clock::time_point t0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

int size_class(int n) { return n <= 128 ? 0 : (n <= 512 ? 1 : (n <= 1024 ? 2 : 3)); }

// Lanes are affine to size classes, so that the long steps of large problems never delay
// the steps of small ones: with L >= 4 lanes lane l serves class l mod 4, with fewer lanes
// class c goes to lane c mod L.
bool lane_serves(int lane, int lanes, int cls) {
  return lanes >= 4 ? (lane % 4 == cls) : (cls % lanes == lane);
}

// A cohort of a lane and the arena blocks it holds.
struct LaneCohort {
  Cohort c;
  std::vector<SrvReq> req;          // by Member::idx
  std::vector<char*> ws;            // workspace of each request (null once returned)
  std::vector<size_t> ws_bytes;
  char* meta = nullptr;
  size_t meta_bytes = 0;
  double t_start = 0.0;
  int members = 0;
};

// Posts the records of the members that left `lc` since the last call and returns their
// workspaces to the arena.  Caller holds S->mu.
void post_left(Server* S, LaneCohort& lc, size_t& seen) {
  const double t = S->now();
  for (; seen < lc.c.left.size(); ++seen) {
    const Cohort::Left& l = lc.c.left[seen];
    const SrvReq& r = lc.req[l.idx];
    je_done d{};
    d.tag = r.tag;
    d.status = l.status;
    d.n = r.n;
    d.batch = lc.members;
    d.rotations = l.st.rotations;
    d.t_submit = r.t_submit;
    d.t_start = lc.t_start;
    d.t_done = t;
    S->done.push_back(d);
    if (lc.ws[l.idx]) {
      S->arena.put(lc.ws[l.idx], lc.ws_bytes[l.idx]);
      lc.ws[l.idx] = nullptr;
      ++S->mem_gen;
    }
    --S->in_flight;
  }
}

void server_lane(Server* S, int lane) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->error = JE_ERR_DEVICE;
    S->cv_done.notify_all();
    return;
  }
  std::vector<std::unique_ptr<LaneCohort>> cohorts;
  std::vector<size_t> seen;
  long long gen_seen = -1;  // arena generation of this lane's last failed admission
  for (;;) {
    // ---- admission at the step boundary
    std::unique_ptr<LaneCohort> nc;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      // an idle lane sleeps until there is a request it has not yet failed to place
      const int lanes = (int)S->lanes_n;
      auto mine = [&]() -> const SrvReq* {
        for (const SrvReq& r : S->queue)
          if (lane_serves(lane, lanes, size_class(r.n))) return &r;
        return nullptr;
      };
      if (cohorts.empty())
        S->cv_work.wait(lk, [&] { return S->stop || (mine() && S->mem_gen != gen_seen); });
      if (cohorts.empty() && !mine() && S->stop) break;
      if (cohorts.empty() && S->mem_gen == gen_seen) continue;  // stop requested, memory held
      if (const SrvReq* first = (cohorts.size() < (size_t)kLaneCohorts) ? mine() : nullptr) {
        const int cls = size_class(first->n);
        std::vector<SrvReq> take;
        std::vector<char*> ws;
        std::vector<size_t> wb;
        for (auto it = S->queue.begin(); it != S->queue.end();) {
          if (size_class(it->n) != cls) { ++it; continue; }
          const size_t b = bws_bytes(it->n, S->precond, kBatchLogCap);
          char* p = S->arena.get(b);
          if (!p) break;  // admission by footprint: the rest waits for memory
          take.push_back(*it);
          ws.push_back(p);
          wb.push_back(b);
          it = S->queue.erase(it);
        }
        char* meta = nullptr;
        const size_t mb = take.empty() ? 0 : cohort_meta_bytes((int)take.size());
        if (!take.empty()) meta = S->arena.get(mb);
        if (!take.empty() && !meta) {
          // no room for the tables: give the requests back, in order
          for (size_t i = 0; i < take.size(); ++i) S->arena.put(ws[i], wb[i]);
          for (size_t i = take.size(); i-- > 0;) S->queue.push_front(take[i]);
          take.clear();
        }
        if (take.empty()) gen_seen = S->mem_gen;
        if (!take.empty()) {
          nc.reset(new LaneCohort());
          nc->req = take;
          nc->ws = ws;
          nc->ws_bytes = wb;
          nc->meta = meta;
          nc->meta_bytes = mb;
          nc->members = (int)take.size();
          S->in_flight += (long long)take.size();
        }
      }
    }
    if (nc) {
      std::vector<Member> mem(nc->req.size());
      for (size_t i = 0; i < nc->req.size(); ++i) {
        const SrvReq& r = nc->req[i];
        mem[i] = Member{r.A, r.n, r.lda, r.W, r.V, r.ldv, nc->ws[i], (int)i};
      }
      nc->t_start = S->now();
      int r = nc->c.begin(mem, nc->meta, S->tol, S->pivot, S->precond, S->o, st, kServeStepRot);
      if (r != JE_OK) {
        // the whole cohort failed: every member gets the error
        std::lock_guard<std::mutex> lk(S->mu);
        for (size_t i = 0; i < nc->req.size(); ++i)
          nc->c.left.push_back(Cohort::Left{(int)i, r, je_stats{}});
        nc->c.phase = Cohort::DONE;
      }
      cohorts.push_back(std::move(nc));
      seen.push_back(0);
    }
    // ---- one step of every cohort of this lane
    for (size_t k = 0; k < cohorts.size(); ++k) {
      LaneCohort& lc = *cohorts[k];
      if (lc.c.phase != Cohort::DONE) {
        const int r = lc.c.step();
        if (r != JE_OK) {
          // a device error ends the cohort: its remaining members get the status
          for (int i = 0; i < lc.c.cnt; ++i) lc.c.leave(i, r, nullptr);
          lc.c.cnt = 0;
          lc.c.phase = Cohort::DONE;
        }
      }
      std::lock_guard<std::mutex> lk(S->mu);
      post_left(S, lc, seen[k]);
    }
    // ---- finished cohorts return their tables
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (size_t k = 0; k < cohorts.size();) {
        if (cohorts[k]->c.phase == Cohort::DONE) {
          S->arena.put(cohorts[k]->meta, cohorts[k]->meta_bytes);
          ++S->mem_gen;
          cohorts.erase(cohorts.begin() + k);
          seen.erase(seen.begin() + k);
        } else {
          ++k;
        }
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();  // memory may have been freed for queued requests
  }
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
}

int check_args(const double* A, int n, int lda, const double* W, const double* V, int ldv,
               double tol, int pivot, int precond, const je_opts& o) {
  if (!A && n > 0) return -1;
  if (n < 0) return -2;
  if (lda < std::max(1, n)) return -3;
  if (!W && n > 0) return -4;
  if (V && ldv < std::max(1, n)) return -6;
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    if (!(o.abs_thr > 0.0)) return -7;
  }
  if (pivot != JE_PIVOT_GREEDY && pivot != JE_PIVOT_GAP) return -8;
  if (precond != JE_PRECOND_NONE && precond != JE_PRECOND_FP32) return -9;
  if (o.stop < JE_STOP_CERT || o.stop > JE_STOP_SCORE) return -10;
  if (o.fp32_max_sweeps < 0 || o.fp32_passes < 1 || o.fp32_passes > 2) return -10;
  if (o.split_gemm != 0 && o.split_gemm != 1) return -10;
  if (o.sort != 0 && o.sort != 1) return -10;
  if (o.update_mode < 0 || o.update_mode > 2) return -10;
  if (o.tune != 0 && o.tune != 1) return -10;
  if (o.graph != 0 && o.graph != 1) return -10;
  if (o.profile != 0 && o.profile != 1) return -10;
  if (o.fp32_block != 0 && o.fp32_block != 16 && o.fp32_block != 32) return -10;
  if (o.jacobi_wgs < 0 || o.jacobi_wgs > 2) return -10;
  if (o.batch_threads != 0 && o.batch_threads != 128 && o.batch_threads != 256 &&
      o.batch_threads != 512)
    return -10;
  return 0;
}

// ------------------------------------------------------------------ no-allocation solves
// Workspace of jacobi_eigh_noalloc: a file-scope device array (one copy per device, held
// until the process ends).  Its size covers ws_bytes(JE_NOALLOC_MAX_N, precond = 1,
// kNoAllocLogCap); the entry point checks every call against it.
constexpr long long kNoAllocLogCap = 1ll << 16;
constexpr size_t kNoAllocBytes = JE_NOALLOC_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

// Device address of `scratch` on each device, taken once with that device current (in host
// code the array's name is only a stand-in for the symbol).
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

void* scratch_address(int* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { *err = JE_ERR_DEVICE; return nullptr; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    *err = JE_ERR_DEVICE;
    return nullptr;
  }
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

}  // namespace

extern "C" {

void je_opts_default(je_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->stop = JE_STOP_CERT;
  o->polish_v = 1;
  o->fp32_max_sweeps = 20;
  o->fp32_passes = 2;
  o->max_rotations = 0;
  o->abs_thr = 0.0;
  o->pivot_log = nullptr;
  o->pivot_log_cap = 0;
  o->split_gemm = 0;
  o->sort = 1;
  o->update_mode = 0;
  o->tune = 1;
  o->graph = 0;
  o->profile = 0;
  o->fp32_block = 0;
  o->jacobi_wgs = 0;
  o->batch_threads = 0;
}

int jacobi_eigh_ex(const double* A, int n, int lda, double* W, double* V, int ldv, double tol,
                   int pivot, int precond, const je_opts* opts, je_stats* stats,
                   je_stream stream) {
  je_opts o;
  if (opts) o = *opts;
  else je_opts_default(&o);
  int a = check_args(A, n, lda, W, V, ldv, tol, pivot, precond, o);
  if (a) return a;
  if (n > JE_MAX_N) return JE_ERR_TOO_LARGE;
  hipStream_t s = (hipStream_t)stream;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return JE_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  if (n == 1) {
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, A, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!std::isfinite(v)) return JE_ERR_NONFINITE;
    HIPCHK(hipMemcpyAsync(W, A, 8, hipMemcpyDeviceToDevice, s));
    if (V) {
      static const double one = 1.0;
      HIPCHK(hipMemcpyAsync(V, &one, 8, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (stats) stats->normF = std::fabs(v);
    return JE_OK;
  }
  const long long maxrot = o.max_rotations > 0 ? o.max_rotations : default_maxrot(n);
  const long long cap = log_cap_for(n, maxrot);
  int err = JE_OK;
  void* base = pool_get(ws_bytes(n, precond, cap, o.split_gemm), &err);
  if (!base) return err;
  return solve_one(A, n, lda, W, V, ldv, tol, pivot, precond, o, stats, s, base, cap);
}

int jacobi_eigh_noalloc(const double* A, int n, int lda, double* W, double* V, int ldv,
                        double tol, int pivot, int precond, const je_opts* opts,
                        je_stats* stats, je_stream stream) {
  je_opts o;
  if (opts) o = *opts;
  else je_opts_default(&o);
  int a = check_args(A, n, lda, W, V, ldv, tol, pivot, precond, o);
  if (a) return a;
  if (n > JE_NOALLOC_MAX_N) return JE_ERR_TOO_LARGE;
  o.graph = 0;  // graph instantiation would create runtime objects
  hipStream_t s = (hipStream_t)stream;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return JE_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  if (n == 1) {
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, A, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!std::isfinite(v)) return JE_ERR_NONFINITE;
    HIPCHK(hipMemcpyAsync(W, A, 8, hipMemcpyDeviceToDevice, s));
    if (V) {
      static const double one = 1.0;
      HIPCHK(hipMemcpyAsync(V, &one, 8, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    if (stats) stats->normF = std::fabs(v);
    return JE_OK;
  }
  const long long maxrot = o.max_rotations > 0 ? o.max_rotations : default_maxrot(n);
  const long long cap = log_cap_for(n, std::min(maxrot, kNoAllocLogCap));
  if (ws_bytes(n, precond, cap, o.split_gemm) > kNoAllocBytes) return JE_ERR_TOO_LARGE;
  int err = JE_OK;
  void* base = scratch_address(&err);
  if (!base) return err;
  t_timers_off = true;
  const int r = solve_one(A, n, lda, W, V, ldv, tol, pivot, precond, o, stats, s, base, cap);
  t_timers_off = false;
  return r;
}

int jacobi_eigh(const double* A, int n, int lda, double* W, double* V, double tol, int pivot,
                int precond) {
  return jacobi_eigh_ex(A, n, lda, W, V, n, tol, pivot, precond, nullptr, nullptr, nullptr);
}

int jacobi_svd(const double* B, int m, int n, int ldb, double* S, double* U, int ldu, double* V,
               int ldv, double tol, int pivot, int precond, const je_opts* opts,
               je_stats* stats, je_stream stream) {
  je_opts o;
  if (opts) o = *opts;
  else je_opts_default(&o);
  int a = check_svd_args(B, m, n, ldb, S, U, ldu, V, ldv, tol, pivot, precond, o);
  if (a) return a;
  if (n > JE_MAX_N) return JE_ERR_TOO_LARGE;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return JE_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  return svd_one(B, m, n, ldb, S, U, ldu, V, ldv, tol, pivot, precond, o, stats,
                 (hipStream_t)stream);
}

int jacobi_eigh_batched_host(int batch, const double* const* A, const int* n, const int* lda,
                             double* const* W, double* const* V, const int* ldv, double tol,
                             int pivot, int precond, const je_opts* opts, int* info,
                             je_stats* stats, je_stream stream) {
  if (batch < 0) return -1;
  if (batch > 0 && (!A || !n || !lda || !W || !info)) return -2;
  je_opts o;
  if (opts) o = *opts;
  else je_opts_default(&o);
  o.pivot_log = nullptr;
  // argument checks first: a bad problem rejects the whole call before any work
  for (int b = 0; b < batch; ++b) {
    // argument k of the single call is argument k + 1 here
    int a = check_args(A[b], n[b], lda[b], W[b], V ? V[b] : nullptr, ldv ? ldv[b] : n[b], tol,
                       pivot, precond, o);
    if (a) { info[b] = a - 1; return a - 1; }
    if (n[b] > JE_MAX_N) { info[b] = JE_ERR_TOO_LARGE; return JE_ERR_TOO_LARGE; }
  }
  int worst = JE_OK;
  std::vector<int> mem;
  for (int b = 0; b < batch; ++b) {
    if (n[b] >= 2) { mem.push_back(b); info[b] = JE_ERR_DEVICE; continue; }
    je_stats* sb = stats ? &stats[b] : nullptr;
    int r = jacobi_eigh_ex(A[b], n[b], lda[b], W[b], V ? V[b] : nullptr, ldv ? ldv[b] : n[b], tol,
                           pivot, precond, &o, sb, stream);
    info[b] = r;
    worst = std::max(worst, r);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  int r = solve_batched(mem, A, n, lda, W, V, ldv, tol, pivot, precond, o, info, stats,
                        (hipStream_t)stream);
  return std::max(worst, r);  // errors (>= 3) rank above warnings (1, 2)
}

int jacobi_eigh_batched(int batch, const double* const* A, const int* n, const int* lda,
                        double* const* W, double* const* V, double tol, int pivot,
                        int precond, const je_opts* opts, int* info, je_stream stream) {
  if (batch < 0) return -1;
  if (batch == 0) return JE_OK;
  if (!A) return -2;
  if (!n) return -3;
  if (!lda) return -4;
  if (!W) return -5;
  if (!info) return -11;
  hipStream_t s = (hipStream_t)stream;
  // the batch's description is read to the host: the workspace of each member is carved
  // by its size
  std::vector<const double*> hA(batch);
  std::vector<double*> hW(batch), hV(V ? batch : 0);
  std::vector<int> hn(batch), hlda(batch), hinfo(batch, 0);
  HIPCHK(hipMemcpyAsync(hA.data(), A, sizeof(double*) * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hW.data(), W, sizeof(double*) * batch, hipMemcpyDeviceToHost, s));
  if (V) HIPCHK(hipMemcpyAsync(hV.data(), V, sizeof(double*) * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hn.data(), n, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hlda.data(), lda, sizeof(int) * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int r = jacobi_eigh_batched_host(batch, hA.data(), hn.data(), hlda.data(), hW.data(),
                                   V ? hV.data() : nullptr, nullptr, tol, pivot, precond, opts,
                                   hinfo.data(), nullptr, stream);
  // argument numbers of the host form past V are one higher (its ldv)
  if (r < -7) r += 1;
  for (int& x : hinfo)
    if (x < -7) x += 1;
  HIPCHK(hipMemcpyAsync(info, hinfo.data(), sizeof(int) * batch, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return r;
}

size_t jacobi_workspace_size(int n, int precond) {
  if (n <= 1) return 0;
  return ws_bytes(n, precond ? 1 : 0, log_cap_for(n, default_maxrot(n)));
}

const char* jacobi_strerror(int status) {
  if (status < 0) return "invalid argument";
  switch (status) {
    case JE_OK: return "ok";
    case JE_WARN_MAXROT: return "rotation cap reached before the stop rule held";
    case JE_WARN_STALL: return "best remaining pivot is zero before the stop rule held";
    case JE_ERR_NONFINITE: return "input holds NaN or Inf";
    case JE_ERR_NOMEM: return "device workspace allocation failed";
    case JE_ERR_DEVICE: return "HIP runtime error";
    case JE_ERR_TOO_LARGE: return "n exceeds JE_MAX_N";
    default: return "unknown status";
  }
}

je_server* jacobi_server_create(int workers, size_t hbm_budget, double tol, int pivot,
                                int precond, const je_opts* opts) {
  je_opts o;
  if (opts) o = *opts;
  else je_opts_default(&o);
  o.pivot_log = nullptr;
  if (workers < 1 || workers > 16) return nullptr;
  if (!(tol > 0.0) && !(o.abs_thr > 0.0)) return nullptr;
  if (pivot != JE_PIVOT_GREEDY && pivot != JE_PIVOT_GAP) return nullptr;
  if (precond != JE_PRECOND_NONE && precond != JE_PRECOND_FP32) return nullptr;
  if (check_args((const double*)1, 2, 2, (const double*)1, nullptr, 2, tol, pivot, precond, o))
    return nullptr;
  Server* S = new Server();
  if (hipGetDevice(&S->device) != hipSuccess) { delete S; return nullptr; }
  S->tol = tol; S->pivot = pivot; S->precond = precond; S->o = o;
  S->budget = std::max<size_t>(hbm_budget, (size_t)1 << 20);
  if (hipMalloc(&S->buffer, S->budget) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return nullptr;
  }
  S->arena.init((char*)S->buffer, S->budget);
  S->t0 = std::chrono::steady_clock::now();
  S->lanes_n = workers;
  for (int i = 0; i < workers; ++i) S->lanes.emplace_back(server_lane, S, i);
  return reinterpret_cast<je_server*>(S);
}

int jacobi_server_submit(je_server* srv, const double* A, int n, int lda, double* W, double* V,
                         int ldv, long long tag) {
  Server* S = reinterpret_cast<Server*>(srv);
  if (!S) return -1;
  int a = check_args(A, n, lda, W, V, ldv, S->tol, S->pivot, S->precond, S->o);
  if (a) return a - 1;  // argument k of the single call is argument k + 1 here
  if (n > JE_MAX_N) return JE_ERR_TOO_LARGE;
  // a request that could never be admitted: its workspace and a one-member cohort's tables
  // exceed the whole budget
  if (n >= 2 && al(bws_bytes(n, S->precond, kBatchLogCap)) + al(cohort_meta_bytes(1)) >
                    S->arena.bytes)
    return JE_ERR_NOMEM;
  if (n < 2) {
    // trivial problems complete at once, through the single-problem call
    int r = jacobi_eigh_ex(A, n, lda, W, V, ldv, S->tol, S->pivot, S->precond, &S->o, nullptr,
                           nullptr);
    std::lock_guard<std::mutex> lk(S->mu);
    je_done d{};
    d.tag = tag; d.status = r; d.n = n; d.batch = 1;
    d.t_submit = d.t_start = d.t_done = S->now();
    S->done.push_back(d);
    S->cv_done.notify_all();
    return JE_OK;
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error) return S->error;
    S->queue.push_back(SrvReq{A, n, lda, W, V, ldv, tag, S->now()});
  }
  S->cv_work.notify_all();  // the lane serving this size class may be any of them
  return JE_OK;
}

int jacobi_server_poll(je_server* srv, je_done* out, int max, int wait) {
  Server* S = reinterpret_cast<Server*>(srv);
  if (!S || (!out && max > 0) || max < 0) return -1;
  std::unique_lock<std::mutex> lk(S->mu);
  if (wait)
    S->cv_done.wait(lk, [&] {
      return !S->done.empty() || (S->queue.empty() && S->in_flight == 0) || S->error;
    });
  int k = 0;
  while (k < max && !S->done.empty()) {
    out[k++] = S->done.front();
    S->done.pop_front();
  }
  return k;
}

long long jacobi_server_pending(je_server* srv) {
  Server* S = reinterpret_cast<Server*>(srv);
  if (!S) return -1;
  std::lock_guard<std::mutex> lk(S->mu);
  return (long long)S->queue.size() + S->in_flight;
}

double jacobi_server_clock(je_server* srv) {
  Server* S = reinterpret_cast<Server*>(srv);
  return S ? S->now() : -1.0;
}

void jacobi_server_destroy(je_server* srv) {
  Server* S = reinterpret_cast<Server*>(srv);
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->lanes) t.join();
  if (S->buffer) (void)hipFree(S->buffer);
  delete S;
}

void jacobi_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  for (auto& p : g_pools) {
    if (p.ptr) (void)hipFree(p.ptr);
    p.ptr = nullptr;
    p.bytes = 0;
  }
}

}  // extern "C"
