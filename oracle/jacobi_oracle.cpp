// Oracle for the preconditioned Jacobi eigensolver with gap-aware pivoting
// (N. Shao, Y. Nakatsukasa, "Accelerating preconditioned Jacobi methods via
// perturbation-inspired pivoting").
//
// TEST INFRASTRUCTURE ONLY.  This is a plain, slow, CPU implementation written for
// readability, used by the test-suite and by the benchmark's CPU baseline to check the
// HIP implementation.  It shares no code, header, table or helper with the HIP path,
// and the product never calls it.
//
// Everything is row-major, full symmetric storage, FP64 (FP32 for the low-precision
// preconditioner), built with -O2 -ffp-contract=off and no fast-math so that each
// operation below is one correctly rounded IEEE operation in the order written.
//
// Readings of points the paper leaves open (every one is also listed in the design notes):
//   * score when a_ij^2 == 0 in FP64: defined as 0 (eq. (1) is 0/0 when also a_ii == a_jj);
//   * rotation: the small-angle root of t^2 + 2 theta t - 1 = 0, theta = (a_pp - a_qq)/(2 a_pq),
//     evaluated as t = sgn(delta) 2 a_pq / (|delta| + sqrt(delta^2 + 4 a_pq^2)),
//     delta = a_pp - a_qq, sgn(0) = +1 (no division by a_pq, no theta^2 overflow);
//   * argmax ties: the lexicographically smallest (i, j), i < j;
//   * stop rules: certificate max_{i!=j} L_ij <= thr (Theorem 1), off(A) <= thr, or
//     the selection score of the best pivot <= thr.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

namespace {

// eq. (1): L_ij = 2|a_ij|^2 / (|a_ii - a_jj| + sqrt(|a_ii - a_jj|^2 + 4|a_ij|^2)).
// Defined as 0 when a_ij^2 is 0 in FP64 (a_ij == 0, or |a_ij| < 2^-537 so that the
// square underflows): eq. (1) would be 0/0 when also a_ii == a_jj.
double gap_score(double aii, double ajj, double aij) {
  double a2 = aij * aij;
  if (a2 == 0.0) return 0.0;
  double d = std::fabs(aii - ajj);
  return (2.0 * a2) / (d + std::sqrt(d * d + 4.0 * a2));
}

// Classical greedy score: the magnitude of the off-diagonal entry.
double greedy_score(double aij) { return std::fabs(aij); }

// Relative score of Sec. 4.2 for a symmetric positive definite A:
//   Lhat_ij = (1/a_ii + 1/a_jj) L_ij,
// the sum of the relative shifts of the two eigenvalues of the 2 x 2 block.  Lhat does not
// change when the block is scaled, so a_ii, a_jj, a_ij are first multiplied by the power of
// two that brings max(a_ii, a_jj) into [1/2, 1) (exact): for a pair of tiny diagonal
// entries a_ij^2 then stays in range.  0 when a_ij == 0, or when the scaled a_ij^2
// underflows.
double rel_score(double aii, double ajj, double aij) {
  if (aij == 0.0) return 0.0;
  int e;
  (void)std::frexp(std::max(aii, ajj), &e);
  double x = std::ldexp(aii, -e), y = std::ldexp(ajj, -e), a = std::ldexp(aij, -e);
  double l = gap_score(x, y, a);
  if (l == 0.0) return 0.0;
  return (1.0 / x + 1.0 / y) * l;
}

// c, s such that G^T [[app, apq], [apq, aqq]] G is diagonal, G = [[c, -s], [s, c]] (Sec. 2).
// t = s / c is the root of modulus <= 1 of t^2 + 2 theta t - 1 = 0, theta = (app - aqq)/(2 apq),
// written without theta: t = sgn(delta) 2 apq / (|delta| + sqrt(delta^2 + 4 apq^2)),
// delta = app - aqq, sgn(0) = +1.  t depends only on the ratio delta : apq, so when both
// are tiny or huge they are first scaled by the same power of two (exactly) to keep the
// squares in range.  Then c = 1/sqrt(1 + t^2), s = t c, and the new diagonal entries are
// app + t apq and aqq - t apq.
template <typename T>
void rotation(T app, T aqq, T apq, T* t, T* c, T* s) {
  const T lo = sizeof(T) == 8 ? T(0x1p-400) : T(0x1p-50);
  const T hi = sizeof(T) == 8 ? T(0x1p400) : T(0x1p50);
  T d = app - aqq;
  T a = apq;
  T m = std::max(std::fabs(d), std::fabs(a));
  if (m < lo || m > hi) {
    int e;
    (void)std::frexp(m, &e);
    d = std::ldexp(d, -e);
    a = std::ldexp(a, -e);
  }
  T den = std::fabs(d) + std::sqrt(d * d + T(4) * (a * a));
  T tt = (T(2) * a) / den;
  if (d < T(0)) tt = -tt;
  T cc = T(1) / std::sqrt(T(1) + tt * tt);
  *t = tt;
  *c = cc;
  *s = tt * cc;
}

struct Matrix {
  double* a;
  int n;
  double at(int i, int j) const { return a[(size_t)i * n + j]; }
};

// Score of pair (i, j) under a strategy: 0 = greedy |a_ij|, 1 = gap L_ij, 2 = relative Lhat_ij.
double pair_score(const Matrix& m, int i, int j, int strategy) {
  if (strategy == 1) return gap_score(m.at(i, i), m.at(j, j), m.at(i, j));
  if (strategy == 2) return rel_score(m.at(i, i), m.at(j, j), m.at(i, j));
  return greedy_score(m.at(i, j));
}

// Best (score, column) of row k over l != k; ties go to the smallest column.
void row_best(const Matrix& m, int k, int strategy, double* best, int* arg) {
  double b = -1.0;
  int a = -1;
  for (int l = 0; l < m.n; ++l) {
    if (l == k) continue;
    double v = pair_score(m, k, l, strategy);
    if (v > b) {
      b = v;
      a = l;
    }
  }
  *best = b;
  *arg = a;
}

double row_off2(const Matrix& m, int k) {
  double s = 0.0;
  for (int l = 0; l < m.n; ++l)
    if (l != k) s += m.at(k, l) * m.at(k, l);
  return s;
}

// Per-row best-score cache (the O(n) maintenance the paper describes in Sec. 3.2).
struct RowCache {
  int strategy;
  std::vector<double> best;
  std::vector<int> arg;
  long long rescans = 0;

  void build(const Matrix& m) {
    best.assign(m.n, 0.0);
    arg.assign(m.n, -1);
    for (int k = 0; k < m.n; ++k) row_best(m, k, strategy, &best[k], &arg[k]);
  }

  // Called after rotation (p, q) has been applied to m.
  void refresh(const Matrix& m, int p, int q) {
    for (int k = 0; k < m.n; ++k) {
      if (k == p || k == q) {
        row_best(m, k, strategy, &best[k], &arg[k]);
        continue;
      }
      double sp = pair_score(m, k, p, strategy);
      double sq = pair_score(m, k, q, strategy);
      if (arg[k] == p || arg[k] == q) {
        // the cached maximum itself moved; every other entry is still <= best[k]
        double v = sp;
        int col = p;
        if (sq > v) {
          v = sq;
          col = q;
        }
        if (v > best[k] || (v == best[k] && col <= arg[k])) {
          best[k] = v;
          arg[k] = col;
        } else {
          row_best(m, k, strategy, &best[k], &arg[k]);
          ++rescans;
        }
      } else {
        if (sp > best[k] || (sp == best[k] && p < arg[k])) {
          best[k] = sp;
          arg[k] = p;
        }
        if (sq > best[k] || (sq == best[k] && q < arg[k])) {
          best[k] = sq;
          arg[k] = q;
        }
      }
    }
  }

  // Row with the largest cached value (smallest row on ties) -> lexicographic argmax.
  void argmax(double* v, int* i, int* j) const {
    double b = -1.0;
    int r = -1;
    for (int k = 0; k < (int)best.size(); ++k)
      if (best[k] > b) {
        b = best[k];
        r = k;
      }
    *v = b;
    if (r < 0) {
      *i = *j = -1;
      return;
    }
    *i = std::min(r, arg[r]);
    *j = std::max(r, arg[r]);
  }
};

}  // namespace

extern "C" {

enum { OR_GREEDY = 0, OR_GAP = 1, OR_REL = 2 };
enum { OR_STOP_CERT = 0, OR_STOP_OFF = 1, OR_STOP_SCORE = 2 };
enum { OR_OK = 0, OR_MAXROT = 1, OR_STALL = 2, OR_NONFINITE = 3 };

struct OrStats {
  long long rotations;
  long long rescans;
  double final_sel;   // selection score of the last candidate pivot
  double final_cert;  // max_{i != j} L_ij at exit
  double final_off;   // sqrt(sum_{i != j} a_ij^2) at exit
  int status;
};

double orc_score_gap(double aii, double ajj, double aij) { return gap_score(aii, ajj, aij); }

double orc_score_rel(double aii, double ajj, double aij) { return rel_score(aii, ajj, aij); }

void orc_rotation(double app, double aqq, double apq, double* t, double* c, double* s) {
  rotation<double>(app, aqq, apq, t, c, s);
}

// Two-sided Jacobi (Algorithm 1) on the full symmetric row-major n x n matrix A, in place.
//   pivot : 0 greedy |a_ij|, 1 gap-aware L_ij (eq. (1))
//   stop  : 0 max L_ij <= thr (Theorem 1 certificate), 1 off(A) <= thr, 2 best selection score <= thr
//   scan  : 0 full O(n^2) scan per rotation, 1 per-row best cache (Sec. 3.2)
//   VJ    : optional n x n row-major, set to the product of the rotations (starts at I)
//   plog  : optional int[2*logcap] pivots (p, q), 0-based, p < q
//   cslog : optional double[2*logcap] (c, s) of each rotation
int orc_jacobi(double* A, int n, int pivot, int stop, double thr, long long maxrot, int scan,
               double* VJ, int* plog, double* cslog, long long logcap, OrStats* st) {
  Matrix m{A, n};
  std::memset(st, 0, sizeof(*st));
  for (long long i = 0; i < (long long)n * n; ++i)
    if (!std::isfinite(A[i])) {
      st->status = OR_NONFINITE;
      return OR_NONFINITE;
    }
  if (VJ) {
    std::fill(VJ, VJ + (size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) VJ[(size_t)i * n + i] = 1.0;
  }
  RowCache sel{pivot}, cert{OR_GAP};
  std::vector<double> off2;
  bool need_cert = (stop == OR_STOP_CERT);
  if (scan == 1) {
    sel.build(m);
    if (need_cert && pivot != OR_GAP) cert.build(m);
    off2.resize(n);
    for (int k = 0; k < n; ++k) off2[k] = row_off2(m, k);
  }
  long long rot = 0;
  int status = OR_OK;
  double vsel = 0.0, vcert = 0.0, voff = 0.0;
  for (;;) {
    int p = -1, q = -1;
    // --- pivot candidate and stop quantities
    if (scan == 0) {
      vsel = -1.0;
      vcert = 0.0;
      double s2 = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
          double v = pair_score(m, i, j, pivot);
          if (v > vsel) {
            vsel = v;
            p = i;
            q = j;
          }
          double l = gap_score(m.at(i, i), m.at(j, j), m.at(i, j));
          if (l > vcert) vcert = l;
          s2 += m.at(i, j) * m.at(i, j);
        }
      voff = std::sqrt(2.0 * s2);
    } else {
      sel.argmax(&vsel, &p, &q);
      if (pivot == OR_GAP) {
        vcert = vsel;
      } else if (need_cert) {
        int a, b;
        cert.argmax(&vcert, &a, &b);
      }
      double s2 = 0.0;
      for (int k = 0; k < n; ++k) s2 += off2[k];
      voff = std::sqrt(s2);
    }
    if (n < 2) break;
    if (stop == OR_STOP_CERT && vcert <= thr) break;
    if (stop == OR_STOP_OFF && voff <= thr) break;
    if (stop == OR_STOP_SCORE && vsel <= thr) break;
    if (rot >= maxrot) {
      status = OR_MAXROT;
      break;
    }
    double apq = m.at(p, q);
    if (apq == 0.0) {  // the best candidate has nothing to annihilate
      status = OR_STALL;
      break;
    }
    // --- rotation (Sec. 2): A <- G^T A G with G = G(c, s, p, q)
    double t, c, s;
    rotation<double>(m.at(p, p), m.at(q, q), apq, &t, &c, &s);
    for (int k = 0; k < n; ++k) {
      if (k == p || k == q) continue;
      double akp = m.at(k, p), akq = m.at(k, q);
      double xn = c * akp + s * akq;
      double yn = c * akq - s * akp;
      A[(size_t)k * n + p] = xn;
      A[(size_t)p * n + k] = xn;
      A[(size_t)k * n + q] = yn;
      A[(size_t)q * n + k] = yn;
    }
    double app = m.at(p, p), aqq = m.at(q, q);
    A[(size_t)p * n + p] = app + t * apq;
    A[(size_t)q * n + q] = aqq - t * apq;
    A[(size_t)p * n + q] = 0.0;
    A[(size_t)q * n + p] = 0.0;
    if (VJ) {
      for (int i = 0; i < n; ++i) {
        double vp = VJ[(size_t)i * n + p], vq = VJ[(size_t)i * n + q];
        VJ[(size_t)i * n + p] = c * vp + s * vq;
        VJ[(size_t)i * n + q] = c * vq - s * vp;
      }
    }
    if (plog && rot < logcap) {
      plog[2 * rot] = p;
      plog[2 * rot + 1] = q;
    }
    if (cslog && rot < logcap) {
      cslog[2 * rot] = c;
      cslog[2 * rot + 1] = s;
    }
    ++rot;
    if (scan == 1) {
      sel.refresh(m, p, q);
      if (need_cert && pivot != OR_GAP) cert.refresh(m, p, q);
      off2[p] = row_off2(m, p);
      off2[q] = row_off2(m, q);
    }
  }
  st->rotations = rot;
  st->rescans = sel.rescans + cert.rescans;
  st->final_sel = vsel;
  st->final_cert = vcert;
  st->final_off = voff;
  st->status = status;
  return status;
}

// Low-precision spectral decomposition (Sec. 2.1): cyclic-by-rows two-sided Jacobi in
// FP32 on the full symmetric row-major A32 (in place), accumulating V32 (row-major,
// starts at I).  A sweep visits every pair (p, q), p < q, in row order.  Sweeps stop once
// off(A32) <= tol * ||A32||_F, once a sweep fails to reduce off(A32), or after max_sweeps.
// Returns the number of sweeps performed.
// Cyclic-by-rows FP32 Jacobi (the low-precision decomposition of Sec. 2.1, whose method the
// paper leaves open).  A pair is skipped when a_pq and a_pp - a_qq both lie within
// 2^-22 (|a_pp| + |a_qq|): at that level FP32 cannot separate the two eigenvalues and the
// rotation angle would be decided by rounding; the FP64 phase resolves such pairs.  Sweeps
// stop at off <= tol ||A32||_F, when a sweep leaves off >= rho times its previous value,
// or after max_sweeps.
static bool f32_noise_pair(float app, float aqq, float apq) {
  float nz = 0x1p-22f * (std::fabs(app) + std::fabs(aqq));
  return std::fabs(app - aqq) <= nz && std::fabs(apq) <= nz;
}

// verbose != 0: one line per sweep on stderr (progress of long runs).
int orc_jacobi_f32(float* A32, int n, float* V32, int max_sweeps, double tol, double rho,
                   int verbose) {
  std::fill(V32, V32 + (size_t)n * n, 0.0f);
  for (int i = 0; i < n; ++i) V32[(size_t)i * n + i] = 1.0f;
  auto off_and_norm = [&](double* off, double* nrm) {
    double so = 0.0, sd = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double v = A32[(size_t)i * n + j];
        if (i == j)
          sd += v * v;
        else
          so += v * v;
      }
    *off = std::sqrt(so);
    *nrm = std::sqrt(so + sd);
  };
  double off, nrm;
  off_and_norm(&off, &nrm);
  int sweeps = 0;
  while (sweeps < max_sweeps && off > tol * nrm) {
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        float apq = A32[(size_t)p * n + q];
        if (apq == 0.0f) continue;
        if (f32_noise_pair(A32[(size_t)p * n + p], A32[(size_t)q * n + q], apq)) continue;
        float t, c, s;
        rotation<float>(A32[(size_t)p * n + p], A32[(size_t)q * n + q], apq, &t, &c, &s);
        for (int k = 0; k < n; ++k) {
          if (k == p || k == q) continue;
          float akp = A32[(size_t)k * n + p], akq = A32[(size_t)k * n + q];
          float xn = c * akp + s * akq;
          float yn = c * akq - s * akp;
          A32[(size_t)k * n + p] = xn;
          A32[(size_t)p * n + k] = xn;
          A32[(size_t)k * n + q] = yn;
          A32[(size_t)q * n + k] = yn;
        }
        float app = A32[(size_t)p * n + p], aqq = A32[(size_t)q * n + q];
        A32[(size_t)p * n + p] = app + t * apq;
        A32[(size_t)q * n + q] = aqq - t * apq;
        A32[(size_t)p * n + q] = 0.0f;
        A32[(size_t)q * n + p] = 0.0f;
        for (int i = 0; i < n; ++i) {
          float vp = V32[(size_t)i * n + p], vq = V32[(size_t)i * n + q];
          V32[(size_t)i * n + p] = c * vp + s * vq;
          V32[(size_t)i * n + q] = c * vq - s * vp;
        }
      }
    ++sweeps;
    double prev = off;
    off_and_norm(&off, &nrm);
    if (verbose) std::fprintf(stderr, "oracle fp32 sweep %d: off/norm %.3e\n", sweeps, off / nrm);
    if (off >= rho * prev) break;
  }
  return sweeps;
}


// Dot product of rows i and j of the row-major n x m array X, summed in index order.
static double dot_rows(const double* X, int m, int i, int j) {
  const double* x = X + (size_t)i * m;
  const double* y = X + (size_t)j * m;
  double s = 0.0;
  for (int r = 0; r < m; ++r) s += x[r] * y[r];
  return s;
}

// One-sided Jacobi SVD (Algorithm 2) of B (m x n, m >= n), held transposed: row k of the
// row-major n x m array X is column b_k of B.  A pivot (p, q) is chosen on the Gram matrix
// A = B^T B (the matrix the pivot scores of Sec. 3 are evaluated on, Sec. 2.1), the rotation
// that makes b_p and b_q orthogonal is the one that diagonalises [[a_pp, a_pq], [a_pq, a_qq]]
// (Sec. 2), and B <- B G(c, s, p, q).  A is never rotated: every entry is the dot product of
// the current columns (dot_rows), so after the rotation rows p and q of A are recomputed.
//   pivot : 0 greedy |a_ij|, 1 gap L_ij (eq. (1)), 2 relative Lhat_ij (Sec. 4.2)
//   stop  : the best selection score is <= thr, or maxrot rotations
//   scan  : 0 full O(n^2) scan per rotation, 1 per-row best cache (Sec. 3.2)
//   Vt    : optional n x n row-major; its rows are rotated with those of X (so Vt^T = V
//           accumulates B's right factor); the caller initialises it
//   G     : n x n row-major output: A of the final columns
//   plog, cslog : optional logs of (p, q) and (c, s)
int orc_svd1(double* X, int m, int n, int pivot, double thr, long long maxrot, int scan,
             double* Vt, double* G, int* plog, double* cslog, long long logcap, OrStats* st) {
  std::memset(st, 0, sizeof(*st));
  for (long long i = 0; i < (long long)n * m; ++i)
    if (!std::isfinite(X[i])) {
      st->status = OR_NONFINITE;
      return OR_NONFINITE;
    }
  Matrix g{G, n};
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double v = dot_rows(X, m, i, j);
      G[(size_t)i * n + j] = v;
      G[(size_t)j * n + i] = v;
    }
  RowCache sel{pivot};
  if (scan == 1) sel.build(g);
  long long rot = 0;
  int status = OR_OK;
  double vsel = 0.0;
  for (;;) {
    int p = -1, q = -1;
    if (scan == 0) {
      vsel = -1.0;
      for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
          double v = pair_score(g, i, j, pivot);
          if (v > vsel) {
            vsel = v;
            p = i;
            q = j;
          }
        }
    } else {
      sel.argmax(&vsel, &p, &q);
    }
    if (n < 2) break;
    if (vsel <= thr) break;
    if (rot >= maxrot) {
      status = OR_MAXROT;
      break;
    }
    double apq = g.at(p, q);
    if (apq == 0.0) {
      status = OR_STALL;
      break;
    }
    double t, c, s;
    rotation<double>(g.at(p, p), g.at(q, q), apq, &t, &c, &s);
    // [b_p, b_q] <- [b_p, b_q] [[c, -s], [s, c]]
    double* xp = X + (size_t)p * m;
    double* xq = X + (size_t)q * m;
    for (int r = 0; r < m; ++r) {
      double u = xp[r], w = xq[r];
      xp[r] = c * u + s * w;
      xq[r] = c * w - s * u;
    }
    if (Vt) {
      double* vp = Vt + (size_t)p * n;
      double* vq = Vt + (size_t)q * n;
      for (int r = 0; r < n; ++r) {
        double u = vp[r], w = vq[r];
        vp[r] = c * u + s * w;
        vq[r] = c * w - s * u;
      }
    }
    if (plog && rot < logcap) {
      plog[2 * rot] = p;
      plog[2 * rot + 1] = q;
    }
    if (cslog && rot < logcap) {
      cslog[2 * rot] = c;
      cslog[2 * rot + 1] = s;
    }
    ++rot;
    for (int k = 0; k < n; ++k) {
      double v = dot_rows(X, m, p, k);
      G[(size_t)p * n + k] = v;
      G[(size_t)k * n + p] = v;
    }
    for (int k = 0; k < n; ++k) {
      if (k == p) continue;
      double v = dot_rows(X, m, q, k);
      G[(size_t)q * n + k] = v;
      G[(size_t)k * n + q] = v;
    }
    if (scan == 1) sel.refresh(g, p, q);
  }
  st->rotations = rot;
  st->rescans = sel.rescans;
  st->final_sel = vsel;
  st->status = status;
  return status;
}

}  // extern "C"
