// One-sided Jacobi SVD (Algorithm 2) with the pivot scores of Sec. 3 evaluated on the Gram
// matrix A = B^T B (Sec. 2.1), including the relative score of Sec. 4.2.
//
// Layout: B (m x n, m >= n) is held row-major, Y[r][k] = b_rk with row stride ldy, so that
// the lanes computing a_pk for consecutive k read consecutive addresses while b_rp is a
// broadcast.  A is row-major n x n.  A is never rotated: every entry is the dot product of
// the current columns summed in index order (one lane per entry, no split of the sum), and
// after a rotation of columns p and q the rows p and q of A are recomputed.  With
// -ffp-contract=off every value is then a function of the input bits alone.
//
// One persistent workgroup runs the whole rotation sequence.  When B and the per-row state
// fit, B lives in LDS for the whole run (written back at the end); otherwise it stays in
// HBM.  Per rotation:
//   argmax over the per-row best scores (each wave redundantly: no cross-wave exchange),
//   rotation of columns p, q of B and of rows p, q of the right factor V^T, barrier,
//   the dot products of rows p and q of A, barrier,
//   per-row cache refresh (Sec. 3.2), rows needing a full rescan queued in LDS, barrier,
//   full rescans, one wave per queued row, barrier.
#include "device_common.h"
#include "kernels.h"

namespace je {

// Relative score of Sec. 4.2, (1/a_ii + 1/a_jj) L_ij: the sum of the relative shifts of the
// two eigenvalues of the 2 x 2 block.  It is invariant under scaling of the block, so the
// entries are first multiplied by the power of two that brings max(a_ii, a_jj) into
// [1/2, 1) (exact): a pair of tiny columns keeps a_ij^2 in range.  0 when a_ij == 0 or the
// scaled a_ij^2 underflows.
__device__ __forceinline__ double rel_score(double aii, double ajj, double aij) {
  if (aij == 0.0) return 0.0;
  int e;
  (void)frexp(fmax(aii, ajj), &e);
  const double x = ldexp(aii, -e), y = ldexp(ajj, -e), a = ldexp(aij, -e);
  const double l = gap_score(x, y, a);
  if (l == 0.0) return 0.0;
  return (1.0 / x + 1.0 / y) * l;
}

// PIV: 0 greedy |a_ij|, 1 gap L_ij (eq. (1)), 2 relative (Sec. 4.2)
template <int PIV>
__device__ __forceinline__ double svd_score(double aii, double ajj, double aij) {
  if constexpr (PIV == 0) return fabs(aij);
  else if constexpr (PIV == 1) return gap_score(aii, ajj, aij);
  else return rel_score(aii, ajj, aij);
}

// (score, index) maximum over the wave: larger score, then smaller index.  Every lane ends
// with the result.
__device__ __forceinline__ void wave_best(double& v, int& k) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int ok = __shfl_xor(k, o);
    if (ov > v || (ov == v && ok < k)) {
      v = ov;
      k = ok;
    }
  }
}

// ------------------------------------------------------------------ set-up kernels
// Y[r][k] = B[r + k ldb]; flags a non-finite entry.  32 x 32 tiles through LDS so that
// both the column-major reads and the row-major writes are coalesced.
__global__ __launch_bounds__(256) void k_svd_load(const double* __restrict__ B, int m, int n,
                                                  int ldb, double* __restrict__ Y, int ldy,
                                                  int* __restrict__ flag) {
  __shared__ double t[32][33];
  const int r0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty in [0, 8)
  bool bad = false;
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + tx, k = k0 + j;
    if (r < m && k < n) {
      const double v = B[(size_t)k * ldb + r];
      bad |= !isfinite(v);
      t[j][tx] = v;
    }
  }
  if (bad) *flag = 1;
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + j, k = k0 + tx;
    if (r < m && k < n) Y[(size_t)r * ldy + k] = t[tx][j];
  }
}

// A = B^T B: entry (i, j), i <= j, by one lane (j across the lanes of a row of 16), summed
// in index order, mirrored.
__global__ __launch_bounds__(256) void k_svd_gram(const double* __restrict__ Y, int ldy, int m,
                                                  int n, double* __restrict__ G, int ldg) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= n || j >= n || i > j) return;
  double s = 0.0;
#pragma unroll 8
  for (int r = 0; r < m; ++r) s += Y[(size_t)r * ldy + i] * Y[(size_t)r * ldy + j];
  G[(size_t)i * ldg + j] = s;
  G[(size_t)j * ldg + i] = s;
}

// Best (score, column) of every row, one wave per row (smallest column on ties); also the
// diagonal of A.
template <int PIV>
__global__ __launch_bounds__(256) void k_svd_rowbest(const double* __restrict__ G, int ldg,
                                                     int n, double* __restrict__ best,
                                                     int* __restrict__ arg,
                                                     double* __restrict__ diag) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n) return;
  const double* gk = G + (size_t)k * ldg;
  const double akk = gk[k];
  double v = -1.0;
  int c = INT_MAX;
  for (int l = lane; l < n; l += 64) {
    if (l == k) continue;
    const double x = svd_score<PIV>(akk, G[(size_t)l * ldg + l], gk[l]);
    if (x > v) {
      v = x;
      c = l;
    }
  }
  wave_best(v, c);
  if (lane == 0) {
    best[k] = v;
    arg[k] = c == INT_MAX ? -1 : c;
    diag[k] = akk;
  }
}

// Z = Y Q (Z[r][k] = sum_i Y[r][i] Q[i][k], summed in index order): B times the
// preconditioner.
__global__ __launch_bounds__(256) void k_svd_rowmix(const double* __restrict__ Y, int ldy,
                                                    const double* __restrict__ Q, int ldq,
                                                    int m, int n, double* __restrict__ Z,
                                                    int ldz) {
  const int r = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const double* yr = Y + (size_t)r * ldy;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += yr[i] * Q[(size_t)i * ldq + k];
  Z[(size_t)r * ldz + k] = s;
}

// Vt = Q^T.
__global__ __launch_bounds__(256) void k_svd_transpose(const double* __restrict__ Q, int ldq,
                                                       int n, double* __restrict__ Vt,
                                                       int ldv) {
  const int k = blockIdx.y;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    Vt[(size_t)k * ldv + i] = Q[(size_t)i * ldq + k];
}

// ------------------------------------------------------------------ the rotation sequence
// Barrier for phases that communicate through LDS only: waits for this wave's LDS accesses,
// not for its stores to device memory (which no other wave reads before the kernel ends).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave-uniform (score, index) maximum, larger score then smaller index, of per-lane
// candidates (v < 0: none).  Returns false when no lane has a candidate.
__device__ __forceinline__ bool wave_best_fast(double& v, int& k) {
  const int w = wave_argmax_lane(v, k);
  if (w < 0) return false;
  v = readlane_d(v, w);
  k = readlane_i(k, w);
  return true;
}

// Packed upper triangle: position of (i, j), i <= j, of an n x n symmetric matrix.
__device__ __forceinline__ int tri(int i, int j, int n) { return i * (2 * n - i - 1) / 2 + j; }

// LDS bytes of the resident mode: B with an odd row stride (the column accesses of the
// rotation then fall in distinct banks), A as a packed upper triangle, the new columns p
// and q contiguous, and best, diag, rows p and q of A, arg and the rescan queue.
__host__ __device__ __forceinline__ int svd_lds_ld(int n) { return n | 1; }
__host__ __device__ __forceinline__ size_t svd_lds_bytes(int m, int n) {
  return 8 * ((size_t)m * svd_lds_ld(n) + (size_t)n * (n + 1) / 2 + 2 * (size_t)m +
              4 * (size_t)n) +
         8 * (size_t)n;
}

// Resident mode: B and A stay in LDS for the whole run, every exchange between waves goes
// through LDS.  Per rotation:
//   B  (all lanes) argmax, rotation parameters, columns p and q of B rotated in place and
//      copied contiguously; this lane's entries of rows p, q of V^T loaded (each lane owns
//      the same entries for the whole run).                                      barrier
//   C  the 2n dot products of rows p and q of A, one per lane; V^T entries stored.
//                                                                                barrier
//   D  A's rows p, q and diagonal stored; per-row cache refresh with rows whose cached best
//      moved down queued; full rescans of rows p and q by two waves (entries stored by
//      other lanes in this phase, diag[p] and diag[q], are taken from rows p, q).  barrier
//   E  (only if the queue is not empty) full rescans of the queued rows.          barrier
template <int PIV>
__global__ __launch_bounds__(256) void k_svd_res(const SDesc d) {
  constexpr int NT = 256, NW = NT / 64;
  extern __shared__ double smem[];
  __shared__ int s_cnt, s_resc;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = d.n, m = d.m, ldy = svd_lds_ld(n);
  const size_t ldv = d.ldv, ldg = d.ldg;
  double* Y = smem;
  double* Gp = Y + (size_t)m * ldy;
  double* colp = Gp + (size_t)n * (n + 1) / 2;
  double* colq = colp + m;
  double* best = colq + m;
  double* diag = best + n;
  double* rowp = diag + n;
  double* rowq = rowp + n;
  int* arg = (int*)(rowq + n);
  int* list = arg + n;
  for (int i = tid; i < m * n; i += NT) {
    const int r = i / n, k = i - r * n;
    Y[r * ldy + k] = d.Y[(size_t)r * d.ldy + k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + tid; j < n; j += NT) Gp[tri(i, j, n)] = d.G[(size_t)i * ldg + j];
  for (int k = tid; k < n; k += NT) {
    best[k] = d.best[k];
    arg[k] = d.arg[k];
    diag[k] = d.diag[k];
  }
  if (tid == 0) {
    s_resc = 0;
    s_cnt = 0;
  }
  __syncthreads();
  long long rot = 0;
  int status = ST_OK;
  double vsel = -1.0;
  for (;;) {
    // ---- B
    double v = -1.0;
    int r = INT_MAX;
    for (int k = lane; k < n; k += 64) {
      const double x = best[k];
      if (x > v) {
        v = x;
        r = k;
      }
    }
    if (!wave_best_fast(v, r)) v = -1.0;
    vsel = v;
    if (n < 2 || v <= d.thr) break;
    if (rot >= d.maxrot) {
      status = ST_MAXROT;
      break;
    }
    const int a = arg[r];
    const int p = min(r, a), q = max(r, a);
    const double apq = Gp[tri(p, q, n)];
    if (apq == 0.0) {
      status = ST_STALL;
      break;
    }
    double t, c, s;
    rot_params<double>(diag[p], diag[q], apq, t, c, s);
    // this lane's entries of rows p, q of V^T (n <= NT here): loaded now, stored after the
    // dot products so that the memory latency overlaps them
    const bool hv = d.Vt != nullptr && tid < n;
    double vu = 0.0, vw = 0.0;
    if (hv) {
      vu = d.Vt[(size_t)p * ldv + tid];
      vw = d.Vt[(size_t)q * ldv + tid];
    }
    if (tid == 0 && d.plog && rot < d.logcap) {
      d.plog[2 * rot] = p;
      d.plog[2 * rot + 1] = q;
    }
    ++rot;
    for (int i = tid; i < m; i += NT) {
      double* yi = Y + i * ldy;
      const double u = yi[p], w = yi[q];
      const double np_ = c * u + s * w, nq_ = c * w - s * u;
      yi[p] = np_;
      yi[q] = nq_;
      colp[i] = np_;
      colq[i] = nq_;
    }
    lds_barrier();
    // ---- C: a_pk = sum_i b_ip b_ik (tasks 0..n-1) and a_qk = sum_i b_iq b_ik (tasks n..2n-1),
    // each by one lane in index order; the loads of a block of rows are issued before its sums
    for (int task = tid; task < 2 * n; task += NT) {
      const bool onp = task < n;
      const int k = onp ? task : task - n;
      const double* yc = onp ? colp : colq;
      const double* yk = Y + k;
      constexpr int kB = 8;
      double x = 0.0;
      int i = 0;
      for (; i + kB <= m; i += kB) {
        double u[kB], z[kB];
#pragma unroll
        for (int e = 0; e < kB; ++e) {
          u[e] = yc[i + e];
          z[e] = yk[(i + e) * ldy];
        }
#pragma unroll
        for (int e = 0; e < kB; ++e) x += u[e] * z[e];
      }
      for (; i < m; ++i) x += yc[i] * yk[i * ldy];
      (onp ? rowp : rowq)[k] = x;
    }
    if (hv) {
      d.Vt[(size_t)p * ldv + tid] = c * vu + s * vw;
      d.Vt[(size_t)q * ldv + tid] = c * vw - s * vu;
    }
    lds_barrier();
    // ---- D
    const double app = rowp[p], aqq = rowq[q];
    for (int k = tid; k < n; k += NT) {
      // a_pq is stored once, from row p (the same bits as rowq[p])
      Gp[tri(min(p, k), max(p, k), n)] = rowp[k];
      if (k != p) Gp[tri(min(q, k), max(q, k), n)] = rowq[k];
      if (k == p) {
        diag[p] = app;
        continue;
      }
      if (k == q) {
        diag[q] = aqq;
        continue;
      }
      const double akk = diag[k];
      const double sp = svd_score<PIV>(akk, app, rowp[k]);
      const double sq = svd_score<PIV>(akk, aqq, rowq[k]);
      double b = best[k];
      int ak = arg[k];
      if (ak == p || ak == q) {
        double x = sp;
        int col = p;
        if (sq > x) {
          x = sq;
          col = q;
        }
        if (x > b || (x == b && col <= ak)) {
          best[k] = x;
          arg[k] = col;
        } else {
          list[atomicAdd(&s_cnt, 1)] = k;
          atomicAdd(&s_resc, 1);
        }
      } else {
        if (sp > b || (sp == b && p < ak)) {
          b = sp;
          ak = p;
        }
        if (sq > b || (sq == b && q < ak)) {
          b = sq;
          ak = q;
        }
        best[k] = b;
        arg[k] = ak;
      }
    }
    if (wv >= NW - 2) {
      // rows p and q: their entries are rowp / rowq; diag[p], diag[q] are being stored in
      // this phase, so their new values are taken from rowp[p], rowq[q]
      const int k = wv == NW - 2 ? p : q;
      const double* gk = wv == NW - 2 ? rowp : rowq;
      const double akk = gk[k];
      double bv = -1.0;
      int bc = INT_MAX;
      for (int l = lane; l < n; l += 64) {
        if (l == k) continue;
        const double all = l == p ? app : (l == q ? aqq : diag[l]);
        const double x = svd_score<PIV>(akk, all, gk[l]);
        if (x > bv) {
          bv = x;
          bc = l;
        }
      }
      wave_best_fast(bv, bc);
      if (lane == 0) {
        best[k] = bv;
        arg[k] = bc;
      }
    }
    lds_barrier();
    // ---- E
    const int cnt = s_cnt;
    if (cnt > 0) {
      for (int e = wv; e < cnt; e += NW) {
        const int k = list[e];
        const double akk = diag[k];
        double bv = -1.0;
        int bc = INT_MAX;
        for (int l = lane; l < n; l += 64) {
          if (l == k) continue;
          const double x = svd_score<PIV>(akk, diag[l], Gp[tri(min(k, l), max(k, l), n)]);
          if (x > bv) {
            bv = x;
            bc = l;
          }
        }
        wave_best_fast(bv, bc);
        if (lane == 0) {
          best[k] = bv;
          arg[k] = bc;
        }
      }
      lds_barrier();
      if (tid == 0) s_cnt = 0;
    }
  }
  __syncthreads();
  for (int i = tid; i < m * n; i += NT) {
    const int r = i / n, k = i - r * n;
    d.Y[(size_t)r * d.ldy + k] = Y[r * ldy + k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + tid; j < n; j += NT) {
      const double x = Gp[tri(i, j, n)];
      d.G[(size_t)i * ldg + j] = x;
      d.G[(size_t)j * ldg + i] = x;
    }
  if (tid == 0) {
    d.ctl->rotations = rot;
    d.ctl->rescans = s_resc;
    d.ctl->status = status;
    d.ctl->done = 1;
    d.ctl->final_sel = vsel;
  }
}

// HBM mode (B too large for LDS): B, A and the per-row state in device memory, the rescan
// queue in LDS; the same steps with full barriers.
template <int PIV, int NT>
__global__ __launch_bounds__(NT) void k_svd1(const SDesc d) {
  constexpr int NW = NT / 64;
  extern __shared__ int list[];
  __shared__ int s_cnt, s_resc;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = d.n, m = d.m;
  double* __restrict__ G = d.G;
  double* __restrict__ Y = d.Y;
  double* __restrict__ best = d.best;
  double* __restrict__ diag = d.diag;
  double* __restrict__ rowp = d.rowp;
  double* __restrict__ rowq = d.rowq;
  int* __restrict__ arg = d.arg;
  const size_t ldg = d.ldg, ldv = d.ldv, ldy = d.ldy;
  if (tid == 0) s_resc = 0;
  __syncthreads();
  long long rot = 0;
  int status = ST_OK;
  double vsel = -1.0;
  for (;;) {
    double v = -1.0;
    int r = INT_MAX;
    for (int k = lane; k < n; k += 64) {
      const double x = best[k];
      if (x > v) {
        v = x;
        r = k;
      }
    }
    if (!wave_best_fast(v, r)) v = -1.0;
    vsel = v;
    if (n < 2 || v <= d.thr) break;
    if (rot >= d.maxrot) {
      status = ST_MAXROT;
      break;
    }
    const int a = arg[r];
    const int p = min(r, a), q = max(r, a);
    const double apq = G[(size_t)p * ldg + q];
    if (apq == 0.0) {
      status = ST_STALL;
      break;
    }
    double t, c, s;
    rot_params<double>(diag[p], diag[q], apq, t, c, s);
    for (int i = tid; i < m; i += NT) {
      double* yi = Y + (size_t)i * ldy;
      const double u = yi[p], w = yi[q];
      yi[p] = c * u + s * w;
      yi[q] = c * w - s * u;
    }
    if (d.Vt) {
      double* vp = d.Vt + (size_t)p * ldv;
      double* vq = d.Vt + (size_t)q * ldv;
      for (int i = tid; i < n; i += NT) {
        const double u = vp[i], w = vq[i];
        vp[i] = c * u + s * w;
        vq[i] = c * w - s * u;
      }
    }
    if (tid == 0) {
      if (d.plog && rot < d.logcap) {
        d.plog[2 * rot] = p;
        d.plog[2 * rot + 1] = q;
      }
      s_cnt = 0;
    }
    ++rot;
    __syncthreads();
    // both dot products of column k in one pass over B
    for (int k = tid; k < n; k += NT) {
      constexpr int kB = 16;
      double xp = 0.0, xq = 0.0;
      int i = 0;
      for (; i + kB <= m; i += kB) {
        double u[kB], w[kB], z[kB];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
          const double* yi = Y + (size_t)(i + j) * ldy;
          u[j] = yi[p];
          w[j] = yi[q];
          z[j] = yi[k];
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
          xp += u[j] * z[j];
          xq += w[j] * z[j];
        }
      }
      for (; i < m; ++i) {
        const double* yi = Y + (size_t)i * ldy;
        const double yk = yi[k];
        xp += yi[p] * yk;
        xq += yi[q] * yk;
      }
      rowp[k] = xp;
      rowq[k] = xq;
      G[(size_t)p * ldg + k] = xp;
      G[(size_t)k * ldg + p] = xp;
      G[(size_t)q * ldg + k] = xq;
      G[(size_t)k * ldg + q] = xq;
      if (k == p) diag[p] = xp;
      if (k == q) diag[q] = xq;
    }
    __syncthreads();
    const double app = diag[p], aqq = diag[q];
    for (int k = tid; k < n; k += NT) {
      if (k == p || k == q) {
        list[atomicAdd(&s_cnt, 1)] = k;
        continue;
      }
      const double akk = diag[k];
      const double sp = svd_score<PIV>(akk, app, rowp[k]);
      const double sq = svd_score<PIV>(akk, aqq, rowq[k]);
      double b = best[k];
      int ak = arg[k];
      if (ak == p || ak == q) {
        double x = sp;
        int col = p;
        if (sq > x) {
          x = sq;
          col = q;
        }
        if (x > b || (x == b && col <= ak)) {
          best[k] = x;
          arg[k] = col;
        } else {
          list[atomicAdd(&s_cnt, 1)] = k;
          atomicAdd(&s_resc, 1);
        }
      } else {
        if (sp > b || (sp == b && p < ak)) {
          b = sp;
          ak = p;
        }
        if (sq > b || (sq == b && q < ak)) {
          b = sq;
          ak = q;
        }
        best[k] = b;
        arg[k] = ak;
      }
    }
    __syncthreads();
    const int cnt = s_cnt;
    for (int e = wv; e < cnt; e += NW) {
      const int k = list[e];
      const double* gk = G + (size_t)k * ldg;
      const double akk = diag[k];
      double bv = -1.0;
      int bc = INT_MAX;
      for (int l = lane; l < n; l += 64) {
        if (l == k) continue;
        const double x = svd_score<PIV>(akk, diag[l], gk[l]);
        if (x > bv) {
          bv = x;
          bc = l;
        }
      }
      wave_best_fast(bv, bc);
      if (lane == 0) {
        best[k] = bv;
        arg[k] = bc;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    d.ctl->rotations = rot;
    d.ctl->rescans = s_resc;
    d.ctl->status = status;
    d.ctl->done = 1;
    d.ctl->final_sel = vsel;
  }
}

// ------------------------------------------------------------------ output
// rank[k] = position of column k in descending order of sigma_k = sqrt(a_kk) (stable);
// S[rank[k]] = sigma_k.
__global__ __launch_bounds__(256) void k_svd_rank(const double* __restrict__ G, int ldg, int n,
                                                  int* __restrict__ rank, double* __restrict__ S) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const double sk = sqrt(G[(size_t)k * ldg + k]);
  int rk = 0;
  for (int j = 0; j < n; ++j) {
    const double sj = sqrt(G[(size_t)j * ldg + j]);
    rk += (sj > sk) || (sj == sk && j < k);
  }
  rank[k] = rk;
  S[rk] = sk;
}

// U[:, rank k] = b_k / sigma_k (0 when sigma_k == 0); V[:, rank k] = row k of Vt.
__global__ __launch_bounds__(256) void k_svd_vectors(const double* __restrict__ Y, int ldy, int m,
                                                     const double* __restrict__ G, int ldg,
                                                     const double* __restrict__ Vt, int ldvt,
                                                     int n, const int* __restrict__ rank,
                                                     double* __restrict__ U, int ldu,
                                                     double* __restrict__ V, int ldv) {
  const int k = blockIdx.y;
  const int rk = rank[k];
  const double sk = sqrt(G[(size_t)k * ldg + k]);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
    if (U) U[(size_t)rk * ldu + i] = sk > 0.0 ? Y[(size_t)i * ldy + k] / sk : 0.0;
    if (V && i < n) V[(size_t)rk * ldv + i] = Vt[(size_t)k * ldvt + i];
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_svd_load(const double* B, int m, int n, int ldb, double* Y, int ldy, int* flag,
                           hipStream_t s) {
  dim3 g((m + 31) / 32, (n + 31) / 32);
  hipLaunchKernelGGL(k_svd_load, g, dim3(256), 0, s, B, m, n, ldb, Y, ldy, flag);
  return hipGetLastError();
}

hipError_t launch_svd_gram(const double* Y, int ldy, int m, int n, double* G, int ldg,
                           hipStream_t s) {
  dim3 g((n + 15) / 16, (n + 15) / 16);
  hipLaunchKernelGGL(k_svd_gram, g, dim3(256), 0, s, Y, ldy, m, n, G, ldg);
  return hipGetLastError();
}

hipError_t launch_svd_rowmix(const double* Y, int ldy, const double* Q, int ldq, int m, int n,
                             double* Z, int ldz, hipStream_t s) {
  dim3 g((n + 255) / 256, m);
  hipLaunchKernelGGL(k_svd_rowmix, g, dim3(256), 0, s, Y, ldy, Q, ldq, m, n, Z, ldz);
  return hipGetLastError();
}

hipError_t launch_svd_transpose(const double* Q, int ldq, int n, double* Vt, int ldv,
                                hipStream_t s) {
  dim3 g((n + 255) / 256, n);
  hipLaunchKernelGGL(k_svd_transpose, g, dim3(256), 0, s, Q, ldq, n, Vt, ldv);
  return hipGetLastError();
}

static int svd_max_lds() {
  static int v = -1;
  if (v < 0) {
    int dev = 0, x = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      x = 65536;
    v = x;
  }
  return v;
}

bool svd_resident(int m, int n) {
  // one lane per entry of a row of V^T; the static LDS of the kernel (two counters) and a
  // margin stay free
  return n <= 256 && svd_lds_bytes(m, n) + 1024 <= (size_t)svd_max_lds();
}

template <typename K>
static hipError_t svd_launch_main(K fn, int nt, size_t sh, const SDesc& d, hipStream_t s) {
  if (sh > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(1), dim3(nt), sh, s, d);
  return hipGetLastError();
}

template <int PIV>
static hipError_t svd_jacobi_t(const SDesc& d, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_rowbest<PIV>, dim3((d.n + 3) / 4), dim3(256), 0, s, d.G, d.ldg,
                     d.n, d.best, d.arg, d.diag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (svd_resident(d.m, d.n))
    return svd_launch_main(k_svd_res<PIV>, 256, svd_lds_bytes(d.m, d.n), d, s);
  // one workgroup; more lanes once the dot products of a rotation outnumber 256
  if (d.n > 256) return svd_launch_main(k_svd1<PIV, 1024>, 1024, (size_t)d.n * 4, d, s);
  return svd_launch_main(k_svd1<PIV, 256>, 256, (size_t)d.n * 4, d, s);
}

hipError_t launch_svd_jacobi(const SDesc& d, hipStream_t s) {
  if (d.n > kSvdMaxN) return hipErrorInvalidValue;
  if (d.pivot == 0) return svd_jacobi_t<0>(d, s);
  if (d.pivot == 1) return svd_jacobi_t<1>(d, s);
  return svd_jacobi_t<2>(d, s);
}

hipError_t launch_svd_out(const double* Y, int ldy, int m, const double* G, int ldg,
                          const double* Vt, int ldvt, int n, int* rank, double* S, double* U,
                          int ldu, double* V, int ldv, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_rank, dim3((n + 255) / 256), dim3(256), 0, s, G, ldg, n, rank, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || (!U && !V)) return e;
  dim3 g((m + 255) / 256, n);
  hipLaunchKernelGGL(k_svd_vectors, g, dim3(256), 0, s, Y, ldy, m, G, ldg, Vt, ldvt, n, rank, U,
                     ldu, V, ldv);
  return hipGetLastError();
}

}  // namespace je
