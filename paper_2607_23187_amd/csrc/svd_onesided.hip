// One-sided Jacobi SVD (Algorithm 2) with the pivot scores of Sec. 3 evaluated on the Gram
// matrix A = B^T B (Sec. 2.1), including the relative score of Sec. 4.2.
//
// Layout: B (m x n, m >= n) is held transposed, X = B^T row-major with row stride ldx, so
// that column b_k of B is the contiguous row k of X and rotating two columns of B touches
// two contiguous rows.  A is row-major n x n.  A is never rotated: every entry is the dot
// product of the current columns summed in index order (one lane per entry, no split of the
// sum), and after a rotation of columns p and q the rows p and q of A are recomputed.  With
// -ffp-contract=off every value is then a function of the input bits alone.
//
// One persistent workgroup runs the whole rotation sequence; per rotation:
//   argmax over the per-row best scores (each wave redundantly: no cross-wave exchange),
//   rotation of rows p, q of X and of the right factor, barrier,
//   2n - 1 dot products for rows p and q of A, barrier,
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

// Dot product of rows a and b of X, in index order.
__device__ __forceinline__ double dot_rows(const double* __restrict__ xa,
                                           const double* __restrict__ xb, int m) {
  double s = 0.0;
#pragma unroll 8
  for (int r = 0; r < m; ++r) s += xa[r] * xb[r];
  return s;
}

// ------------------------------------------------------------------ set-up kernels
// X[k][r] = B[r + k ldb]; flags a non-finite entry.
__global__ __launch_bounds__(256) void k_svd_load(const double* __restrict__ B, int m, int n,
                                                  int ldb, double* __restrict__ X, int ldx,
                                                  int* __restrict__ flag) {
  const int k = blockIdx.y;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < m; r += gridDim.x * 256) {
    const double v = B[(size_t)k * ldb + r];
    if (!isfinite(v)) *flag = 1;
    X[(size_t)k * ldx + r] = v;
  }
}

// A = X X^T, entry (i, j), i <= j, by one lane, mirrored.
__global__ __launch_bounds__(256) void k_svd_gram(const double* __restrict__ X, int ldx, int m,
                                                  int n, double* __restrict__ G, int ldg) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= n || j >= n || i > j) return;
  const double v = dot_rows(X + (size_t)i * ldx, X + (size_t)j * ldx, m);
  G[(size_t)i * ldg + j] = v;
  G[(size_t)j * ldg + i] = v;
}

// Best (score, column) of every row, one wave per row (smallest column on ties).
template <int PIV>
__global__ __launch_bounds__(256) void k_svd_rowbest(const double* __restrict__ G, int ldg,
                                                     int n, double* __restrict__ best,
                                                     int* __restrict__ arg) {
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
  }
}

// Y = Q^T X (Y[k][r] = sum_i Q[i][k] X[i][r], summed in index order): the columns of B Q.
__global__ __launch_bounds__(256) void k_svd_rowmix(const double* __restrict__ Q, int ldq,
                                                    const double* __restrict__ X, int ldx,
                                                    int n, int m, double* __restrict__ Y,
                                                    int ldy) {
  const int k = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= m) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += Q[(size_t)i * ldq + k] * X[(size_t)i * ldx + r];
  Y[(size_t)k * ldy + r] = s;
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
template <int PIV, int NT>
__global__ __launch_bounds__(NT) void k_svd1(const SDesc d) {
  constexpr int NW = NT / 64;
  __shared__ int s_list[kSvdMaxN];
  __shared__ int s_cnt, s_resc;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = d.n, m = d.m;
  double* __restrict__ X = d.X;
  double* __restrict__ G = d.G;
  double* __restrict__ best = d.best;
  int* __restrict__ arg = d.arg;
  const size_t ldx = d.ldx, ldg = d.ldg, ldv = d.ldv;
  if (tid == 0) s_resc = 0;
  long long rot = 0;
  int status = ST_OK;
  double vsel = -1.0;
  for (;;) {
    // ---- argmax over the row cache (lexicographically smallest pair among equal scores)
    double v = -1.0;
    int r = INT_MAX;
    for (int k = lane; k < n; k += 64) {
      const double x = best[k];
      if (x > v) {
        v = x;
        r = k;
      }
    }
    wave_best(v, r);
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
    rot_params<double>(G[(size_t)p * ldg + p], G[(size_t)q * ldg + q], apq, t, c, s);
    // ---- [b_p, b_q] <- [b_p, b_q] [[c, -s], [s, c]], same for the right factor
    double* xp = X + (size_t)p * ldx;
    double* xq = X + (size_t)q * ldx;
    for (int i = tid; i < m; i += NT) {
      const double u = xp[i], w = xq[i];
      xp[i] = c * u + s * w;
      xq[i] = c * w - s * u;
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
    // ---- rows p and q of A from the new columns
    for (int task = tid; task < 2 * n; task += NT) {
      int row = p, k = task;
      if (task >= n) {
        row = q;
        k = task - n;
        if (k == p) continue;
      }
      const double x = dot_rows(X + (size_t)row * ldx, X + (size_t)k * ldx, m);
      G[(size_t)row * ldg + k] = x;
      G[(size_t)k * ldg + row] = x;
    }
    __syncthreads();
    // ---- per-row cache refresh; rows whose cached best moved down are queued
    const double app = G[(size_t)p * ldg + p], aqq = G[(size_t)q * ldg + q];
    for (int k = tid; k < n; k += NT) {
      if (k == p || k == q) {
        s_list[atomicAdd(&s_cnt, 1)] = k;
        continue;
      }
      const double akk = G[(size_t)k * ldg + k];
      const double sp = svd_score<PIV>(akk, app, G[(size_t)k * ldg + p]);
      const double sq = svd_score<PIV>(akk, aqq, G[(size_t)k * ldg + q]);
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
          s_list[atomicAdd(&s_cnt, 1)] = k;
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
    // ---- full rescans, one wave per queued row
    const int cnt = s_cnt;
    for (int e = wv; e < cnt; e += NW) {
      const int k = s_list[e];
      const double* gk = G + (size_t)k * ldg;
      const double akk = gk[k];
      double bv = -1.0;
      int bc = INT_MAX;
      for (int l = lane; l < n; l += 64) {
        if (l == k) continue;
        const double x = svd_score<PIV>(akk, G[(size_t)l * ldg + l], gk[l]);
        if (x > bv) {
          bv = x;
          bc = l;
        }
      }
      wave_best(bv, bc);
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
__global__ __launch_bounds__(256) void k_svd_vectors(const double* __restrict__ X, int ldx, int m,
                                                     const double* __restrict__ G, int ldg,
                                                     const double* __restrict__ Vt, int ldvt,
                                                     int n, const int* __restrict__ rank,
                                                     double* __restrict__ U, int ldu,
                                                     double* __restrict__ V, int ldv) {
  const int k = blockIdx.y;
  const int rk = rank[k];
  const double sk = sqrt(G[(size_t)k * ldg + k]);
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
    if (U) U[(size_t)rk * ldu + i] = sk > 0.0 ? X[(size_t)k * ldx + i] / sk : 0.0;
    if (V && i < n) V[(size_t)rk * ldv + i] = Vt[(size_t)k * ldvt + i];
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_svd_load(const double* B, int m, int n, int ldb, double* X, int ldx, int* flag,
                           hipStream_t s) {
  dim3 g((m + 255) / 256, n);
  hipLaunchKernelGGL(k_svd_load, g, dim3(256), 0, s, B, m, n, ldb, X, ldx, flag);
  return hipGetLastError();
}

hipError_t launch_svd_gram(const double* X, int ldx, int m, int n, double* G, int ldg,
                           hipStream_t s) {
  dim3 g((n + 15) / 16, (n + 15) / 16);
  hipLaunchKernelGGL(k_svd_gram, g, dim3(256), 0, s, X, ldx, m, n, G, ldg);
  return hipGetLastError();
}

hipError_t launch_svd_rowmix(const double* Q, int ldq, const double* X, int ldx, int n, int m,
                             double* Y, int ldy, hipStream_t s) {
  dim3 g((m + 255) / 256, n);
  hipLaunchKernelGGL(k_svd_rowmix, g, dim3(256), 0, s, Q, ldq, X, ldx, n, m, Y, ldy);
  return hipGetLastError();
}

hipError_t launch_svd_transpose(const double* Q, int ldq, int n, double* Vt, int ldv,
                                hipStream_t s) {
  dim3 g((n + 255) / 256, n);
  hipLaunchKernelGGL(k_svd_transpose, g, dim3(256), 0, s, Q, ldq, n, Vt, ldv);
  return hipGetLastError();
}

template <int PIV>
static hipError_t svd_jacobi_t(const SDesc& d, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_rowbest<PIV>, dim3((d.n + 3) / 4), dim3(256), 0, s, d.G, d.ldg,
                     d.n, d.best, d.arg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // one workgroup; more lanes once the 2n dot products of a rotation outnumber 256
  if (d.n > 256) hipLaunchKernelGGL((k_svd1<PIV, 1024>), dim3(1), dim3(1024), 0, s, d);
  else hipLaunchKernelGGL((k_svd1<PIV, 256>), dim3(1), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_svd_jacobi(const SDesc& d, hipStream_t s) {
  if (d.n > kSvdMaxN) return hipErrorInvalidValue;
  if (d.pivot == 0) return svd_jacobi_t<0>(d, s);
  if (d.pivot == 1) return svd_jacobi_t<1>(d, s);
  return svd_jacobi_t<2>(d, s);
}

hipError_t launch_svd_out(const double* X, int ldx, int m, const double* G, int ldg,
                          const double* Vt, int ldvt, int n, int* rank, double* S, double* U,
                          int ldu, double* V, int ldv, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_rank, dim3((n + 255) / 256), dim3(256), 0, s, G, ldg, n, rank, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || (!U && !V)) return e;
  dim3 g((m + 255) / 256, n);
  hipLaunchKernelGGL(k_svd_vectors, g, dim3(256), 0, s, X, ldx, m, G, ldg, Vt, ldvt, n, rank, U,
                     ldu, V, ldv);
  return hipGetLastError();
}

}  // namespace je
