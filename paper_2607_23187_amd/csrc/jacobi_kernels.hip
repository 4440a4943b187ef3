// FP64 pivoted Jacobi phase of the preconditioned eigensolver (Algorithm 1 with the
// greedy or the gap-aware pivot score of eq. (1)), for gfx950.
//
// Data layout (one problem):
//   A      row-major n x ld FP64, full symmetric storage, kept current in one of two
//          modes.  Mirror mode (one matrix): a rotation (p, q) stores rows p and q
//          (coalesced) and mirrors them into columns p and q, so every load is a
//          contiguous row segment.  Timestamp mode (batches): rows p and q only; each row
//          carries the rotation number ts[k] that last wrote it, and the current value of
//          entry (k, l) is A[k][l] if ts[k] >= ts[l] and A[l][k] otherwise, which trades
//          the 2n scattered column stores for a per-element choice of address on load.
//          Both modes perform the same arithmetic.  A LDS-resident A (small n) is mirrored.
//   diag   the diagonal lives in LDS / registers, never in A.
//   caches per row k: best selection score over l != k (value, column, a_kl, stale flag)
//          and, for greedy pivoting with the Theorem 1 stop rule, the best L_kl.  A stale
//          row keeps an upper bound; it is rescanned only when it would win the argmax
//          (Sec. 3.2: only O(n) scores change per rotation).
//   V      is not touched by the Jacobi kernel: every rotation is appended to a log
//          (p, q, c, s) and applied to the rows of V by a separate, fully parallel kernel.
#include <hip/hip_runtime.h>
#include <algorithm>

#include "device_common.h"
#include "jacobi_device.h"
#include "kernels.h"

namespace je {

// ------------------------------------------------------------------ symmetric copy
// Au (column-major, lda, upper triangle read) -> A (row-major, ld, full symmetric),
// diag[k] = a_kk, nonfinite flag.
constexpr int kTile = 32;

__device__ __forceinline__ void symcopy_tile(const double* __restrict__ Au, int n, int lda,
                                             double* __restrict__ A, int ld,
                                             double* __restrict__ diag, int* nonfinite, int bi,
                                             int bj) {
  if (bi > bj) return;
  __shared__ double t[kTile][kTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int i0 = bi * kTile, j0 = bj * kTile;
  bool bad = false;
  for (int r = ty; r < kTile; r += 8) {
    int i = i0 + tx, j = j0 + r;  // element (i, j) of Au, column-major -> coalesced in i
    double v = 0.0;
    if (i < n && j < n && (bi < bj || tx <= r)) {
      v = Au[(size_t)j * lda + i];
      if (!isfinite(v)) bad = true;
    }
    t[tx][r] = v;  // t[i_local][j_local]
  }
  if (bad) atomicOr(nonfinite, 1);
  __syncthreads();
  for (int r = ty; r < kTile; r += 8) {
    // row i0 + r of A, columns j0 + tx  (upper part, or mirrored lower part on diagonal tiles)
    int i = i0 + r, j = j0 + tx;
    if (i < n && j < n) {
      double v = (bi < bj || r <= tx) ? t[r][tx] : t[tx][r];
      A[(size_t)i * ld + j] = v;
      if (i == j) diag[i] = v;
    }
    if (bi < bj) {  // mirror: row j0 + r, columns i0 + tx
      int i2 = j0 + r, j2 = i0 + tx;
      if (i2 < n && j2 < n) A[(size_t)i2 * ld + j2] = t[tx][r];
    }
  }
}

__global__ __launch_bounds__(256) void k_symcopy(const double* __restrict__ Au, int n, int lda,
                                                 double* __restrict__ A, int ld,
                                                 double* __restrict__ diag, int* nonfinite) {
  symcopy_tile(Au, n, lda, A, ld, diag, nonfinite, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_symcopy_b(BMat* __restrict__ mats) {
  BMat& b = mats[blockIdx.z];
  if ((int)blockIdx.y * kTile >= b.n || (int)blockIdx.x * kTile >= b.n) return;
  symcopy_tile(b.Au, b.n, b.lda, b.Asym, b.ld, b.diag, b.flag, blockIdx.y, blockIdx.x);
}

__global__ void k_reset_b(BMat* __restrict__ mats, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  mats[i].flag[0] = 0;
  JCtl* c = mats[i].jd.ctl;
  c->rotations = 0; c->rescans = 0; c->status = 0; c->done = 0;
  c->final_sel = 0.0; c->final_cert = 0.0; c->final_off = 0.0;
}

__global__ void k_collect_b(const BMat* __restrict__ mats, int count, BInfo* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BMat& b = mats[i];
  BInfo x;
  x.normF = b.scal[0];
  x.rnorm = b.scal[1];
  x.maxabs = b.scal[4];
  x.nonfinite = b.flag[0];
  x.sweeps32 = b.f_pass_sweeps;
  x.ctl = *b.jd.ctl;
  out[i] = x;
}

hipError_t launch_reset_b(BMat* m, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count);
  return hipGetLastError();
}

hipError_t launch_collect_b(const BMat* m, int count, BInfo* out, hipStream_t s) {
  hipLaunchKernelGGL(k_collect_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count, out);
  return hipGetLastError();
}

hipError_t launch_symcopy_b(BMat* m, int count, int nmax, hipStream_t s) {
  int nb = (nmax + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_symcopy_b, dim3(nb, nb, count), dim3(256), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_symcopy(const double* Au, int n, int lda, double* A, int ld, double* diag,
                          double* rowsq, int* nonfinite, hipStream_t s) {
  (void)rowsq;
  int nb = (n + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_symcopy, dim3(nb, nb), dim3(256), 0, s, Au, n, lda, A, ld, diag,
                     nonfinite);
  return hipGetLastError();
}

__global__ void k_get_diag(const double* __restrict__ A, int n, int ld, double* __restrict__ diag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) diag[k] = A[(size_t)k * ld + k];
}

__device__ __forceinline__ double* bm_mat(BMat& b, size_t off) {
  return *reinterpret_cast<double**>(reinterpret_cast<char*>(&b) + off);
}

__global__ void k_get_diag_b(BMat* __restrict__ mats, size_t off) {
  BMat& b = mats[blockIdx.y];
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < b.n) b.diag[k] = bm_mat(b, off)[(size_t)k * b.ld + k];
}

hipError_t launch_get_diag_b(BMat* m, int count, int nmax, size_t off, hipStream_t s) {
  hipLaunchKernelGGL(k_get_diag_b, dim3((nmax + 255) / 256, count), dim3(256), 0, s, m, off);
  return hipGetLastError();
}

hipError_t launch_get_diag(const double* A, int n, int ld, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_get_diag, dim3((n + 255) / 256), dim3(256), 0, s, A, n, ld, diag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ ||A||_F
// Deterministic: per-row sums in a fixed order, then one block sums the rows in order.
__global__ __launch_bounds__(256) void k_rowsq(const double* __restrict__ A, int n, int ld,
                                               double* __restrict__ partial) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int l = lane; l < n; l += 64) {
    double v = A[(size_t)row * ld + l];
    s += v * v;
  }
  s = wave_sum_d(s);
  if (lane == 0) partial[row] = s;
}

__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ partial, int n,
                                                  double* out) {
  __shared__ double w[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += partial[k];
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = sqrt(((w[0] + w[1]) + w[2]) + w[3]);
}

__global__ __launch_bounds__(256) void k_rowsq_b(BMat* __restrict__ mats, size_t off) {
  BMat& b = mats[blockIdx.y];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= b.n) return;
  const double* A = bm_mat(b, off);
  double s = 0.0;
  for (int l = lane; l < b.n; l += 64) {
    double v = A[(size_t)row * b.ld + l];
    s += v * v;
  }
  s = wave_sum_d(s);
  if (lane == 0) b.rowsq[row] = s;
}

__global__ __launch_bounds__(256) void k_sum_rows_b(BMat* __restrict__ mats, int slot) {
  BMat& b = mats[blockIdx.x];
  __shared__ double w[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < b.n; k += 256) s += b.rowsq[k];
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) b.scal[slot] = sqrt(((w[0] + w[1]) + w[2]) + w[3]);
}

hipError_t launch_fro2_b(BMat* m, int count, int nmax, size_t off, int out_slot,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_rowsq_b, dim3((nmax + 3) / 4, count), dim3(256), 0, s, m, off);
  hipLaunchKernelGGL(k_sum_rows_b, dim3(count), dim3(256), 0, s, m, out_slot);
  return hipGetLastError();
}

hipError_t launch_fro2(const double* A, int n, int ld, double* partial, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_rowsq, dim3((n + 3) / 4), dim3(256), 0, s, A, n, ld, partial);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partial, n, out);
  return hipGetLastError();
}

// off(A): per-row sums of the off-diagonal squares, then the fixed-order row sum.
__global__ __launch_bounds__(256) void k_rowsq_off(const double* __restrict__ A, int n, int ld,
                                                   double* __restrict__ partial) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int l = lane; l < n; l += 64) {
    double v = (l == row) ? 0.0 : A[(size_t)row * ld + l];
    s += v * v;
  }
  s = wave_sum_d(s);
  if (lane == 0) partial[row] = s;
}

hipError_t launch_offnorm(const double* A, int n, int ld, double* partial, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_rowsq_off, dim3((n + 3) / 4), dim3(256), 0, s, A, n, ld, partial);
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, partial, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ zero fill
// A fill kernel rather than a runtime memset, so that the call sequence holds kernels and
// copies only.
__global__ void k_zero_words(int* __restrict__ p, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

hipError_t launch_zero_words(void* p, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((count + 255) / 256), dim3(256), 0, s, (int*)p, count);
  return hipGetLastError();
}

// ------------------------------------------------------------------ range of A
// max |a_ij| (per-row maxima, then one block), and an exact scaling by a power of two.
__global__ __launch_bounds__(256) void k_rowmax(const double* __restrict__ A, int n, int ld,
                                                double* __restrict__ partial) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double m = 0.0;
  for (int l = lane; l < n; l += 64) m = fmax(m, fabs(A[(size_t)row * ld + l]));
  m = wave_max_d(m);
  if (lane == 0) partial[row] = m;
}

__global__ __launch_bounds__(256) void k_max_rows(const double* __restrict__ partial, int n,
                                                  double* out) {
  __shared__ double w[4];
  double m = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) m = fmax(m, partial[k]);
  m = wave_max_d(m);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = fmax(fmax(w[0], w[1]), fmax(w[2], w[3]));
}

hipError_t launch_maxabs(const double* A, int n, int ld, double* partial, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_rowmax, dim3((n + 3) / 4), dim3(256), 0, s, A, n, ld, partial);
  hipLaunchKernelGGL(k_max_rows, dim3(1), dim3(256), 0, s, partial, n, out);
  return hipGetLastError();
}

// A <- 2^e A and diag <- 2^e diag (exact: no entry leaves the normal range for the scalings
// the host chooses).
__global__ void k_scale(double* __restrict__ A, int n, int ld, double* __restrict__ diag,
                        int e) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
  double v = ldexp(A[(size_t)i * ld + j], e);
  A[(size_t)i * ld + j] = v;
  if (i == j && diag) diag[i] = v;
}

hipError_t launch_scale(double* A, int n, int ld, double* diag, int e, hipStream_t s) {
  size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A, n, ld,
                     diag, e);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_rowmax_b(BMat* __restrict__ mats, size_t off) {
  BMat& b = mats[blockIdx.y];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= b.n) return;
  const double* A = bm_mat(b, off);
  double m = 0.0;
  for (int l = lane; l < b.n; l += 64) m = fmax(m, fabs(A[(size_t)row * b.ld + l]));
  m = wave_max_d(m);
  if (lane == 0) b.rowsq[row] = m;
}

__global__ __launch_bounds__(256) void k_max_rows_b(BMat* __restrict__ mats, int slot) {
  BMat& b = mats[blockIdx.x];
  __shared__ double w[4];
  double m = 0.0;
  for (int k = threadIdx.x; k < b.n; k += 256) m = fmax(m, b.rowsq[k]);
  m = wave_max_d(m);
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) b.scal[slot] = fmax(fmax(w[0], w[1]), fmax(w[2], w[3]));
}

hipError_t launch_maxabs_b(BMat* m, int count, int nmax, size_t off, int out_slot,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_rowmax_b, dim3((nmax + 3) / 4, count), dim3(256), 0, s, m, off);
  hipLaunchKernelGGL(k_max_rows_b, dim3(count), dim3(256), 0, s, m, out_slot);
  return hipGetLastError();
}

// members with a_exp != 0: the matrix at `off` and the diagonal scaled by 2^a_exp
__global__ void k_scale_b(BMat* __restrict__ mats, size_t off) {
  BMat& b = mats[blockIdx.y];
  if (b.a_exp == 0) return;
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)b.n * b.n) return;
  int i = (int)(idx / b.n), j = (int)(idx - (size_t)i * b.n);
  double* A = bm_mat(b, off);
  double v = ldexp(A[(size_t)i * b.ld + j], b.a_exp);
  A[(size_t)i * b.ld + j] = v;
  if (i == j) b.diag[i] = v;
}

hipError_t launch_scale_b(BMat* m, int count, int nmax, size_t off, hipStream_t s) {
  size_t tot = (size_t)nmax * nmax;
  hipLaunchKernelGGL(k_scale_b, dim3((unsigned)((tot + 255) / 256), count), dim3(256), 0, s, m,
                     off);
  return hipGetLastError();
}

hipError_t launch_normf(const double* rowsq, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, rowsq, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ J0: initial row scores
// Per-lane top two of a row: value and column of the best (smallest column on ties, since
// columns arrive in ascending order), and the best value among the other columns.
__device__ __forceinline__ void top2(double v, int col, double a, double& s1, int& c1, double& a1,
                                     double& s2) {
  if (v > s1) { s2 = s1; s1 = v; c1 = col; a1 = a; }
  else if (v > s2) s2 = v;
}

// Wave-uniform bound of all values except the winner's: the winner lane offers its second
// value, every other lane its best.
__device__ __forceinline__ double wave_second(double s1, double s2, int wlane) {
  return wave_max_ub(lane_id() == wlane ? s2 : s1);
}

// One wave per row: best selection score over l != k (smallest l on ties) and the largest
// score over the other columns; the same for L_kl (greedy + certificate only);
// off2[k] = sum_{l != k} a_kl^2.
template <bool GAP>
__device__ __forceinline__ void init_rows_body(const JDesc& d, int use_cert) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= d.n) return;
  const int n = d.n;
  const double* row = d.A + (size_t)k * d.ld;
  const double dkk = d.diag[k];
  double bs = -1.0, bv = 0.0, b2 = -1.0, cb = -1.0, cav = 0.0, c2 = -1.0, o2 = 0.0;
  int ba = 0x7fffffff, ca = 0x7fffffff;
  for (int l = lane; l < n; l += 64) {
    if (l == k) continue;
    double a = row[l];
    double dl = d.diag[l];
    top2(sel_score<GAP>(dkk, dl, a), l, a, bs, ba, bv, b2);
    if (use_cert) top2(gap_score(dkk, dl, a), l, 0.0, cb, ca, cav, c2);
    o2 += a * a;
  }
  int w = wave_argmax_lane(bs, ba);
  double wbs = -1.0, wbv = 0.0, wbu = -1.0;
  int wba = -1;
  if (w >= 0) {
    wbs = readlane_d(bs, w); wbv = readlane_d(bv, w); wba = readlane_i(ba, w);
    wbu = wave_second(bs, b2, w);
  }
  double wcb = -1.0, wcu = -1.0;
  int wca = -1;
  if (use_cert) {
    int w2 = wave_argmax_lane(cb, ca);
    if (w2 >= 0) { wcb = readlane_d(cb, w2); wca = readlane_i(ca, w2); wcu = wave_second(cb, c2, w2); }
  }
  o2 = wave_sum_fast(o2);
  if (lane == 0) {
    d.bs[k] = wbs; d.ba[k] = wba; d.bv[k] = wbv; d.bst[k] = 0; d.bu[k] = wbu;
    if (use_cert) { d.cb[k] = wcb; d.ca[k] = wca; d.cst[k] = 0; d.cu[k] = wcu; }
    d.off2[k] = o2;
    d.ts[k] = 0;
  }
}

template <bool GAP>
__global__ __launch_bounds__(256) void k_init_rows(JDesc d, int use_cert) {
  init_rows_body<GAP>(d, use_cert);
}

template <bool GAP>
__global__ __launch_bounds__(256) void k_init_rows_b(BMat* __restrict__ mats, int use_cert) {
  const JDesc d = mats[blockIdx.y].jd;
  init_rows_body<GAP>(d, use_cert);
}

hipError_t launch_init_rows_b(BMat* m, int count, int nmax, int pivot, int use_cert,
                              hipStream_t s) {
  dim3 g((nmax + 3) / 4, count), b(256);
  if (pivot == 1) hipLaunchKernelGGL(k_init_rows_b<true>, g, b, 0, s, m, use_cert);
  else hipLaunchKernelGGL(k_init_rows_b<false>, g, b, 0, s, m, use_cert);
  return hipGetLastError();
}

hipError_t launch_init_rows(const JDesc& d, hipStream_t s) {
  int use_cert = (d.pivot == 0 && d.stop == STOP_CERT) ? 1 : 0;
  dim3 g((d.n + 3) / 4), b(256);
  if (d.pivot == 1) hipLaunchKernelGGL(k_init_rows<true>, g, b, 0, s, d, use_cert);
  else hipLaunchKernelGGL(k_init_rows<false>, g, b, 0, s, d, use_cert);
  return hipGetLastError();
}

// ------------------------------------------------------------------ J1..J6: pivoted Jacobi
// Slot indices of the per-wave partial results exchanged through LDS.
enum {
  SL_SEL = 0,   // best cached selection candidate over the wave's rows (rows p, q excluded)
  SL_RP = 1,    // new row p: best (score, column) and bound of its other scores
  SL_RQ = 2,    // new row q
  SL_CERT = 3,  // best cached certificate value (greedy) over the wave's rows
  SL_CP = 4,    // new row p, certificate
  SL_CQ = 5,    // new row q, certificate
  SL_N = 6
};

template <int NW>
struct Slots {
  Cand c[2][SL_N][NW];
  double sum[2][3][NW];  // off2 of the wave's rows, of the new row p, of the new row q
};

// Cross-wave reduction of three slot groups at once: lane 16 g + w holds entry w of group
// g (g = 0, 1, 2; w < NW <= 16).  One DPP butterfly inside each 16-lane row yields the
// three group maxima; ties of the float keys are settled exactly.  Group 0 is keyed by
// row, groups 1 and 2 by column; for groups 1 and 2 u bounds every value but the winner's.
template <int NW>
__device__ __forceinline__ void reduce_groups3(const Cand* g0, const Cand* g1, const Cand* g2,
                                               Cand& r0, Cand& r1, Cand& r2) {
  const int lane = lane_id();
  const int grp = lane >> 4, w = lane & 15;
  Cand x = empty_cand();
  if (w < NW && grp < 3) x = (grp == 0 ? g0 : (grp == 1 ? g1 : g2))[w];
  const int key = (grp == 0) ? x.i : x.c;
  const int k32 = key32(x.s);
  int m = k32;
  m = max(m, dpp_i<0xB1>(m));
  m = max(m, dpp_i<0x4E>(m));
  m = max(m, dpp_i<0x141>(m));
  m = max(m, dpp_i<0x140>(m));
  const unsigned long long hit = __ballot(k32 == m && x.s >= 0.0);
  int win[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    unsigned long long b = hit & (0xffffull << (16 * g));
    int wl = b ? __ffsll((long long)b) - 1 : -1;
    if (b & (b - 1)) {  // equal float keys: exact comparison
      double bs = readlane_d(x.s, wl);
      int bk = readlane_i(key, wl);
      b &= b - 1;
      while (b) {
        int l = __ffsll((long long)b) - 1;
        b &= b - 1;
        double v = readlane_d(x.s, l);
        int kv = readlane_i(key, l);
        if (v > bs || (v == bs && kv < bk)) { bs = v; bk = kv; wl = l; }
      }
    }
    win[g] = wl;
  }
  // bound of the other values in groups 1 and 2: the winner offers its u, the rest their s
  const bool mine = (grp == 1 && lane == win[1]) || (grp == 2 && lane == win[2]);
  int mu = key32(mine ? x.u : x.s);
  mu = max(mu, dpp_i<0xB1>(mu));
  mu = max(mu, dpp_i<0x4E>(mu));
  mu = max(mu, dpp_i<0x141>(mu));
  mu = max(mu, dpp_i<0x140>(mu));
  const int mu1 = readlane_i(mu, 16), mu2 = readlane_i(mu, 32);
  r0 = read_cand(x, win[0], false);
  r1 = read_cand(x, win[1], false);
  r2 = read_cand(x, win[2], false);
  r1.u = key_ub(mu1);
  r2.u = key_ub(mu2);
}

// Cross-wave argmax of slot k over the NW waves: every lane scans the same NW entries
// (broadcast LDS reads), keeping the first maximum in (score desc, key asc) order; u is
// the bound of all values but the winner's.
template <int NW>
__device__ __forceinline__ Cand reduce_slot(const Slots<NW>& S, int b, int k, bool by_col) {
  Cand best = S.c[b][k][0];
  int bw = 0;
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    const Cand x = S.c[b][k][w];
    const int kx = by_col ? x.c : x.i, kb = by_col ? best.c : best.i;
    if (better(x.s, kx, best.s, kb)) { best = x; bw = w; }
  }
  double u = best.u;
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if (w != bw) u = fmax(u, S.c[b][k][w].s);
  best.u = u;
  return best;
}

template <int NW>
__device__ __forceinline__ double reduce_sum_slot(const Slots<NW>& S, int b, int k) {
  double v = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) v += S.sum[b][k][w];  // fixed order: wave 0, 1, ...
  return v;
}

// NT threads (NW waves), RM rows per thread (row k = tid + i * NT).  LDSA: A lives in
// LDS.  MIR: columns p and q are stored as well (mirrored update; rows are then always
// current and every load is a contiguous row segment); otherwise rows only, with the
// per-row write timestamps choosing the current copy of each entry.
template <int NT, int RM, bool GAP, bool LDSA, bool MIR>
__device__ __forceinline__ void jacobi_body(const JDesc d, long long log_base) {
  constexpr int NW = NT / kWave;
  extern __shared__ double smem[];
  __shared__ Slots<NW> S;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int n = d.n;
  const bool use_cert = !GAP && d.stop == STOP_CERT;
  const bool use_off = d.stop == STOP_OFF;

  double* s_diag = smem;
  int* s_ts = reinterpret_cast<int*>(s_diag + n);
  double* s_A = s_diag + n + (n + 1) / 2;  // after the int array, 8-byte aligned
  const int ldl = n | 1;
  const int ld = d.ld;
  double* gA = d.A;

  auto ld_a = [&](int r, int c) -> double {
    if constexpr (LDSA) return s_A[r * ldl + c];
    else return gA[(size_t)r * ld + c];
  };
  auto st_a = [&](int r, int c, double v) {
    if constexpr (LDSA) s_A[r * ldl + c] = v;
    else gA[(size_t)r * ld + c] = v;
  };
  auto sync = [&]() {
    if constexpr (NW > 1) __syncthreads();
  };

  // ---- per-thread rows k = tid + i * NT
  double dk[RM], bs[RM], bv[RM], bu[RM], cb[RM], cu[RM], of2[RM];
  int ba[RM], bst[RM], ca[RM], cst[RM], tk[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    int k = tid + i * NT;
    if (k < n) {
      dk[i] = d.diag[k]; bs[i] = d.bs[k]; ba[i] = d.ba[k]; bv[i] = d.bv[k]; bst[i] = d.bst[k];
      bu[i] = d.bu[k]; of2[i] = d.off2[k]; tk[i] = d.ts[k];
      if (use_cert) { cb[i] = d.cb[k]; ca[i] = d.ca[k]; cst[i] = d.cst[k]; cu[i] = d.cu[k]; }
      else { cb[i] = -1.0; ca[i] = -1; cst[i] = 0; cu[i] = -1.0; }
      s_diag[k] = dk[i];
      s_ts[k] = tk[i];
    } else {
      dk[i] = 0.0; bs[i] = -1.0; ba[i] = -1; bv[i] = 0.0; bst[i] = 0; bu[i] = -1.0; of2[i] = 0.0;
      tk[i] = 0; cb[i] = -1.0; ca[i] = -1; cst[i] = 0; cu[i] = -1.0;
    }
  }
  if constexpr (LDSA) {
    for (int idx = tid; idx < n * n; idx += NT) {
      int r = idx / n, c = idx - r * n;
      s_A[r * ldl + c] = gA[(size_t)r * ld + c];
    }
  }
  __syncthreads();

  long long rot = d.ctl->rotations;
  long long rescans = 0;
  int status = ST_OK, done = 0;
  const double thr = d.thr;
  // last rotation (its diagonal entries and timestamps reach LDS one iteration later)
  int lp = -1, lq = -1, lrot = 0;
  double lapp = 0.0, laqq = 0.0;
  bool pend = false;
  // per-thread top two of the new rows p and q (filled by a rotation)
  Cand rp = empty_cand(), rq = rp, cp = rp, cq = rp;
  double op = 0.0, oq = 0.0;
  Cand W = empty_cand(), C = empty_cand();
  double off_tot = 0.0;
  int it = 0;

  auto diag_of = [&](int x) -> double { return x == lp ? lapp : (x == lq ? laqq : s_diag[x]); };
  auto ts_of = [&](int x) -> int { return (x == lp || x == lq) ? lrot : s_ts[x]; };
  // current value of entry (r, l), l owned by this thread with timestamp tl
  auto entry = [&](int r, int l, int tl, int tr) -> double {
    if constexpr (MIR) return ld_a(r, l);
    else return (tl > tr) ? ld_a(l, r) : ld_a(r, l);
  };
  // optional phase timers: wave reductions, barrier, cross-wave, rescans, rotation
  const bool prof = d.prof != nullptr;
  long long tw = 0, tb = 0, tx = 0, tr = 0, tp = 0, tu = 0, tmark = 0;
  auto tick = [&]() -> long long { return prof ? (long long)wall_clock64() : 0; };
  const long long clk0 = prof ? (long long)clock64() : 0, wall0 = tick();

  // Full rescan of row r's selection (which == 0) or certificate (which == 1) cache:
  // exact best and the bound of the other scores.
  auto rescan = [&](int r, int which) {
    const int b = it & 1;
    const double arr = diag_of(r);
    const int trr = MIR ? 0 : ts_of(r);
    double vals[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int l = tid + i * NT;
      vals[i] = (l < n && l != r) ? entry(r, l, tk[i], trr) : 0.0;
    }
    Cand x = empty_cand();
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int l = tid + i * NT;
      if (l >= n || l == r) continue;
      double v = vals[i];
      double sc = which == 0 ? sel_score<GAP>(arr, dk[i], v) : gap_score(arr, dk[i], v);
      cand_top2(x, sc, l, v);
    }
    Cand e1 = empty_cand(), e2 = empty_cand();
    wave_best3(e1, 0, x, x.c, e2, 0);
    if (NW > 1) {
      if (lane == 0) S.c[b][SL_RP][wid] = x;
      __syncthreads();
      x = reduce_slot(S, b, SL_RP, true);
    }
    ++it;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      if (tid + i * NT == r) {
        if (which == 0) { bs[i] = x.s; ba[i] = x.c; bv[i] = x.a; bu[i] = x.u; bst[i] = 0; }
        else { cb[i] = x.s; ca[i] = x.c; cu[i] = x.u; cst[i] = 0; }
      }
    }
    ++rescans;
  };

  for (;;) {
    const int b = it & 1;
    tmark = tick();
    // ---- per-thread candidates over own rows
    Cand x1 = empty_cand(), x4 = empty_cand();
    double o7 = 0.0;
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int k = tid + i * NT;
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
    if (prof) { long long t = tick(); tw += t - tmark; tmark = t; }
    if constexpr (NW > 1) {
      if (lane == 0) {
        S.c[b][SL_SEL][wid] = w1; S.c[b][SL_RP][wid] = w2; S.c[b][SL_RQ][wid] = w3;
        if (use_cert) { S.c[b][SL_CERT][wid] = w4; S.c[b][SL_CP][wid] = w5; S.c[b][SL_CQ][wid] = w6; }
        if (use_off) { S.sum[b][0][wid] = s7; S.sum[b][1][wid] = s8; S.sum[b][2][wid] = s9; }
      }
      __syncthreads();
      if (prof) { long long t = tick(); tb += t - tmark; tmark = t; }
      reduce_groups3<NW>(S.c[b][SL_SEL], S.c[b][SL_RP], S.c[b][SL_RQ], w1, w2, w3);
      if (use_cert)
        reduce_groups3<NW>(S.c[b][SL_CERT], S.c[b][SL_CP], S.c[b][SL_CQ], w4, w5, w6);
      if (use_off) {
        s7 = reduce_sum_slot(S, b, 0);
        s8 = reduce_sum_slot(S, b, 1);
        s9 = reduce_sum_slot(S, b, 2);
      }
    }
    ++it;
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
        int k = tid + i * NT;
        if (k == lp) {
          bs[i] = w2.s; ba[i] = w2.c; bv[i] = w2.a; bu[i] = w2.u; bst[i] = 0; of2[i] = s8;
          if (use_cert) { cb[i] = w5.s; ca[i] = w5.c; cu[i] = w5.u; cst[i] = 0; }
        } else if (k == lq) {
          bs[i] = w3.s; ba[i] = w3.c; bv[i] = w3.a; bu[i] = w3.u; bst[i] = 0; of2[i] = s9;
          if (use_cert) { cb[i] = w6.s; ca[i] = w6.c; cu[i] = w6.u; cst[i] = 0; }
        }
      }
      if (tid == 0) {
        s_diag[lp] = lapp; s_diag[lq] = laqq;
        s_ts[lp] = lrot; s_ts[lq] = lrot;
      }
      pend = false;
      rp = empty_cand(); rq = rp; cp = rp; cq = rp;
      op = 0.0; oq = 0.0;
    }
    if (prof) { long long t = tick(); tx += t - tmark; tmark = t; }
    if (n < 2) { done = 1; break; }
    // ---- the winner must be exact
    if (W.f) {
      rescan(W.i, 0);
      if (prof) { long long t = tick(); tr += t - tmark; }
      continue;
    }
    // ---- stop rules (checked before every rotation)
    if (d.stop == STOP_CERT) {
      if (GAP) {
        if (W.s <= thr) { done = 1; break; }
      } else {
        if (C.s <= thr) { done = 1; break; }
        if (C.f) {
          rescan(C.i, 1);
          if (prof) { long long t = tick(); tr += t - tmark; }
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
    const int tsp = MIR ? 0 : ts_of(p), tsq = MIR ? 0 : ts_of(q);
    double xv[RM], yv[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int k = tid + i * NT;
      xv[i] = 0.0; yv[i] = 0.0;
      if (k >= n || k == p || k == q) continue;
      xv[i] = entry(p, k, tk[i], tsp);
      yv[i] = entry(q, k, tk[i], tsq);
    }
    const double apq = W.a;
    const double app = diag_of(p), aqq = diag_of(q);
    double t, c, s;
    rot_params<double>(app, aqq, apq, t, c, s);
    const double napp = app + t * apq;
    const double naqq = aqq - t * apq;
    const int nts = (int)(rot + 1);
    if (prof) { long long tt = tick(); tp += tt - tmark; tmark = tt; }
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      int k = tid + i * NT;
      if (k >= n) continue;
      if (k == p) {
        st_a(q, p, 0.0);
        if (MIR) st_a(p, q, 0.0);
        dk[i] = napp; tk[i] = nts;
        cand_top2(rq, 0.0, p, 0.0);
        if (use_cert) cand_top2(cq, 0.0, p, 0.0);
        continue;
      }
      if (k == q) {
        if (!MIR) st_a(p, q, 0.0);
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
      if (MIR) { st_a(k, p, xn); st_a(k, q, yn); }
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
    if (tid == 0) d.log[rot - log_base] = RotEntry{p, q, c, s};
    if (prof) { long long tt = tick(); tu += tt - tmark; }
    lp = p; lq = q; lapp = napp; laqq = naqq; lrot = nts;
    pend = true;
    ++rot;
  }

  // ---- write the state back (a later launch may resume from it)
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    int k = tid + i * NT;
    if (k < n) {
      d.diag[k] = dk[i]; d.bs[k] = bs[i]; d.ba[k] = ba[i]; d.bv[k] = bv[i]; d.bst[k] = bst[i];
      d.bu[k] = bu[i]; d.off2[k] = of2[i]; d.ts[k] = tk[i];
      if (use_cert) { d.cb[k] = cb[i]; d.ca[k] = ca[i]; d.cst[k] = cst[i]; d.cu[k] = cu[i]; }
    }
  }
  if constexpr (LDSA) {
    if (!done) {
      __syncthreads();
      for (int idx = tid; idx < n * n; idx += NT) {
        int r = idx / n, c = idx - r * n;
        gA[(size_t)r * ld + c] = s_A[r * ldl + c];
      }
    }
  }
  if (prof && tid == 0) {
    d.prof[0] += tw; d.prof[1] += tb; d.prof[2] += tx; d.prof[3] += tr; d.prof[4] += tp;
    d.prof[5] += tu;
    d.prof[6] += (long long)clock64() - clk0;
    d.prof[7] += tick() - wall0;
  }
  if (tid == 0) {
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

template <int NT, int RM, bool GAP, bool LDSA, bool MIR>
__global__ __launch_bounds__(NT) void k_jacobi(JDesc d, long long log_base) {
  jacobi_body<NT, RM, GAP, LDSA, MIR>(d, log_base);
}

// Persistent form for a batch: each workgroup takes the next matrix from a device counter
// (the host orders idx largest first) and runs the same pivoted Jacobi on it, until the
// list is exhausted.  Workgroups never wait for each other.
template <int NT, int RM, bool GAP, bool LDSA, bool MIR>
__global__ __launch_bounds__(NT) void k_jacobi_queue(BMat* __restrict__ mats,
                                                     const int* __restrict__ idx, int count,
                                                     int* counter) {
  __shared__ int s_next;
  for (;;) {
    __syncthreads();  // the previous matrix is finished with LDS
    if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_next;
    if (t >= count) return;
    const BMat& b = mats[idx[t]];
    jacobi_body<NT, RM, GAP, LDSA, MIR>(b.jd, b.log_base);
  }
}

// LDS budget of the kernel's dynamic part (diagonal, timestamps, and A if LDS-resident).
static size_t lds_bytes(int n, bool ldsa) {
  size_t b = (size_t)n * 8 + (size_t)((n + 1) / 2) * 8;
  if (ldsa) b += (size_t)n * (size_t)(n | 1) * 8;
  return b;
}

static int g_max_lds = -1;

static int max_lds() {
  if (g_max_lds < 0) {
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
      g_max_lds = v;
    else
      g_max_lds = 65536;
  }
  return g_max_lds;
}

bool jacobi_fits_lds(int n) {
  return n <= 128 && lds_bytes(n, true) + 8192 <= (size_t)max_lds();
}

template <int NT, int RM, bool GAP, bool LDSA, bool MIR>
static hipError_t launch_one(const JDesc& d, long long log_base, hipStream_t s) {
  // thread tid owns rows tid + i NT, i < RM: every row of the matrix needs an owner
  if ((long long)NT * RM < d.n) return hipErrorInvalidValue;
  size_t sh = lds_bytes(d.n, LDSA);
  auto fn = k_jacobi<NT, RM, GAP, LDSA, MIR>;
  if (sh > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(1), dim3(NT), sh, s, d, log_base);
  return hipGetLastError();
}

// Threads per workgroup for the HBM-resident kernel: 512 (two waves per SIMD, 256 VGPRs
// per lane); rows per thread RM = ceil(n / NT).
template <bool GAP, bool MIR>
static hipError_t launch_global(const JDesc& d, long long log_base, hipStream_t s) {
  const int n = d.n;
  if (n <= 256) return launch_one<256, 1, GAP, false, MIR>(d, log_base, s);
  if (n <= 512) return launch_one<512, 1, GAP, false, MIR>(d, log_base, s);
  if (n <= 1024) return launch_one<512, 2, GAP, false, MIR>(d, log_base, s);
  if (n <= 2048) return launch_one<512, 4, GAP, false, MIR>(d, log_base, s);
  if (n <= 4096) return launch_one<512, 8, GAP, false, MIR>(d, log_base, s);
  return launch_one<1024, 8, GAP, false, MIR>(d, log_base, s);
}

// HBM-resident matrices: mirror mode (rows and columns p, q stored, every load a contiguous
// row segment) or timestamp mode (rows only, the newer copy of each entry chosen by per-row
// write timestamps).  Both give the same arithmetic and the same pivot sequence.
template <bool GAP>
static hipError_t launch_jacobi_t(const JDesc& d, long long log_base, bool lds, bool mirror,
                                  hipStream_t s) {
  const int n = d.n;
  if (lds) {
    if (n <= 64) return launch_one<64, 1, GAP, true, true>(d, log_base, s);
    return launch_one<64, 2, GAP, true, true>(d, log_base, s);
  }
  if (mirror) return launch_global<GAP, true>(d, log_base, s);
  return launch_global<GAP, false>(d, log_base, s);
}

template <int NT, int RM, bool GAP, bool LDSA>
static hipError_t launch_queue_one(BMat* m, const int* idx, int count, int nmax, bool mirror,
                                   int* counter, int grid, hipStream_t s) {
  if ((long long)NT * RM < nmax) return hipErrorInvalidValue;
  size_t sh = lds_bytes(nmax, LDSA);
  auto fn = (LDSA || mirror) ? k_jacobi_queue<NT, RM, GAP, LDSA, true>
                             : k_jacobi_queue<NT, RM, GAP, LDSA, false>;
  // under graph capture the attribute was set by a preparing call (grid 0) beforehand
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return hipGetLastError();
  if (sh > 65536 && cs == hipStreamCaptureStatusNone) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  if (grid <= 0) return hipSuccess;  // attributes only (before a graph capture)
  hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), sh, s, m, idx, count, counter);
  return hipGetLastError();
}

// Workgroup shapes of the batched Jacobi: LDS-resident matrices (n <= 128) with one or two
// waves, HBM-resident ones with 128, 256 or 512 threads (128 and 256 up to n = 512; 1024
// threads above n = 4096); rows per thread = ceil(nmax / threads).
template <bool GAP>
static hipError_t launch_queue_t(BMat* m, const int* idx, int count, int nmax, bool lds,
                                 bool mirror, int threads, int* counter, int grid,
                                 hipStream_t s) {
  if (lds) {
    if (threads == 128 && nmax <= 128)
      return launch_queue_one<128, 1, GAP, true>(m, idx, count, nmax, mirror, counter, grid, s);
    if (nmax <= 64)
      return launch_queue_one<64, 1, GAP, true>(m, idx, count, nmax, mirror, counter, grid, s);
    return launch_queue_one<64, 2, GAP, true>(m, idx, count, nmax, mirror, counter, grid, s);
  }
  if (threads == 256) {
    if (nmax <= 256)
      return launch_queue_one<256, 1, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
    if (nmax <= 512)
      return launch_queue_one<256, 2, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
  }
  if (threads == 128) {
    if (nmax <= 128)
      return launch_queue_one<128, 1, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
    if (nmax <= 256)
      return launch_queue_one<128, 2, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
    if (nmax <= 512)
      return launch_queue_one<128, 4, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
  }
  if (nmax <= 512)
    return launch_queue_one<512, 1, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
  if (nmax <= 1024)
    return launch_queue_one<512, 2, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
  if (nmax <= 2048)
    return launch_queue_one<512, 4, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
  if (nmax <= 4096)
    return launch_queue_one<512, 8, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
  return launch_queue_one<1024, 8, GAP, false>(m, idx, count, nmax, mirror, counter, grid, s);
}

hipError_t launch_jacobi_queue(BMat* m, const int* idx, int count, int nmax, int pivot,
                               bool lds_mode, bool mirror, int threads, int* counter, int grid,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (pivot == 1)
    return launch_queue_t<true>(m, idx, count, nmax, lds_mode, mirror, threads, counter, grid, s);
  return launch_queue_t<false>(m, idx, count, nmax, lds_mode, mirror, threads, counter, grid, s);
}

hipError_t launch_jacobi(const JDesc& d, long long log_base, bool lds_mode, bool mirror,
                         hipStream_t s) {
  if (d.pivot == 1) return launch_jacobi_t<true>(d, log_base, lds_mode, mirror, s);
  return launch_jacobi_t<false>(d, log_base, lds_mode, mirror, s);
}

// ------------------------------------------------------------------ J5: apply the log to V
// Each block (one wave) holds `R` rows of V in LDS, transposed (column index major) so that
// lane r touches row r's entries p and q in consecutive banks.  Rotations on pairwise
// disjoint column pairs commute, which both forms below use; either way every entry of V
// sees the rotations that touch it in log order, with the same arithmetic.
//   R > 32 (n up to about 200; apply_log_rows): all lanes work on the same rotation.  The
//     log is staged 64 entries at a time, one per lane (a coalesced load, the next 64 in
//     flight while these are applied), each entry broadcast with readlane; up to four
//     consecutive rotations issue their LDS loads together when their columns are
//     disjoint (consecutive pivots are, in about four groups of four out of five).
//   R <= 32 (apply_log_groups, further below): the lanes split into 64 / R groups, each
//     applying one rotation of a run of consecutive disjoint ones.

// Global-memory views: accesses through them are global instructions, which count on the
// vector-memory counter only, so they never hold up a wait for LDS results.
template <class T>
using gmem = __attribute__((address_space(1))) T;

__device__ __forceinline__ void rot_col(double* __restrict__ t, int p, int q, int R, int off,
                                        double c, double s) {
  double* xp = t + p * R + off;
  double* xq = t + q * R + off;
  const double x = *xp, y = *xq;
  *xp = c * x + s * y;
  *xq = c * y - s * x;
}

template <int K>
__device__ __forceinline__ void rot_cols_disjoint(double* __restrict__ t, const int* p,
                                                  const int* q, int R, int off,
                                                  const double* c, const double* s) {
  double x[K], y[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    x[u] = t[p[u] * R + off];
    y[u] = t[q[u] * R + off];
  }
#pragma unroll
  for (int u = 0; u < K; ++u) {
    t[p[u] * R + off] = c[u] * x[u] + s[u] * y[u];
    t[q[u] * R + off] = c[u] * y[u] - s[u] * x[u];
  }
}

__device__ __forceinline__ bool pairs_disjoint(int p0, int q0, int p1, int q1) {
  return p0 != p1 && p0 != q1 && q0 != p1 && q0 != q1;
}

// Log entries k .. k + 3 of the staged chunk (lane j holds entry j: columns p | q << 16,
// cosine, sine) applied to the tile.
__device__ __forceinline__ void rot_group4(double* __restrict__ tile, int R, int off, int cpq,
                                           double cc, double cs, int k) {
  int p[4], q[4];
  double c[4], s[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int pq = __builtin_amdgcn_readlane(cpq, k + u);
    p[u] = pq & 0xffff; q[u] = pq >> 16;
    c[u] = readlane_d(cc, k + u); s[u] = readlane_d(cs, k + u);
  }
  const bool d01 = pairs_disjoint(p[0], q[0], p[1], q[1]);
  const bool d23 = pairs_disjoint(p[2], q[2], p[3], q[3]);
  const bool dx = pairs_disjoint(p[0], q[0], p[2], q[2]) &&
                  pairs_disjoint(p[0], q[0], p[3], q[3]) &&
                  pairs_disjoint(p[1], q[1], p[2], q[2]) &&
                  pairs_disjoint(p[1], q[1], p[3], q[3]);
  if (d01 && d23 && dx) {
    rot_cols_disjoint<4>(tile, p, q, R, off, c, s);
    return;
  }
  if (d01) {
    rot_cols_disjoint<2>(tile, p, q, R, off, c, s);
  } else {
    rot_col(tile, p[0], q[0], R, off, c[0], s[0]);
    rot_col(tile, p[1], q[1], R, off, c[1], s[1]);
  }
  if (d23) {
    rot_cols_disjoint<2>(tile, p + 2, q + 2, R, off, c + 2, s + 2);
  } else {
    rot_col(tile, p[2], q[2], R, off, c[2], s[2]);
    rot_col(tile, p[3], q[3], R, off, c[3], s[3]);
  }
}

// Applies log entries [0, m) to the tile.  Lanes past the block's rows repeat the work of
// lane (lane mod R): same addresses, same inputs, same results, so no lane diverges.  A full
// chunk of 64 entries is unrolled, so the loads of the next chunk stay in flight until it
// is done.
__device__ __forceinline__ void apply_log_rows(double* __restrict__ tile, int R,
                                               const RotEntry* log_, long long m) {
  const gmem<RotEntry>* log = (const gmem<RotEntry>*)log_;
  const int lane = threadIdx.x;
  const int off = lane % R;
  // the chunk being loaded: entry e0 + lane (identity rotations past the end)
  int np = 0, nq = 0;
  double nc = 1.0, ns = 0.0;
  if (lane < m) {
    np = log[lane].p; nq = log[lane].q; nc = log[lane].c; ns = log[lane].s;
  }
  // the first chunk is complete before the loop, as every later one is at its top, so no
  // wait inside the loop has to cover loads from before it
  __builtin_amdgcn_s_waitcnt(0);
  for (long long e0 = 0; e0 < m; e0 += 64) {
    const int cnt = __builtin_amdgcn_readfirstlane((int)(m - e0 < 64 ? m - e0 : 64));
    const int cpq = np | (nq << 16);  // n <= 8192
    const double cc = nc, cs = ns;
    np = 0; nq = 0; nc = 1.0; ns = 0.0;
    if (e0 + 64 + lane < m) {
      const gmem<RotEntry>* g = log + e0 + 64 + lane;
      np = g->p; nq = g->q; nc = g->c; ns = g->s;
    }
    if (cnt == 64) {
#pragma unroll
      for (int k = 0; k < 64; k += 4) rot_group4(tile, R, off, cpq, cc, cs, k);
    } else {
      int k = 0;
      for (; k + 4 <= cnt; k += 4) rot_group4(tile, R, off, cpq, cc, cs, k);
      for (; k < cnt; ++k) {
        const int pq = __builtin_amdgcn_readlane(cpq, k);
        rot_col(tile, pq & 0xffff, pq >> 16, R, off, readlane_d(cc, k), readlane_d(cs, k));
      }
    }
  }
}

// Rows [r0, r0 + rows) of V (row stride ldv) into the transposed tile and back, eight
// loads per lane in flight.  Indices past the end are clamped to the last element, whose
// lane then repeats the same load or store.
__device__ __forceinline__ void tile_in(double* __restrict__ tile, int R, int rows, int n,
                                        const double* V_, int ldv, int r0) {
  const gmem<double>* V = (const gmem<double>*)V_;
  const int total = rows * n;
  for (int base = threadIdx.x; base < total + 63; base += 512) {
    double v[8];
    int at[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = min(base + 64 * u, total - 1);
      const int r = idx / n, j = idx - r * n;
      v[u] = V[(size_t)(r0 + r) * ldv + j];
      at[u] = j * R + r;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) tile[at[u]] = v[u];
  }
}

__device__ __forceinline__ void tile_out(const double* __restrict__ tile, int R, int rows, int n,
                                         double* V_, int ldv, int r0) {
  gmem<double>* V = (gmem<double>*)V_;
  const int total = rows * n;
  for (int base = threadIdx.x; base < total + 63; base += 512) {
    double v[8];
    size_t at[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = min(base + 64 * u, total - 1);
      const int r = idx / n, j = idx - r * n;
      v[u] = tile[j * R + r];
      at[u] = (size_t)(r0 + r) * ldv + j;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) V[at[u]] = v[u];
  }
}

// Geometry of a log-drain workgroup (one wave, 64 KB of LDS) for V with n columns: rows
// R of V per workgroup, and lane groups G.  With R <= 32 the wave applies up to G = 64 / R
// (at most 32) rotations at once (lane group u, lanes u R .. u R + R - 1, rotation k + u of the log on
// the R rows) for the longest run of consecutive rotations on pairwise disjoint columns
// (they commute); the log chunk and a small column-mark table then share the LDS with the
// tile.  Larger R (small n) keeps one rotation per step over R lanes, and so does R = 1
// (n > 7776), where the tile alone fills the LDS.
constexpr int kApplyLds = 65536;
constexpr int kMarkSlots = 512;  // column marks, indexed by column mod 512
constexpr int kStageBytes = 64 * 16 + 64 * 4 + kMarkSlots * 4;

struct ApplyGeom {
  int R, G;
};

__host__ __device__ __forceinline__ ApplyGeom apply_geom(int n) {
  const int r1 = (kApplyLds - kStageBytes) / (n * 8);
  if (r1 >= 1 && r1 <= 32) return {r1, r1 == 1 ? 32 : 64 / r1};  // 2 G marking lanes <= 64
  int r0 = kApplyLds / (n * 8);
  r0 = r0 > 64 ? 64 : (r0 < 1 ? 1 : r0);
  return {r0, 1};
}

// Lane-group form of the drain (G >= 2; `stage` is the LDS after the tile, 16-byte
// aligned).  Each step: (1) lane i < 2 Ge reads column i mod 2 of rotation k + i / 2 and
// the lanes mark their columns with an LDS minimum of their lane index; a lane that finds
// a smaller index on its column shares it with an earlier rotation of the window, so the
// run of pairwise disjoint rotations ends before the rotation of the lowest such lane
// (columns are marked modulo kMarkSlots: a false clash only shortens the run, which always
// holds the first rotation); (2) lane group u < L applies rotation k + u.  Every entry of
// V sees the rotations touching it in log order, with the same arithmetic as one at a time.
__device__ __forceinline__ void apply_log_groups(double* __restrict__ tile, char* stage, int R,
                                                 int G, const RotEntry* log_, long long m) {
  const gmem<RotEntry>* log = (const gmem<RotEntry>*)log_;
  double2* ecs = reinterpret_cast<double2*>(stage);             // 64 (c, s)
  int* epq = reinterpret_cast<int*>(stage + 64 * 16);           // 64 (p | q << 16)
  int* mark = reinterpret_cast<int*>(stage + 64 * 16 + 64 * 4);  // kMarkSlots
  const int lane = threadIdx.x;
  const int u = lane / R, rr = lane - u * R;
  for (long long e0 = 0; e0 < m; e0 += 64) {
    const int cnt = __builtin_amdgcn_readfirstlane((int)(m - e0 < 64 ? m - e0 : 64));
    if (lane < cnt) {
      const gmem<RotEntry>* g = log + e0 + lane;
      epq[lane] = g->p | (g->q << 16);  // n <= 8192
      ecs[lane] = make_double2(g->c, g->s);
    }
    __syncthreads();  // one wave: orders the staging before the reads below
    int k = 0;
    while (k < cnt) {
      const int ge = min(G, cnt - k);
      const bool marker = lane < 2 * ge;
      int slot = 0;
      if (marker) {
        const int pq = epq[k + (lane >> 1)];
        slot = ((lane & 1) ? (pq >> 16) : (pq & 0xffff)) & (kMarkSlots - 1);
        mark[slot] = 0x7fffffff;
      }
      // the applying lanes read their rotation meanwhile (it does not depend on the run)
      const bool applier = u < ge;
      int apq = 0;
      double2 acs = make_double2(1.0, 0.0);
      if (applier) {
        apq = epq[k + u];
        acs = ecs[k + u];
      }
      if (marker) atomicMin(&mark[slot], lane);
      const bool clash = marker && mark[slot] != lane;
      const unsigned long long lost = __ballot(clash);
      int L = lost ? (__ffsll((long long)lost) - 1) >> 1 : ge;
      L = __builtin_amdgcn_readfirstlane(L < 1 ? 1 : L);
      if (u < L) {
        double* xp = tile + (apq & 0xffff) * R + rr;
        double* xq = tile + (apq >> 16) * R + rr;
        const double x = *xp, y = *xq;
        *xp = acs.x * x + acs.y * y;
        *xq = acs.x * y - acs.y * x;
      }
      k += L;
    }
    __syncthreads();  // the next chunk's staging overwrites this one
  }
}

__device__ __forceinline__ void apply_log_block(double* __restrict__ tile, ApplyGeom g, int n,
                                                const RotEntry* log, long long m) {
  if (g.G >= 2) {
    char* stage = reinterpret_cast<char*>(tile) + (((size_t)g.R * n * 8 + 15) & ~(size_t)15);
    apply_log_groups(tile, stage, g.R, g.G, log, m);
  } else {
    apply_log_rows(tile, g.R, log, m);
  }
}

__global__ __launch_bounds__(64) void k_apply_log(double* __restrict__ V, int n, int ldv,
                                                  const RotEntry* __restrict__ log,
                                                  long long m) {
  extern __shared__ double tile[];  // tile[j * R + r]
  const ApplyGeom g = apply_geom(n);
  const int r0 = blockIdx.x * g.R;
  const int rows = min(g.R, n - r0);
  tile_in(tile, g.R, rows, n, V, ldv, r0);
  __syncthreads();
  apply_log_block(tile, g, n, log, m);
  __syncthreads();
  tile_out(tile, g.R, rows, n, V, ldv, r0);
}

__global__ __launch_bounds__(64) void k_apply_log_b(BMat* __restrict__ mats) {
  extern __shared__ double tile[];
  const BMat& b = mats[blockIdx.y];
  const int n = b.n;
  const ApplyGeom g = apply_geom(n);
  const int r0 = blockIdx.x * g.R;
  if (r0 >= n) return;
  const long long m = b.jd.ctl->rotations - b.log_base;
  if (m <= 0) return;
  const int rows = min(g.R, n - r0);
  tile_in(tile, g.R, rows, n, b.Vw, b.ld, r0);
  __syncthreads();
  apply_log_block(tile, g, n, b.jd.log, m);
  __syncthreads();
  tile_out(tile, g.R, rows, n, b.Vw, b.ld, r0);
}

// LDS bytes of a drain workgroup (at most kApplyLds for every n <= 8192).
static size_t apply_lds_bytes(int n) {
  const ApplyGeom g = apply_geom(n);
  const size_t t = (size_t)g.R * n * 8;
  return g.G >= 2 ? ((t + 15) & ~(size_t)15) + kStageBytes : t;
}

// After the drain: the log of every matrix is empty again.
__global__ void k_log_drained_b(BMat* __restrict__ mats, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) mats[i].log_base = mats[i].jd.ctl->rotations;
}

hipError_t launch_apply_log_b(BMat* m, int count, int nmax, hipStream_t s) {
  // blocks per matrix: ceil(n / R(n)) does not decrease with n (R(n) does not increase), so
  // the largest matrix sets the grid
  const int R = apply_geom(nmax).R;
  const int gx = (nmax + R - 1) / R;
  hipLaunchKernelGGL(k_apply_log_b, dim3(gx, count), dim3(64), kApplyLds, s, m);
  hipLaunchKernelGGL(k_log_drained_b, dim3((count + 255) / 256), dim3(256), 0, s, m, count);
  return hipGetLastError();
}

hipError_t launch_apply_log(double* V, int n, int ldv, const RotEntry* log, long long m,
                            hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int R = apply_geom(n).R;
  hipLaunchKernelGGL(k_apply_log, dim3((n + R - 1) / R), dim3(64), apply_lds_bytes(n), s, V, n,
                     ldv, log, m);
  return hipGetLastError();
}

__global__ void k_set_identity(double* V, int n, int ldv) {
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
  V[(size_t)i * ldv + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_set_identity_b(BMat* __restrict__ mats, size_t off) {
  BMat& b = mats[blockIdx.y];
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)b.n * b.n) return;
  int i = (int)(idx / b.n), j = (int)(idx - (size_t)i * b.n);
  bm_mat(b, off)[(size_t)i * b.ld + j] = (i == j) ? 1.0 : 0.0;
}

__global__ void k_copy_mat_b(BMat* __restrict__ mats, size_t dst, size_t src) {
  BMat& b = mats[blockIdx.y];
  size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)b.n * b.n) return;
  int i = (int)(idx / b.n), j = (int)(idx - (size_t)i * b.n);
  bm_mat(b, dst)[(size_t)i * b.ld + j] = bm_mat(b, src)[(size_t)i * b.ld + j];
}

hipError_t launch_set_identity_b(BMat* m, int count, int nmax, size_t off, hipStream_t s) {
  size_t tot = (size_t)nmax * nmax;
  hipLaunchKernelGGL(k_set_identity_b, dim3((unsigned)((tot + 255) / 256), count), dim3(256), 0,
                     s, m, off);
  return hipGetLastError();
}

hipError_t launch_copy_mat_b(BMat* m, int count, int nmax, size_t dst, size_t src,
                             hipStream_t s) {
  size_t tot = (size_t)nmax * nmax;
  hipLaunchKernelGGL(k_copy_mat_b, dim3((unsigned)((tot + 255) / 256), count), dim3(256), 0, s,
                     m, dst, src);
  return hipGetLastError();
}

hipError_t launch_set_identity(double* V, int n, int ldv, hipStream_t s) {
  size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(k_set_identity, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, V, n,
                     ldv);
  return hipGetLastError();
}

// ------------------------------------------------------------------ J7: sort and output
// rank[k] = #{l : d_l < d_k} + #{l < k : d_l == d_k}  (ascending, stable)
// (sort == 0: rank[k] = k, the diagonal order.)  W[rank[k]] = 2^w_exp d_k (exact).
__global__ __launch_bounds__(256) void k_rank(const double* __restrict__ diag, int n,
                                              int* __restrict__ rank, double* __restrict__ W,
                                              int sort, int w_exp) {
  extern __shared__ double sd[];
  if (sort)
    for (int l = threadIdx.x; l < n; l += 256) sd[l] = diag[l];
  __syncthreads();
  int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double v = sort ? sd[k] : diag[k];
  int r = k;
  if (sort) {
    r = 0;
    for (int l = 0; l < n; ++l) {
      double u = sd[l];
      r += (u < v) || (u == v && l < k);
    }
  }
  rank[k] = r;
  W[r] = w_exp ? ldexp(v, w_exp) : v;
}

// Vout[i + rank[k] * ldvo] = Vw[i][k]   (32 x 32 tiles through LDS)
__global__ __launch_bounds__(256) void k_permute_out(const double* __restrict__ Vw, int n, int ldw,
                                                     const int* __restrict__ rank,
                                                     double* __restrict__ Vout, int ldvo) {
  __shared__ double t[kTile][kTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int i0 = blockIdx.y * kTile, k0 = blockIdx.x * kTile;
  for (int r = ty; r < kTile; r += 8) {
    int i = i0 + r, k = k0 + tx;
    t[r][tx] = (i < n && k < n) ? Vw[(size_t)i * ldw + k] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < kTile; r += 8) {
    int k = k0 + r, i = i0 + tx;
    if (i < n && k < n) Vout[(size_t)rank[k] * ldvo + i] = t[tx][r];
  }
}

__global__ __launch_bounds__(256) void k_rank_b(BMat* __restrict__ mats, int sort) {
  extern __shared__ double sd[];
  BMat& b = mats[blockIdx.y];
  const int n = b.n;
  if ((int)blockIdx.x * 256 >= n) return;
  if (sort)
    for (int l = threadIdx.x; l < n; l += 256) sd[l] = b.diag[l];
  __syncthreads();
  int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double v = sort ? sd[k] : b.diag[k];
  int r = k;
  if (sort) {
    r = 0;
    for (int l = 0; l < n; ++l) {
      double u = sd[l];
      r += (u < v) || (u == v && l < k);
    }
  }
  b.rank[k] = r;
  // the member's input was scaled by 2^a_exp
  b.Wout[r] = b.a_exp ? ldexp(v, -b.a_exp) : v;
}

__global__ __launch_bounds__(256) void k_permute_out_b(BMat* __restrict__ mats) {
  BMat& b = mats[blockIdx.z];
  const int n = b.n;
  if (!b.Vout || (int)blockIdx.y * kTile >= n || (int)blockIdx.x * kTile >= n) return;
  __shared__ double t[kTile][kTile + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int i0 = blockIdx.y * kTile, k0 = blockIdx.x * kTile;
  for (int r = ty; r < kTile; r += 8) {
    int i = i0 + r, k = k0 + tx;
    t[r][tx] = (i < n && k < n) ? b.Vw[(size_t)i * b.ld + k] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < kTile; r += 8) {
    int k = k0 + r, i = i0 + tx;
    if (i < n && k < n) b.Vout[(size_t)b.rank[k] * b.ldv + i] = t[tx][r];
  }
}

hipError_t launch_sort_output_b(BMat* m, int count, int nmax, int sort, hipStream_t s) {
  size_t sh = (size_t)nmax * 8;
  if (sh > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_rank_b,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rank_b, dim3((nmax + 255) / 256, count), dim3(256), sh, s, m, sort);
  int nb = (nmax + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_permute_out_b, dim3(nb, nb, count), dim3(256), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_sort_output(const double* diag, int n, const double* Vw, int ldw, double* W,
                              double* Vout, int ldvo, int* rank, int sort, int w_exp,
                              hipStream_t s) {
  size_t sh = (size_t)n * 8;
  if (sh > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_rank,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rank, dim3((n + 255) / 256), dim3(256), sh, s, diag, n, rank, W, sort,
                     w_exp);
  if (Vout) {
    int nb = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_permute_out, dim3(nb, nb), dim3(256), 0, s, Vw, n, ldw, rank, Vout,
                       ldvo);
  }
  return hipGetLastError();
}

__global__ void k_copy_pivots(const RotEntry* __restrict__ log, long long m, int* __restrict__ out) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  out[2 * e] = log[e].p;
  out[2 * e + 1] = log[e].q;
}

hipError_t launch_copy_pivots(const RotEntry* log, long long m, int* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_pivots, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, log, m,
                     out);
  return hipGetLastError();
}

}  // namespace je
