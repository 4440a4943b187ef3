// Internal interface between the host API (api.hip) and the kernel files.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace je {

enum { STOP_CERT = 0, STOP_OFF = 1, STOP_SCORE = 2 };
enum { ST_OK = 0, ST_MAXROT = 1, ST_STALL = 2 };

// One entry of the rotation log written by the pivoted Jacobi kernel: the rotation
// G(c, s, p, q) of Sec. 2 applied at that step.
struct RotEntry {
  int p, q;
  double c, s;
};

// Control block of one FP64 Jacobi phase (device memory).
struct JCtl {
  long long rotations;   // absolute rotation count so far
  long long rescans;
  int status;            // ST_*
  int done;              // 1 once the stop rule, the rotation cap or a stall ended it
  double final_sel;      // selection score of the best remaining pivot at exit
  double final_cert;     // certificate value (max L_ij, an upper bound) at exit
  double final_off;      // off(A) from the per-row sums at exit
};

// Device state of one FP64 pivoted-Jacobi problem.  A is row-major with leading
// dimension ld; entry (i, j) is current in row i if ts[i] >= ts[j], else in row j
// (rows are only ever written whole; see the Jacobi kernel).
struct JDesc {
  double* A;
  int n, ld;
  double* diag;                 // [n]
  double* bs; int* ba; double* bv; int* bst;   // per-row selection cache
  double* bu;                   // per row: upper bound of the row's scores off its best column
  double* cb; int* ca; int* cst;               // per-row certificate (L) cache, greedy only
  double* cu;                   // certificate analogue of bu
  double* off2;                 // [n] sum_{l != k} a_kl^2
  int* ts;                      // [n] rotation number that last wrote row k (0 = input)
  RotEntry* log;                // rotation log
  long long log_cap;
  JCtl* ctl;
  double thr;
  long long maxrot;
  int pivot, stop;
  long long* prof;              // optional [8] phase timers (10 ns ticks), accumulated
};

// Kernel launchers (all asynchronous on `s`).
hipError_t launch_symcopy(const double* Au, int n, int lda, double* A, int ld, double* diag,
                          double* rowsq, int* nonfinite, hipStream_t s);
hipError_t launch_normf(const double* rowsq, int n, double* out, hipStream_t s);
hipError_t launch_init_rows(const JDesc& d, hipStream_t s);
hipError_t launch_get_diag(const double* A, int n, int ld, double* diag, hipStream_t s);
// Runs the pivoted Jacobi until the stop rule holds, the cap is reached or the log is
// full (then ctl->done stays 0 and the launch can be repeated after the log is drained).
// lds_mode: A held in LDS (jacobi_fits_lds); otherwise mirror selects the HBM update mode
// (rows and columns p, q stored) over the timestamp mode (rows only).
hipError_t launch_jacobi(const JDesc& d, long long log_base, bool lds_mode, bool mirror,
                         hipStream_t s);
bool jacobi_fits_lds(int n);
// V[i][:] <- V[i][:] * G_1 ... G_m for every row (rotations of `log`, in order).
hipError_t launch_apply_log(double* V, int n, int ldv, const RotEntry* log, long long m,
                            hipStream_t s);

// Multi-workgroup form of launch_jacobi (mirror mode, A in HBM): G one-wave workgroups on
// one XCD exchange their candidates through L2 every rotation.  `buf` holds the control
// block and the exchange area (mw_bytes(n) bytes).  After the launch, MwCtl::misplaced = 1
// means the kernel returned without touching the state (run launch_jacobi instead);
// abort = 1 without it means a wait ran out mid-run (device error).
constexpr int kMwMaxGroups = 32;
struct MwCtl {
  int counter;                // arrivals at the exchange barriers
  int abort;                  // a wait ran out
  int misplaced;              // the workgroups were not all resident on one XCD
  int pad;
  int xcc[kMwMaxGroups];      // XCC id of every workgroup
};
void mw_shape(int n, int* G, int* RM);
size_t mw_bytes(int n);
hipError_t launch_jacobi_mw(const JDesc& d, long long log_base, void* buf, hipStream_t s);
hipError_t launch_set_identity(double* V, int n, int ldv, hipStream_t s);
// W[rank[k]] = 2^w_exp diag[k], Vout[:, rank[k]] = column k of Vw; rank ascending and
// stable when sort != 0, else rank[k] = k.
hipError_t launch_sort_output(const double* diag, int n, const double* Vw, int ldw, double* W,
                              double* Vout, int ldvo, int* perm, int sort, int w_exp,
                              hipStream_t s);
// count 4-byte words at p set to zero
hipError_t launch_zero_words(void* p, int count, hipStream_t s);
// out[0] = max |a_ij|
hipError_t launch_maxabs(const double* A, int n, int ld, double* partial, double* out,
                         hipStream_t s);
// A <- 2^e A, diag <- 2^e diag (diag may be null)
hipError_t launch_scale(double* A, int n, int ld, double* diag, int e, hipStream_t s);
hipError_t launch_copy_pivots(const RotEntry* log, long long m, int* out, hipStream_t s);

// FP64 GEMM on MFMA: C = alpha * op(A) * B + beta * Cin (all row-major, square n).
// op(A) = A if transA == 0 else A^T.  Cin may equal C only if beta == 0 or the tiles
// of C are only read by their own block (always true here).
// C = alpha A^T B for a symmetric product (X^T X, Q^T (A Q)): the tiles on and above the
// diagonal are computed and mirrored, so C is exactly symmetric.
hipError_t launch_dgemm_sym(int n, double alpha, const double* A, int lda, const double* B,
                            int ldb, double* C, int ldc, hipStream_t s);
hipError_t launch_dgemm(int n, int transA, double alpha, const double* A, int lda,
                        const double* B, int ldb, double beta, const double* Cin, int ldcin,
                        double* C, int ldc, hipStream_t s);
hipError_t launch_add_identity(double* C, int n, int ldc, double scale, hipStream_t s);
// C = op(A) * B on the BF16 matrix cores with FP64 accuracy: rows of op(A) and columns of
// B scaled by powers of two and cut into 8-bit integer slices (exact in BF16), slice
// products summed exactly in FP32 per K block of 32 and level, each level added into FP64
// (the precision variant of Q^T A Q).  `work`: gemm_split_bytes(n) bytes of device memory.
size_t gemm_split_bytes(int n);
hipError_t launch_gemm_split(int n, int transA, const double* A, int lda, const double* B,
                             int ldb, double* C, int ldc, void* work, hipStream_t s);
hipError_t launch_symmetrize(double* A, int n, int ld, hipStream_t s);
hipError_t launch_fro2(const double* A, int n, int ld, double* partial, double* out,
                       hipStream_t s);
// out[0] = off(A) = sqrt(sum_{i != j} a_ij^2)
hipError_t launch_offnorm(const double* A, int n, int ld, double* partial, double* out,
                          hipStream_t s);

// FP32 preconditioner.
size_t precond_f32_bytes(int n);
// Sweeps stop at off(A32) <= tol ||A32||_F, when a sweep leaves off(A32) >= rho times its
// value before the sweep, or after max_sweeps.  block: rows per block (16, 32; 0 = chosen
// by n); graphs: replay the sweeps from captured HIP graphs.
hipError_t run_precond_f32(const double* Asym, int n, int ld, double* Q, int ldq,
                           void* scratch, int max_sweeps, double tol, double rho, int* sweeps,
                           int block, bool graphs, hipStream_t s);

// ------------------------------------------------------------------ batches
// One matrix of a batch (device memory).  The batched kernels take an array of these and
// put the matrix index in their last grid dimension; blocks past a matrix's size exit, so
// one launch covers matrices of uneven n.  Workspace matrices are row-major n x ld.
struct BMat {
  const double* Au; int n, lda;      // input (column-major, upper triangle read)
  double* Wout; double* Vout; int ldv;
  int ld;
  double *Asym, *A, *Vw, *X, *Xb, *T, *R;
  double *diag, *rowsq, *scal;       // scal[0] = ||A||_F, scal[1] = ||I - X^T X||_F
  int *rank, *flag;                  // flag[0]: non-finite input
  // FP32 stage (np = n padded to 2 PB, nb = np / PB blocks, nb - 1 rounds per sweep)
  float *A32, *V32, *U;
  double* part;
  int np, nb;
  int f_round, f_sweeps, f_done, f_pass_sweeps;
  double f_off, f_nrm;
  // FP64 Jacobi phase
  JDesc jd;
  long long log_base;
  int j_done;
  // Newton-Schulz: set once the member has converged; its later steps are exact no-ops
  int ns_done;
  // the input was scaled by 2^a_exp (exact) to keep squares and FP32 values in range; the
  // eigenvalues are scaled back
  int a_exp;
};

// Per-matrix results gathered into one array, so the host reads a batch with one copy.
struct BInfo {
  double normF, rnorm, maxabs;
  int nonfinite, sweeps32;  // sweeps32: FP32 sweeps of all passes so far
  JCtl ctl;
};

// field of a BMat that holds an n x ld FP64 matrix, as an offset for the generic kernels
#define BM_FIELD(f) offsetof(::je::BMat, f)

hipError_t launch_symcopy_b(BMat* m, int count, int nmax, hipStream_t s);
// flag[0] = 0 and the Jacobi control block zeroed, for every matrix
hipError_t launch_reset_b(BMat* m, int count, hipStream_t s);
hipError_t launch_collect_b(const BMat* m, int count, BInfo* out, hipStream_t s);
hipError_t launch_fro2_b(BMat* m, int count, int nmax, size_t off, int out_slot,
                         hipStream_t s);
hipError_t launch_get_diag_b(BMat* m, int count, int nmax, size_t off, hipStream_t s);
hipError_t launch_set_identity_b(BMat* m, int count, int nmax, size_t off, hipStream_t s);
hipError_t launch_copy_mat_b(BMat* m, int count, int nmax, size_t dst, size_t src, hipStream_t s);
hipError_t launch_init_rows_b(BMat* m, int count, int nmax, int pivot, int use_cert,
                              hipStream_t s);
// Persistent Jacobi over the matrices idx[0..count) (one workgroup per matrix at a time,
// taken from a device counter in the given order); lds_mode as for launch_jacobi.  With
// grid <= 0 only the kernel's attributes are set (before a graph capture).
hipError_t launch_jacobi_queue(BMat* m, const int* idx, int count, int nmax, int pivot,
                               bool lds_mode, bool mirror, int threads, int* counter, int grid,
                               hipStream_t s);
hipError_t launch_apply_log_b(BMat* m, int count, int nmax, hipStream_t s);
hipError_t launch_sort_output_b(BMat* m, int count, int nmax, int sort, hipStream_t s);
// scal[out_slot] = max |a_ij| of the matrix at `off`
hipError_t launch_maxabs_b(BMat* m, int count, int nmax, size_t off, int out_slot,
                           hipStream_t s);
// members with a_exp != 0: matrix at `off` and diag scaled by 2^a_exp
hipError_t launch_scale_b(BMat* m, int count, int nmax, size_t off, hipStream_t s);
// ns_mask: members with ns_done get C = 0 (no product), resp. no identity added
hipError_t launch_dgemm_sym_b(BMat* m, int count, int nmax, double alpha, size_t offA,
                              size_t offB, size_t offC, hipStream_t s, int ns_mask = 0);
hipError_t launch_dgemm_b(BMat* m, int count, int nmax, int transA, double alpha, size_t offA,
                          size_t offB, double beta, size_t offCin, size_t offC, hipStream_t s,
                          int ns_mask = 0);
hipError_t launch_add_identity_b(BMat* m, int count, int nmax, size_t off, double scale,
                                 hipStream_t s, int ns_mask = 0);
// Newton-Schulz bookkeeping of a batch: clear every ns_done, or set it for the members whose
// residual of this step (scal[1]) meets the convergence rule
hipError_t launch_ns_reset_b(BMat* m, int count, hipStream_t s);
hipError_t launch_ns_flag_b(BMat* m, int count, hipStream_t s);
hipError_t launch_symmetrize_b(BMat* m, int count, int nmax, size_t off, hipStream_t s);
// FP32 stage of a batch: fl32 of the matrix at `off` (padded), V32 = I, sweeps with the
// given stop rule until every matrix is done (each at its own pace, at most max_sweeps);
// then the first n columns of V32 (FP64) into the matrix at `qoff`.  nvec: host array of
// the sizes; dwork: device ints, 5 per matrix.
// Batched FP32 stage: bytes of one matrix's state with blocks of pb rows (and the part
// before its per-block sums), and the block rows of a batch whose largest n is nmax
// (request 16 or 32 overrides the choice).
size_t precond_f32_bytes_b(int n, int pb);
size_t precond_f32_part_b(int n, int pb);
int precond_f32_block_b(int nmax, int request);
hipError_t run_precond_f32_b(BMat* m, const int* nvec, int count, int nmax, int* dwork,
                             size_t off, size_t qoff, int max_sweeps, double tol, double rho,
                             hipStream_t s);

// The same stage in bounded pieces: begin() starts it, every advance(k) performs up to k
// steps (a step = the next round of every matrix not yet done); `finished` is set, and the
// FP64 eigenvector matrices gathered, once every matrix is done.  nvec must stay valid.
struct F32Batch {
  BMat* m = nullptr;
  const int* nvec = nullptr;
  int count = 0, nmax = 0;
  int* dwork = nullptr;
  size_t qoff = 0;
  int max_sweeps = 0;
  double tol = 0.0, rho = 0.0;
  hipStream_t s = nullptr;
  long long step = 0, max_steps = 0;
  bool finished = false;
  std::vector<int> done, act, ps, pa, pv;
  int tps = 0, tpa = 0, tpv = 0, na = 0, max_rounds = 1;
  // graph replay: the steps between two polls of the done flags are one graph, captured
  // at the first advance and replayed; the launch lists are kept (matrices that are done
  // leave every launch at once) until a quarter of the listed matrices are done, then
  // rebuilt and the graph captured again
  // (captured on stream cap, which the caller owns, and launched on s)
  bool graph = false;
  hipStream_t cap = nullptr;
  hipGraphExec_t gx = nullptr;
  int live = 0;  // matrices not yet done (graph replay)
  int pb = 32;  // block rows
  hipError_t begin(BMat* m, const int* nvec, int count, int nmax, int* dwork, size_t off,
                   size_t qoff, int max_sweeps, double tol, double rho, hipStream_t s,
                   bool graph = false, hipStream_t cap = nullptr, int pb = 32);
  hipError_t advance(int steps);
  void release();
  F32Batch() = default;
  F32Batch(const F32Batch&) = delete;
  F32Batch& operator=(const F32Batch&) = delete;
  ~F32Batch() { release(); }

 private:
  hipError_t rebuild();
  hipError_t poll();
  hipError_t launch_steps(int k);
};

// ------------------------------------------------------------------ one-sided SVD
constexpr int kSvdMaxN = 8192;

// Device state of the one-sided Jacobi SVD: Y = B row-major (row stride ldy), the right
// factor Vt = V^T (rows rotated with the columns of B; may be null), the Gram matrix
// G = B^T B (row-major), the per-row best score cache, the diagonal of G and the last
// recomputed rows p and q of G (device scratch of n entries each), the control block.
struct SDesc {
  double* Y;
  int m, ldy;
  double* Vt;
  int ldv;
  double* G;
  int n, ldg;
  double* best;
  int* arg;
  double *diag, *rowp, *rowq;
  double thr;
  long long maxrot;
  int pivot;                    // 0 greedy, 1 gap, 2 relative
  int* plog;                    // optional (p, q) log, logcap entries
  long long logcap;
  JCtl* ctl;
};

hipError_t launch_svd_load(const double* B, int m, int n, int ldb, double* Y, int ldy, int* flag,
                           hipStream_t s);
hipError_t launch_svd_gram(const double* Y, int ldy, int m, int n, double* G, int ldg,
                           hipStream_t s);
// Z = Y Q: the rows of B times the preconditioner.
hipError_t launch_svd_rowmix(const double* Y, int ldy, const double* Q, int ldq, int m, int n,
                             double* Z, int ldz, hipStream_t s);
hipError_t launch_svd_transpose(const double* Q, int ldq, int n, double* Vt, int ldv,
                                hipStream_t s);
// Row cache, then the whole rotation sequence in one launch (ends at the stop rule, the
// rotation cap or a stall; ctl->done = 1).
hipError_t launch_svd_jacobi(const SDesc& d, hipStream_t s);
// true when B and the per-row state of the rotation kernel fit in LDS
bool svd_resident(int m, int n);
hipError_t launch_svd_out(const double* Y, int ldy, int m, const double* G, int ldg,
                          const double* Vt, int ldvt, int n, int* rank, double* S, double* U,
                          int ldu, double* V, int ldv, hipStream_t s);

}  // namespace je
