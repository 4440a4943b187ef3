/*
 * jacobi.h -- C ABI of the MI355X (gfx950) preconditioned Jacobi eigensolver with the
 * gap-aware pivot score of Shao & Nakatsukasa, "Accelerating preconditioned Jacobi
 * methods via perturbation-inspired pivoting".
 *
 * Problem (Algorithm 1): given a real symmetric A (n x n), compute its eigenvalues as
 * the diagonal of a sequence of Jacobi rotations A <- G^T A G (Sec. 2), each rotation
 * annihilating the off-diagonal entry chosen by a pivot rule:
 *   greedy: argmax_{i != j} |a_ij|                                  (Sec. 1)
 *   gap   : argmax_{i != j} L_ij,                                    (eq. (1))
 *           L_ij = 2 a_ij^2 / (|a_ii - a_jj| + sqrt((a_ii - a_jj)^2 + 4 a_ij^2)),
 *           with L_ij := 0 when a_ij^2 is 0 in FP64.
 * Ties go to the lexicographically smallest (i, j), i < j.
 * The eigenvectors are the preconditioner times the accumulated rotations (Sec. 2.1).
 *
 * Preconditioner (Sec. 2.1): with JE_PRECOND_FP32 the library first computes an FP32
 * spectral decomposition by a parallel cyclic Jacobi in FP32, re-orthogonalises its
 * eigenvector matrix in FP64 by Newton-Schulz, and runs the FP64 pivoted Jacobi on
 * Q^T A Q, whose off-diagonal entries are O(||A|| u_32).  By default the FP32
 * decomposition is refined once (fp32_passes = 2): the FP32 Jacobi runs again on
 * fl32(Q^T A Q) and Q <- Q V_2, re-orthogonalised; fp32_passes = 1 is the single FP32
 * decomposition.  FP32 sweeps stop when off(A32) <= 2^-22 ||A32||_F or a sweep does not
 * lower it (single pass); the first of two passes stops at 2^-18; the refinement sweeps
 * until a sweep fails to halve off or off <= 2^-30 ||A32||_F (jacobi_svd: no 2^-30 bound);
 * every pass is capped at fp32_max_sweeps.
 *
 * Stop rule (default, Theorem 1): stop once max_{i != j} L_ij <= eps with
 *   eps = tol * ||A||_F / (2 n (n - 1)),
 * which guarantees |lambda_k - a_kk| <= tol * ||A||_F for the sorted diagonal.
 *
 * Conventions for every entry point:
 *   - All matrix/vector pointers are DEVICE pointers (hipMalloc'd memory or torch CUDA
 *     tensors) unless stated otherwise.  The library never frees caller memory.
 *   - A is column-major with leading dimension lda >= max(1, n): element (i, j) is
 *     A[i + j*lda].  Only the upper triangle (i <= j) is read; it is mirrored.  A is
 *     never modified.
 *   - W receives n eigenvalues in ascending order (stable: equal values keep the order
 *     of the diagonal positions that produced them).
 *   - V (may be NULL = eigenvalues only) is column-major with leading dimension ldv >= n:
 *     component i of the eigenvector of W[k] is V[i + k*ldv].
 *   - All calls are blocking: work is enqueued on `stream` (NULL = the null stream of
 *     the current device) and the call returns once it has completed, so statistics are
 *     valid on return.  (The solve takes decisions on the host from device state between
 *     its launches: when the rotation log is full it is drained into V, and Newton-Schulz
 *     stops once converged; an asynchronous form would have to move these decisions onto
 *     the device.)
 *   - Inputs whose largest entry lies outside [2^-60, 2^60] are scaled by a power of two
 *     (exact) before the solve and the eigenvalues scaled back, so squares and the FP32
 *     copy stay in range; other inputs are solved as given.
 *   - The library owns a per-device workspace pool (grown on demand, released by
 *     jacobi_release()).  Calls from several host threads are serialised internally.
 *
 * Return status (int):
 *   0                 JE_OK
 *   -k (k >= 1)       the k-th argument is invalid (LAPACK info convention)
 *   JE_WARN_MAXROT    the rotation cap was reached; W, V hold the current iterate (V is
 *                     still orthogonal)
 *   JE_WARN_STALL     the best remaining pivot has a_pq == 0 (nothing to annihilate)
 *                     while the stop rule does not hold; W, V hold the current iterate
 *   JE_ERR_NONFINITE  A holds NaN or Inf in its upper triangle (outputs untouched), or
 *                     the preconditioned matrix is not finite
 *   JE_ERR_NOMEM      device memory for the workspace could not be allocated
 *   JE_ERR_DEVICE     a HIP runtime call failed (no device, launch failure, ...)
 *   JE_ERR_TOO_LARGE  n exceeds JE_MAX_N
 */
#ifndef JACOBI_GAP_JACOBI_H
#define JACOBI_GAP_JACOBI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A HIP stream handle (hipStream_t) passed as an opaque pointer. */
typedef void* je_stream;

#define JE_MAX_N 8192

/* JE_PIVOT_RELATIVE is the relative score of Sec. 4.2, (1/a_ii + 1/a_jj) L_ij, for the
 * positive semidefinite Gram matrix of jacobi_svd only. */
enum je_pivot { JE_PIVOT_GREEDY = 0, JE_PIVOT_GAP = 1, JE_PIVOT_RELATIVE = 2 };
enum je_precond { JE_PRECOND_NONE = 0, JE_PRECOND_FP32 = 1 };
enum je_stop {
  JE_STOP_CERT = 0,  /* max_{i!=j} L_ij <= tol*||A||_F / (2n(n-1))   (Theorem 1)           */
  JE_STOP_OFF = 1,   /* off(A) = sqrt(sum_{i!=j} a_ij^2) <= tol*||A||_F                      */
  JE_STOP_SCORE = 2  /* selection score of the best pivot (|a_pq| or L_pq) <= tol*||A||_F  */
};
enum je_status {
  JE_OK = 0,
  JE_WARN_MAXROT = 1,
  JE_WARN_STALL = 2,
  JE_ERR_NONFINITE = 3,
  JE_ERR_NOMEM = 4,
  JE_ERR_DEVICE = 5,
  JE_ERR_TOO_LARGE = 6
};

/* Options of the _ex / _batched entry points.  Fill with je_opts_default() first. */
typedef struct je_opts {
  int stop;                  /* enum je_stop                              (JE_STOP_CERT) */
  int polish_v;              /* 1: one FP64 Newton-Schulz step on V             (1)   */
  int fp32_max_sweeps;       /* sweeps cap of each FP32 preconditioner pass     (20)   */
  int fp32_passes;           /* FP32 decompositions (1 or 2)                    (2)    */
  long long max_rotations;   /* <= 0: 40 n^2 + 64                              (0)    */
  double abs_thr;            /* > 0: absolute threshold of the stop rule,             */
                             /*      overriding the one derived from tol         (0)  */
  int* pivot_log;            /* device int32[2*pivot_log_cap]: (p, q) of every        */
                             /* rotation of the FP64 phase, 0-based, p < q; NULL = off */
  long long pivot_log_cap;
  int split_gemm;            /* 1: form Q^T A Q on the BF16 matrix cores from 8-bit   */
                             /* integer slices of the row- and column-scaled         */
                             /* operands, summed exactly in FP32 per block of 32 and */
                             /* added into FP64 (FP64-accurate A_hat, the precision  */
                             /* variant); 0: FP64 MFMA products                  (0)  */
  int sort;                  /* 1: W ascending, V's columns permuted to match; 0: W in  */
                             /* the order of the final diagonal                  (1)  */
  int update_mode;           /* HBM-resident FP64 phase: 0 automatic (mirror for one    */
                             /* problem, timestamp for batches), 1 mirror (rows and   */
                             /* columns p, q stored), 2 timestamp (rows only); same   */
                             /* results                                          (0)  */
  int tune;                  /* batched: time the workgroup shapes of each size class  */
                             /* once per process and keep the faster (same results)(1)*/
  int graph;                 /* 1: replay from captured HIP graphs: the FP32 sweeps (0)  */
                             /* of one problem; for batches and served requests the  */
                             /* FP32 rounds between two polls, a Newton-Schulz step, */
                             /* the persistent FP64 launches and the log drain (same */
                             /* results as direct launches)                          */
  int profile;               /* 1: phase timers of the FP64 Jacobi kernel into        */
                             /* je_stats.prof_ns (slows the kernel slightly)     (0)  */
  int fp32_block;            /* rows per block of the FP32 stage: 0 by n (batches:  (0) */
                             /* 32), 16 or 32                                         */
  int jacobi_wgs;            /* FP64 phase of one problem: 0 automatic (several       */
                             /* workgroups from n = 768), 1 one workgroup, 2 several */
                             /* workgroups when the matrix lives in HBM; same results */
                             /* (0); batches always use one workgroup per matrix      */
  int batch_threads;         /* batches: threads per workgroup of the persistent FP64  */
                             /* launch for the HBM-resident members: 0 tuned (tune=1) */
                             /* or 512; 128 or 256 (members up to n = 512), or 512;   */
                             /* same results                                     (0)  */
} je_opts;

/* Statistics of one solve (host struct, filled before return). */
typedef struct je_stats {
  long long rotations;       /* FP64 Jacobi rotations performed                     */
  long long rescans;         /* full row rescans of the per-row score cache         */
  double final_max_score;    /* max_{i!=j} L_ij of the final iterate (certificate)  */
  double final_off;          /* off(A) of the final iterate                         */
  double normF;              /* ||A||_F of the input                                */
  double thr;                /* absolute stop threshold used                        */
  int sweeps32;              /* FP32 preconditioner sweeps (all passes)             */
  int status;
  float ms_precond;          /* FP32 Jacobi + re-orthogonalisation                  */
  float ms_gemm;             /* Q^T A Q contraction                                 */
  float ms_jacobi;           /* FP64 pivoted Jacobi (initial scores + rotations)    */
  float ms_finalize;         /* eigenvectors, polish, sort                          */
  float ms_jacobi_kernel;    /* the persistent Jacobi kernel launches alone (HIP    */
                             /* events on `stream` around each launch)             */
  double a_hat_off;          /* off(A_hat) = sqrt(sum_{i != j} a_ij^2) of the matrix   */
                             /* the FP64 phase starts from (0 if not measured)       */
  double prof_ns[6];         /* opts.profile: ns per rotation in the wave reductions,  */
                             /* the barrier, the cross-wave reduction, row rescans,  */
                             /* the rotation parameters and the row updates          */
  float ms_apply_log;        /* applying the rotation log to V (HIP events on stream) */
  int scale_exp;             /* the input was scaled by 2^scale_exp (0: not scaled)   */
  int jacobi_wgs;            /* workgroups of the FP64 Jacobi kernel                  */
} je_stats;

void je_opts_default(je_opts* opts);

/* Eigenvalues W (and eigenvectors V, ldv = n) of the symmetric A, stop rule of Theorem 1
 * with tolerance tol > 0 relative to ||A||_F.  pivot: enum je_pivot, precond: enum
 * je_precond.  Null stream, default options. */
int jacobi_eigh(const double* A, int n, int lda, double* W, double* V, double tol, int pivot,
                int precond);

/* As jacobi_eigh with explicit ldv, options (NULL = defaults), statistics (host pointer,
 * may be NULL) and stream. */
int jacobi_eigh_ex(const double* A, int n, int lda, double* W, double* V, int ldv, double tol,
                   int pivot, int precond, const je_opts* opts, je_stats* stats,
                   je_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): jacobi_eigh_ex with the same arguments,
 * results and statistics (the timings stay 0), whose workspace is a fixed array of
 * JE_NOALLOC_BYTES in device memory that the library holds on each device it runs on until
 * the process ends, instead of the allocated workspace pool.  It calls no device allocation
 * routine and creates no events or graphs (opts->graph is ignored).  n <= JE_NOALLOC_MAX_N,
 * else JE_ERR_TOO_LARGE before any device work.  Every call on a device shares that
 * device's array and leaves its contents there: calls on one device must not overlap (calls
 * of one process are serialised internally and return when done; two processes each hold
 * their own array).  The rotation log holds 2^16 entries, so longer solves drain it more
 * often (same results). */
#define JE_NOALLOC_MAX_N 512
#define JE_NOALLOC_BYTES (24u << 20)
int jacobi_eigh_noalloc(const double* A, int n, int lda, double* W, double* V, int ldv,
                        double tol, int pivot, int precond, const je_opts* opts,
                        je_stats* stats, je_stream stream);

/* `batch` independent problems of (possibly different) sizes solved together: the same
 * phases as jacobi_eigh_ex, each launch covering the whole batch, the FP64 phase as
 * persistent launches whose workgroups take the next matrix from a device queue.  Every
 * problem gives the same bits as a solve of its own.
 * All arrays are DEVICE memory: A, W, V are device arrays of `batch` device pointers (V may
 * be NULL = eigenvalues only, or hold NULL entries), n and lda device int arrays, info a
 * device int array receiving each problem's status; V[b] has leading dimension n[b].  The
 * whole batch shares tol, pivot, precond and opts (opts->pivot_log is ignored).  Returns
 * the worst status (errors before warnings) or a negative argument index
 * (A = 2 ... stream = 12).  Stream-ordered like the other calls, and blocking. */
int jacobi_eigh_batched(int batch, const double* const* A, const int* n, const int* lda,
                        double* const* W, double* const* V, double tol, int pivot,
                        int precond, const je_opts* opts, int* info, je_stream stream);

/* As jacobi_eigh_batched with the arrays in HOST memory (each entry still a device
 * pointer), explicit ldv (NULL = n) and per-problem statistics (HOST array of `batch`
 * je_stats, or NULL): the form for callers that build the batch on the host. */
int jacobi_eigh_batched_host(int batch, const double* const* A, const int* n, const int* lda,
                             double* const* W, double* const* V, const int* ldv, double tol,
                             int pivot, int precond, const je_opts* opts, int* info,
                             je_stats* stats, je_stream stream);

/* ---------------------------------------------------------------- one-sided SVD
 * Singular values (and vectors) of B (m x n, m >= n) by the one-sided Jacobi method of
 * Algorithm 2: a pivot (p, q) is chosen on the Gram matrix A = B^T B (the matrix the scores
 * are evaluated on, Sec. 2.1), columns b_p and b_q are made orthogonal by the rotation
 * that diagonalises [[a_pp, a_pq], [a_pq, a_qq]], and B <- B G(c, s, p, q).  A is never
 * rotated: each entry is the dot product of the current columns, summed in index order, and
 * rows p and q are recomputed after every rotation, so a_pp, a_qq, a_pq are always those of
 * the columns being rotated.  Ties go to the lexicographically smallest pair.
 *   pivot   JE_PIVOT_GREEDY |a_ij|, JE_PIVOT_GAP L_ij (eq. (1)), or JE_PIVOT_RELATIVE
 *           (1/a_ii + 1/a_jj) L_ij (Sec. 4.2; evaluated on the block scaled by a power of
 *           two so that max(a_ii, a_jj) is in [1/2, 1), which leaves it unchanged).
 *   precond JE_PRECOND_FP32 (Sec. 2.1): right singular vectors from the FP32 decomposition
 *           of fl32(B^T B) (passes and sweep caps from opts, as jacobi_eigh_ex),
 *           re-orthogonalised in FP64 -> Q; the method then runs on B Q.  JE_PRECOND_NONE:
 *           on B itself (Sec. 4.2: the global transformation would spoil the relative
 *           accuracy of tiny singular values).
 *   stop    best selection score <= thr, with thr = tol ||B^T B||_F / (2 n (n-1))
 *           (Theorem 1 on A; greedy implies it since |a_ij| >= L_ij) for greedy and gap, and
 *           thr = tol / (2 n (n-1)) for the scale-free relative score; opts->abs_thr > 0
 *           overrides it.  At exit the columns satisfy |cos(b_i, b_j)| <= sqrt(1.5 thr) under
 *           the relative score.  The greedy rule cannot go below the rounding level of the dot
 *           products (about m u ||b_i|| ||b_j||): give it a tol above that.
 *
 * B: device, column-major, ldb >= m, read only.  S: device, n singular values in
 * descending order (stable: equal values keep their column order); sigma_k = sqrt(a_kk)
 * of the final columns.  U (may be NULL): device, column-major m x n, ldu >= m, column k =
 * b_k / sigma_k (0 where sigma_k = 0).  V (may be NULL): device, column-major n x n,
 * ldv >= n, the accumulated right factor (Q times the rotations), B V = U diag(S).
 * opts (NULL = defaults): max_rotations (<= 0: 40 n^2 + 64), abs_thr, fp32_passes,
 * fp32_max_sweeps, and pivot_log, which here is written directly by the kernel (device
 * int32[2 * pivot_log_cap]: (p, q), 0-based, p < q).  opts->stop, polish_v and split_gemm
 * are not used.  stats: rotations, rescans, final_max_score (the best selection score at
 * exit), final_off (off(A) at exit), normF (||B^T B||_F), thr, sweeps32, a_hat_off (off of
 * the preconditioned Gram matrix), timings.
 * Range: the entries of B^T B must be finite (JE_ERR_NONFINITE otherwise), and under the
 * gap or greedy score their squares too.
 * Returns as jacobi_eigh_ex, with arguments numbered B = 1 ... opts = 13. */
int jacobi_svd(const double* B, int m, int n, int ldb, double* S, double* U, int ldu, double* V,
               int ldv, double tol, int pivot, int precond, const je_opts* opts,
               je_stats* stats, je_stream stream);

/* Device bytes the workspace pool holds for one solve of size n. */
size_t jacobi_workspace_size(int n, int precond);

/* Static description of a status code. */
const char* jacobi_strerror(int status);

/* Free the workspace pool of every device. */
void jacobi_release(void);

/* ---------------------------------------------------------------- serving
 * A request server for streams of independent problems of different sizes, with continuous
 * batching.  Each problem is solved by the batched method (jacobi_eigh_batched) with the
 * server's tol, pivot, precond and opts, and gives the same bits as in a batch of its own.
 * One device buffer of `hbm_budget` bytes, allocated at creation, holds the workspaces of
 * all requests in flight.  `workers` lanes (host threads, 1..16, each with its own HIP
 * stream on the device current at creation) run cohorts in bounded steps (a few FP32
 * rounds, one Newton-Schulz step, a few thousand FP64 rotations per member, ...).  At
 * every step boundary a lane admits queued requests of the size classes it serves
 * (n <= 128, <= 512, <= 1024, larger: with 4 or more lanes lane l serves class l mod 4,
 * with fewer, class c goes to lane c mod workers), in arrival order and as far as their
 * workspaces fit in the buffer, as a new cohort beside the (at most one) other it is
 * running; a request that does not fit, or whose lane runs two cohorts, waits and joins the
 * lane's next cohort.  A problem whose solve has ended
 * leaves its cohort at once: its completion record is posted and its memory returned.
 * Cohorts of different lanes run concurrently on the device (when the process has at least
 * as many hardware queues as lanes: HIP's GPU_MAX_HW_QUEUES, 4 by default, is read when the
 * runtime starts; with fewer, lanes share queues and their launches serialize).
 *
 * Ownership: A, W and V of a request are the caller's device memory and must stay valid
 * (A unmodified) until the request's completion record has been polled.  The server owns
 * its threads, streams and buffer; jacobi_server_destroy waits for queued requests. */
typedef struct je_server je_server;

typedef struct {
  long long tag;        /* the caller's tag from jacobi_server_submit                    */
  int status;           /* as jacobi_eigh_ex                                              */
  int n;
  int batch;            /* requests admitted in the same cohort                          */
  int pad;
  long long rotations;
  double t_submit;      /* seconds on the server's clock (jacobi_server_clock)           */
  double t_start;       /* admission of its cohort                                        */
  double t_done;        /* the request left its cohort: results are in W, V               */
} je_done;

/* NULL on an invalid argument or device error. */
je_server* jacobi_server_create(int workers, size_t hbm_budget, double tol, int pivot,
                                int precond, const je_opts* opts);
/* Queues one problem (arguments as jacobi_eigh_ex, numbered from 2).  Returns 0, a
 * negative argument index, JE_ERR_TOO_LARGE, JE_ERR_NOMEM when the problem's workspace
 * exceeds the whole hbm_budget (it could never be admitted), or a device error seen by a
 * lane. */
int jacobi_server_submit(je_server* srv, const double* A, int n, int lda, double* W, double* V,
                         int ldv, long long tag);
/* Moves up to `max` completion records to `out` (host array) and returns their number;
 * with wait != 0 it first blocks until a record exists or nothing is queued or running. */
int jacobi_server_poll(je_server* srv, je_done* out, int max, int wait);
/* Requests queued or being solved. */
long long jacobi_server_pending(je_server* srv);
/* Seconds since the server's creation (the clock of je_done). */
double jacobi_server_clock(je_server* srv);
void jacobi_server_destroy(je_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_GAP_JACOBI_H */
