/*
 * mbl.h -- C ABI of the MI355X matrix-free interior eigensolver for the
 * random-field spin-1/2 chain (Van Beeumen, Ibrahim, Kahanamoku-Meyer, Yao,
 * Yang, "Enhancing Scalability of a Matrix-Free Eigensolver for Studying
 * Many-Body Localization", arXiv 2012.00217).
 *
 * Model (paper eq. (1)/(2), Sec. 2.1), open chain of L sites, S = sigma/2:
 *   H = J sum_{i=0}^{L-2} [S^x_i S^x_{i+1} + S^y_i S^y_{i+1} + Delta S^z_i S^z_{i+1}]
 *       + sum_{i=0}^{L-1} h_i S^z_i
 * J = Delta = 1 is eq. (1).  H conserves total S^z; every call works in one
 * sector, nup = Sz + L/2 up spins, dimension n = C(L, nup) (Table 1).
 *
 * Basis convention: site i is bit i of an integer state; bit 1 = spin up.
 * Row r of every block is the r-th state of the sector in ascending integer
 * order.  Blocks are row-major n x b with an explicit leading dimension
 * (in elements); FP64 blocks are double, FP32 blocks are float.
 *
 * Ownership: h is copied at create time; the handle owns its device tables.
 * Block arguments (X, Y, R, W, evecs, Gram outputs) are device pointers owned
 * by the caller.  Host pointers are marked _host.  Work buffers are device
 * memory the library allocates (hipMalloc, or the callback installed with
 * mbl_set_allocator) and frees before the call returns, except the per-handle
 * tables, freed by mbl_hamiltonian_destroy.
 *
 * Errors: every call returns an mbl_status (MBL_OK == 0, errors < 0).  No C++
 * exception and no abort crosses this boundary.  mbl_last_error() returns a
 * thread-local message for the last failure on the calling thread.
 * Arguments are validated before any device work is enqueued; a call that
 * returns MBL_EINVAL has not touched device memory.
 *
 * Streams: calls marked "async" only enqueue work on the given stream and
 * return; the others synchronise that stream before returning.  Handles are
 * thread-compatible, not thread-safe: do not use one handle from two threads
 * at once.
 */
#ifndef MBL_H_
#define MBL_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MBL_OK = 0,
  MBL_EINVAL = -1,      /* invalid argument (nothing was enqueued)           */
  MBL_ENOMEM = -2,      /* device allocation failed                           */
  MBL_EDEVICE = -3,     /* a HIP runtime call failed                          */
  MBL_ENOCONV = -4,     /* solver hit its iteration limit; best pairs returned */
  MBL_EBREAKDOWN = -5,  /* basis collapsed (e.g. starting block rank-deficient) */
  MBL_ETIMEOUT = -6,    /* mbl_server_wait: request not finished in time      */
  MBL_ECANCELLED = -7,  /* solve stopped by its cancel flag or time limit (or
                           a server request cancelled); best pairs returned  */
  MBL_EINTERNAL = -8    /* unexpected internal failure                        */
} mbl_status;

typedef enum {
  MBL_F64 = 0,    /* everything in FP64                                       */
  MBL_F32 = 1,    /* FP32 blocks (apply / PCG kernels only; not a solve mode) */
  MBL_MIXED = 2,  /* solve: FP32 apply, block updates, FP32-MFMA Gram and FP32
                     PCG; FP64 small dense algebra; then a closing FP64 pass
                     (FP64 blocks, FP32 PCG) down to the tolerance           */
  MBL_PCG32 = 3   /* solve: FP64 blocks and Rayleigh-Ritz, FP32 PCG only
                     (the precision split of the paper, Sec. 6)               */
} mbl_precision;

typedef struct mbl_ham_s* mbl_ham;

/* Allocation callbacks (optional).  alloc returns device memory of at least
 * `bytes` usable on `stream`, or NULL; free releases it.  NULL, NULL restores
 * hipMalloc/hipFree.  Not thread-safe with concurrent library calls. */
typedef void* (*mbl_alloc_fn)(size_t bytes, hipStream_t stream, void* ctx);
typedef void (*mbl_free_fn)(void* ptr, hipStream_t stream, void* ctx);
mbl_status mbl_set_allocator(mbl_alloc_fn alloc, mbl_free_fn free_fn, void* ctx);

const char* mbl_last_error(void);
int mbl_version(void);

/* ---- sector and Hamiltonian (paper Sec. 2.1, eq. (1)/(2)) ---------------- */

/* Build the handle for one sector: validates 2 <= L <= 32, 2*Sz integer with
 * the parity of L and |Sz| <= L/2, finite J, Delta, h_host[0..L-1].  Builds
 * the Pascal table C(i, t), the state list (uint32 per row) and the diagonal
 * <s|H|s> on the device (async on `stream`, which is synchronised before
 * return).  The sector's sparsity pattern is independent of h (Sec. 4.2), so
 * the tables could be shared between realisations; here each handle owns its
 * own. */
mbl_status mbl_hamiltonian_create(int L, double Sz, double J, double Delta,
                                  const double* h_host, hipStream_t stream,
                                  mbl_ham* out);
mbl_status mbl_hamiltonian_destroy(mbl_ham H);
mbl_status mbl_hamiltonian_dim(mbl_ham H, int64_t* n);

/* The n sector states in row order, as 64-bit integers (host output). */
mbl_status mbl_sector_states(mbl_ham H, uint64_t* states_host);

/* Row index of each query state (host arrays); -1 if the state is not in the
 * sector (wrong number of up spins or a bit at position >= L). */
mbl_status mbl_rank(mbl_ham H, const uint64_t* states_host, int64_t count,
                    int64_t* idx_host);

/* diag_dev[r] = <s_r|H|s_r>; jacobi_dev[r] = diag of (H - sigma I)^2 for row
 * r, the Jacobi preconditioner of the PCG inner solve (Sec. 3.2).  Either
 * output may be NULL.  Device FP64 arrays of length n.  Async. */
mbl_status mbl_diagonal(mbl_ham H, double sigma, double* diag_dev,
                        double* jacobi_dev, hipStream_t stream);

/* ---- matrix-free block apply (paper Sec. 3.2 and 4.1) -------------------- */

/* Y = (H - sigma I) X for an n x b block, never forming H.  prec MBL_F64 or
 * MBL_F32 selects the element type of X and Y.  ldx, ldy >= b.  X and Y must
 * not overlap.  Async.  The launch schedule comes from the library's table of
 * tuned schedules (nearest sector size, same row width); the environment
 * variables MBL_APPLY_CHUNK_BYTES, MBL_APPLY_LANE_BYTES, MBL_APPLY_XCD_GROUP and
 * MBL_APPLY_SLOTS_PER_XCD override its fields (they also apply to mbl_pcg).
 * MBL_APPLY_SPLIT=1 selects the two-pass kernel instead (the chain cut in two
 * halves, each half's flips gathered from an LDS tile; also used by mbl_pcg
 * and the solvers); MBL_SPLIT_PANEL_BYTES and MBL_SPLIT_SLOTS override its
 * column-panel width and workgroups per XCD.  Both kernels compute the same
 * sums in different orders. */
mbl_status mbl_apply_block(mbl_ham H, double sigma, mbl_precision prec,
                           const void* X, int64_t ldx, void* Y, int64_t ldy,
                           int b, hipStream_t stream);

/* Y = (H - sigma I)^2 X, the spectral fold (Sec. 3.2), as two applies through
 * the caller's intermediate T = (H - sigma I) X (n x b, ldt >= b).  Async. */
mbl_status mbl_fold_apply(mbl_ham H, double sigma, mbl_precision prec,
                          const void* X, int64_t ldx, void* T, int64_t ldt,
                          void* Y, int64_t ldy, int b, hipStream_t stream);

/* W = m steps of Jacobi-preconditioned CG on (H - sigma I)^2 W = R, each
 * column independently, starting from W = 0 (the LOBPCG preconditioner,
 * Sec. 3.2).  prec MBL_F64 or MBL_F32 is the element type of R, W and of the
 * CG arithmetic.  m >= 0.  Synchronises `stream`. */
mbl_status mbl_pcg(mbl_ham H, double sigma, mbl_precision prec, const void* R,
                   int64_t ldr, void* W, int64_t ldw, int b, int m,
                   hipStream_t stream);

/* ---- dense block kernels (LOBPCG's matrix-matrix work, Sec. 3.2 (ii)) ---- */

/* C_dev (p x q, row-major, ldc >= q, FP64) = A^T B for n x p A and n x q B of
 * element type prec (MBL_F64 or MBL_F32), reduced in a fixed order (results
 * are bitwise reproducible).  Matrix-core (MFMA) kernel.  Async. */
mbl_status mbl_gram(mbl_precision prec, int64_t n, const void* A, int64_t lda,
                    int p, const void* B, int64_t ldb, int q, double* C_dev,
                    int64_t ldc, hipStream_t stream);

/* mbl_gram without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels, reduction order and
 * results (bitwise) as mbl_gram.  The per-split partial sums go to a fixed
 * array of MBL_GRAM_SCRATCH_BYTES in device memory, one per GPU, held from
 * the library's first use of this call on that GPU until the process ends.
 * Shapes whose partials do not fit (p, q beyond about 2048 columns; the
 * library computes splits x p x q x 8 bytes) return MBL_EINVAL.  All calls on
 * one GPU share the array: calls that may overlap on that GPU (two streams,
 * two threads) race and must be serialised by the caller.  Async. */
#define MBL_GRAM_SCRATCH_BYTES ((size_t)64 << 20)
mbl_status mbl_gram_noalloc(mbl_precision prec, int64_t n, const void* A,
                            int64_t lda, int p, const void* B, int64_t ldb,
                            int q, double* C_dev, int64_t ldc,
                            hipStream_t stream);

/* Y (n x q) = A (n x p) C (p x q, FP64 device, row-major ldc) in element type
 * prec.  Y must not overlap A.  Async. */
mbl_status mbl_block_combine(mbl_precision prec, int64_t n, const void* A,
                             int64_t lda, int p, const double* C_dev,
                             int64_t ldc, void* Y, int64_t ldy, int q,
                             hipStream_t stream);

/* Symmetric eigendecomposition of an m x m FP64 device matrix (row-major,
 * lda >= m; only read): w_dev ascending, V_dev columns the eigenvectors
 * (row-major, ldv >= m).  One-workgroup cyclic Jacobi.  m <= 1024.  Async. */
mbl_status mbl_small_eigh(int m, const double* A_dev, int64_t lda,
                          double* w_dev, double* V_dev, int64_t ldv,
                          hipStream_t stream);

/* ---- eigensolver (paper Sec. 3.2) ---------------------------------------- */

/* Extreme eigenvalues of H in the sector, each to absolute accuracy `tol`
 * (tol >= 1e-14), by LOBPCG on H and on -H.  Synchronises `stream`. */
mbl_status mbl_spectrum_bounds(mbl_ham H, double tol, double* emin,
                               double* emax, hipStream_t stream);

typedef struct {
  int max_iter;          /* LOBPCG outer iterations (default 400)            */
  int pcg_iters;         /* CG steps per LOBPCG iteration; 0 = by dimension  */
  int precision;         /* mbl_precision: MBL_F64, MBL_MIXED or MBL_PCG32   */
  int verbose;           /* 1: one line per outer iteration on stderr        */
  int timing;            /* 1: time the two fused CG apply kernels with HIP
                            events on the solve's stream (the first 64 CG
                            steps of every inner CG call and column chunk,
                            extrapolated to all its steps), and the apply,
                            Gram and small dense phases                      */
  uint64_t seed;         /* starting block (device counter-based generator)  */
  int lock;              /* 1: soft locking.  Wanted pairs whose tracked
                            residual is <= tol/10 keep their place in X and
                            in every Rayleigh-Ritz step but get no new
                            preconditioned direction: the fold residual is
                            rotated into the H-Ritz basis of span(X), their
                            columns are left out, and the remaining width is
                            rounded up to whole 128-byte rows of the CG's
                            scalars (least converged locked pairs stay
                            active), so the inner CG runs on fewer columns.
                            With guard columns (guard_cg) the unlocked
                            wanted pairs lead the rotated block and run all
                            the CG steps.  Results satisfy the same
                            tolerance; iterates differ from lock = 0.
                            Default 0.                                       */
  double max_seconds;    /* > 0: wall-clock limit of the call.  Checked
                            between outer iterations and every 32 CG steps;
                            when it passes, the solve finishes the CG chunk
                            in flight, extracts the current best pairs with
                            fresh FP64 residuals and returns MBL_ECANCELLED
                            (MBL_OK if they already meet tol).  0 = none.   */
  const volatile int* cancel;  /* host flag, may be NULL: a nonzero value
                            stops the solve the same way (set it from
                            another thread).                                 */
  double guard_cg;       /* fraction (0, 1] of the pcg_iters CG steps given to
                            the guard columns of the block (those beyond the
                            nev smallest fold Ritz values); the nev leading
                            columns always run all pcg_iters steps.  0 = by
                            shape: 0.05 for sectors of n >= 500000 with
                            nev >= 64 (measured 1.47x faster at L = 22 and
                            L = 24, nev 64, block 128), else 1 (with nev 16,
                            block 32 the
                            narrowed CG saves too little per step: 1.68x
                            slower at L = 22).  With soft locking the guard
                            columns are those beyond the unlocked wanted
                            pairs.                                           */
} mbl_solve_opts;

typedef struct {
  int iters;             /* outer LOBPCG iterations in total                 */
  int iters_fp64;        /* of which in the closing FP64 pass (MBL_MIXED)    */
  int nconv;             /* wanted pairs with residual <= tol                */
  int64_t applies;       /* block applies of (H - sigma I), all kernels      */
  int64_t pcg_steps;     /* CG steps in total                                */
  double seconds;        /* wall time of the call                            */
  double t_pcg;          /* seconds in the PCG inner solves                  */
  double t_rr;           /* seconds in Gram / Rayleigh-Ritz / orthonormalising */
  double max_resid;      /* max ||H x - lambda x||_2 over the returned pairs */
  /* opts.timing: timed launches and their summed milliseconds of the CG
     kernels T = (H - sigma) p (+ |T|^2) and q = (H - sigma) T (+ x, r update,
     r.z); FP32 and FP64 inner solves are counted separately.               */
  int64_t cg_apply1_launches[2], cg_apply2_launches[2];  /* [0]=FP64 [1]=FP32 */
  double cg_apply1_ms[2], cg_apply2_ms[2];
  /* algorithmic bytes of those launches: apply1 2nws + 12n, apply2
     6nws + (12 + s)n for a launch over w columns of s-byte scalars          */
  double cg_apply1_bytes[2], cg_apply2_bytes[2];
  int64_t pcg_columns;   /* CG steps times block columns, summed over inner
                            solves (fewer than pcg_steps * block with lock or
                            guard columns)                                   */
  /* opts.timing: device seconds (HIP events) of the applies outside the CG
     (residual blocks, new directions, fresh residuals), the Gram products and
     the small dense kernels (eigensolver, Cholesky, small products)        */
  double t_apply, t_gram, t_small;
  int cg_split;          /* the timed CG steps ran the two-pass kernels      */
  /* opts.timing: every CG step of the solve (the timed ones are the first up
     to 64 of each inner CG call, of each column chunk): launches of each CG
     kernel, their algorithmic bytes, and their device milliseconds estimated
     per inner CG call as the timed launches' mean times its steps (the other
     steps replay the same launches from a captured graph).  [0]=FP64 [1]=FP32 */
  int64_t cg_launches_all[2];
  double cg_apply1_ms_all[2], cg_apply2_ms_all[2];
  double cg_apply1_bytes_all[2], cg_apply2_bytes_all[2];
} mbl_solve_info;

mbl_status mbl_solve_opts_default(mbl_solve_opts* opts);

/* The nev eigenpairs of H with eigenvalues nearest sigma, by LOBPCG with
 * block size `block` on the spectral fold (H - sigma I)^2, preconditioned by
 * Jacobi-PCG (Sec. 3.2).  Converged when every wanted pair has
 * ||H x - lambda x||_2 <= tol (absolute, unit x, evaluated in FP64 with a
 * fresh apply).  Requires 1 <= nev <= block, 2 * block <= n, tol > 0.
 * Outputs: evals_host[nev] ascending, resid_host[nev], evecs_dev (n x nev
 * FP64 row-major, ldv >= nev; may be NULL), info (may be NULL); opts NULL =
 * defaults.  Returns MBL_ENOCONV with the best pairs if max_iter is reached.
 * Synchronises `stream`. */
mbl_status mbl_lobpcg_solve(mbl_ham H, double sigma, int nev, int block,
                            double tol, const mbl_solve_opts* opts,
                            double* evals_host, double* evecs_dev, int64_t ldv,
                            double* resid_host, mbl_solve_info* info,
                            hipStream_t stream);

/* ---- MBL observables and spectrum slices (paper Sec. 2.2, 3.1) ----------- */

/* Von Neumann entanglement entropy (natural log) of each of the nev unit
 * eigenvectors (device, n x nev FP64, ld ldv) across the cut between sites
 * cut-1 and cut (left part: sites 0..cut-1).  1 <= cut <= L-1 and
 * L - cut <= 26.  S_host[nev].  Synchronises `stream`. */
mbl_status mbl_entanglement_entropy(mbl_ham H, const double* V_dev, int64_t ldv, int nev,
                                    int cut, double* S_host, hipStream_t stream);

/* Mean adjacent gap ratio <min(d_n, d_n+1) / max(d_n, d_n+1)> of `count`
 * eigenvalues (host; sorted internally; count >= 3). */
mbl_status mbl_gap_ratio(const double* evals_host, int count, double* mean_r);

/* Eigenvalue chunks of one H: for each of `count` shifts, the nev eigenpairs
 * nearest it (as mbl_lobpcg_solve, eigenvalues and residuals only), solved
 * `concurrency` at a time on worker streams sharing the handle.
 * evals_host[count*nev], resid_host[count*nev] (may be NULL). */
mbl_status mbl_slices_solve(mbl_ham H, int count, const double* sigmas_host, int nev, int block,
                            double tol, const mbl_solve_opts* opts, double* evals_host,
                            double* resid_host, int concurrency);

/* ---- many independent solves (paper Sec. 3.1: realisations, disorder
 * strengths and spectral regions are independent levels of concurrency) ---- */

typedef struct {
  int L;
  double Sz, J, Delta;
  const double* h_host;  /* length L; copied by submit / read during batch   */
  double sigma;          /* used when eps < 0                                */
  double eps;            /* >= 0: sigma = Emin + eps (Emax - Emin), with the
                            bounds computed on the GPU (mbl_spectrum_bounds) */
  int nev, block;
  double tol;
  int precision;         /* MBL_F64, MBL_MIXED or MBL_PCG32                  */
  int max_iter, pcg_iters;
  uint64_t seed;
  int want_vectors;      /* server only: keep the n x nev FP64 eigenvectors on
                            the device until wait() copies them to
                            out->evecs_dev (batch: results[i].evecs_dev)     */
} mbl_problem;

typedef struct {
  int status;            /* mbl_status of this problem                       */
  double sigma;          /* shift actually used                              */
  int nconv, iters;
  int64_t applies;
  double max_resid;
  double seconds;        /* wall time of this problem's solve                */
  double latency;        /* submit (or batch start) to completion, seconds   */
  double* evals_host;    /* caller-provided, nev entries (may be NULL)       */
  double* resid_host;    /* caller-provided, nev entries (may be NULL)       */
  double* evecs_dev;     /* caller-provided device n x nev, ld ldv (or NULL) */
  int64_t ldv;
} mbl_result;

/* Device bytes one solve holds at its peak (n-length blocks of the LOBPCG and
 * PCG work space plus the sector tables).  Pure host function: this is the
 * admission model of the server below. */
mbl_status mbl_footprint_bytes(int L, double Sz, int block, int precision, size_t* bytes);

/* Solve `count` independent problems, `concurrency` at a time (>= 1), each on
 * its own non-blocking stream of the current device.  Every solve is the same
 * deterministic computation as mbl_lobpcg_solve, so a problem's result does
 * not depend on what runs beside it.  Per-problem outcomes are in results[i]
 * (status, sigma, counts, timings; evals/resid/evecs into caller buffers).
 * Returns MBL_OK if every problem converged, else the first problem's error.
 * With the environment variable MBL_VERBOSE=1, batch and server solves print
 * one line per outer iteration to stderr.  MBL_BATCH_FUSE=1 runs the inner CG
 * calls of concurrent solves that share a launch plan as one launch per
 * kernel (problem j's workgroups are its own grid, so results keep their
 * bits); MBL_FUSE_WAIT_MS (default 0.5) is how long the first call of a group
 * waits for the others, and MBL_FUSE_STATS=1 prints the groups formed. */
mbl_status mbl_batch_solve(int count, const mbl_problem* problems, mbl_result* results,
                           int concurrency);

/* Serving loop with continuous batching on HIP device `device`: submit()
 * queues a request and returns at once; `max_slots` worker threads take
 * requests in arrival order as soon as a slot is free and the sum of admitted
 * footprints stays within hbm_budget (bytes; 0 = 90% of the device's free
 * memory at creation), so requests that arrive while others run are started
 * beside them.  A request whose footprint exceeds the whole budget is refused
 * at submit (MBL_ENOMEM).  wait() blocks for a ticket (timeout_s < 0: forever)
 * and fills `out` (its buffers must stay valid until wait returns).  Results
 * are kept until waited for.  Thread-safe.  The statistics call is named
 * mbl_server_stats_get because mbl_server_stats names its struct. */
typedef struct mbl_server_s* mbl_server;
typedef struct {
  int64_t submitted, admitted, completed, rejected, in_flight;
  double p50_latency, p99_latency;  /* seconds, submit to completion        */
  double throughput_pairs;          /* converged pairs / s since creation   */
  size_t budget_bytes, peak_bytes;
} mbl_server_stats;

mbl_status mbl_server_create(int device, size_t hbm_budget, int max_slots, mbl_server* out);
mbl_status mbl_server_submit(mbl_server srv, const mbl_problem* request, uint64_t* ticket);
/* Returns MBL_OK when the request finished (its own status is out->status),
 * MBL_ETIMEOUT if it is still running after timeout_s. */
mbl_status mbl_server_wait(mbl_server srv, uint64_t ticket, double timeout_s, mbl_result* out);
/* Cancels a request that has not finished: a queued one is dropped, a running
 * one stops within one chunk of CG steps.  Its result (still to be waited for)
 * has status MBL_ECANCELLED (a running solve returns its best pairs so far).
 * MBL_EINVAL for an unknown or already finished ticket. */
mbl_status mbl_server_cancel(mbl_server srv, uint64_t ticket);
mbl_status mbl_server_stats_get(mbl_server srv, mbl_server_stats* st);
/* Waits for every submitted request, then stops the workers. */
mbl_status mbl_server_destroy(mbl_server srv);

#ifdef __cplusplus
}
#endif
#endif /* MBL_H_ */
