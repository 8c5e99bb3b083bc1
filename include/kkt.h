/*
 * kkt.h -- C ABI of a GPU-resident solver for sequences of sparse KKT systems that share
 * one sparsity pattern, on AMD Instinct MI355X (gfx950).
 *
 * Method (Swirydowicz, Koukpaizan, Alam, Regev, Saunders, Peles, "Iterative Methods in
 * GPU-Resident Linear Solvers for Nonlinear Constrained Optimization"):
 *   - the systems K_k dx_k = r_k of eq. (kktlinear) share one pattern (Section 1.2, "Summary");
 *   - the first system gets a full symbolic analysis and a factorization with pivoting on the
 *     host; every later system gets a numeric refactorization on the GPU that reuses the
 *     pattern and the pivot sequence (static pivoting, Section 1.3);
 *   - the direct solution x0 = Q U^-1 L^-1 P r is refined by FGMRES with the LU factors as a
 *     right preconditioner, CGS2 orthogonalization, the estimated residual as stopping test
 *     and the solution formed only at restart/convergence (Section 2.1); refinement runs only
 *     when ||r - K x0|| / ||r|| >= delta_tol (Section 2.3).
 *
 * Conventions for every entry point:
 *   - Matrices are CSR: int64 row pointers (N+1), int32 column indices sorted ascending
 *     within each row with no duplicates, float64 values.  The FULL symmetric matrix is
 *     passed (both triangles).  Indices are 0-based.
 *   - "host" pointers are read during the call only; the library keeps its own copies.
 *   - "device" pointers are caller-owned HIP device memory, read or written only on the
 *     given stream for the duration of the call (the call returns after the work on that
 *     stream has been issued, or after it completes where stated).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - No exception crosses the ABI: every call returns a kkt_status_t; kkt_last_error()
 *     gives a message for the last failing call on the handle.
 *   - One handle is used by one host thread at a time; distinct handles are independent.
 */
#ifndef KKT_H
#define KKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kkt_handle_s *kkt_handle_t;

typedef enum {
    KKT_OK = 0,
    KKT_EINVAL = 1,     /* invalid argument or input (bad CSR, non-finite values, ...) */
    KKT_ENOMEM = 2,     /* host allocation failed or the workspace is too small */
    KKT_ESINGULAR = 3,  /* singular column in the pivoted analysis, or a guarded pivot with
                           guard_policy = KKT_GUARD_FAIL */
    KKT_ENOCONV = 4,    /* FGMRES-IR did not meet the tolerance; x holds the iterate with the
                           lowest true residual ||r - K x||_2 seen (x0 included) and the info
                           describes that iterate */
    KKT_EDEVICE = 5,    /* a HIP call failed; the handle accepts only kkt_release() */
    KKT_ESTATE = 6      /* call out of order (solve before refactor, no workspace, ...) */
} kkt_status_t;

enum { KKT_PREC_FP64 = 0, KKT_PREC_MIXED = 1 };     /* factor / preconditioner precision */
enum { KKT_GUARD_PERTURB = 0, KKT_GUARD_FAIL = 1 }; /* tiny static pivot policy */
enum { KKT_STOP_PAPER = 0, KKT_STOP_NRBE = 1 };     /* FGMRES-IR stopping control */

enum { KKT_ORDER_MD = 0, KKT_ORDER_ND = 1 };      /* fill-reducing ordering */

typedef struct {
    int32_t ordering;       /* KKT_ORDER_MD: exact minimum degree on the elimination graph of
                               K + K^T (ties: smallest index), default; KKT_ORDER_ND: BFS nested
                               dissection */
    int32_t nd_leaf;        /* nested dissection: sets of <= nd_leaf vertices are not dissected (64) */
    double pivot_tau;       /* threshold partial pivoting: keep the diagonal row when
                               |x_c| >= tau * max |x_i| (1e-10).  K_k of eq. (kktlinear) with a
                               dual regularization -delta I (delta > 0) is quasi-definite, so every
                               diagonal pivot of a symmetric ordering is nonzero; a small tau keeps
                               them, gives P = Q (symmetric factor patterns, least fill) and a
                               pivot sequence that stays valid when D is redrawn.  tau = 0.1
                               (textbook threshold pivoting) picks off-diagonal pivots from system
                               1's D that later systems no longer support. */
    int32_t restart;        /* FGMRES restart length R (10, Section 4.1.1) */
    int32_t max_restarts;   /* cycles after the first (20) */
    double delta_tol;       /* refine/stop tolerance delta_tol (1e-14, Section 4.1.2) */
    double nrbe_target;     /* accept only when NRBE (eq. (nbre)) <= this (1e-12) */
    int32_t precision;      /* KKT_PREC_FP64 or KKT_PREC_MIXED (FP32 factors and triangular
                               solves as preconditioner, FP64 Krylov) */
    int32_t guard_policy;   /* KKT_GUARD_PERTURB: replace a static pivot with
                               |u_jj| <= u * max_i |K(i,Q[j])| by sign(u_jj) u colmax and count
                               it; KKT_GUARD_FAIL: report KKT_ESINGULAR */
    int32_t stop_mode;      /* KKT_STOP_PAPER: refine iff ||rho0||/||r|| >= delta_tol, stop
                               on estimated RR < delta_tol, accept iff also NRBE <=
                               nrbe_target; KKT_STOP_NRBE: refine iff NRBE(x0) > nrbe_target,
                               inner test |g| <= nrbe_target (||K||inf ||x|| + ||r||) */
    int32_t mixed_fallback; /* mixed precision: on non-convergence refactor in FP64 and
                               solve again (1) or return KKT_ENOCONV (0) */
    int32_t mixed_max_cycles; /* mixed precision: restart cycles tried with the FP32
                               preconditioner before the fallback (3) */
    int32_t ir_method;      /* KKT_IR_FGMRES (the method of Section 2.1, default),
                               KKT_IR_RICHARDSON (x += M^-1 (r - K x), Section 1.3) or
                               KKT_IR_ERROR_FGMRES (Richardson whose correction solves the error
                               system K d = rho with FGMRES(restart), Section 2.1) */
    int32_t richardson_max_it; /* Richardson: corrections at most (50) */
    double ratio_stop;      /* Richardson: stop when NSR_new > ratio_stop * NSR_old, MA57's
                               ratio test (0.5) */
    double inner_tol;       /* error-system FGMRES: relative tolerance of each inner solve (1e-2) */
    int32_t residual;       /* KKT_RESID_FP64 (default) or KKT_RESID_DD: every true residual
                               rho = b - K x of the refinement carried in double-double and
                               rounded once (the extended-precision residual of three-precision
                               iterative refinement, Section 2) */
    int32_t repivot_cycles; /* when > 0: if FGMRES-IR with the current pivot sequence has not
                               converged after this many restart cycles, the solve downloads
                               the system's values, repeats the threshold-pivoted factorization
                               on the host (ordering kept), rebuilds the schedules in the bound
                               workspace, refactors and solves again; later systems use the new
                               pivot sequence (3).  0: the pivot sequence of system 1 is kept. */
    int32_t gram_schmidt;   /* KKT_GS_CGS2: two classical Gram-Schmidt passes per Arnoldi step
                               (Section 2.1, default).  KKT_GS_DCGS2: delayed CGS2, one of the
                               low-synchronization FGMRES variants Section 2.1 cites (Bielich et
                               al. 2022): one reduction per step, the second pass and the
                               normalization of each vector deferred to the next step's
                               reduction; 2 kernels per step after the triangular solves
                               instead of 4, the same Krylov basis, and one preconditioner
                               application more per cycle that converges before its restart */
    int32_t tile_lds_kib;   /* LDS budget of one staged triangular-solve tile in KiB, 16..150
                               (0: 32).  Larger tiles hold more levels of the elimination tree,
                               so fewer cross-block hands-offs lie on a solve's critical path;
                               smaller ones let more blocks share a compute unit (measured
                               faster at 32 than at 64 on 60k and 2M unknowns); above 80 KiB
                               one solve block occupies a compute unit alone */
    int32_t narrow_columns; /* refactorization levels with at most this many columns are handed
                               out one column per wavefront, wider ones as lane items (64
                               short columns, one per lane) and chunks of 8 longer columns (0:
                               automatic, the larger of 3,072 (the refactorization's resident
                               wavefronts) and n/64 capped at 16,384; measured best at 60k,
                               500k and 2M unknowns); negative values are rejected
                               (KKT_EINVAL).  The factors do not depend on it. */
    int32_t deterministic;  /* 1 (default): bitwise-repeatable results.  Every kernel reduces in
                               a fixed order and none uses floating-point atomics, so a solve
                               gives the same bits alone, batched, in a serving mix or on a
                               rerun; there is no faster nondeterministic mode, and any value
                               other than 1 is rejected (KKT_EINVAL) */
} kkt_opts_t;

enum { KKT_IR_FGMRES = 0, KKT_IR_RICHARDSON = 1, KKT_IR_ERROR_FGMRES = 2 };
enum { KKT_RESID_FP64 = 0, KKT_RESID_DD = 1 };
enum { KKT_GS_CGS2 = 0, KKT_GS_DCGS2 = 1 };

/* Kernel classes reported by kkt_get_kernel_times. */
enum {
    KKT_K_INGEST = 0,   /* values into factor storage, ||K||_inf, finiteness checks */
    KKT_K_REFACTOR = 1, /* numeric refactorization */
    KKT_K_TRSV_L = 2,   /* forward substitution with L (one launch per preconditioner use) */
    KKT_K_TRSV_U = 3,   /* backward substitution with U */
    KKT_K_SPMV = 4,     /* w = K z_j with the first Gram-Schmidt projections */
    KKT_K_CGS = 5,      /* second Gram-Schmidt pass, norm, rotation, normalization */
    KKT_K_RESID = 6,    /* true residual rho = b - K x with norms */
    KKT_K_OTHER = 7,    /* cycle start, least squares, solution update, sentinel reset */
    KKT_K_CLASSES = 8
};

typedef struct {
    int64_t launches[KKT_K_CLASSES]; /* timed launches per class */
    double ms[KKT_K_CLASSES];        /* summed device time per class (HIP events) */
} kkt_kernel_times_t;

typedef struct {
    int64_t n;              /* N */
    int64_t nnz;            /* nonzeros of K (full) */
    int64_t nnz_l;          /* strictly lower nonzeros of L */
    int64_t nnz_u;          /* nonzeros of U including the diagonal */
    int64_t offdiag_pivots; /* analysis pivots not on the diagonal of K(:,Q) */
    int64_t levels_refactor;/* depth of the column dependency DAG of the refactorization */
    int64_t levels_l;       /* depth of the row DAG of the L solve */
    int64_t levels_u;       /* depth of the row DAG of the U solve */
    int64_t updates;        /* scalar multiply-subtract updates per refactorization */
    double analysis_seconds;/* host time spent in kkt_analyze */
    int64_t max_column;     /* longest factor column (U part, diagonal and L part); columns
                               beyond the refactorization's LDS stage are updated in HBM */
    int64_t tiles_l;        /* triangular-solve tiles of L (see kkt_bind_workspace) */
    int64_t tiles_u;        /* ... and of U */
    int64_t unstaged_l;     /* tiles of L whose row is too long for LDS (read from HBM) */
    int64_t unstaged_u;     /* ... and of U */
} kkt_analysis_info_t;

typedef struct {
    int32_t converged;       /* 1 if the accept test passed */
    int32_t iterations;      /* FGMRES (Arnoldi) iterations in total */
    int32_t cycles;          /* restart cycles run (0 when refinement was skipped) */
    int32_t refined;         /* 1 if the refine test asked for FGMRES */
    int32_t precision;       /* precision of the factors that produced x */
    int32_t fallback;        /* 1 if a mixed solve fell back to FP64 factors */
    int64_t pivots_perturbed;/* guarded static pivots in the last refactorization */
    double nrbe;             /* ||r - K x||_2 / (||K||_inf ||x||_2 + ||r||_2) */
    double nrbe0;            /* the same for the direct solution x0 */
    double rel_resid;        /* ||r - K x||_2 / ||r||_2 */
    double rr;               /* ||r - K x||_2 / ||r - K x0||_2 (true residuals) */
    double est_resid;        /* last estimated FGMRES residual norm */
    double true_resid;       /* ||r - K x||_2 */
    double knorm_inf;        /* ||K||_inf */
    double nsr;              /* ||r - K x||_inf / (||K||_inf ||x||_inf), MA57's measure */
    int64_t precond_applications; /* triangular-solve pairs (x0 included) */
    int32_t repivoted;       /* 1 if this solve re-pivoted (opts.repivot_cycles) */
    int32_t restored_best;   /* 1 if the solve did not converge and x was set back to an
                                earlier iterate with a lower true residual */
} kkt_solve_info_t;

/* Fill *opts with the defaults listed above. */
void kkt_opts_default(kkt_opts_t *opts);

/* Analyse a pattern on the host with the values of the first system (Section 1.3: symbolic
 * analysis plus factorization with pivoting on system 1): validates the CSR, computes the
 * fill-reducing ordering Q and a threshold-pivoted left-looking LU of K(:,Q), and builds
 * every schedule the GPU kernels need.  rowptr/colidx/values_first are HOST pointers.  Does
 * not touch the GPU.  On success *out owns a new handle (release with kkt_release).
 * Errors: KKT_EINVAL (bad CSR, N < 1, non-finite value), KKT_ESINGULAR (no nonzero pivot
 * candidate; the column is named in kkt_last_error), KKT_ENOMEM. */
kkt_status_t kkt_analyze(const kkt_opts_t *opts, int64_t n, const int64_t *rowptr,
                         const int32_t *colidx, const double *values_first, kkt_handle_t *out);

/* Sizes and schedule statistics of the analysis (host only). */
kkt_status_t kkt_get_analysis_info(kkt_handle_t h, kkt_analysis_info_t *info);

/* Pivot sequence and ordering: prow[k] = row of K pivoted at step k, q[k] = column of K
 * eliminated at step k, so that P K Q = L U (host arrays of n entries). */
kkt_status_t kkt_get_permutations(kkt_handle_t h, int32_t *prow, int32_t *q);

/* Factor patterns in column-compressed form (host arrays): L strictly lower with ORIGINAL
 * row indices of K ascending per column (lp: n+1, li: nnz_l); U upper with pivot-step row
 * indices ascending per column, diagonal last (up: n+1, ui: nnz_u). */
kkt_status_t kkt_get_factor_pattern(kkt_handle_t h, int64_t *lp, int32_t *li, int64_t *up,
                                    int32_t *ui);

/* Values of the host analysis factorization (system 1), in the layout of
 * kkt_get_factor_pattern (host arrays, nnz_l and nnz_u entries). */
kkt_status_t kkt_get_analysis_values(kkt_handle_t h, double *lx, double *ux);

/* Device bytes needed by kkt_bind_workspace for `batch` >= 1 handles of this analysis (each
 * handle of a kkt_refactor_batch call binds a workspace of its own: factor values in FP64 and
 * FP32, structure arrays, Krylov basis V and Z for the restart length, scratch), i.e. batch
 * times the size of one.  Errors: KKT_EINVAL (batch < 1). */
kkt_status_t kkt_workspace_size(kkt_handle_t h, int32_t batch, size_t *bytes);

/* Bind caller-owned device memory (>= kkt_workspace_size bytes, 256-byte aligned) and upload
 * the structure arrays on `stream` (synchronous on return).  The current HIP device at this
 * call is the handle's device.  Rebinding replaces the previous workspace. */
kkt_status_t kkt_bind_workspace(kkt_handle_t h, void *dev_ptr, size_t bytes, void *stream);

/* Numeric refactorization of a new system with the fixed pattern and pivot sequence
 * (Section 1.3 / 2.1).  dev_values: DEVICE array of nnz float64 values in the CSR order of
 * the analysed pattern; copied into the workspace, so it may be reused after the call's
 * work completes.  Work is enqueued on `stream`; tiny-pivot guards are counted on the device
 * and reported by the next kkt_solve.  Errors: KKT_ESTATE (no workspace). */
kkt_status_t kkt_refactor(kkt_handle_t h, const double *dev_values, void *stream);

/* kkt_refactor for `count` (1..8) systems of one pattern in one refactorization launch: handle
 * hs[b] refactors the values at DEVICE array dev_values[b] (nnz float64 each).  The handles
 * must be distinct, bound, and share one analysis (kkt_clone copies of one handle, none of
 * them re-pivoted since) with the same precision and guard policy.  Ingest runs per system;
 * the columns of all systems are then handed out together, so each system's factors are the
 * same bits as its own kkt_refactor.  Enqueued on `stream`.  Errors: KKT_EINVAL (count out of
 * range, a handle twice, different analyses, options or devices), KKT_ESTATE (a handle not
 * bound), KKT_EDEVICE. */
kkt_status_t kkt_refactor_batch(const kkt_handle_t *hs, const double *const *dev_values, int32_t count,
                                void *stream);

/* kkt_refactor_batch through a HIP graph: the values are first copied into each handle's
 * workspace (device to device, on `stream`); the ingest and refactorization kernels of the
 * batch are captured once per (handles, their current workspace bindings, precision) and the
 * instantiated graph is replayed on later calls with the same handles (no kernel launches from
 * the host).  The result is the same as kkt_refactor_batch's, bit for bit.  A graph is dropped
 * when one of its handles is released; rebinding a handle's workspace makes a new graph.
 * Errors: those of kkt_refactor_batch. */
kkt_status_t kkt_refactor_batch_graph(const kkt_handle_t *hs, const double *const *dev_values, int32_t count,
                                      void *stream);

/* Refactorizations of this handle replayed from a captured graph so far. */
kkt_status_t kkt_graph_launches(kkt_handle_t h, int64_t *launches);

/* Solve K x = b for the last refactored K: direct solve, refine decision, FGMRES-IR
 * (Section 2).  dev_b, dev_x: DEVICE arrays of n float64 (distinct).  tol <= 0 uses
 * opts.delta_tol.  Waits for each Arnoldi step's stop flag while the next step runs, and
 * synchronizes `stream` at each restart and before returning; *info
 * (may be NULL) is filled on return.  Errors: KKT_ESTATE (no refactor yet), KKT_EINVAL
 * (non-finite K values or b), KKT_ESINGULAR (guard_policy = FAIL and a guarded pivot),
 * KKT_ENOCONV (tolerance not met; x holds the iterate with the lowest true residual seen,
 * x0 included, and info describes it).  An iterate whose true residual exceeds that of x0 is
 * never accepted, in either stop_mode. */
kkt_status_t kkt_solve(kkt_handle_t h, const double *dev_b, double *dev_x, double tol,
                       kkt_solve_info_t *info, void *stream);

/* Apply the current preconditioner once: x = Q U^-1 L^-1 P b with the last refactored
 * factors (the direct solve of Section 1.3, no refinement).  DEVICE arrays of n float64.
 * Enqueued on `stream`, not synchronized. */
kkt_status_t kkt_direct_solve(kkt_handle_t h, const double *dev_b, double *dev_x, void *stream);

/* kkt_direct_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result bit for bit, but the intermediate vectors of the two sweeps and their tile counters
 * live in a static device array of the library (32 MiB + 256 B per GPU, held until the process
 * ends) instead of the handle's workspace.  It calls no allocating routine.  The handle must be
 * bound and refactored (its factors are read from its workspace), n <= 2,097,152 (else
 * KKT_EINVAL, checked before any device call) and the handle's device current (else
 * KKT_EINVAL).  DEVICE arrays of n float64; enqueued on `stream`, not synchronized.  Every
 * call on one GPU uses that GPU's single copy of the array: calls that overlap on one GPU
 * (other streams, other threads) race and give undefined results; serialize them. */
kkt_status_t kkt_direct_solve_noalloc(kkt_handle_t h, const double *dev_b, double *dev_x, void *stream);

/* Residual rho = b - K x of the last refactored K (original ordering), each row summed in
 * CSR order; with opts.residual = KKT_RESID_DD the row is carried as a double-double sum
 * (error-free products and the accurate double-word addition of Joldes, Muller and Popescu)
 * and rounded once.  DEVICE arrays of n float64 (dev_r distinct from the others).  Enqueued
 * on `stream`, not synchronized.  Errors: KKT_ESTATE (no refactor yet). */
kkt_status_t kkt_residual(kkt_handle_t h, const double *dev_b, const double *dev_x, double *dev_r,
                          void *stream);

/* Copy the current device factor values (last kkt_refactor) to HOST arrays in the layout
 * of kkt_get_factor_pattern; precision 0 = FP64 factors, 1 = FP32 factors widened to
 * float64.  Synchronizes `stream`. */
kkt_status_t kkt_get_factor_values(kkt_handle_t h, int32_t precision, double *lx, double *ux,
                                   void *stream);

/* Enable (1) or disable (0) per-launch timing with HIP events on the work stream; enabling
 * clears the totals.  Timing adds two event records per kernel launch. */
kkt_status_t kkt_set_profiling(kkt_handle_t h, int32_t on);

/* Time only the kernel classes whose bits are set in class_mask (bit c: class c of
 * kkt_kernel_class_t; 0 disables timing) and clear the totals.  Timing one class keeps the
 * event records, and their cost on the host and the stream, to that class's launches.
 * KKT_EINVAL for bits at or beyond KKT_K_CLASSES. */
kkt_status_t kkt_set_profiling_mask(kkt_handle_t h, uint32_t class_mask);

/* Totals since profiling was enabled: launches and device milliseconds per kernel class.
 * Synchronizes `stream` (the stream the work was issued on). */
kkt_status_t kkt_get_kernel_times(kkt_handle_t h, kkt_kernel_times_t *times, void *stream);

/* New unbound handle with a copy of src's options and analysis (no host re-analysis): for
 * several solvers of one pattern running at once (each needs its own workspace).  Errors:
 * KKT_ENOMEM. */
kkt_status_t kkt_clone(kkt_handle_t src, kkt_handle_t *out);

/* Free the handle and its host memory (the workspace stays owned by the caller). */
kkt_status_t kkt_release(kkt_handle_t h);

/* Message for the last failing call on h ("" if none; h may be NULL for kkt_analyze
 * failures, which keep a per-thread message). */
const char *kkt_last_error(kkt_handle_t h);

/* ------------------------------------------------------------------------------------------
 * Serving: KKT solves of several patterns arriving from concurrent optimizer instances.
 *
 * The server keeps one host analysis per registered pattern and a set of resident solver
 * *slots* (a cloned handle with its own workspace).  Slot workspaces are carved first-fit
 * from one caller-owned device pool, so admission is by HBM footprint: a request starts when
 * a free slot of its pattern exists or a new slot fits in the pool (idle slots of other
 * patterns are evicted, least recently used first, to make room); otherwise it waits while
 * later requests that fit go ahead.  `workers` host threads, each with its own HIP stream
 * (default priority), run admitted requests concurrently, so their kernels overlap on the
 * device; each request is one refactorization plus one FGMRES-IR solve, exactly as
 * kkt_refactor + kkt_solve on a handle of that pattern (the same kernels and schedules, hence
 * the same result bit for bit, alone or in a mix).
 * ---------------------------------------------------------------------------------------- */
typedef struct kkt_server_s *kkt_server_t;

typedef struct {
    double queued_ms;   /* submit -> start of service */
    double service_ms;  /* start of service -> solution ready (stream synchronized) */
    double latency_ms;  /* submit -> solution ready */
    int32_t slot;       /* slot that served the request */
    int32_t new_slot;   /* 1 if the slot was created (workspace carved and bound) for it */
} kkt_request_times_t;

/* Create a server on the current HIP device.  dev_pool: DEVICE memory of pool_bytes
 * (256-byte aligned, caller-owned, outlives the server).  workers >= 1.  Errors:
 * KKT_EINVAL, KKT_ENOMEM, KKT_EDEVICE. */
kkt_status_t kkt_server_create(void *dev_pool, size_t pool_bytes, int32_t workers, kkt_server_t *out);

/* Register a pattern: host analysis as kkt_analyze (HOST arrays, copied).  *pattern_id
 * receives its id (0, 1, ...).  Errors: those of kkt_analyze; KKT_ENOMEM when one slot of
 * this pattern cannot fit in the pool at all. */
kkt_status_t kkt_server_add_pattern(kkt_server_t srv, const kkt_opts_t *opts, int64_t n, const int64_t *rowptr,
                                    const int32_t *colidx, const double *values_first, int32_t *pattern_id);

/* Queue one solve of pattern_id: DEVICE arrays dev_values (nnz, CSR order of the pattern),
 * dev_b and dev_x (n float64), which must stay valid (and b, values unchanged) until the
 * request completes; tol <= 0 uses the pattern's delta_tol.  *ticket identifies it.
 * Never blocks.  Errors: KKT_EINVAL (unknown pattern, null pointers). */
kkt_status_t kkt_server_submit(kkt_server_t srv, int32_t pattern_id, const double *dev_values,
                               const double *dev_b, double *dev_x, double tol, int64_t *ticket);

/* Block until the request completes; fill *info and *times (either may be NULL) and forget
 * the ticket.  Returns the request's status (that of kkt_refactor / kkt_solve; KKT_ENOCONV
 * with x and info filled as for kkt_solve).  KKT_EINVAL for an unknown ticket. */
kkt_status_t kkt_server_wait(kkt_server_t srv, int64_t ticket, kkt_solve_info_t *info,
                             kkt_request_times_t *times);

/* Non-blocking: *done = 1 when the request has completed (then kkt_server_wait returns at
 * once), else 0.  KKT_EINVAL for an unknown ticket. */
kkt_status_t kkt_server_poll(kkt_server_t srv, int64_t ticket, int32_t *done);

/* Counters: requests completed, slots created, slots evicted, pool bytes in use. */
kkt_status_t kkt_server_stats(kkt_server_t srv, int64_t *completed, int64_t *slots_created,
                              int64_t *slots_evicted, int64_t *pool_in_use);

/* Batching: a worker that admits a request also admits up to max_batch - 1 (1..8, default 4)
 * queued requests of the same pattern that can get a slot, refactors them in one launch
 * (kkt_refactor_batch, or kkt_refactor_batch_graph when use_graphs = 1, the default) and then
 * solves them one after another on its stream.  A slot whose solve re-pivoted is retired, so
 * that every request is served on its pattern's own analysis.  Errors: KKT_EINVAL. */
kkt_status_t kkt_server_configure(kkt_server_t srv, int32_t max_batch, int32_t use_graphs);

/* Batches of more than one request, the requests they held, and batch refactorizations
 * launched through a graph (any batch size). */
kkt_status_t kkt_server_batch_stats(kkt_server_t srv, int64_t *batches, int64_t *batched_requests,
                                    int64_t *graph_launches);

/* Finish every queued request, stop the workers, release all slots and patterns. */
kkt_status_t kkt_server_destroy(kkt_server_t srv);

/* ------------------------------------------------------------------------------------------
 * HyKKT (Section 5, eq. (kktlineargamma)): for KKT systems [[H + D, J^T], [J, 0]] with a zero
 * (2,2) block (eq. (kktlinear)).  Adding gamma J^T times the second block row to the first
 * leaves the solution unchanged and gives H_gamma = H + D + gamma J^T J, symmetric positive
 * definite; the multipliers solve S dl = J H_gamma^-1 (r_x + gamma J^T r_l) - r_l with the SPD
 * Schur complement S = J H_gamma^-1 J^T by conjugate gradients (S applied as products, never
 * formed), then dx = H_gamma^-1 (r_x + gamma J^T r_l - J^T dl).  The pattern of H_gamma and the
 * map from K's values to its entries are built once (a sparse product with a fixed pattern);
 * H_gamma is refactored per system with the analysis of the first (diagonal pivots: Cholesky
 * up to the diagonal scaling) and applied with the staged triangular solves.
 * ---------------------------------------------------------------------------------------- */
typedef struct kkt_hykkt_s *kkt_hykkt_t;

typedef struct {
    double gamma;        /* > 0: this gamma; 0 (default): gamma_scale * max_i (H + D)_ii /
                            max_i (J^T J)_ii of the first system, kept for the sequence */
    double gamma_scale;  /* 1e4 (the paper asks for a gamma "large enough"; CG on S converges in
                            a few tens of iterations once gamma J^T J dominates H + D) */
    double cg_tol;       /* stop when ||r_k||_2 <= cg_tol ||r_0||_2 (1e-12) */
    int32_t cg_max_iter; /* iteration cap (1000); reaching it gives KKT_ENOCONV */
    int32_t reserved;
    kkt_opts_t lu;       /* options of the H_gamma factorization (ordering, tile budget, ...) */
} kkt_hykkt_opts_t;

typedef struct {
    int32_t converged;      /* 1 if the CG met cg_tol */
    int32_t cg_iterations;
    double gamma;
    double cg_rel_resid;    /* ||r_k|| / ||r_0|| of the CG on S */
    double nrbe;            /* eq. (nbre) of x = [dx; dl] for the original K */
    double rel_resid;       /* ||b - K x||_2 / ||b||_2 */
    double true_resid;      /* ||b - K x||_2 */
    double knorm_inf;       /* ||K||_inf */
} kkt_hykkt_info_t;

/* Fill *opts with the defaults above (lu: kkt_opts_default). */
void kkt_hykkt_opts_default(kkt_hykkt_opts_t *opts);

/* Analyse a KKT pattern with n_primal primal rows (rows and columns 0..n_primal-1 hold H + D,
 * the rest the constraints) and the values of the first system: J, J^T and the H_gamma pattern,
 * gamma, and the factorization analysis of H_gamma (kkt_analyze).  HOST arrays in the CSR
 * conventions above.  Errors: KKT_EINVAL (bad CSR, 1 <= n_primal < n violated, non-finite
 * value, a nonzero in the (2,2) block, J zero), KKT_ESINGULAR (from the H_gamma analysis),
 * KKT_ENOMEM. */
kkt_status_t kkt_hykkt_analyze(const kkt_hykkt_opts_t *opts, int64_t n, int64_t n_primal, const int64_t *rowptr,
                               const int32_t *colidx, const double *values_first, kkt_hykkt_t *out);

/* Device bytes for kkt_hykkt_bind_workspace (HyKKT arrays plus the H_gamma factorization's
 * workspace). */
kkt_status_t kkt_hykkt_workspace_size(kkt_hykkt_t h, size_t *bytes);

/* Bind caller-owned device memory (>= kkt_hykkt_workspace_size bytes, 256-byte aligned) and
 * upload the structure (synchronous on return). */
kkt_status_t kkt_hykkt_bind_workspace(kkt_hykkt_t h, void *dev_ptr, size_t bytes, void *stream);

/* New values (DEVICE, nnz float64 in the pattern's CSR order): H_gamma's entries formed on the
 * device, then its refactorization.  Enqueued on `stream`.  Errors: KKT_ESTATE (no workspace),
 * those of kkt_refactor. */
kkt_status_t kkt_hykkt_refactor(kkt_hykkt_t h, const double *dev_values, void *stream);

/* x = K^-1 b by HyKKT for the last refactored K.  DEVICE arrays of n float64 (distinct).
 * Synchronizes `stream` once per 8 CG iterations and before returning; *info (may be NULL) is
 * filled.  Errors: KKT_ESTATE (no refactorization), KKT_EINVAL (non-finite K), KKT_ENOCONV (the
 * CG reached cg_max_iter; x holds the solution recovered from the last iterate). */
kkt_status_t kkt_hykkt_solve(kkt_hykkt_t h, const double *dev_b, double *dev_x, kkt_hykkt_info_t *info,
                             void *stream);

/* H_gamma's pattern (HOST rp: n_primal+1, ci: nnz_hgamma), gamma, and (vals != NULL) its current
 * values after kkt_hykkt_refactor (HOST, synchronizes `stream`). */
kkt_status_t kkt_hykkt_get_hgamma(kkt_hykkt_t h, int64_t *rp, int32_t *ci, double *vals, double *gamma,
                                  void *stream);

/* Entries of H_gamma and products in its entries' sums (sizes of the map). */
kkt_status_t kkt_hykkt_sizes(kkt_hykkt_t h, int64_t *nnz_hgamma, int64_t *pairs);

/* The handle of the H_gamma factorization (owned by h: do not release; its getters give the
 * permutations, factor pattern and values). */
kkt_status_t kkt_hykkt_factor_handle(kkt_hykkt_t h, kkt_handle_t *lu);

/* Message for the last failing call on h (h may be NULL for kkt_hykkt_analyze failures). */
const char *kkt_hykkt_last_error(kkt_hykkt_t h);

/* Free the handle, its H_gamma factorization handle and host memory. */
kkt_status_t kkt_hykkt_release(kkt_hykkt_t h);

#ifdef __cplusplus
}
#endif

#endif /* KKT_H */
