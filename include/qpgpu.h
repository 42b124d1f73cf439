/*
 * qpgpu.h -- C ABI of the MI355X (gfx950) interior point search-direction library.
 *
 * The library solves the convex QP of Section 3.1, eq. (qp), of Liu,
 * Fredriksson and Markidis, "A GPU-Accelerated Interior Point Method for
 * Radiation Therapy Optimization":
 *
 *     min  1/2 x^T H x + p^T x
 *     s.t. lo_A <= A x <= hi_A,   lo_x <= x <= hi_x,
 *
 * with the variable bounds kept apart from the rows of A (Section 4, the text
 * before eq. (2x2_reduced)) and the Hessian in the matrix-free form of
 * eq. (bfgs_hessian), H = H_0 + U diag(w) U^T, where here
 * H_0 = gamma*I + J^T diag(W) J for a sparse dose-influence matrix J.
 *
 * Every search direction is the solution of the condensed Newton system
 * (H + A^T Sigma_A A + Sigma_x) dx = r (the Schur complement of the doubly
 * augmented system eq. (2x2_augmented)), computed by Jacobi-preconditioned
 * conjugate gradients (Section 4.1) on the GPU; the rest of Algorithm 1
 * (direction recovery, step lengths, updates, residuals, the barrier rule)
 * also runs on the GPU.
 *
 * Conventions shared by every entry point:
 *  - All array arguments are HOST pointers unless the name says otherwise;
 *    the library copies inputs to device memory it owns and copies outputs
 *    back into caller buffers of the stated length.  The caller keeps
 *    ownership of every buffer it passes and may free it on return.
 *  - Sparse matrices are 0-based CSR with strictly increasing column indices
 *    in each row; nnz must be below 2^31.
 *  - Infinite bounds (+-INFINITY) mark an absent side.
 *  - Errors are returned as qp_status codes; no C++ exception crosses the
 *    ABI.  Inputs are validated before any GPU call: on QP_ERR_INVALID no
 *    device work was done and outputs are untouched.  qp_last_error() gives a
 *    message for the most recent failure.
 *  - One handle is used by one host thread at a time.  Distinct handles may
 *    run concurrently on distinct streams.
 */
#ifndef QPGPU_H
#define QPGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qp_handle qp_handle;

typedef enum {
    QP_OK = 0,
    QP_ERR_INVALID = 1,        /* bad argument; nothing was done */
    QP_ERR_NOMEM = 2,          /* device or host allocation failed */
    QP_ERR_DEVICE = 3,         /* a HIP call failed (no GPU, launch error, ...) */
    QP_ERR_NOT_CONVERGED = 4,  /* iteration limit reached; best iterate returned */
    QP_ERR_NUMERIC = 5         /* PCG breakdown (p^T K p <= 0 or non-finite) */
} qp_status;

/* Storage of the J values inside the PCG operator (Section 4.1 keeps FP64).
 * FP32/BF16 keep a rounded copy (round to nearest even) with FP32
 * accumulation; residuals, PCG scalars and dot products stay FP64, and the
 * direction is refined against the FP64 operator: each low-precision PCG
 * solve stops at refine_tol times its own right-hand side, and refinement
 * passes (at most refine_steps) go on until the FP64 residual is below
 * pcg_tol times the original right-hand side.  When it is still above after
 * refine_steps passes (the rounded operator too far from K for refinement to
 * converge, e.g. J without full column rank and a small gamma), the direction
 * is solved again by FP64 PCG.  refine_steps = 0: the low-precision solve to
 * pcg_tol is the direction, unrefined. */
typedef enum { QP_FP64 = 0, QP_FP32 = 1, QP_BF16 = 2 } qp_precision;

typedef struct {
    int32_t rows, cols;
    int64_t nnz;
    const int64_t* row_ptr;   /* rows+1 entries, row_ptr[0] = 0, nondecreasing */
    const int32_t* col_idx;   /* nnz entries, sorted strictly increasing per row */
    const double*  val;       /* nnz entries, finite */
} qp_csr;

/* H = gamma*I + J^T diag(W) J + U diag(w) U^T (eq. (bfgs_hessian)); the J part
 * is passed to qp_create separately. */
typedef struct {
    double gamma;             /* >= 0 */
    const double* p;          /* n: linear term of eq. (qp) */
    int32_t k;                /* columns of U; 0 = no low-rank term */
    const double* U;          /* n*k, column-major (U[j + n*c]); may be NULL when k = 0 */
    const double* w;          /* k, >= 0 */
} qp_hessian;

typedef struct {
    const double* lo;         /* may be NULL: all -INFINITY */
    const double* hi;         /* may be NULL: all +INFINITY */
} qp_range;

typedef struct {
    int32_t precision;        /* qp_precision, default QP_FP64 */
    int32_t refine_steps;     /* at most this many FP64 refinement passes per low-precision direction,
                                 default 6 (they stop once the FP64 residual meets pcg_tol) */
    double  pcg_tol;          /* stop at ||r||_2 <= pcg_tol*||rhs||_2, default 1e-8 */
    int32_t pcg_max_iter;     /* per PCG solve, default 20000 */
    double  mu0;              /* <= 0: average complementarity of the start point (default) */
    double  mu_tol;           /* barrier rule exit, default 1e-10 (objective scaled, see below) */
    double  tau;              /* fraction to the boundary, default 0.995 */
    int32_t max_ipm_iter;     /* default 200 */
    int32_t step_mode;        /* 0: separate primal/dual steps (Algorithm 1), 1: equal */
    int32_t scale_objective;  /* 1 (default): divide H, p by max(1, ||H x0 + p||_inf) */
    int32_t schedule;         /* CSR SpMV schedule (results are the same bits for every one):
                                 0: autotuned; 4..64: lanes per row; 1: the J pass over
                                 nonzero-balanced blocks of rows, default lane counts elsewhere */
    int32_t timing;           /* 1: time the J and J^T SpMV launches with HIP events */
    int32_t log_level;        /* 0: quiet; 1: one line per IPM iteration on stderr */
    int32_t precond;          /* 0: Jacobi, diag(K) (Section 4.1.2); 1 (default): Jacobi on the H
                                 part, diag(H + Sigma_x), with the constraint block A^T Sigma_A A
                                 applied exactly (Woodbury identity) for the rows with
                                 Sigma_i sum_j A_ij^2 / D_j >= 1 through the dense inverse of their
                                 Schur complement, the other rows folded into the diagonal;
                                 falls back to 0 when m = 0 or m > 8192.  A solve with it that
                                 reaches its attempt cap (the larger of 2000 and 4 times the
                                 longest converged constraint-block solve of the call so far) or
                                 breaks down (r^T z <= 0: late in
                                 the IPM the block's rounding can cost it definiteness) is
                                 repeated with the block's Sigma capped so that no diagonal entry
                                 of its Schur complement exceeds 1 + 1e4, and a solve that stalls
                                 with that too, with 0; qp_solve keeps the tier reached for the
                                 rest of the QP */
    int32_t spmv_format;      /* 0 (default): line format for J when its rows come in lines of 64
                                 that share most of their columns (the 64-voxel bands): each line
                                 stores the union of its rows' column lists, zeros where a row
                                 lacks one, taken when that stores at most 2 nnz(J) values; else
                                 CSR.  1: CSR */
    double  refine_tol;       /* relative residual target of each low-precision PCG solve when
                                 refine_steps > 0, in [pcg_tol, 1); default 1e-3 */
    int32_t graphs;           /* 1 (default): PCG iterations are launched as HIP graphs of four
                                 iterations, captured once per operator and replayed; 0: one launch
                                 per kernel.  Results are identical.  timing = 1 launches directly. */
    int32_t kkt_system;       /* linear system PCG runs on.  0 (default): the condensed system
                                 (H + Sigma_x + A^T Sigma_A A) dx = r, the Schur complement of
                                 eq. (2x2_augmented).  1: the doubly augmented system of
                                 eq. (2x2_augmented) itself (Section 4), of size n + |L_A| + |U_A|,
                                 with the Jacobi preconditioner of Section 4.1.2 (precond is then
                                 ignored); dx is its x part.  qp_operator_apply always applies the
                                 condensed operator. */
    int32_t batch_mode;       /* how qp_solve_batch runs a batch of handles that all set it:
                                 0 (default): each QP's own solve, several in flight on their
                                 own streams (host workers); 1: the persistent batched path where
                                 it applies (see qp_solve_batch).  Results are identical. */
} qp_settings;

typedef struct {
    int32_t status;           /* qp_status of the call */
    int32_t ipm_iters;
    int64_t pcg_iters;        /* all PCG iterations of the call, refinement solves included */
    int32_t pcg_solves;
    int32_t pcg_capped;       /* PCG solves that stopped at pcg_max_iter */
    double  mu;               /* final barrier parameter (scaled units) */
    double  rnorm;            /* final ||r|| of the barrier rule */
    double  zeta;             /* objective scale used */
    double  objective;        /* 1/2 x^T H x + p^T x at the returned x */
    double  pcg_relres;       /* last PCG solve: ||r||_2 / ||rhs||_2 */
    double  t_solve_ms;       /* wall time of the call on the device stream */
    double  t_pcg_ms;         /* part of it inside PCG loops */
    double  t_spmv_fwd_ms;    /* summed J (and A) SpMV launch time, when timing = 1 */
    double  t_spmv_bwd_ms;    /* summed J^T (and A^T) SpMV launch time, when timing = 1 */
    int64_t n_spmv_fwd, n_spmv_bwd;
    int32_t spmv_format;      /* format the PCG operator used: 0 CSR, 1 line format */
    int32_t prec_fallbacks;   /* PCG solves repeated with the next preconditioner tier (capped block,
                                 then the Jacobi diagonal) */
    /* KKT certificate of the returned (x, lam_x, lam_A) in the original units
     * (qp_solve / qp_solve_from only, 0 elsewhere), with y_x = lam_x, y_A = lam_A
     * and lambda_l = max(-y, 0), lambda_u = max(y, 0) per side:
     *   eps_d = ||H x + p + y_x + A^T y_A||_inf / (1 + max(||H x||, ||p||, ||y_x||, ||A^T y_A||))
     *   eps_p = largest bound or row violation / (1 + largest finite |bound|)
     *   eps_c = largest lambda * slack / (1 + |x^T H x|/2 + |p^T x|)
     *   gap   = |f - (-x^T H x/2 + sum lambda_l lo - sum lambda_u hi)| / (1 + |x^T H x|/2 + |p^T x|)
     * (the optimality conditions of eq. (qp) with mu = 0 in eq. (perturbed_KKT)). */
    double  eps_d, eps_p, eps_c, gap;
    int32_t prec_tier;        /* preconditioner tier the call ended on: 0 constraint block, 1 capped
                                 block, 2 Jacobi diagonal (see precond) */
    int32_t spmv_schedule;    /* CSR format: the J pass's schedule (1: nonzero-balanced row
                                 blocks, else lanes per row; see settings.schedule); 0: line format */
} qp_info;

/* Defaults listed above. */
void qp_default_settings(qp_settings* s);

/* qp_create: validate, copy to the device, build the stored transposes J^T
 * and A^T (Section 4.1: transposes are precomputed so every SpMV is
 * transpose-free), the low-precision J copies, diag(H) (cached once, Section
 * 4.1.2) and the SpMV row schedule.
 *   H      : gamma, p (n), optional U (n x k), w (k); n = J->cols.
 *   J      : nJ x n dose matrix; W: nJ weights >= 0.
 *   A      : m x n constraint matrix or NULL (m = 0); b: its row bounds (m).
 *   bounds : variable bounds (n); NULL = free variables.
 *   s      : NULL = defaults.  hip_stream: hipStream_t to enqueue on, NULL =
 *            a stream the handle creates and owns.
 * Errors: QP_ERR_INVALID (shapes, unsorted or out-of-range indices, non-finite
 * values, lo > hi, W < 0, gamma < 0, w < 0), QP_ERR_NOMEM, QP_ERR_DEVICE. */
qp_status qp_create(qp_handle** out, const qp_hessian* H, const qp_csr* J, const double* W,
                    const qp_csr* A, const qp_range* b, const qp_range* bounds,
                    const qp_settings* s, void* hip_stream);

/* qp_create_device: qp_create with every array in device memory of the
 * current HIP device (the structs themselves on the host): H->p, H->U, H->w,
 * J's and A's row_ptr/col_idx/val, W, b->lo/hi and bounds->lo/hi are device
 * pointers, for callers whose data already sit in GPU memory (e.g. tensors
 * allocated by a framework through the same HIP runtime).  The arrays are
 * read on hip_stream (NULL: the null stream) and copied to host memory for
 * the one-time preparation of qp_create (transposes, line format, value
 * copies), which then runs unchanged; the caller keeps ownership and may free
 * the arrays on return.  Validation runs on those host copies, before any
 * device allocation.  Errors: as qp_create; QP_ERR_DEVICE when a pointer is
 * not readable device memory. */
qp_status qp_create_device(qp_handle** out, const qp_hessian* H, const qp_csr* J, const double* W,
                           const qp_csr* A, const qp_range* b, const qp_range* bounds,
                           const qp_settings* s, void* hip_stream);

/* qp_solve: run Algorithm 1 from the default start point.
 *   x     (n) : minimiser.
 *   lam_A (m) : lambda_uA - lambda_lA per row of A (> 0 where the upper side
 *               binds); may be NULL.
 *   lam_x (n) : lambda_ux - lambda_lx per variable; may be NULL.
 *   info      : may be NULL.
 * Returns QP_OK, QP_ERR_NOT_CONVERGED (best iterate in the outputs),
 * QP_ERR_NUMERIC or QP_ERR_DEVICE. */
qp_status qp_solve(qp_handle* h, double* x, double* lam_A, double* lam_x, qp_info* info);

/* qp_solve_from: qp_solve started at the caller's primal point x0 (n finite
 * doubles, host memory; NULL = the default start).  Meant for a sequence of
 * related QPs (SQP sub-problems, Section 3.2), x0 being the previous QP's
 * minimiser.  The paper gives no warm-start rule: x0 replaces the default x
 * of the start point and the slacks (max(x0 - lo, 1), max(hi - x0, 1) and
 * the same for A x0), multipliers (1) and mu0 follow the default rule, so x0
 * need not be feasible.  Outputs and errors as qp_solve; QP_ERR_INVALID for
 * a non-finite x0 (no device work). */
qp_status qp_solve_from(qp_handle* h, const double* x0, double* x, double* lam_A, double* lam_x,
                        qp_info* info);

/* qp_update_hessian: replace the objective of a handle (gamma, p, U, w, k;
 * see qp_hessian) and keep J, W, A and the bounds resident.  In SQP
 * (Section 3.2) the quasi-Newton term U w U^T of eq. (bfgs_hessian) gains
 * two columns from one QP sub-problem to the next (Section 5.2); the J and A
 * preparation of qp_create is not repeated.  Recomputes the cached diag(H) and drops the
 * handle's captured PCG graphs.  k may grow or shrink (storage grows to
 * max(k, 2 * capacity) when k exceeds it).  Waits for the handle's queued
 * work first; H's arrays are copied before return.  Errors: QP_ERR_INVALID
 * (as qp_create's checks of H: gamma < 0, w < 0, non-finite entries, NULL
 * arrays; the handle is unchanged), QP_ERR_NOMEM (a larger U did not fit),
 * QP_ERR_DEVICE; after these two the handle's objective is unspecified until
 * a later call succeeds. */
qp_status qp_update_hessian(qp_handle* h, const qp_hessian* H);

/* qp_newton_step: one PCG solve of (H + diag(sigma_x) + A^T diag(sigma_A) A) dx = rhs
 * (the Newton system of Algorithm 1 in condensed form) with the
 * handle's precision and refinement settings and no objective scaling.
 *   sigma_x (n) >= 0, sigma_A (m) >= 0 (may be NULL when m = 0), rhs (n),
 *   dx (n) output.  Returns QP_OK, QP_ERR_NOT_CONVERGED (pcg_max_iter hit;
 *   dx holds the last iterate), QP_ERR_NUMERIC, QP_ERR_INVALID. */
qp_status qp_newton_step(qp_handle* h, const double* sigma_x, const double* sigma_A,
                         const double* rhs, double* dx, qp_info* info);

/* qp_operator_apply: y = (H + diag(sigma_x) + A^T diag(sigma_A) A) v, the
 * matrix-free product of Section 4.1.1 in condensed form, with the J values
 * stored in `precision` (FP64 accumulation for QP_FP64, FP32 otherwise).
 * reps > 1 repeats the product (for timing); the result is the same. */
qp_status qp_operator_apply(qp_handle* h, const double* sigma_x, const double* sigma_A,
                            const double* v, double* y, int32_t precision, int32_t reps,
                            qp_info* info);

/* qp_operator_apply_noalloc: the product of qp_operator_apply,
 *   y = (H + diag(sigma_x) + A^T diag(sigma_A) A) v,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree, copy or synchronisation, only enqueues the product's
 * kernels on hip_stream (NULL: the handle's stream) and returns; y is ready
 * when the stream reaches that point.
 *   sigma_x (n), sigma_A (m; may be NULL when m = 0), v (n), y (n): DEVICE
 *   pointers of the handle's device, caller-owned; sigma entries must be
 *   finite and >= 0 (not checked: the arrays are in device memory).
 *   precision: as qp_operator_apply; the J copy of that precision must
 *   already be resident (a handle created with it, or one earlier
 *   qp_operator_apply call with it), else QP_ERR_INVALID.
 * The intermediates (per-slot or per-row products of J, the rows of A, the
 * low-rank partials) go to one static 32 MiB device array of the library per
 * GPU, held until the process ends: problems needing more (line slots or J
 * rows, plus m, plus 256*k + k doubles, each part rounded up to 32, above
 * 4,194,304) get QP_ERR_INVALID.  Every call on one GPU uses that same array:
 * calls whose products overlap in time on one GPU (different streams, or
 * several host threads) race; calls on one stream are ordered.
 * Errors: QP_ERR_INVALID (NULL argument, precision, size, copy not resident;
 * nothing enqueued), QP_ERR_DEVICE (launch failure). */
qp_status qp_operator_apply_noalloc(qp_handle* h, const double* sigma_x, const double* sigma_A,
                                    const double* v, double* y, int32_t precision, void* hip_stream);

/* qp_solve_batch: solve `count` independent QPs (each a handle from
 * qp_create) together; xs[i] (n_i doubles) receives QP i's minimiser and
 * infos[i] (may be NULL) its info, each bitwise what qp_solve of that handle
 * returns.  Many QPs of uneven size are the intended use.  Two ways to run
 * them (settings.batch_mode):
 *   0: handles run concurrently, each its own qp_solve on its own stream
 *      (create them with hip_stream = NULL for a stream per handle), by up to
 *      6 host workers (environment QPGPU_BATCH_WORKERS), largest nnz first;
 *   1: when every handle sets it and uses the line format, the condensed
 *      system, no low-rank term and the same precision, refine_steps and
 *      graphs (and timing = 0), 2 to 256 handles on one device: the IPM
 *      iterations of all QPs advance together; each kind of PCG work of
 *      all QPs is ONE launch over a device-built work list of every QP's
 *      blocks (QPs whose solve stopped drop out), the iterations replayed
 *      as a captured HIP graph; each QP's other IPM steps on its own
 *      stream.  Other batches run as with 0.
 * Returns QP_OK when every QP returned QP_OK, else the first failing status
 * (QP_ERR_DEVICE preferred); QP_ERR_INVALID for NULL or repeated handles,
 * or two handles on one stream (text in qp_last_error(NULL)). */
qp_status qp_solve_batch(qp_handle* const* hs, int32_t count, double* const* xs, qp_info* infos);

/* Text of the last error on this handle; h == NULL gives the calling
 * thread's last qp_create error.  Valid until the next call on h. */
const char* qp_last_error(const qp_handle* h);

/* Free all device memory of h (NULL is a no-op). */
void qp_destroy(qp_handle* h);

/* Problem sizes of a handle (any pointer may be NULL). */
void qp_sizes(const qp_handle* h, int32_t* n, int32_t* m, int32_t* nJ, int64_t* nnzJ,
              int64_t* nnzA);

#ifdef __cplusplus
}
#endif

#endif /* QPGPU_H */
