/*
 * hodlr.h -- C ABI of the MI355X HODLRdD library.
 *
 * HODLRdD (Khan, Kandappan, Ambikasaran, arXiv 2209.05819) approximates the
 * N x N kernel matrix K(i,j) = F(x_i, x_j) of N points in d dimensions: the
 * blocks of far-field and vertex-sharing hyper-cube pairs on every level of a
 * 2^d tree are compressed with ACA, and the remaining adjacent leaf pairs are
 * evaluated densely.  This library builds that representation on one AMD
 * Instinct MI355X (gfx950) and applies it to vectors.
 *
 * Conventions for every entry point:
 *   - Only plain C types cross this boundary.  Every call returns a
 *     hodlr_status; none aborts.  On failure hodlr_last_error() returns a
 *     message for the calling thread.
 *   - "Tree order" is the order of the points sorted by (Morton key of their
 *     finest-level cell, original index); "user order" is the caller's order.
 *   - Box indices of a level are positions in that level's list of non-empty
 *     boxes, which is sorted by Morton key.
 *   - Streams are hipStream_t values passed as void*; NULL is the null stream.
 */
#ifndef HODLR_H
#define HODLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hodlr_handle_s* hodlr_t;

typedef enum {
    HODLR_OK = 0,
    HODLR_EINVAL = 1,       /* bad argument (size, tolerance, pointer, level) */
    HODLR_ENOMEM = 2,       /* device allocation failed or exceeded mem_budget_bytes */
    HODLR_EDEVICE = 3,      /* a HIP call failed */
    HODLR_EDUPLICATE = 4,   /* two distinct points coincide under a singular kernel */
    HODLR_ENONFINITE = 5,   /* NaN or Inf in the points, or in a solve's F, guess or residual */
    HODLR_EUNSUPPORTED = 6  /* valid request this library does not handle */
} hodlr_status;

/* Kernel functions of the paper's sec. 3 list (F1 1/r, F2 log r, F5 r,
 * F6 sin r, F7 1/sqrt(1+r), F8 exp(-r)), the 4D Laplace kernel 1/r^2 of
 * sec. 6.2 and the Gaussian of sec. 6.3.  r = |x_i - x_j|_2 (natural log). */
typedef enum {
    HODLR_K_LOG = 0,         /* log r           */
    HODLR_K_INV_R = 1,       /* 1 / r           */
    HODLR_K_INV_R2 = 2,      /* 1 / r^2         */
    HODLR_K_GAUSS = 3,       /* exp(-r^2 / h^2) */
    HODLR_K_EXP = 4,         /* exp(-r / h)     */
    HODLR_K_R = 5,           /* r               */
    HODLR_K_SIN = 6,         /* sin r           */
    HODLR_K_INV_SQRT1P = 7   /* 1 / sqrt(1 + r) */
} hodlr_kernel_kind;

/* K(i,j) = scale * f(r) for i != j and K(i,i) = diag, decided by the
 * points' global indices (sec. 6.1 sets the diagonal of log r to 0). */
typedef struct {
    int kind;       /* hodlr_kernel_kind */
    double h;       /* length scale of GAUSS and EXP (> 0) */
    double scale;
    double diag;
} hodlr_kernel;

typedef enum { HODLR_FP64 = 0, HODLR_FP32 = 1, HODLR_BF16 = 2 } hodlr_prec;

typedef struct {
    /* depth rule (sec. 5.2 / Alg. "HODLRdD Initialization"):
     * 0 = smallest level whose fullest box holds <= leaf_size points;
     * 1 = smallest kappa with leaf_size * 2^(d kappa) >= N;
     * 2 = adaptive 2^d tree (the option sec. 5.2 names beside the balanced
     *     tree): depth as rule 0, but a box is subdivided only while it holds
     *     more than leaf_size points.  Leaves then lie on several levels; the
     *     lists take only boxes whose parent was subdivided (active boxes),
     *     and a pair that is not admissible with a leaf on either side is a
     *     dense near-field pair of its level (hodlr_export_near_level). */
    int level_rule;
    /* computational hyper-cube: [domain_lo, domain_lo + domain_side]^d when
     * has_domain != 0 (points outside -> HODLR_EINVAL), else the bounding cube */
    int has_domain;
    double domain_lo[8];
    double domain_side;
    /* hodlr_prec of the stored U/V factors: FP64, FP32 or BF16 (rounded to
     * nearest even; BF16 factors are applied in FP32 arithmetic, on matrix
     * cores when nrhs > 1) */
    int storage;
    /* 1: store one factor pair per unordered block pair {A,B} and apply
     * K(B,A) = K(A,B)^T (the kernel is symmetric and both index sets are the
     * same point set); 0: store a pair for every ordered block (A,B) */
    int symmetric;
    int max_rank;         /* cap on every ACA rank; 0 = min(|I|,|J|) */
    int skip_aca;         /* 1: tree and lists only; factors come from hodlr_import_factors */
    size_t mem_budget_bytes;  /* cap on device memory held by the handle; 0 = none */
    /* admissibility (sec. 5): adjacent boxes sharing a hyper-surface of
     * dimension <= adm_dim are compressed, far ones always; -1 = far field
     * only (strong admissibility of H-matrices), 0 = HODLRdD (vertex sharing,
     * the default), d-1 = every pair (weak admissibility of HODLR) */
    int adm_dim;
    /* 1: store each block in the skeleton form of eqs. keq1/keq2 (the ACA
     * pivots sigma, tau and the LU of K(sigma, tau): r^2 elements instead of
     * r (|I| + |J|)) and evaluate K(I, tau) and K(sigma, J) inside every
     * product.  FP64 storage and FP64 arithmetic only: the pivots on the
     * diagonal of L span the tolerance's range, so the solves cancel unless
     * K(sigma, J) x is accurate to about tol.  One right-hand side per pass;
     * only the ranks can be exported, nothing imported; a block rank above
     * 1024 fails the build with EUNSUPPORTED.  0: store U and V (default). */
    int skeleton;
} hodlr_opts;

/* Defaults: level_rule 1, bounding cube, FP64 storage, symmetric 1,
 * max_rank 0, skip_aca 0, no budget, adm_dim 0, skeleton 0. */
void hodlr_default_opts(hodlr_opts* opts);

/* Build the HODLRdD representation (Alg. "HODLRdD Initialization"): the
 * hyper-cube and 2^d tree (sec. 5.2), the interaction lists of every level
 * and the near lists of the leaves (sec. 5.3, table of notations and the
 * HODLRdD admissibility definition), and the ACA factors of every admissible
 * block (eq. keq1) to relative tolerance tol.
 *   points    host or device pointer (the copy infers which), N x d
 *             row-major FP64, user order; copied before the call returns.
 *   N >= 1, 1 <= d <= 8, leaf_size >= 1, 0 <= tol < 1, -1 <= opts->adm_dim <= d-1.
 *   kernel    host pointer; h > 0 for GAUSS and EXP.
 *   opts      host pointer or NULL for the defaults.
 *   stream    work is queued on it; the call returns after the build finished.
 *   out       receives the handle (unchanged on failure).
 * Errors: EINVAL, ENONFINITE, EDUPLICATE (coincident distinct points under
 * LOG, INV_R or INV_R2), ENOMEM, EDEVICE. */
hodlr_status hodlr_build(const double* points, int64_t N, int d, const hodlr_kernel* kernel,
                         int leaf_size, double tol, const hodlr_opts* opts, void* stream,
                         hodlr_t* out);

/* Y = K~ X (Alg. "HODLRdD matrix-vector Product"): the low-rank blocks of
 * every level plus the near field of the leaves, evaluated on the fly.
 *   X, Y     device pointers, N x nrhs column-major in user order with
 *            leading dimensions ldx, ldy >= N; element type x_prec
 *            (FP64 or FP32) for both.  Y must not overlap X.
 *   compute_prec  FP64: FP64 arithmetic throughout; FP32: FP32 near field
 *            and FP32 accumulation (factors are read in their storage type).
 *            BF16 storage requires FP32; with nrhs > 1 the blocks of at most
 *            512 rows and columns are applied on BF16 matrix cores (x and the
 *            projections V x rounded to BF16, FP32 accumulation), 16 or 32
 *            right-hand sides per pass.
 *   Asynchronous on stream.  The near field runs on a second stream owned by
 *   the handle (default priority), beside the low-rank stages: it starts
 *   after the work queued on `stream` before the call, and `stream` waits
 *   for it before the final stage.  Owns a workspace inside the handle, so
 *   calls on one handle must not overlap in time (serialize them on one
 *   stream).
 * Errors: EINVAL (nrhs < 1, ld < N, bad prec, BF16 storage with FP64
 * compute, skeleton form with FP32 compute, factors missing), EDEVICE. */
hodlr_status hodlr_matvec(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec,
                          void* Y, int64_t ldy, int compute_prec, void* stream);

/* hodlr_matvec that also records caller-created hipEvent_t (passed as
 * void*) on the stream, for timing.  nevents == 5: before the product and
 * after each of its four stages (permutation into tree order; projections
 * and one-pass applications of the stored blocks; expansions of the blocks
 * split over several workgroups; gather of the contributions and the
 * near-field sums plus permutation back; the near field itself runs on the
 * handle's second stream beside the second and third stages, and with BF16
 * matrix cores beside both passes, joined before the permutation back).
 * Stage times are those of the caller's stream.  nevents == 11: the
 * same five, then events[5 + c] recorded after the launch of block-size
 * class c = 0..5 inside the second stage (classes of hodlr_info
 * class_blocks).  Same results and errors as hodlr_matvec (EINVAL if events
 * is NULL or nevents is neither 5 nor 11). */
hodlr_status hodlr_matvec_events(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec,
                                 void* Y, int64_t ldy, int compute_prec, void* stream,
                                 void* const* events, int nevents);

/* Reserves the product's device workspace for nrhs columns in compute_prec
 * (the largest request so far is kept).  hodlr_matvec reserves on demand;
 * reserving first makes a later hodlr_matvec / hodlr_matvec_events with at
 * most nrhs columns free of allocations, host synchronisation and memsets:
 * only kernel launches and events on the caller's stream and on the
 * handle's second stream (created here, forked from and joined back into the
 * caller's stream within each call), so the call can be captured into a HIP
 * graph and replayed (inputs and outputs at the captured addresses).  A call under stream capture that would have to grow
 * the workspace returns HODLR_EINVAL instead.  EINVAL for a null handle,
 * nrhs < 1 or a bad precision. */
hodlr_status hodlr_reserve_workspace(hodlr_t h, int nrhs, int compute_prec);

/* Route of hodlr_matvec for this handle (Alg. "HODLRdD matrix-vector
 * Product" either way): 1 = one persistent launch that walks every stage
 * (permutation, the blocks of every level, the near field, the sums of the
 * segmented blocks, the gather) as an ordered queue of work; 0 = one launch
 * per stage and block size class, the near field on a second stream; 2 = the
 * same launches all on the caller's stream (no fork and join: fewer
 * operations for a launch-bound product); -1 (default, not chosen) = route
 * 0.  The
 * persistent route applies to FP64 factors in FP64 arithmetic and FP32
 * factors in FP32 arithmetic (not BF16, not the skeleton form); other
 * products take the per-class route whatever is set.  EINVAL for a null
 * handle or another route. */
hodlr_status hodlr_set_route(hodlr_t h, int route);

/* What hodlr_autotune measured and chose. */
typedef struct {
    int route;              /* product route kept: 0 per-class launches, 1 persistent, 2 per-class on one stream */
    int class_choice[8];    /* tile shape kept per single-RHS block class (index below) */
    double class_ms[8];     /* that shape's time per launch of the class, ms */
    double class_route_ms;  /* product time on the per-class route, ms */
    double persistent_ms;   /* product time on the persistent route, ms (0: not applicable) */
    int seg_side;           /* persistent route: widest block one workgroup streams alone */
    double one_stream_ms;   /* product time on route 2 (per-class, one stream), ms */
} hodlr_tuning;

/* Autotuner of this handle's product (Alg. "HODLRdD matrix-vector Product"
 * as the handle applies it), for nrhs columns of X in x_prec and
 * compute_prec arithmetic: for nrhs = 1, every candidate tile shape
 * <W waves per block, CH rows per lane, KB terms per batch> of the
 * block-size classes 2..5 is timed alone on the handle's own blocks and the
 * fastest is kept (class 2, blocks up to 64: <1,1,8> <1,1,4> <1,1,16>;
 * class 3, up to 128: <1,2,4> <1,2,8> <2,1,8>; class 4, up to 1024:
 * <4,4,K> <4,4,2K> <8,2,K>; class 5, up to 4608: <8,9,K'> <8,9,2K'>, with
 * K = 2 and K' = 1 in FP64 arithmetic, 4 and 2 in FP32); then the product
 * is timed on the per-class route (near field on a second stream, or all
 * on the caller's stream) and on the persistent route (there with the
 * class-4 blocks wider than 1024, 512 or 256 rows segmented over many
 * workgroups, the fastest of the three kept) and the fastest route is kept
 * (hodlr_set_route).  Every time is the least of three timings of five
 * back-to-back calls.  Allocates scratch X and Y, reserves
 * the workspace, synchronises stream; out (host) receives the times.
 * Errors: those of hodlr_matvec. */
hodlr_status hodlr_autotune(hodlr_t h, int nrhs, int x_prec, int compute_prec,
                            hodlr_tuning* out, void* stream);

/* Products of several handles (different point sets, sizes, dimensions and
 * kernels) in one persistent launch: Y[t] = K~_t X[t] for t < nslots, each
 * N_t x nrhs[t] column-major in its own user order, device pointers.  The
 * handles must all store FP64 or all store FP32 factors (the arithmetic
 * follows the storage) and appear once each; x_prec is that of every X and
 * Y.  Each handle's workspace grows as hodlr_matvec's would; the call
 * returns after the launch finished.  Calls must not overlap other calls on
 * the same handles.  On this GPU the launch is slower than the handles'
 * own per-class launches (it saves host launches, not device time).
 * Errors: EINVAL (arguments, mixed or BF16 storage, the skeleton form, a
 * repeated handle, factors missing), EUNSUPPORTED (a handle with more than
 * 1632 columns: the launch holds at most 1024 stages, five per eight
 * columns), ENOMEM, EDEVICE. */
hodlr_status hodlr_matvec_batch(int nslots, const hodlr_t* hs, const void* const* X,
                                const int64_t* ldx, const int* nrhs, int x_prec, void* const* Y,
                                const int64_t* ldy, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of hodlr_matvec with the same arguments and result, whose
 * workspace is the library's static device scratch array of
 * HODLR_NOALLOC_SCRATCH_BYTES (one per GPU, held until the process ends)
 * and whose near field runs on `stream` itself (no second stream).  The call
 * allocates nothing and creates nothing; the handle must belong to the
 * current device.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams, other threads, other handles) race and
 * must be ordered by the caller.  Errors: those of hodlr_matvec, and EINVAL
 * when the product's workspace (which grows with N, the number of stored
 * blocks and nrhs) exceeds the scratch array. */
#define HODLR_NOALLOC_SCRATCH_BYTES (64u << 20)
hodlr_status hodlr_matvec_noalloc(hodlr_t h, const void* X, int64_t ldx, int nrhs, int x_prec,
                                  void* Y, int64_t ldy, int compute_prec, void* stream);

/* Largest byte offset the matrix-core product (BF16 factors, several
 * right-hand sides; the blocks of Alg. "HODLRdD matrix-vector Product")
 * forms within one factor of rank `rank` and length `len` or within the x
 * rows it reads.  Those offsets address buffer resources of a 2^31-byte
 * range, and a build whose BF16 factors exceed it fails with
 * HODLR_EUNSUPPORTED; this call exposes the same check.  Host computation
 * only (no device needed).  Returns OK and *extent, EUNSUPPORTED (with
 * *extent set) when *extent >= 2^31, EINVAL for negative sizes, nrhs
 * outside 1..32 or a null extent. */
hodlr_status hodlr_mfma_extent(int64_t rank, int64_t len, int nrhs, int64_t* extent);

/* Options of hodlr_solve. */
typedef struct {
    double tol;           /* outer stop: max over columns of |F - A U| / |F| (FP64 operator) */
    double inner_tol;     /* inner GMRES stop: residual estimate <= inner_tol |r| */
    int restart;          /* Krylov dimension of one inner cycle, 1..512 */
    int max_outer;        /* refinement steps, >= 0 */
    int lo_compute;       /* hodlr_prec of the inner products' arithmetic (FP32 forced for BF16) */
    int use_initial_guess;/* 1: start from U; 0: from zero */
} hodlr_solve_opts;

typedef struct {
    int outer_iters;      /* refinement steps taken */
    int inner_iters;      /* Arnoldi steps taken in total (one product with lo each) */
    int converged;        /* 1 if the outer tolerance was met */
    double rel_residual;  /* final max over columns of |F - A U| / |F| */
    double history[64];   /* the same before each of the first 64 refinement steps */
} hodlr_solve_info;

/* Defaults: tol 1e-10, inner_tol 1e-4, restart 50, max_outer 30,
 * lo_compute FP32, use_initial_guess 0. */
void hodlr_default_solve_opts(hodlr_solve_opts* opts);

/* Solve (alpha I + beta K~) U = F (the paper's GMRES use of the product,
 * sec. 6.2) by iterative refinement: residuals r = F - A U with the FP64
 * representation `hi`, corrections from one restarted GMRES cycle on `lo`
 * (a lower-precision representation of the same points, e.g. BF16 or FP32
 * factors; lo == hi gives plain restarted GMRES).  Krylov basis,
 * orthogonalisation (classical Gram-Schmidt applied twice) and norms in FP64.
 *   hi, lo   handles built on the same points and kernel; hi holds FP64 or FP32
 *            factors and is applied in FP64 arithmetic.
 *   F, U     device pointers, N x nrhs column-major FP64 in user order,
 *            leading dimensions ldf, ldu >= N; U receives the solution.
 *            U is read only when opts->use_initial_guess is 1 (any
 *            contents otherwise).
 *   opts     host pointer or NULL for the defaults; info host pointer (may be NULL).
 *   Allocates a workspace of about (restart + 4) N nrhs doubles for the
 *   call; synchronous on stream.  Calls must not overlap other calls on hi or lo.
 * Errors: EINVAL (arguments, mismatched handles, hi with BF16 factors, factors
 * missing), ENONFINITE (NaN or Inf in F, in the initial guess, or in a
 * residual), ENOMEM, EDEVICE.  Not converging is not an error: check
 * info->converged.  A column of F that is zero is measured by its absolute
 * residual. */
hodlr_status hodlr_solve(hodlr_t hi, hodlr_t lo, double alpha, double beta, const double* F,
                         int64_t ldf, int nrhs, double* U, int64_t ldu,
                         const hodlr_solve_opts* opts, hodlr_solve_info* info, void* stream);

/* ---- Serving: resident point sets, continuous batching of requests ---- */

typedef struct hodlr_server_s* hodlr_server_t;

typedef struct {
    size_t mem_budget_bytes;  /* device memory for resident sets, batch buffers and
                               * running solves; 0 = 90% of the free memory at creation */
    int max_concurrent;       /* stream slots: launches in flight at once, 1..64 */
    int max_batch_cols;       /* columns of one batched product = largest nrhs, 1..1024 */
    int64_t max_points;       /* largest set (sizes the batch buffers), >= 1 */
    /* 1: queued products of several sets with FP64 or FP32 factors (not the
     * skeleton form) share one persistent launch (hodlr_matvec_batch); 0, the
     * default: one launch per set (on this GPU the per-class route of each
     * set is faster than the persistent launch, so the shared launch saves
     * host launches but not GPU time) */
    int multiset;
} hodlr_server_opts;

typedef enum { HODLR_REQ_MATVEC = 0, HODLR_REQ_SOLVE = 1 } hodlr_request_kind;

typedef struct {
    int kind;                 /* hodlr_request_kind */
    int set;                  /* from hodlr_server_add_set */
    int nrhs;                 /* 1 .. max_batch_cols */
    const double* X;          /* device, N x nrhs column-major (ld N), FP64, user order */
    double* Y;                /* device, same shape: the product, or the solution */
    double alpha, beta;       /* solve: (alpha I + beta K~) Y = X */
    double tol;               /* solve: relative residual to reach */
    void* stream;             /* hipStream_t on which X was produced (NULL: the null
                               * stream): the request reads X only after the work
                               * queued there before hodlr_server_submit */
} hodlr_request;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t launches;          /* products and solves started */
    int64_t batched_requests;  /* products that shared a launch with others */
    int64_t multiset_launches; /* launches that applied the products of several sets */
    int64_t max_concurrent;    /* most launches in flight at once */
    size_t used_bytes, budget_bytes;
    int sets;
} hodlr_server_stats;

/* Defaults: budget 0 (90% of free), 8 slots, 64 columns, 2^18 points. */
void hodlr_server_default_opts(hodlr_server_opts* opts);

/* Start a server (one scheduler thread, max_concurrent HIP streams of default
 * priority, batch buffers of 2 max_points max_batch_cols doubles per slot).
 * Errors: EINVAL, ENOMEM, EDEVICE. */
hodlr_status hodlr_server_create(const hodlr_server_opts* opts, hodlr_server_t* out);

/* Build and keep resident the representation of a point set (arguments as
 * hodlr_build, points on the host; opts->mem_budget_bytes is replaced by the
 * server's remaining room).  Blocks until built.  *set_id receives its index.
 * Errors: those of hodlr_build; ENOMEM when it does not fit the budget. */
hodlr_status hodlr_server_add_set(hodlr_server_t srv, const double* points, int64_t N, int d,
                                  const hodlr_kernel* kernel, int leaf_size, double tol,
                                  const hodlr_opts* opts, int* set_id);

/* Queue a request; returns at once with its id.  The scheduler starts it when
 * its set is idle, a slot is free and its workspace fits the budget; queued
 * products of one set are applied together as one product of their columns,
 * and, with the server option multiset, queued products of other idle sets
 * with the same factor precision (FP64 or FP32) join the same launch: one
 * persistent launch applies up to 16 sets (as far as the slot's buffer of
 * max_points x max_batch_cols doubles holds their columns).
 * Solves run GMRES with iterative refinement on the set itself (FP64
 * residuals; inner GMRES(30) in FP32 arithmetic, to tol).  X and Y must stay
 * valid until the request completes.  Ordering: an event is recorded on
 * req->stream at submission and the request's stream slot waits on it
 * before reading X, so X may still be in production there; Y is complete
 * when hodlr_server_wait or a successful hodlr_server_poll returns.
 * Errors: EINVAL (unknown set, nrhs out of range, solve on BF16 factors, set
 * larger than max_points), EDEVICE (the event could not be recorded). */
hodlr_status hodlr_server_submit(hodlr_server_t srv, const hodlr_request* req, int64_t* id);

/* Block until request id completes; returns its status (a solve that misses
 * its tolerance: EUNSUPPORTED) and its time in the queue and running, in
 * microseconds (either pointer may be NULL).  A completed request is
 * reported once; its id is then unknown (EINVAL). */
hodlr_status hodlr_server_wait(hodlr_server_t srv, int64_t id, double* queue_us, double* run_us);

/* Non-blocking hodlr_server_wait: *done = 0 while the request is queued or
 * running (status OK, nothing else written). */
hodlr_status hodlr_server_poll(hodlr_server_t srv, int64_t id, int* done, double* queue_us,
                               double* run_us);

hodlr_status hodlr_server_get_stats(hodlr_server_t srv, hodlr_server_stats* stats);

/* Finish every queued request, stop the scheduler, free the sets. */
void hodlr_server_destroy(hodlr_server_t srv);

typedef struct {
    int64_t N;
    int d;
    int kappa;            /* depth of the tree (leaves are level kappa) */
    int lmax;             /* finest representable level of the Morton keys */
    int symmetric;
    int storage;
    double domain_lo[8];
    double domain_side;
    int64_t nboxes[32];       /* non-empty boxes per level 0..kappa */
    int64_t il_entries[32];   /* interaction-list entries per level */
    int64_t stored_blocks[32];/* factor pairs held per level */
    int32_t rank_min[32], rank_max[32];
    double rank_mean[32];     /* over stored blocks */
    int64_t factor_elems[32]; /* stored factor elements: sum of r(|I|+|J|) (r^2 in the skeleton form) */
    /* blocks applied by one workgroup, by size class (0, 1: at most 8 / 16
     * rows, columns and terms; 2..5: |A|, |B| up to 64, 128, 1024, 4608),
     * their factor elements sum r(|I|+|J|) and vector elements 2(|I|+|J|) */
    int64_t class_blocks[8];
    int64_t class_factor_elems[8];
    int64_t class_vector_elems[8];
    int64_t split_blocks;         /* larger blocks, split over workgroups */
    int64_t split_factor_elems;
    int64_t near_entries;     /* near-list entries at the leaves */
    int64_t near_pairs;       /* point pairs of the near field */
    size_t device_bytes;      /* device memory held by the handle */
    double build_ms[4];       /* tree, lists, ACA, packing */
    /* BF16 storage, several right-hand sides (matrix cores, two passes):
     * projection jobs by workgroup width W = 1, 2, 4, 8 waves (a job
     * projects one side of a stored block over a panel of at most 64 W
     * columns), the factor elements and the x elements per right-hand side
     * they read; the factor elements the expansion pass reads (every
     * interaction-list entry's factor with |I| rows); projection elements per
     * right-hand side */
    int64_t mfma_proj_jobs[4];
    int64_t mfma_proj_factor_elems[4];
    int64_t mfma_proj_vector_elems[4];
    int64_t mfma_expand_factor_elems;
    int64_t mfma_proj_elems;
} hodlr_info;

hodlr_status hodlr_get_info(hodlr_t h, hodlr_info* info);

/* Tree export (host pointers): perm[N] maps tree position -> user index,
 * keys[N] the sorted Morton keys.  Either may be NULL. */
hodlr_status hodlr_export_tree(hodlr_t h, int64_t* perm, uint64_t* keys);

/* Boxes of level l (0..kappa), host pointers: start[nb+1] offsets into tree
 * order, key[nb] level keys, coord[nb*d] integer box coordinates.  Any may be NULL. */
hodlr_status hodlr_export_boxes(hodlr_t h, int level, int64_t* start, uint64_t* key,
                                int32_t* coord);

/* Interaction list of level l (1..kappa) in CSR form over the level's boxes,
 * columns ascending: ptr[nb+1], col[nnz].  *nnz receives the entry count;
 * ptr/col may be NULL to query it. */
hodlr_status hodlr_export_il(hodlr_t h, int level, int64_t* nnz, int64_t* ptr, int32_t* col);

/* Near list of the leaves ({A} and boxes sharing a hyper-surface of
 * dimension 1..d-1 with A), same CSR convention: the dense pairs of level
 * kappa (every dense pair of a uniform tree). */
hodlr_status hodlr_export_near(hodlr_t h, int64_t* nnz, int64_t* ptr, int32_t* col);

/* Dense near-field pairs of level l (0..kappa), same CSR convention over the
 * level's boxes: (A, B) both active, not admissible, and A or B a leaf.  In
 * a uniform tree only level kappa has any. */
hodlr_status hodlr_export_near_level(hodlr_t h, int level, int64_t* nnz, int64_t* ptr,
                                     int32_t* col);

/* Box flags of level l (0..kappa), host pointer flags[nb]: bit 0 active (the
 * box's parent was subdivided), bit 1 leaf. */
hodlr_status hodlr_export_box_flags(hodlr_t h, int level, uint8_t* flags);

/* Factors of level l in the interaction list's CSR order, for every entry
 * (A,B): U (|A| x r, column after column) and V (r x |B|, row after row),
 * concatenated; FP64 host pointers.  ranks[nnz] receives r per entry;
 * *u_elems / *v_elems receive the totals (U, V may be NULL to query).
 * In symmetric mode the entry (B,A) is exported as the transpose of the
 * stored pair of (A,B). */
hodlr_status hodlr_export_factors(hodlr_t h, int level, int32_t* ranks, int64_t* u_elems,
                                  int64_t* v_elems, double* U, double* V);

/* Install factors of level l from host memory in the layout of
 * hodlr_export_factors (replacing any present).  In symmetric mode only the
 * entries (A,B) with A < B are read; the others are ignored.  Meant for
 * testing the apply with externally computed factors. */
hodlr_status hodlr_import_factors(hodlr_t h, int level, const int32_t* ranks, const double* U,
                                  const double* V);

void hodlr_destroy(hodlr_t h);

/* Message of the calling thread's last failure ("" if none). */
const char* hodlr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
