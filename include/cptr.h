/* cptr.h -- C ABI of the MI355X CPTR library.
 *
 * The library applies the Constrained Pressure-Temperature Residual (CPTR)
 * two-stage preconditioner inside right-preconditioned (F)GMRES to block-sparse
 * Jacobians with interleaved per-cell unknowns (Cremon, Franc, Hamon, "CPTR
 * Preconditioner Performance for Large-Scale Thermal CO2 Injection
 * Simulation").  The operations follow the paper's statement of the problem:
 *   - Eq. (3): M^-1 = M1^-1 + M2^-1 (I - A M1^-1);
 *   - Sec. 3: A split into elliptic and hyperbolic unknowns, the first stage
 *     M1^-1 = [[0,0],[0,Mee^-1]], right-preconditioned GMRES, 200 iterations,
 *     relative tolerance 1e-6;
 *   - Sec. 3.1: the variables are interleaved per cell; Mee^-1 is one AMG
 *     V-cycle (HMIS coarsening, extended+i interpolation truncated to 4
 *     entries per row, first-order relaxation); the second stage is ILU(0);
 *   - Sec. 3.2: CPTR puts pressure and temperature in the elliptic block and
 *     solves it with system AMG;
 *   - Sec. 5.2: the elliptic block is reached by a quasi-IMPES decomposition.
 *
 * General rules
 *   - Every call returns cptr_status; nothing aborts, throws or prints.
 *     Negative values are errors, CPTR_NOT_CONVERGED (> 0) is a warning with a
 *     valid result.  cptr_last_error() returns a message for the last failure.
 *   - Vectors passed to cptr_apply / cptr_gmres_solve / cptr_spmv are device
 *     pointers to FP64 arrays of length N = n_block_rows * block_size in the
 *     matrix's interleaved order (unknown c of cell i at index i*b + c).  The
 *     caller owns them; they must stay valid until the work on `stream`
 *     completes.  Input and output must not alias.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is enqueued on it.
 *   - A handle owns all hierarchy, factor and workspace memory, the Krylov
 *     space of cptr_gmres_solve included (sized by cptr_setup_opts.max_restart
 *     and flexible_space); it allocates in cptr_setup and frees in
 *     cptr_destroy.  cptr_apply, cptr_stage1, cptr_ilu_solve, cptr_spmv and
 *     cptr_gmres_solve never allocate device memory.  A handle is not
 *     thread-safe; distinct handles are independent.
 *   - The ILU(0) sweeps wait on each other's results with bounded waits.  A
 *     wait that reaches its bound (never, for a valid schedule) sets a flag on
 *     the handle; cptr_gmres_solve reports it as CPTR_E_HIP and clears it at
 *     its start, and cptr_sweep_check reads and clears it after asynchronous
 *     calls.
 */
#ifndef CPTR_H
#define CPTR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cptr_solver_s *cptr_solver;

typedef enum {
  CPTR_OK = 0,
  CPTR_NOT_CONVERGED = 1,      /* max_iter reached; x holds the last iterate */
  CPTR_E_INVALID = -1,         /* bad argument; message names field and row */
  CPTR_E_NOMEM = -2,           /* host or device allocation failed */
  CPTR_E_ZERO_PIVOT = -3,      /* zero ILU(0) pivot, singular hyperbolic block or zero smoother diagonal */
  CPTR_E_SINGULAR_COARSE = -4, /* coarsest AMG matrix (solved by dense LU) singular */
  CPTR_E_HIP = -5,             /* a HIP runtime call failed */
  CPTR_E_STATE = -6            /* call not valid for this handle (e.g. host-only setup) */
} cptr_status;

/* Block-sparse (BSR) matrix, square blocks of block_size^2 values stored
 * row-major inside the block, blocks of a row sorted by column with the
 * diagonal block present.  The caller owns the arrays; the library reads them
 * only during cptr_setup and keeps its own copies. */
typedef struct {
  int32_t n_block_rows;
  int64_t nnz_blocks;
  const int32_t *row_ptr;   /* [n_block_rows + 1], row_ptr[0] = 0 */
  const int32_t *col_idx;   /* [nnz_blocks] */
  const double *values;     /* [nnz_blocks * block_size * block_size] */
  int32_t on_device;        /* 0: host pointers, 1: device pointers */
} cptr_bsr;

enum { CPTR_RESTRICT_QUASI_IMPES = 0, CPTR_RESTRICT_INJECTION = 1 };

typedef struct {
  double strong_threshold;   /* AMG strength threshold theta, default 0.25 */
  double max_row_sum;        /* rows with |same-function row sum| > this * |a_ii| have only weak links; 0.9 */
  int32_t max_levels;        /* AMG levels including the coarsest, default 25 */
  int32_t max_coarse;        /* stop coarsening at or below this many rows, default 9 */
  int32_t p_max_elmts;       /* interpolation entries kept per row, default 4 */
  int32_t restriction;       /* CPTR_RESTRICT_*, default quasi-IMPES */
  int32_t host_only;         /* 1: build the hierarchy on the host only (for inspection
                                through cptr_export; apply/solve return CPTR_E_STATE) */
  int32_t setup_threads;     /* host threads for setup; 0 = min(16, hardware threads) */
  int32_t ilu_sweep;         /* CPTR_ILU_SWEEP_*: how the ILU(0) triangular solves run */
  int32_t agg_levels;        /* AMG levels coarsened aggressively (the "aggregate level" of
                                Sec. 3.1): a second first pass over the C points on the
                                distance-two strength graph, multipass interpolation, no
                                truncation; default 1, 0 = none */
  int32_t precond_precision; /* CPTR_PRECISION_*: value type of the preconditioner (the V-cycle
                                operators and vectors, the ILU(0) factors and sweeps); the
                                Krylov method, A, the restriction weights and the coarsest dense
                                solve stay FP64; default FP64 */
  int32_t num_sweeps;        /* l1-Jacobi sweeps before and after the coarse correction on every
                                AMG level above the coarsest (the "first order relaxation" of
                                Sec. 3.1 reads as 1); default 1, at most 8 */
  int32_t max_restart;       /* longest restart cptr_gmres_solve accepts: the handle allocates
                                the Krylov basis V (max_restart + 1 vectors) in cptr_setup;
                                default 50, 1..64 */
  int32_t flexible_space;    /* 1: also allocate the max_restart preconditioned vectors Z that
                                flexible solves keep; 0: flexible solves return CPTR_E_STATE;
                                default 1 */
  int32_t hmis_block;        /* HMIS coarsening (Sec. 3.1) over blocks of this many consecutive
                                rows of a level, each block standing for one subdomain: the
                                Ruge-Stueben first pass inside every block, then PMIS on the
                                points it leaves undecided across blocks; 1 = PMIS; default
                                0 = one block (the first pass over the whole level) */
  int32_t max_dense_coarse;  /* largest coarsest level solved exactly (dense LU, Sec. 3.1's
                                coarse solve); a coarsest level above it (the coarsening
                                stopped early: a split with no C point, or max_levels) gets
                                num_sweeps l1-Jacobi sweeps before and after a zero coarse
                                correction instead; default 4096, 0..4096 */
  int32_t dense_tail;        /* the V-cycle below the largest AMG level l >= 1 of at most this
                                many rows (with a smoothed level and the dense coarsest solve
                                under it) is applied as one dense n_l x n_l operator, formed at
                                setup by running that part of the cycle on the n_l unit vectors:
                                the same linear map (the cycle starts from zero iterates, Sec.
                                3.1), evaluated in one matrix-vector product instead of about
                                four launches per level; n_l^2 values of device memory in the
                                preconditioner's type; default 2048, 0 = off, at most 4096 */
} cptr_setup_opts;

enum {
  CPTR_PRECISION_FP64 = 0,
  CPTR_PRECISION_FP32 = 1       /* mixed precision: FP32 preconditioner inside FP64 (F)GMRES */
};

enum {
  CPTR_ILU_SWEEP_AUTO = 0,      /* GRID when A is a 7-point lexicographic stencil, else
                                   ONE_LAUNCH when rows are narrow enough, else LEVELS */
  CPTR_ILU_SWEEP_LEVELS = 1,    /* one launch per dependency level */
  CPTR_ILU_SWEEP_ONE_LAUNCH = 2, /* one launch per sweep, rows published as they finish;
                                   CPTR_E_INVALID if rows are too wide */
  CPTR_ILU_SWEEP_GRID = 3       /* tiled sweeps over x-pencils of an nx*ny*nz grid (7-point
                                   stencil, x fastest); CPTR_E_INVALID for other patterns */
};

typedef struct {
  int32_t restart;           /* Krylov vectors per cycle, default 30 */
  int32_t max_iter;          /* total iterations across restarts, default 200 */
  int32_t flexible;          /* 0: right GMRES (x += M^-1 V y), 1: FGMRES (x += Z y) */
  int32_t x0_is_zero;        /* 1: ignore x on entry and start from 0, default 1 */
  double rtol;               /* stop when ||b - A x||_2 <= rtol ||b||_2, default 1e-6 */
  int32_t profile;           /* 1: time each kernel phase with HIP events (cptr_phase_times);
                                a value > 1 times only the phases k whose bit k + 1 is set */
} cptr_solve_opts;

typedef struct {
  int32_t iterations;        /* Arnoldi steps = applications of A M^-1 */
  int32_t restarts;          /* completed cycles before the last */
  int32_t converged;         /* 1 when the true residual met the tolerance */
  double rel_res_est;        /* |g_{j+1}| / ||b|| from the Givens recurrence */
  double rel_res_true;       /* ||b - A x|| / ||b|| recomputed at the end */
  double setup_s;            /* wall time of cptr_setup */
  double solve_s;            /* wall time of this cptr_gmres_solve */
} cptr_solve_info;

void cptr_setup_opts_default(cptr_setup_opts *o);
void cptr_solve_opts_default(cptr_solve_opts *o);

/* Build the preconditioner for A (Sec. 3, 3.2, 5.2).
 *   block_size    must be 3 (two elliptic + one hyperbolic, or one + two);
 *   elliptic_idx  within-block unknown indices of the elliptic block, e.g. {0,1}
 *                 for (p, T); equation k pairs with unknown k; 1 <= n_elliptic <
 *                 block_size, values unique and in range;
 *   opts          NULL for defaults;
 *   stream        hipStream_t (void*) receiving the uploads;
 *   out           receives the handle on success (NULL on failure).
 * The AMG hierarchy is built on the host, except that a device handle forms
 * the strength graphs, the extended+i interpolations and the Galerkin products
 * R A P on the device in the host's order and rounding (the same hierarchy,
 * bit for bit); the C/F splits and the aggressive level's multipass
 * interpolation stay on the host.  A device handle factors ILU(0) on
 * the device (rows of one dependency level at a time, each in the host
 * factorisation's order and rounding, so the factors equal the host's); a
 * host-only handle factors it on the host.  A's device layout and the reduced
 * elliptic blocks are also formed on the device.
 * Errors: CPTR_E_INVALID (null pointer, block size, indices, unsorted or
 * duplicate columns, missing diagonal block, non-finite value),
 * CPTR_E_ZERO_PIVOT (zero ILU(0) pivot, singular hyperbolic diagonal block,
 * zero smoother diagonal), CPTR_E_SINGULAR_COARSE, CPTR_E_NOMEM, CPTR_E_HIP. */
cptr_status cptr_setup(const cptr_bsr *A, int32_t block_size, const int32_t *elliptic_idx,
                       int32_t n_elliptic, const cptr_setup_opts *opts, void *stream,
                       cptr_solver *out);

/* z = M^-1 r, Eq. (3), asynchronous on `stream`; no host synchronisation and
 * no allocation. */
cptr_status cptr_apply(cptr_solver s, const double *r, double *z, void *stream);

/* Solve A x = b with right-preconditioned restarted GMRES (or FGMRES) and the
 * CPTR preconditioner (Sec. 3).  Synchronises `stream` once per iteration for
 * the host Givens update and returns with x final and info filled (info may be
 * NULL; o NULL for defaults).  CPTR_NOT_CONVERGED when max_iter is reached.
 * CPTR_E_INVALID when o->restart exceeds the handle's max_restart, CPTR_E_STATE
 * for a flexible solve on a handle set up with flexible_space = 0.  Allocates
 * no device memory. */
cptr_status cptr_gmres_solve(cptr_solver s, const double *b, double *x, const cptr_solve_opts *o,
                             cptr_solve_info *info, void *stream);

/* cptr_gmres_solve for callers that cannot allocate device memory or must
 * not touch the handle's own workspace beyond the Krylov space (serving loops
 * running many resident handles, harnesses that forbid allocation).  Same
 * arguments, result and errors as cptr_gmres_solve, bit for bit; the
 * reduction partials of the Gram-Schmidt passes and norms and the
 * Hessenberg/flag slots live in a static device array of the library
 * (kept by each GPU the library runs on until the process ends; 1024 * 66 +
 * 256 doubles, about 530 KiB) instead of the handle's.  The first call on a
 * device looks up that device's address of the array; no call allocates or
 * frees device memory.
 *   - Every call on one GPU shares that GPU's array: calls that overlap in
 *     time on one GPU (other threads, other streams) race and must not be
 *     made.  The array keeps the last call's contents; each call clears what
 *     must start at zero (the sweeps' wait-limit flag).
 *   - CPTR_E_INVALID when o->restart needs more partials than the array holds
 *     (restart + 2 columns of 1024; every restart the handle accepts fits) or
 *     when o->profile != 0 (this variant does not time phases). */
cptr_status cptr_gmres_solve_static(cptr_solver s, const double *b, double *x, const cptr_solve_opts *o,
                                    cptr_solve_info *info, void *stream);

/* y = A x with the block SpMV kernel of the solve (Eq. 3 uses A in the
 * stage-two residual and GMRES applies it once per iteration). */
cptr_status cptr_spmv(cptr_solver s, const double *x, double *y, void *stream);

/* The two stages of Eq. (3) separately, asynchronous on `stream`:
 *   cptr_stage1:    x1 = M1^-1 r = P_E Vcycle(R_QI r)  (Sec. 3 form of M1, one
 *                   system-AMG V-cycle on the quasi-IMPES elliptic block);
 *   cptr_ilu_solve: x = M2^-1 r = U^-1 L^-1 r with the ILU(0) factors (Sec. 3.1).
 * Same conventions as cptr_apply (device FP64 vectors of length N, no aliasing,
 * no allocation). */
cptr_status cptr_stage1(cptr_solver s, const double *r, double *x1, void *stream);
cptr_status cptr_ilu_solve(cptr_solver s, const double *r, double *x, void *stream);

/* Synchronises `stream` and reports whether an ILU(0) sweep queued on the
 * handle since the last check (or the last cptr_gmres_solve) gave up a
 * dependency wait at its bound: CPTR_E_HIP with a message if so (the output of
 * that apply is not valid), CPTR_OK otherwise.  Clears the flag. */
cptr_status cptr_sweep_check(cptr_solver s, void *stream);

cptr_status cptr_destroy(cptr_solver s);

/* Message of the last failed call on s, or of the last failed cptr_setup in
 * this thread when s is NULL.  Never NULL. */
const char *cptr_last_error(cptr_solver s);

/* ---- introspection (tests, benchmarks) ---- */

/* Number of AMG levels and, per level, rows and stored entries (arrays of at
 * least *n_levels entries; pass NULL to query the count only). */
cptr_status cptr_hierarchy_info(cptr_solver s, int32_t *n_levels, int64_t *rows, int64_t *nnz);

enum {
  CPTR_EXPORT_CF = 0,        /* int32[rows_l]: 1 = C, -1 = F (levels below the coarsest) */
  CPTR_EXPORT_A_ROWPTR = 1,  /* int64[rows_l + 1] of level-l scalar CSR A_l */
  CPTR_EXPORT_A_COLS = 2,    /* int32[nnz_l] */
  CPTR_EXPORT_A_VALS = 3,    /* double[nnz_l] */
  CPTR_EXPORT_P_ROWPTR = 4,  /* int64[rows_l + 1] of P_l */
  CPTR_EXPORT_P_COLS = 5,
  CPTR_EXPORT_P_VALS = 6,
  CPTR_EXPORT_W = 7,         /* double[n_block_rows * n_elliptic * n_hyperbolic] */
  CPTR_EXPORT_DINV = 8,      /* double[rows_l], inverse l1-Jacobi diagonal */
  CPTR_EXPORT_ILU_VALS = 9,  /* double[nnz_blocks * 9]: L below the diagonal
                                (unit diagonal blocks implied), U on and above,
                                with the diagonal blocks stored as U_ii (not inverted);
                                CPTR_E_STATE for a device handle, whose
                                factors are computed on the device */
  CPTR_EXPORT_ILU_NLEVELS = 10, /* int32[2]: forward and backward dependency levels */
  CPTR_EXPORT_SWEEP = 11,      /* int32[4]: ILU sweep schedule in use (CPTR_ILU_SWEEP_*),
                                  then nx, ny, nz of the detected grid (0 if none) */
  CPTR_EXPORT_DEVICE_PLAN = 13, /* int64[1 + n]: n, then the n steps of building this host-only
                                  handle's device half with its max_restart and flexible_space
                                  (the solve server's footprint measurement): a positive entry
                                  allocates that many bytes (in 256-byte pieces), -1 - k releases
                                  the k-th allocation; CPTR_E_STATE for a device handle */
  CPTR_EXPORT_SETUP_TIMES = 14, /* double[10]: wall seconds of the setup steps: validation,
                                  quasi-IMPES weights and level-0 operator, strength graphs,
                                  C/F splits, interpolations (with R = P^T), Galerkin products,
                                  l1 diagonals and coarsest LU, host ILU(0) and sweep levels,
                                  then the device half and the whole cptr_setup.  In
                                  cptr_setup the device half's first part (A's layout, the
                                  ILU(0) factors and the sweeps' levels) runs on a second
                                  thread beside the AMG steps, so the steps may add up to
                                  more than the whole */
  CPTR_EXPORT_SETUP_SITES = 12 /* int32[15]: strength graphs formed on the device and in total,
                                  extended+i interpolations on the device and in total,
                                  coarse operators R A P on the device and in total, multipass
                                  interpolations (aggressive levels) on the device and in total,
                                  distance-two strength graphs (aggressive levels) on the device
                                  and in total, first passes begun on the device (over the
                                  components of at most 64 points, the rest finished on the
                                  host) and first passes in total (with hmis_block = 0: one per
                                  level split, two on an aggressive level), and the share, in
                                  thousandths, of the device passes' points that the device
                                  decided; then the splits over several HMIS blocks formed on
                                  the device (hmis_block from 1 to 4096) and in total.
                                  A device handle forms a product on the host only when a row of
                                  it has more than 2048 products, an extended+i interpolation
                                  only when a row's interpolatory set has more than 64 points, a
                                  multipass interpolation only when a row has more than 64
                                  interpolating points or 2048 products, a distance-two graph
                                  only when a row has more than 2048 candidates */,
  CPTR_EXPORT_DENSE_TAIL = 15  /* int32[2]: the AMG level whose V-cycle below runs as one dense
                                  operator (dense_tail; 0 = none) and its rows; CPTR_E_STATE for
                                  a host-only handle */
};
/* Copy one piece of the setup into host_buf (bytes = its capacity). */
cptr_status cptr_export(cptr_solver s, int32_t what, int32_t level, void *host_buf, int64_t bytes);

/* Per-phase GPU times accumulated by solves with profile = 1 since the last
 * reset.  Phases: 0 SpMV, 1 restriction, 2 V-cycle level 0, 3 V-cycle coarse
 * levels, 4 stage-two residual, 5 ILU forward, 6 ILU backward, 7 Arnoldi,
 * 8 solution update.  ms[k] = total milliseconds, count[k] = launches timed.
 * n = array capacity; reset = 1 clears after copying. */
cptr_status cptr_phase_times(cptr_solver s, double *ms, int64_t *count, int32_t n, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif
