/* cptr_oracle.h -- plain sequential FP64 reference of CPTR-preconditioned GMRES.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this code; only the tests, the package's smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no source with the GPU library.
 *
 * What it computes (paper: Cremon, Franc, Hamon, "Constrained
 * Pressure-Temperature Residual (CPTR) Preconditioner Performance for
 * Large-Scale Thermal CO2 Injection Simulation"):
 *   - the two-stage preconditioner M^-1 = M1^-1 + M2^-1 (I - A M1^-1), Eq. (3);
 *   - the first stage acting on the elliptic (p, T) block, Sec. 3 and 3.2,
 *     reached through a quasi-IMPES reduction (Sec. 5.2 names the
 *     decomposition) and approximated by one system-AMG V-cycle with the
 *     parameters listed in Sec. 3.1 (HMIS coarsening, extended+i
 *     interpolation truncated to 4 entries per row, first-order relaxation);
 *   - the second stage, ILU(0) on the whole system, Sec. 3.1;
 *   - right-preconditioned restarted GMRES (and its flexible variant),
 *     200 iterations at most, relative tolerance 1e-6 by default, Sec. 3.
 *
 * Conventions: all arrays are host memory owned by the caller unless a
 * function returns an object, which the caller releases with the matching
 * *_free call.  Scalar CSR rows have sorted column indices.  Every call that
 * can fail returns an OR_* status; or_last_error() holds the message.
 */
#ifndef CPTR_ORACLE_H
#define CPTR_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_E_INVALID = -1, OR_E_NOMEM = -2,
       OR_E_ZERO_PIVOT = -3, OR_E_SINGULAR_COARSE = -4 };

const char *or_last_error(void);

/* ---------- scalar CSR matrices produced by the oracle ---------- */
typedef struct or_mat or_mat;
void or_mat_info(const or_mat *m, int *nrows, int *ncols, long *nnz);
void or_mat_copy(const or_mat *m, long *rp, int *ci, double *v);
void or_mat_free(or_mat *m);

/* y = A x for a block-CSR matrix with nb block rows of size bs x bs. */
void or_bsr_spmv(int nb, int bs, const int *rp, const int *ci, const double *v,
                 const double *x, double *y);

/* ---------- AMG building blocks (exposed for pins) ---------- */
/* Strength matrix pattern (values are 1.0) of a scalar CSR matrix. */
or_mat *or_strength(int n, const long *rp, const int *ci, const double *v,
                    const int *func, double theta, double max_row_sum);
/* Ruge-Stueben first pass on a strength pattern: cf[i] = 1 (C) or -1 (F). */
void or_rs_first_pass(int n, const long *srp, const int *sci, int *cf);
/* Extended+i interpolation for a given C/F split; pmax <= 0: no truncation. */
or_mat *or_extpi(int n, const long *rp, const int *ci, const double *v,
                 const long *srp, const int *sci, const int *cf, const int *func,
                 int pmax);
/* distance-two strength among the C points of cf (rows = C points in order) */
or_mat *or_strength2(int n, const long *srp, const int *sci, const int *cf);
/* HMIS split over blocks of `block` consecutive points (<= 0: one block) */
void or_hmis_split(int n, const long *srp, const int *sci, int block, int *cf);
/* aggressive split: HMIS, then HMIS over the C points with or_strength2 */
void or_aggressive_hmis(int n, const long *srp, const int *sci, int block, int *cf);
/* the same with one block (first passes over the whole level) */
void or_aggressive_split(int n, const long *srp, const int *sci, int *cf);
/* multipass interpolation for a split (no truncation) */
or_mat *or_multipass(int n, const long *rp, const int *ci, const double *v,
                     const long *srp, const int *sci, const int *cf, const int *func);

typedef struct {
  double theta;        /* strength threshold, 0.25 */
  double max_row_sum;  /* 0.9 */
  int max_levels;      /* 25 */
  int max_coarse;      /* 9 */
  int pmax;            /* 4 */
  int agg_levels;      /* 1: levels coarsened aggressively (multipass interpolation) */
  int num_sweeps;      /* 1: l1-Jacobi sweeps before and after the coarse correction */
  int hmis_block;      /* 0: points per HMIS block (0: one block per level) */
  int max_dense;       /* 4096: largest coarsest level solved by dense LU; a larger
                          one (coarsening stopped early) is smoothed instead */
} or_amg_opts;
void or_amg_opts_default(or_amg_opts *o);

typedef struct or_amg or_amg;
int or_amg_setup(int n, const long *rp, const int *ci, const double *v,
                 const int *func, const or_amg_opts *o, or_amg **out);
int or_amg_nlevels(const or_amg *a);
/* what: 0 = A_l, 1 = P_l (levels 0..L-2), 2 = R_l = P_l^T.  Returns a copy. */
or_mat *or_amg_get(const or_amg *a, int level, int what);
void or_amg_get_cf(const or_amg *a, int level, int *cf);
void or_amg_get_func(const or_amg *a, int level, int *func);
void or_amg_get_dinv(const or_amg *a, int level, double *dinv);
void or_amg_vcycle(const or_amg *a, const double *b, double *x);
void or_amg_free(or_amg *a);

/* ---------- CPTR ---------- */
typedef struct or_cptr or_cptr;
/* qi = 1: quasi-IMPES restriction; qi = 0: plain injection (W = 0). */
int or_cptr_setup(int nb, int bs, const int *rp, const int *ci, const double *v,
                  const int *eidx, int ne, int qi, const or_amg_opts *o,
                  or_cptr **out);
const or_amg *or_cptr_amg(const or_cptr *h);
or_mat *or_cptr_get_ahat(const or_cptr *h);
void or_cptr_get_w(const or_cptr *h, double *w);        /* [nb][ne][nh] */
or_mat *or_cptr_get_ilu(const or_cptr *h);              /* L\U in one CSR */
void or_cptr_restrict(const or_cptr *h, const double *r, double *rhat);
void or_cptr_prolong(const or_cptr *h, const double *e, double *x);
void or_cptr_ilu_solve(const or_cptr *h, const double *r, double *x);
void or_cptr_stage1(const or_cptr *h, const double *r, double *x1);
void or_cptr_apply(const or_cptr *h, const double *r, double *z);
void or_cptr_free(or_cptr *h);

/* ---------- GMRES ---------- */
enum { OR_PC_NONE = 0, OR_PC_ILU = 1, OR_PC_STAGE1 = 2, OR_PC_CPTR = 3 };
typedef struct {
  int restart;   /* 30 */
  int max_iter;  /* 200 */
  int flexible;  /* 0: right GMRES, 1: FGMRES */
  int precond;   /* OR_PC_* */
  double rtol;   /* 1e-6 */
} or_gmres_opts;
void or_gmres_opts_default(or_gmres_opts *o);
/* hist (may be NULL) receives max_iter+1 residual estimates |g_{j+1}|/|b|
 * (hist[0] = |r0|/|b|); hist_n receives how many were written. */
int or_gmres(int nb, int bs, const int *rp, const int *ci, const double *v,
             const or_cptr *pc, const double *b, double *x,
             const or_gmres_opts *o, int *iters, double *rel_est,
             double *rel_true, double *hist, int *hist_n);

#ifdef __cplusplus
}
#endif
#endif
