// kernels.hpp -- device data layouts and launchers of the CPTR hot path (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cptr {

constexpr int kLanes = 64;      // rows per SELL slice = one wavefront
constexpr int kBlock = 256;     // threads per workgroup for streaming kernels
constexpr int kRedBlocks = 1024;  // workgroups of the deterministic reductions

// Sliced-ELL layout with one 64-row slice per wavefront.  Slice s owns the
// k-columns [sptr[s], sptr[s+1]); k-column k holds, for each of the 64 lanes,
// one block: col[k*64 + lane] and the block's `nv` values stored as planes
// val[(k*nv + e)*64 + lane], so lane-consecutive loads of one entry are
// contiguous.  Padding slots repeat a valid column with zero values.  Values
// are FP64, or FP32 for the preconditioner's operators in mixed precision.
template <class T>
struct SellT {
  int32_t nrows = 0;      // block rows (or positions) covered
  int32_t nslices = 0;
  int32_t nv = 0;         // values per block (9 for 3x3, 4 for 2x2)
  int32_t* sptr = nullptr;
  int32_t* col = nullptr;
  T* val = nullptr;
  int64_t nslots = 0;     // total k-columns
};
using Sell = SellT<double>;

// Scalar CSR on the device.
template <class T>
struct DCsrT {
  int32_t n = 0, m = 0;
  int64_t nnz = 0;
  int32_t* rp = nullptr;
  int32_t* ci = nullptr;
  T* v = nullptr;
  int group = 1;          // lanes cooperating on one row
};
using DCsr = DCsrT<double>;

// ---- launchers (all asynchronous on `st`) ----
void launch_bsr3_spmv(const Sell& A, const double* x, const double* b, double* y, bool resid,
                      hipStream_t st);
// The preconditioner's launchers take its value type T: double, or float in
// the mixed-precision mode (A, the restriction weights and the coarsest LU stay
// FP64 in both).
// Level 0 of the V-cycle on Ahat:
//   restrict: b0 = quasi-IMPES restriction of r, and with dinv also the
//             pre-smoothed iterate x0 = D^-1 b0 (dinv null: b0 only)
//   resid:    r0 = b0 - Ahat x0
//   post:     e0 = x0 + D^-1 (b0 - Ahat x0)
template <class T>
void launch_l0_restrict(int32_t nc, int ne, const double* r, const double* W, const int32_t* eidx,
                        const int32_t* hidx, T* b0, const T* dinv, T* x0, hipStream_t st);
template <class T>
void launch_l0_resid(const SellT<T>& Ah, int ne, const T* x0, const T* b0, T* r0, hipStream_t st);
template <class T>
void launch_l0_post(const SellT<T>& Ah, int ne, const T* x0, const T* b0, const T* dinv, T* e0,
                    hipStream_t st);
// Coarse-level V-cycle operators (scalar CSR, G lanes per row):
//   resid:    r = b - A x0, with x0 = D^-1 b the pre-smoothed iterate
//   spmv:     y = A x
//   restrict: bc = R r and xc = D_c^-1 bc (the next level's right-hand side
//             and pre-smoothed iterate)
//   prolong:  x = D^-1 b + P xc
//   post:     e = x + D^-1 (b - A x)
template <class T>
void launch_csr_resid(const DCsrT<T>& A, const T* x0, const T* b, T* r, hipStream_t st);
template <class T>
void launch_csr_spmv(const DCsrT<T>& A, const T* x, T* y, hipStream_t st);
template <class T>
void launch_csr_restrict(const DCsrT<T>& R, const T* r, const T* dinv_c, T* bc, T* xc, hipStream_t st);
template <class T>
void launch_csr_prolong(const DCsrT<T>& P, const T* xc, const T* b, const T* dinv, T* x,
                        hipStream_t st);
// prolong_add: y = x + P xc (x: a pre-smoothed iterate of several sweeps)
template <class T>
void launch_csr_prolong_add(const DCsrT<T>& P, const T* xc, const T* x, T* y, hipStream_t st);
template <class T>
void launch_csr_post(const DCsrT<T>& A, const T* x, const T* b, const T* dinv, T* e, hipStream_t st);
// resid and post on a scalar SELL-64 operator (nv = 1, one thread per row)
template <class T>
void launch_sell_resid(const SellT<T>& A, const T* x0, const T* b, T* r, hipStream_t st);
template <class T>
void launch_sell_post(const SellT<T>& A, const T* x, const T* b, const T* dinv, T* e, hipStream_t st);
template <class T>
void launch_coarse_solve(int n, const double* lu, const int32_t* piv, const T* b, T* x,
                         hipStream_t st);
// The V-cycle below a small level as one dense operator B (kernels.hip): the
// setup passes over row-major n_l x w FP64 blocks, the operators (S: A_l, R_l
// or P_l; null for kBlkScale) in the preconditioner's type T:
//   kBlkScale   y = dinv x             kBlkResid  y = x - S z
//   kBlkJacobi  y = z + dinv (x - S z) kBlkProduct y = S z      kBlkAdd y += S z
enum BlkOp { kBlkScale = 0, kBlkResid = 1, kBlkJacobi = 2, kBlkProduct = 3, kBlkAdd = 4 };
template <class T>
void launch_blk_csr(int op, int nrows, int w, const DCsrT<T>* S, const T* dinv, const double* z,
                    const double* x, double* y, hipStream_t st);
// the coarsest LU solve on every column of the n x w block x; the n x n identity
void launch_blk_lu(int n, int w, const double* lu, const int32_t* piv, double* x, hipStream_t st);
void launch_blk_identity(int n, double* x, hipStream_t st);
// y = x rounded to T (m values)
template <class T>
void launch_blk_to(int64_t m, const double* x, T* y, hipStream_t st);
// e = B b with B row-major n x n in T
template <class T>
void launch_dense_gemv(int n, const T* B, const T* b, T* e, hipStream_t st);
template <class T>
void launch_stage2_resid(const Sell& A, int ne, const int32_t* eidx, const T* e0, const double* r,
                         T* r2, hipStream_t st);
template <class T>
void launch_ilu_fwd_level(const SellT<T>& L, const int32_t* perm, int32_t p0, int32_t p1, const T* r2,
                          T* y, hipStream_t st);
template <class T>
void launch_ilu_bwd_level(const SellT<T>& U, const int32_t* perm, const T* uinv, int32_t p0,
                          int32_t p1, const T* y, const T* e0, int ne, const int32_t* eidx, T* x2,
                          double* z, hipStream_t st);

// one-launch ILU sweeps (see kernels.hip); width = register slots per row
int ilu_sf_width(int max_width);  // 0 when the rows are too wide for the one-launch kernels
// r2 = r - A P_E e0 in T (e0 null: r2 = r), y, x2 := sentinel, tickets := 0
template <class T>
void launch_stage2_resid_sf(const Sell& A, int ne, const int32_t* eidx, const T* e0,
                            const double* r, T* r2, T* y, T* x2, int* tickets, hipStream_t st);
// 7-point lexicographic grids: tiled systolic sweeps.  Lt / Ut: per-cell L
// (27 values) and U + U_ii^-1 (36 values) in the tile layout of grid_tile_slot;
// ytile: forward results in the backward sweep's tile layout.
constexpr int kGridTJ = 16, kGridTK = 4;
__host__ __device__ inline int grid_nsteps(int nx) { return nx + kGridTJ - 1 + kGridTK - 1; }
inline int64_t grid_ntiles(int ny, int nz) {
  return (int64_t)((ny + kGridTJ - 1) / kGridTJ) * ((nz + kGridTK - 1) / kGridTK);
}
// slot (in units of 64-lane rows) of cell (i, j, k) in the forward / backward layout
__host__ __device__ inline void grid_tile_slot(int nx, int ny, int i, int j, int k, int64_t& fwd_row, int64_t& bwd_row,
                           int& lane) {
  const int nJ = (ny + kGridTJ - 1) / kGridTJ;
  const int J = j / kGridTJ, jj = j % kGridTJ, K = k / kGridTK, kk = k % kGridTK;
  const int64_t t = J + (int64_t)nJ * K;
  const int ns = grid_nsteps(nx);
  lane = jj + kGridTJ * kk;
  fwd_row = t * ns + (i + jj + kk);
  bwd_row = t * ns + ((nx - 1 - i) + (kGridTJ - 1 - jj) + (kGridTK - 1 - kk));
}
// r2t: stage-two residual in the forward tile layout (3 per slot); e0t: the
// V-cycle result in the backward tile layout (ne per slot), or null (x1 = 0).
// faces: the face buffers of the two sweeps, grid_face_values() each
// (forward first); the stage-two kernel fills both with the sentinel.
int64_t grid_face_values(int nx, int ny, int nz);
// Block ILU(0) of A on an nx*ny*nz 7-point grid, on the device.  One call per
// forward dependency level (positions [p0, p1) of fperm): U_cc^-1 of the
// level's cells into uinv (FP64, 9 per cell); a singular U_cc leaves zeros and
// lowers *bad to the smallest such cell.  Then launch_grid_ilu_pack writes the
// sweeps' tile layouts (Lt forward, Ut backward; cleared beforehand).
void launch_grid_ilu_diag(const Sell& A, const int32_t* fperm, int32_t p0, int32_t p1, int nx, int nxy,
                          double* uinv, int* bad, hipStream_t st);
template <class T>
void launch_grid_ilu_pack(const Sell& A, int nx, int ny, const double* uinv, T* Lt, T* Ut,
                          hipStream_t st);
// Strength of connection of one AMG level in the host construction's order
// and rounding (scalar CSR A, int32): row i's strong columns at ocol[arp[i]..],
// their count in cnt[i]; launch_compact_cols moves them to CSR order (off:
// padded row starts, rp: exclusive prefix of cnt).
void launch_strength(int n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* func,
                     double theta, double mrs, int32_t* ocol, int32_t* cnt, hipStream_t st);
void launch_compact_cols(int n, const int32_t* off, const int32_t* rp, const int32_t* ocol, int32_t* ci,
                         hipStream_t st);
// Extended+i interpolation of one AMG level in the host construction's order
// and rounding (scalar CSR A and strength pattern S, int32; cf 1 = C, -1 =
// F; func: unknown type per row; cidx: coarse index of each C point).  Row i
// goes to ocol/oval at i * outcap (outcap >= pmax, or >= interp_set_cap()
// without truncation), its length to cnt[i]; a row whose interpolatory set has
// more than interp_set_cap() points adds 1 to *overflow.  long_rows: one
// workgroup per row instead of one thread (same results; faster when rows
// are long).
void launch_interp_exti(int n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* srp,
                        const int32_t* sci, const int32_t* cf, const int32_t* func, const int32_t* cidx, int pmax,
                        int outcap, int32_t* ocol, double* oval, int32_t* cnt, int* overflow, bool long_rows,
                        hipStream_t st);
int interp_set_cap();
// Sparse product C = X Y of scalar CSR matrices in the host product's
// summation order (each entry from 0.0, products in the order of X's and Y's
// stored entries; rows sorted by column).  bound: products per row of X (at
// most spgemm_row_cap()); off: exclusive prefix of bound (int64) into the
// padded outputs ocol/oval; cnt: unique entries per row; then, with rp the
// exclusive prefix of cnt, launch_spgemm_compact writes C's ci/v.
void launch_spgemm_bound(int n, const int32_t* xrp, const int32_t* xci, const int32_t* yrp, int32_t* bound,
                         hipStream_t st);
void launch_spgemm_rows(int n, const int32_t* xrp, const int32_t* xci, const double* xv, const int32_t* yrp,
                        const int32_t* yci, const double* yv, const int64_t* off, int32_t* ocol, double* oval,
                        int32_t* cnt, int max_bound, hipStream_t st);
void launch_spgemm_compact(int n, const int64_t* off, const int32_t* rp, const int32_t* ocol, const double* oval,
                           int32_t* ci, double* v, hipStream_t st);
int spgemm_row_cap();
// Multipass interpolation (Stueben 2001) of an aggressive AMG level, one pass
// at a time, rows in the host construction's order and rounding (scalar CSR
// A and strength pattern S, int32; func: unknown type per row).  pass[i]: 0
// for C points, the pass that gave row i of P, -1 while it has none; P is CSR
// over all rows.  launch_mp_mark: flag[i] = 1 when i has no row and a strong
// dependency of i has one.  For the pass's rows now[0..m): launch_mp_bound
// gives bound[r], the products of row now[r] (or spgemm_row_cap() + 1 when it
// has more than mp_point_cap() interpolating points); with off the exclusive prefix of
// bound (every bound at most spgemm_row_cap()), launch_mp_rows writes row r
// sorted by column at off[r] of ocol/oval and its length to cnt[r].
// launch_mp_merge forms the next P (nrp: its row pointers) from P and the new
// rows, sets the pass's points to pass number pass_no and leaves rowpos (n
// entries, -1 outside a call) at -1.
void launch_mp_mark(int n, const int32_t* srp, const int32_t* sci, const int32_t* pass, int32_t* flag,
                    hipStream_t st);
// now[pos[i]] = i where flag[i] != 0 (pos: exclusive prefix of flag)
void launch_select(int n, const int32_t* flag, const int32_t* pos, int32_t* now, hipStream_t st);
// len[now[r]] = cnt[r]
void launch_mp_setlen(int m, const int32_t* now, const int32_t* cnt, int32_t* len, hipStream_t st);
void launch_mp_bound(int m, const int32_t* now, const int32_t* arp, const int32_t* aci, const double* av,
                     const int32_t* srp, const int32_t* sci, const int32_t* pass, const int32_t* func,
                     const int32_t* prp, int32_t* bound, hipStream_t st);
void launch_mp_rows(int m, const int32_t* now, const int32_t* arp, const int32_t* aci, const double* av,
                    const int32_t* srp, const int32_t* sci, const int32_t* pass, const int32_t* func,
                    const int32_t* prp, const int32_t* pci, const double* pv, const int64_t* off, int32_t* ocol,
                    double* oval, int32_t* cnt, int max_bound, hipStream_t st);
void launch_mp_merge(int n, int pass_no, int32_t* rowpos, const int32_t* now, int m, const int64_t* off,
                     const int32_t* ocol, const double* oval, const int32_t* prp, const int32_t* pci,
                     const double* pv, const int32_t* nrp, int32_t* nci, double* nv, int32_t* pass,
                     hipStream_t st);
void launch_fill_i32(int64_t n, int32_t* x, int32_t v, hipStream_t st);
int mp_point_cap();
// Distance-two strength among the C points of a first pass (aggressive
// level), as the host forms it: row r is C point cpts[r], its columns the
// coarse indices (cidx, -1 for F points) of the other C points one or two
// strong links away, sorted, each once.  bound[r]: candidates of row r (must
// be at most s2_row_cap()); launch_s2_rows with rp == nullptr writes the
// column counts to cnt, with rp (exclusive prefix of cnt) the columns to ci.
void launch_s2_bound(int nc, const int32_t* cpts, const int32_t* srp, const int32_t* sci, int32_t* bound,
                     hipStream_t st);
void launch_s2_rows(int nc, const int32_t* cpts, const int32_t* srp, const int32_t* sci, const int32_t* cidx,
                    const int32_t* rp, int32_t* ci, int32_t* cnt, hipStream_t st);
int s2_row_cap();
// HMIS over blocks of `block` (at most hmis_block_cap()) consecutive points
// of a strength pattern S (n points, int32 CSR), as the host's hmis_split.
// launch_transpose_pattern: phase 0 adds each point's dependents to deg
// (zeroed beforehand); phase 1, with cursor = the exclusive prefix of deg
// (trp), writes them to tci (any order within a row).  launch_hmis_blocks:
// the first pass inside every block (cf1: 1 for its C points, else 0), then
// cf = 1 (C), -1 (depends strongly on a C point) or 0.  launch_pmis_start:
// the undecided points' counts (cnt) and the ones without undecided
// dependents made F; launch_pmis_round: one round of picks (isnew) and their
// F points; *left = the undecided points at the round's start (0: done).
void launch_transpose_pattern(int n, const int32_t* srp, const int32_t* sci, int32_t* deg, int32_t* cursor,
                              int32_t* tci, int phase, hipStream_t st);
void launch_hmis_blocks(int n, int block, const int32_t* srp, const int32_t* sci, const int32_t* trp,
                        const int32_t* tci, int32_t* cf1, int32_t* cf, hipStream_t st);
void launch_pmis_start(int n, const int32_t* srp, const int32_t* sci, int32_t* cf, int32_t* cnt, hipStream_t st);
void launch_pmis_round(int n, const int32_t* srp, const int32_t* sci, const int32_t* trp, const int32_t* tci,
                       const int32_t* cnt, int32_t* cf, int32_t* isnew, int* left, hipStream_t st);
int hmis_block_cap();
// Exclusive prefix sums of n int32 counts: out[0..n) the offsets, out[n] the
// total (O = int64_t, or int32_t when the total fits); *maxv (if not null,
// set beforehand) is raised to the largest count.  tmp: scan_tmp_size(n)
// int64 of scratch.
template <class O>
void launch_scan(int64_t n, const int32_t* in, O* out, int64_t* tmp, int* maxv, hipStream_t st);
int64_t scan_tmp_size(int64_t n);
// Ruge-Stueben first pass over the small weakly connected components of a
// strength pattern S (n points, int32 CSR).  launch_fp_components: lam[i] =
// the number of points depending strongly on i, root[i] = the smallest point
// of i's component, size[r] = the size of the component with root r, cf[i] =
// -1 for points without any strong link, else 0.  With cursor[r] = the
// offset of root r's component in `members` (-1 for components not taken)
// and coff the offsets of the ncomp components taken (ascending roots),
// launch_fp_small lists their members and runs the pass over each (one thread
// per component: cf 1 = C, -1 = F), leaving the other points untouched.
void launch_fp_components(int n, const int32_t* srp, const int32_t* sci, int32_t* parent, int32_t* lam,
                          int32_t* root, int32_t* size, int32_t* cf, hipStream_t st);
void launch_fp_small(int n, const int32_t* root, int32_t* cursor, int32_t* members, int ncomp, const int32_t* coff,
                     const int32_t* srp, const int32_t* sci, int32_t* lam, int32_t* cf, hipStream_t st);
// Block ILU(0) of any block-sparse A on the device.  W: a copy of A's SELL-64
// values, factored in place (L left of the diagonal, U on and right of it);
// one launch_ilu_rows per forward dependency level (positions [p0, p1) of
// fperm), rows in the host factorisation's order and rounding; uinv (FP64, 9
// per row) gets U_ii^-1, a singular U_ii leaves zeros and lowers *bad to the
// row.  rp: A's row pointers, dslot: the diagonal's slot in each row (device).
// launch_ilu_pack then writes the sweeps' layouts: Lf (by forward position),
// Ub and uinv_t (planar, by backward position), their sptr filled beforehand.
void launch_ilu_rows(const Sell& A, const int32_t* fperm, int32_t p0, int32_t p1, const int32_t* rp,
                     const int32_t* dslot, double* W, double* uinv, int* bad, hipStream_t st);
template <class T>
void launch_ilu_pack(const Sell& A, const int32_t* rp, const int32_t* dslot, const double* W, const double* uinv,
                     const int32_t* fperm, const int32_t* bperm, SellT<T>& Lf, SellT<T>& Ub, T* uinv_t,
                     hipStream_t st);
// A (3x3 blocks, CSR order) into its SELL-64 layout, for the whole slices of
// rows [r0, r_end) (r0 a multiple of 64, r_end a multiple of 64 or the padded
// end); rp on the device; the rows' columns and blocks staged from q0 = rp[r0].
// A.sptr is filled beforehand.
void launch_bsr_to_sell(int nrows, int r0, int r_end, const int32_t* rp, int32_t q0, const int32_t* ci_chunk,
                        const double* v_chunk, Sell& A, hipStream_t st);
// Ahat_ij = A_ij[E,E] - W_i A_ij[H,E] in A's SELL-64 slots (ne*ne values per
// slot, A's sptr and col apply); W: 2 per cell; eidx/hidx: host arrays.
template <class T>
void launch_sell_ahat(const Sell& A, const double* W, int ne, const int32_t* eidx, const int32_t* hidx,
                      T* out, hipStream_t st);
template <class T>
void launch_stage2_grid(int nx, int ny, int nz, const Sell& A, int ne, const int32_t* eidx, const T* e0,
                        const double* r, T* r2t, T* e0t, T* faces, int* tickets, hipStream_t st);
template <class T>
void launch_ilu_fwd_grid(int nx, int ny, int nz, const T* Lt, const T* r2t, T* ytile, T* faces,
                         int* tickets, double* err, long spin_limit, hipStream_t st);
template <class T>
void launch_ilu_bwd_grid(int nx, int ny, int nz, const T* Ut, T* ytile, const T* e0t, int ne,
                         const int32_t* eidx, T* faces, double* z, int* tickets, double* err,
                         long spin_limit, hipStream_t st);
template <class T>
void launch_ilu_fwd_sf(const SellT<T>& L, int width, const int32_t* perm, const T* r2, T* y,
                       int* tickets, double* err, long spin_limit, hipStream_t st);
template <class T>
void launch_ilu_bwd_sf(const SellT<T>& U, int width, const int32_t* perm, const T* uinv,
                       const T* y, const T* e0, int ne, const int32_t* eidx, T* x2,
                       double* z, int* tickets, double* err, long spin_limit, hipStream_t st);
template <class T>
void launch_prolong_e(int32_t nrows, int ne, const int32_t* eidx, const T* e0, double* x1,
                      hipStream_t st);
void launch_sweep_prepare(int64_t n, double* y, double* x2, int* tickets, hipStream_t st);
// x[0..n) = v (a kernel, so that it may sit in a captured graph)
void launch_fill(int64_t n, double* x, double v, hipStream_t st);

// Arnoldi / BLAS-1 (deterministic two-stage reductions into `part`)
void launch_mdot(int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* part,
                 hipStream_t st);
void launch_maxpy_dot(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                      double* w, double* part, hipStream_t st);
void launch_maxpy_norm(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                       double* w, double* part, hipStream_t st);
void launch_reduce(int ncols, const double* part, double* out, int add_to_out, hipStream_t st);
void launch_scale(int64_t n, const double* w, const double* nrm2, double* v, hipStream_t st);
void launch_scale_host(int64_t n, const double* w, double s, double* v, hipStream_t st);
void launch_norm2(int64_t n, const double* x, double* part, hipStream_t st);
void launch_update_host_coef(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                             double* x, hipStream_t st);

}  // namespace cptr
