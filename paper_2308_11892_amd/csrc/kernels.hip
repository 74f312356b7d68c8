// kernels.hip -- HIP kernels of the CPTR hot path for gfx950 (MI355X), FP64.
//
// Paper mapping (Cremon, Franc, Hamon, CPTR):
//   bsr3 SpMV            A z in GMRES and in the residual of Eq. (3)
//   l0 restrict          quasi-IMPES restriction to the (p, T) block (Sec. 5.2)
//   l0 / csr V-cycle     one system-AMG V-cycle with one l1-Jacobi sweep before
//                        and after the coarse correction (Sec. 3.1, 3.2)
//   stage2 resid         r - A M1^-1 r with M1^-1 injecting into (p, T) (Eq. 3)
//   ilu fwd / bwd        ILU(0) triangular sweeps, second stage (Sec. 3.1)
//   mdot / maxpy         Arnoldi orthogonalisation of right-preconditioned GMRES
//   setup                A's device layout, the reduced elliptic blocks (Sec. 5.2),
//                        block ILU(0) (Sec. 3.1), the Galerkin products of the
//                        AMG hierarchy (Sec. 3.1)
//
// Everything here is bandwidth-bound sparse or vector work: no MFMA.  Block
// values are stored as lane-contiguous planes (see Sell in kernels.hpp) so a
// wavefront reads each entry of 64 blocks as one contiguous 512-byte segment.
// Reductions are two-stage with a fixed order, so results are bit-identical
// from run to run.
#include "kernels.hpp"

#include <algorithm>
#include <climits>

namespace cptr {

namespace {

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD walks one contiguous range of logical blocks (its L2 then sees
// neighbouring rows and shares their gathered vector entries).
__device__ __forceinline__ int xcd_block(int b, int nblk) {
  const int x = b & 7, k = b >> 3;
  const int q = nblk >> 3, r = nblk & 7;
  return x * q + min(x, r) + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_down(v, off, G);
  return v;
}

inline int nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

// --------------------------------------------------------------------------
// y = A x  or  y = b - A x, A 3x3 block-sparse in SELL-64
template <bool RESID>
__global__ __launch_bounds__(kBlock) void k_bsr3_spmv(int nrows, int nblk, const int32_t* __restrict__ sptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ y) {
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= nrows) return;
  const int s = row >> 6, lane = row & 63;
  const int k0 = sptr[s], k1 = sptr[s + 1];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  // A is read once per product: non-temporal loads keep it from displacing x
  // in the caches
#pragma unroll 4
  for (int k = k0; k < k1; ++k) {
    const int c = __builtin_nontemporal_load(col + (size_t)k * 64 + lane);
    const double* v = val + (size_t)k * 9 * 64 + lane;
    double m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = __builtin_nontemporal_load(v + e * 64);
    const double x0 = x[3 * (size_t)c], x1 = x[3 * (size_t)c + 1], x2 = x[3 * (size_t)c + 2];
    a0 += m[0] * x0 + m[1] * x1 + m[2] * x2;
    a1 += m[3] * x0 + m[4] * x1 + m[5] * x2;
    a2 += m[6] * x0 + m[7] * x1 + m[8] * x2;
  }
  double* yo = y + 3 * (size_t)row;
  if (RESID) {
    const double* bo = b + 3 * (size_t)row;
    yo[0] = bo[0] - a0;
    yo[1] = bo[1] - a1;
    yo[2] = bo[2] - a2;
  } else {
    yo[0] = a0;
    yo[1] = a1;
    yo[2] = a2;
  }
}

// --------------------------------------------------------------------------
// quasi-IMPES restriction: b0_i = r_i[E] - W_i r_i[H]
// (computed in FP64, stored in the preconditioner's type T)
// (with dinv, also the pre-smoothed iterate x0 = D^-1 b0 of the V-cycle)
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_l0_restrict(int nc, const double* __restrict__ r,
                                                        const double* __restrict__ W, int e0,
                                                        int e1, int h0, int h1,
                                                        T* __restrict__ b0, const T* __restrict__ dinv,
                                                        T* __restrict__ x0) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nc) return;
  const double* ri = r + 3 * (size_t)i;
  T bv[NE];
  if (NE == 2) {
    const double rh = ri[h0];
    bv[0] = (T)(ri[e0] - W[2 * (size_t)i] * rh);
    bv[NE - 1] = (T)(ri[e1] - W[2 * (size_t)i + 1] * rh);
  } else {
    bv[0] = (T)(ri[e0] - W[2 * (size_t)i] * ri[h0] - W[2 * (size_t)i + 1] * ri[h1]);
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) {
    b0[(size_t)i * NE + a] = bv[a];
    if (dinv) x0[(size_t)i * NE + a] = dinv[(size_t)i * NE + a] * bv[a];
  }
}

// r0 = b0 - Ahat x0 with x0 = D^-1 b0: the residual after pre-smoothing from
// zero
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_l0_resid(int nc, int nblk, const int32_t* __restrict__ sptr,
                                                     const int32_t* __restrict__ col,
                                                     const T* __restrict__ val,
                                                     const T* __restrict__ x0,
                                                     const T* __restrict__ b0,
                                                     T* __restrict__ r0) {
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= nc) return;
  const int s = row >> 6, lane = row & 63;
  T acc[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = 0;
#pragma unroll 4
  for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
    const int c = __builtin_nontemporal_load(col + (size_t)k * 64 + lane);
    const T* v = val + (size_t)k * NE * NE * 64 + lane;
    T xc[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) xc[q] = x0[(size_t)c * NE + q];
#pragma unroll
    for (int a = 0; a < NE; ++a)
#pragma unroll
      for (int q = 0; q < NE; ++q) acc[a] += __builtin_nontemporal_load(v + (a * NE + q) * 64) * xc[q];
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) r0[(size_t)row * NE + a] = b0[(size_t)row * NE + a] - acc[a];
}

// e0 = x0 + D^-1 (b0 - Ahat x0): post-smoothing at level 0
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_l0_post(int nc, int nblk, const int32_t* __restrict__ sptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const T* __restrict__ x0,
                                                    const T* __restrict__ b0,
                                                    const T* __restrict__ dinv,
                                                    T* __restrict__ e0) {
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= nc) return;
  const int s = row >> 6, lane = row & 63;
  T acc[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) acc[a] = 0;
#pragma unroll 4
  for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
    const int c = __builtin_nontemporal_load(col + (size_t)k * 64 + lane);
    const T* v = val + (size_t)k * NE * NE * 64 + lane;
    T xc[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) xc[q] = x0[(size_t)c * NE + q];
#pragma unroll
    for (int a = 0; a < NE; ++a)
#pragma unroll
      for (int q = 0; q < NE; ++q) acc[a] += __builtin_nontemporal_load(v + (a * NE + q) * 64) * xc[q];
  }
#pragma unroll
  for (int a = 0; a < NE; ++a) {
    const size_t i = (size_t)row * NE + a;
    e0[i] = x0[i] + dinv[i] * (b0[i] - acc[a]);
  }
}

// --------------------------------------------------------------------------
// scalar CSR kernels: G lanes per row
// kRestrict: y = A x and y2 = D^-1 y (the next level's right-hand side and its
// pre-smoothed iterate); kResid: y = b - A x with x = D^-1 b, the residual
// after one l1-Jacobi sweep from zero; kProlong: y = D^-1 b + A x; kPost:
// y = x + D^-1 (b - A x); kProlongAdd: y = b + A x (b: the pre-smoothed
// iterate, when it took more than one sweep)
enum CsrOp { kSpmv = 0, kResid = 1, kProlong = 2, kPost = 3, kRestrict = 4, kProlongAdd = 5 };

// entries per lane and chunk of the scalar CSR kernels
constexpr int kCsrE = 4;
template <int G, int OP, class T>
__global__ __launch_bounds__(kBlock) void k_csr(int n, const int32_t* __restrict__ rp,
                                                const int32_t* __restrict__ ci,
                                                const T* __restrict__ v,
                                                const T* __restrict__ x,
                                                const T* __restrict__ b,
                                                const T* __restrict__ dinv,
                                                T* __restrict__ y, T* __restrict__ y2) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int row = (int)(t / G), sub = (int)(t % G);
  const bool live = row < n;
  T acc = 0;
  // the row in chunks of kCsrE entries per lane whose loads all go out
  // before the chunk's first product (indices clamped to the row's last
  // entry, surplus products dropped); the sum runs in entry order
  const int k1 = live ? rp[row + 1] : 0;
  for (int kb = (live ? rp[row] : 0) + sub; kb < k1; kb += kCsrE * G) {
    int cc[kCsrE];
    T vv[kCsrE], xx[kCsrE];
#pragma unroll
    for (int q = 0; q < kCsrE; ++q) {
      const int k = min(kb + q * G, k1 - 1);
      cc[q] = ci[k];
      vv[q] = v[k];
    }
#pragma unroll
    for (int q = 0; q < kCsrE; ++q) xx[q] = x[cc[q]];
#pragma unroll
    for (int q = 0; q < kCsrE; ++q)
      if (kb + q * G < k1) acc += vv[q] * xx[q];
  }
  acc = group_sum<G, T>(acc);
  if (!live || sub != 0) return;
  switch (OP) {
    case kSpmv: y[row] = acc; break;
    case kRestrict:
      y[row] = acc;
      y2[row] = dinv[row] * acc;
      break;
    case kResid: y[row] = b[row] - acc; break;
    case kProlong: y[row] = dinv[row] * b[row] + acc; break;
    case kProlongAdd: y[row] = b[row] + acc; break;
    case kPost: y[row] = x[row] + dinv[row] * (b[row] - acc); break;
  }
}

// scalar SELL-64 operator (kResid or kPost), one thread per row, each row
// summing its entries in stored order
template <int OP, class T>
__global__ __launch_bounds__(kBlock) void k_sell_scalar(int n, int nblk, const int32_t* __restrict__ sptr,
                                                        const int32_t* __restrict__ col,
                                                        const T* __restrict__ val, const T* __restrict__ x,
                                                        const T* __restrict__ b, const T* __restrict__ dinv,
                                                        T* __restrict__ y) {
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= n) return;
  const int s = row >> 6, lane = row & 63;
  T acc = 0;
  // slots in chunks whose loads all go out before the first product (slot
  // clamped to the slice's last, surplus products dropped); entry order kept
  constexpr int CH = 8;
  const int k1 = sptr[s + 1];
  for (int kb = sptr[s]; kb < k1; kb += CH) {
    int cc[CH];
    T vv[CH], xx[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const size_t k = (size_t)min(kb + q, k1 - 1);
      cc[q] = col[k * 64 + lane];
      vv[q] = val[k * 64 + lane];
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) xx[q] = x[cc[q]];
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (kb + q < k1) acc += vv[q] * xx[q];
  }
  if (OP == kResid)
    y[row] = b[row] - acc;
  else
    y[row] = x[row] + dinv[row] * (b[row] - acc);
}

template <int OP, class T>
void launch_csr_op(const DCsrT<T>& A, const T* x, const T* b, const T* dinv, T* y, hipStream_t st,
                   T* y2 = nullptr) {
  if (A.n == 0) return;
  const int64_t threads = (int64_t)A.n * A.group;
  const int grid = nblocks(threads, kBlock);
  switch (A.group) {
#define CSR_CASE(G) \
  case G: k_csr<G, OP, T><<<grid, kBlock, 0, st>>>(A.n, A.rp, A.ci, A.v, x, b, dinv, y, y2); break;
    CSR_CASE(1) CSR_CASE(2) CSR_CASE(4) CSR_CASE(8) CSR_CASE(16) CSR_CASE(32) CSR_CASE(64)
#undef CSR_CASE
    default:
      k_csr<8, OP, T><<<nblocks((int64_t)A.n * 8, kBlock), kBlock, 0, st>>>(A.n, A.rp, A.ci, A.v, x, b, dinv, y, y2);
  }
}

// --------------------------------------------------------------------------
// coarsest level: x = (LU)^-1 b with row swaps piv (one workgroup)
// (FP64 factors and arithmetic; b and x in the preconditioner's type)
template <class T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int n, const double* __restrict__ lu,
                                                         const int32_t* __restrict__ piv,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ x) {
  extern __shared__ double s[];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kBlock) s[i] = b[i];
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < n; ++k) {
      const int p = piv[k];
      if (p != k) {
        const double t = s[k];
        s[k] = s[p];
        s[p] = t;
      }
    }
  __syncthreads();
  for (int i = 0; i < n; ++i) {  // unit lower
    const double xi = s[i];
    for (int j = i + 1 + tid; j < n; j += kBlock) s[j] -= lu[(size_t)j * n + i] * xi;
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {  // upper
    if (tid == 0) s[i] /= lu[(size_t)i * n + i];
    __syncthreads();
    const double xi = s[i];
    for (int j = tid; j < i; j += kBlock) s[j] -= lu[(size_t)j * n + i] * xi;
    __syncthreads();
  }
  for (int i = tid; i < n; i += kBlock) x[i] = (T)s[i];
}

// --------------------------------------------------------------------------
// The bottom of the V-cycle as one dense operator.  The cycle of Sec. 3.1
// starts every level's iterate from zero, so the part below a small level t
// (its smoothing, the coarser levels and the coarsest solve) is a fixed linear
// map e_t = B_t b_t.  Setup forms B_t by running exactly that part of the
// cycle on the n_t unit vectors at once: every level's vectors become
// row-major blocks of n_l x w FP64 values (w = n_t columns), every operator
// pass a pass over all columns.  Each apply then replaces the ~4 launches per
// level below t by one dense matrix-vector product.

// one sparse row (blockIdx.y) times the block z, the threads over columns:
//   scale:   y = dinv x                   (the first sweep from zero)
//   resid:   y = x - A z                  (x: right-hand sides)
//   jacobi:  y = z + dinv (x - A z)       (one l1-Jacobi sweep from iterate z)
//   product: y = S z                      (restriction)
//   add:     y += S z                     (prolongation into the iterate)
template <int OP, class T>
__global__ __launch_bounds__(kBlock) void k_blk_csr(int w, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci, const T* __restrict__ v,
                                                    const T* __restrict__ dinv, const double* __restrict__ z,
                                                    const double* __restrict__ x, double* __restrict__ y) {
  const int row = blockIdx.y;
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= w) return;
  const size_t o = (size_t)row * w + c;
  if (OP == kBlkScale) {
    y[o] = (double)dinv[row] * x[o];
    return;
  }
  double acc = 0.0;
  for (int k = rp[row]; k < rp[row + 1]; ++k) acc += (double)v[k] * z[(size_t)ci[k] * w + c];
  switch (OP) {
    case kBlkResid: y[o] = x[o] - acc; break;
    case kBlkJacobi: y[o] = z[o] + (double)dinv[row] * (x[o] - acc); break;
    case kBlkProduct: y[o] = acc; break;
    case kBlkAdd: y[o] += acc; break;
    default: break;
  }
}

// the coarsest dense LU solve (the same steps as k_coarse_solve) on every
// column of the n x w block x, one thread per column
__global__ __launch_bounds__(kBlock) void k_blk_lu(int n, int w, const double* __restrict__ lu,
                                                   const int32_t* __restrict__ piv, double* __restrict__ x) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= w) return;
  double* xc = x + c;
  for (int k = 0; k < n; ++k) {
    const int p = piv[k];
    if (p != k) {
      const double t = xc[(size_t)k * w];
      xc[(size_t)k * w] = xc[(size_t)p * w];
      xc[(size_t)p * w] = t;
    }
  }
  for (int i = 0; i < n; ++i) {
    const double xi = xc[(size_t)i * w];
    for (int j = i + 1; j < n; ++j) xc[(size_t)j * w] -= lu[(size_t)j * n + i] * xi;
  }
  for (int i = n - 1; i >= 0; --i) {
    xc[(size_t)i * w] /= lu[(size_t)i * n + i];
    const double xi = xc[(size_t)i * w];
    for (int j = 0; j < i; ++j) xc[(size_t)j * w] -= lu[(size_t)j * n + i] * xi;
  }
}

// the n x n identity block; the finished B in the preconditioner's type
__global__ __launch_bounds__(kBlock) void k_blk_identity(int n, double* __restrict__ x) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q < (int64_t)n * n) x[q] = q / n == q % n ? 1.0 : 0.0;
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_blk_to(int64_t m, const double* __restrict__ x, T* __restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (q < m) y[q] = (T)x[q];
}

// e = B b, B row-major n x n: one workgroup per row, each thread PER columns
// (n <= PER * kBlock) whose loads all go out before the first product; the
// index is clamped and the surplus products dropped, so no load waits on a
// branch.  Accumulates in T like the other operators of the preconditioner.
template <int PER, class T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(int n, const T* __restrict__ B, const T* __restrict__ b,
                                                       T* __restrict__ e) {
  const T* r = B + (size_t)blockIdx.x * n;
  T bv[PER], rv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int c = min((int)threadIdx.x + q * kBlock, n - 1);
    rv[q] = r[c];
    bv[q] = b[c];
  }
  T acc = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q)
    if ((int)threadIdx.x + q * kBlock < n) acc += rv[q] * bv[q];
  acc = group_sum<64, T>(acc);
  __shared__ T part[kBlock / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T sum = 0;
    for (int w = 0; w < kBlock / 64; ++w) sum += part[w];
    e[blockIdx.x] = sum;
  }
}

// --------------------------------------------------------------------------
// stage-two residual r2 = r - A x1 with x1[E] = e0, x1[H] = 0: only the
// elliptic columns of each block are read
// (A and the arithmetic in FP64, e0 and r2 in the preconditioner's type T;
// without e0 this only converts r)
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_stage2_resid(int nrows, int nblk, const int32_t* __restrict__ sptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val, int ea,
                                                         int eb, const T* __restrict__ e0,
                                                         const double* __restrict__ r,
                                                         T* __restrict__ r2) {
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= nrows) return;
  const int s = row >> 6, lane = row & 63;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  // e0 == nullptr (no first stage): r2 = r, converted to T
  for (int k = sptr[s]; e0 && k < sptr[s + 1]; ++k) {
    const int c = col[(size_t)k * 64 + lane];
    const double* v = val + (size_t)k * 9 * 64 + lane;
    const double u = e0[(size_t)c * NE];
    a0 += v[(0 * 3 + ea) * 64] * u;
    a1 += v[(1 * 3 + ea) * 64] * u;
    a2 += v[(2 * 3 + ea) * 64] * u;
    if (NE == 2) {
      const double w = e0[(size_t)c * NE + 1];
      a0 += v[(0 * 3 + eb) * 64] * w;
      a1 += v[(1 * 3 + eb) * 64] * w;
      a2 += v[(2 * 3 + eb) * 64] * w;
    }
  }
  const double* ri = r + 3 * (size_t)row;
  T* o = r2 + 3 * (size_t)row;
  o[0] = (T)(ri[0] - a0);
  o[1] = (T)(ri[1] - a1);
  o[2] = (T)(ri[2] - a2);
}

// --------------------------------------------------------------------------
// ILU(0) sweeps, one launch per dependency level.  Positions are rows sorted
// by level; slot columns < 0 are padding.
template <class T>
__global__ __launch_bounds__(kBlock) void k_ilu_fwd(int p0, int p1, const int32_t* __restrict__ sptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const int32_t* __restrict__ perm,
                                                    const T* __restrict__ r2,
                                                    T* __restrict__ y) {
  const int p = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (p >= p1) return;
  const int i = perm[p];
  const int s = p >> 6, lane = p & 63;
  T a0 = r2[3 * (size_t)i], a1 = r2[3 * (size_t)i + 1], a2 = r2[3 * (size_t)i + 2];
  for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
    const int c = col[(size_t)k * 64 + lane];
    if (c < 0) continue;
    const T* v = val + (size_t)k * 9 * 64 + lane;
    const T x0 = y[3 * (size_t)c], x1 = y[3 * (size_t)c + 1], x2 = y[3 * (size_t)c + 2];
    a0 -= v[0] * x0 + v[64] * x1 + v[128] * x2;
    a1 -= v[192] * x0 + v[256] * x1 + v[320] * x2;
    a2 -= v[384] * x0 + v[448] * x1 + v[512] * x2;
  }
  y[3 * (size_t)i] = a0;
  y[3 * (size_t)i + 1] = a1;
  y[3 * (size_t)i + 2] = a2;
}

template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_ilu_bwd(int p0, int p1, int npad, const int32_t* __restrict__ sptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const int32_t* __restrict__ perm,
                                                    const T* __restrict__ uinv,
                                                    const T* __restrict__ y, const T* __restrict__ e0,
                                                    int ea, int eb, T* __restrict__ x2,
                                                    double* __restrict__ z) {
  const int p = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (p >= p1) return;
  const int i = perm[p];
  const int s = p >> 6, lane = p & 63;
  T a0 = y[3 * (size_t)i], a1 = y[3 * (size_t)i + 1], a2 = y[3 * (size_t)i + 2];
  for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
    const int c = col[(size_t)k * 64 + lane];
    if (c < 0) continue;
    const T* v = val + (size_t)k * 9 * 64 + lane;
    const T x0 = x2[3 * (size_t)c], x1 = x2[3 * (size_t)c + 1], xx = x2[3 * (size_t)c + 2];
    a0 -= v[0] * x0 + v[64] * x1 + v[128] * xx;
    a1 -= v[192] * x0 + v[256] * x1 + v[320] * xx;
    a2 -= v[384] * x0 + v[448] * x1 + v[512] * xx;
  }
  const T* u = uinv + p;
  const T o0 = u[0] * a0 + u[(size_t)npad] * a1 + u[2 * (size_t)npad] * a2;
  const T o1 = u[3 * (size_t)npad] * a0 + u[4 * (size_t)npad] * a1 + u[5 * (size_t)npad] * a2;
  const T o2 = u[6 * (size_t)npad] * a0 + u[7 * (size_t)npad] * a1 + u[8 * (size_t)npad] * a2;
  x2[3 * (size_t)i] = o0;
  x2[3 * (size_t)i + 1] = o1;
  x2[3 * (size_t)i + 2] = o2;
  // z = x1 + x2 with x1[E] = e0 and x1[H] = 0 (e0 == nullptr: x1 = 0), in FP64
  const double ex = e0 ? (double)e0[(size_t)i * NE] : 0.0;
  const double ey = (NE == 2 && e0) ? (double)e0[(size_t)i * NE + 1] : 0.0;
  z[3 * (size_t)i] = (double)o0 + (ea == 0 ? ex : 0.0) + (NE == 2 && eb == 0 ? ey : 0.0);
  z[3 * (size_t)i + 1] = (double)o1 + (ea == 1 ? ex : 0.0) + (NE == 2 && eb == 1 ? ey : 0.0);
  z[3 * (size_t)i + 2] = (double)o2 + (ea == 2 ? ex : 0.0) + (NE == 2 && eb == 2 ? ey : 0.0);
}

// --------------------------------------------------------------------------
// ILU(0) sweeps in one launch each, without level barriers.
//
// A row may start as soon as the rows it depends on are written.  Readiness is
// carried by the solution vector itself: the kernel that runs before a sweep
// fills the sweep's output with a sentinel NaN pattern, rows are published
// with device-coherent (sc1) stores and dependencies are polled with
// device-coherent loads until no sentinel is left.  Arithmetic never yields
// this payload (NaNs produced by arithmetic are the canonical quiet NaN), so
// a published value can not be mistaken for "not ready".
//
// Deadlock freedom: positions are sorted by dependency level, so every
// dependency sits at a lower position.  Each workgroup takes its block of
// positions from a ticket counter when it starts, hence it only waits on
// workgroups that started before it (resident or finished).  Inside a wave
// the lanes retry until every lane is done, so lanes waiting on lower lanes
// of the same wave do not block them.  Every wait is bounded: after
// `spin_limit` rounds the wave records an error flag and exits.
// The FP32 sweeps use a signalling-NaN payload of their own.
constexpr unsigned long long kSentinel = 0x7FF4C0DE5E1F0BADull;
constexpr unsigned kSentinelF = 0x7FA5C0DEu;

template <class T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool is_sent(double v) {
  return (unsigned long long)__double_as_longlong(v) == kSentinel;
}
__device__ __forceinline__ bool is_sent(float v) { return __float_as_uint(v) == kSentinelF; }
template <class T>
__device__ __forceinline__ T sentinel_value();
template <>
__device__ __forceinline__ double sentinel_value<double>() {
  return __longlong_as_double((long long)kSentinel);
}
template <>
__device__ __forceinline__ float sentinel_value<float>() {
  return __uint_as_float(kSentinelF);
}

__device__ __forceinline__ int take_ticket(int* ctr) {
  __shared__ int s_ticket;
  if (threadIdx.x == 0) s_ticket = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return s_ticket;
}

// Forward sweep y = L^-1 r2 (unit block-lower L), in the factors' type T.
template <int W, class T>
__global__ __launch_bounds__(kBlock) void k_ilu_fwd_sf(int npos, const int32_t* __restrict__ sptr,
                                                       const int32_t* __restrict__ col,
                                                       const T* __restrict__ val,
                                                       const int32_t* __restrict__ perm,
                                                       const T* __restrict__ r2, T* y,
                                                       int* tickets, double* err, long spin_limit) {
  const int blk = take_ticket(tickets);
  const int p = blk * kBlock + threadIdx.x;
  const bool active = p < npos;
  int i = 0;
  T a0 = T(0), a1 = T(0), a2 = T(0);
  int c[W];
  T Lv[W][9];
  T yv[W][3];
  unsigned need = 0;
  if (active) {
    i = perm[p];
    a0 = r2[3 * (size_t)i];
    a1 = r2[3 * (size_t)i + 1];
    a2 = r2[3 * (size_t)i + 2];
    const int s = p >> 6, lane = p & 63;
    const int k0 = sptr[s], w = sptr[s + 1] - k0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      c[k] = -1;
      if (k < w) {
        c[k] = col[(size_t)(k0 + k) * 64 + lane];
        const T* v = val + (size_t)(k0 + k) * 9 * 64 + lane;
#pragma unroll
        for (int e = 0; e < 9; ++e) Lv[k][e] = v[e * 64];
      }
      if (c[k] >= 0) need |= 1u << k;
    }
  }
  bool done = !active;
  for (long spin = 0;; ++spin) {
    if (!done) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (need & (1u << k)) {
          const T* q = y + 3 * (size_t)c[k];
          const T u0 = ld_dev(q), u1 = ld_dev(q + 1), u2 = ld_dev(q + 2);
          if (!is_sent(u0) && !is_sent(u1) && !is_sent(u2)) {
            yv[k][0] = u0;
            yv[k][1] = u1;
            yv[k][2] = u2;
            need &= ~(1u << k);
          }
        }
      }
      if (need == 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          if (c[k] < 0) continue;
          a0 -= Lv[k][0] * yv[k][0] + Lv[k][1] * yv[k][1] + Lv[k][2] * yv[k][2];
          a1 -= Lv[k][3] * yv[k][0] + Lv[k][4] * yv[k][1] + Lv[k][5] * yv[k][2];
          a2 -= Lv[k][6] * yv[k][0] + Lv[k][7] * yv[k][1] + Lv[k][8] * yv[k][2];
        }
        st_dev(y + 3 * (size_t)i, a0);
        st_dev(y + 3 * (size_t)i + 1, a1);
        st_dev(y + 3 * (size_t)i + 2, a2);
        done = true;
      }
    }
    if (__all(done)) break;
    if (spin >= spin_limit) {
      st_dev(err, 1.0);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Backward sweep x2 = U^-1 y with U_ii^-1 stored per position, and z = x1 + x2
// (the sweep in T, z in FP64).
template <int W, int NE, class T>
__global__ __launch_bounds__(kBlock) void k_ilu_bwd_sf(int npos, int npad, const int32_t* __restrict__ sptr,
                                                       const int32_t* __restrict__ col,
                                                       const T* __restrict__ val,
                                                       const int32_t* __restrict__ perm,
                                                       const T* __restrict__ uinv,
                                                       const T* y, const T* __restrict__ e0,
                                                       int ea, int eb, T* x2,
                                                       double* __restrict__ z, int* tickets,
                                                       double* err, long spin_limit) {
  const int blk = take_ticket(tickets + 1);
  const int p = blk * kBlock + threadIdx.x;
  const bool active = p < npos;
  int i = 0;
  T a0 = T(0), a1 = T(0), a2 = T(0);
  int c[W];
  T Uv[W][9];
  T xv[W][3];
  unsigned need = 0;
  if (active) {
    i = perm[p];
    a0 = ld_dev(y + 3 * (size_t)i);
    a1 = ld_dev(y + 3 * (size_t)i + 1);
    a2 = ld_dev(y + 3 * (size_t)i + 2);
    const int s = p >> 6, lane = p & 63;
    const int k0 = sptr[s], w = sptr[s + 1] - k0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      c[k] = -1;
      if (k < w) {
        c[k] = col[(size_t)(k0 + k) * 64 + lane];
        const T* v = val + (size_t)(k0 + k) * 9 * 64 + lane;
#pragma unroll
        for (int e = 0; e < 9; ++e) Uv[k][e] = v[e * 64];
      }
      if (c[k] >= 0) need |= 1u << k;
    }
  }
  bool done = !active;
  for (long spin = 0;; ++spin) {
    if (!done) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        if (need & (1u << k)) {
          const T* q = x2 + 3 * (size_t)c[k];
          const T u0 = ld_dev(q), u1 = ld_dev(q + 1), u2 = ld_dev(q + 2);
          if (!is_sent(u0) && !is_sent(u1) && !is_sent(u2)) {
            xv[k][0] = u0;
            xv[k][1] = u1;
            xv[k][2] = u2;
            need &= ~(1u << k);
          }
        }
      }
      if (need == 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          if (c[k] < 0) continue;
          a0 -= Uv[k][0] * xv[k][0] + Uv[k][1] * xv[k][1] + Uv[k][2] * xv[k][2];
          a1 -= Uv[k][3] * xv[k][0] + Uv[k][4] * xv[k][1] + Uv[k][5] * xv[k][2];
          a2 -= Uv[k][6] * xv[k][0] + Uv[k][7] * xv[k][1] + Uv[k][8] * xv[k][2];
        }
        const T* u = uinv + p;
        const T o0 = u[0] * a0 + u[(size_t)npad] * a1 + u[2 * (size_t)npad] * a2;
        const T o1 = u[3 * (size_t)npad] * a0 + u[4 * (size_t)npad] * a1 + u[5 * (size_t)npad] * a2;
        const T o2 = u[6 * (size_t)npad] * a0 + u[7 * (size_t)npad] * a1 + u[8 * (size_t)npad] * a2;
        st_dev(x2 + 3 * (size_t)i, o0);
        st_dev(x2 + 3 * (size_t)i + 1, o1);
        st_dev(x2 + 3 * (size_t)i + 2, o2);
        const double ex = e0 ? (double)e0[(size_t)i * NE] : 0.0;
        const double ey = (NE == 2 && e0) ? (double)e0[(size_t)i * NE + 1] : 0.0;
        z[3 * (size_t)i] = (double)o0 + (ea == 0 ? ex : 0.0) + (NE == 2 && eb == 0 ? ey : 0.0);
        z[3 * (size_t)i + 1] = (double)o1 + (ea == 1 ? ex : 0.0) + (NE == 2 && eb == 1 ? ey : 0.0);
        z[3 * (size_t)i + 2] = (double)o2 + (ea == 2 ? ex : 0.0) + (NE == 2 && eb == 2 ? ey : 0.0);
        done = true;
      }
    }
    if (__all(done)) break;
    if (spin >= spin_limit) {
      st_dev(err, 1.0);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}


// --------------------------------------------------------------------------
// x1 = P_E e0: elliptic unknowns from e0, hyperbolic unknowns zero
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_prolong_e(int nrows, const T* __restrict__ e0, int ea,
                                                      int eb, double* __restrict__ x1) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nrows) return;
  double o[3] = {0.0, 0.0, 0.0};
  const double ex = e0[(size_t)i * NE];
  const double ey = NE == 2 ? (double)e0[(size_t)i * NE + 1] : 0.0;
  x1[3 * (size_t)i] = (ea == 0 ? ex : 0.0) + (NE == 2 && eb == 0 ? ey : 0.0) + o[0];
  x1[3 * (size_t)i + 1] = (ea == 1 ? ex : 0.0) + (NE == 2 && eb == 1 ? ey : 0.0) + o[1];
  x1[3 * (size_t)i + 2] = (ea == 2 ? ex : 0.0) + (NE == 2 && eb == 2 ? ey : 0.0) + o[2];
}

// prepares one-launch sweeps on an arbitrary right-hand side:
// y, x2 := sentinel, both ticket counters := 0
__global__ __launch_bounds__(kBlock) void k_sweep_prepare(int64_t n, double* __restrict__ y,
                                                          double* __restrict__ x2, int* tickets) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i == 0) {
    tickets[0] = 0;
    tickets[1] = 0;
  }
  if (i < n) {
    const double s0 = __longlong_as_double((long long)kSentinel);
    y[i] = s0;
    x2[i] = s0;
  }
}


// --------------------------------------------------------------------------
// ILU(0) sweeps for a 7-point stencil in lexicographic order (x fastest).
//
// One workgroup owns a tile of 16 x 4 x-pencils (lane = jj + 16 kk, pencil
// (j, k) = (16 J + jj, 4 K + kk)) and walks it as a skewed systolic array: at
// step s lane (jj, kk) handles cell i = s - jj - kk of its pencil.  The three
// lower neighbours of that cell were handled one step earlier by the lane
// itself (i-1), by lane jj-1 (j-1) and by lane kk-1 (k-1), so they arrive in
// registers or through cross-lane moves.  Only lanes on the tile's low faces
// (jj = 0, kk = 0) need values of another tile; those are polled from the
// device-coherent, sentinel-filled output as in the one-launch sweeps.  Tiles
// take tickets in (K, J) order, so a tile only waits on tiles that started
// before it.  The backward sweep is the mirror image (high faces, tiles in
// reverse order).
//
// Matrix data per cell: L = blocks (-x, -y, -z); U = blocks (+x, +y, +z) then
// U_ii^-1; blocks of absent neighbours are zero.
constexpr int kTJ = 16, kTK = 4;

template <class T>
struct Vec3 {
  T v0, v1, v2;
};

template <class T>
__device__ __forceinline__ Vec3<T> shfl_up3(Vec3<T> a, int d) {
  return {__shfl_up(a.v0, d, 64), __shfl_up(a.v1, d, 64), __shfl_up(a.v2, d, 64)};
}
template <class T>
__device__ __forceinline__ Vec3<T> shfl_down3(Vec3<T> a, int d) {
  return {__shfl_down(a.v0, d, 64), __shfl_down(a.v1, d, 64), __shfl_down(a.v2, d, 64)};
}
template <class T>
__device__ __forceinline__ Vec3<T> ld3_dev(const T* p) { return {ld_dev(p), ld_dev(p + 1), ld_dev(p + 2)}; }
template <class T>
__device__ __forceinline__ bool sent3(const Vec3<T>& a) { return is_sent(a.v0) || is_sent(a.v1) || is_sent(a.v2); }
template <class T>
__device__ __forceinline__ void mv3_sub(const T* b, const Vec3<T>& x, T& a0, T& a1, T& a2) {
  a0 -= b[0] * x.v0 + b[1] * x.v1 + b[2] * x.v2;
  a1 -= b[3] * x.v0 + b[4] * x.v1 + b[5] * x.v2;
  a2 -= b[6] * x.v0 + b[7] * x.v1 + b[8] * x.v2;
}

// Both directions share one kernel.
//   FWD: y = L^-1 r2.  M = L blocks (-x, -y, -z), rhs = r2, both in the
//        forward tile layout.  y goes to `ytile` in the backward tile layout
//        (all lanes of a forward step land in one backward step: coalesced);
//        the lanes whose values other tiles read (high faces jj = 15,
//        kk = 3) also publish them to the tile's face buffer.
//   BWD: x2 = U^-1 y, z = P_E e0 + x2.  M = U blocks (+x, +y, +z) then
//        U_ii^-1, rhs = ytile, e0 (NE values), all in the backward tile layout;
//        low-face lanes (jj = 0, kk = 0) publish x2.
// Face buffer of a sweep: per tile and step 60 values, the J face (3
// components x 4 lanes kk) then the K face (3 components x 16 lanes jj),
// ((tile * nsteps + step) * 60 + ...), written with device-coherent stores at
// the step that computes them and filled with the sentinel before the sweep.
// A tile needs the J-face values of its upstream J neighbour from that tile's
// step s + 15 and the K-face values of its K neighbour from step s + 3 (the
// skew), so both the stores of one step and the loads of one step are
// contiguous.
// Tile layout of per-cell data with NV values: ((tile * nsteps + step) * NV +
// e) * 64 + lane, tile = J + nJ K, step = the step that handles the cell in
// this direction; slots of absent cells hold zeros.
constexpr int kFaceVals = 3 * (kTK + kTJ);  // face-buffer values per tile and step
constexpr int kSkewJ = kTJ - 1, kSkewK = kTK - 1;

template <bool FWD, int NE, class T>
struct GridTile {
  static constexpr int NV = FWD ? 27 : 36;
  int nx, ny, lag, nsteps;
  long base;
  bool valid, pollJ, pollK, pubJ, pubK;
  int jj, kk, t, tJ, tK;
  T* faces;

  // tile t_ of an nJ-wide tile grid, seen by lane `lane`
  __device__ __forceinline__ void init(int nx_, int ny_, int nz, int nJ, int t_, int lane, T* faces_) {
    t = t_;
    const int J = t % nJ, K = t / nJ;
    nx = nx_;
    ny = ny_;
    jj = lane & (kTJ - 1);
    kk = lane / kTJ;
    const int j = J * kTJ + jj, k = K * kTK + kk;
    valid = j < ny && k < nz;
    base = valid ? (long)nx * ((long)j + (long)ny * k) : 0;
    lag = FWD ? jj + kk : (kTJ - 1 - jj) + (kTK - 1 - kk);
    nsteps = nx + (kTJ - 1) + (kTK - 1);
    pollJ = valid && (FWD ? (jj == 0 && j > 0) : (jj == kTJ - 1 && j + 1 < ny));
    pollK = valid && (FWD ? (kk == 0 && k > 0) : (kk == kTK - 1 && k + 1 < nz));
    pubJ = valid && (FWD ? jj == kTJ - 1 : jj == 0);
    pubK = valid && (FWD ? kk == kTK - 1 : kk == 0);
    tJ = FWD ? t - 1 : t + 1;    // the tiles whose faces this tile reads
    tK = FWD ? t - nJ : t + nJ;
    faces = faces_;
  }
  __device__ __forceinline__ int cell_i(int step) const { return FWD ? step - lag : nx - 1 - (step - lag); }
  __device__ __forceinline__ bool active(int step) const {
    const int i = cell_i(step);
    return valid && i >= 0 && i < nx;
  }
  // component q of the J-face value of lane (., kk) / K-face value of lane (jj, .)
  __device__ __forceinline__ T* jface(int tile, int step, int q) const {
    return faces + ((size_t)tile * nsteps + step) * kFaceVals + q * kTK + kk;
  }
  __device__ __forceinline__ T* kface(int tile, int step, int q) const {
    return faces + ((size_t)tile * nsteps + step) * kFaceVals + 3 * kTK + q * kTJ + jj;
  }
  __device__ __forceinline__ void poll(int step, Vec3<T>& bj, Vec3<T>& bk) const {
    if (active(step)) {
      if (pollJ) bj = {ld_dev(jface(tJ, step + kSkewJ, 0)), ld_dev(jface(tJ, step + kSkewJ, 1)),
                       ld_dev(jface(tJ, step + kSkewJ, 2))};
      if (pollK) bk = {ld_dev(kface(tK, step + kSkewK, 0)), ld_dev(kface(tK, step + kSkewK, 1)),
                       ld_dev(kface(tK, step + kSkewK, 2))};
    }
  }
  // the value one waiting lane spins on: the last component of a missing face
  __device__ __forceinline__ const T* spin_addr(int step, const Vec3<T>& bj) const {
    return pollJ && sent3(bj) ? jface(tJ, step + kSkewJ, 2) : kface(tK, step + kSkewK, 2);
  }
  __device__ __forceinline__ void publish(int step, T a0, T a1, T a2) const {
    if (pubJ) {
      st_dev(jface(t, step, 0), a0);
      st_dev(jface(t, step, 1), a1);
      st_dev(jface(t, step, 2), a2);
    }
    if (pubK) {
      st_dev(kface(t, step, 0), a0);
      st_dev(kface(t, step, 1), a1);
      st_dev(kface(t, step, 2), a2);
    }
  }
  __device__ __forceinline__ bool ready(int step, const Vec3<T>& bj, const Vec3<T>& bk) const {
    return !(active(step) && ((pollJ && sent3(bj)) || (pollK && sent3(bk))));
  }
};

// j-shift of the systolic array (lane = jj + 16 kk): the j-neighbour is one
// lane over inside a 16-lane row, a DPP row shift in which the row's edge lane
// keeps `old` (the value of the neighbouring tile).
template <bool FWD>
__device__ __forceinline__ double dpp_row_shift(double x, double old) {
  constexpr int ctrl = FWD ? 0x111 : 0x101;  // row_shr:1 / row_shl:1
  const long long xi = __double_as_longlong(x), oi = __double_as_longlong(old);
  const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)xi, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(xi >> 32), ctrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <bool FWD>
__device__ __forceinline__ float dpp_row_shift(float x, float old) {
  constexpr int ctrl = FWD ? 0x111 : 0x101;
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), ctrl, 0xF, 0xF, false));
}
template <bool FWD, class T>
__device__ __forceinline__ Vec3<T> grid_shift_j(const Vec3<T>& x, const Vec3<T>& old) {
  return {dpp_row_shift<FWD>(x.v0, old.v0), dpp_row_shift<FWD>(x.v1, old.v1), dpp_row_shift<FWD>(x.v2, old.v2)};
}

// One lane's place in the sweep and the cell update of a step: m holds the 27
// off-diagonal block values, ui the 9 of U_ii^-1 (backward), r the right-hand
// side (3, then NE values of e0 backward); vj and vk are the values of the two
// other lower (upper) neighbours.
template <bool FWD, int NE, class T>
struct GridCell {
  GridTile<FWD, NE, T> g;
  Vec3<T> prev, last;  // own result one cell earlier / of the last step
  T* yo;            // forward: this tile's last backward-layout row of ytile
  double* z;
  bool has_e0;
  int ea, eb;
  // backward: z goes out in pairs of cells (c, c + 1), c even, as three
  // 16-byte stores (half the lanes storing per step, half the cache lines
  // touched); the odd cell's values wait here for their partner.  Single
  // cells at a pencil's ends, and every cell when z is not 16-byte aligned.
  bool pairs;
  double h0, h1, h2;

  __device__ __forceinline__ void init(int nx, int ny, int nz, int nJ, int t, int lane, T* faces,
                                       T* ytile, const T* e0t, int ea_, int eb_, double* z_) {
    g.init(nx, ny, nz, nJ, t, lane, faces);
    const size_t trow = (size_t)t * g.nsteps;
    yo = FWD ? ytile + (trow + g.nsteps - 1) * 3 * 64 + lane : nullptr;
    z = z_;
    pairs = ((uintptr_t)z_ & 15) == 0;
    h0 = h1 = h2 = 0.0;
    has_e0 = e0t != nullptr;
    ea = ea_;
    eb = eb_;
    prev = last = {T(0), T(0), T(0)};
  }

  __device__ __forceinline__ void update(int s, const Vec3<T>& vj, const Vec3<T>& vk, const T* m,
                                         const T* ui, const T* r) {
    if (!g.active(s)) return;
    T a0 = r[0], a1 = r[1], a2 = r[2];
    mv3_sub(&m[0], prev, a0, a1, a2);
    mv3_sub(&m[9], vj, a0, a1, a2);
    mv3_sub(&m[18], vk, a0, a1, a2);
    const long c = g.base + g.cell_i(s);
    if (FWD) {
      // the backward sweep handles this cell at step nsteps - 1 - s
      T* yw = yo - (size_t)s * 3 * 64;
      yw[0] = a0;
      yw[64] = a1;
      yw[128] = a2;
      g.publish(s, a0, a1, a2);
      prev = {a0, a1, a2};
    } else {
      const T o0 = ui[0] * a0 + ui[1] * a1 + ui[2] * a2;
      const T o1 = ui[3] * a0 + ui[4] * a1 + ui[5] * a2;
      const T o2 = ui[6] * a0 + ui[7] * a1 + ui[8] * a2;
      g.publish(s, o0, o1, o2);
      // z = P_E e0 + x2 in FP64
      const double ex = has_e0 ? (double)r[3] : 0.0;
      const double ey = (NE == 2 && has_e0) ? (double)r[3 + NE - 1] : 0.0;
      const double z0 = (double)o0 + (ea == 0 ? ex : 0.0) + (NE == 2 && eb == 0 ? ey : 0.0);
      const double z1 = (double)o1 + (ea == 1 ? ex : 0.0) + (NE == 2 && eb == 1 ? ey : 0.0);
      const double z2 = (double)o2 + (ea == 2 ? ex : 0.0) + (NE == 2 && eb == 2 ? ey : 0.0);
      const int i = g.cell_i(s);  // the sweep visits i = nx - 1 down to 0
      if (pairs && (c & 1) == 0 && i + 1 < g.nx) {
        double2* q = reinterpret_cast<double2*>(z + 3 * c);  // 48 c bytes: 16-byte aligned
        q[0] = make_double2(z0, z1);
        q[1] = make_double2(z2, h0);
        q[2] = make_double2(h1, h2);
      } else if (pairs && (c & 1) == 1 && i > 0) {
        h0 = z0;
        h1 = z1;
        h2 = z2;
      } else {
        z[3 * c] = z0;
        z[3 * c + 1] = z1;
        z[3 * c + 2] = z2;
      }
      prev = {o0, o1, o2};
    }
    last = prev;
  }
};

// The kernel: one workgroup per tile.  Wave 0 runs the systolic steps and
// reads no global memory; waves 1..H stage each step into a ring of R step
// slots in LDS (wave l takes steps l - 1, l - 1 + H, ...): the matrix data,
// right-hand side and e0 go from HBM to the slot directly, and the values of
// the neighbouring tiles are polled (until the sentinel is gone) and written
// next to them.  So up to R - 1 steps are staged ahead of wave 0, and wave 0's
// own memory traffic is its stores.  Hand-over is through workgroup-scope
// flags with release / acquire fences restricted to LDS:
//   ready[slot] = step     the slot holds that step;
//   consumed = n           wave 0 has read the slots of steps < n.
// A stager of step s first waits for consumed > s - R, wave 0 only waits for
// a step whose slot it has freed, and the polled tiles only wait on tiles
// that started earlier, so nothing waits in a cycle.  Every wait is bounded;
// on failure a wave raises `abort` so the others stop waiting too.
__device__ __forceinline__ int lds_ld(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local"); }
__device__ __forceinline__ void lds_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local"); }

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

// copy of N values of T (N * sizeof(T) a multiple of 256 bytes, 16-byte
// aligned) from global memory straight into LDS by one wave: each instruction
// moves 64 x 16 bytes, the lanes past the end of the last one stay masked.
// The loads are non-temporal (cache policy nt): the staged factors and
// right-hand sides are read once per sweep, and streaming them past the L2
// keeps the face hand-offs' lines there (sweeps 4 % faster).
template <class T, int N>
__device__ __forceinline__ void wave_copy_to_lds(const T* src, T* dst, int lane, bool on = true) {
  constexpr int PL = 16 / (int)sizeof(T);  // values per lane and instruction
  constexpr int PI = 64 * PL;              // values per instruction
  constexpr int kNonTemporal = 2;          // the nt bit of the load's cache policy
#pragma unroll
  for (int q = 0; q < (N + PI - 1) / PI; ++q) {
    if (on && (N % PI == 0 || q * PI + PL * lane < N))
      __builtin_amdgcn_global_load_lds((glb_void*)(src + q * PI + PL * lane), (lds_void*)(dst + q * PI),
                                       16, 0, kNonTemporal);
  }
}

template <bool FWD, int NE, int H, int R, class T>
__global__ __launch_bounds__(64 * (H + 1)) void k_ilu_grid(int nx, int ny, int nz, int nJ, int nK,
                                                               const T* __restrict__ M,
                                                               const T* rhs, T* ytile,
                                                               T* faces,
                                                               const T* __restrict__ e0t,
                                                               int ea, int eb, double* __restrict__ z,
                                                               int* tickets, double* err,
                                                               long spin_limit) {
  constexpr int NV = GridTile<FWD, NE, T>::NV;
  constexpr int NE0 = FWD ? 0 : NE;
  constexpr int NR = 3 + NE0;
  // slot: M (NV), rhs (3), e0 (NE0), polled j and k values (3 + 3); x 64 lanes
  constexpr int OR = NV * 64, OE = (NV + 3) * 64, OF = (NV + NR) * 64;
  constexpr int SLOT = (NV + NR + 6) * 64;
  __shared__ T ring[R * SLOT];
  __shared__ int s_ready[R];
  __shared__ int s_t, s_consumed, s_abort;
  if (threadIdx.x == 0) {
    s_t = __hip_atomic_fetch_add(tickets + (FWD ? 0 : 1), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_consumed = 0;
    s_abort = 0;
  }
  if (threadIdx.x < R) s_ready[threadIdx.x] = -1;
  __syncthreads();
  const int t = FWD ? s_t : nJ * nK - 1 - s_t;
  // the wave index is uniform per wave: keep it (and the stagers' loops) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int wait_limit = (int)min(4 * spin_limit, (long)1 << 30);
  GridCell<FWD, NE, T> w;
  w.init(nx, ny, nz, nJ, t, lane, faces, ytile, e0t, ea, eb, z);
  const GridTile<FWD, NE, T>& g = w.g;
  const int nsteps = g.nsteps;
  const size_t trow = (size_t)t * nsteps;

  // wave 0 runs an even number of steps and reads two slots past them: the
  // stagers fill steps up to nst + 1 (beyond nsteps - 1 with copies of the
  // last step's data, no lane active), so no read is conditional
  const int nst = (nsteps + 1) & ~1;
  if (wave > 0) {
    // stager
    int spin = 0;
    for (int s = wave - 1; s <= nst + 1; s += H) {
      while (lds_ld(&s_consumed) <= s - R) {
        if (lds_ld(&s_abort)) return;
        if (++spin > wait_limit) {
          lds_st(&s_abort, 1);
          if (lane == 0) st_dev(err, 1.0);
          return;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      lds_acquire();
      T* slot = ring + (s % R) * SLOT;
      const size_t row = trow + min(s, nsteps - 1);
      // a load lane moves the values of PL consecutive cell lanes of one row
      // of the tile (the same lanes in every instruction): in FP64 it is
      // skipped when none of them is active at step s (padding pencils, the
      // skew's ramps), whose slot values the sweeping wave never uses (1 %
      // faster; in FP32, four cells per load lane, the masked copies made
      // the sweeps slower, also with the test reduced to two comparisons)
      bool on = true;
      if constexpr (sizeof(T) == 8) {
        constexpr int PL = 16 / (int)sizeof(T);
        const int c0 = PL * (lane % (64 / PL));
        const int kk = c0 / kTJ, k = (t / nJ) * kTK + kk;
        on = false;
#pragma unroll
        for (int u = 0; u < PL; ++u) {
          const int jj = (c0 + u) % kTJ, j = (t % nJ) * kTJ + jj;
          const int lag = FWD ? jj + kk : (kTJ - 1 - jj) + (kTK - 1 - kk);
          on = on || (j < ny && k < nz && s >= lag && s < lag + nx);
        }
      }
      wave_copy_to_lds<T, NV * 64>(M + row * NV * 64, slot, lane, on);
      wave_copy_to_lds<T, 3 * 64>(rhs + row * 3 * 64, slot + OR, lane, on);
      // without e0 (M2^-1 alone) the slot's e0 part is left as it is: unused
      if (!FWD && e0t) wave_copy_to_lds<T, NE0 * 64>(e0t + row * NE0 * 64, slot + OE, lane, on);
      // values of the neighbouring tiles, once published.  All face values a
      // step needs from one neighbour come from one step of that tile, so
      // while they are missing a single lane waits on one of them and the
      // whole face is read again once it is there.
      Vec3<T> bj = {T(0), T(0), T(0)}, bk = bj;
      bool need = g.active(s) && (g.pollJ || g.pollK);
      for (;;) {
        if (need) {
          g.poll(s, bj, bk);
          need = !g.ready(s, bj, bk);
        }
        const unsigned long long waiting = __ballot(need);
        if (!waiting) break;
        const int leader = __builtin_ctzll(waiting);
        for (;;) {
          if (lds_ld(&s_abort)) return;
          if (++spin > wait_limit) {
            lds_st(&s_abort, 1);
            if (lane == 0) st_dev(err, 1.0);
            return;
          }
          __builtin_amdgcn_s_sleep(2);
          bool there = true;
          if (lane == leader) {
            there = !is_sent(ld_dev(g.spin_addr(s, bj)));
          }
          if (__all(there)) break;
        }
      }
      T* f = slot + OF + lane;
      f[0] = bj.v0;
      f[64] = bj.v1;
      f[128] = bj.v2;
      f[192] = bk.v0;
      f[256] = bk.v1;
      f[320] = bk.v2;
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the copies have landed in LDS
      lds_release();
      lds_st(&s_ready[s % R], s);
    }
    return;
  }

  // wave 0: the systolic sweep.  A step first sends its k-shift through the
  // LDS crossbar, then issues the reads of the next step's slot and the ready
  // flag of the step after it, and computes while they are in flight; the
  // j-shift is a DPP move whose edge lanes keep the polled value.
  T ma[NV], mb[NV], ra[NR], rb[NR];
  Vec3<T> ja, ka, jb, kb;
  const bool kedge = FWD ? g.kk == 0 : g.kk == kTK - 1;
  auto wait_ready = [&](int s) __attribute__((always_inline)) -> bool {
    const int slot = s % R;
    int sp = 0;
    while (lds_ld(&s_ready[slot]) != s) {
      if (lds_ld(&s_abort) || ++sp > wait_limit) return false;
      __builtin_amdgcn_s_sleep(1);
    }
    return true;
  };
  // (the caller has seen the ready flag of step s and fenced)
  auto read = [&](T* m, T* r, Vec3<T>& bj, Vec3<T>& bk, int s) __attribute__((always_inline)) {
    const T* sl = ring + (s % R) * SLOT + lane;
#pragma unroll
    for (int e = 0; e < NV; ++e) m[e] = sl[e * 64];
#pragma unroll
    for (int q = 0; q < NR; ++q) r[q] = sl[OR + q * 64];
    bj = {sl[OF], sl[OF + 64], sl[OF + 128]};
    bk = {sl[OF + 192], sl[OF + 256], sl[OF + 320]};
  };
  auto consumed = [&](int n) __attribute__((always_inline)) {
    lds_release();
    lds_st(&s_consumed, n);
  };
  // step s on (m, r, bj, bk) while the slot of step s + 1 is read into
  // (mn, rn, bjn, bkn); returns the ready flag of step s + 2
  auto step = [&](int s, const T* m, const T* r, const Vec3<T>& bj, const Vec3<T>& bk, T* mn,
                  T* rn, Vec3<T>& bjn, Vec3<T>& bkn) __attribute__((always_inline)) -> int {
    const Vec3<T> fk = FWD ? shfl_up3(w.last, kTJ) : shfl_down3(w.last, kTJ);
    __builtin_amdgcn_sched_barrier(0);
    read(mn, rn, bjn, bkn, s + 1);
    const int f = lds_ld(&s_ready[(s + 2) % R]);
    __builtin_amdgcn_sched_barrier(0);
    const Vec3<T> vj = grid_shift_j<FWD>(w.last, bj);
    w.update(s, vj, kedge ? bk : fk, m, m + 27, r);
    consumed(s + 1);
    return f;
  };
  bool ok = wait_ready(0);
  if (ok) {
    lds_acquire();
    read(ma, ra, ja, ka, 0);
    ok = wait_ready(1);
    lds_acquire();
  }
  for (int s = 0; ok && s < nst; s += 2) {
    int f = step(s, ma, ra, ja, ka, mb, rb, jb, kb);
    if (f != s + 2 && !(ok = wait_ready(s + 2))) break;
    lds_acquire();
    f = step(s + 1, mb, rb, jb, kb, ma, ra, ja, ka);
    if (f != s + 3 && !(ok = wait_ready(s + 3))) break;
    lds_acquire();
  }
  if (!ok) {
    lds_st(&s_abort, 1);
    if (lane == 0) st_dev(err, 1.0);
  }
}

// A P_E e0 on one SELL-64 row: only the elliptic columns ea (and eb) of each
// block are read, slots in chunks of CH whose loads all go out before the
// chunk's first product (slot clamped to the slice's last, surplus products
// dropped; entry order kept).  A is read once per product: non-temporal loads.
// HOLD keeps all of a chunk's loads in flight at the cost of occupancy (the
// compiler otherwise trades them for more waves); which is faster was
// measured per kernel and type.
template <int NE, int CH, bool HOLD, class T>
__device__ __forceinline__ void stage2_row_sum(int k0, int k1, int lane, const int32_t* __restrict__ col,
                                               const double* __restrict__ val, int ea, int eb,
                                               const T* __restrict__ e0, double& a0, double& a1,
                                               double& a2) {
  for (int kb = k0; kb < k1; kb += CH) {
    int cc[CH];
    double m[CH][6];
    T uu[CH][2];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const size_t kq = (size_t)min(kb + q, k1 - 1);
      cc[q] = __builtin_nontemporal_load(col + kq * 64 + lane);
      const double* v = val + kq * 9 * 64 + lane;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        m[q][a] = __builtin_nontemporal_load(v + (a * 3 + ea) * 64);
        if (NE == 2) m[q][3 + a] = __builtin_nontemporal_load(v + (a * 3 + eb) * 64);
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      uu[q][0] = e0[(size_t)cc[q] * NE];
      if (NE == 2) uu[q][1] = e0[(size_t)cc[q] * NE + 1];
    }
    if (HOLD) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (kb + q < k1) {
        const double u = uu[q][0];
        a0 += m[q][0] * u;
        a1 += m[q][1] * u;
        a2 += m[q][2] * u;
        if (NE == 2) {
          const double w = uu[q][1];
          a0 += m[q][3] * w;
          a1 += m[q][4] * w;
          a2 += m[q][5] * w;
        }
      }
  }
}

// stage-two residual for the grid sweeps: r2 and e0 are also written in the
// tile layouts (r2 forward, e0 backward), the face buffers of both sweeps
// (nfaces values) get the sentinel, and both ticket counters := 0
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_stage2_grid(int nx, int ny, int nz, int nrows, int nblk,
                                                        const int32_t* __restrict__ sptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, int ea,
                                                        int eb, const T* __restrict__ e0,
                                                        const double* __restrict__ r,
                                                        T* __restrict__ r2t,
                                                        T* __restrict__ e0t,
                                                        T* __restrict__ faces, int64_t nfaces,
                                                        int* tickets) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    tickets[0] = 0;
    tickets[1] = 0;
  }
  {
    const T s0 = sentinel_value<T>();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nfaces; q += stride) faces[q] = s0;
  }
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= nrows) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (e0) {
    const int s = row >> 6, lane = row & 63;
    stage2_row_sum<NE, 8, sizeof(T) == 8>(sptr[s], sptr[s + 1], lane, col, val, ea, eb, e0, a0, a1, a2);
  }
  const int i = row % nx, jg = (row / nx) % ny, kg = row / (nx * ny);
  const int nJ = (ny + kTJ - 1) / kTJ;
  const int J = jg / kTJ, jj = jg % kTJ, K = kg / kTK, kk = kg % kTK;
  const size_t t = (size_t)J + (size_t)nJ * K;
  const int ns = nx + (kTJ - 1) + (kTK - 1);
  const int lane = jj + kTJ * kk;
  const size_t frow = t * ns + (i + jj + kk);
  const size_t brow = t * ns + ((nx - 1 - i) + (kTJ - 1 - jj) + (kTK - 1 - kk));
  const double* ri = r + 3 * (size_t)row;
  T* o = r2t + frow * 3 * 64 + lane;
  o[0] = (T)(ri[0] - a0);
  o[64] = (T)(ri[1] - a1);
  o[128] = (T)(ri[2] - a2);
  if (e0) {
    T* eo = e0t + brow * NE * 64 + lane;
    eo[0] = e0[(size_t)row * NE];
    if (NE == 2) eo[64] = e0[(size_t)row * NE + 1];
  }
  (void)nz;
}

// stage-two residual that also prepares the one-launch sweeps: y, x2 :=
// sentinel and both ticket counters := 0
template <int NE, class T>
__global__ __launch_bounds__(kBlock) void k_stage2_resid_sf(int nrows, int nblk, const int32_t* __restrict__ sptr,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ val, int ea,
                                                            int eb, const T* __restrict__ e0,
                                                            const double* __restrict__ r,
                                                            T* __restrict__ r2,
                                                            T* __restrict__ y,
                                                            T* __restrict__ x2, int* tickets) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    tickets[0] = 0;
    tickets[1] = 0;
  }
  const int row = xcd_block(blockIdx.x, nblk) * kBlock + threadIdx.x;
  if (row >= nrows) return;
  const int s = row >> 6, lane = row & 63;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  // without e0 (M2^-1 alone) this only converts r to T
  if (e0) stage2_row_sum<NE, 4, true>(sptr[s], sptr[s + 1], lane, col, val, ea, eb, e0, a0, a1, a2);
  const double* ri = r + 3 * (size_t)row;
  T* o = r2 + 3 * (size_t)row;
  o[0] = (T)(ri[0] - a0);
  o[1] = (T)(ri[1] - a1);
  o[2] = (T)(ri[2] - a2);
  const T s0 = sentinel_value<T>();
  y[3 * (size_t)row] = s0;
  y[3 * (size_t)row + 1] = s0;
  y[3 * (size_t)row + 2] = s0;
  x2[3 * (size_t)row] = s0;
  x2[3 * (size_t)row + 1] = s0;
  x2[3 * (size_t)row + 2] = s0;
}

// --------------------------------------------------------------------------
// Arnoldi BLAS-1.  part[blk * ncol + j] holds each workgroup's partial sums.
template <int MAXV>
__device__ __forceinline__ void block_store(const double* acc, int nv, double* part, int ncol) {
  __shared__ double red[kBlock / 64][MAXV + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < MAXV + 1; ++j) {
    if (j < ncol) {
      const double v = wave_sum(acc[j]);
      if (lane == 0) red[wave][j] = v;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ncol; j += kBlock) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][j];
    part[(size_t)blockIdx.x * ncol + j] = s;
  }
  (void)nv;
}

// Element i of basis columns jb .. jb+G-1, with columns past the first nv read
// as column nv-1 (always present: nv >= 1).  The group's loads are issued
// together, with no branch between them to wait at.  The callers give the
// extra columns zero coefficients and drop their sums, so the results equal
// those of a loop over the nv columns alone.  Kernels with MAXV <= 8 are
// launched with nv == MAXV (one group, no extra column); larger ones read
// groups of 8.
template <int MAXV>
constexpr int col_group() { return MAXV < 8 ? MAXV : 8; }
template <int G>
__device__ __forceinline__ void load_cols(const double* __restrict__ V, int64_t ldv, int nv, int jb, int64_t i,
                                          double* v) {
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int j = jb + q < nv ? jb + q : nv - 1;
    v[q] = V[(size_t)j * ldv + i];
  }
  // keep the scheduler from interleaving the group's loads with their uses
  // (it otherwise issues some of them one at a time, each waited for)
  __builtin_amdgcn_sched_barrier(0);
}

template <int MAXV>
__global__ __launch_bounds__(kBlock) void k_mdot(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ w, double* __restrict__ part) {
  double acc[MAXV + 1];
#pragma unroll
  for (int j = 0; j <= MAXV; ++j) acc[j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double wi = w[i];
#pragma unroll
    for (int jb = 0; jb < MAXV; jb += col_group<MAXV>())
      if (jb < nv) {
        double v[col_group<MAXV>()];
        load_cols<col_group<MAXV>()>(V, ldv, nv, jb, i, v);
#pragma unroll
        for (int q = 0; q < col_group<MAXV>(); ++q) acc[jb + q] += v[q] * wi;
      }
  }
  block_store<MAXV>(acc, nv, part, nv);
}

// w -= sum_j coef_j V_j, then partial dots V_j . w (second Gram-Schmidt pass)
template <int MAXV>
__global__ __launch_bounds__(kBlock) void k_maxpy_dot(int64_t n, int nv, const double* __restrict__ V,
                                                      int64_t ldv, const double* __restrict__ coef,
                                                      double* __restrict__ w, double* __restrict__ part) {
  double acc[MAXV + 1];
  double c[MAXV];
#pragma unroll
  for (int j = 0; j <= MAXV; ++j) acc[j] = 0.0;
#pragma unroll
  for (int j = 0; j < MAXV; ++j) c[j] = j < nv ? coef[j] : 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double wi = w[i];
#pragma unroll
    for (int jb = 0; jb < MAXV; jb += col_group<MAXV>())
      if (jb < nv) {
        double v[col_group<MAXV>()];
        load_cols<col_group<MAXV>()>(V, ldv, nv, jb, i, v);
#pragma unroll
        for (int q = 0; q < col_group<MAXV>(); ++q) wi -= c[jb + q] * v[q];
      }
    w[i] = wi;
#pragma unroll
    for (int jb = 0; jb < MAXV; jb += col_group<MAXV>())
      if (jb < nv) {
        double v[col_group<MAXV>()];
        load_cols<col_group<MAXV>()>(V, ldv, nv, jb, i, v);
#pragma unroll
        for (int q = 0; q < col_group<MAXV>(); ++q) acc[jb + q] += v[q] * wi;
      }
  }
  block_store<MAXV>(acc, nv, part, nv);
}

// w -= sum_j coef_j V_j, then the partial squared norm of w
template <int MAXV>
__global__ __launch_bounds__(kBlock) void k_maxpy_norm(int64_t n, int nv, const double* __restrict__ V,
                                                       int64_t ldv, const double* __restrict__ coef,
                                                       double* __restrict__ w, double* __restrict__ part) {
  double c[MAXV];
#pragma unroll
  for (int j = 0; j < MAXV; ++j) c[j] = j < nv ? coef[j] : 0.0;
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double wi = w[i];
#pragma unroll
    for (int jb = 0; jb < MAXV; jb += col_group<MAXV>())
      if (jb < nv) {
        double v[col_group<MAXV>()];
        load_cols<col_group<MAXV>()>(V, ldv, nv, jb, i, v);
#pragma unroll
        for (int q = 0; q < col_group<MAXV>(); ++q) wi -= c[jb + q] * v[q];
      }
    w[i] = wi;
    acc[0] += wi * wi;
  }
  block_store<0>(acc, 1, part, 1);
}

__global__ __launch_bounds__(kBlock) void k_norm2(int64_t n, const double* __restrict__ x,
                                                  double* __restrict__ part) {
  double acc[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) acc[0] += x[i] * x[i];
  block_store<0>(acc, 1, part, 1);
}

// out[j] (+)= sum over workgroups of part[b * ncol + j], fixed tree order
__global__ __launch_bounds__(kBlock) void k_reduce(int ncol, const double* __restrict__ part,
                                                   double* __restrict__ out, int add) {
  __shared__ double red[kBlock];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < kRedBlocks; b += kBlock) s += part[(size_t)b * ncol + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = add ? out[j] + red[0] : red[0];
}

// in place allowed (w == v)
__global__ __launch_bounds__(kBlock) void k_scale(int64_t n, const double* w, const double* nrm2, double* v) {
  const double h = sqrt(nrm2[0]);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) v[i] = w[i] / h;
}

__global__ __launch_bounds__(kBlock) void k_scale_host(int64_t n, const double* __restrict__ w, double s,
                                                       double* __restrict__ v) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) v[i] = w[i] / s;
}

struct Coef64 {
  double c[64];
};

// x += sum_j coef_j V_j (coefficients past nv are zero)
template <int MAXV>
__global__ __launch_bounds__(kBlock) void k_update(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                   Coef64 coef, double* __restrict__ x) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double s = x[i];
#pragma unroll
    for (int jb = 0; jb < MAXV; jb += col_group<MAXV>())
      if (jb < nv) {
        double v[col_group<MAXV>()];
        load_cols<col_group<MAXV>()>(V, ldv, nv, jb, i, v);
#pragma unroll
        for (int q = 0; q < col_group<MAXV>(); ++q) s += coef.c[jb + q] * v[q];
      }
    x[i] = s;
  }
}

}  // namespace

// ============================================================================
// launchers
void launch_bsr3_spmv(const Sell& A, const double* x, const double* b, double* y, bool resid,
                      hipStream_t st) {
  const int g = nblocks(A.nrows, kBlock);
  if (resid)
    k_bsr3_spmv<true><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, x, b, y);
  else
    k_bsr3_spmv<false><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, x, b, y);
}

template <class T>
void launch_l0_restrict(int32_t nc, int ne, const double* r, const double* W, const int32_t* eidx,
                        const int32_t* hidx, T* b0, const T* dinv, T* x0, hipStream_t st) {
  const int g = nblocks(nc, kBlock);
  if (ne == 2)
    k_l0_restrict<2, T><<<g, kBlock, 0, st>>>(nc, r, W, eidx[0], eidx[1], hidx[0], 0, b0, dinv, x0);
  else
    k_l0_restrict<1, T><<<g, kBlock, 0, st>>>(nc, r, W, eidx[0], 0, hidx[0], hidx[1], b0, dinv, x0);
}

template <class T>
void launch_l0_resid(const SellT<T>& Ah, int ne, const T* x0, const T* b0, T* r0, hipStream_t st) {
  const int g = nblocks(Ah.nrows, kBlock);
  if (ne == 2)
    k_l0_resid<2, T><<<g, kBlock, 0, st>>>(Ah.nrows, g, Ah.sptr, Ah.col, Ah.val, x0, b0, r0);
  else
    k_l0_resid<1, T><<<g, kBlock, 0, st>>>(Ah.nrows, g, Ah.sptr, Ah.col, Ah.val, x0, b0, r0);
}

template <class T>
void launch_l0_post(const SellT<T>& Ah, int ne, const T* x0, const T* b0, const T* dinv, T* e0,
                    hipStream_t st) {
  const int g = nblocks(Ah.nrows, kBlock);
  if (ne == 2)
    k_l0_post<2, T><<<g, kBlock, 0, st>>>(Ah.nrows, g, Ah.sptr, Ah.col, Ah.val, x0, b0, dinv, e0);
  else
    k_l0_post<1, T><<<g, kBlock, 0, st>>>(Ah.nrows, g, Ah.sptr, Ah.col, Ah.val, x0, b0, dinv, e0);
}

template <class T>
void launch_csr_resid(const DCsrT<T>& A, const T* x0, const T* b, T* r, hipStream_t st) {
  launch_csr_op<kResid, T>(A, x0, b, nullptr, r, st);
}
template <class T>
void launch_csr_spmv(const DCsrT<T>& A, const T* x, T* y, hipStream_t st) {
  launch_csr_op<kSpmv, T>(A, x, nullptr, nullptr, y, st);
}
template <class T>
void launch_csr_restrict(const DCsrT<T>& R, const T* r, const T* dinv_c, T* bc, T* xc, hipStream_t st) {
  launch_csr_op<kRestrict, T>(R, r, nullptr, dinv_c, bc, st, xc);
}
template <class T>
void launch_csr_prolong(const DCsrT<T>& P, const T* xc, const T* b, const T* dinv, T* x,
                        hipStream_t st) {
  launch_csr_op<kProlong, T>(P, xc, b, dinv, x, st);
}
template <class T>
void launch_csr_prolong_add(const DCsrT<T>& P, const T* xc, const T* x, T* y, hipStream_t st) {
  launch_csr_op<kProlongAdd, T>(P, xc, x, nullptr, y, st);
}
template <class T>
void launch_csr_post(const DCsrT<T>& A, const T* x, const T* b, const T* dinv, T* e, hipStream_t st) {
  launch_csr_op<kPost, T>(A, x, b, dinv, e, st);
}
template <class T>
void launch_sell_resid(const SellT<T>& A, const T* x0, const T* b, T* r, hipStream_t st) {
  if (A.nrows == 0) return;
  const int g = nblocks(A.nrows, kBlock);
  k_sell_scalar<kResid, T><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, x0, b, nullptr, r);
}
template <class T>
void launch_sell_post(const SellT<T>& A, const T* x, const T* b, const T* dinv, T* e, hipStream_t st) {
  if (A.nrows == 0) return;
  const int g = nblocks(A.nrows, kBlock);
  k_sell_scalar<kPost, T><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, x, b, dinv, e);
}

template <class T>
void launch_coarse_solve(int n, const double* lu, const int32_t* piv, const T* b, T* x,
                         hipStream_t st) {
  k_coarse_solve<T><<<1, kBlock, sizeof(double) * (size_t)n, st>>>(n, lu, piv, b, x);
}

template <class T>
void launch_blk_csr(int op, int nrows, int w, const DCsrT<T>* S, const T* dinv, const double* z,
                    const double* x, double* y, hipStream_t st) {
  if (nrows <= 0 || w <= 0) return;
  const dim3 g(nblocks(w, kBlock), nrows);
  const int32_t* rp = S ? S->rp : nullptr;
  const int32_t* ci = S ? S->ci : nullptr;
  const T* v = S ? S->v : nullptr;
  switch (op) {
    case kBlkScale: k_blk_csr<kBlkScale, T><<<g, kBlock, 0, st>>>(w, rp, ci, v, dinv, z, x, y); break;
    case kBlkResid: k_blk_csr<kBlkResid, T><<<g, kBlock, 0, st>>>(w, rp, ci, v, dinv, z, x, y); break;
    case kBlkJacobi: k_blk_csr<kBlkJacobi, T><<<g, kBlock, 0, st>>>(w, rp, ci, v, dinv, z, x, y); break;
    case kBlkProduct: k_blk_csr<kBlkProduct, T><<<g, kBlock, 0, st>>>(w, rp, ci, v, dinv, z, x, y); break;
    case kBlkAdd: k_blk_csr<kBlkAdd, T><<<g, kBlock, 0, st>>>(w, rp, ci, v, dinv, z, x, y); break;
  }
}
void launch_blk_lu(int n, int w, const double* lu, const int32_t* piv, double* x, hipStream_t st) {
  if (n > 0 && w > 0) k_blk_lu<<<nblocks(w, kBlock), kBlock, 0, st>>>(n, w, lu, piv, x);
}
void launch_blk_identity(int n, double* x, hipStream_t st) {
  if (n > 0) k_blk_identity<<<nblocks((int64_t)n * n, kBlock), kBlock, 0, st>>>(n, x);
}
template <class T>
void launch_blk_to(int64_t m, const double* x, T* y, hipStream_t st) {
  if (m > 0) k_blk_to<T><<<nblocks(m, kBlock), kBlock, 0, st>>>(m, x, y);
}
template <class T>
void launch_dense_gemv(int n, const T* B, const T* b, T* e, hipStream_t st) {
  if (n <= 0) return;
  if (n <= kBlock) k_dense_gemv<1, T><<<n, kBlock, 0, st>>>(n, B, b, e);
  else if (n <= 2 * kBlock) k_dense_gemv<2, T><<<n, kBlock, 0, st>>>(n, B, b, e);
  else if (n <= 4 * kBlock) k_dense_gemv<4, T><<<n, kBlock, 0, st>>>(n, B, b, e);
  else if (n <= 8 * kBlock) k_dense_gemv<8, T><<<n, kBlock, 0, st>>>(n, B, b, e);
  else k_dense_gemv<16, T><<<n, kBlock, 0, st>>>(n, B, b, e);  // n <= 4096 (dense_tail)
}

template <class T>
void launch_stage2_resid(const Sell& A, int ne, const int32_t* eidx, const T* e0, const double* r,
                         T* r2, hipStream_t st) {
  const int g = nblocks(A.nrows, kBlock);
  if (ne == 2)
    k_stage2_resid<2, T><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, eidx[0], eidx[1], e0, r, r2);
  else
    k_stage2_resid<1, T><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, eidx[0], 0, e0, r, r2);
}

template <class T>
void launch_ilu_fwd_level(const SellT<T>& L, const int32_t* perm, int32_t p0, int32_t p1, const T* r2,
                          T* y, hipStream_t st) {
  if (p1 <= p0) return;
  k_ilu_fwd<T><<<nblocks(p1 - p0, kBlock), kBlock, 0, st>>>(p0, p1, L.sptr, L.col, L.val, perm, r2, y);
}

template <class T>
void launch_ilu_bwd_level(const SellT<T>& U, const int32_t* perm, const T* uinv, int32_t p0,
                          int32_t p1, const T* y, const T* e0, int ne, const int32_t* eidx, T* x2,
                          double* z, hipStream_t st) {
  if (p1 <= p0) return;
  const int npad = U.nslices * 64;
  const int g = nblocks(p1 - p0, kBlock);
  if (ne == 2)
    k_ilu_bwd<2, T><<<g, kBlock, 0, st>>>(p0, p1, npad, U.sptr, U.col, U.val, perm, uinv, y, e0,
                                          eidx[0], eidx[1], x2, z);
  else
    k_ilu_bwd<1, T><<<g, kBlock, 0, st>>>(p0, p1, npad, U.sptr, U.col, U.val, perm, uinv, y, e0,
                                          eidx[0], 0, x2, z);
}


template <class T>
void launch_stage2_resid_sf(const Sell& A, int ne, const int32_t* eidx, const T* e0,
                            const double* r, T* r2, T* y, T* x2, int* tickets, hipStream_t st) {
  const int g = nblocks(A.nrows, kBlock);
  if (ne == 2)
    k_stage2_resid_sf<2, T><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, eidx[0], eidx[1], e0, r, r2, y, x2, tickets);
  else
    k_stage2_resid_sf<1, T><<<g, kBlock, 0, st>>>(A.nrows, g, A.sptr, A.col, A.val, eidx[0], 0, e0, r, r2, y, x2, tickets);
}


template <class T>
void launch_prolong_e(int32_t nrows, int ne, const int32_t* eidx, const T* e0, double* x1,
                      hipStream_t st) {
  const int g = nblocks(nrows, kBlock);
  if (ne == 2) k_prolong_e<2, T><<<g, kBlock, 0, st>>>(nrows, e0, eidx[0], eidx[1], x1);
  else k_prolong_e<1, T><<<g, kBlock, 0, st>>>(nrows, e0, eidx[0], 0, x1);
}
void launch_sweep_prepare(int64_t n, double* y, double* x2, int* tickets, hipStream_t st) {
  k_sweep_prepare<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, y, x2, tickets);
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, double* __restrict__ x, double v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = v;
}
void launch_fill(int64_t n, double* x, double v, hipStream_t st) {
  if (n > 0) k_fill<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, x, v);
}


int64_t grid_face_values(int nx, int ny, int nz) {
  return grid_ntiles(ny, nz) * grid_nsteps(nx) * kFaceVals;
}

template <class T>
void launch_stage2_grid(int nx, int ny, int nz, const Sell& A, int ne, const int32_t* eidx, const T* e0,
                        const double* r, T* r2t, T* e0t, T* faces, int* tickets, hipStream_t st) {
  const int g = nblocks(A.nrows, kBlock);
  const int64_t nfaces = 2 * grid_face_values(nx, ny, nz);
  if (ne == 2)
    k_stage2_grid<2, T><<<g, kBlock, 0, st>>>(nx, ny, nz, A.nrows, g, A.sptr, A.col, A.val, eidx[0],
                                              eidx[1], e0, r, r2t, e0t, faces, nfaces, tickets);
  else
    k_stage2_grid<1, T><<<g, kBlock, 0, st>>>(nx, ny, nz, A.nrows, g, A.sptr, A.col, A.val, eidx[0], 0,
                                              e0, r, r2t, e0t, faces, nfaces, tickets);
}

// --------------------------------------------------------------------------
// Block ILU(0) of a 7-point stencil in lexicographic order (Sec. 3.1).  On this
// pattern the elimination has no fill and touches only diagonal blocks: a lower
// neighbour k of cell c (c - nx*ny, c - nx, c - 1) contributes L_ck = A_ck
// U_kk^-1 and U_cc = A_cc - sum_k L_ck A_kc (k in increasing column order), the
// blocks right of the diagonal are A's own.
// (no FP contraction in these two: they round like the host factorisation's)
__device__ __forceinline__ void mm3_dev(const double* a, const double* b, double* c) {
#pragma clang fp contract(off)
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) s += a[r * 3 + q] * b[q * 3 + k];
      c[r * 3 + k] = s;
    }
}
// 3x3 inverse by Gauss-Jordan with partial pivoting; false for a zero pivot
__device__ __forceinline__ bool inv3_dev(const double* m, double* out) {
#pragma clang fp contract(off)
  double a[3][6];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 6; ++c) a[r][c] = c < 3 ? m[r * 3 + c] : (c - 3 == r ? 1.0 : 0.0);
  for (int k = 0; k < 3; ++k) {
    int p = k;
    for (int r = k + 1; r < 3; ++r)
      if (fabs(a[r][k]) > fabs(a[p][k])) p = r;
    if (a[p][k] == 0.0) return false;
    if (p != k)
      for (int c = 0; c < 6; ++c) {
        const double t = a[k][c];
        a[k][c] = a[p][c];
        a[p][c] = t;
      }
    const double d = a[k][k];
    for (int c = 0; c < 6; ++c) a[k][c] /= d;
    for (int r = 0; r < 3; ++r)
      if (r != k) {
        const double f = a[r][k];
        for (int c = 0; c < 6; ++c) a[r][c] -= f * a[k][c];
      }
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) out[r * 3 + c] = a[r][c + 3];
  return true;
}

__global__ __launch_bounds__(kBlock) void k_grid_ilu_diag(int p0, int p1, const int32_t* __restrict__ perm,
                                                          const int32_t* __restrict__ sptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val, int nx, int nxy,
                                                          double* __restrict__ uinv, int* bad) {
  const int p = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (p >= p1) return;
  const int c = perm[p];
  const int ny = nxy / nx;
  // A's pattern is the 7-point stencil in sorted column order, so a row's
  // slot of each neighbour follows from which of its neighbours exist: the
  // blocks are read directly instead of searching the row's columns
  auto slot = [&](int r, int d) -> size_t {  // slot in row r of column r + d
    const int xr = r % nx, yr = (r / nx) % ny, zr = r / nxy;
    int k = 0;
    if (d > -nxy) k += zr > 0;
    if (d > -nx) k += yr > 0;
    if (d > -1) k += xr > 0;
    if (d > 0) k += 1;
    if (d > 1) k += xr < nx - 1;
    if (d > nx) k += yr < ny - 1;
    return (size_t)sptr[r >> 6] + k;
  };
  auto block_at = [&](int r, size_t q, double* out) {
#pragma unroll
    for (int e = 0; e < 9; ++e) out[e] = val[(q * 9 + e) * 64 + (r & 63)];
  };
  double D[9];
  block_at(c, slot(c, 0), D);
  const int x = c % nx, y = (c / nx) % ny, z = c / nxy;
  const int dl[3] = {nxy, nx, 1};  // lower neighbours in increasing column order
  const bool has[3] = {z > 0, y > 0, x > 0};
  for (int q = 0; q < 3; ++q) {
    if (!has[q]) continue;
    const int k = c - dl[q];
    double Ack[9], Akc[9], Lq[9], prod[9];
    block_at(c, slot(c, -dl[q]), Ack);
    bool present = false;
#pragma unroll
    for (int e = 0; e < 9; ++e) present |= Ack[e] != 0.0;
    if (!present) continue;
    mm3_dev(Ack, uinv + (size_t)k * 9, Lq);
    block_at(k, slot(k, dl[q]), Akc);
    mm3_dev(Lq, Akc, prod);
#pragma unroll
    for (int e = 0; e < 9; ++e) D[e] -= prod[e];
  }
  double inv[9];
  if (!inv3_dev(D, inv)) {
#pragma unroll
    for (int e = 0; e < 9; ++e) inv[e] = 0.0;
    atomicMin(bad, c);
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) uinv[(size_t)c * 9 + e] = inv[e];
}

// tile layouts of the grid sweeps: L_ck = A_ck U_kk^-1 (forward, slots -x, -y,
// -z), A_ck (backward, slots +x, +y, +z) and U_cc^-1 (backward, values 27..35)
template <class T>
__global__ __launch_bounds__(kBlock) void k_grid_ilu_pack(int nb, int nx, int ny, const int32_t* __restrict__ sptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ uinv, T* __restrict__ Lt,
                                                          T* __restrict__ Ut) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= nb) return;
  const int nxy = nx * ny;
  const int i = c % nx, j = (c / nx) % ny, k = c / nxy;
  int64_t fr, br;
  int lane;
  grid_tile_slot(nx, ny, i, j, k, fr, br, lane);
  const int s = c >> 6, sl = c & 63;
  for (int q = sptr[s]; q < sptr[s + 1]; ++q) {
    const int cc = col[(size_t)q * 64 + sl];
    const int d = cc - c;
    double blk[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) blk[e] = val[((size_t)q * 9 + e) * 64 + sl];
    if (d == -1 || d == -nx || d == -nxy) {
      const int slot = d == -1 ? 0 : d == -nx ? 1 : 2;
      double Lq[9];
      mm3_dev(blk, uinv + (size_t)cc * 9, Lq);
#pragma unroll
      for (int e = 0; e < 9; ++e) Lt[((size_t)fr * 27 + 9 * slot + e) * 64 + lane] = (T)Lq[e];
    } else if (d == 1 || d == nx || d == nxy) {
      const int slot = d == 1 ? 0 : d == nx ? 1 : 2;
#pragma unroll
      for (int e = 0; e < 9; ++e) Ut[((size_t)br * 36 + 9 * slot + e) * 64 + lane] = (T)blk[e];
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) Ut[((size_t)br * 36 + 27 + e) * 64 + lane] = (T)uinv[(size_t)c * 9 + e];
}

// Strength of connection of one AMG level, one thread per row, in the host
// construction's order and rounding: j (j != i, of i's unknown type) is a
// strong dependency of i when -sign(a_ii) a_ij >= theta * max over same-type
// k != i of (-sign(a_ii) a_ik); none when that maximum is not positive or
// the same-type row sum exceeds mrs |a_ii| (mrs < 1).  Row i's strong columns
// go to ocol at arp[i] (A's own row offsets), their count to cnt[i].
__global__ __launch_bounds__(kBlock) void k_strength(int n, const int32_t* __restrict__ arp,
                                                     const int32_t* __restrict__ aci,
                                                     const double* __restrict__ av,
                                                     const int32_t* __restrict__ func, double theta, double mrs,
                                                     int32_t* __restrict__ ocol, int32_t* __restrict__ cnt) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int b = arp[i], e = arp[i + 1];
  double aii = 0.0;
  for (int k = b; k < e; ++k)
    if (aci[k] == i) aii = av[k];
  const double sg = aii < 0.0 ? -1.0 : 1.0;
  double sum = 0.0, best = 0.0;
  bool any = false;
  const int32_t fi = func[i];
  for (int k = b; k < e; ++k) {
    const int32_t j = aci[k];
    if (func[j] != fi) continue;
    sum = sum + av[k];
    if (j != i) {
      const double t = -sg * av[k];
      best = any ? (best < t ? t : best) : t;
      any = true;
    }
  }
  int c = 0;
  if (any && best > 0.0 && !(mrs < 1.0 && fabs(sum) > mrs * fabs(aii))) {
    const double cut = theta * best;
    for (int k = b; k < e; ++k) {
      const int32_t j = aci[k];
      if (j != i && func[j] == fi && -sg * av[k] >= cut) ocol[b + c++] = j;
    }
  }
  cnt[i] = c;
}

void launch_strength(int n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* func,
                     double theta, double mrs, int32_t* ocol, int32_t* cnt, hipStream_t st) {
  if (n > 0) k_strength<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, arp, aci, av, func, theta, mrs, ocol, cnt);
}

// the entries of each row from their padded places (off) to CSR order (rp),
// columns only
__global__ __launch_bounds__(kBlock) void k_compact_cols(int n, const int32_t* __restrict__ off,
                                                         const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ocol, int32_t* __restrict__ ci) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int q = rp[i]; q < rp[i + 1]; ++q) ci[q] = ocol[off[i] + (q - rp[i])];
}

void launch_compact_cols(int n, const int32_t* off, const int32_t* rp, const int32_t* ocol, int32_t* ci,
                         hipStream_t st) {
  if (n > 0) k_compact_cols<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, off, rp, ocol, ci);
}

// Extended+i interpolation weights of one AMG level (De Sterck, Falgout,
// Nolting, Yang 2008), one thread per row, in the host construction's order
// and rounding: the interpolatory set of an F row is its strong C points and
// the strong C points of its strong F points, in the order met; each same-type
// off-diagonal a_im goes to its set point, through a strong F point m to the
// set points (and i) in proportion to a_ml, or to the diagonal.  Rows keep
// the pmax largest |w| (smaller column on ties), rescaled to the full row sum,
// then are sorted by column.  The row's set and sums live in LDS (at most
// kInterpCap points; more sets *overflow).  Output: row i's entries at
// i * outcap of ocol/oval, their count in cnt[i].
constexpr int kInterpCap = 64;

__global__ __launch_bounds__(64) void k_interp_exti(int n, const int32_t* __restrict__ arp,
                                                    const int32_t* __restrict__ aci,
                                                    const double* __restrict__ av,
                                                    const int32_t* __restrict__ srp,
                                                    const int32_t* __restrict__ sci,
                                                    const int32_t* __restrict__ cf,
                                                    const int32_t* __restrict__ func,
                                                    const int32_t* __restrict__ cidx, int pmax, int outcap,
                                                    int32_t* __restrict__ ocol, double* __restrict__ oval,
                                                    int32_t* __restrict__ cnt, int* __restrict__ overflow) {
#pragma clang fp contract(off)
  // each thread's set and sums run down a column, so that the 64 threads
  // reading their q-th entries hit 64 consecutive words (no bank conflicts)
  __shared__ int32_t s_set[kInterpCap][64];
  __shared__ double s_acc[kInterpCap][64];
  struct Col {
    int32_t* p;
    __device__ int32_t& operator[](int q) const { return p[q * 64]; }
  };
  struct ColD {
    double* p;
    __device__ double& operator[](int q) const { return p[q * 64]; }
  };
  const Col set{&s_set[0][threadIdx.x]};
  const ColD acc{&s_acc[0][threadIdx.x]};
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  const size_t o = (size_t)i * outcap;
  if (cf[i] == 1) {
    ocol[o] = cidx[i];
    oval[o] = 1.0;
    cnt[i] = 1;
    return;
  }
  int ns = 0;
  bool full = false;
  auto in_set = [&](int32_t c) -> int {
    for (int q = 0; q < ns; ++q)
      if (set[q] == c) return q;
    return -1;
  };
  auto add = [&](int32_t c) {
    if (in_set(c) >= 0) return;
    if (ns == kInterpCap) {
      full = true;
      return;
    }
    set[ns++] = c;
  };
  for (int k = srp[i]; k < srp[i + 1]; ++k) {
    const int32_t j = sci[k];
    if (cf[j] == 1) {
      add(j);
    } else {
      for (int q = srp[j]; q < srp[j + 1]; ++q)
        if (cf[sci[q]] == 1) add(sci[q]);
    }
  }
  if (full) {
    atomicAdd(overflow, 1);
    cnt[i] = 0;
    return;
  }
  auto a_diag = [&](int32_t r) -> double {
    for (int k = arp[r]; k < arp[r + 1]; ++k)
      if (aci[k] == r) return av[k];
    return 0.0;
  };
  auto strong = [&](int32_t m) -> bool {
    for (int k = srp[i]; k < srp[i + 1]; ++k)
      if (sci[k] == m) return true;
    return false;
  };
  int nout = 0;
  if (ns > 0) {
    for (int q = 0; q < ns; ++q) acc[q] = 0.0;
    double dg = a_diag(i);
    const int32_t fi = func[i];
    for (int k = arp[i]; k < arp[i + 1]; ++k) {
      const int32_t m = aci[k];
      if (m == i || func[m] != fi) continue;
      const double aim = av[k];
      const int pos = in_set(m);
      if (pos >= 0) {
        acc[pos] = acc[pos] + aim;
        continue;
      }
      if (cf[m] != 1 && strong(m)) {
        const double sm = a_diag(m) < 0.0 ? -1.0 : 1.0;
        double den = 0.0;
        for (int q = arp[m]; q < arp[m + 1]; ++q) {
          const int32_t l = aci[q];
          const double aml = av[q];
          if (sm * aml < 0.0 && (l == i || in_set(l) >= 0)) den = den + aml;
        }
        if (den == 0.0) {
          dg = dg + aim;
          continue;
        }
        for (int q = arp[m]; q < arp[m + 1]; ++q) {
          const int32_t l = aci[q];
          const double aml = av[q];
          if (!(sm * aml < 0.0)) continue;
          const double share = aim * aml / den;
          if (l == i) {
            dg = dg + share;
          } else {
            const int p = in_set(l);
            if (p >= 0) acc[p] = acc[p] + share;
          }
        }
        continue;
      }
      dg = dg + aim;
    }
    if (dg != 0.0) {
      // the row in set order: columns in set[], weights in acc[]
      for (int q = 0; q < ns; ++q) {
        set[q] = cidx[set[q]];
        acc[q] = -acc[q] / dg;
      }
      nout = ns;
      if (pmax > 0 && ns > pmax) {
        double total = 0.0, kept = 0.0;
        for (int q = 0; q < ns; ++q) total = total + acc[q];
        // the pmax best by (|w| descending, column ascending), in that order,
        // moved to the front
        for (int r = 0; r < pmax; ++r) {
          int best = r;
          for (int q = r + 1; q < ns; ++q) {
            const double fa = fabs(acc[q]), fb = fabs(acc[best]);
            if (fa != fb ? fa > fb : set[q] < set[best]) best = q;
          }
          const int32_t tc = set[r];
          set[r] = set[best];
          set[best] = tc;
          const double tw = acc[r];
          acc[r] = acc[best];
          acc[best] = tw;
        }
        for (int r = 0; r < pmax; ++r) kept = kept + acc[r];
        nout = pmax;
        if (kept != 0.0) {
          const double scale = total / kept;
          for (int r = 0; r < pmax; ++r) acc[r] = acc[r] * scale;
        }
      }
      // by column (columns are distinct)
      for (int a = 1; a < nout; ++a) {
        const int32_t c = set[a];
        const double w = acc[a];
        int b = a;
        for (; b > 0 && set[b - 1] > c; --b) {
          set[b] = set[b - 1];
          acc[b] = acc[b - 1];
        }
        set[b] = c;
        acc[b] = w;
      }
      for (int q = 0; q < nout; ++q) {
        ocol[o + q] = set[q];
        oval[o + q] = acc[q];
      }
    }
  }
  cnt[i] = nout;
}

// The same rows with one 64-lane workgroup per row, for levels whose rows are
// long: every step of k_interp_exti in the same order (the lanes compute the
// same uniform values), but a lookup in the interpolatory set or in row i of
// S is one ballot over the lanes, which hold one entry each, and rows of A
// are read 64 entries at a time and walked with shuffles.
__global__ __launch_bounds__(64) void k_interp_exti_wave(int n, const int32_t* __restrict__ arp,
                                                         const int32_t* __restrict__ aci,
                                                         const double* __restrict__ av,
                                                         const int32_t* __restrict__ srp,
                                                         const int32_t* __restrict__ sci,
                                                         const int32_t* __restrict__ cf,
                                                         const int32_t* __restrict__ func,
                                                         const int32_t* __restrict__ cidx, int pmax, int outcap,
                                                         int32_t* __restrict__ ocol, double* __restrict__ oval,
                                                         int32_t* __restrict__ cnt, int* __restrict__ overflow) {
#pragma clang fp contract(off)
  __shared__ int32_t s_set[kInterpCap];
  __shared__ double s_acc[kInterpCap];
  const int lane = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const size_t o = (size_t)i * outcap;
    if (cf[i] == 1) {
      if (lane == 0) {
        ocol[o] = cidx[i];
        oval[o] = 1.0;
        cnt[i] = 1;
      }
      continue;
    }
    // the set: lane q holds entry q (q < ns), in insertion order
    int32_t my_set = -1;
    int ns = 0;
    bool full = false;
    auto find = [&](int32_t c) -> int {
      const unsigned long long b = __ballot(lane < ns && my_set == c);
      return b ? __ffsll(b) - 1 : -1;
    };
    auto add = [&](int32_t c) {
      if (find(c) >= 0) return;
      if (ns == kInterpCap) {
        full = true;
        return;
      }
      if (lane == ns) my_set = c;
      ++ns;
    };
    const int s0 = srp[i], s1 = srp[i + 1];
    for (int k = s0; k < s1; ++k) {
      const int32_t j = sci[k];
      if (cf[j] == 1) {
        add(j);
      } else {
        for (int qb = srp[j]; qb < srp[j + 1]; qb += 64) {
          const int len = min(64, srp[j + 1] - qb);
          int32_t c = -1;
          bool isc = false;
          if (lane < len) {
            c = sci[qb + lane];
            isc = cf[c] == 1;
          }
          const unsigned long long cm = __ballot(isc);
          for (int t = 0; t < len; ++t)
            if ((cm >> t) & 1ull) add(__shfl(c, t, 64));
        }
      }
    }
    if (full) {
      if (lane == 0) {
        atomicAdd(overflow, 1);
        cnt[i] = 0;
      }
      continue;
    }
    if (ns == 0) {
      if (lane == 0) cnt[i] = 0;
      continue;
    }
    const int slen = s1 - s0;
    const int32_t my_s = lane < slen ? sci[s0 + lane] : -1;
    auto strong = [&](int32_t m) -> bool {
      if (slen <= 64) return __ballot(my_s == m) != 0;
      bool hit = false;
      for (int kb = s0; kb < s1; kb += 64) {
        const int32_t v = kb + lane < s1 ? sci[kb + lane] : -1;
        hit = hit || __ballot(v == m) != 0;
      }
      return hit;
    };
    auto a_diag = [&](int32_t r) -> double {
      for (int kb = arp[r]; kb < arp[r + 1]; kb += 64) {
        const bool hit = kb + lane < arp[r + 1] && aci[kb + lane] == r;
        const unsigned long long b = __ballot(hit);
        if (b) return av[kb + __ffsll(b) - 1];
      }
      return 0.0;
    };
    double my_acc = 0.0;
    double dg = a_diag(i);
    const int32_t fi = func[i];
    for (int kb = arp[i]; kb < arp[i + 1]; kb += 64) {
      const int len = min(64, arp[i + 1] - kb);
      int32_t mm = -1, fm = -1, cm = 0;
      double va = 0.0;
      if (lane < len) {
        mm = aci[kb + lane];
        va = av[kb + lane];
        fm = func[mm];
        cm = cf[mm];
      }
      for (int t = 0; t < len; ++t) {
        const int32_t m = __shfl(mm, t, 64);
        const double aim = __shfl(va, t, 64);
        if (m == i || __shfl(fm, t, 64) != fi) continue;
        const int pos = find(m);
        if (pos >= 0) {
          if (lane == pos) my_acc = my_acc + aim;
          continue;
        }
        if (__shfl(cm, t, 64) != 1 && strong(m)) {
          const double sm = a_diag(m) < 0.0 ? -1.0 : 1.0;
          double den = 0.0;
          for (int qb = arp[m]; qb < arp[m + 1]; qb += 64) {
            const int ln = min(64, arp[m + 1] - qb);
            int32_t lq = -1;
            double aq = 0.0;
            if (lane < ln) {
              lq = aci[qb + lane];
              aq = av[qb + lane];
            }
            for (int u = 0; u < ln; ++u) {
              const int32_t l = __shfl(lq, u, 64);
              const double aml = __shfl(aq, u, 64);
              if (sm * aml < 0.0 && (l == i || find(l) >= 0)) den = den + aml;
            }
          }
          if (den == 0.0) {
            dg = dg + aim;
            continue;
          }
          for (int qb = arp[m]; qb < arp[m + 1]; qb += 64) {
            const int ln = min(64, arp[m + 1] - qb);
            int32_t lq = -1;
            double aq = 0.0;
            if (lane < ln) {
              lq = aci[qb + lane];
              aq = av[qb + lane];
            }
            for (int u = 0; u < ln; ++u) {
              const int32_t l = __shfl(lq, u, 64);
              const double aml = __shfl(aq, u, 64);
              if (!(sm * aml < 0.0)) continue;
              const double share = aim * aml / den;
              if (l == i) {
                dg = dg + share;
              } else {
                const int p = find(l);
                if (p >= 0 && lane == p) my_acc = my_acc + share;
              }
            }
          }
          continue;
        }
        dg = dg + aim;
      }
    }
    if (dg == 0.0) {
      if (lane == 0) cnt[i] = 0;
      continue;
    }
    if (lane < ns) {
      s_set[lane] = cidx[my_set];
      s_acc[lane] = -my_acc / dg;
    }
    __syncthreads();
    if (lane == 0) {  // truncation and order exactly as in k_interp_exti
      int32_t* set = s_set;
      double* acc = s_acc;
      int nout = ns;
      if (pmax > 0 && ns > pmax) {
        double total = 0.0, kept = 0.0;
        for (int q = 0; q < ns; ++q) total = total + acc[q];
        for (int r = 0; r < pmax; ++r) {
          int best = r;
          for (int q = r + 1; q < ns; ++q) {
            const double fa = fabs(acc[q]), fb = fabs(acc[best]);
            if (fa != fb ? fa > fb : set[q] < set[best]) best = q;
          }
          const int32_t tc = set[r];
          set[r] = set[best];
          set[best] = tc;
          const double tw = acc[r];
          acc[r] = acc[best];
          acc[best] = tw;
        }
        for (int r = 0; r < pmax; ++r) kept = kept + acc[r];
        nout = pmax;
        if (kept != 0.0) {
          const double scale = total / kept;
          for (int r = 0; r < pmax; ++r) acc[r] = acc[r] * scale;
        }
      }
      for (int a = 1; a < nout; ++a) {
        const int32_t c = set[a];
        const double w = acc[a];
        int b = a;
        for (; b > 0 && set[b - 1] > c; --b) {
          set[b] = set[b - 1];
          acc[b] = acc[b - 1];
        }
        set[b] = c;
        acc[b] = w;
      }
      for (int q = 0; q < nout; ++q) {
        ocol[o + q] = set[q];
        oval[o + q] = acc[q];
      }
      cnt[i] = nout;
    }
    __syncthreads();
  }
}

void launch_interp_exti(int n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* srp,
                        const int32_t* sci, const int32_t* cf, const int32_t* func, const int32_t* cidx, int pmax,
                        int outcap, int32_t* ocol, double* oval, int32_t* cnt, int* overflow, bool long_rows,
                        hipStream_t st) {
  if (n <= 0) return;
  if (long_rows)
    k_interp_exti_wave<<<std::min(n, 16384), 64, 0, st>>>(n, arp, aci, av, srp, sci, cf, func, cidx, pmax, outcap,
                                                          ocol, oval, cnt, overflow);
  else
    k_interp_exti<<<(n + 63) / 64, 64, 0, st>>>(n, arp, aci, av, srp, sci, cf, func, cidx, pmax, outcap, ocol, oval,
                                               cnt, overflow);
}
int interp_set_cap() { return kInterpCap; }

// Sparse product C = X Y of scalar CSR matrices (int32 indices, FP64
// values) with the summation order of the host's product: each entry of row
// i of C is 0.0 plus the products x_ik y_kj added in the order of the stored
// entries of row i of X and, within row k of Y, of Y's stored entries; rows
// of C are sorted by column.  One 64-thread workgroup per row of X: the
// row's products are expanded into LDS in that order, sorted by (column,
// position) and each run of equal columns is summed from its first product
// on by one lane.  bound[i] = the number of products of row i (at most
// kGemmCap); the unique entries go to ocol/oval at off[i], their count to
// cnt[i].
constexpr int kGemmCap = 2048;

__global__ __launch_bounds__(kBlock) void k_spgemm_bound(int n, const int32_t* __restrict__ xrp,
                                                         const int32_t* __restrict__ xci,
                                                         const int32_t* __restrict__ yrp,
                                                         int32_t* __restrict__ bound) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int b = 0;
  for (int q = xrp[i]; q < xrp[i + 1]; ++q) b += yrp[xci[q] + 1] - yrp[xci[q]];
  bound[i] = b;
}

__global__ __launch_bounds__(64) void k_spgemm_rows(int n, const int32_t* __restrict__ xrp,
                                                    const int32_t* __restrict__ xci,
                                                    const double* __restrict__ xv,
                                                    const int32_t* __restrict__ yrp,
                                                    const int32_t* __restrict__ yci,
                                                    const double* __restrict__ yv,
                                                    const int64_t* __restrict__ off,
                                                    int32_t* __restrict__ ocol, double* __restrict__ oval,
                                                    int32_t* __restrict__ cnt, int cap) {
#pragma clang fp contract(off)
  // cap (a power of two, at least every row's product count) keys and values
  // in dynamic LDS, so short rows leave room for many workgroups per CU
  extern __shared__ double gemm_lds[];
  long long* key = reinterpret_cast<long long*>(gemm_lds);  // column * kGemmCap + position
  double* val = gemm_lds + cap;
  const int lane = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int q0 = xrp[i], q1 = xrp[i + 1];
    int m = 0;
    for (int qb = q0; qb < q1; qb += 64) {
      const int q = qb + lane;
      int len = 0, k = 0;
      double x = 0.0;
      if (q < q1) {
        k = xci[q];
        x = xv[q];
        len = yrp[k + 1] - yrp[k];
      }
      int incl = len;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
      }
      const int start = m + incl - len;
      for (int p = 0; p < len; ++p) {
        const int e = yrp[k] + p;
        key[start + p] = (long long)yci[e] * kGemmCap + (start + p);
        val[start + p] = x * yv[e];
      }
      m += __shfl(incl, 63, 64);
    }
    int np = 1;
    while (np < m) np <<= 1;
    for (int t = m + lane; t < np; t += 64) key[t] = LLONG_MAX;
    __syncthreads();
    // bitonic sort of (key, val); keys are unique, so the order is total
    for (int size = 2; size <= np; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = lane; t < np / 2; t += 64) {
          const int a = 2 * t - (t & (stride - 1)), b = a + stride;
          const bool up = (a & size) == 0;
          const long long ka = key[a], kb = key[b];
          if ((ka > kb) == up) {
            key[a] = kb;
            key[b] = ka;
            const double va = val[a];
            val[a] = val[b];
            val[b] = va;
          }
        }
        __syncthreads();
      }
    int runs = 0;
    const int64_t o = off[i];
    for (int t0 = 0; t0 < m; t0 += 64) {
      const int t = t0 + lane;
      long long c = -1;
      bool first = false;
      if (t < m) {
        c = key[t] / kGemmCap;
        first = t == 0 || key[t - 1] / kGemmCap != c;
      }
      const unsigned long long b = __ballot(first);
      if (first) {
        double sum = 0.0;
        for (int u = t; u < m && key[u] / kGemmCap == c; ++u) sum = sum + val[u];
        const int r = runs + __popcll(b & ((1ull << lane) - 1));
        ocol[o + r] = (int32_t)c;
        oval[o + r] = sum;
      }
      runs += __popcll(b);
    }
    if (lane == 0) cnt[i] = runs;
    __syncthreads();
  }
}

// rows of the product from their padded places (off) to CSR order (rp)
__global__ __launch_bounds__(kBlock) void k_spgemm_compact(int n, const int64_t* __restrict__ off,
                                                           const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ocol,
                                                           const double* __restrict__ oval,
                                                           int32_t* __restrict__ ci, double* __restrict__ v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t o = off[i];
  for (int q = rp[i]; q < rp[i + 1]; ++q) {
    ci[q] = ocol[o + (q - rp[i])];
    v[q] = oval[o + (q - rp[i])];
  }
}

void launch_spgemm_bound(int n, const int32_t* xrp, const int32_t* xci, const int32_t* yrp, int32_t* bound,
                         hipStream_t st) {
  if (n > 0) k_spgemm_bound<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, xrp, xci, yrp, bound);
}
static int lds_cap(int max_count) {
  int cap = 64;
  while (cap < max_count) cap <<= 1;
  return std::min(cap, kGemmCap);
}
void launch_spgemm_rows(int n, const int32_t* xrp, const int32_t* xci, const double* xv, const int32_t* yrp,
                        const int32_t* yci, const double* yv, const int64_t* off, int32_t* ocol, double* oval,
                        int32_t* cnt, int max_bound, hipStream_t st) {
  const int cap = lds_cap(max_bound);
  if (n > 0)
    k_spgemm_rows<<<std::min(n, 16384), 64, (size_t)cap * 16, st>>>(n, xrp, xci, xv, yrp, yci, yv, off, ocol, oval,
                                                                     cnt, cap);
}
void launch_spgemm_compact(int n, const int64_t* off, const int32_t* rp, const int32_t* ocol, const double* oval,
                           int32_t* ci, double* v, hipStream_t st) {
  if (n > 0) k_spgemm_compact<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, off, rp, ocol, oval, ci, v);
}
int spgemm_row_cap() { return kGemmCap; }

// --------------------------------------------------------------------------
// Multipass interpolation (Stueben 2001) of the aggressive level, one pass at
// a time, each row in the host construction's order and rounding.  In row i,
// "negative" means of sign opposite to a_ii, N_i are the same-type
// off-diagonal entries and P_i the strong dependencies of i that already have
// a row of P (pass[q] != -1): alpha = negative sum over N_i / negative sum
// over P_i, d = a_ii + the non-negative rest of N_i, and c_q = -alpha a_iq / d
// for q in P_i in A's column order; row i of P is the sum of c_q times row q
// (entries from 0.0, terms in the order of q and of row q's entries), sorted
// by column.  A row with d = 0 or a zero negative sum over P_i is empty.
constexpr int kMpCap = 64;  // interpolating points per row

__global__ __launch_bounds__(kBlock) void k_mp_mark(int n, const int32_t* __restrict__ srp,
                                                    const int32_t* __restrict__ sci,
                                                    const int32_t* __restrict__ pass, int32_t* __restrict__ flag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int32_t f = 0;
  if (pass[i] == -1)
    for (int a = srp[i]; a < srp[i + 1]; ++a)
      if (pass[sci[a]] != -1) {
        f = 1;
        break;
      }
  flag[i] = f;
}

// the interpolating points of row i and their coefficients, in A's column
// order; visit(q, c) for each; returns their count (0 for an empty row)
template <class Visit>
__device__ int mp_coefs(int i, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                        const double* __restrict__ av, const int32_t* __restrict__ srp,
                        const int32_t* __restrict__ sci, const int32_t* __restrict__ pass,
                        const int32_t* __restrict__ func, Visit visit) {
#pragma clang fp contract(off)
  const int b = arp[i], e = arp[i + 1], s0 = srp[i], s1 = srp[i + 1];
  double aii = 0.0;
  for (int k = b; k < e; ++k)
    if (aci[k] == i) aii = av[k];
  const int32_t fi = func[i];
  // is column q in P_i?  walks row i of S (sorted) alongside A's sorted row
  auto in_p = [&](int& sa, int32_t q) {
    while (sa < s1 && sci[sa] < q) ++sa;
    return sa < s1 && sci[sa] == q && pass[q] != -1;
  };
  double negn = 0.0, posn = 0.0, negp = 0.0;
  int sa = s0;
  for (int k = b; k < e; ++k) {
    const int32_t j = aci[k];
    if (j == i || func[j] != fi) continue;
    const bool opp = aii < 0.0 ? av[k] > 0.0 : av[k] < 0.0;
    if (opp)
      negn = negn + av[k];
    else
      posn = posn + av[k];
    if (opp && in_p(sa, j)) negp = negp + av[k];
  }
  const double d = aii + posn;
  if (d == 0.0 || negp == 0.0) return 0;
  const double alpha = negn / negp;
  int cnt = 0;
  sa = s0;
  for (int k = b; k < e; ++k) {
    const int32_t q = aci[k];
    if (q == i || func[q] != fi || !in_p(sa, q)) continue;
    visit(cnt++, q, -alpha * av[k] / d);
  }
  return cnt;
}

__global__ __launch_bounds__(kBlock) void k_mp_bound(int m, const int32_t* __restrict__ now,
                                                     const int32_t* __restrict__ arp,
                                                     const int32_t* __restrict__ aci,
                                                     const double* __restrict__ av,
                                                     const int32_t* __restrict__ srp,
                                                     const int32_t* __restrict__ sci,
                                                     const int32_t* __restrict__ pass,
                                                     const int32_t* __restrict__ func,
                                                     const int32_t* __restrict__ prp, int32_t* __restrict__ bound) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= m) return;
  int b = 0;
  const int cnt = mp_coefs(now[r], arp, aci, av, srp, sci, pass, func,
                           [&](int, int32_t q, double) { b += prp[q + 1] - prp[q]; });
  bound[r] = cnt > kMpCap ? kGemmCap + 1 : b;  // beyond any row cap: the host takes the level
}

// one 64-lane workgroup per row of the pass: the interpolating points and
// coefficients into LDS (lane 0, in order), the products c_q p_qj expanded in
// that order, sorted by (column, position), each run summed from its first
// product on
__global__ __launch_bounds__(64) void k_mp_rows(int m, const int32_t* __restrict__ now,
                                                const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                                                const double* __restrict__ av, const int32_t* __restrict__ srp,
                                                const int32_t* __restrict__ sci, const int32_t* __restrict__ pass,
                                                const int32_t* __restrict__ func, const int32_t* __restrict__ prp,
                                                const int32_t* __restrict__ pci, const double* __restrict__ pv,
                                                const int64_t* __restrict__ off, int32_t* __restrict__ ocol,
                                                double* __restrict__ oval, int32_t* __restrict__ cnt, int cap) {
#pragma clang fp contract(off)
  extern __shared__ double mp_lds[];  // cap keys and values (cap: see k_spgemm_rows)
  long long* key = reinterpret_cast<long long*>(mp_lds);  // column * kGemmCap + position
  double* val = mp_lds + cap;
  __shared__ int32_t qs[kMpCap];
  __shared__ double cs[kMpCap];
  __shared__ int nq;
  const int lane = threadIdx.x;
  for (int r = blockIdx.x; r < m; r += gridDim.x) {
    if (lane == 0)
      nq = mp_coefs(now[r], arp, aci, av, srp, sci, pass, func, [&](int t, int32_t q, double c) {
        if (t < kMpCap) {
          qs[t] = q;
          cs[t] = c;
        }
      });
    __syncthreads();
    const int nqr = min(nq, kMpCap);  // the bound kernel rejected longer sets
    int len = 0, q = 0;
    double c = 0.0;
    if (lane < nqr) {
      q = qs[lane];
      c = cs[lane];
      len = prp[q + 1] - prp[q];
    }
    int incl = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(incl, d, 64);
      if (lane >= d) incl += t;
    }
    const int start = incl - len;
    const int np_total = __shfl(incl, 63, 64);
    const int total = min(np_total, cap);  // the host sized cap to the largest bound
    for (int p = 0; p < len && start + p < total; ++p) {
      const int e = prp[q] + p;
      key[start + p] = (long long)pci[e] * kGemmCap + (start + p);
      val[start + p] = c * pv[e];
    }
    int np = 1;
    while (np < total) np <<= 1;
    for (int t = total + lane; t < np; t += 64) key[t] = LLONG_MAX;
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = lane; t < np / 2; t += 64) {
          const int a = 2 * t - (t & (stride - 1)), b = a + stride;
          const bool up = (a & size) == 0;
          const long long ka = key[a], kb = key[b];
          if ((ka > kb) == up) {
            key[a] = kb;
            key[b] = ka;
            const double va = val[a];
            val[a] = val[b];
            val[b] = va;
          }
        }
        __syncthreads();
      }
    int runs = 0;
    const int64_t o = off[r];
    for (int t0 = 0; t0 < total; t0 += 64) {
      const int t = t0 + lane;
      long long col = -1;
      bool first = false;
      if (t < total) {
        col = key[t] / kGemmCap;
        first = t == 0 || key[t - 1] / kGemmCap != col;
      }
      const unsigned long long bal = __ballot(first);
      if (first) {
        double sum = 0.0;
        for (int u = t; u < total && key[u] / kGemmCap == col; ++u) sum = sum + val[u];
        const int w = runs + __popcll(bal & ((1ull << lane) - 1));
        ocol[o + w] = (int32_t)col;
        oval[o + w] = sum;
      }
      runs += __popcll(bal);
    }
    if (lane == 0) cnt[r] = runs;
    __syncthreads();
  }
}

// next P: the pass's rows from their padded places, every other row copied;
// the pass's points get pass number pass_no and their rowpos is reset
__global__ __launch_bounds__(kBlock) void k_mp_merge(int n, int pass_no, int32_t* __restrict__ rowpos,
                                                     const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ ocol,
                                                     const double* __restrict__ oval,
                                                     const int32_t* __restrict__ prp,
                                                     const int32_t* __restrict__ pci,
                                                     const double* __restrict__ pv,
                                                     const int32_t* __restrict__ nrp, int32_t* __restrict__ nci,
                                                     double* __restrict__ nv, int32_t* __restrict__ pass) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int r = rowpos[i];
  const int o = nrp[i], len = nrp[i + 1] - nrp[i];
  if (r >= 0) {
    for (int t = 0; t < len; ++t) {
      nci[o + t] = ocol[off[r] + t];
      nv[o + t] = oval[off[r] + t];
    }
    pass[i] = pass_no;
    rowpos[i] = -1;
  } else {
    for (int t = 0; t < len; ++t) {
      nci[o + t] = pci[prp[i] + t];
      nv[o + t] = pv[prp[i] + t];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_mp_scatter(int m, const int32_t* __restrict__ now,
                                                       int32_t* __restrict__ rowpos) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r < m) rowpos[now[r]] = r;
}

// now[pos[i]] = i for the flagged points (pos: exclusive prefix of flag)
__global__ __launch_bounds__(kBlock) void k_select(int n, const int32_t* __restrict__ flag,
                                                   const int32_t* __restrict__ pos, int32_t* __restrict__ now) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && flag[i]) now[pos[i]] = i;
}

__global__ __launch_bounds__(kBlock) void k_mp_setlen(int m, const int32_t* __restrict__ now,
                                                      const int32_t* __restrict__ cnt, int32_t* __restrict__ len) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r < m) len[now[r]] = cnt[r];
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int64_t n, int32_t* __restrict__ x, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = v;
}

void launch_mp_mark(int n, const int32_t* srp, const int32_t* sci, const int32_t* pass, int32_t* flag,
                    hipStream_t st) {
  if (n > 0) k_mp_mark<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, pass, flag);
}
void launch_select(int n, const int32_t* flag, const int32_t* pos, int32_t* now, hipStream_t st) {
  if (n > 0) k_select<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, flag, pos, now);
}
void launch_mp_setlen(int m, const int32_t* now, const int32_t* cnt, int32_t* len, hipStream_t st) {
  if (m > 0) k_mp_setlen<<<nblocks(m, kBlock), kBlock, 0, st>>>(m, now, cnt, len);
}
void launch_mp_bound(int m, const int32_t* now, const int32_t* arp, const int32_t* aci, const double* av,
                     const int32_t* srp, const int32_t* sci, const int32_t* pass, const int32_t* func,
                     const int32_t* prp, int32_t* bound, hipStream_t st) {
  if (m > 0) k_mp_bound<<<nblocks(m, kBlock), kBlock, 0, st>>>(m, now, arp, aci, av, srp, sci, pass, func, prp, bound);
}
void launch_mp_rows(int m, const int32_t* now, const int32_t* arp, const int32_t* aci, const double* av,
                    const int32_t* srp, const int32_t* sci, const int32_t* pass, const int32_t* func,
                    const int32_t* prp, const int32_t* pci, const double* pv, const int64_t* off, int32_t* ocol,
                    double* oval, int32_t* cnt, int max_bound, hipStream_t st) {
  const int cap = lds_cap(max_bound);
  if (m > 0)
    k_mp_rows<<<std::min(m, 16384), 64, (size_t)cap * 16, st>>>(m, now, arp, aci, av, srp, sci, pass, func, prp, pci,
                                                                 pv, off, ocol, oval, cnt, cap);
}
void launch_mp_merge(int n, int pass_no, int32_t* rowpos, const int32_t* now, int m, const int64_t* off,
                     const int32_t* ocol, const double* oval, const int32_t* prp, const int32_t* pci,
                     const double* pv, const int32_t* nrp, int32_t* nci, double* nv, int32_t* pass,
                     hipStream_t st) {
  if (m > 0) k_mp_scatter<<<nblocks(m, kBlock), kBlock, 0, st>>>(m, now, rowpos);
  if (n > 0)
    k_mp_merge<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, pass_no, rowpos, off, ocol, oval, prp, pci, pv, nrp, nci,
                                                      nv, pass);
}
void launch_fill_i32(int64_t n, int32_t* x, int32_t v, hipStream_t st) {
  if (n > 0) k_fill_i32<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, x, v);
}
int mp_point_cap() { return kMpCap; }

// --------------------------------------------------------------------------
// Distance-two strength among the C points of a first pass (the aggressive
// level): row r is C point i = cpts[r]; its columns are the coarse indices of
// the C points j != i reached from i by one strong link (j in S_i) or two
// (j in S_k, k in S_i), sorted, each once.  One 64-lane workgroup per row:
// the candidates go to LDS, are sorted and the first of each run is kept.
// bound[r] = 1 + |S_k| summed over k in S_i (at most s2_row_cap()); a first
// launch with rp == nullptr counts the columns into cnt, a second writes them
// at rp[r].
constexpr int kS2Cap = 2048;

__global__ __launch_bounds__(kBlock) void k_s2_bound(int nc, const int32_t* __restrict__ cpts,
                                                     const int32_t* __restrict__ srp,
                                                     const int32_t* __restrict__ sci, int32_t* __restrict__ bound) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= nc) return;
  const int i = cpts[r];
  int b = 0;
  for (int a = srp[i]; a < srp[i + 1]; ++a) b += 1 + srp[sci[a] + 1] - srp[sci[a]];
  bound[r] = b;
}

__global__ __launch_bounds__(64) void k_s2_rows(int nc, const int32_t* __restrict__ cpts,
                                                const int32_t* __restrict__ srp, const int32_t* __restrict__ sci,
                                                const int32_t* __restrict__ cidx, const int32_t* __restrict__ rp,
                                                int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
  __shared__ int32_t key[kS2Cap];
  const int lane = threadIdx.x;
  for (int r = blockIdx.x; r < nc; r += gridDim.x) {
    const int i = cpts[r], a0 = srp[i], a1 = srp[i + 1];
    int m = 0;  // candidates so far
    for (int ab = a0; ab < a1; ab += 64) {
      const int a = ab + lane;
      int k = 0, len = 0;
      if (a < a1) {
        k = sci[a];
        len = 1 + srp[k + 1] - srp[k];
      }
      int incl = len;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
      }
      const int start = m + incl - len;
      for (int p = 0; p < len && start + p < kS2Cap; ++p) {
        const int j = p == 0 ? k : sci[srp[k] + p - 1];
        const int c = j == i ? -1 : cidx[j];  // -1: not a C point, or i itself
        key[start + p] = c < 0 ? INT_MAX : c;
      }
      m += __shfl(incl, 63, 64);
    }
    m = min(m, kS2Cap);  // the host rejects rows with more candidates
    int np = 1;
    while (np < m) np <<= 1;
    for (int t = m + lane; t < np; t += 64) key[t] = INT_MAX;
    __syncthreads();
    for (int size = 2; size <= np; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = lane; t < np / 2; t += 64) {
          const int a = 2 * t - (t & (stride - 1)), b = a + stride;
          const bool up = (a & size) == 0;
          const int ka = key[a], kb = key[b];
          if ((ka > kb) == up) {
            key[a] = kb;
            key[b] = ka;
          }
        }
        __syncthreads();
      }
    int runs = 0;
    for (int t0 = 0; t0 < m; t0 += 64) {
      const int t = t0 + lane;
      const int c = t < m ? key[t] : INT_MAX;
      const bool first = c != INT_MAX && (t == 0 || key[t - 1] != c);
      const unsigned long long bal = __ballot(first);
      if (first && rp) ci[rp[r] + runs + __popcll(bal & ((1ull << lane) - 1))] = c;
      runs += __popcll(bal);
    }
    if (lane == 0 && !rp) cnt[r] = runs;
    __syncthreads();
  }
}

void launch_s2_bound(int nc, const int32_t* cpts, const int32_t* srp, const int32_t* sci, int32_t* bound,
                     hipStream_t st) {
  if (nc > 0) k_s2_bound<<<nblocks(nc, kBlock), kBlock, 0, st>>>(nc, cpts, srp, sci, bound);
}
void launch_s2_rows(int nc, const int32_t* cpts, const int32_t* srp, const int32_t* sci, const int32_t* cidx,
                    const int32_t* rp, int32_t* ci, int32_t* cnt, hipStream_t st) {
  if (nc > 0) k_s2_rows<<<std::min(nc, 8192), 64, 0, st>>>(nc, cpts, srp, sci, cidx, rp, ci, cnt);
}
int s2_row_cap() { return kS2Cap; }

// --------------------------------------------------------------------------
// HMIS over blocks of consecutive points (the hmis_block reading): the first
// pass inside every block on its in-block links, then the points depending
// on a C point are F, then PMIS with the priority (count, SplitMix64(i), i).

// the transpose's columns: dependents of each point, in any order within a row
__global__ __launch_bounds__(kBlock) void k_tr_count(int n, const int32_t* __restrict__ srp,
                                                     const int32_t* __restrict__ sci, int32_t* __restrict__ deg) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int a = srp[i]; a < srp[i + 1]; ++a) atomicAdd(&deg[sci[a]], 1);
}
__global__ __launch_bounds__(kBlock) void k_tr_fill(int n, const int32_t* __restrict__ srp,
                                                    const int32_t* __restrict__ sci, int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ tci) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int a = srp[i]; a < srp[i + 1]; ++a) tci[atomicAdd(&cursor[sci[a]], 1)] = i;
}

// one 64-lane workgroup per block: measures and states of the block's points
// in LDS (dynamic, 8 bytes a point); each pick is the largest measure >= 1,
// smallest index, found by a scan and a wave reduction; the points of the
// block depending on it (its row of the transpose) become F and raise their
// undecided in-block dependencies, then its own undecided in-block
// dependencies drop.  cf1[i] = 1 for the block's C points, else 0.
__global__ __launch_bounds__(64) void k_hmis_block(int n, int block, const int32_t* __restrict__ srp,
                                                   const int32_t* __restrict__ sci,
                                                   const int32_t* __restrict__ trp,
                                                   const int32_t* __restrict__ tci, int32_t* __restrict__ cf1) {
  extern __shared__ int32_t hmis_lds[];
  int32_t* lam = hmis_lds;
  int32_t* st = hmis_lds + block;  // 0 undecided, 1 C, -1 F (a count while starting)
  const int lane = threadIdx.x;
  const int lo = blockIdx.x * block, hi = min(n, lo + block), m = hi - lo;
  for (int t = lane; t < m; t += 64) {
    lam[t] = 0;
    st[t] = 0;
  }
  __syncthreads();
  for (int t = lane; t < m; t += 64) {
    const int i = lo + t;
    int out = 0;
    for (int a = srp[i]; a < srp[i + 1]; ++a) {
      const int j = sci[a];
      if (j >= lo && j < hi) {
        atomicAdd(&lam[j - lo], 1);
        ++out;
      }
    }
    st[t] = out;
  }
  __syncthreads();
  for (int t = lane; t < m; t += 64) st[t] = (st[t] == 0 && lam[t] == 0) ? -1 : 0;
  __syncthreads();
  for (;;) {
    int bl = 0, bt = -1;
    for (int t = lane; t < m; t += 64)
      if (st[t] == 0 && lam[t] >= 1 && lam[t] > bl) {
        bl = lam[t];
        bt = t;
      }
    for (int off = 32; off > 0; off >>= 1) {
      const int ol = __shfl_xor(bl, off, 64), ot = __shfl_xor(bt, off, 64);
      if (ot >= 0 && (bt < 0 || ol > bl || (ol == bl && ot < bt))) {
        bl = ol;
        bt = ot;
      }
    }
    if (bt < 0) break;
    const int c = lo + bt;
    if (lane == 0) st[bt] = 1;
    __syncthreads();
    for (int k = trp[c] + lane; k < trp[c + 1]; k += 64) {
      const int f = tci[k];
      if (f < lo || f >= hi || st[f - lo] != 0) continue;
      st[f - lo] = -1;
      for (int a = srp[f]; a < srp[f + 1]; ++a) {
        const int q = sci[a];
        if (q >= lo && q < hi && st[q - lo] == 0) atomicAdd(&lam[q - lo], 1);
      }
    }
    __syncthreads();
    for (int a = srp[c] + lane; a < srp[c + 1]; a += 64) {
      const int q = sci[a];
      if (q >= lo && q < hi && st[q - lo] == 0) atomicSub(&lam[q - lo], 1);
    }
    __syncthreads();
  }
  for (int t = lane; t < m; t += 64) cf1[lo + t] = st[t] == 1 ? 1 : 0;
}

// step 2: C stays C, a point depending strongly on a C point is F, the rest
// undecided (0)
__global__ __launch_bounds__(kBlock) void k_hmis_cover(int n, const int32_t* __restrict__ srp,
                                                       const int32_t* __restrict__ sci,
                                                       const int32_t* __restrict__ cf1, int32_t* __restrict__ cf) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int v = cf1[i] == 1 ? 1 : 0;
  if (v == 0)
    for (int a = srp[i]; a < srp[i + 1]; ++a)
      if (cf1[sci[a]] == 1) {
        v = -1;
        break;
      }
  cf[i] = v;
}

// PMIS counts: cnt[i] += 1 for every undecided j depending on i
__global__ __launch_bounds__(kBlock) void k_pmis_count(int n, const int32_t* __restrict__ srp,
                                                       const int32_t* __restrict__ sci,
                                                       const int32_t* __restrict__ cf, int32_t* __restrict__ cnt) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n || cf[j] != 0) return;
  for (int a = srp[j]; a < srp[j + 1]; ++a) atomicAdd(&cnt[sci[a]], 1);
}

// undecided points nobody undecided depends on are F
__global__ __launch_bounds__(kBlock) void k_pmis_drop(int n, const int32_t* __restrict__ cnt,
                                                      int32_t* __restrict__ cf) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && cf[i] == 0 && cnt[i] == 0) cf[i] = -1;
}

// SplitMix64 (Steele, Lea, Flood 2014): the output for counter value x
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ bool pmis_beats(int32_t ca, int a, int32_t cb, int b) {
  if (ca != cb) return ca > cb;
  const uint64_t ha = splitmix64((uint64_t)a), hb = splitmix64((uint64_t)b);
  if (ha != hb) return ha > hb;
  return a > b;
}

// one round: isnew[i] = 1 for the undecided points whose priority beats every
// undecided strong neighbour's (links either way); *left counts the
// undecided points
__global__ __launch_bounds__(kBlock) void k_pmis_pick(int n, const int32_t* __restrict__ srp,
                                                      const int32_t* __restrict__ sci,
                                                      const int32_t* __restrict__ trp,
                                                      const int32_t* __restrict__ tci,
                                                      const int32_t* __restrict__ cnt,
                                                      const int32_t* __restrict__ cf, int32_t* __restrict__ isnew,
                                                      int* __restrict__ left) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int top = 0;
  if (cf[i] == 0) {
    atomicAdd(left, 1);
    top = 1;
    for (int a = srp[i]; a < srp[i + 1] && top; ++a) {
      const int j = sci[a];
      if (cf[j] == 0 && pmis_beats(cnt[j], j, cnt[i], i)) top = 0;
    }
    for (int a = trp[i]; a < trp[i + 1] && top; ++a) {
      const int j = tci[a];
      if (cf[j] == 0 && pmis_beats(cnt[j], j, cnt[i], i)) top = 0;
    }
  }
  isnew[i] = top;
}

// the round's C points, then the undecided points depending on one are F
__global__ __launch_bounds__(kBlock) void k_pmis_c(int n, const int32_t* __restrict__ isnew,
                                                   int32_t* __restrict__ cf) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n && isnew[i]) cf[i] = 1;
}
__global__ __launch_bounds__(kBlock) void k_pmis_f(int n, const int32_t* __restrict__ srp,
                                                   const int32_t* __restrict__ sci,
                                                   const int32_t* __restrict__ isnew, int32_t* __restrict__ cf) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || cf[i] != 0) return;
  for (int a = srp[i]; a < srp[i + 1]; ++a)
    if (isnew[sci[a]]) {
      cf[i] = -1;
      return;
    }
}

void launch_transpose_pattern(int n, const int32_t* srp, const int32_t* sci, int32_t* deg, int32_t* cursor,
                              int32_t* tci, int phase, hipStream_t st) {
  if (n <= 0) return;
  if (phase == 0)
    k_tr_count<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, deg);
  else
    k_tr_fill<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, cursor, tci);
}
void launch_hmis_blocks(int n, int block, const int32_t* srp, const int32_t* sci, const int32_t* trp,
                        const int32_t* tci, int32_t* cf1, int32_t* cf, hipStream_t st) {
  if (n <= 0) return;
  k_hmis_block<<<nblocks(n, block), 64, (size_t)block * 8, st>>>(n, block, srp, sci, trp, tci, cf1);
  k_hmis_cover<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, cf1, cf);
}
void launch_pmis_start(int n, const int32_t* srp, const int32_t* sci, int32_t* cf, int32_t* cnt, hipStream_t st) {
  if (n <= 0) return;
  k_fill_i32<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, cnt, 0);
  k_pmis_count<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, cf, cnt);
  k_pmis_drop<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, cnt, cf);
}
void launch_pmis_round(int n, const int32_t* srp, const int32_t* sci, const int32_t* trp, const int32_t* tci,
                       const int32_t* cnt, int32_t* cf, int32_t* isnew, int* left, hipStream_t st) {
  if (n <= 0) return;
  k_fill_i32<<<1, kBlock, 0, st>>>(1, left, 0);
  k_pmis_pick<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, trp, tci, cnt, cf, isnew, left);
  k_pmis_c<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, isnew, cf);
  k_pmis_f<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, isnew, cf);
}
int hmis_block_cap() { return 4096; }

// --------------------------------------------------------------------------
// Exclusive prefix sums of int32 counts on the device (setup row pointers):
// each 256-thread workgroup sums 16 consecutive counts per thread and scans
// the thread sums in LDS; one workgroup then scans the workgroup totals in
// chunks with a running carry; a last pass adds each workgroup's offset.
// out[0..n) are the offsets, out[n] the total; also the largest count.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kBlock * kScanPer;

template <class O>
__global__ __launch_bounds__(kBlock) void k_scan_local(int64_t n, const int32_t* __restrict__ in,
                                                       O* __restrict__ out, int64_t* __restrict__ bsum,
                                                       int* __restrict__ maxv) {
  __shared__ int64_t part[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  int64_t sum = 0;
  int mx = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    sum += v[k];
    mx = max(mx, v[k]);
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int d = 1; d < kBlock; d <<= 1) {  // inclusive Hillis-Steele scan of the thread sums
    const int64_t t = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - sum;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = (O)run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = part[kBlock - 1];
  if (maxv) {
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_down(mx, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(maxv, mx);
  }
}

// exclusive scan of the nb workgroup totals, in place, one workgroup; the
// grand total to *total
__global__ __launch_bounds__(kBlock) void k_scan_sums(int64_t nb, int64_t* __restrict__ bsum,
                                                      int64_t* __restrict__ total) {
  __shared__ int64_t part[kBlock];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kBlock) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t x = i < nb ? bsum[i] : 0;
    part[threadIdx.x] = x;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
      const int64_t t = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + part[threadIdx.x] - x;
    carry += part[kBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

template <class O>
__global__ __launch_bounds__(kBlock) void k_scan_add(int64_t n, O* __restrict__ out,
                                                     const int64_t* __restrict__ bsum,
                                                     const int64_t* __restrict__ total) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (O)(out[i] + bsum[i / kScanChunk]);
  if (i == 0) out[n] = (O)*total;
}

int64_t scan_tmp_size(int64_t n) { return std::max<int64_t>(1, (n + kScanChunk - 1) / kScanChunk) + 1; }

template <class O>
void launch_scan(int64_t n, const int32_t* in, O* out, int64_t* tmp, int* maxv, hipStream_t st) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanChunk - 1) / kScanChunk);
  int64_t* total = tmp + nb;
  k_scan_local<O><<<(unsigned)nb, kBlock, 0, st>>>(n, in, out, tmp, maxv);
  k_scan_sums<<<1, kBlock, 0, st>>>(nb, tmp, total);
  k_scan_add<O><<<(unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock), kBlock, 0, st>>>(n, out, tmp, total);
}
template void launch_scan<int64_t>(int64_t, const int32_t*, int64_t*, int64_t*, int*, hipStream_t);
template void launch_scan<int32_t>(int64_t, const int32_t*, int32_t*, int64_t*, int*, hipStream_t);

// --------------------------------------------------------------------------
// Ruge-Stueben first pass over the small weakly connected components of a
// strength graph.  The pass reads and changes only the strong neighbours of a
// pick, so components never interact, and the picks inside one component are
// those of a pass over it alone, in the same order.  Components come from a
// lock-free union-find (a root is hooked under a smaller root by
// compare-and-swap, a failed swap retries from the value it found; paths are
// halved on the way up), so every root is its component's smallest point.

// parent[i] = i, lam[i] = 0, size[i] = 0
__global__ __launch_bounds__(kBlock) void k_fp_init(int n, int32_t* __restrict__ parent, int32_t* __restrict__ lam,
                                                    int32_t* __restrict__ size) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  parent[i] = i;
  lam[i] = 0;
  size[i] = 0;
}

__device__ __forceinline__ int32_t uf_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// the root of x, halving the path: each visited point is pointed at its
// grandparent (still an ancestor, so concurrent hooks stay valid)
__device__ int32_t uf_root(int32_t* parent, int32_t x) {
  int32_t p = uf_load(&parent[x]);
  while (p != x) {
    const int32_t g = uf_load(&parent[p]);
    if (g == p) return p;
    __hip_atomic_store(&parent[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = g;
    p = uf_load(&parent[x]);
  }
  return x;
}

// every strong link i -> j: lam[j] += 1 (the points depending on j) and the
// union of i's and j's sets
__global__ __launch_bounds__(kBlock) void k_fp_links(int n, const int32_t* __restrict__ srp,
                                                     const int32_t* __restrict__ sci, int32_t* parent,
                                                     int32_t* __restrict__ lam) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int a = srp[i]; a < srp[i + 1]; ++a) {
    const int32_t j = sci[a];
    atomicAdd(&lam[j], 1);
    int32_t ri = uf_root(parent, i), rj = uf_root(parent, j);
    while (ri != rj) {
      if (ri < rj) {  // hook rj under ri
        const int32_t seen = atomicCAS(&parent[rj], rj, ri);
        if (seen == rj) break;
        rj = uf_root(parent, seen);
      } else {
        const int32_t seen = atomicCAS(&parent[ri], ri, rj);
        if (seen == ri) break;
        ri = uf_root(parent, seen);
      }
    }
  }
}

// root[i] and the component sizes; isolated points (no link either way) are
// F, the rest undecided.  The forest no longer changes: plain (cached)
// loads walk up to the root.
__global__ __launch_bounds__(kBlock) void k_fp_roots(int n, const int32_t* __restrict__ srp,
                                                     const int32_t* __restrict__ parent,
                                                     const int32_t* __restrict__ lam, int32_t* __restrict__ root,
                                                     int32_t* __restrict__ size, int32_t* __restrict__ cf) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int32_t r = i, p = parent[i];
  while (p != r) {
    r = p;
    p = parent[r];
  }
  root[i] = r;
  atomicAdd(&size[r], 1);
  cf[i] = (srp[i + 1] == srp[i] && lam[i] == 0) ? -1 : 0;
}

// members of the components picked by the host: cursor[r] starts at the
// component's offset (-1 for components not taken)
__global__ __launch_bounds__(kBlock) void k_fp_members(int n, const int32_t* __restrict__ root,
                                                       int32_t* __restrict__ cursor, int32_t* __restrict__ members) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t r = root[i];
  if (cursor[r] >= 0) members[atomicAdd(&cursor[r], 1)] = i;
}

// one thread per small component: the first pass over its members (picks by
// scanning them: the largest measure >= 1, the smallest index on ties), with
// the points depending on a pick found by scanning the members' rows
__global__ __launch_bounds__(kBlock) void k_fp_small(int ncomp, const int32_t* __restrict__ coff,
                                                     const int32_t* __restrict__ members,
                                                     const int32_t* __restrict__ srp,
                                                     const int32_t* __restrict__ sci, int32_t* __restrict__ lam,
                                                     int32_t* __restrict__ cf) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= ncomp) return;
  const int32_t* mem = members + coff[q];
  const int m = coff[q + 1] - coff[q];
  for (;;) {
    int32_t best = -1, bl = 0;
    for (int t = 0; t < m; ++t) {
      const int32_t i = mem[t];
      if (cf[i] != 0) continue;
      const int32_t l = lam[i];
      if (l >= 1 && (best < 0 || l > bl || (l == bl && i < best))) {
        best = i;
        bl = l;
      }
    }
    if (best < 0) break;
    cf[best] = 1;
    for (int t = 0; t < m; ++t) {  // the undecided points depending on best become F
      const int32_t f = mem[t];
      if (cf[f] != 0) continue;
      bool dep = false;
      for (int a = srp[f]; a < srp[f + 1] && !dep; ++a) dep = sci[a] == best;
      if (!dep) continue;
      cf[f] = -1;
      for (int a = srp[f]; a < srp[f + 1]; ++a)
        if (cf[sci[a]] == 0) ++lam[sci[a]];
    }
    for (int a = srp[best]; a < srp[best + 1]; ++a)
      if (cf[sci[a]] == 0) --lam[sci[a]];
  }
  for (int t = 0; t < m; ++t)
    if (cf[mem[t]] == 0) cf[mem[t]] = -1;
}

void launch_fp_components(int n, const int32_t* srp, const int32_t* sci, int32_t* parent, int32_t* lam,
                          int32_t* root, int32_t* size, int32_t* cf, hipStream_t st) {
  if (n <= 0) return;
  k_fp_init<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, parent, lam, size);
  k_fp_links<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, sci, parent, lam);
  k_fp_roots<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, srp, parent, lam, root, size, cf);
}
void launch_fp_small(int n, const int32_t* root, int32_t* cursor, int32_t* members, int ncomp, const int32_t* coff,
                     const int32_t* srp, const int32_t* sci, int32_t* lam, int32_t* cf, hipStream_t st) {
  if (n <= 0 || ncomp <= 0) return;
  k_fp_members<<<nblocks(n, kBlock), kBlock, 0, st>>>(n, root, cursor, members);
  k_fp_small<<<nblocks(ncomp, kBlock), kBlock, 0, st>>>(ncomp, coff, members, srp, sci, lam, cf);
}

// Block ILU(0) of any block-sparse A (Sec. 3.1) on W, a copy of A's SELL-64
// values: one launch per forward dependency level, one thread per row, each
// row in the host factorisation's order: for its lower blocks in column
// order, L_ic = W_ic U_cc^-1 and W_it -= L_ic U_ct over the U blocks of row c
// that row i also holds; then U_ii^-1.  Rows of a level depend only on rows
// of earlier levels.  dslot: the diagonal's slot in each row.  A singular
// U_ii leaves zeros and lowers *bad to the row.
__global__ __launch_bounds__(kBlock) void k_ilu_rows(int p0, int p1, const int32_t* __restrict__ fperm,
                                                     const int32_t* __restrict__ sptr,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ dslot, double* __restrict__ W,
                                                     double* __restrict__ uinv, int* __restrict__ bad) {
#pragma clang fp contract(off)
  const int p = p0 + blockIdx.x * kBlock + threadIdx.x;
  if (p >= p1) return;
  const int i = fperm[p];
  const int lane = i & 63;
  const size_t k0 = (size_t)sptr[i >> 6];
  const int n = rp[i + 1] - rp[i], d = dslot[i];
  for (int q = 0; q < d; ++q) {
    const int c = col[(k0 + q) * 64 + lane];
    double a[9], Lq[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) a[e] = W[((k0 + q) * 9 + e) * 64 + lane];
    mm3_dev(a, uinv + (size_t)c * 9, Lq);
#pragma unroll
    for (int e = 0; e < 9; ++e) W[((k0 + q) * 9 + e) * 64 + lane] = Lq[e];
    const int lc = c & 63;
    const size_t kc0 = (size_t)sptr[c >> 6];
    const int nc = rp[c + 1] - rp[c];
    int t = q + 1;
    for (int u = dslot[c] + 1; u < nc; ++u) {
      const int cu = col[(kc0 + u) * 64 + lc];
      while (t < n && col[(k0 + t) * 64 + lane] < cu) ++t;
      if (t == n) break;
      if (col[(k0 + t) * 64 + lane] != cu) continue;
      double ub[9], prod[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) ub[e] = W[((kc0 + u) * 9 + e) * 64 + lc];
      mm3_dev(Lq, ub, prod);
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        double& x = W[((k0 + t) * 9 + e) * 64 + lane];
        x = x - prod[e];
      }
    }
  }
  double dg[9], inv[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) dg[e] = W[((k0 + d) * 9 + e) * 64 + lane];
  if (!inv3_dev(dg, inv)) {
#pragma unroll
    for (int e = 0; e < 9; ++e) inv[e] = 0.0;
    atomicMin(bad, i);
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) uinv[(size_t)i * 9 + e] = inv[e];
}

// The factored blocks of the rows perm[p] into a SELL-64 over positions p:
// the L blocks (lower) or the U blocks right of the diagonal; padding slots
// get column -1 and zero values.
template <class T>
__global__ __launch_bounds__(kBlock) void k_ilu_pack_sell(int nb, int npos, const int32_t* __restrict__ perm,
                                                          int lower, const int32_t* __restrict__ sptrA,
                                                          const int32_t* __restrict__ colA,
                                                          const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ dslot,
                                                          const double* __restrict__ W,
                                                          const int32_t* __restrict__ sptrF,
                                                          int32_t* __restrict__ colF, T* __restrict__ valF) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= npos) return;
  const int sl = p >> 6, lp = p & 63;
  const int w = sptrF[sl + 1] - sptrF[sl];
  const bool live = p < nb;
  const int i = live ? perm[p] : 0;
  const int li = i & 63;
  const size_t k0 = (size_t)sptrA[i >> 6];
  const int d = dslot[i];
  const int first = lower ? 0 : d + 1;
  const int cnt = live ? (lower ? d : rp[i + 1] - rp[i] - d - 1) : 0;
  for (int k = 0; k < w; ++k) {
    const size_t slot = (size_t)sptrF[sl] + k;
    const bool real = k < cnt;
    colF[slot * 64 + lp] = real ? colA[(k0 + first + k) * 64 + li] : -1;
#pragma unroll
    for (int e = 0; e < 9; ++e)
      valF[(slot * 9 + e) * 64 + lp] = real ? (T)W[((k0 + first + k) * 9 + e) * 64 + li] : T(0);
  }
}

// U_ii^-1 by backward position, planar: out[e * npad + p] (zero past nb)
template <class T>
__global__ __launch_bounds__(kBlock) void k_ilu_pack_uinv(int nb, int npad, const int32_t* __restrict__ bperm,
                                                          const double* __restrict__ uinv,
                                                          T* __restrict__ out) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= npad) return;
#pragma unroll
  for (int e = 0; e < 9; ++e) out[(size_t)e * npad + p] = p < nb ? (T)uinv[(size_t)bperm[p] * 9 + e] : T(0);
}

void launch_ilu_rows(const Sell& A, const int32_t* fperm, int32_t p0, int32_t p1, const int32_t* rp,
                     const int32_t* dslot, double* W, double* uinv, int* bad, hipStream_t st) {
  if (p1 <= p0) return;
  k_ilu_rows<<<nblocks(p1 - p0, kBlock), kBlock, 0, st>>>(p0, p1, fperm, A.sptr, A.col, rp, dslot, W, uinv,
                                                          bad);
}

template <class T>
void launch_ilu_pack(const Sell& A, const int32_t* rp, const int32_t* dslot, const double* W, const double* uinv,
                     const int32_t* fperm, const int32_t* bperm, SellT<T>& Lf, SellT<T>& Ub, T* uinv_t,
                     hipStream_t st) {
  const int nb = A.nrows;
  const int nl = Lf.nslices * 64, nu = Ub.nslices * 64;
  k_ilu_pack_sell<T><<<nblocks(nl, kBlock), kBlock, 0, st>>>(nb, nl, fperm, 1, A.sptr, A.col, rp, dslot, W,
                                                             Lf.sptr, Lf.col, Lf.val);
  k_ilu_pack_sell<T><<<nblocks(nu, kBlock), kBlock, 0, st>>>(nb, nu, bperm, 0, A.sptr, A.col, rp, dslot, W,
                                                             Ub.sptr, Ub.col, Ub.val);
  k_ilu_pack_uinv<T><<<nblocks(nu, kBlock), kBlock, 0, st>>>(nb, nu, bperm, uinv, uinv_t);
}

// A's 3x3 blocks into SELL-64 slots, one thread per row of the whole slices
// [r0, r_end): the blocks of those rows (from q0 = rp[r0] on) are staged in
// ci_chunk / v_chunk in CSR order.  Padding slots get the row's own column
// (column 0 in padding rows) and a zero block, as every SELL-64 operator here.
__global__ __launch_bounds__(kBlock) void k_bsr_to_sell(int nrows, int r0, int r_end,
                                                        const int32_t* __restrict__ rp, int32_t q0,
                                                        const int32_t* __restrict__ ci_chunk,
                                                        const double* __restrict__ v_chunk,
                                                        const int32_t* __restrict__ sptr,
                                                        int32_t* __restrict__ col, double* __restrict__ val) {
  const int row = r0 + blockIdx.x * kBlock + threadIdx.x;
  if (row >= r_end) return;
  const int s = row >> 6, lane = row & 63;
  const bool live = row < nrows;
  const int n = live ? rp[row + 1] - rp[row] : 0;
  const int64_t qb = live ? (int64_t)rp[row] - q0 : 0;
  const int w = sptr[s + 1] - sptr[s];
  for (int k = 0; k < w; ++k) {
    const size_t slot = (size_t)sptr[s] + k;
    const bool real = k < n;
    col[slot * 64 + lane] = real ? ci_chunk[qb + k] : (live ? row : 0);
#pragma unroll
    for (int e = 0; e < 9; ++e) val[(slot * 9 + e) * 64 + lane] = real ? v_chunk[(qb + k) * 9 + e] : 0.0;
  }
}

void launch_bsr_to_sell(int nrows, int r0, int r_end, const int32_t* rp, int32_t q0, const int32_t* ci_chunk,
                        const double* v_chunk, Sell& A, hipStream_t st) {
  if (r_end <= r0) return;
  k_bsr_to_sell<<<nblocks(r_end - r0, kBlock), kBlock, 0, st>>>(nrows, r0, r_end, rp, q0, ci_chunk, v_chunk,
                                                                A.sptr, A.col, A.val);
}

// reduced elliptic blocks Ahat_ij = A_ij[E,E] - W_i A_ij[H,E] (Sec. 5.2) in
// A's SELL-64 slots: one thread per row, ne*ne values per slot.  Products are
// rounded before each subtraction, in the order t = 0, 1, ..., so the values
// are the ones the host computes (and, in FP32, their rounding).  Padding
// slots hold zero blocks and give zero blocks.
template <class T>
__global__ __launch_bounds__(kBlock) void k_sell_ahat(int nrows, int nslices, const int32_t* __restrict__ sptr,
                                                      const double* __restrict__ aval,
                                                      const double* __restrict__ W, int ne, int e0, int e1,
                                                      int h0, int h1, T* __restrict__ out) {
#pragma clang fp contract(off)
  const int row = blockIdx.x * kBlock + threadIdx.x;
  const int s = row >> 6, lane = row & 63;
  if (s >= nslices) return;
  const int nh = 3 - ne;
  const int eidx[2] = {e0, e1}, hidx[2] = {h0, h1};
  double w[2] = {0.0, 0.0};
  if (row < nrows) {
    w[0] = W[(size_t)row * 2];
    w[1] = W[(size_t)row * 2 + 1];
  }
  const int nv = ne * ne;
  for (int q = sptr[s]; q < sptr[s + 1]; ++q) {
    const double* B = aval + (size_t)q * 9 * 64 + lane;
    for (int a = 0; a < ne; ++a)
      for (int c = 0; c < ne; ++c) {
        double v = B[(eidx[a] * 3 + eidx[c]) * 64];
        for (int t = 0; t < nh; ++t) {
          const double prod = w[a * nh + t] * B[(hidx[t] * 3 + eidx[c]) * 64];
          v = v - prod;
        }
        out[((size_t)q * nv + a * ne + c) * 64 + lane] = (T)v;
      }
  }
}

template <class T>
void launch_sell_ahat(const Sell& A, const double* W, int ne, const int32_t* eidx, const int32_t* hidx,
                      T* out, hipStream_t st) {
  if (A.nslices == 0) return;
  k_sell_ahat<T><<<nblocks((int64_t)A.nslices * 64, kBlock), kBlock, 0, st>>>(
      A.nrows, A.nslices, A.sptr, A.val, W, ne, eidx[0], ne > 1 ? eidx[1] : 0, hidx[0],
      ne < 2 ? hidx[1] : 0, out);
}

void launch_grid_ilu_diag(const Sell& A, const int32_t* fperm, int32_t p0, int32_t p1, int nx, int nxy,
                          double* uinv, int* bad, hipStream_t st) {
  if (p1 <= p0) return;
  k_grid_ilu_diag<<<nblocks(p1 - p0, kBlock), kBlock, 0, st>>>(p0, p1, fperm, A.sptr, A.col, A.val, nx, nxy,
                                                                  uinv, bad);
}

template <class T>
void launch_grid_ilu_pack(const Sell& A, int nx, int ny, const double* uinv, T* Lt, T* Ut, hipStream_t st) {
  k_grid_ilu_pack<T><<<nblocks(A.nrows, kBlock), kBlock, 0, st>>>(A.nrows, nx, ny, A.sptr, A.col, A.val, uinv,
                                                                  Lt, Ut);
}

// workgroup: the sweeping wave and the staging waves.  The forward sweep keeps
// five steps in flight from HBM; the backward sweeping wave needs more than
// 256 VGPRs in FP64, which leaves room for one wave per SIMD only (three
// stagers).  Ring slots (18 KB forward, 24 KB backward per slot in FP64; the
// FP32 slots are half that): measured on 250x250x50, rings of 6 forward and
// 4 backward slots beat the 8 and 6 that fit in LDS (the sweeps took 0.347
// and 0.510 ms against 0.356 and 0.537); with fewer slots the staging waves
// wait more and compete less with the sweeping wave for LDS.
#ifndef CPTR_GRID_STAGERS_FWD
#define CPTR_GRID_STAGERS_FWD 5
#endif
#ifndef CPTR_GRID_STAGERS_BWD
#define CPTR_GRID_STAGERS_BWD 3
#endif
#ifndef CPTR_GRID_SLOTS_FWD
#define CPTR_GRID_SLOTS_FWD 6
#endif
#ifndef CPTR_GRID_SLOTS_BWD
#define CPTR_GRID_SLOTS_BWD 4
#endif
constexpr int kGridStagersFwd = CPTR_GRID_STAGERS_FWD, kGridStagersBwd = CPTR_GRID_STAGERS_BWD;
constexpr int kGridSlotsFwd = CPTR_GRID_SLOTS_FWD, kGridSlotsBwd = CPTR_GRID_SLOTS_BWD;

template <class T>
void launch_ilu_fwd_grid(int nx, int ny, int nz, const T* Lt, const T* r2t, T* ytile, T* faces,
                         int* tickets, double* err, long spin_limit, hipStream_t st) {
  const int nJ = (ny + kTJ - 1) / kTJ, nK = (nz + kTK - 1) / kTK;
  k_ilu_grid<true, 2, kGridStagersFwd, kGridSlotsFwd, T><<<nJ * nK, 64 * (kGridStagersFwd + 1), 0, st>>>(
      nx, ny, nz, nJ, nK, Lt, r2t, ytile, faces, nullptr, 0, 0, nullptr, tickets, err, spin_limit);
}

template <class T>
void launch_ilu_bwd_grid(int nx, int ny, int nz, const T* Ut, T* ytile, const T* e0t, int ne,
                         const int32_t* eidx, T* faces, double* z, int* tickets, double* err,
                         long spin_limit, hipStream_t st) {
  const int nJ = (ny + kTJ - 1) / kTJ, nK = (nz + kTK - 1) / kTK;
  if (ne == 2)
    k_ilu_grid<false, 2, kGridStagersBwd, kGridSlotsBwd, T><<<nJ * nK, 64 * (kGridStagersBwd + 1), 0, st>>>(
        nx, ny, nz, nJ, nK, Ut, ytile, nullptr, faces, e0t, eidx[0], eidx[1], z, tickets, err, spin_limit);
  else
    k_ilu_grid<false, 1, kGridStagersBwd, kGridSlotsBwd, T><<<nJ * nK, 64 * (kGridStagersBwd + 1), 0, st>>>(
        nx, ny, nz, nJ, nK, Ut, ytile, nullptr, faces, e0t, eidx[0], 0, z, tickets, err, spin_limit);
}

int ilu_sf_width(int max_width) {
  if (max_width <= 4) return 4;
  if (max_width <= 8) return 8;
  if (max_width <= 16) return 16;
  return 0;
}

template <class T>
void launch_ilu_fwd_sf(const SellT<T>& L, int width, const int32_t* perm, const T* r2, T* y,
                       int* tickets, double* err, long spin_limit, hipStream_t st) {
  const int g = nblocks(L.nrows, kBlock);
  switch (width) {
    case 4: k_ilu_fwd_sf<4, T><<<g, kBlock, 0, st>>>(L.nrows, L.sptr, L.col, L.val, perm, r2, y, tickets, err, spin_limit); break;
    case 8: k_ilu_fwd_sf<8, T><<<g, kBlock, 0, st>>>(L.nrows, L.sptr, L.col, L.val, perm, r2, y, tickets, err, spin_limit); break;
    default: k_ilu_fwd_sf<16, T><<<g, kBlock, 0, st>>>(L.nrows, L.sptr, L.col, L.val, perm, r2, y, tickets, err, spin_limit); break;
  }
}

template <class T>
void launch_ilu_bwd_sf(const SellT<T>& U, int width, const int32_t* perm, const T* uinv,
                       const T* y, const T* e0, int ne, const int32_t* eidx, T* x2,
                       double* z, int* tickets, double* err, long spin_limit, hipStream_t st) {
  const int g = nblocks(U.nrows, kBlock);
  const int npad = U.nslices * 64;
#define BWD(WW, NN) k_ilu_bwd_sf<WW, NN, T><<<g, kBlock, 0, st>>>(U.nrows, npad, U.sptr, U.col, U.val, perm, uinv, y, e0, eidx[0], NN == 2 ? eidx[1] : 0, x2, z, tickets, err, spin_limit)
  if (ne == 2) {
    if (width == 4) BWD(4, 2); else if (width == 8) BWD(8, 2); else BWD(16, 2);
  } else {
    if (width == 4) BWD(4, 1); else if (width == 8) BWD(8, 1); else BWD(16, 1);
  }
#undef BWD
}

#define MAXV_DISPATCH(KERNEL, nv, ...)                                                     \
  do {                                                                                     \
    if ((nv) == 1) KERNEL<1><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);                  \
    else if ((nv) == 2) KERNEL<2><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) == 3) KERNEL<3><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) == 4) KERNEL<4><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) == 5) KERNEL<5><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) == 6) KERNEL<6><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) == 7) KERNEL<7><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) == 8) KERNEL<8><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);             \
    else if ((nv) <= 16) KERNEL<16><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);           \
    else if ((nv) <= 32) KERNEL<32><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);           \
    else KERNEL<64><<<kRedBlocks, kBlock, 0, st>>>(__VA_ARGS__);                           \
  } while (0)

void launch_mdot(int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* part,
                 hipStream_t st) {
  if (nv <= 0) return;  // callers pass 1 <= nv <= 64; the kernel reads column nv - 1
  MAXV_DISPATCH(k_mdot, nv, n, nv, V, ldv, w, part);
}
void launch_maxpy_dot(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                      double* w, double* part, hipStream_t st) {
  if (nv <= 0) return;  // callers pass 1 <= nv <= 64; the kernel reads column nv - 1
  MAXV_DISPATCH(k_maxpy_dot, nv, n, nv, V, ldv, coef, w, part);
}
void launch_maxpy_norm(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                       double* w, double* part, hipStream_t st) {
  if (nv <= 0) return;  // callers pass 1 <= nv <= 64; the kernel reads column nv - 1
  MAXV_DISPATCH(k_maxpy_norm, nv, n, nv, V, ldv, coef, w, part);
}
void launch_reduce(int ncols, const double* part, double* out, int add_to_out, hipStream_t st) {
  k_reduce<<<ncols, kBlock, 0, st>>>(ncols, part, out, add_to_out);
}
void launch_scale(int64_t n, const double* w, const double* nrm2, double* v, hipStream_t st) {
  k_scale<<<kRedBlocks, kBlock, 0, st>>>(n, w, nrm2, v);
}
void launch_scale_host(int64_t n, const double* w, double s, double* v, hipStream_t st) {
  k_scale_host<<<kRedBlocks, kBlock, 0, st>>>(n, w, s, v);
}
void launch_norm2(int64_t n, const double* x, double* part, hipStream_t st) {
  k_norm2<<<kRedBlocks, kBlock, 0, st>>>(n, x, part);
}
void launch_update_host_coef(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                             double* x, hipStream_t st) {
  if (nv <= 0 || n <= 0) return;  // nothing to add (the kernel reads column nv - 1)
  Coef64 c;
  for (int j = 0; j < 64; ++j) c.c[j] = j < nv ? coef[j] : 0.0;
  MAXV_DISPATCH(k_update, nv, n, nv, V, ldv, c, x);
}

// the preconditioner runs in FP64 or, in the mixed-precision mode, in FP32
#define CPTR_PREC_LAUNCHERS(T)                                                                      \
  template void launch_l0_restrict<T>(int32_t, int, const double*, const double*, const int32_t*,   \
                                      const int32_t*, T*, const T*, T*, hipStream_t);                 \
  template void launch_l0_resid<T>(const SellT<T>&, int, const T*, const T*, T*, hipStream_t);        \
  template void launch_l0_post<T>(const SellT<T>&, int, const T*, const T*, const T*, T*, hipStream_t); \
  template void launch_csr_resid<T>(const DCsrT<T>&, const T*, const T*, T*, hipStream_t);           \
  template void launch_csr_spmv<T>(const DCsrT<T>&, const T*, T*, hipStream_t);                      \
  template void launch_csr_restrict<T>(const DCsrT<T>&, const T*, const T*, T*, T*, hipStream_t);    \
  template void launch_csr_prolong<T>(const DCsrT<T>&, const T*, const T*, const T*, T*, hipStream_t); \
  template void launch_csr_prolong_add<T>(const DCsrT<T>&, const T*, const T*, T*, hipStream_t);     \
  template void launch_csr_post<T>(const DCsrT<T>&, const T*, const T*, const T*, T*, hipStream_t);  \
  template void launch_sell_resid<T>(const SellT<T>&, const T*, const T*, T*, hipStream_t);          \
  template void launch_sell_post<T>(const SellT<T>&, const T*, const T*, const T*, T*, hipStream_t); \
  template void launch_coarse_solve<T>(int, const double*, const int32_t*, const T*, T*, hipStream_t); \
  template void launch_blk_csr<T>(int, int, int, const DCsrT<T>*, const T*, const double*,            \
                                  const double*, double*, hipStream_t);                              \
  template void launch_blk_to<T>(int64_t, const double*, T*, hipStream_t);                           \
  template void launch_dense_gemv<T>(int, const T*, const T*, T*, hipStream_t);                      \
  template void launch_stage2_resid<T>(const Sell&, int, const int32_t*, const T*, const double*, T*, \
                                       hipStream_t);                                                 \
  template void launch_ilu_fwd_level<T>(const SellT<T>&, const int32_t*, int32_t, int32_t, const T*, \
                                        T*, hipStream_t);                                            \
  template void launch_ilu_bwd_level<T>(const SellT<T>&, const int32_t*, const T*, int32_t, int32_t,  \
                                        const T*, const T*, int, const int32_t*, T*, double*,        \
                                        hipStream_t);                                                \
  template void launch_prolong_e<T>(int32_t, int, const int32_t*, const T*, double*, hipStream_t);   \
  template void launch_stage2_grid<T>(int, int, int, const Sell&, int, const int32_t*, const T*,     \
                                      const double*, T*, T*, T*, int*, hipStream_t);                 \
  template void launch_grid_ilu_pack<T>(const Sell&, int, int, const double*, T*, T*, hipStream_t);  \
  template void launch_ilu_pack<T>(const Sell&, const int32_t*, const int32_t*, const double*,       \
                                   const double*, const int32_t*, const int32_t*, SellT<T>&, SellT<T>&, \
                                   T*, hipStream_t);                                                 \
  template void launch_sell_ahat<T>(const Sell&, const double*, int, const int32_t*, const int32_t*,  \
                                    T*, hipStream_t);                                                 \
  template void launch_ilu_fwd_grid<T>(int, int, int, const T*, const T*, T*, T*, int*, double*, long, \
                                       hipStream_t);                                                 \
  template void launch_ilu_bwd_grid<T>(int, int, int, const T*, T*, const T*, int, const int32_t*, T*, \
                                       double*, int*, double*, long, hipStream_t);                   \
  template void launch_stage2_resid_sf<T>(const Sell&, int, const int32_t*, const T*, const double*,  \
                                          T*, T*, T*, int*, hipStream_t);                            \
  template void launch_ilu_fwd_sf<T>(const SellT<T>&, int, const int32_t*, const T*, T*, int*,       \
                                     double*, long, hipStream_t);                                    \
  template void launch_ilu_bwd_sf<T>(const SellT<T>&, int, const int32_t*, const T*, const T*,       \
                                     const T*, int, const int32_t*, T*, double*, int*, double*, long, \
                                     hipStream_t);
CPTR_PREC_LAUNCHERS(double)
CPTR_PREC_LAUNCHERS(float)
#undef CPTR_PREC_LAUNCHERS

}  // namespace cptr
