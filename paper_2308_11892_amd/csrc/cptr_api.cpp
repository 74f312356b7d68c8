// cptr_api.cpp -- C ABI of the CPTR library: setup, apply, (F)GMRES solve.
//
// Device work for one preconditioner application (Eq. 3 of the paper):
//   b0 = R_QI r                              quasi-IMPES restriction (Sec. 5.2)
//   e0 = one V-cycle on Ahat b0              system AMG, (p, T) block (Sec. 3.1, 3.2)
//   r2 = r - A P_E e0                        stage-two residual
//   z  = P_E e0 + U^-1 L^-1 r2               ILU(0) on the full system (Sec. 3.1)
// The solver is right-preconditioned restarted GMRES (Sec. 3) with classical
// Gram-Schmidt applied twice on the device and the Hessenberg least-squares
// problem updated by Givens rotations on the host in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "cptr.h"
#include "dev_arena.hpp"
#include "host_setup.hpp"
#include "kernels.hpp"
#include "solver_internal.hpp"

using namespace cptr;

namespace {

thread_local std::string g_setup_error;

// ---------------------------------------------------------------------------
// Large copies between pageable host memory and the device.  Copies from or
// to pageable memory run well below the link's rate (the runtime stages them
// itself; ~4 GB/s device to host, ~22 GB/s host to device here), so large ones
// go through pinned buffers in chunks: the DMA of one chunk overlaps the host
// copy of the next (or the previous) one, and the host copies are split over
// threads.  The pinned buffers live as long as the process and are shared by
// the setups in flight on a device, one pair each (a pair's events belong to
// the device it was made on).
namespace staged {

constexpr size_t kChunk = size_t(16) << 20;  // bytes per chunk and buffer
constexpr size_t kDirect = size_t(2) << 20;  // smaller copies go direct

struct Pair {
  int device = -1;
  char* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
};

std::mutex g_mu;
std::vector<Pair> g_free;  // idle pairs

// a pair for the current device (false: copy directly)
bool take(Pair& p) {
  if (hipGetDevice(&p.device) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  {
    std::lock_guard<std::mutex> g(g_mu);
    for (size_t k = 0; k < g_free.size(); ++k)
      if (g_free[k].device == p.device) {
        p = g_free[k];
        g_free.erase(g_free.begin() + (ptrdiff_t)k);
        return true;
      }
  }
  for (int b = 0; b < 2; ++b) {
    void* q = nullptr;
    if (hipHostMalloc(&q, kChunk, hipHostMallocDefault) != hipSuccess ||
        (p.buf[b] = static_cast<char*>(q), hipEventCreateWithFlags(&p.ev[b], hipEventDisableTiming)) != hipSuccess) {
      (void)hipGetLastError();
      for (int c = 0; c <= b; ++c) {
        if (p.buf[c]) (void)hipHostFree(p.buf[c]);
        if (p.ev[c]) (void)hipEventDestroy(p.ev[c]);
      }
      return false;
    }
  }
  return true;
}

void give(const Pair& p) {
  std::lock_guard<std::mutex> g(g_mu);
  g_free.push_back(p);
}

// dst[0, n) = src[0, n) on the host, split over threads in pieces of >= 1 MB
void host_copy(char* dst, const char* src, size_t n, int threads) {
  const int64_t pieces = std::max<int64_t>(1, std::min<int64_t>(threads, (int64_t)(n >> 20)));
  if (pieces == 1) {
    std::memcpy(dst, src, n);
    return;
  }
  std::vector<std::thread> th;
  for (int64_t k = 1; k < pieces; ++k)
    th.emplace_back([=] {
      const size_t lo = n * k / pieces, hi = n * (k + 1) / pieces;
      std::memcpy(dst + lo, src + lo, hi - lo);
    });
  std::memcpy(dst, src, n / pieces);
  for (auto& t : th) t.join();
}

// device -> pageable host, after the stream's earlier work; complete on return
hipError_t to_host(void* dst, const void* src, size_t n, hipStream_t st, int threads) {
  hipError_t e;
  Pair p;
  if (n < kDirect || !take(p)) {
    if ((e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    return hipStreamSynchronize(st);
  }
  char* d = static_cast<char*>(dst);
  const char* q = static_cast<const char*>(src);
  const size_t nc = (n + kChunk - 1) / kChunk;
  auto len = [&](size_t i) { return std::min(kChunk, n - i * kChunk); };
  e = hipSuccess;
  for (size_t i = 0; i <= nc && e == hipSuccess; ++i) {
    // chunk i's DMA goes out before the host copies chunk i - 1 (buffer
    // (i - 1) & 1); chunk i + 1 reuses buffer (i + 1) & 1 only after that copy
    if (i < nc) {
      e = hipMemcpyAsync(p.buf[i & 1], q + i * kChunk, len(i), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipEventRecord(p.ev[i & 1], st);
    }
    if (i > 0 && e == hipSuccess) {
      e = hipEventSynchronize(p.ev[(i - 1) & 1]);
      if (e == hipSuccess) host_copy(d + (i - 1) * kChunk, p.buf[(i - 1) & 1], len(i - 1), threads);
    }
  }
  if (e != hipSuccess) (void)hipStreamSynchronize(st);  // no DMA left into the pair
  give(p);
  return e;
}

// pageable host -> device on the stream; the source may die on return (the
// copies into pinned memory are done, and the DMAs complete before return)
hipError_t to_device(void* dst, const void* src, size_t n, hipStream_t st, int threads) {
  hipError_t e;
  Pair p;
  if (n < kDirect || !take(p)) {
    if ((e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    return hipStreamSynchronize(st);
  }
  char* d = static_cast<char*>(dst);
  const char* q = static_cast<const char*>(src);
  const size_t nc = (n + kChunk - 1) / kChunk;
  e = hipSuccess;
  for (size_t i = 0; i < nc && e == hipSuccess; ++i) {
    const size_t m = std::min(kChunk, n - i * kChunk);
    // buffer i & 1 is free once chunk i - 2's DMA is done
    if (i >= 2) e = hipEventSynchronize(p.ev[i & 1]);
    if (e != hipSuccess) break;
    host_copy(p.buf[i & 1], q + i * kChunk, m, threads);
    e = hipMemcpyAsync(d + i * kChunk, p.buf[i & 1], m, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(p.ev[i & 1], st);
  }
  const hipError_t s2 = hipStreamSynchronize(st);
  give(p);
  return e != hipSuccess ? e : s2;
}

}  // namespace staged

constexpr int kMaxRestart = 64;
// Rounds a wave of the one-launch sweeps polls before it gives up and raises
// the wait-limit flag (seconds of waiting; never reached when the schedule is
// valid).
constexpr long kSweepSpinLimit = 1L << 22;
constexpr int kPhases = 9;
enum Phase { PH_SPMV = 0, PH_RESTRICT, PH_VC0, PH_VCC, PH_STAGE2, PH_ILU_F, PH_ILU_B, PH_ARNOLDI, PH_UPDATE };

struct HostSell {
  int32_t nrows = 0, nslices = 0, nv = 0;
  std::vector<int32_t> sptr, col;
  std::vector<double> val;
};

// run body(lo, hi) over [0, n) split into `threads` contiguous ranges
template <class Body>
void parallel_ranges(int64_t n, int threads, Body body) {
  const int t = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n / 4096));
  if (t <= 1) {
    body((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  for (int k = 0; k < t; ++k) th.emplace_back(body, n * k / t, n * (k + 1) / t);
  for (auto& x : th) x.join();
}

// Pack rows (or positions) into SELL-64; len(r) blocks per row, fill(r, k, col, vals).
// With sizes_only only the slice pointers are built (col and val stay empty).
template <class Len, class Fill>
HostSell pack_sell(int32_t nrows, int nv, Len len, Fill fill, int32_t pad_col_mode, bool sizes_only,
                   int threads) {
  HostSell s;
  s.nrows = nrows;
  s.nv = nv;
  s.nslices = (nrows + kLanes - 1) / kLanes;
  s.sptr.assign(s.nslices + 1, 0);
  for (int32_t sl = 0; sl < s.nslices; ++sl) {
    int32_t w = 0;
    for (int l = 0; l < kLanes; ++l) {
      const int32_t r = sl * kLanes + l;
      if (r < nrows) w = std::max<int32_t>(w, len(r));
    }
    s.sptr[sl + 1] = s.sptr[sl] + w;
  }
  const int64_t slots = s.sptr[s.nslices];
  if (sizes_only) return s;
  s.col.assign((size_t)slots * kLanes, 0);
  s.val.assign((size_t)slots * kLanes * nv, 0.0);
  parallel_ranges(s.nslices, threads, [&](int64_t s0, int64_t s1) {
  for (int32_t sl = (int32_t)s0; sl < (int32_t)s1; ++sl) {
    const int32_t w = s.sptr[sl + 1] - s.sptr[sl];
    for (int l = 0; l < kLanes; ++l) {
      const int32_t r = sl * kLanes + l;
      const int32_t n = r < nrows ? len(r) : 0;
      for (int32_t k = 0; k < w; ++k) {
        const int64_t slot = (int64_t)s.sptr[sl] + k;
        double vals[9] = {0};
        int32_t c;
        if (k < n) {
          fill(r, k, c, vals);
        } else {
          c = pad_col_mode < 0 ? -1 : (r < nrows ? r : 0);  // padding: own row, zero block
        }
        s.col[(size_t)slot * kLanes + l] = c;
        for (int e = 0; e < nv; ++e) s.val[((size_t)slot * nv + e) * kLanes + l] = k < n ? vals[e] : 0.0;
      }
    }
  }
  });
  return s;
}

// Device operators and workspace of the preconditioner in its value type T
// (double, or float in the mixed-precision mode).
template <class T>
struct PrecDev {
  SellT<T> Ahat, Lf, Ub;     // elliptic blocks; ILU factors by dependency level
  T* uinv = nullptr;         // U_ii^-1 per level-sorted position
  T* Lg = nullptr;           // L blocks (-x, -y, -z), tile layout of the forward sweep
  T* Ug = nullptr;           // U blocks (+x, +y, +z) and U_ii^-1, tile layout of the backward sweep
  T* ytile = nullptr;        // forward-sweep results in the backward tile layout
  T* r2tile = nullptr;       // stage-two residual in the forward tile layout
  T* e0tile = nullptr;       // V-cycle result in the backward tile layout
  T* faces = nullptr;        // face buffers of the forward then the backward grid sweep
  struct Lev {
    DCsrT<T> A, P, R;
    SellT<T> As;             // A in SELL-64 instead (levels of many short rows)
    bool sell = false;
    T* dinv = nullptr;
    T *b = nullptr, *r = nullptr, *x = nullptr, *e = nullptr;
    T* t = nullptr;          // second iterate of the smoothing sweeps (num_sweeps > 1)
    int32_t n = 0;
  };
  std::vector<Lev> lev;
  T *r2 = nullptr, *y = nullptr, *x2 = nullptr;  // apply workspace
  // the V-cycle below level `tail` (0: none) as one dense operator, row-major
  // n_tail x n_tail (kernels.hip, "the bottom of the V-cycle")
  int tail = 0;
  T* tailB = nullptr;
};

}  // namespace

// AMG construction steps a setup did on the device (levels)
struct SetupSiteCounts {
  int strength = 0, interp = 0, galerkin = 0, multipass = 0, strength2 = 0;
  int split = 0;              // first passes begun on the device
  int hmis = 0;               // splits over several HMIS blocks on the device
  int64_t split_points = 0;   // points those decided on the device
  int64_t first_points = 0;   // points of all first passes of a one-block split
};

struct cptr_solver_s {
  HostSetup host;
  bool device = false;
  int ilu_mode = CPTR_ILU_SWEEP_AUTO;
  std::string err;
  double setup_s = 0.0;
  double device_build_s = 0.0;  // wall time of the device half (both parts)
  bool dev_a_done = false;      // the device half's first part was built during setup_host
  int ne = 2;
  int nsweeps = 1;           // l1-Jacobi sweeps before and after the coarse correction
  int dense_tail = 0;        // largest level whose cycle below runs as one dense operator
  int max_restart = 0;       // Krylov space of cptr_setup (cptr_setup_opts.max_restart)
  bool flex_space = false;   // ... with the FGMRES vectors Z
  int32_t eidx_h[3] = {0, 1, 2}, hidx_h[3] = {2, 0, 0};
  int64_t N = 0;  // DOF
  std::vector<void*> allocs;
  DevArena* arena = nullptr;  // device memory comes from here when set (serving)
  bool measure = false;       // count device bytes only: no allocation, copy or launch
  std::vector<int64_t>* plan = nullptr;  // measure mode: the build's allocations (+bytes) and
                                         // releases (-1 - index of the allocation), in order
  int threads = 1;            // host threads for packing device layouts
  int64_t dev_bytes = 0;      // device bytes held (or counted), in DevArena pieces
  // device operators shared by both precisions
  Sell A;
  double* W = nullptr;
  int32_t* fperm = nullptr;
  int32_t* bperm = nullptr;
  std::vector<int32_t> flev_ptr, blev_ptr;
  int sf_width = 0;          // register slots of the one-launch sweeps; 0 = per-level launches
  int grid[3] = {0, 0, 0};   // nx, ny, nz when A is a 7-point stencil in lexicographic order
  bool use_grid = false;     // tiled systolic sweeps on that grid
  bool device_ilu = false;   // ILU(0) factored on the device (every device handle; no host factors)
  SetupSiteCounts device_steps;        // AMG construction steps done on the device
  int32_t agg_levels_used = 0;         // levels with the aggressive (multipass) interpolation
  int* tickets = nullptr;    // [2] workgroup ticket counters of the one-launch sweeps
  double* coarse_lu = nullptr;
  int32_t* coarse_piv = nullptr;
  int32_t ncoarse = 0;
  // the preconditioner in FP64 or FP32 (cptr_setup_opts.precond_precision)
  int prec = CPTR_PRECISION_FP64;
  PrecDev<double> p64;
  PrecDev<float> p32;
  // solve workspace
  int restart_cap = 0;
  bool have_z = false;
  double* V = nullptr;
  double* Z = nullptr;
  int64_t ldv = 0;
  double *wr = nullptr, *wt = nullptr, *wu = nullptr;
  double* part = nullptr;
  double* hdev = nullptr;   // [0,64): first CGS pass, [64,128): second, [128]: ||w||^2,
                            // [136]: scratch norm, [140]: sweep wait-limit flag
  double* hhost = nullptr;  // pinned copy
  double* sweep_flag = nullptr;  // where the sweeps raise the wait-limit flag (hdev + 140,
                                 // or the static scratch's slot during cptr_gmres_solve_static)
  // profiling
  bool profiling = false;
  uint32_t profile_mask = 0;  // phases timed while profiling
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  hipEvent_t ev_copy = nullptr;  // marks the Hessenberg column's copy to the host
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double phase_ms[kPhases] = {0};
  int64_t phase_cnt[kPhases] = {0};
};

namespace {

int fail(cptr_solver s, int code, const std::string& msg) {
  if (s) s->err = msg;
  else g_setup_error = msg;
  return code;
}

int hip_fail(cptr_solver s, hipError_t e, const char* what) {
  return fail(s, CPTR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(s, call)                                  \
  do {                                                    \
    hipError_t _e = (call);                               \
    if (_e != hipSuccess) return (cptr_status)hip_fail((s), _e, #call); \
  } while (0)

// In measure mode pointers are this placeholder: never dereferenced, never
// passed to a kernel or a copy.
char g_measure_placeholder[DevArena::kAlign];

template <class T>
int dalloc(cptr_solver s, T*& p, int64_t count) {
  p = nullptr;
  if (count <= 0) count = 1;
  const size_t bytes = sizeof(T) * (size_t)count;
  if (s->measure) {
    s->dev_bytes += (int64_t)DevArena::round(bytes);
    p = reinterpret_cast<T*>(g_measure_placeholder);
    if (s->plan) {
      // a distinct stand-in per allocation, so that its release can be
      // recorded; never dereferenced, never passed to a kernel or a copy
      const int64_t k = (int64_t)s->allocs.size();
      void* q = reinterpret_cast<void*>((uintptr_t(1) << 44) + (uintptr_t)k * DevArena::kAlign);
      s->allocs.push_back(q);
      s->plan->push_back((int64_t)DevArena::round(bytes));
      p = static_cast<T*>(q);
    }
    return CPTR_OK;
  }
  void* q = nullptr;
  if (s->arena) {
    q = s->arena->alloc(bytes);
    if (!q)
      return fail(s, CPTR_E_NOMEM, "HBM arena has no free piece of " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(s, CPTR_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  s->allocs.push_back(q);
  s->dev_bytes += (int64_t)DevArena::round(bytes);
  p = static_cast<T*>(q);
  return CPTR_OK;
}

// returns one allocation of the handle (to the arena when there is one)
void dfree(cptr_solver s, void* p) {
  auto it = std::find(s->allocs.begin(), s->allocs.end(), p);
  if (it == s->allocs.end()) return;
  if (s->measure) {  // a recorded plan: stand-ins are never released
    if (s->plan) s->plan->push_back(-1 - (int64_t)(it - s->allocs.begin()));
    return;
  }
  s->allocs.erase(it);
  if (s->arena) (void)s->arena->release(p);
  else (void)hipFree(p);
}

void dfree_all(cptr_solver s) {
  for (void* p : s->allocs) {
    if (s->arena) (void)s->arena->release(p);
    else (void)hipFree(p);
  }
  s->allocs.clear();
  s->dev_bytes = 0;
}

template <class T>
int upload(cptr_solver s, T*& p, const T* src, int64_t count, hipStream_t st) {
  int rc = dalloc(s, p, count);
  if (rc) return rc;
  // on the build's stream, which the kernels reading p use too, and complete
  // before returning: the host staging vectors die right after the upload
  if (count > 0 && !s->measure) HIP_TRY(s, staged::to_device(p, src, sizeof(T) * (size_t)count, st, s->threads));
  return CPTR_OK;
}

// FP64 host values uploaded as T (rounded to nearest when T is float)
template <class T>
int upload_as(cptr_solver s, T*& p, const double* src, int64_t count, hipStream_t st) {
  if constexpr (std::is_same<T, double>::value) {
    return upload(s, p, src, count, st);
  } else {
    if (s->measure) return dalloc(s, p, count);
    std::vector<T> tmp((size_t)count);
    parallel_ranges(count, s->threads, [&](int64_t lo, int64_t hi) {
      for (int64_t q = lo; q < hi; ++q) tmp[(size_t)q] = (T)src[q];
    });
    return upload(s, p, tmp.data(), count, st);
  }
}

template <class T>
int upload_sell(cptr_solver s, SellT<T>& d, const HostSell& h, hipStream_t st) {
  d.nrows = h.nrows;
  d.nslices = h.nslices;
  d.nv = h.nv;
  d.nslots = h.sptr.back();
  int rc;
  if ((rc = upload(s, d.sptr, h.sptr.data(), (int64_t)h.sptr.size(), st))) return rc;
  const int64_t slots = h.sptr.back();
  if ((rc = upload(s, d.col, h.col.data(), slots * kLanes, st))) return rc;
  if ((rc = upload_as(s, d.val, h.val.data(), slots * kLanes * h.nv, st))) return rc;
  return CPTR_OK;
}

// lanes per row of the scalar CSR kernels: about four nonzeros per lane, so
// each lane keeps several independent index/value/gather loads in flight
int pick_group(int64_t nnz, int32_t n) {
  const double avg = n > 0 ? (double)nnz / n / 4.0 : 1.0;
  int g = 1;
  while (g < 32 && g < avg) g <<= 1;
  return g;
}

template <class T>
int upload_csr(cptr_solver s, DCsrT<T>& d, const Csr& h, hipStream_t st) {
  d.n = h.n;
  d.m = h.m;
  d.nnz = h.nnz();
  if (d.nnz >= INT32_MAX) return fail(s, CPTR_E_INVALID, "AMG level too large for 32-bit offsets");
  std::vector<int32_t> rp32(h.rp.begin(), h.rp.end());
  d.group = pick_group(d.nnz, d.n);
  int rc;
  if ((rc = upload(s, d.rp, rp32.data(), (int64_t)rp32.size(), st))) return rc;
  if ((rc = upload(s, d.ci, h.ci.data(), (int64_t)h.ci.size(), st))) return rc;
  if ((rc = upload_as(s, d.v, h.v.data(), (int64_t)h.v.size(), st))) return rc;
  return CPTR_OK;
}

// A coarse level's operator: SELL-64 (one thread per row, fully coalesced)
// for many short rows of similar length, where the slices pad by at most
// 10 %; otherwise CSR with several lanes per row, which keeps enough loads in
// flight for long rows and small levels.
template <class Lev>
int upload_level_op(cptr_solver s, Lev& dl, const Csr& h, hipStream_t st) {
  const int32_t n = h.n;
  auto len = [&](int32_t r) { return (int32_t)(h.rp[r + 1] - h.rp[r]); };
  int64_t padded = 0;
  int32_t maxlen = 0;
  for (int32_t a = 0; a < n; a += kLanes) {
    int32_t w = 0;
    for (int32_t r = a; r < std::min(n, a + kLanes); ++r) w = std::max(w, len(r));
    padded += (int64_t)w * kLanes;
    maxlen = std::max(maxlen, w);
  }
  dl.sell = n >= (1 << 18) && maxlen <= 32 && padded <= 1.1 * (double)h.nnz();
  if (!dl.sell) return upload_csr(s, dl.A, h, st);
  HostSell hs = pack_sell(
      n, 1, len,
      [&](int32_t r, int32_t k, int32_t& c, double* v) {
        const int64_t q = h.rp[r] + k;
        c = h.ci[q];
        v[0] = h.v[q];
      },
      0, s->measure, s->threads);
  return upload_sell(s, dl.As, hs, st);
}

// Is A's block pattern exactly the 7-point stencil of an nx*ny*nz grid in
// lexicographic order (x fastest)?  Requires nx, ny, nz >= 2.  (rp, ci:
// a validated pattern with sorted rows.)
bool detect_grid(int32_t nb, const int32_t* rp, const int32_t* ci, int dims[3], int threads = 1) {
  if (rp[1] - rp[0] != 4) return false;  // corner cell: itself, +x, +y, +z
  const int32_t nx = ci[rp[0] + 1] == 1 ? ci[rp[0] + 2] : 0;
  const int32_t nxy = ci[rp[0] + 3];
  if (ci[rp[0]] != 0 || ci[rp[0] + 1] != 1 || nx < 2 || nxy % nx != 0 || nxy / nx < 2) return false;
  if (nb % nxy != 0 || nb / nxy < 2) return false;
  const int32_t ny = nxy / nx, nz = nb / nxy;
  std::atomic<bool> ok{true};
  parallel_ranges(nb, threads, [&](int64_t lo, int64_t hi) {
    for (int64_t c = lo; c < hi && ok.load(std::memory_order_relaxed); ++c) {
      const int32_t x = (int32_t)(c % nx), yy = (int32_t)((c / nx) % ny), zz = (int32_t)(c / nxy);
      int32_t want[7], m = 0;
      if (zz > 0) want[m++] = (int32_t)c - nxy;
      if (yy > 0) want[m++] = (int32_t)c - nx;
      if (x > 0) want[m++] = (int32_t)c - 1;
      want[m++] = (int32_t)c;
      if (x < nx - 1) want[m++] = (int32_t)c + 1;
      if (yy < ny - 1) want[m++] = (int32_t)c + nx;
      if (zz < nz - 1) want[m++] = (int32_t)c + nxy;
      bool same = rp[c + 1] - rp[c] == m;
      for (int q = 0; q < m && same; ++q) same = ci[rp[c] + q] == want[q];
      if (!same) ok.store(false, std::memory_order_relaxed);
    }
  });
  if (!ok.load()) return false;
  dims[0] = nx;
  dims[1] = ny;
  dims[2] = nz;
  return true;
}
bool detect_grid(const HostSetup& h, int dims[3], int threads) {
  return detect_grid(h.nb, h.rp.data(), h.ci.data(), dims, threads);
}

// The grid factors computed on the device from A (see launch_grid_ilu_diag):
// U_cc^-1 level by level into a temporary FP64 array, then the tile layouts.
template <class T>
int build_grid_factors_device(cptr_solver s, PrecDev<T>& d, hipStream_t st) {
  const int nx = s->grid[0], ny = s->grid[1], nz = s->grid[2];
  const int64_t rows = grid_ntiles(ny, nz) * grid_nsteps(nx);
  const int32_t nb = s->host.nb;
  double* uinv = nullptr;
  int* bad = nullptr;
  int rc;
  if ((rc = dalloc(s, d.Lg, rows * 27 * 64)) || (rc = dalloc(s, d.Ug, rows * 36 * 64)) ||
      (rc = dalloc(s, d.ytile, rows * 3 * 64)) || (rc = dalloc(s, d.r2tile, rows * 3 * 64)) ||
      (rc = dalloc(s, d.e0tile, rows * 2 * 64)) || (rc = dalloc(s, d.faces, 2 * grid_face_values(nx, ny, nz))) ||
      (rc = dalloc(s, uinv, (int64_t)nb * 9)) || (rc = dalloc(s, bad, 1)))
    return rc;
  if (s->measure) {  // the temporaries' releases, as below
    dfree(s, uinv);
    dfree(s, bad);
    return CPTR_OK;
  }
  // every fill and copy of the build goes on `st`: a null-stream operation is
  // not ordered with the kernels of a non-blocking stream
  HIP_TRY(s, hipMemsetAsync(d.Lg, 0, sizeof(T) * (size_t)rows * 27 * 64, st));
  HIP_TRY(s, hipMemsetAsync(d.Ug, 0, sizeof(T) * (size_t)rows * 36 * 64, st));
  HIP_TRY(s, hipMemsetAsync(d.ytile, 0, sizeof(T) * (size_t)rows * 3 * 64, st));
  HIP_TRY(s, hipMemsetAsync(d.r2tile, 0, sizeof(T) * (size_t)rows * 3 * 64, st));
  HIP_TRY(s, hipMemsetAsync(d.e0tile, 0, sizeof(T) * (size_t)rows * 2 * 64, st));
  const int none = INT32_MAX;  // lives until the synchronisation below
  HIP_TRY(s, hipMemcpyAsync(bad, &none, sizeof(int), hipMemcpyHostToDevice, st));
  for (size_t l = 0; l + 1 < s->flev_ptr.size(); ++l)
    launch_grid_ilu_diag(s->A, s->fperm, s->flev_ptr[l], s->flev_ptr[l + 1], nx, nx * ny, uinv, bad, st);
  launch_grid_ilu_pack(s->A, nx, ny, uinv, d.Lg, d.Ug, st);
  HIP_TRY(s, hipGetLastError());
  int first_bad = none;
  HIP_TRY(s, hipMemcpyAsync(&first_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(s, hipStreamSynchronize(st));
  // the temporaries go back; the handle's counted footprint keeps them (peak)
  dfree(s, uinv);
  dfree(s, bad);
  if (first_bad != none)
    return fail(s, CPTR_E_ZERO_PIVOT,
                "zero ILU(0) pivot (singular diagonal block) in block row " + std::to_string(first_bad));
  return CPTR_OK;
}

// ILU(0) factors of any matrix for the level-ordered sweeps, factored on the
// device: the slice widths of Lf (forward positions) and Ub (backward
// positions) come from the host's row pointers and diagonals, the values from
// launch_ilu_rows on a copy of A's SELL values.
template <class T>
int build_ilu_factors_device(cptr_solver s, PrecDev<T>& d, const std::vector<int32_t>& fp,
                             const std::vector<int32_t>& bp, hipStream_t st) {
  const HostSetup& h = s->host;
  const int32_t nb = h.nb;
  auto nolen = [](int32_t, int32_t, int32_t&, double*) {};
  HostSell Lh = pack_sell(nb, 9, [&](int32_t p) { return h.diag[fp[p]] - h.rp[fp[p]]; }, nolen, -1, true, 1);
  HostSell Uh = pack_sell(nb, 9, [&](int32_t p) { return h.rp[bp[p] + 1] - h.diag[bp[p]] - 1; }, nolen, -1, true, 1);
  if (s->sf_width == 0 && s->ilu_mode != CPTR_ILU_SWEEP_LEVELS) {
    int maxw = 0;
    for (int32_t sl = 0; sl < Lh.nslices; ++sl) maxw = std::max(maxw, Lh.sptr[sl + 1] - Lh.sptr[sl]);
    for (int32_t sl = 0; sl < Uh.nslices; ++sl) maxw = std::max(maxw, Uh.sptr[sl + 1] - Uh.sptr[sl]);
    const int w = ilu_sf_width(maxw);
    if (s->ilu_mode == CPTR_ILU_SWEEP_ONE_LAUNCH && w == 0)
      return fail(s, CPTR_E_INVALID,
                  "rows too wide (" + std::to_string(maxw) + " blocks) for one-launch ILU sweeps");
    s->sf_width = w;
  }
  int rc;
  auto alloc_sell = [&](SellT<T>& o, const HostSell& hs) -> int {
    o.nrows = hs.nrows;
    o.nslices = hs.nslices;
    o.nv = 9;
    o.nslots = hs.sptr.back();
    int r = upload(s, o.sptr, hs.sptr.data(), (int64_t)hs.sptr.size(), st);
    if (!r) r = dalloc(s, o.col, o.nslots * kLanes);
    if (!r) r = dalloc(s, o.val, o.nslots * kLanes * 9);
    return r;
  };
  if ((rc = alloc_sell(d.Lf, Lh)) || (rc = alloc_sell(d.Ub, Uh))) return rc;
  const int64_t npad = (int64_t)Uh.nslices * kLanes;
  if ((rc = dalloc(s, d.uinv, npad * 9))) return rc;
  // temporaries: the factored copy of A, U_ii^-1 in FP64, rows, diagonal slots
  std::vector<int32_t> dslot((size_t)nb);
  for (int32_t i = 0; i < nb; ++i) dslot[i] = h.diag[i] - h.rp[i];
  double* W = nullptr;
  double* uinv = nullptr;
  int32_t* rp_d = nullptr;
  int32_t* ds_d = nullptr;
  int* bad = nullptr;
  if ((rc = dalloc(s, W, s->A.nslots * kLanes * 9)) || (rc = dalloc(s, uinv, (int64_t)nb * 9)) ||
      (rc = upload(s, rp_d, h.rp.data(), (int64_t)nb + 1, st)) ||
      (rc = upload(s, ds_d, dslot.data(), (int64_t)nb, st)) || (rc = dalloc(s, bad, 1)))
    return rc;
  if (s->measure) {  // the temporaries' releases, as below
    dfree(s, W);
    dfree(s, uinv);
    dfree(s, rp_d);
    dfree(s, ds_d);
    dfree(s, bad);
    return CPTR_OK;
  }
  const int none = INT32_MAX;  // lives until the synchronisation below
  HIP_TRY(s, hipMemcpyAsync(bad, &none, sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(s, hipMemcpyAsync(W, s->A.val, sizeof(double) * (size_t)s->A.nslots * kLanes * 9,
                            hipMemcpyDeviceToDevice, st));
  for (size_t l = 0; l + 1 < s->flev_ptr.size(); ++l)
    launch_ilu_rows(s->A, s->fperm, s->flev_ptr[l], s->flev_ptr[l + 1], rp_d, ds_d, W, uinv, bad, st);
  launch_ilu_pack(s->A, rp_d, ds_d, W, uinv, s->fperm, s->bperm, d.Lf, d.Ub, d.uinv, st);
  HIP_TRY(s, hipGetLastError());
  int first_bad = none;
  HIP_TRY(s, hipMemcpyAsync(&first_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(s, hipStreamSynchronize(st));
  // the temporaries go back; the handle's counted footprint keeps them (peak)
  dfree(s, W);
  dfree(s, uinv);
  dfree(s, rp_d);
  dfree(s, ds_d);
  dfree(s, bad);
  if (first_bad != none)
    return fail(s, CPTR_E_ZERO_PIVOT,
                "zero ILU(0) pivot (singular diagonal block) in block row " + std::to_string(first_bad));
  return CPTR_OK;
}

// The preconditioner's own operators in its value type T.
// The preconditioner's operators that need only A: Ahat and the ILU factors.
template <class T>
int build_prec_ilu(cptr_solver s, PrecDev<T>& d, const std::vector<int32_t>& fp,
                   const std::vector<int32_t>& bp, hipStream_t st) {
  const HostSetup& h = s->host;
  const int ne = h.ne;
  int rc;
  // Ahat (ne x ne blocks) in A's SELL-64 slots, formed on the device from A
  // and W (slice pointers and columns are A's)
  {
    d.Ahat.nrows = s->A.nrows;
    d.Ahat.nslices = s->A.nslices;
    d.Ahat.nv = ne * ne;
    d.Ahat.nslots = s->A.nslots;
    d.Ahat.sptr = s->A.sptr;
    d.Ahat.col = s->A.col;
    if ((rc = dalloc(s, d.Ahat.val, s->A.nslots * kLanes * ne * ne))) return rc;
    if (!s->measure) {
      launch_sell_ahat(s->A, s->W, ne, s->eidx_h, s->hidx_h, d.Ahat.val, st);
      HIP_TRY(s, hipGetLastError());
    }
  }
  // ILU factors: in the tile layouts of the grid sweeps, or by dependency
  // level for the one-launch and per-level sweeps (only one of the two is kept)
  if (s->use_grid) {
    if ((rc = build_grid_factors_device(s, d, st))) return rc;
  } else {
    if ((rc = build_ilu_factors_device(s, d, fp, bp, st))) return rc;
  }
  return CPTR_OK;
}

// The rest: the AMG hierarchy (the coarsest LU stays FP64 and is shared) and
// the sweeps' work vectors.
template <class T>
int build_prec_amg(cptr_solver s, PrecDev<T>& d, hipStream_t st) {
  const HostSetup& h = s->host;
  const int32_t nb = h.nb;
  int rc;
  const int L = (int)h.lev.size();
  d.lev.resize(L);
  for (int l = 0; l < L; ++l) {
    const AmgLevel& hl = h.lev[l];
    auto& dl = d.lev[l];
    dl.n = hl.A.n;
    // smoothed: every level but a coarsest one solved by dense LU
    const bool smoothed = l + 1 < L || h.coarse_relax;
    if (l > 0 && smoothed && (rc = upload_level_op(s, dl, hl.A, st))) return rc;
    if (l + 1 < L) {
      if ((rc = upload_csr(s, dl.P, hl.P, st))) return rc;
      if ((rc = upload_csr(s, dl.R, hl.R, st))) return rc;
    }
    if (smoothed && (rc = upload_as(s, dl.dinv, hl.dinv.data(), (int64_t)hl.dinv.size(), st))) return rc;
    if ((rc = dalloc(s, dl.b, dl.n)) || (rc = dalloc(s, dl.r, dl.n)) || (rc = dalloc(s, dl.x, dl.n)) ||
        (rc = dalloc(s, dl.e, dl.n)))
      return rc;
    if (s->nsweeps > 1 && smoothed && (rc = dalloc(s, dl.t, dl.n))) return rc;
  }
  const int64_t N = (int64_t)nb * 3;
  if (!s->use_grid && ((rc = dalloc(s, d.r2, N)) || (rc = dalloc(s, d.y, N)) || (rc = dalloc(s, d.x2, N))))
    return rc;
  // the dense bottom: the largest level l >= 1 of at most dense_tail rows
  // with a smoothed level and the coarsest LU below it (level 0 keeps its
  // block operator, a smoothed coarsest level its sweeps)
  d.tail = 0;
  if (!h.coarse_relax)
    for (int l = 1; l + 2 <= L; ++l)
      if (h.lev[l].A.n <= s->dense_tail) {
        d.tail = l;
        break;
      }
  return CPTR_OK;
}

// B = the V-cycle from level d.tail down as a dense operator: the cycle's
// passes over that level and the coarser ones (the same sweeps, residuals,
// restrictions, coarsest LU solve and prolongations as an apply, over the
// level operators of type T, in FP64) run once on the n_t unit vectors at
// once; B is then rounded to T.
template <class T>
int build_tail(cptr_solver s, PrecDev<T>& d, hipStream_t st) {
  const int t = d.tail;
  if (t <= 0) return CPTR_OK;
  const int L = (int)d.lev.size();
  const int w = d.lev[t].n;
  const int ns = s->nsweeps;
  int rc;
  if ((rc = dalloc(s, d.tailB, (int64_t)w * w))) return rc;
  // per level: right-hand sides b, iterate x, and y (a residual, or the next
  // sweep's iterate); the coarsest solves in place in b
  std::vector<double*> b((size_t)L, nullptr), x((size_t)L, nullptr), y((size_t)L, nullptr);
  for (int l = t; l < L; ++l) {
    const int64_t m = (int64_t)d.lev[l].n * w;
    if ((rc = dalloc(s, b[l], m))) return rc;
    if (l + 1 < L && ((rc = dalloc(s, x[l], m)) || (rc = dalloc(s, y[l], m)))) return rc;
  }
  auto release = [&] {
    for (int l = t; l < L; ++l) {
      dfree(s, b[l]);
      if (l + 1 < L) {
        dfree(s, x[l]);
        dfree(s, y[l]);
      }
    }
  };
  if (s->measure) {
    release();
    return CPTR_OK;
  }
  launch_blk_identity(w, b[t], st);
  for (int l = t; l + 1 < L; ++l) {
    auto& dl = d.lev[l];
    launch_blk_csr<T>(kBlkScale, dl.n, w, nullptr, dl.dinv, nullptr, b[l], x[l], st);
    for (int k = 1; k < ns; ++k) {
      launch_blk_csr<T>(kBlkJacobi, dl.n, w, &dl.A, dl.dinv, x[l], b[l], y[l], st);
      std::swap(x[l], y[l]);
    }
    launch_blk_csr<T>(kBlkResid, dl.n, w, &dl.A, nullptr, x[l], b[l], y[l], st);
    launch_blk_csr<T>(kBlkProduct, d.lev[l + 1].n, w, &dl.R, nullptr, y[l], nullptr, b[l + 1], st);
  }
  launch_blk_lu(s->ncoarse, w, s->coarse_lu, s->coarse_piv, b[L - 1], st);
  x[L - 1] = b[L - 1];
  for (int l = L - 2; l >= t; --l) {
    auto& dl = d.lev[l];
    launch_blk_csr<T>(kBlkAdd, dl.n, w, &dl.P, nullptr, x[l + 1], nullptr, x[l], st);
    for (int k = 0; k < ns; ++k) {
      launch_blk_csr<T>(kBlkJacobi, dl.n, w, &dl.A, dl.dinv, x[l], b[l], y[l], st);
      std::swap(x[l], y[l]);
    }
  }
  launch_blk_to<T>((int64_t)w * w, x[t], d.tailB, st);
  HIP_TRY(s, hipGetLastError());
  // the temporaries go back once the kernels reading them are done
  HIP_TRY(s, hipStreamSynchronize(st));
  release();
  return CPTR_OK;
}

// device-side members back to their initial (host-only) values; no freeing
void reset_device_state(cptr_solver s) {
  s->allocs.clear();
  s->dev_bytes = 0;
  s->A = Sell();
  s->W = nullptr;
  s->fperm = s->bperm = nullptr;
  s->flev_ptr.clear();
  s->blev_ptr.clear();
  s->sf_width = 0;
  s->grid[0] = s->grid[1] = s->grid[2] = 0;
  s->use_grid = false;
  s->tickets = nullptr;
  s->coarse_lu = nullptr;
  s->coarse_piv = nullptr;
  s->ncoarse = 0;
  s->p64 = PrecDev<double>();
  s->p32 = PrecDev<float>();
  s->dev_a_done = false;
  s->device_build_s = 0.0;
  s->restart_cap = 0;
  s->have_z = false;
  s->V = s->Z = nullptr;
  s->ldv = 0;
  s->wr = s->wt = s->wu = nullptr;
  s->part = nullptr;
  s->hdev = nullptr;
  s->hhost = nullptr;
  s->sweep_flag = nullptr;
}

// The device half's first part, which needs only A and the host steps that
// depend on A alone (diagonals, weights, dependency levels).
int build_device_a(cptr_solver s, hipStream_t st) {
  const HostSetup& h = s->host;
  const int32_t nb = h.nb;
  const int ne = h.ne;
  int rc;
  // A in SELL-64, natural order (FP64 in both precisions).  Slice widths come
  // from the row pointers on the host; A's columns and blocks go to the device
  // as they are, in chunks of whole slices through a staging buffer, and a
  // kernel places them in the slots.
  {
    Sell& d = s->A;
    d.nrows = nb;
    d.nslices = (nb + kLanes - 1) / kLanes;
    d.nv = 9;
    std::vector<int32_t> sptr((size_t)d.nslices + 1, 0);
    parallel_ranges(d.nslices, s->threads, [&](int64_t s0, int64_t s1) {
      for (int64_t sl = s0; sl < s1; ++sl) {
        const int32_t r0 = (int32_t)sl * kLanes, r1 = std::min(nb, r0 + kLanes);
        int32_t w = 0;
        for (int32_t r = r0; r < r1; ++r) w = std::max(w, h.rp[r + 1] - h.rp[r]);
        sptr[sl + 1] = w;
      }
    });
    int64_t max_slice_blocks = 0;
    for (int32_t sl = 0; sl < d.nslices; ++sl) {
      const int32_t r0 = sl * kLanes, r1 = std::min(nb, r0 + kLanes);
      sptr[sl + 1] += sptr[sl];
      max_slice_blocks = std::max<int64_t>(max_slice_blocks, h.rp[r1] - h.rp[r0]);
    }
    d.nslots = sptr[d.nslices];
    if ((rc = upload(s, d.sptr, sptr.data(), (int64_t)sptr.size(), st))) return rc;
    if ((rc = dalloc(s, d.col, d.nslots * kLanes)) || (rc = dalloc(s, d.val, d.nslots * kLanes * 9)))
      return rc;
    // staging: up to 1M blocks, never more than A itself
    const int64_t cap = std::max<int64_t>(std::min<int64_t>(int64_t(1) << 20, h.rp[nb]), max_slice_blocks);
    int32_t* rp_d = nullptr;
    int32_t* ci_st = nullptr;
    double* v_st = nullptr;
    if ((rc = upload(s, rp_d, h.rp.data(), (int64_t)nb + 1, st)) || (rc = dalloc(s, ci_st, cap)) ||
        (rc = dalloc(s, v_st, cap * 9)))
      return rc;
    if (!s->measure) {
      for (int32_t s0 = 0; s0 < d.nslices;) {
        const int32_t q0 = h.rp[(int64_t)s0 * kLanes];
        int32_t s1 = s0 + 1;
        while (s1 < d.nslices && h.rp[std::min<int64_t>(nb, (int64_t)(s1 + 1) * kLanes)] - q0 <= cap) ++s1;
        const int32_t q1 = h.rp[std::min<int64_t>(nb, (int64_t)s1 * kLanes)];
        if (q1 > q0) {
          HIP_TRY(s, staged::to_device(ci_st, h.ci.data() + q0, sizeof(int32_t) * (size_t)(q1 - q0), st,
                                       s->threads));
          HIP_TRY(s, staged::to_device(v_st, h.av + (size_t)q0 * 9, sizeof(double) * 9 * (size_t)(q1 - q0), st,
                                       s->threads));
        }
        launch_bsr_to_sell(nb, s0 * kLanes, s1 * kLanes, rp_d, q0, ci_st, v_st, d, st);
        HIP_TRY(s, hipGetLastError());
        s0 = s1;
      }
      HIP_TRY(s, hipStreamSynchronize(st));
    }
    dfree(s, rp_d);
    dfree(s, ci_st);
    dfree(s, v_st);
  }
  // W padded to 2 per cell
  {
    std::vector<double> w2((size_t)nb * 2);
    parallel_ranges(nb, s->threads, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i)
        for (int t = 0; t < 2; ++t) w2[(size_t)i * 2 + t] = t < ne * h.nh ? h.W[(size_t)i * ne * h.nh + t] : 0.0;
    });
    if ((rc = upload(s, s->W, w2.data(), (int64_t)w2.size(), st))) return rc;
  }
  // ILU sweeps: positions sorted by level (stable in row order): a counting
  // sort whose threads each count, then place, one contiguous range of rows
  std::vector<int32_t> fp, bp;
  {
    auto order = [&](const std::vector<int32_t>& lvl, int32_t nl, std::vector<int32_t>& perm,
                     std::vector<int32_t>& ptr) {
      const int t = (int)std::max<int64_t>(1, std::min<int64_t>(s->threads, nb / 65536));
      std::vector<int64_t> cnt((size_t)t * nl, 0);  // [thread][level]
      auto range = [&](int k) { return std::make_pair((int64_t)nb * k / t, (int64_t)nb * (k + 1) / t); };
      auto each = [&](auto&& f) {
        std::vector<std::thread> th;
        for (int k = 1; k < t; ++k) th.emplace_back(f, k);
        f(0);
        for (auto& x : th) x.join();
      };
      each([&](int k) {
        for (int64_t i = range(k).first; i < range(k).second; ++i) ++cnt[(size_t)k * nl + lvl[i]];
      });
      ptr.assign(nl + 1, 0);
      int64_t run = 0;
      for (int32_t l = 0; l < nl; ++l) {
        ptr[l] = (int32_t)run;
        for (int k = 0; k < t; ++k) {
          const int64_t c = cnt[(size_t)k * nl + l];
          cnt[(size_t)k * nl + l] = run;
          run += c;
        }
      }
      ptr[nl] = (int32_t)run;
      perm.resize(nb);
      each([&](int k) {
        for (int64_t i = range(k).first; i < range(k).second; ++i)
          perm[cnt[(size_t)k * nl + lvl[i]]++] = (int32_t)i;
      });
    };
    order(h.fwd_level, h.n_fwd_levels, fp, s->flev_ptr);
    order(h.bwd_level, h.n_bwd_levels, bp, s->blev_ptr);
    if ((rc = dalloc(s, s->tickets, 2))) return rc;
    if (!s->measure) HIP_TRY(s, hipMemsetAsync(s->tickets, 0, 2 * sizeof(int), st));
    const bool grid = detect_grid(h, s->grid, s->threads);
    if (s->ilu_mode == CPTR_ILU_SWEEP_GRID && !grid)
      return fail(s, CPTR_E_INVALID, "ilu_sweep = GRID needs a 7-point stencil in lexicographic order");
    s->use_grid = grid && (s->ilu_mode == CPTR_ILU_SWEEP_AUTO || s->ilu_mode == CPTR_ILU_SWEEP_GRID);
    s->sf_width = 0;
    if ((rc = upload(s, s->fperm, fp.data(), nb, st))) return rc;
    if ((rc = upload(s, s->bperm, bp.data(), nb, st))) return rc;
  }
  rc = s->prec == CPTR_PRECISION_FP32 ? build_prec_ilu(s, s->p32, fp, bp, st)
                                      : build_prec_ilu(s, s->p64, fp, bp, st);
  if (rc) return rc;
  if (!s->measure) HIP_TRY(s, hipStreamSynchronize(st));
  return CPTR_OK;
}

// The rest of the device half: the AMG hierarchy and the solve's buffers.
int build_device_b(cptr_solver s, hipStream_t st) {
  const HostSetup& h = s->host;
  int rc = s->prec == CPTR_PRECISION_FP32 ? build_prec_amg(s, s->p32, st) : build_prec_amg(s, s->p64, st);
  if (rc) return rc;
  s->ncoarse = h.lev.back().A.n;
  if ((rc = upload(s, s->coarse_lu, h.coarse_lu.data(), (int64_t)h.coarse_lu.size(), st))) return rc;
  if ((rc = upload(s, s->coarse_piv, h.coarse_piv.data(), (int64_t)h.coarse_piv.size(), st))) return rc;
  rc = s->prec == CPTR_PRECISION_FP32 ? build_tail(s, s->p32, st) : build_tail(s, s->p64, st);
  if (rc) return rc;
  if ((rc = dalloc(s, s->part, (int64_t)kRedBlocks * (kMaxRestart + 2)))) return rc;
  if ((rc = dalloc(s, s->hdev, 256))) return rc;
  s->sweep_flag = s->hdev + 140;
  if (s->measure) return CPTR_OK;
  HIP_TRY(s, hipMemsetAsync(s->hdev, 0, 256 * sizeof(double), st));
  {
    void* hp = nullptr;
    HIP_TRY(s, hipHostMalloc(&hp, 256 * sizeof(double), hipHostMallocDefault));
    s->hhost = static_cast<double*>(hp);
  }
  // marks the Hessenberg column's copy to the host in each Arnoldi step
  HIP_TRY(s, hipEventCreateWithFlags(&s->ev_copy, hipEventDisableTiming));
  HIP_TRY(s, hipStreamSynchronize(st));
  return CPTR_OK;
}

int build_device(cptr_solver s, hipStream_t st) {
  int rc = build_device_a(s, st);
  return rc ? rc : build_device_b(s, st);
}

// ---------------------------------------------------------------- profiling
void ph_begin(cptr_solver s, hipStream_t st, int phase, hipEvent_t& ev) {
  ev = nullptr;
  if (!s->profiling || !(s->profile_mask & (1u << phase))) return;
  if (s->ev_used + 2 > s->ev_pool.size()) return;
  ev = s->ev_pool[s->ev_used++];
  (void)hipEventRecord(ev, st);
}
void ph_end(cptr_solver s, hipStream_t st, int phase, hipEvent_t ev0) {
  if (!s->profiling || !ev0) return;
  hipEvent_t ev1 = s->ev_pool[s->ev_used++];
  (void)hipEventRecord(ev1, st);
  s->ev_pending.push_back({phase, {ev0, ev1}});
}
void ph_harvest(cptr_solver s) {  // call after the stream is synchronised
  for (auto& p : s->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
      s->phase_ms[p.first] += ms;
      s->phase_cnt[p.first] += 1;
    }
  }
  s->ev_pending.clear();
  s->ev_used = 0;
}

// ---------------------------------------------------------------- apply
// e0 = V-cycle(R_QI r) on the elliptic block (first stage without
// prolongation), in the preconditioner's type T
// b0 = R_QI r and, with a smoothed level 0, its pre-smoothed iterate D^-1 b0
template <class T>
void enqueue_restrict(cptr_solver s, PrecDev<T>& d, const double* r, hipStream_t st) {
  auto& l0 = d.lev[0];
  const bool smoothed = d.lev.size() > 1 || s->host.coarse_relax;
  launch_l0_restrict(s->host.nb, s->ne, r, s->W, s->eidx_h, s->hidx_h, l0.b, smoothed ? l0.dinv : nullptr, l0.x,
                     st);
}
void enqueue_restrict(cptr_solver s, const double* r, hipStream_t st) {
  if (s->prec == CPTR_PRECISION_FP32)
    enqueue_restrict(s, s->p32, r, st);
  else
    enqueue_restrict(s, s->p64, r, st);
}

// `restricted`: the restriction of r is already queued on st
template <class T>
void enqueue_stage1(cptr_solver s, PrecDev<T>& d, const double* r, hipStream_t st, bool restricted) {
  const int ne = s->ne;
  const int L = (int)d.lev.size();
  auto& l0 = d.lev[0];
  hipEvent_t ev;
  if (!restricted) {
    ph_begin(s, st, PH_RESTRICT, ev);
    enqueue_restrict(s, d, r, st);
    ph_end(s, st, PH_RESTRICT, ev);
  }
  const bool relax = s->host.coarse_relax;
  if (L == 1 && !relax) {
    ph_begin(s, st, PH_VCC, ev);
    launch_coarse_solve(s->ncoarse, s->coarse_lu, s->coarse_piv, l0.b, l0.e, st);
    ph_end(s, st, PH_VCC, ev);
  } else {
    const int ns = s->nsweeps;
    // the iterate after the pre-smoothing sweeps of each level: the first
    // sweep from zero is written by the restriction to the level (x = D^-1 b),
    // further sweeps alternate between x and t
    std::vector<T*> cur((size_t)L, nullptr);
    auto presmooth = [&](int l) {
      auto& dl = d.lev[l];
      T* c = dl.x;
      for (int k = 1; k < ns; ++k) {
        T* o = c == dl.x ? dl.t : dl.x;
        if (l == 0)
          launch_l0_post(d.Ahat, ne, c, dl.b, dl.dinv, o, st);
        else if (dl.sell)
          launch_sell_post(dl.As, c, dl.b, dl.dinv, o, st);
        else
          launch_csr_post(dl.A, c, dl.b, dl.dinv, o, st);
        c = o;
      }
      cur[(size_t)l] = c;
    };
    // one sweep out = in + D^-1 (b - A in) on level l
    auto post_l = [&](int l, const T* in, T* out) {
      auto& dl = d.lev[l];
      if (l == 0)
        launch_l0_post(d.Ahat, ne, in, dl.b, dl.dinv, out, st);
      else if (dl.sell)
        launch_sell_post(dl.As, in, dl.b, dl.dinv, out, st);
      else
        launch_csr_post(dl.A, in, dl.b, dl.dinv, out, st);
    };
    // a coarsest level above the dense limit: its pre-smoothing sweeps, no
    // coarse correction, its post-smoothing sweeps; the result goes to e
    auto relax_coarsest = [&](int l) {
      auto& dl = d.lev[l];
      presmooth(l);
      T* c = cur[(size_t)l];
      for (int k = 0; k < ns; ++k) {
        T* n = k + 1 == ns ? dl.e : (c == dl.x ? dl.t : dl.x);
        post_l(l, c, n);
        c = n;
      }
    };
    // coarse correction and post-smoothing of level l; the result goes to e
    auto correct = [&](int l) {
      auto& dl = d.lev[l];
      const T* ec = d.lev[l + 1].e;
      auto post = [&](const T* in, T* out) { post_l(l, in, out); };
      if (ns == 1) {
        // x = D^-1 b + P ec recomputes the one pre-smoothing sweep
        launch_csr_prolong(dl.P, ec, dl.b, dl.dinv, dl.x, st);
        post(dl.x, dl.e);
        return;
      }
      T* c = cur[(size_t)l];
      T* o = c == dl.x ? dl.t : dl.x;
      launch_csr_prolong_add(dl.P, ec, c, o, st);
      for (int k = 0; k < ns; ++k) {
        T* n = k + 1 == ns ? dl.e : (o == dl.x ? dl.t : dl.x);
        post(o, n);
        o = n;
      }
    };
    if (L == 1) {  // level 0 is a coarsest level above the dense limit
      ph_begin(s, st, PH_VC0, ev);
      relax_coarsest(0);
      ph_end(s, st, PH_VC0, ev);
      return;
    }
    ph_begin(s, st, PH_VC0, ev);
    // restrictions to a smoothed level also write its pre-smoothed iterate
    // x = D^-1 b, which its residual then reads
    auto restrict_to = [&](int l, const T* r) {
      auto& nx = d.lev[l + 1];
      if (l + 2 < L || relax)
        launch_csr_restrict(d.lev[l].R, r, nx.dinv, nx.b, nx.x, st);
      else
        launch_csr_spmv(d.lev[l].R, r, nx.b, st);
    };
    presmooth(0);
    launch_l0_resid(d.Ahat, ne, cur[0], l0.b, l0.r, st);
    restrict_to(0, l0.r);
    ph_end(s, st, PH_VC0, ev);
    ph_begin(s, st, PH_VCC, ev);
    // levels 1 .. top - 1 run pass by pass; below them one operator: the
    // dense bottom B (e_top = B b_top), or the coarsest solve or sweeps
    const int top = d.tail > 0 ? d.tail : L - 1;
    for (int l = 1; l < top; ++l) {
      auto& dl = d.lev[l];
      presmooth(l);
      if (dl.sell)
        launch_sell_resid(dl.As, cur[(size_t)l], dl.b, dl.r, st);
      else
        launch_csr_resid(dl.A, cur[(size_t)l], dl.b, dl.r, st);
      restrict_to(l, dl.r);
    }
    if (d.tail > 0)
      launch_dense_gemv(d.lev[top].n, d.tailB, d.lev[top].b, d.lev[top].e, st);
    else if (relax)
      relax_coarsest(L - 1);
    else
      launch_coarse_solve(s->ncoarse, s->coarse_lu, s->coarse_piv, d.lev[L - 1].b, d.lev[L - 1].e, st);
    for (int l = top - 1; l >= 1; --l) correct(l);
    ph_end(s, st, PH_VCC, ev);
    ph_begin(s, st, PH_VC0, ev);
    correct(0);
    ph_end(s, st, PH_VC0, ev);
  }
}

// z = P_E e0 + M2^-1 (r - A P_E e0); e0 == nullptr gives z = M2^-1 r
template <class T>
void enqueue_stage2(cptr_solver s, PrecDev<T>& d, const double* r, const T* e0, double* z,
                    hipStream_t st) {
  const int ne = s->ne;
  hipEvent_t ev;
  if (s->use_grid) {
    const int nx = s->grid[0], ny = s->grid[1], nz = s->grid[2];
    ph_begin(s, st, PH_STAGE2, ev);
    launch_stage2_grid(nx, ny, nz, s->A, ne, s->eidx_h, e0, r, d.r2tile, d.e0tile, d.faces, s->tickets,
                       st);
    ph_end(s, st, PH_STAGE2, ev);
    ph_begin(s, st, PH_ILU_F, ev);
    launch_ilu_fwd_grid(nx, ny, nz, d.Lg, d.r2tile, d.ytile, d.faces, s->tickets, s->sweep_flag,
                        kSweepSpinLimit, st);
    ph_end(s, st, PH_ILU_F, ev);
    ph_begin(s, st, PH_ILU_B, ev);
    launch_ilu_bwd_grid(nx, ny, nz, d.Ug, d.ytile, e0 ? d.e0tile : nullptr, ne, s->eidx_h,
                        d.faces + grid_face_values(nx, ny, nz), z, s->tickets, s->sweep_flag,
                        kSweepSpinLimit, st);
    ph_end(s, st, PH_ILU_B, ev);
    return;
  }
  const T* rhs = d.r2;
  constexpr bool f64 = std::is_same<T, double>::value;
  if (s->sf_width > 0) {  // one-launch sweeps
    ph_begin(s, st, PH_STAGE2, ev);
    if (e0 || !f64) {
      // the stage-two residual (or, without e0, r converted to T)
      launch_stage2_resid_sf(s->A, ne, s->eidx_h, e0, r, d.r2, d.y, d.x2, s->tickets, st);
    } else if constexpr (f64) {
      launch_sweep_prepare(s->N, d.y, d.x2, s->tickets, st);
      rhs = r;
    }
    ph_end(s, st, PH_STAGE2, ev);
    ph_begin(s, st, PH_ILU_F, ev);
    launch_ilu_fwd_sf(d.Lf, s->sf_width, s->fperm, rhs, d.y, s->tickets, s->sweep_flag,
                      kSweepSpinLimit, st);
    ph_end(s, st, PH_ILU_F, ev);
    ph_begin(s, st, PH_ILU_B, ev);
    launch_ilu_bwd_sf(d.Ub, s->sf_width, s->bperm, d.uinv, d.y, e0, ne, s->eidx_h, d.x2, z,
                      s->tickets, s->sweep_flag, kSweepSpinLimit, st);
    ph_end(s, st, PH_ILU_B, ev);
    return;
  }
  if constexpr (f64) {
    if (!e0) rhs = r;
  }
  // per-level launches; the stage-two residual also converts r to T
  if (rhs == d.r2) {
    ph_begin(s, st, PH_STAGE2, ev);
    launch_stage2_resid(s->A, ne, s->eidx_h, e0, r, d.r2, st);
    ph_end(s, st, PH_STAGE2, ev);
  }
  ph_begin(s, st, PH_ILU_F, ev);
  for (size_t l = 0; l + 1 < s->flev_ptr.size(); ++l)
    launch_ilu_fwd_level(d.Lf, s->fperm, s->flev_ptr[l], s->flev_ptr[l + 1], rhs, d.y, st);
  ph_end(s, st, PH_ILU_F, ev);
  ph_begin(s, st, PH_ILU_B, ev);
  for (size_t l = 0; l + 1 < s->blev_ptr.size(); ++l)
    launch_ilu_bwd_level(d.Ub, s->bperm, d.uinv, s->blev_ptr[l], s->blev_ptr[l + 1], d.y, e0, ne,
                         s->eidx_h, d.x2, z, st);
  ph_end(s, st, PH_ILU_B, ev);
}

template <class T>
void enqueue_apply(cptr_solver s, PrecDev<T>& d, const double* r, double* z, hipStream_t st, bool restricted) {
  enqueue_stage1(s, d, r, st, restricted);
  enqueue_stage2(s, d, r, (const T*)d.lev[0].e, z, st);
}

void enqueue_apply(cptr_solver s, const double* r, double* z, hipStream_t st, bool restricted = false) {
  if (s->prec == CPTR_PRECISION_FP32)
    enqueue_apply(s, s->p32, r, z, st, restricted);
  else
    enqueue_apply(s, s->p64, r, z, st, restricted);
}

// The Krylov space of (F)GMRES(m): V (m + 1 vectors), Z (m vectors, flexible
// solves) and three work vectors, allocated once when the device half is
// built.  A failure leaves the handle's other memory to the caller's release.
int alloc_solve_space(cptr_solver s, int m, bool flexible) {
  const int64_t ld = (s->N + 63) / 64 * 64;
  int rc;
  if ((rc = dalloc(s, s->V, ld * (m + 1)))) return rc;
  if (flexible && (rc = dalloc(s, s->Z, ld * m))) return rc;
  if ((rc = dalloc(s, s->wr, s->N)) || (rc = dalloc(s, s->wt, s->N)) || (rc = dalloc(s, s->wu, s->N)))
    return rc;
  s->restart_cap = m;
  s->have_z = flexible;
  s->ldv = ld;
  return CPTR_OK;
}

// ||x||_2 on the device, synchronising st (part, hd: the reduction scratch)
int device_norm(cptr_solver s, const double* x, double& out, hipStream_t st, double* part, double* hd) {
  launch_norm2(s->N, x, part, st);
  launch_reduce(1, part, hd + 136, 0, st);
  HIP_TRY(s, hipMemcpyAsync(s->hhost + 136, hd + 136, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(s, hipStreamSynchronize(st));
  out = std::sqrt(s->hhost[136]);
  return CPTR_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- Galerkin
// A CSR matrix on the device (int32 row pointers and columns, FP64 values),
// allocated stream-ordered so that setups running beside solves never
// synchronise the device.
struct DevCsr {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t* rp = nullptr;
  int32_t* ci = nullptr;
  double* v = nullptr;
};

// The steps of one AMG level's construction on the device for a device
// handle: strength, extended+i interpolation and the Galerkin product, each
// giving the host construction's result bit for bit.  The level's operator
// goes to the device once.  A step returns false when it cannot take the
// level (a row too long for the kernels, a HIP error); the host then forms
// that piece itself.  Counts of the steps done here go to `done`.
class DeviceLevelSteps : public LevelSteps {
 public:
  DeviceLevelSteps(const Csr& A, SetupSiteCounts& done, int threads)
      : A_(A), done_(done), threads_(std::max(1, threads)) {
    ok_ = hipStreamCreateWithFlags(&st_, hipStreamNonBlocking) == hipSuccess && upload(A, a_);
  }
  ~DeviceLevelSteps() override {
    for (void* p : mem_) (void)hipFreeAsync(p, st_);
    if (st_) {
      (void)hipStreamSynchronize(st_);
      (void)hipStreamDestroy(st_);
    }
  }

  bool strength(const std::vector<int32_t>& func, double theta, double mrs, Csr& S) override {
    if (!ok_) return false;
    const int32_t n = A_.n;
    int32_t *dfunc = nullptr, *ocol = nullptr, *cnt = nullptr;
    if (!put(dfunc, func.data(), n) || !alloc(ocol, a_.nnz) || !alloc(cnt, n)) return fail();
    launch_strength(n, a_.rp, a_.ci, a_.v, dfunc, theta, mrs, ocol, cnt, st_);
    std::vector<int32_t> hc((size_t)n);
    if (!get(hc.data(), cnt, n)) return fail();
    std::vector<int32_t> rp((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) rp[i + 1] = rp[i] + hc[i];
    DevCsr sd;
    sd.n = n;
    sd.nnz = rp[n];
    if (!put(sd.rp, rp.data(), (int64_t)n + 1) || !alloc(sd.ci, sd.nnz)) return fail();
    launch_compact_cols(n, a_.rp, sd.rp, ocol, sd.ci, st_);
    S.n = S.m = n;
    S.rp.assign(rp.begin(), rp.end());
    S.ci.resize(sd.nnz);
    S.v.clear();
    if (!get(S.ci.data(), sd.ci, sd.nnz)) return fail();
    s_ = sd;
    have_s_ = true;
    ++done_.strength;
    return true;
  }

  bool interp(const Csr& S, const std::vector<int32_t>& cf, const std::vector<int32_t>& func, int pmax,
              Csr& P) override {
    if (!ok_) return false;
    const int32_t n = A_.n;
    std::vector<int32_t> cidx((size_t)n, -1);
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i)
      if (cf[i] == 1) cidx[i] = nc++;
    const int outcap = pmax > 0 ? std::max(1, pmax) : interp_set_cap();
    if (!have_s_ && !upload_pattern(S, s_)) return fail();
    have_s_ = true;
    int32_t *dcf = nullptr, *dfunc = nullptr, *dcidx = nullptr, *ocol = nullptr, *cnt = nullptr;
    double* oval = nullptr;
    int* over = nullptr;
    if (!put(dcf, cf.data(), n) || !put(dfunc, func.data(), n) || !put(dcidx, cidx.data(), n) ||
        !alloc(ocol, (int64_t)n * outcap) || !alloc(oval, (int64_t)n * outcap) || !alloc(cnt, n) ||
        !alloc(over, 1) || hipMemsetAsync(over, 0, sizeof(int), st_) != hipSuccess)
      return fail();
    // a workgroup per row once rows average 16 entries (the coarse levels)
    const bool long_rows = a_.nnz >= 16 * (int64_t)n;
    launch_interp_exti(n, a_.rp, a_.ci, a_.v, s_.rp, s_.ci, dcf, dfunc, dcidx, pmax, outcap, ocol, oval, cnt, over,
                       long_rows,
                       st_);
    std::vector<int32_t> hc((size_t)n);
    int h_over = 0;
    if (!get(hc.data(), cnt, n) || !get(&h_over, over, 1)) return fail();
    if (h_over != 0) return false;
    std::vector<int64_t> off((size_t)n + 1);
    std::vector<int32_t> rp((size_t)n + 1, 0);
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
      off[i] = (int64_t)i * outcap;
      total += hc[i];
      rp[i + 1] = (int32_t)total;
    }
    int64_t* doff = nullptr;
    int32_t *drp = nullptr, *pci = nullptr;
    double* pv = nullptr;
    if (!put(doff, off.data(), n) || !put(drp, rp.data(), (int64_t)n + 1) || !alloc(pci, total) ||
        !alloc(pv, total))
      return fail();
    launch_spgemm_compact(n, doff, drp, ocol, oval, pci, pv, st_);
    P.n = n;
    P.m = nc;
    P.rp.assign(rp.begin(), rp.end());
    P.ci.resize(total);
    P.v.resize(total);
    if (!get(P.ci.data(), pci, total) || !get(P.v.data(), pv, total)) return fail();
    ++done_.interp;
    return true;
  }

  // The first pass over the components of at most kSmallComponent points:
  // components and measures from the union-find kernels, the components
  // picked here by size, their passes on the device (one thread each).
  static constexpr int32_t kSmallComponent = 64;
  bool first_pass_small(const Csr& G, bool second, std::vector<int32_t>& cf) override {
    if (!ok_) return false;
    if (second && !have_s2_) return false;
    if (!second && !have_s_) {
      if (!upload_pattern(G, s_)) return fail();
      have_s_ = true;
    }
    const DevCsr& g = second ? s2_ : s_;
    const int32_t n = G.n;
    int32_t *parent = nullptr, *lam = nullptr, *root = nullptr, *size = nullptr, *dcf = nullptr;
    if (!alloc(parent, n) || !alloc(lam, n) || !alloc(root, n) || !alloc(size, n) || !alloc(dcf, n)) return fail();
    launch_fp_components(n, g.rp, g.ci, parent, lam, root, size, dcf, st_);
    std::vector<int32_t> hs((size_t)n);
    if (!get(hs.data(), size, n)) return fail();
    std::vector<int32_t> cursor((size_t)n, -1), coff(1, 0);
    for (int32_t r = 0; r < n; ++r)
      if (hs[r] >= 2 && hs[r] <= kSmallComponent) {
        cursor[r] = coff.back();
        coff.push_back(coff.back() + hs[r]);
      }
    const int32_t ncomp = (int32_t)coff.size() - 1;
    if (ncomp > 0) {
      int32_t *dcur = nullptr, *dcoff = nullptr, *members = nullptr;
      if (!put(dcur, cursor.data(), n) || !put(dcoff, coff.data(), (int64_t)ncomp + 1) ||
          !alloc(members, coff.back()))
        return fail();
      launch_fp_small(n, root, dcur, members, ncomp, dcoff, g.rp, g.ci, lam, dcf, st_);
    }
    cf.resize(n);
    if (!get(cf.data(), dcf, n)) return fail();
    ++done_.split;
    done_.split_points += coff.back();
    done_.first_points += n;
    return true;
  }

  // HMIS over blocks on the device: the graph's transpose, the blocks' first
  // passes, the cover by their C points, then PMIS rounds until no point is
  // undecided (one count back per round).
  bool hmis(const Csr& G, bool second, int32_t block, std::vector<int32_t>& cf) override {
    if (!ok_ || block < 1 || block > hmis_block_cap()) return false;
    if (second && !have_s2_) return false;
    if (!second && !have_s_) {
      if (!upload_pattern(G, s_)) return fail();
      have_s_ = true;
    }
    const DevCsr& g = second ? s2_ : s_;
    const int32_t n = G.n;
    int32_t *deg = nullptr, *trp = nullptr, *cursor = nullptr, *tci = nullptr, *cf1 = nullptr, *dcf = nullptr;
    int32_t *cnt = nullptr, *isnew = nullptr;
    int* left = nullptr;
    if (!alloc(deg, n) || !alloc(trp, (int64_t)n + 1) || !alloc(cursor, (int64_t)n + 1) || !alloc(cf1, n) ||
        !alloc(dcf, n) || !alloc(cnt, n) || !alloc(isnew, n) || !alloc(left, 1))
      return fail();
    launch_fill_i32(n, deg, 0, st_);
    launch_transpose_pattern(n, g.rp, g.ci, deg, nullptr, nullptr, 0, st_);
    const int64_t nt = scan<int32_t>(deg, n, trp, nullptr);
    if (nt < 0) return fail();
    if (!alloc(tci, nt) ||
        hipMemcpyAsync(cursor, trp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, st_) != hipSuccess)
      return fail();
    launch_transpose_pattern(n, g.rp, g.ci, nullptr, cursor, tci, 1, st_);
    launch_hmis_blocks(n, block, g.rp, g.ci, trp, tci, cf1, dcf, st_);
    launch_pmis_start(n, g.rp, g.ci, dcf, cnt, st_);
    // every round with a point left decides at least the best of them
    for (int64_t round = 0;; ++round) {
      launch_pmis_round(n, g.rp, g.ci, trp, tci, cnt, dcf, isnew, left, st_);
      int h_left = 0;
      if (!get(&h_left, left, 1)) return fail();
      if (h_left == 0) break;
      if (round > n) return false;
    }
    cf.resize(n);
    if (!get(cf.data(), dcf, n)) return fail();
    ++done_.hmis;
    return true;
  }

  // Distance-two strength of an aggressive level: candidates counted, rows
  // counted, then written at their CSR places.
  bool strength2(const Csr& S, const std::vector<int32_t>& cf, Csr& S2) override {
    if (!ok_) return false;
    const int32_t n = A_.n;
    if (!have_s_ && !upload_pattern(S, s_)) return fail();
    have_s_ = true;
    std::vector<int32_t> cidx((size_t)n, -1), cpts;
    for (int32_t i = 0; i < n; ++i)
      if (cf[i] == 1) {
        cidx[i] = (int32_t)cpts.size();
        cpts.push_back(i);
      }
    const int32_t nc = (int32_t)cpts.size();
    int32_t *dcpts = nullptr, *dcidx = nullptr, *bound = nullptr, *cnt = nullptr;
    if (!put(dcpts, cpts.data(), nc) || !put(dcidx, cidx.data(), n) || !alloc(bound, nc) || !alloc(cnt, nc))
      return fail();
    launch_s2_bound(nc, dcpts, s_.rp, s_.ci, bound, st_);
    std::vector<int32_t> h((size_t)nc);
    if (!get(h.data(), bound, nc)) return fail();
    for (int32_t r = 0; r < nc; ++r)
      if (h[r] > s2_row_cap()) return false;
    launch_s2_rows(nc, dcpts, s_.rp, s_.ci, dcidx, nullptr, nullptr, cnt, st_);
    if (!get(h.data(), cnt, nc)) return fail();
    std::vector<int32_t> rp((size_t)nc + 1, 0);
    for (int32_t r = 0; r < nc; ++r) {
      if ((int64_t)rp[r] + h[r] >= INT32_MAX) return false;
      rp[r + 1] = rp[r] + h[r];
    }
    int32_t *drp = nullptr, *dci = nullptr;
    if (!put(drp, rp.data(), (int64_t)nc + 1) || !alloc(dci, rp[nc])) return fail();
    launch_s2_rows(nc, dcpts, s_.rp, s_.ci, dcidx, drp, dci, nullptr, st_);
    S2.n = S2.m = nc;
    S2.rp.assign(rp.begin(), rp.end());
    S2.ci.resize(rp[nc]);
    S2.v.clear();
    if (!get(S2.ci.data(), dci, rp[nc])) return fail();
    s2_.n = nc;
    s2_.nnz = rp[nc];
    s2_.rp = drp;
    s2_.ci = dci;
    have_s2_ = true;
    ++done_.strength2;
    return true;
  }

  // Multipass interpolation of an aggressive level, pass by pass: the rows of
  // a pass are those without interpolation next to a point with one; their
  // coefficients and products come from the kernels, the row pointers of each
  // next P from here.
  bool multipass(const Csr& S, const std::vector<int32_t>& cf, const std::vector<int32_t>& func,
                 Csr& P) override {
    if (!ok_) return false;
    const int32_t n = A_.n;
    if (!have_s_ && !upload_pattern(S, s_)) return fail();
    have_s_ = true;
    std::vector<int32_t> pass((size_t)n), lens((size_t)n, 0), prp((size_t)n + 1, 0), pci;
    int32_t nc = 0;
    for (int32_t i = 0; i < n; ++i) {
      pass[i] = cf[i] == 1 ? 0 : -1;
      if (cf[i] == 1) {
        lens[i] = 1;
        pci.push_back(nc++);
      }
      prp[i + 1] = prp[i] + lens[i];
    }
    const std::vector<double> pv(pci.size(), 1.0);
    int32_t *dpass = nullptr, *dfunc = nullptr, *drp = nullptr, *dci = nullptr, *rowpos = nullptr;
    int32_t *flag = nullptr, *pos = nullptr, *dlens = nullptr;
    double* dv = nullptr;
    if (!put(dpass, pass.data(), n) || !put(dfunc, func.data(), n) || !put(drp, prp.data(), (int64_t)n + 1) ||
        !put(dci, pci.data(), nc) || !put(dv, pv.data(), nc) || !put(dlens, lens.data(), n) || !alloc(flag, n) ||
        !alloc(pos, (int64_t)n + 1) || !alloc(rowpos, n))
      return fail();
    launch_fill_i32(n, rowpos, -1, st_);
    int64_t nnz = nc;
    for (int pass_no = 1;; ++pass_no) {
      launch_mp_mark(n, s_.rp, s_.ci, dpass, flag, st_);
      const int64_t m = scan<int32_t>(flag, n, pos, nullptr);
      if (m < 0) return fail();
      if (m == 0) break;
      int32_t *dnow = nullptr, *bound = nullptr, *cnt = nullptr, *ocol = nullptr, *nrp = nullptr, *nci = nullptr;
      int64_t* doff = nullptr;
      double *oval = nullptr, *nv = nullptr;
      if (!alloc(dnow, m) || !alloc(bound, m) || !alloc(doff, m + 1) || !alloc(cnt, m) || !alloc(nrp, (int64_t)n + 1))
        return fail();
      launch_select(n, flag, pos, dnow, st_);
      launch_mp_bound((int)m, dnow, a_.rp, a_.ci, a_.v, s_.rp, s_.ci, dpass, dfunc, drp, bound, st_);
      int32_t maxb = 0;
      const int64_t nprod = scan<int64_t>(bound, m, doff, &maxb);
      if (nprod < 0) return fail();
      if (maxb > spgemm_row_cap()) return false;
      if (!alloc(ocol, nprod) || !alloc(oval, nprod)) return fail();
      launch_mp_rows((int)m, dnow, a_.rp, a_.ci, a_.v, s_.rp, s_.ci, dpass, dfunc, drp, dci, dv, doff, ocol, oval,
                     cnt, maxb, st_);
      launch_mp_setlen((int)m, dnow, cnt, dlens, st_);
      const int64_t total = scan<int32_t>(dlens, n, nrp, nullptr);
      if (total < 0) return fail();
      if (total >= INT32_MAX) return false;
      if (!alloc(nci, total) || !alloc(nv, total)) return fail();
      launch_mp_merge(n, pass_no, rowpos, dnow, (int)m, doff, ocol, oval, drp, dci, dv, nrp, nci, nv, dpass, st_);
      drp = nrp;
      dci = nci;
      dv = nv;
      nnz = total;
    }
    P.n = n;
    P.m = nc;
    if (!get(prp.data(), drp, (int64_t)n + 1)) return fail();
    P.rp.assign(prp.begin(), prp.end());
    P.ci.resize(nnz);
    P.v.resize(nnz);
    if (!get(P.ci.data(), dci, nnz) || !get(P.v.data(), dv, nnz)) return fail();
    ++done_.multipass;
    return true;
  }

  // C = R (A P) in the host product's order
  bool galerkin(const Csr& R, const Csr& P, Csr& C) override {
    if (!ok_) return false;
    DevCsr p, r, ap, c;
    std::vector<int32_t> crp;
    if (!upload(P, p) || !upload(R, r)) return fail();
    if (!product(a_, p, ap, nullptr) || !product(r, ap, c, &crp)) return false;
    C.n = R.n;
    C.m = P.m;
    C.rp.assign(crp.begin(), crp.end());
    C.ci.resize(c.nnz);
    C.v.resize(c.nnz);
    if (!get(C.ci.data(), c.ci, c.nnz) || !get(C.v.data(), c.v, c.nnz)) return fail();
    ++done_.galerkin;
    return true;
  }

 private:
  bool fail() {
    (void)hipGetLastError();
    ok_ = false;
    return false;
  }
  template <class T>
  bool alloc(T*& p, int64_t count) {
    void* q = nullptr;
    if (hipMallocAsync(&q, sizeof(T) * (size_t)std::max<int64_t>(1, count), st_) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    mem_.push_back(q);
    p = static_cast<T*>(q);
    return true;
  }
  // host -> device; the source may die when this returns
  template <class T>
  bool put(T*& p, const T* src, int64_t count) {
    return alloc(p, count) &&
           (count == 0 || staged::to_device(p, src, sizeof(T) * count, st_, threads_) == hipSuccess);
  }
  // device -> host, after the stream's earlier work
  template <class T>
  bool get(T* dst, const T* src, int64_t count) {
    if (count > 0 && staged::to_host(dst, src, sizeof(T) * count, st_, threads_) != hipSuccess) return false;
    return hipStreamSynchronize(st_) == hipSuccess && hipGetLastError() == hipSuccess;
  }
  bool upload_pattern(const Csr& h, DevCsr& d) {
    if (h.nnz() >= INT32_MAX) return false;
    std::vector<int32_t> rp32(h.rp.begin(), h.rp.end());
    d.n = h.n;
    d.nnz = h.nnz();
    return put(d.rp, rp32.data(), (int64_t)rp32.size()) && put(d.ci, h.ci.data(), d.nnz);
  }
  bool upload(const Csr& h, DevCsr& d) {
    if (h.v.size() != h.ci.size()) return false;
    return upload_pattern(h, d) && put(d.v, h.v.data(), d.nnz);
  }
  // exclusive prefix sums of n device counts into out (n + 1 entries, the
  // total last); returns the total (and the largest count in *maxc), -1 on a
  // HIP error
  template <class O>
  int64_t scan(const int32_t* in, int64_t n, O* out, int32_t* maxc) {
    const int64_t ntmp = scan_tmp_size(n);
    int64_t* tmp = nullptr;
    int32_t* dmax = nullptr;
    if (!alloc(tmp, ntmp) || !alloc(dmax, 1)) return -1;
    launch_fill_i32(1, dmax, 0, st_);
    launch_scan<O>(n, in, out, tmp, dmax, st_);
    int64_t total = 0;
    int32_t mx = 0;
    if (!get(&total, tmp + ntmp - 1, 1) || !get(&mx, dmax, 1)) return -1;
    if (maxc) *maxc = mx;
    return total;
  }
  // out = x y; row pointers prefixed on the device, copied to *rp_host if asked
  bool product(const DevCsr& x, const DevCsr& y, DevCsr& out, std::vector<int32_t>* rp_host) {
    const int32_t n = x.n;
    int32_t *bound = nullptr, *ocol = nullptr, *cnt = nullptr;
    int64_t* doff = nullptr;
    double* oval = nullptr;
    if (!alloc(bound, n) || !alloc(doff, (int64_t)n + 1) || !alloc(cnt, n) || !alloc(out.rp, (int64_t)n + 1))
      return fail();
    launch_spgemm_bound(n, x.rp, x.ci, y.rp, bound, st_);
    int32_t maxb = 0;
    const int64_t nprod = scan<int64_t>(bound, n, doff, &maxb);
    if (nprod < 0) return fail();
    if (maxb > spgemm_row_cap()) return false;
    if (!alloc(ocol, nprod) || !alloc(oval, nprod)) return fail();
    launch_spgemm_rows(n, x.rp, x.ci, x.v, y.rp, y.ci, y.v, doff, ocol, oval, cnt, maxb, st_);
    const int64_t total = scan<int32_t>(cnt, n, out.rp, nullptr);
    if (total < 0) return fail();
    if (total >= INT32_MAX) return false;
    out.n = n;
    out.nnz = total;
    if (!alloc(out.ci, total) || !alloc(out.v, total)) return fail();
    launch_spgemm_compact(n, doff, out.rp, ocol, oval, out.ci, out.v, st_);
    if (rp_host) {
      rp_host->resize((size_t)n + 1);
      if (!get(rp_host->data(), out.rp, (int64_t)n + 1)) return fail();
    }
    return hipGetLastError() == hipSuccess || fail();
  }

  const Csr& A_;
  SetupSiteCounts& done_;
  int threads_ = 1;  // host threads for the staged copies
  hipStream_t st_ = nullptr;
  bool ok_ = false;
  DevCsr a_, s_, s2_;
  bool have_s_ = false, have_s2_ = false;
  std::vector<void*> mem_;
};

}  // namespace

// ============================================================================
extern "C" {

void cptr_setup_opts_default(cptr_setup_opts* o) {
  if (!o) return;
  o->strong_threshold = 0.25;
  o->max_row_sum = 0.9;
  o->max_levels = 25;
  o->max_coarse = 9;
  o->p_max_elmts = 4;
  o->restriction = CPTR_RESTRICT_QUASI_IMPES;
  o->host_only = 0;
  o->setup_threads = 0;
  o->ilu_sweep = CPTR_ILU_SWEEP_AUTO;
  o->agg_levels = 1;
  o->precond_precision = CPTR_PRECISION_FP64;
  o->num_sweeps = 1;
  o->max_restart = 50;
  o->flexible_space = 1;
  o->hmis_block = 0;
  o->max_dense_coarse = 4096;
  o->dense_tail = 2048;
}

void cptr_solve_opts_default(cptr_solve_opts* o) {
  if (!o) return;
  o->restart = 30;
  o->max_iter = 200;
  o->flexible = 0;
  o->x0_is_zero = 1;
  o->rtol = 1e-6;
  o->profile = 0;
}

const char* cptr_last_error(cptr_solver s) { return s ? s->err.c_str() : g_setup_error.c_str(); }

}  // extern "C"

namespace cptr {

int setup_host(const cptr_bsr* A, int32_t block_size, const int32_t* elliptic_idx, int32_t n_elliptic,
               const cptr_setup_opts* opts, cptr_solver* out, const hipStream_t* early_stream) {
  g_setup_error.clear();
  if (!out) return (cptr_status)fail(nullptr, CPTR_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!A) return (cptr_status)fail(nullptr, CPTR_E_INVALID, "A is NULL");
  if (block_size != kBS)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "block_size must be 3");
  if (!elliptic_idx || n_elliptic < 1 || n_elliptic >= block_size)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "n_elliptic must be 1 or 2 with a non-NULL elliptic_idx");
  for (int e = 0; e < n_elliptic; ++e) {
    if (elliptic_idx[e] < 0 || elliptic_idx[e] >= block_size)
      return (cptr_status)fail(nullptr, CPTR_E_INVALID, "elliptic_idx out of range");
    for (int f = 0; f < e; ++f)
      if (elliptic_idx[f] == elliptic_idx[e])
        return (cptr_status)fail(nullptr, CPTR_E_INVALID, "elliptic_idx has duplicates");
  }
  cptr_setup_opts o;
  cptr_setup_opts_default(&o);
  if (opts) o = *opts;
  if (o.ilu_sweep < 0 || o.ilu_sweep > 3)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "ilu_sweep must be 0, 1, 2 or 3");
  if (o.precond_precision != CPTR_PRECISION_FP64 && o.precond_precision != CPTR_PRECISION_FP32)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "precond_precision must be FP64 or FP32");
  if (o.num_sweeps < 1 || o.num_sweeps > 8)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "num_sweeps must be in [1, 8]");
  if (o.max_restart < 1 || o.max_restart > kMaxRestart)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "max_restart must be in [1, 64]");
  if (o.flexible_space != 0 && o.flexible_space != 1)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "flexible_space must be 0 or 1");
  if (o.max_levels < 1 || o.max_levels > 64 || o.max_coarse < 1 || o.p_max_elmts < 0 ||
      o.agg_levels < 0 || o.hmis_block < 0 || o.max_dense_coarse < 0 || o.max_dense_coarse > 4096 ||
      o.dense_tail < 0 || o.dense_tail > 4096 ||
      !(o.strong_threshold >= 0.0) || !(o.max_row_sum > 0.0))
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "setup options out of range");
  if (A->n_block_rows <= 0 || A->nnz_blocks <= 0 || A->nnz_blocks >= INT32_MAX)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "A.n_block_rows / A.nnz_blocks out of range");
  if (!A->row_ptr || !A->col_idx || !A->values)
    return (cptr_status)fail(nullptr, CPTR_E_INVALID, "A has a NULL array");

  std::unique_ptr<cptr_solver_s> s(new (std::nothrow) cptr_solver_s());
  if (!s) return (cptr_status)fail(nullptr, CPTR_E_NOMEM, "host allocation failed");
  const int32_t nb = A->n_block_rows;
  const int64_t nnzb = A->nnz_blocks;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
  const int32_t* prp = A->row_ptr;
  const int32_t* pci = A->col_idx;
  const double* pv = A->values;
  try {
    if (A->on_device) {
      if (o.host_only)
        return (cptr_status)fail(nullptr, CPTR_E_INVALID, "host_only setup needs host arrays");
      rp.resize(nb + 1);
      ci.resize(nnzb);
      v.resize(nnzb * 9);
      hipError_t e1 = hipMemcpy(rp.data(), prp, sizeof(int32_t) * (nb + 1), hipMemcpyDeviceToHost);
      hipError_t e2 = hipMemcpy(ci.data(), pci, sizeof(int32_t) * nnzb, hipMemcpyDeviceToHost);
      hipError_t e3 = hipMemcpy(v.data(), pv, sizeof(double) * nnzb * 9, hipMemcpyDeviceToHost);
      if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return (cptr_status)fail(nullptr, CPTR_E_HIP, "copying A from the device failed");
      prp = rp.data();
      pci = ci.data();
      pv = v.data();
    }
  } catch (const std::bad_alloc&) {
    return (cptr_status)fail(nullptr, CPTR_E_NOMEM, "host allocation failed");
  }
  std::string err;
  int rc = validate_bsr(nb, nnzb, prp, pci, pv, err);
  if (rc) return (cptr_status)fail(nullptr, rc, err);
  SetupParams prm;
  // a device handle factors ILU(0) on the device
  const bool dev_ilu = !o.host_only;
  prm.skip_ilu = dev_ilu;
  // a device handle forms the Galerkin products on the device (the host's
  // summation order, so the hierarchy is the same); a level whose rows are
  // too long for the kernel is formed on the host
  SetupSiteCounts sites;
  if (!o.host_only)
    prm.level_steps = [&sites, &prm](const Csr& Al) -> std::unique_ptr<LevelSteps> {
      return std::unique_ptr<LevelSteps>(new DeviceLevelSteps(Al, sites, prm.threads));
    };
  prm.theta = o.strong_threshold;
  prm.max_row_sum = o.max_row_sum;
  prm.max_levels = o.max_levels;
  prm.max_coarse = o.max_coarse;
  prm.pmax = o.p_max_elmts;
  prm.agg_levels = o.agg_levels;
  prm.hmis_block = o.hmis_block;
  prm.max_dense_coarse = o.max_dense_coarse;
  prm.quasi_impes = o.restriction == CPTR_RESTRICT_QUASI_IMPES;
  unsigned hw = std::thread::hardware_concurrency();
  prm.threads = o.setup_threads > 0 ? o.setup_threads : (int)std::min<unsigned>(16, hw ? hw : 1);
  s->ne = n_elliptic;
  s->N = (int64_t)nb * 3;
  s->ilu_mode = o.ilu_sweep;
  s->threads = prm.threads;
  s->device_ilu = dev_ilu;
  s->prec = o.precond_precision;
  s->nsweeps = o.num_sweeps;
  s->dense_tail = o.dense_tail;
  s->max_restart = o.max_restart;
  s->flex_space = o.flexible_space != 0;
  // the device half's first part on a second thread, overlapping the AMG
  // levels (it needs A, its diagonals and weights, which are final once the
  // weights are formed, and the sweeps' dependency levels, computed there)
  std::thread early;
  int early_rc = CPTR_OK;
  int early_dev = -1;
  double early_s = 0.0;
  bool early_ran = false;
  if (early_stream && !o.host_only && hipGetDevice(&early_dev) == hipSuccess) {
    const hipStream_t est = *early_stream;
    cptr_solver hs = s.get();
    prm.ilu_levels_elsewhere = true;
    prm.after_weights = [&early, &early_rc, &early_s, &early_ran, early_dev, est, hs](HostSetup& h) {
      early_ran = true;
      for (int e = 0; e < 3; ++e) {
        hs->eidx_h[e] = h.eidx[e];
        hs->hidx_h[e] = h.hidx[e];
      }
      early = std::thread([&early_rc, &early_s, early_dev, est, hs, &h] {
        const double t = now_s();
        if (hipSetDevice(early_dev) != hipSuccess) {
          early_rc = hip_fail(hs, hipGetLastError(), "hipSetDevice for the device half");
          return;
        }
        try {
          ilu_dependency_levels(h);
          early_rc = build_device_a(hs, est);
        } catch (const std::bad_alloc&) {
          early_rc = fail(hs, CPTR_E_NOMEM, "host allocation failed while packing device layouts");
        }
        early_s = now_s() - t;
      });
    };
  } else {
    (void)hipGetLastError();
  }
  bool no_mem = false;
  try {
    rc = build_host_setup(nb, prp, pci, pv, elliptic_idx, n_elliptic, prm, s->host, err);
  } catch (const std::bad_alloc&) {
    no_mem = true;
  }
  if (early.joinable()) early.join();
  if (no_mem || rc || early_rc) {
    const std::string msg = no_mem ? "host allocation failed during setup" : rc ? err : s->err;
    const int code = no_mem ? CPTR_E_NOMEM : rc ? rc : early_rc;
    // kernels of the first part may still run on its stream: its memory goes
    // back only once they are done
    if (early_ran) {
      (void)hipStreamSynchronize(*early_stream);
      release_device(s.get());
    }
    return (cptr_status)fail(nullptr, code, msg);
  }
  s->dev_a_done = early_ran;
  s->device_build_s = early_s;
  if (A->on_device) {
    // the host copy of A's values dies with this call: the handle keeps it
    // until the device half has been built
    s->host.av_owned = std::move(v);
    s->host.av = s->host.av_owned.data();
  }
  for (int e = 0; e < 3; ++e) {
    s->eidx_h[e] = s->host.eidx[e];
    s->hidx_h[e] = s->host.hidx[e];
  }
  s->device_steps = sites;
  s->agg_levels_used = std::min<int32_t>(prm.agg_levels, (int32_t)s->host.lev.size() - 1);
  *out = s.release();
  return CPTR_OK;
}

int measure_device(cptr_solver s, int restart, bool flexible, int64_t* bytes) {
  if (!s || !bytes) return CPTR_E_INVALID;
  if (s->device) return fail(s, CPTR_E_STATE, "handle already has its device half");
  s->measure = true;
  s->dev_bytes = 0;
  int rc = CPTR_OK;
  try {
    rc = build_device(s, nullptr);
    if (!rc) rc = alloc_solve_space(s, std::max(1, std::min(restart, kMaxRestart)), flexible);
  } catch (const std::bad_alloc&) {
    rc = fail(s, CPTR_E_NOMEM, "host allocation failed while packing device layouts");
  }
  *bytes = s->dev_bytes;
  s->measure = false;
  reset_device_state(s);
  return rc;
}

int setup_device(cptr_solver s, DevArena* arena, int restart, bool flexible, hipStream_t st) {
  if (!s) return CPTR_E_INVALID;
  if (s->device) return fail(s, CPTR_E_STATE, "handle already has its device half");
  int dev_count = 0;
  hipError_t he = hipGetDeviceCount(&dev_count);
  if (he != hipSuccess || dev_count == 0) return fail(s, CPTR_E_HIP, "no HIP device available");
  s->arena = arena;
  int rc;
  const double t_dev = now_s();
  try {
    rc = s->dev_a_done ? build_device_b(s, st) : build_device(s, st);
    if (!rc) rc = alloc_solve_space(s, std::max(1, std::min(restart, kMaxRestart)), flexible);
  } catch (const std::bad_alloc&) {
    rc = fail(s, CPTR_E_NOMEM, "host allocation failed while packing device layouts");
  }
  if (rc) {
    // kernels of the failed build may still run on st: its memory goes back
    // (to an arena other requests allocate from) only once they are done
    (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
    release_device(s);
    return rc;
  }
  s->device = true;
  s->device_build_s += now_s() - t_dev;
  return CPTR_OK;
}

void release_device(cptr_solver s) {
  if (!s) return;
  dfree_all(s);
  if (s->hhost) (void)hipHostFree(s->hhost);
  for (auto& e : s->ev_pool)
    if (e) (void)hipEventDestroy(e);
  s->ev_pool.clear();
  if (s->ev_copy) (void)hipEventDestroy(s->ev_copy);
  s->ev_copy = nullptr;
  s->ev_used = 0;
  s->ev_pending.clear();
  reset_device_state(s);
  s->device = false;
}

const char* last_error(cptr_solver s) { return s ? s->err.c_str() : g_setup_error.c_str(); }

void drop_input(cptr_solver s) {
  if (!s) return;
  s->host.av = nullptr;
  std::vector<double>().swap(s->host.av_owned);
}

int64_t device_bytes(cptr_solver s) { return s ? s->dev_bytes : 0; }

}  // namespace cptr

extern "C" {

cptr_status cptr_setup(const cptr_bsr* A, int32_t block_size, const int32_t* elliptic_idx,
                       int32_t n_elliptic, const cptr_setup_opts* opts, void* stream,
                       cptr_solver* out) {
  const double t0 = now_s();
  if (out) *out = nullptr;
  cptr_solver s = nullptr;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = setup_host(A, block_size, elliptic_idx, n_elliptic, opts, &s, &st);
  if (rc) return (cptr_status)rc;
  cptr_setup_opts o;
  cptr_setup_opts_default(&o);
  if (opts) o = *opts;
  if (!o.host_only) {
    rc = setup_device(s, nullptr, o.max_restart, o.flexible_space != 0, st);
    if (rc) {
      g_setup_error = s->err;
      delete s;
      return (cptr_status)rc;
    }
  }
  drop_input(s);  // A's values belong to the caller again
  s->setup_s = now_s() - t0;
  *out = s;
  return CPTR_OK;
}

cptr_status cptr_destroy(cptr_solver s) {
  if (!s) return CPTR_E_INVALID;
  release_device(s);
  delete s;
  return CPTR_OK;
}

cptr_status cptr_apply(cptr_solver s, const double* r, double* z, void* stream) {
  if (!s) return CPTR_E_INVALID;
  if (!s->device) return (cptr_status)fail(s, CPTR_E_STATE, "handle was set up host-only");
  if (!r || !z || r == z) return (cptr_status)fail(s, CPTR_E_INVALID, "r and z must be distinct non-NULL device pointers");
  hipStream_t st = static_cast<hipStream_t>(stream);
  enqueue_apply(s, r, z, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (cptr_status)hip_fail(s, e, "kernel launch in cptr_apply");
  return CPTR_OK;
}

cptr_status cptr_stage1(cptr_solver s, const double* r, double* x1, void* stream) {
  if (!s) return CPTR_E_INVALID;
  if (!s->device) return (cptr_status)fail(s, CPTR_E_STATE, "handle was set up host-only");
  if (!r || !x1 || r == x1) return (cptr_status)fail(s, CPTR_E_INVALID, "r and x1 must be distinct non-NULL device pointers");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->prec == CPTR_PRECISION_FP32) {
    enqueue_stage1(s, s->p32, r, st, false);
    launch_prolong_e(s->host.nb, s->ne, s->eidx_h, s->p32.lev[0].e, x1, st);
  } else {
    enqueue_stage1(s, s->p64, r, st, false);
    launch_prolong_e(s->host.nb, s->ne, s->eidx_h, s->p64.lev[0].e, x1, st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (cptr_status)hip_fail(s, e, "kernel launch in cptr_stage1");
  return CPTR_OK;
}

cptr_status cptr_ilu_solve(cptr_solver s, const double* r, double* x, void* stream) {
  if (!s) return CPTR_E_INVALID;
  if (!s->device) return (cptr_status)fail(s, CPTR_E_STATE, "handle was set up host-only");
  if (!r || !x || r == x) return (cptr_status)fail(s, CPTR_E_INVALID, "r and x must be distinct non-NULL device pointers");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s->prec == CPTR_PRECISION_FP32)
    enqueue_stage2<float>(s, s->p32, r, nullptr, x, st);
  else
    enqueue_stage2<double>(s, s->p64, r, nullptr, x, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (cptr_status)hip_fail(s, e, "kernel launch in cptr_ilu_solve");
  return CPTR_OK;
}

cptr_status cptr_sweep_check(cptr_solver s, void* stream) {
  if (!s) return CPTR_E_INVALID;
  if (!s->device) return (cptr_status)fail(s, CPTR_E_STATE, "handle was set up host-only");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(s, hipMemcpyAsync(s->hhost + 140, s->hdev + 140, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(s, hipStreamSynchronize(st));
  launch_fill(1, s->hdev + 140, 0.0, st);
  HIP_TRY(s, hipGetLastError());
  if (s->hhost[140] != 0.0)
    return (cptr_status)fail(s, CPTR_E_HIP, "ILU sweep dependency wait exceeded its limit");
  return CPTR_OK;
}

cptr_status cptr_spmv(cptr_solver s, const double* x, double* y, void* stream) {
  if (!s) return CPTR_E_INVALID;
  if (!s->device) return (cptr_status)fail(s, CPTR_E_STATE, "handle was set up host-only");
  if (!x || !y || x == y) return (cptr_status)fail(s, CPTR_E_INVALID, "x and y must be distinct non-NULL device pointers");
  launch_bsr3_spmv(s->A, x, nullptr, y, false, static_cast<hipStream_t>(stream));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (cptr_status)hip_fail(s, e, "kernel launch in cptr_spmv");
  return CPTR_OK;
}

}  // extern "C"

namespace {

// Arguments of cptr_gmres_solve and its static-scratch variant.
int check_solve_args(cptr_solver s, const double* b, double* x, const cptr_solve_opts* o_in,
                     cptr_solve_opts& o) {
  if (!s) return CPTR_E_INVALID;
  if (!s->device) return fail(s, CPTR_E_STATE, "handle was set up host-only");
  if (!b || !x || b == x) return fail(s, CPTR_E_INVALID, "b and x must be distinct non-NULL device pointers");
  cptr_solve_opts_default(&o);
  if (o_in) o = *o_in;
  if (o.restart < 1 || o.restart > s->restart_cap)
    return fail(s, CPTR_E_INVALID,
                "restart must be in [1, " + std::to_string(s->restart_cap) + "] (the handle's max_restart)");
  if (o.flexible && !s->have_z)
    return fail(s, CPTR_E_STATE, "flexible solve on a handle set up with flexible_space = 0");
  if (o.max_iter < 0 || !(o.rtol >= 0.0))
    return fail(s, CPTR_E_INVALID, "max_iter must be >= 0 and rtol >= 0");
  return CPTR_OK;
}

// Restarted right-preconditioned (F)GMRES.  part: kRedBlocks * (kMaxRestart
// + 2) doubles of reduction partials; hd: 256 doubles for the Hessenberg
// column ([0,64) first Gram-Schmidt pass, [64,128) second, [128] ||w||^2),
// a norm ([136]) and the sweeps' wait-limit flag ([140], s->sweep_flag).
int gmres_run(cptr_solver s, const double* b, double* x, const cptr_solve_opts& o, cptr_solve_info* info,
              hipStream_t st, double* part, double* hd) {
  const double t0 = now_s();
  int rc = CPTR_OK;
  // the sweeps' wait-limit flag reports on this solve only
  launch_fill(1, hd + 140, 0.0, st);
  if (o.profile != 0 && s->ev_pool.empty()) {
    s->ev_pool.resize(512);
    for (auto& e : s->ev_pool)
      if (hipEventCreate(&e) != hipSuccess) e = nullptr;
  }
  s->profiling = o.profile != 0 && !s->ev_pool.empty() && s->ev_pool[0];
  s->profile_mask = o.profile == 1 ? ~0u : (uint32_t)o.profile >> 1;
  s->ev_used = 0;
  s->ev_pending.clear();
  // queue the next step's restriction early unless its phase is being timed
  const bool prefetch = s->ev_copy && !(s->profiling && (s->profile_mask & (1u << PH_RESTRICT)));
  bool pre = false;  // the restriction of the next basis vector is queued
  const int64_t N = s->N;
  const int m = o.restart;
  const int64_t ld = s->ldv;
  double* V = s->V;
  double* r = s->wr;
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), yv(m);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  hipEvent_t ev;

  double bnorm = 0.0;
  if ((rc = device_norm(s, b, bnorm, st, part, hd))) return rc;
  // the residual the next cycle starts from: b itself when x0 = 0
  const double* r0 = r;
  double beta = 0.0;
  if (o.x0_is_zero || bnorm == 0.0) {
    launch_fill(N, x, 0.0, st);
    r0 = b;
    beta = bnorm;
  } else {
    ph_begin(s, st, PH_SPMV, ev);
    launch_bsr3_spmv(s->A, x, b, r, true, st);
    ph_end(s, st, PH_SPMV, ev);
    if ((rc = device_norm(s, r, beta, st, part, hd))) return rc;
  }
  ph_harvest(s);
  const double bref = bnorm == 0.0 ? 1.0 : bnorm;
  const double target = o.rtol * bref;
  int it = 0, restarts = 0, converged = 0;
  double est = beta;
  for (;;) {
    if (beta <= target) {
      converged = 1;
      break;
    }
    if (it >= o.max_iter) break;
    launch_scale_host(N, r0, beta, V, st);
    pre = false;
    r0 = r;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = -1;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (size_t)j * ld;
      double* zj = o.flexible ? s->Z + (size_t)j * ld : s->wu;
      double* w = V + (size_t)(j + 1) * ld;
      enqueue_apply(s, vj, zj, st, pre);
      pre = false;
      ph_begin(s, st, PH_SPMV, ev);
      launch_bsr3_spmv(s->A, zj, nullptr, w, false, st);
      ph_end(s, st, PH_SPMV, ev);
      // classical Gram-Schmidt, twice
      ph_begin(s, st, PH_ARNOLDI, ev);
      const int nv = j + 1;
      launch_mdot(N, nv, V, ld, w, part, st);
      launch_reduce(nv, part, hd, 0, st);
      launch_maxpy_dot(N, nv, V, ld, hd, w, part, st);
      launch_reduce(nv, part, hd + 64, 0, st);
      launch_maxpy_norm(N, nv, V, ld, hd + 64, w, part, st);
      launch_reduce(1, part, hd + 128, 0, st);
      launch_scale(N, w, hd + 128, w, st);
      ph_end(s, st, PH_ARNOLDI, ev);
      HIP_TRY(s, hipMemcpyAsync(s->hhost, hd, 144 * sizeof(double), hipMemcpyDeviceToHost, st));
      if (prefetch && j + 1 < m) {
        // the next step's restriction reads only v_{j+1}: it is queued before
        // the host waits for the Hessenberg column, so the device has work
        // while the host decides whether that step happens (if it does not,
        // the restriction's level-0 output is scratch that nothing reads)
        HIP_TRY(s, hipEventRecord(s->ev_copy, st));
        enqueue_restrict(s, V + (size_t)(j + 1) * ld, st);
        pre = true;
        HIP_TRY(s, hipEventSynchronize(s->ev_copy));
      } else {
        HIP_TRY(s, hipStreamSynchronize(st));
      }
      {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(s, e, "kernel launch in cptr_gmres_solve");
      }
      ph_harvest(s);
      if (s->hhost[140] != 0.0)
        return fail(s, CPTR_E_HIP, "ILU sweep dependency wait exceeded its limit");
      for (int i = 0; i <= j; ++i) Hij(i, j) = s->hhost[i] + s->hhost[64 + i];
      const double hn = std::sqrt(std::max(0.0, s->hhost[128]));
      Hij(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        const double a = Hij(i, j), c = Hij(i + 1, j);
        Hij(i, j) = cs[i] * a + sn[i] * c;
        Hij(i + 1, j) = -sn[i] * a + cs[i] * c;
      }
      const double a = Hij(j, j), c = Hij(j + 1, j);
      const double rho = std::hypot(a, c);
      if (rho == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / rho;
        sn[j] = c / rho;
      }
      Hij(j, j) = rho;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      est = std::fabs(g[j + 1]);
      jend = j;
      if (hn == 0.0) break;
      if (est <= target || it >= o.max_iter) break;
    }
    const int k = jend + 1;
    for (int i = k - 1; i >= 0; --i) {
      double sum = g[i];
      for (int q = i + 1; q < k; ++q) sum -= Hij(i, q) * yv[q];
      yv[i] = Hij(i, i) != 0.0 ? sum / Hij(i, i) : 0.0;
    }
    ph_begin(s, st, PH_UPDATE, ev);
    if (o.flexible) {
      launch_update_host_coef(N, k, s->Z, ld, yv.data(), x, st);
      ph_end(s, st, PH_UPDATE, ev);
    } else {
      launch_fill(N, s->wt, 0.0, st);
      launch_update_host_coef(N, k, V, ld, yv.data(), s->wt, st);
      ph_end(s, st, PH_UPDATE, ev);
      enqueue_apply(s, s->wt, s->wu, st);
      ph_begin(s, st, PH_UPDATE, ev);
      std::vector<double> one(1, 1.0);
      launch_update_host_coef(N, 1, s->wu, ld, one.data(), x, st);
      ph_end(s, st, PH_UPDATE, ev);
    }
    ph_begin(s, st, PH_SPMV, ev);
    launch_bsr3_spmv(s->A, x, b, r, true, st);
    ph_end(s, st, PH_SPMV, ev);
    if ((rc = device_norm(s, r, beta, st, part, hd))) return rc;
    ph_harvest(s);
    if (beta > target && it < o.max_iter) ++restarts;
  }
  s->profiling = false;
  if (info) {
    info->iterations = it;
    info->restarts = restarts;
    info->converged = converged;
    info->rel_res_est = est / bref;
    info->rel_res_true = beta / bref;
    info->setup_s = s->setup_s;
    info->solve_s = now_s() - t0;
  }
  return converged ? CPTR_OK : CPTR_NOT_CONVERGED;
}

// Scratch of cptr_gmres_solve_static: the reduction partials and the
// Hessenberg / norm / flag slots, in one static device array per GPU instead
// of the handle's own.  Every call on a GPU shares that GPU's copy.
constexpr int64_t kStaticPartDoubles = (int64_t)kRedBlocks * (kMaxRestart + 2);
constexpr int64_t kStaticScratchDoubles = kStaticPartDoubles + 256;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// The current device's address of `scratch`, looked up once per device (with
// that device current) on the first call there.  The host-side name of the
// array is not a device address and is never passed to a kernel or a copy.
int static_scratch(cptr_solver s, double*& out) {
  out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(s, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(s, CPTR_E_HIP, "device ordinal out of range for the static scratch");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(s, CPTR_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  out = g_scratch_ptr[dev];
  return CPTR_OK;
}

}  // namespace

extern "C" {

cptr_status cptr_gmres_solve(cptr_solver s, const double* b, double* x, const cptr_solve_opts* o_in,
                             cptr_solve_info* info, void* stream) {
  cptr_solve_opts o;
  int rc = check_solve_args(s, b, x, o_in, o);
  if (rc) return (cptr_status)rc;
  return (cptr_status)gmres_run(s, b, x, o, info, static_cast<hipStream_t>(stream), s->part, s->hdev);
}

cptr_status cptr_gmres_solve_static(cptr_solver s, const double* b, double* x, const cptr_solve_opts* o_in,
                                    cptr_solve_info* info, void* stream) {
  cptr_solve_opts o;
  int rc = check_solve_args(s, b, x, o_in, o);
  if (rc) return (cptr_status)rc;
  if ((int64_t)kRedBlocks * (o.restart + 2) > kStaticPartDoubles)
    return (cptr_status)fail(s, CPTR_E_INVALID, "restart " + std::to_string(o.restart) +
                                                    " needs more reduction scratch than the static array holds");
  if (o.profile != 0)
    return (cptr_status)fail(s, CPTR_E_INVALID, "cptr_gmres_solve_static does not profile (profile must be 0)");
  double* sc = nullptr;
  if ((rc = static_scratch(s, sc))) return (cptr_status)rc;
  double* hd = sc + kStaticPartDoubles;
  s->sweep_flag = hd + 140;
  rc = gmres_run(s, b, x, o, info, static_cast<hipStream_t>(stream), sc, hd);
  s->sweep_flag = s->hdev + 140;
  return (cptr_status)rc;
}

cptr_status cptr_hierarchy_info(cptr_solver s, int32_t* n_levels, int64_t* rows, int64_t* nnz) {
  if (!s || !n_levels) return CPTR_E_INVALID;
  *n_levels = (int32_t)s->host.lev.size();
  for (size_t l = 0; l < s->host.lev.size(); ++l) {
    if (rows) rows[l] = s->host.lev[l].A.n;
    if (nnz) nnz[l] = s->host.lev[l].A.nnz();
  }
  return CPTR_OK;
}

cptr_status cptr_export(cptr_solver s, int32_t what, int32_t level, void* buf, int64_t bytes) {
  if (!s || !buf) return CPTR_E_INVALID;
  const HostSetup& h = s->host;
  const int L = (int)h.lev.size();
  auto put = [&](const void* src, int64_t nbytes) -> cptr_status {
    if (nbytes > bytes) return (cptr_status)fail(s, CPTR_E_INVALID, "export buffer too small");
    if (nbytes) std::memcpy(buf, src, (size_t)nbytes);
    return CPTR_OK;
  };
  const bool lvl_ok = level >= 0 && level < L;
  const bool has_p = level >= 0 && level + 1 < L;
  switch (what) {
    case CPTR_EXPORT_CF:
      if (!has_p) break;
      return put(h.lev[level].cf.data(), (int64_t)h.lev[level].cf.size() * 4);
    case CPTR_EXPORT_A_ROWPTR:
      if (!lvl_ok) break;
      return put(h.lev[level].A.rp.data(), (int64_t)h.lev[level].A.rp.size() * 8);
    case CPTR_EXPORT_A_COLS:
      if (!lvl_ok) break;
      return put(h.lev[level].A.ci.data(), (int64_t)h.lev[level].A.ci.size() * 4);
    case CPTR_EXPORT_A_VALS:
      if (!lvl_ok) break;
      return put(h.lev[level].A.v.data(), (int64_t)h.lev[level].A.v.size() * 8);
    case CPTR_EXPORT_P_ROWPTR:
      if (!has_p) break;
      return put(h.lev[level].P.rp.data(), (int64_t)h.lev[level].P.rp.size() * 8);
    case CPTR_EXPORT_P_COLS:
      if (!has_p) break;
      return put(h.lev[level].P.ci.data(), (int64_t)h.lev[level].P.ci.size() * 4);
    case CPTR_EXPORT_P_VALS:
      if (!has_p) break;
      return put(h.lev[level].P.v.data(), (int64_t)h.lev[level].P.v.size() * 8);
    case CPTR_EXPORT_W:
      return put(h.W.data(), (int64_t)h.W.size() * 8);
    case CPTR_EXPORT_DINV:
      if (!has_p && !(h.coarse_relax && level + 1 == (int)h.lev.size())) break;
      return put(h.lev[level].dinv.data(), (int64_t)h.lev[level].dinv.size() * 8);
    case CPTR_EXPORT_ILU_VALS:
      if (s->device_ilu)
        return (cptr_status)fail(s, CPTR_E_STATE, "this handle factors ILU(0) on the device (grid sweeps)");
      return put(h.ilu.data(), (int64_t)h.ilu.size() * 8);
    case CPTR_EXPORT_SWEEP: {
      const int32_t mode = !s->device ? -1
                           : s->use_grid ? CPTR_ILU_SWEEP_GRID
                           : s->sf_width > 0 ? CPTR_ILU_SWEEP_ONE_LAUNCH
                                             : CPTR_ILU_SWEEP_LEVELS;
      int32_t v[4] = {mode, s->use_grid ? s->grid[0] : 0, s->use_grid ? s->grid[1] : 0,
                      s->use_grid ? s->grid[2] : 0};
      return put(v, 16);
    }
    case CPTR_EXPORT_DENSE_TAIL: {
      if (!s->device) return (cptr_status)fail(s, CPTR_E_STATE, "a host-only handle has no device V-cycle");
      const int t = s->prec == CPTR_PRECISION_FP32 ? s->p32.tail : s->p64.tail;
      int32_t v[2] = {t, t > 0 ? (int32_t)h.lev[t].A.n : 0};
      return put(v, 8);
    }
    case CPTR_EXPORT_ILU_NLEVELS: {
      int32_t nl[2] = {h.n_fwd_levels, h.n_bwd_levels};
      return put(nl, 8);
    }
    case CPTR_EXPORT_DEVICE_PLAN: {
      if (s->device) return (cptr_status)fail(s, CPTR_E_STATE, "the handle already has its device half");
      std::vector<int64_t> plan;
      int64_t total = 0;
      s->plan = &plan;
      const int rc = cptr::measure_device(s, s->max_restart, s->flex_space, &total);
      s->plan = nullptr;
      if (rc) return (cptr_status)rc;
      plan.insert(plan.begin(), (int64_t)plan.size());
      return put(plan.data(), (int64_t)plan.size() * 8);
    }
    case CPTR_EXPORT_SETUP_TIMES: {
      double t[10];
      for (int k = 0; k < 8; ++k) t[k] = h.step_s[k];
      t[8] = s->device_build_s;
      t[9] = s->setup_s;
      return put(t, sizeof t);
    }
    case CPTR_EXPORT_SETUP_SITES: {
      const int32_t built = (int32_t)h.lev.size() - 1;
      const int32_t agg = std::min(built, s->agg_levels_used);
      const SetupSiteCounts& d = s->device_steps;
      const int32_t permille =
          d.first_points > 0 ? (int32_t)(1000 * d.split_points / d.first_points) : 0;
      int32_t v[15] = {d.strength, built, d.interp, std::max(0, built - s->agg_levels_used), d.galerkin, built,
                       d.multipass, agg, d.strength2, agg, d.split, h.first_passes, permille, d.hmis,
                       h.hmis_splits};
      return put(v, 60);
    }
    default:
      return (cptr_status)fail(s, CPTR_E_INVALID, "unknown export item");
  }
  return (cptr_status)fail(s, CPTR_E_INVALID, "level out of range for this export item");
}

cptr_status cptr_phase_times(cptr_solver s, double* ms, int64_t* count, int32_t n, int32_t reset) {
  if (!s || n < 0) return CPTR_E_INVALID;
  for (int k = 0; k < n && k < kPhases; ++k) {
    if (ms) ms[k] = s->phase_ms[k];
    if (count) count[k] = s->phase_cnt[k];
  }
  if (reset)
    for (int k = 0; k < kPhases; ++k) {
      s->phase_ms[k] = 0.0;
      s->phase_cnt[k] = 0;
    }
  return CPTR_OK;
}

}  // extern "C"
