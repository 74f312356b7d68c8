// host_setup.cpp -- host construction of the CPTR preconditioner.
//
// Paper sections: the two-stage form and the elliptic/hyperbolic split
// (Sec. 3, Eq. 3), the AMG parameters of the first stage and ILU(0) as the
// second stage (Sec. 3.1), CPTR's (p, T) elliptic block solved by system AMG
// (Sec. 3.2), the quasi-IMPES decomposition that produces that block
// (Sec. 5.2).  Where the paper only names a method, the reading used is the
// one stated at each function below.
//
// Compiled with FP contraction off so that the reduced elliptic matrix and the
// strength tests on it are bit-reproducible.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

#include "cptr.h"
#include "host_setup.hpp"

namespace cptr {

void parallel_for(int threads, int64_t n, const std::function<void(int64_t, int64_t, int)>& body) {
  if (threads <= 1 || n < 4096) {
    body(0, n, 0);
    return;
  }
  int t = (int)std::min<int64_t>(threads, n / 1024 + 1);
  std::vector<std::thread> pool;
  pool.reserve(t);
  for (int k = 0; k < t; ++k) {
    int64_t lo = n * k / t, hi = n * (k + 1) / t;
    pool.emplace_back([&body, lo, hi, k] { body(lo, hi, k); });
  }
  for (auto& th : pool) th.join();
}

// Rows [lo, hi) of thread t of parallel_for(threads, n, ...) were written, in
// row order, to part t; each thread of the same partition copies its part to
// offset rp[lo] of the result arrays (sized here).
template <class Part>
static void place_parts(int threads, int64_t n, const std::vector<int64_t>& rp, const std::vector<Part>& parts,
                        HVec<int32_t>& ci, HVec<double>& v) {
  ci.resize(rp[n]);
  v.resize(rp[n]);
  parallel_for(threads, n, [&](int64_t lo, int64_t, int t) {
    std::copy(parts[t].ci.begin(), parts[t].ci.end(), ci.begin() + rp[lo]);
    std::copy(parts[t].v.begin(), parts[t].v.end(), v.begin() + rp[lo]);
  });
}

static void place_parts(int threads, int64_t n, const std::vector<int64_t>& rp,
                        const std::vector<std::vector<int32_t>>& parts, HVec<int32_t>& ci) {
  ci.resize(rp[n]);
  parallel_for(threads, n, [&](int64_t lo, int64_t, int t) {
    std::copy(parts[t].begin(), parts[t].end(), ci.begin() + rp[lo]);
  });
}

int validate_bsr(int32_t nb, int64_t nnzb, const int32_t* rp, const int32_t* ci,
                 const double* v, std::string& err) {
  if (nb <= 0) return err = "A.n_block_rows must be positive", CPTR_E_INVALID;
  if (!rp || !ci || !v) return err = "A has a null array", CPTR_E_INVALID;
  if (rp[0] != 0) return err = "A.row_ptr[0] must be 0", CPTR_E_INVALID;
  if ((int64_t)rp[nb] != nnzb)
    return err = "A.row_ptr[n] != A.nnz_blocks", CPTR_E_INVALID;
  for (int32_t i = 0; i < nb; ++i) {
    if (rp[i + 1] < rp[i])
      return err = "A.row_ptr decreases at row " + std::to_string(i), CPTR_E_INVALID;
    bool diag = false;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= nb)
        return err = "A.col_idx out of range in row " + std::to_string(i), CPTR_E_INVALID;
      if (k > rp[i] && ci[k] <= ci[k - 1])
        return err = "A.col_idx unsorted or duplicated in row " + std::to_string(i),
               CPTR_E_INVALID;
      diag |= ci[k] == i;
    }
    if (!diag) return err = "A has no diagonal block in row " + std::to_string(i), CPTR_E_INVALID;
  }
  for (int64_t k = 0; k < nnzb * kBS * kBS; ++k)
    if (!std::isfinite(v[k]))
      return err = "A.values has a non-finite entry in block " + std::to_string(k / 9),
             CPTR_E_INVALID;
  return CPTR_OK;
}

// ---------------------------------------------------------------------------
// strength of connection, restricted to one unknown type ("unknown" system AMG)
// j is a strong dependency of i when j has i's type, j != i and
//   -sign(a_ii) a_ij >= theta * max over same-type k != i of (-sign(a_ii) a_ik),
// none when that maximum is not positive, and none when the same-type row sum
// exceeds max_row_sum * |a_ii| in magnitude (diagonally dominant row).
Csr strength_graph(const Csr& A, const std::vector<int32_t>& func, double theta, double mrs,
                   int threads) {
  Csr S;
  S.n = S.m = A.n;
  std::vector<int64_t> cnt(A.n + 1, 0);
  auto row_pass = [&](int32_t i, int32_t* out) -> int64_t {
    const int64_t b = A.rp[i], e = A.rp[i + 1];
    double aii = 0.0;
    for (int64_t k = b; k < e; ++k)
      if (A.ci[k] == i) aii = A.v[k];
    const double s = aii < 0.0 ? -1.0 : 1.0;
    double sum = 0.0, best = 0.0;
    bool any = false;
    const int32_t fi = func[i];
    for (int64_t k = b; k < e; ++k) {
      const int32_t j = A.ci[k];
      if (func[j] != fi) continue;
      sum += A.v[k];
      if (j != i) {
        const double t = -s * A.v[k];
        best = any ? std::max(best, t) : t;
        any = true;
      }
    }
    if (!any || !(best > 0.0)) return 0;
    if (mrs < 1.0 && std::fabs(sum) > mrs * std::fabs(aii)) return 0;
    const double cut = theta * best;
    int64_t c = 0;
    for (int64_t k = b; k < e; ++k) {
      const int32_t j = A.ci[k];
      if (j != i && func[j] == fi && -s * A.v[k] >= cut) {
        if (out) out[c] = j;
        ++c;
      }
    }
    return c;
  };
  parallel_for(threads, A.n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i) cnt[i + 1] = row_pass((int32_t)i, nullptr);
  });
  S.rp.assign(A.n + 1, 0);
  for (int32_t i = 0; i < A.n; ++i) S.rp[i + 1] = S.rp[i] + cnt[i + 1];
  S.ci.resize(S.rp[A.n]);
  parallel_for(threads, A.n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i) row_pass((int32_t)i, S.ci.data() + S.rp[i]);
  });
  return S;
}

// Rows of the transpose hold their columns in increasing order.  Large
// matrices are placed with atomic counters by several threads and each row is
// then sorted, which gives the same arrays as the sequential placement.
static Csr transpose(const Csr& a, int threads) {
  Csr t;
  t.n = a.m;
  t.m = a.n;
  const bool values = !a.v.empty();  // a pattern-only matrix stays pattern-only
  const int64_t nnz = a.nnz();
  t.ci.resize(nnz);
  t.v.resize(values ? nnz : 0);
  if (threads <= 1 || nnz < 4096) {
    t.rp.assign(t.n + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) ++t.rp[a.ci[k] + 1];
    for (int32_t j = 0; j < t.n; ++j) t.rp[j + 1] += t.rp[j];
    std::vector<int64_t> fill(t.rp.begin(), t.rp.end() - 1);
    for (int32_t i = 0; i < a.n; ++i)
      for (int64_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
        const int64_t p = fill[a.ci[k]]++;
        t.ci[p] = i;
        if (values) t.v[p] = a.v[k];
      }
    return t;
  }
  std::vector<int64_t> cnt(t.n + 1, 0);
  parallel_for(threads, a.n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t k = a.rp[lo]; k < a.rp[hi]; ++k) __atomic_fetch_add(&cnt[a.ci[k] + 1], 1, __ATOMIC_RELAXED);
  });
  t.rp.assign(t.n + 1, 0);
  for (int32_t j = 0; j < t.n; ++j) t.rp[j + 1] = t.rp[j] + cnt[j + 1];
  std::vector<int64_t> fill(t.rp.begin(), t.rp.end() - 1);
  parallel_for(threads, a.n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
        const int64_t p = __atomic_fetch_add(&fill[a.ci[k]], 1, __ATOMIC_RELAXED);
        t.ci[p] = (int32_t)i;
        if (values) t.v[p] = a.v[k];
      }
  });
  parallel_for(threads, t.n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t j = lo; j < hi; ++j)  // insertion sort: rows are short
      for (int64_t p = t.rp[j] + 1; p < t.rp[j + 1]; ++p) {
        const int32_t c = t.ci[p];
        const double x = values ? t.v[p] : 0.0;
        int64_t q = p;
        for (; q > t.rp[j] && t.ci[q - 1] > c; --q) {
          t.ci[q] = t.ci[q - 1];
          if (values) t.v[q] = t.v[q - 1];
        }
        t.ci[q] = c;
        if (values) t.v[q] = x;
      }
  });
  return t;
}

// ---------------------------------------------------------------------------
// HMIS coarsening on one domain = the Ruge-Stueben first pass.
// Measure = number of points that depend strongly on a point.  Points without
// any strong link become F.  The unassigned point of largest measure (>= 1,
// smallest index on ties) becomes C; unassigned points depending on it become
// F and each unassigned strong dependency of such a new F point gains 1; each
// unassigned strong dependency of the new C point loses 1.  Leftovers are F.
// Selection takes points from a bucket queue keyed on the measure.
namespace {
// Points keyed by a small non-negative integer measure; pick() returns the
// largest key, ties to the smallest index.  Each key value holds its points in
// a three-level bitset (64-way fan-out), so insert, erase and the smallest
// member of a key are O(1); the largest occupied key only drops when its set
// empties.  Keys below 1 are not selectable and are not stored.
struct BucketQueue {
  struct Bits {
    std::vector<uint64_t> w0, w1, w2;
    int64_t count = 0;
  };
  int32_t n;
  std::vector<int64_t> key;  // stored key of each point, -1 = absent
  std::vector<Bits> bucket;
  int64_t top = 0;           // an upper bound of the largest occupied key
  explicit BucketQueue(int32_t n_) : n(n_), key(n_, -1) {}
  Bits& at(int64_t k) {
    if ((int64_t)bucket.size() <= k) bucket.resize(k + 1);
    Bits& b = bucket[k];
    if (b.w0.empty()) {
      b.w0.assign(((size_t)n + 63) / 64, 0);
      b.w1.assign((b.w0.size() + 63) / 64, 0);
      b.w2.assign((b.w1.size() + 63) / 64, 0);
    }
    return b;
  }
  void insert(int32_t i, int64_t k) {
    Bits& b = at(k);
    const size_t a = (size_t)i >> 6, c = a >> 6, d = c >> 6;
    if (!b.w0[a]) {
      if (!b.w1[c]) b.w2[d] |= 1ull << (c & 63);
      b.w1[c] |= 1ull << (a & 63);
    }
    b.w0[a] |= 1ull << (i & 63);
    ++b.count;
    if (k > top) top = k;
  }
  void erase(int32_t i, int64_t k) {
    Bits& b = bucket[k];
    const size_t a = (size_t)i >> 6, c = a >> 6, d = c >> 6;
    b.w0[a] &= ~(1ull << (i & 63));
    if (!b.w0[a]) {
      b.w1[c] &= ~(1ull << (a & 63));
      if (!b.w1[c]) b.w2[d] &= ~(1ull << (c & 63));
    }
    --b.count;
  }
  void set(int32_t i, int64_t k) {
    if (key[i] >= 1) erase(i, key[i]);
    key[i] = k >= 1 ? k : -1;
    if (k >= 1) insert(i, k);
  }
  // the selected point, or -1 when no key >= 1 is left
  int32_t pick() {
    while (top >= 1 && ((int64_t)bucket.size() <= top || bucket[top].count == 0)) --top;
    if (top < 1) return -1;
    const Bits& b = bucket[top];
    size_t d = 0;
    while (!b.w2[d]) ++d;
    const size_t c = d * 64 + (size_t)__builtin_ctzll(b.w2[d]);
    const size_t a = c * 64 + (size_t)__builtin_ctzll(b.w1[c]);
    return (int32_t)(a * 64 + (size_t)__builtin_ctzll(b.w0[a]));
  }
};
}  // namespace

// The pass over the undecided points (cf 0) of S, given their measures; every
// decided point must have no strong link to an undecided one.
static void first_pass_run(const Csr& S, const Csr& St, std::vector<int32_t>& cf, std::vector<int64_t>& lam) {
  const int32_t n = S.n;
  BucketQueue queue(n);
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 0) queue.set(i, lam[i]);
  auto refresh = [&](int32_t m) { queue.set(m, cf[m] == 0 ? lam[m] : -1); };
  for (;;) {
    const int32_t c = queue.pick();
    if (c < 0) break;
    cf[c] = 1;
    refresh(c);
    for (int64_t k = St.rp[c]; k < St.rp[c + 1]; ++k) {
      const int32_t f = St.ci[k];
      if (cf[f] != 0) continue;
      cf[f] = -1;
      refresh(f);
      for (int64_t q = S.rp[f]; q < S.rp[f + 1]; ++q) {
        const int32_t m = S.ci[q];
        if (cf[m] == 0) {
          ++lam[m];
          refresh(m);
        }
      }
    }
    for (int64_t k = S.rp[c]; k < S.rp[c + 1]; ++k) {
      const int32_t m = S.ci[k];
      if (cf[m] == 0) {
        --lam[m];
        refresh(m);
      }
    }
  }
  for (auto& x : cf)
    if (x == 0) x = -1;
}

std::vector<int32_t> first_pass_split(const Csr& S, int threads) {
  const int32_t n = S.n;
  const Csr St = transpose(S, threads);
  std::vector<int32_t> cf(n, 0);
  std::vector<int64_t> lam(n);
  for (int32_t i = 0; i < n; ++i) {
    lam[i] = St.rp[i + 1] - St.rp[i];
    if (lam[i] == 0 && S.rp[i + 1] == S.rp[i]) cf[i] = -1;
  }
  first_pass_run(S, St, cf, lam);
  return cf;
}

// The pass leaves the weakly connected components of S independent (it reads
// and changes only a pick's strong neighbours, and a component's picks come
// in the order a pass over it alone takes them), so components already
// passed elsewhere (cf +-1, as are points without links) are final; the rest
// (cf 0) is passed here.
std::vector<int32_t> first_pass_finish(const Csr& S, std::vector<int32_t> cf, int threads) {
  const int32_t n = S.n;
  if (std::find(cf.begin(), cf.end(), 0) == cf.end()) return cf;
  const Csr St = transpose(S, threads);
  std::vector<int64_t> lam(n);
  for (int32_t i = 0; i < n; ++i) lam[i] = St.rp[i + 1] - St.rp[i];
  first_pass_run(S, St, cf, lam);
  return cf;
}

// ---------------------------------------------------------------------------
// HMIS (De Sterck, Yang, Heys 2006) over blocks of `block` consecutive points,
// a block standing for one processor's subdomain:
//  1. the first pass above inside every block, on the strong links with both
//     ends in the block; its C points are C;
//  2. a point that is not C and depends strongly on a C point is F;
//  3. PMIS on the rest, U: cnt_i = number of points of U depending strongly on
//     i; cnt_i = 0 makes i F; then in rounds every point of U whose priority
//     (cnt_i, splitmix64(i), i) beats that of each strong neighbour still in
//     U (links either way) is C, and the points of U depending on one of those
//     are F.
// One block (block <= 0 or >= n) is the first pass itself: its picks make
// exactly the F points of step 2 and every leftover has cnt = 0.
namespace {
// SplitMix64 (Steele, Lea, Flood 2014): the output for counter value x.
inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline bool beats(int64_t ca, int32_t a, int64_t cb, int32_t b) {
  if (ca != cb) return ca > cb;
  const uint64_t ha = splitmix64((uint64_t)a), hb = splitmix64((uint64_t)b);
  if (ha != hb) return ha > hb;
  return a > b;
}
}  // namespace

std::vector<int32_t> hmis_split(const Csr& S, int32_t block, int threads) {
  const int32_t n = S.n;
  if (block <= 0 || block >= n) return first_pass_split(S, threads);
  const int nthreads = std::max(1, threads);
  const int64_t nblocks = ((int64_t)n + block - 1) / block;
  std::vector<int32_t> cf(n, 0);
  // step 1: the blocks are independent
  parallel_for(nthreads, nblocks, [&](int64_t b0, int64_t b1, int) {
    Csr sub;
    for (int64_t b = b0; b < b1; ++b) {
      const int32_t lo = (int32_t)(b * block), hi = (int32_t)std::min<int64_t>(n, (b + 1) * (int64_t)block);
      sub.n = sub.m = hi - lo;
      sub.rp.assign(sub.n + 1, 0);
      sub.ci.clear();
      for (int32_t i = lo; i < hi; ++i) {
        for (int64_t a = S.rp[i]; a < S.rp[i + 1]; ++a)
          if (S.ci[a] >= lo && S.ci[a] < hi) sub.ci.push_back(S.ci[a] - lo);
        sub.rp[i - lo + 1] = (int64_t)sub.ci.size();
      }
      const std::vector<int32_t> bcf = first_pass_split(sub, 1);
      for (int32_t i = lo; i < hi; ++i) cf[i] = bcf[i - lo] == 1 ? 1 : 0;
    }
  });
  // step 2: marks first, then applied, so every scan sees the C points only
  std::vector<uint8_t> dep_c(n, 0);
  parallel_for(nthreads, n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i) {
      if (cf[i] == 1) continue;
      for (int64_t a = S.rp[i]; a < S.rp[i + 1]; ++a)
        if (cf[S.ci[a]] == 1) {
          dep_c[i] = 1;
          break;
        }
    }
  });
  for (int32_t i = 0; i < n; ++i)
    if (dep_c[i]) cf[i] = -1;
  // step 3
  std::vector<int32_t> und;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 0) und.push_back(i);
  if (und.empty()) return cf;
  const Csr St = transpose(S, nthreads);
  std::vector<int64_t> cnt(n, 0);
  for (int32_t i : und)
    for (int64_t a = St.rp[i]; a < St.rp[i + 1]; ++a) cnt[i] += cf[St.ci[a]] == 0;
  std::vector<int32_t> rest;
  for (int32_t i : und)
    if (cnt[i] == 0)
      cf[i] = -1;
    else
      rest.push_back(i);
  std::vector<int32_t> fresh;
  std::vector<uint8_t> is_new(n, 0);
  while (!rest.empty()) {
    fresh.clear();
    for (int32_t i : rest) {
      bool top = true;
      for (int64_t a = S.rp[i]; a < S.rp[i + 1] && top; ++a)
        if (cf[S.ci[a]] == 0 && beats(cnt[S.ci[a]], S.ci[a], cnt[i], i)) top = false;
      for (int64_t a = St.rp[i]; a < St.rp[i + 1] && top; ++a)
        if (cf[St.ci[a]] == 0 && beats(cnt[St.ci[a]], St.ci[a], cnt[i], i)) top = false;
      if (top) fresh.push_back(i);
    }
    for (int32_t i : fresh) {
      cf[i] = 1;
      is_new[i] = 1;
    }
    std::vector<int32_t> next;
    for (int32_t i : rest) {
      if (cf[i] != 0) continue;
      bool dep = false;
      for (int64_t a = S.rp[i]; a < S.rp[i + 1] && !dep; ++a) dep = is_new[S.ci[a]] != 0;
      if (dep)
        cf[i] = -1;
      else
        next.push_back(i);
    }
    for (int32_t i : fresh) is_new[i] = 0;
    rest.swap(next);
  }
  return cf;
}

// ---------------------------------------------------------------------------
// Aggressive coarsening (the "aggregate level" of Sec. 3.1).  Among the C
// points of a first pass, C point j is a distance-two strong dependency of C
// point i when i depends strongly on j directly or through one intermediate
// point of any kind; a second first pass over the C points on that graph keeps
// the final C points.  Rows of the distance-two graph are the C points in
// ascending order, each row sorted.
Csr distance_two_strength(const Csr& S, const std::vector<int32_t>& cf, int threads) {
  const int32_t n = S.n;
  std::vector<int32_t> cidx(n, -1), cpts;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 1) {
      cidx[i] = (int32_t)cpts.size();
      cpts.push_back(i);
    }
  const int32_t nc = (int32_t)cpts.size();
  const int nthreads = std::max(1, threads);
  std::vector<std::vector<int32_t>> part(nthreads);
  std::vector<int64_t> len(nc + 1, 0);
  parallel_for(nthreads, nc, [&](int64_t lo, int64_t hi, int t) {
    std::vector<int32_t> seen(n, -1);
    auto& out = part[t];
    for (int64_t r = lo; r < hi; ++r) {
      const int32_t i = cpts[r];
      const size_t start = out.size();
      auto take = [&](int32_t j) {
        if (j != i && cf[j] == 1 && seen[j] != i) {
          seen[j] = i;
          out.push_back(cidx[j]);
        }
      };
      for (int64_t a = S.rp[i]; a < S.rp[i + 1]; ++a) {
        const int32_t k = S.ci[a];
        take(k);
        for (int64_t b = S.rp[k]; b < S.rp[k + 1]; ++b) take(S.ci[b]);
      }
      std::sort(out.begin() + start, out.end());
      len[r + 1] = (int64_t)(out.size() - start);
    }
  });
  Csr S2;
  S2.n = S2.m = nc;
  S2.rp.assign(nc + 1, 0);
  for (int32_t r = 0; r < nc; ++r) S2.rp[r + 1] = S2.rp[r] + len[r + 1];
  place_parts(nthreads, nc, S2.rp, part, S2.ci);
  return S2;
}

std::vector<int32_t> aggressive_split(const Csr& S, int32_t block, int threads) {
  std::vector<int32_t> cf1 = hmis_split(S, block, threads);
  const Csr S2 = distance_two_strength(S, cf1, threads);
  const std::vector<int32_t> cf2 = hmis_split(S2, block, threads);
  std::vector<int32_t> cf(S.n, -1);
  for (int32_t i = 0, c = 0; i < S.n; ++i)
    if (cf1[i] == 1) cf[i] = cf2[c++] == 1 ? 1 : -1;
  return cf;
}

// ---------------------------------------------------------------------------
// Multipass interpolation (Stueben 2001) for the aggressive level, within one
// unknown type.  F points are handled in passes: pass 1 takes the F points
// with strong C points, pass m > 1 the remaining F points with strong points
// handled in earlier passes; P_i = those strong points.  In row i, with
// "negative" meaning of sign opposite to a_ii:
//   alpha = (negative same-type off-diagonal sum) / (negative sum over P_i),
//   d     = a_ii + (the rest of the same-type off-diagonal sum),
//   c_k   = -alpha a_ik / d  for k in P_i,   w_ij = sum_k c_k w_kj
// (w_kj = identity for C points).  Sums run over row i in column order and the
// terms of w_ij in increasing k, which is also the oracle's order.  A row with
// d = 0 is empty; unreached F points get empty rows; no truncation.
Csr multipass_interp(const Csr& A, const Csr& S, const std::vector<int32_t>& cf,
                     const std::vector<int32_t>& func, int threads) {
  const int32_t n = A.n;
  std::vector<int32_t> cidx(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  std::vector<int32_t> pass(n, -1);
  // rows live in one growing store: row i = [start[i], start[i] + len[i])
  std::vector<int64_t> start(n, 0), len(n, 0);
  std::vector<int32_t> sc;
  std::vector<double> sv;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 1) {
      pass[i] = 0;
      start[i] = (int64_t)sc.size();
      len[i] = 1;
      sc.push_back(cidx[i]);
      sv.push_back(1.0);
    }
  const int nthreads = std::max(1, threads);
  for (int m = 1;; ++m) {
    std::vector<int32_t> now;
    for (int32_t i = 0; i < n; ++i) {
      if (pass[i] != -1) continue;
      for (int64_t a = S.rp[i]; a < S.rp[i + 1]; ++a)
        if (pass[S.ci[a]] != -1 && pass[S.ci[a]] < m) {
          now.push_back(i);
          break;
        }
    }
    if (now.empty()) break;
    struct Out {
      std::vector<int32_t> c;
      std::vector<double> w;
      std::vector<int64_t> off;  // per row of this part: offset into c / w
    };
    std::vector<Out> parts(nthreads);
    std::vector<int64_t> chunk_lo(nthreads + 1, 0);
    parallel_for(nthreads, (int64_t)now.size(), [&](int64_t lo, int64_t hi, int t) {
      chunk_lo[t] = lo;
      Out& o = parts[t];
      std::vector<double> acc(nc, 0.0);
      std::vector<int32_t> seen(nc, -1), touched;
      for (int64_t r = lo; r < hi; ++r) {
        const int32_t i = now[r];
        o.off.push_back((int64_t)o.c.size());
        // is column q (of row i) in P_i?  walk S_i alongside the sorted row
        auto in_p = [&](int64_t& sa, int32_t q) {
          while (sa < S.rp[i + 1] && S.ci[sa] < q) ++sa;
          return sa < S.rp[i + 1] && S.ci[sa] == q && pass[q] != -1 && pass[q] < m;
        };
        double aii = 0.0, negn = 0.0, posn = 0.0, negp = 0.0;
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
          if (A.ci[k] == i) aii = A.v[k];
        int64_t sa = S.rp[i];
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          const int32_t j = A.ci[k];
          if (j == i || func[j] != func[i]) continue;
          const bool opp = aii < 0.0 ? A.v[k] > 0.0 : A.v[k] < 0.0;
          if (opp)
            negn += A.v[k];
          else
            posn += A.v[k];
          if (opp && in_p(sa, j)) negp += A.v[k];
        }
        const double d = aii + posn;
        touched.clear();
        if (d != 0.0 && negp != 0.0) {
          const double alpha = negn / negp;
          sa = S.rp[i];
          for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t q = A.ci[k];
            if (q == i || func[q] != func[i] || !in_p(sa, q)) continue;
            const double c = -alpha * A.v[k] / d;
            for (int64_t e = start[q]; e < start[q] + len[q]; ++e) {
              const int32_t j = sc[e];
              if (seen[j] != i) {
                seen[j] = i;
                acc[j] = 0.0;
                touched.push_back(j);
              }
              acc[j] += c * sv[e];
            }
          }
        }
        std::sort(touched.begin(), touched.end());
        for (int32_t j : touched) {
          o.c.push_back(j);
          o.w.push_back(acc[j]);
        }
      }
      o.off.push_back((int64_t)o.c.size());
    });
    for (int t = 0; t < nthreads; ++t) {
      const Out& o = parts[t];
      for (size_t r = 0; r + 1 < o.off.size(); ++r) {
        const int32_t i = now[chunk_lo[t] + (int64_t)r];
        start[i] = (int64_t)sc.size();
        len[i] = o.off[r + 1] - o.off[r];
        sc.insert(sc.end(), o.c.begin() + o.off[r], o.c.begin() + o.off[r + 1]);
        sv.insert(sv.end(), o.w.begin() + o.off[r], o.w.begin() + o.off[r + 1]);
      }
    }
    for (int32_t i : now) pass[i] = m;
  }
  Csr P;
  P.n = n;
  P.m = nc;
  P.rp.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) P.rp[i + 1] = P.rp[i] + len[i];
  P.ci.resize(P.rp[n]);
  P.v.resize(P.rp[n]);
  parallel_for(nthreads, n, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t e = 0; e < len[i]; ++e) {
        P.ci[P.rp[i] + e] = sc[start[i] + e];
        P.v[P.rp[i] + e] = sv[start[i] + e];
      }
  });
  return P;
}

// ---------------------------------------------------------------------------
// Extended+i interpolation (De Sterck, Falgout, Nolting, Yang, 2008), within
// one unknown type.  For an F point i: the interpolatory set is its strong C
// points plus the strong C points of its strong F points.  Each off-diagonal
// a_im of i's type goes (a) to w_im if m is in the set, (b) for a strong F
// point m, through row m: a_ml (l in the set or l = i, a_ml of sign opposite
// to a_mm) shares a_im in proportion to a_ml, the share of l = i going to the
// diagonal; if those a_ml sum to zero a_im goes to the diagonal, (c) otherwise
// to the diagonal.  w = -(collected) / (collected diagonal).  Rows keep the
// pmax largest |w| (smaller column on ties), rescaled to the full row sum.
namespace {
struct Entry {
  int32_t col;
  double w;
};
}  // namespace

Csr extended_i_interp(const Csr& A, const Csr& S, const std::vector<int32_t>& cf,
                      const std::vector<int32_t>& func, int pmax, int threads) {
  const int32_t n = A.n;
  std::vector<int32_t> cidx(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == 1) cidx[i] = nc++;
  int nthreads = std::max(1, threads);
  struct Part {
    std::vector<int32_t> ci;
    std::vector<double> v;
  };
  std::vector<Part> parts(nthreads);
  std::vector<int64_t> rowlen(n + 1, 0);
  std::vector<int64_t> chunk_lo(nthreads + 1, 0);
  auto a_diag = [&](int32_t r) {
    for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k)
      if (A.ci[k] == r) return A.v[k];
    return 0.0;
  };
  parallel_for(nthreads, n, [&](int64_t lo, int64_t hi, int t) {
    Part& out = parts[t];
    std::vector<int32_t> set;     // interpolatory C points of the current row
    std::vector<double> acc;
    std::vector<Entry> row;
    for (int64_t ii = lo; ii < hi; ++ii) {
      const int32_t i = (int32_t)ii;
      row.clear();
      if (cf[i] == 1) {
        row.push_back({cidx[i], 1.0});
      } else {
        set.clear();
        auto in_set = [&](int32_t c) -> int {
          for (size_t q = 0; q < set.size(); ++q)
            if (set[q] == c) return (int)q;
          return -1;
        };
        auto strong = [&](int32_t m) {
          for (int64_t k = S.rp[i]; k < S.rp[i + 1]; ++k)
            if (S.ci[k] == m) return true;
          return false;
        };
        for (int64_t k = S.rp[i]; k < S.rp[i + 1]; ++k) {
          const int32_t j = S.ci[k];
          if (cf[j] == 1) {
            if (in_set(j) < 0) set.push_back(j);
          } else {
            for (int64_t q = S.rp[j]; q < S.rp[j + 1]; ++q) {
              const int32_t l = S.ci[q];
              if (cf[l] == 1 && in_set(l) < 0) set.push_back(l);
            }
          }
        }
        if (!set.empty()) {
          acc.assign(set.size(), 0.0);
          double dg = a_diag(i);
          for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t m = A.ci[k];
            if (m == i || func[m] != func[i]) continue;
            const double aim = A.v[k];
            const int pos = in_set(m);
            if (pos >= 0) {
              acc[pos] += aim;
              continue;
            }
            if (cf[m] != 1 && strong(m)) {
              const double sm = a_diag(m) < 0.0 ? -1.0 : 1.0;
              double den = 0.0;
              for (int64_t q = A.rp[m]; q < A.rp[m + 1]; ++q) {
                const int32_t l = A.ci[q];
                const double aml = A.v[q];
                if (sm * aml < 0.0 && (l == i || in_set(l) >= 0)) den += aml;
              }
              if (den == 0.0) {
                dg += aim;
                continue;
              }
              for (int64_t q = A.rp[m]; q < A.rp[m + 1]; ++q) {
                const int32_t l = A.ci[q];
                const double aml = A.v[q];
                if (!(sm * aml < 0.0)) continue;
                const double share = aim * aml / den;
                if (l == i) {
                  dg += share;
                } else {
                  const int p = in_set(l);
                  if (p >= 0) acc[p] += share;
                }
              }
              continue;
            }
            dg += aim;
          }
          if (dg != 0.0)
            for (size_t q = 0; q < set.size(); ++q) row.push_back({cidx[set[q]], -acc[q] / dg});
        }
      }
      if (pmax > 0 && (int)row.size() > pmax) {
        double total = 0.0, kept = 0.0;
        for (const auto& e : row) total += e.w;
        std::partial_sort(row.begin(), row.begin() + pmax, row.end(),
                          [](const Entry& a, const Entry& b) {
                            const double fa = std::fabs(a.w), fb = std::fabs(b.w);
                            return fa != fb ? fa > fb : a.col < b.col;
                          });
        row.resize(pmax);
        for (const auto& e : row) kept += e.w;
        if (kept != 0.0) {
          const double scale = total / kept;
          for (auto& e : row) e.w *= scale;
        }
      }
      std::sort(row.begin(), row.end(), [](const Entry& a, const Entry& b) { return a.col < b.col; });
      rowlen[i + 1] = (int64_t)row.size();
      for (const auto& e : row) {
        out.ci.push_back(e.col);
        out.v.push_back(e.w);
      }
    }
    chunk_lo[t + 1] = hi;  // rows of this part end at hi
  });
  Csr P;
  P.n = n;
  P.m = nc;
  P.rp.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) P.rp[i + 1] = P.rp[i] + rowlen[i + 1];
  place_parts(nthreads, n, P.rp, parts, P.ci, P.v);
  return P;
}

// ---------------------------------------------------------------------------
// Sparse product C = X Y, rows in parallel.  Each output entry is accumulated
// over the stored entries x_ik in increasing k (and, within row k of Y, in
// stored order), starting from 0.0, in a small open-addressing table per row;
// the Galerkin operator R A P is formed as R (A P).  With FP contraction off
// this summation order fixes every coarse operator to the last bit, so the
// strength tests of the next level see exactly the same numbers however the
// rows are distributed over threads.
static Csr spgemm(const Csr& X, const Csr& Y, int threads) {
  const int32_t n = X.n;
  int nthreads = std::max(1, threads);
  struct Part {
    std::vector<int32_t> ci;
    std::vector<double> v;
  };
  std::vector<Part> parts(nthreads);
  std::vector<int64_t> len(n + 1, 0);
  parallel_for(nthreads, n, [&](int64_t lo, int64_t hi, int t) {
    std::vector<int32_t> keys(64, -1);
    std::vector<double> vals(64, 0.0);
    std::vector<int32_t> used;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = lo; i < hi; ++i) {
      int64_t bound = 0;
      for (int64_t q = X.rp[i]; q < X.rp[i + 1]; ++q) bound += Y.rp[X.ci[q] + 1] - Y.rp[X.ci[q]];
      size_t want = 64;
      while ((int64_t)want < 2 * bound) want <<= 1;
      if (want > keys.size()) {
        keys.assign(want, -1);
        vals.assign(want, 0.0);
      }
      const uint32_t mask = (uint32_t)keys.size() - 1;
      used.clear();
      for (int64_t q = X.rp[i]; q < X.rp[i + 1]; ++q) {
        const int32_t k = X.ci[q];
        const double xik = X.v[q];
        for (int64_t p = Y.rp[k]; p < Y.rp[k + 1]; ++p) {
          const int32_t col = Y.ci[p];
          uint32_t hsh = ((uint32_t)col * 2654435761u) & mask;
          while (keys[hsh] != -1 && keys[hsh] != col) hsh = (hsh + 1) & mask;
          if (keys[hsh] == -1) {
            keys[hsh] = col;
            vals[hsh] = 0.0;
            used.push_back((int32_t)hsh);
          }
          vals[hsh] += xik * Y.v[p];
        }
      }
      row.clear();
      for (int32_t hh : used) {
        row.emplace_back(keys[hh], vals[hh]);
        keys[hh] = -1;
      }
      std::sort(row.begin(), row.end());
      len[i + 1] = (int64_t)row.size();
      for (auto& e : row) {
        parts[t].ci.push_back(e.first);
        parts[t].v.push_back(e.second);
      }
    }
  });
  Csr C;
  C.n = n;
  C.m = Y.m;
  C.rp.assign(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) C.rp[i + 1] = C.rp[i] + len[i + 1];
  place_parts(nthreads, n, C.rp, parts, C.ci, C.v);
  return C;
}

static Csr galerkin(const Csr& R, const Csr& A, const Csr& P, int threads) {
  Csr AP = spgemm(A, P, threads);
  return spgemm(R, AP, threads);
}

// l1-Jacobi (point blocks): d_i = a_ii + sign(a_ii) sum_{j != i} |a_ij|.
static int l1_inverse_diag(const Csr& A, std::vector<double>& dinv, int threads, std::string& err) {
  dinv.resize(A.n);
  std::vector<int32_t> first_bad(std::max(1, threads), INT32_MAX);
  parallel_for(threads, A.n, [&](int64_t lo, int64_t hi, int t) {
    for (int64_t i = lo; i < hi; ++i) {
      double d = 0.0, off = 0.0;
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        if (A.ci[k] == i) d = A.v[k];
        else off += std::fabs(A.v[k]);
      }
      const double l1 = d < 0.0 ? d - off : d + off;
      if (l1 == 0.0) first_bad[t] = std::min(first_bad[t], (int32_t)i);
      dinv[i] = l1 == 0.0 ? 0.0 : 1.0 / l1;
    }
  });
  const int32_t bad = *std::min_element(first_bad.begin(), first_bad.end());
  if (bad != INT32_MAX)
    return err = "zero smoother diagonal at AMG row " + std::to_string(bad), CPTR_E_ZERO_PIVOT;
  return CPTR_OK;
}

static int dense_lu(int n, std::vector<double>& a, std::vector<int32_t>& piv, std::string& err) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[(size_t)i * n + k]) > std::fabs(a[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (a[(size_t)p * n + k] == 0.0)
      return err = "singular coarsest AMG matrix", CPTR_E_SINGULAR_COARSE;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
    const double inv = a[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      const double l = a[(size_t)i * n + k] / inv;
      a[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
    }
  }
  return CPTR_OK;
}

// 3x3 inverse by Gauss-Jordan with partial pivoting; false when singular.
static bool inv3(const double* m, double* out) {
  double a[3][6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 6; ++c) a[r][c] = c < 3 ? m[r * 3 + c] : (c - 3 == r ? 1.0 : 0.0);
  for (int k = 0; k < 3; ++k) {
    int p = k;
    for (int r = k + 1; r < 3; ++r)
      if (std::fabs(a[r][k]) > std::fabs(a[p][k])) p = r;
    if (a[p][k] == 0.0) return false;
    if (p != k)
      for (int c = 0; c < 6; ++c) std::swap(a[k][c], a[p][c]);
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

static inline void mm3(const double* a, const double* b, double* c) {
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int q = 0; q < 3; ++q) s += a[r * 3 + q] * b[q * 3 + k];
      c[r * 3 + k] = s;
    }
}

// ---------------------------------------------------------------------------
int build_host_setup(int32_t nb, const int32_t* rp, const int32_t* ci, const double* v,
                     const int32_t* elliptic, int ne, const SetupParams& prm, HostSetup& h,
                     std::string& err) {
  using clock = std::chrono::steady_clock;
  auto tick = clock::now();
  // adds the time since the last mark to step k
  auto mark = [&](int k) {
    const auto now = clock::now();
    h.step_s[k] += std::chrono::duration<double>(now - tick).count();
    tick = now;
  };
  const int threads = std::max(1, prm.threads);
  h.nb = nb;
  h.ne = ne;
  h.nh = kBS - ne;
  bool used[kBS] = {false, false, false};
  for (int e = 0; e < ne; ++e) {
    h.eidx[e] = elliptic[e];
    used[elliptic[e]] = true;
  }
  for (int c = 0, t = 0; c < kBS; ++c)
    if (!used[c]) h.hidx[t++] = c;
  const int64_t nnzb = rp[nb];
  h.rp.assign(rp, rp + nb + 1);
  h.ci.assign(ci, ci + nnzb);
  h.av = v;  // read in place: no copy of the largest input
  h.diag.resize(nb);
  parallel_for(threads, nb, [&](int64_t lo, int64_t hi, int) {
    for (int64_t i = lo; i < hi; ++i)
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) h.diag[i] = k;
  });
  mark(kStepValidate);

  // ---- quasi-IMPES weights W_i = A_ii[E,H] A_ii[H,H]^-1 (Sec. 5.2) ----
  const int nh = h.nh;
  h.W.assign((size_t)nb * ne * nh, 0.0);
  if (prm.quasi_impes) {
    std::vector<int32_t> first_bad(threads, INT32_MAX);
    parallel_for(threads, nb, [&](int64_t lo, int64_t hi, int th) {
      for (int64_t i = lo; i < hi; ++i) {
        const double* D = &h.av[(size_t)h.diag[i] * 9];
        double* w = &h.W[(size_t)i * ne * nh];
        if (nh == 1) {
          const double dhh = D[h.hidx[0] * 3 + h.hidx[0]];
          if (dhh == 0.0) {
            first_bad[th] = std::min(first_bad[th], (int32_t)i);
            continue;
          }
          for (int e = 0; e < ne; ++e) w[e] = D[h.eidx[e] * 3 + h.hidx[0]] / dhh;
        } else {  // nh == 2: explicit 2x2 inverse
          const int p = h.hidx[0], q = h.hidx[1];
          const double a = D[p * 3 + p], b = D[p * 3 + q], c = D[q * 3 + p], d = D[q * 3 + q];
          const double det = a * d - b * c;
          if (det == 0.0) {
            first_bad[th] = std::min(first_bad[th], (int32_t)i);
            continue;
          }
          const double ia = d / det, ib = -b / det, ic = -c / det, id = a / det;
          for (int e = 0; e < ne; ++e) {
            const double u = D[h.eidx[e] * 3 + p], t = D[h.eidx[e] * 3 + q];
            w[e * 2 + 0] = u * ia + t * ic;
            w[e * 2 + 1] = u * ib + t * id;
          }
        }
      }
    });
    const int32_t bad = *std::min_element(first_bad.begin(), first_bad.end());
    if (bad != INT32_MAX)
      return err = "singular hyperbolic diagonal block in row " + std::to_string(bad),
             CPTR_E_ZERO_PIVOT;
  }
  if (prm.after_weights) prm.after_weights(h);
  // ---- system AMG on Ahat, unknowns interleaved per cell (Sec. 3.1, 3.2) ----
  // Level 0 is Ahat as a scalar matrix, formed here from the reduced elliptic
  // blocks Ahat_ij = A_ij[E,E] - W_i A_ij[H,E]: each product rounded before
  // its subtraction, t = 0, 1, ... (the device forms the same values).
  h.lev.clear();
  h.lev.emplace_back();
  {
    AmgLevel& L0 = h.lev[0];
    Csr& A0 = L0.A;
    A0.n = A0.m = nb * ne;
    A0.rp.assign(A0.n + 1, 0);
    for (int32_t i = 0; i < nb; ++i)
      for (int a = 0; a < ne; ++a) A0.rp[(int64_t)i * ne + a + 1] = (int64_t)(rp[i + 1] - rp[i]) * ne;
    for (int32_t r = 0; r < A0.n; ++r) A0.rp[r + 1] += A0.rp[r];
    A0.ci.resize(A0.rp[A0.n]);
    A0.v.resize(A0.rp[A0.n]);
    parallel_for(threads, nb, [&](int64_t lo, int64_t hi, int) {
      for (int64_t i = lo; i < hi; ++i) {
        const double* w = &h.W[(size_t)i * ne * nh];
        for (int a = 0; a < ne; ++a) {
          int64_t p = A0.rp[i * ne + a];
          for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const double* B = &h.av[(size_t)k * 9];
            for (int c = 0; c < ne; ++c) {
              double x = B[h.eidx[a] * 3 + h.eidx[c]];
              for (int t = 0; t < nh; ++t) x -= w[a * nh + t] * B[h.hidx[t] * 3 + h.eidx[c]];
              A0.ci[p] = ci[k] * ne + c;
              A0.v[p] = x;
              ++p;
            }
          }
        }
      }
    });
    L0.func.resize(A0.n);
    for (int32_t r = 0; r < A0.n; ++r) L0.func[r] = r % ne;
  }
  mark(kStepReduce);
  for (;;) {
    const size_t l = h.lev.size() - 1;
    const Csr& A = h.lev[l].A;
    if (A.n <= prm.max_coarse || (int)l + 1 >= prm.max_levels) break;
    std::unique_ptr<LevelSteps> dev = prm.level_steps ? prm.level_steps(A) : nullptr;
    Csr S;
    if (!dev || !dev->strength(h.lev[l].func, prm.theta, prm.max_row_sum, S))
      S = strength_graph(A, h.lev[l].func, prm.theta, prm.max_row_sum, threads);
    mark(kStepStrength);
    const bool agg = (int)l < prm.agg_levels;
    // a first pass (one HMIS block) starts with dev's passes over the small
    // components of the graph, and a split over several blocks runs on dev,
    // when dev holds the graph (which: 0 = S, 1 = the distance-two graph it
    // formed, -1 = neither)
    auto split = [&](const Csr& G, int which) {
      const bool one_block = prm.hmis_block <= 0 || prm.hmis_block >= G.n;
      if (one_block)
        ++h.first_passes;
      else
        ++h.hmis_splits;
      std::vector<int32_t> part;
      if (dev && which >= 0) {
        if (one_block && dev->first_pass_small(G, which == 1, part))
          return first_pass_finish(G, std::move(part), threads);
        if (!one_block && dev->hmis(G, which == 1, prm.hmis_block, part)) return part;
      }
      return hmis_split(G, prm.hmis_block, threads);
    };
    std::vector<int32_t> cf;
    if (agg) {  // aggressive_split, with the distance-two graph formed where dev says
      std::vector<int32_t> cf1 = split(S, 0);
      Csr S2;
      const bool s2_dev = dev && dev->strength2(S, cf1, S2);
      if (!s2_dev) S2 = distance_two_strength(S, cf1, threads);
      const std::vector<int32_t> cf2 = split(S2, s2_dev ? 1 : -1);
      cf.assign(S.n, -1);
      for (int32_t i = 0, c = 0; i < S.n; ++i)
        if (cf1[i] == 1) cf[i] = cf2[c++] == 1 ? 1 : -1;
    } else {
      cf = split(S, 0);
    }
    mark(kStepSplit);
    int32_t nc = 0;
    for (auto x : cf) nc += x == 1;
    if (nc == 0 || nc == A.n) break;
    Csr P;
    if (agg) {
      if (!dev || !dev->multipass(S, cf, h.lev[l].func, P)) P = multipass_interp(A, S, cf, h.lev[l].func, threads);
    } else if (!dev || !dev->interp(S, cf, h.lev[l].func, prm.pmax, P))
      P = extended_i_interp(A, S, cf, h.lev[l].func, prm.pmax, threads);
    Csr R = transpose(P, threads);
    mark(kStepInterp);
    Csr Ac;
    if (!dev || !dev->galerkin(R, P, Ac)) Ac = galerkin(R, A, P, threads);
    mark(kStepGalerkin);
    std::vector<int32_t> fc;
    fc.reserve(nc);
    for (int32_t i = 0; i < A.n; ++i)
      if (cf[i] == 1) fc.push_back(h.lev[l].func[i]);
    h.lev[l].cf = std::move(cf);
    h.lev[l].P = std::move(P);
    h.lev[l].R = std::move(R);
    AmgLevel next;
    next.A = std::move(Ac);
    next.func = std::move(fc);
    h.lev.push_back(std::move(next));
  }
  // a coarsest level above the dense limit (the coarsening stopped early) is
  // smoothed like the others, with no coarse correction
  h.coarse_relax = h.lev.back().A.n > prm.max_dense_coarse;
  for (size_t l = 0; l + 1 < h.lev.size() + (h.coarse_relax ? 1 : 0); ++l) {
    int st = l1_inverse_diag(h.lev[l].A, h.lev[l].dinv, threads, err);
    if (st != CPTR_OK) return st;
  }
  if (!h.coarse_relax) {
    const Csr& Ac = h.lev.back().A;
    h.coarse_lu.assign((size_t)Ac.n * Ac.n, 0.0);
    for (int32_t i = 0; i < Ac.n; ++i)
      for (int64_t k = Ac.rp[i]; k < Ac.rp[i + 1]; ++k) h.coarse_lu[(size_t)i * Ac.n + Ac.ci[k]] += Ac.v[k];
    int st = dense_lu(Ac.n, h.coarse_lu, h.coarse_piv, err);
    if (st != CPTR_OK) return st;
  }
  mark(kStepSmoother);

  // ---- block ILU(0) on A's pattern, matrix ordering (Sec. 3.1) ----
  if (!prm.skip_ilu) {
    h.ilu.assign(h.av, h.av + (size_t)nnzb * 9);
    h.uinv.assign((size_t)nb * 9, 0.0);
    for (int32_t i = 0; i < nb; ++i) {
      const int32_t d = h.diag[i];
      for (int32_t q = rp[i]; q < d; ++q) {
        const int32_t c = ci[q];
        double Lq[9];
        mm3(&h.ilu[(size_t)q * 9], &h.uinv[(size_t)c * 9], Lq);
        std::memcpy(&h.ilu[(size_t)q * 9], Lq, sizeof Lq);
        // merge the U part of row c (columns > c) into row i's later blocks
        int32_t t = q + 1;
        for (int32_t u = h.diag[c] + 1; u < rp[c + 1]; ++u) {
          const int32_t col = ci[u];
          while (t < rp[i + 1] && ci[t] < col) ++t;
          if (t == rp[i + 1]) break;
          if (ci[t] != col) continue;
          double prod[9];
          mm3(Lq, &h.ilu[(size_t)u * 9], prod);
          double* dst = &h.ilu[(size_t)t * 9];
          for (int e = 0; e < 9; ++e) dst[e] -= prod[e];
        }
      }
      if (!inv3(&h.ilu[(size_t)d * 9], &h.uinv[(size_t)i * 9]))
        return err = "zero ILU(0) pivot (singular diagonal block) in block row " + std::to_string(i),
               CPTR_E_ZERO_PIVOT;
    }
  }
  if (!prm.ilu_levels_elsewhere) ilu_dependency_levels(h);
  mark(kStepIlu);
  return CPTR_OK;
}

void ilu_dependency_levels(HostSetup& h) {
  const int32_t nb = h.nb;
  const int32_t* rp = h.rp.data();
  const int32_t* ci = h.ci.data();
  h.fwd_level.assign(nb, 0);
  h.bwd_level.assign(nb, 0);
  int32_t nf = 0, nbk = 0;
  for (int32_t i = 0; i < nb; ++i) {
    int32_t lv = 0;
    for (int32_t k = rp[i]; k < h.diag[i]; ++k) lv = std::max(lv, h.fwd_level[ci[k]] + 1);
    h.fwd_level[i] = lv;
    nf = std::max(nf, lv + 1);
  }
  for (int32_t i = nb - 1; i >= 0; --i) {
    int32_t lv = 0;
    for (int32_t k = h.diag[i] + 1; k < rp[i + 1]; ++k) lv = std::max(lv, h.bwd_level[ci[k]] + 1);
    h.bwd_level[i] = lv;
    nbk = std::max(nbk, lv + 1);
  }
  h.n_fwd_levels = nf;
  h.n_bwd_levels = nbk;
}

}  // namespace cptr
