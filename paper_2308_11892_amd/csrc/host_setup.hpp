// host_setup.hpp -- host-side construction of the CPTR preconditioner.
//
// Everything here runs once per matrix inside cptr_setup, before any device
// work: validation of the block-sparse input, the quasi-IMPES reduction of the
// elliptic block (Sec. 5.2 of the paper), the system-AMG hierarchy on it
// (Sec. 3.1 and 3.2) and the block ILU(0) factors of the whole matrix
// (Sec. 3.1), plus the dependency levels the triangular sweeps run in.
// The device layouts are produced from these host structures by the API layer.
#pragma once
#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

namespace cptr {

constexpr int kBS = 3;   // unknowns per cell supported by the kernels

// std::vector whose resize() leaves new elements of trivial types
// uninitialised (assign() and value-taking constructors still fill), so that a
// large array is first written by the threads that fill it instead of being
// zeroed by one thread beforehand.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <class T>
using HVec = std::vector<T, NoInitAlloc<T>>;

struct Csr {
  int32_t n = 0, m = 0;
  std::vector<int64_t> rp;
  HVec<int32_t> ci;
  HVec<double> v;  // empty for a pattern-only matrix (strength graphs)
  int64_t nnz() const { return rp.empty() ? 0 : rp[n]; }
};

struct AmgLevel {
  Csr A;                       // scalar operator of this level
  Csr P, R;                    // interpolation to this level from the next, R = P^T
  std::vector<int32_t> cf;     // 1 = C, -1 = F (empty on the coarsest level)
  std::vector<int32_t> func;   // unknown type (0 = first elliptic unknown, ...)
  std::vector<double> dinv;    // inverse l1-Jacobi diagonal (empty on the coarsest)
};

// Steps of one level's construction done elsewhere (on the device) with the
// results this file's functions give, bit for bit; a step that returns false
// did not produce its result, which is then formed here.
struct LevelSteps {
  virtual ~LevelSteps() = default;
  virtual bool strength(const std::vector<int32_t>& func, double theta, double mrs, Csr& S) = 0;
  virtual bool interp(const Csr& S, const std::vector<int32_t>& cf, const std::vector<int32_t>& func, int pmax,
                      Csr& P) = 0;
  virtual bool galerkin(const Csr& R, const Csr& P, Csr& C) = 0;
  // the first pass over the small weakly connected components of the level's
  // strength graph S (second: of the distance-two graph strength2 formed):
  // cf = 1 / -1 for their points and for points without links, 0 for the rest
  virtual bool first_pass_small(const Csr& G, bool second, std::vector<int32_t>& cf) {
    (void)G, (void)second, (void)cf;
    return false;
  }
  // the HMIS split over blocks of `block` points of G (as first_pass_small's
  // G and second), the whole split
  virtual bool hmis(const Csr& G, bool second, int32_t block, std::vector<int32_t>& cf) {
    (void)G, (void)second, (void)block, (void)cf;
    return false;
  }
  // distance-two strength among the C points of cf (aggressive level)
  virtual bool strength2(const Csr& S, const std::vector<int32_t>& cf, Csr& S2) {
    (void)S, (void)cf, (void)S2;
    return false;
  }
  // multipass interpolation of an aggressive level
  virtual bool multipass(const Csr& S, const std::vector<int32_t>& cf, const std::vector<int32_t>& func,
                         Csr& P) {
    (void)S, (void)cf, (void)func, (void)P;
    return false;
  }
};

struct HostSetup;

struct SetupParams {
  double theta = 0.25;
  double max_row_sum = 0.9;
  int max_levels = 25;
  int max_coarse = 9;
  int pmax = 4;
  int agg_levels = 1;           // levels coarsened aggressively (multipass interpolation)
  bool quasi_impes = true;
  int threads = 1;
  int max_dense_coarse = 4096;  // largest coarsest level solved by dense LU (a larger one is smoothed)
  int32_t hmis_block = 0;       // points per HMIS block, 0 = one block per level
  bool skip_ilu = false;        // ILU(0) is factored elsewhere (on the device)
  // the steps of the level with operator A done elsewhere (null: all here):
  // strength, extended+i or multipass interpolation and the Galerkin product
  std::function<std::unique_ptr<LevelSteps>(const Csr& A)> level_steps;
  // called once the quasi-IMPES weights are formed, before the AMG levels:
  // from then on A's arrays, diag and W do not change (null: nothing)
  std::function<void(HostSetup& h)> after_weights;
  // the sweeps' dependency levels (ilu_dependency_levels) are computed by
  // whoever after_weights started, not at the end of the setup
  bool ilu_levels_elsewhere = false;
};

struct HostSetup {
  int32_t nb = 0;              // block rows (cells)
  int ne = 0, nh = 0;          // elliptic / hyperbolic unknowns per cell
  int eidx[kBS] = {0}, hidx[kBS] = {0};
  std::vector<int32_t> rp, ci; // validated copy of A's pattern
  const double* av = nullptr;  // A values [nnzb][3][3]: the caller's array (or av_owned),
                               // valid while the setup runs, cleared afterwards
  std::vector<double> av_owned;  // A values when the caller's array does not outlive the setup
  std::vector<int32_t> diag;   // position of the diagonal block of each row
  std::vector<double> W;       // [nb][ne][nh]
  std::vector<AmgLevel> lev;   // lev.back() is the coarsest level
  bool coarse_relax = false;      // coarsest level above the dense limit: smoothed, no LU
  std::vector<double> coarse_lu;  // dense LU of the coarsest matrix, row-major
  std::vector<int32_t> coarse_piv;
  std::vector<double> ilu;     // [nnzb][3][3]: L blocks left of the diagonal, U on/right
  std::vector<double> uinv;    // [nb][3][3] inverse of each U_ii (both empty with skip_ilu)
  std::vector<int32_t> fwd_level, bwd_level;  // dependency level of each row
  int32_t n_fwd_levels = 0, n_bwd_levels = 0;
  int first_passes = 0;         // one-block splits run (first passes over a whole graph)
  int hmis_splits = 0;          // splits over several HMIS blocks
  // wall seconds of the setup steps (kSetupStep*), summed over levels
  double step_s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};
enum SetupStep {
  kStepValidate = 0,   // validation, diagonal search
  kStepReduce = 1,     // quasi-IMPES weights and the level-0 operator
  kStepStrength = 2,   // strength graphs
  kStepSplit = 3,      // C/F splits (first passes, aggressive second pass)
  kStepInterp = 4,     // interpolation and its transpose
  kStepGalerkin = 5,   // R A P
  kStepSmoother = 6,   // l1 diagonals, coarsest dense LU
  kStepIlu = 7         // host ILU(0) (host-only handles) and the sweeps' dependency levels
};

// Returns a cptr_status value; on failure `err` holds the message.
int validate_bsr(int32_t nb, int64_t nnzb, const int32_t* rp, const int32_t* ci,
                 const double* v, std::string& err);
int build_host_setup(int32_t nb, const int32_t* rp, const int32_t* ci, const double* v,
                     const int32_t* elliptic, int ne, const SetupParams& prm, HostSetup& out,
                     std::string& err);
// The dependency levels of the sweeps' rows (h.fwd_level, h.bwd_level and
// their counts) from A's pattern and diagonals.
void ilu_dependency_levels(HostSetup& h);

// Building blocks, exported for the library's own host tests.
Csr strength_graph(const Csr& A, const std::vector<int32_t>& func, double theta, double mrs,
                   int threads);
std::vector<int32_t> first_pass_split(const Csr& S, int threads = 1);
// the first pass over the points with cf 0, the others being final
std::vector<int32_t> first_pass_finish(const Csr& S, std::vector<int32_t> cf, int threads);
Csr extended_i_interp(const Csr& A, const Csr& S, const std::vector<int32_t>& cf,
                      const std::vector<int32_t>& func, int pmax, int threads);
Csr distance_two_strength(const Csr& S, const std::vector<int32_t>& cf, int threads);
std::vector<int32_t> aggressive_split(const Csr& S, int32_t block, int threads);
// HMIS split over blocks of `block` consecutive points (<= 0: one block)
std::vector<int32_t> hmis_split(const Csr& S, int32_t block, int threads);
Csr multipass_interp(const Csr& A, const Csr& S, const std::vector<int32_t>& cf,
                     const std::vector<int32_t>& func, int threads);

void parallel_for(int threads, int64_t n, const std::function<void(int64_t, int64_t, int)>& body);

}  // namespace cptr
