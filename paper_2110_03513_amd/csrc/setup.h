// setup.h -- host-side FP64 setup of a fit (see setup.cpp).
#pragma once
#include <cstdint>
#include <string>
#include <memory>
#include <utility>
#include <vector>

#include "../../include/cwb.h"
#include "cwb_internal.h"

namespace cwb {

// Allocator that leaves new elements uninitialised (for the large index
// matrices, every element of which setup writes).
template <class T>
struct UninitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = UninitAlloc<U>;
  };
  UninitAlloc() = default;
  template <class U>
  UninitAlloc(const UninitAlloc<U>&) {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};

struct HostLearner {
  int kind = 0;
  int nb = 0;      // design points or levels
  int band = 0;    // nonzeros per reduced-design row
  int d = 0;       // basis size
  double xmin = 0, xmax = 0;
  int degree = 0, n_int = 0;     // P-spline degree and interior knots
  std::vector<int32_t> bstart;   // nb
  std::vector<double> bval;      // nb x kMaxBand
  std::vector<int32_t> jr;       // d x 2
  std::vector<double> ainv[2];   // d x d, [0] training rows, [1] all rows
  std::vector<double> gram[2];
  double lambda[2] = {0, 0};
  int64_t cnt_max = 0;           // binned: the largest bin count over all rows
  bool solve_on_device = false;  // Grams, lambda and inverses left to the device pass
};

// Learners up to this basis size can take their solves (Gram, lambda,
// inverse) in the device setup pass (12 d^2 + d doubles of LDS each).
constexpr int kDeviceSolveMaxD = 32;

struct HostFit {
  int64_t n = 0, n_pad = 0, n_train = 0;
  int p = 0;
  int loss = 0, variant = 0, M = 0, patience = 0;
  double nu = 0, gamma = 0, f0 = 0;
  int nb_max = 0, d_max = 0, sum_d = 0;
  std::vector<int64_t> perm;     // internal row -> original row
  std::vector<uint16_t, UninitAlloc<uint16_t>> X;  // p x n_pad, feature-major (binned learners)
  bool unbinned = false;         // every learner is an unbinned cubic P-spline
  std::vector<uint32_t, UninitAlloc<uint32_t>> XU;  // p x n_pad knot-interval codes (unbinned)
  std::vector<float> y;          // n_pad
  std::vector<HostLearner> L;
};

// Design points of a P-spline learner for the n_bins setting of its spec:
// the value itself when positive, floor(sqrt(n)) for -1, floor(n^(1/4)) for
// -2 (at least 2).
int bins_for(int32_t n_bins, int64_t n);
int bin_one_feature(const double* x, int64_t n, int nb, uint16_t* ind, double* z, std::string* err);
int validate_problem(const cwb_problem* pr, std::string* err);
// The smoothing parameter lambda with df(lambda) = target for a learner's
// Gram matrix G and penalty D (d x d, row-major): 0, -1 (target out of
// reach) or -5 (degenerate or not positive definite), with a message.
int lambda_for_df(int d, const std::vector<double>& G, const std::vector<double>& D, double target,
                  double* lam_out, std::string* err);
// Host setup of a fit in full: validation, row order, labels, binning, bin
// counts and every learner's tables.
int build_host_fit(const cwb_problem* pr, HostFit* hf, std::string* err,
                   const std::vector<int64_t>* order = nullptr);
// Its first phase only (nothing that reads x): validation, row order,
// labels, intercept and each learner's kind and sizes.
int prepare_host_fit(const cwb_problem* pr, HostFit* hf, std::string* err,
                     const std::vector<int64_t>* order = nullptr);
// Its last phase after a device binning pass: every learner's tables from
// the feature ranges (xrange[2j], xrange[2j+1]) and bin counts (feature j's
// training-row counts at counts[j * counts_stride], all-row counts
// counts_stride / 2 further).  With `device_solves`, learners of basis size
// up to kDeviceSolveMaxD get zero placeholders for their Grams and inverses
// (solve_on_device), which the device solve pass computes.
int finish_host_fit(const cwb_problem* pr, HostFit* hf, const double* xrange,
                    const uint32_t* counts, int64_t counts_stride, std::string* err,
                    bool device_solves = false);
// Host setup of the K folds of a cross-validation (fold[i] in [0, K) for
// every row): `full` bins all rows once, in their own order, and keeps the
// index matrix that the folds share, with the rows grouped by fold (fold 0's
// rows first, each group in the original order: full->perm); each fold's
// HostFit has that row order, and its intercept and learner tables from the
// training rows of every other fold.
int cv_host_fits(const cwb_problem* pr, int K, const int32_t* fold, HostFit* full,
                 std::vector<HostFit>* folds, std::string* err);

}  // namespace cwb
