// setup.cpp -- one-off FP64 host setup of a fit (runs once in cwb_fit_create).
//
//  * equal-grid binning of every numeric feature with ties to the lower
//    design point (Section 3.1.1), written as uint16 index vectors;
//  * B-spline bases at the design points by de Boor's triangular scheme,
//    kept banded (degree+1 nonzeros per design point);
//  * bin counts and Gram matrices G = Z^bT diag(counts) Z^b (binMatMat,
//    Algorithm 1 with unit weights), separately for the training rows and
//    for all rows (HCWB trains on D_train, then on D; Algorithm 3);
//  * difference penalties (Appendix A.2) and, for a requested df, the
//    smoothing parameter from the Demmler-Reinsch orthogonalisation:
//    with G = L L^T and L^-1 D L^-T = U diag(w) U^T, df(lambda) =
//    sum_i 1 / (1 + lambda w_i), solved by a safeguarded Newton iteration;
//  * categorical ridge learners in closed form (Appendix A.3.1);
//  * the inverse penalised Gram matrix (cached factorisation, Section 2.4).
// The dense algebra is alg:: (algebra.h), which the device setup pass runs
// as well; with device binning the Grams, lambdas and inverses of learners
// up to kDeviceSolveMaxD basis functions are left to that pass.
// Compiled with -ffp-contract=off so the binning distances and the algebra
// are not fused.
#include "setup.h"

#include "algebra.h"

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <thread>

namespace cwb {

// lambda with df(lambda) = target (App. A.2): alg::lambda_for_df, the
// routine the device setup pass runs too.
int lambda_for_df(int d, const std::vector<double>& G, const std::vector<double>& D, double target,
                  double* lam_out, std::string* err) {
  std::vector<double> scr((size_t)alg::lambda_scratch(d));
  const int rc = alg::lambda_for_df(alg::Serial(), d, G.data(), D.data(), target, lam_out, scr.data());
  if (rc == -5) *err = "degenerate or not positive definite penalised Gram matrix";
  else if (rc) *err = "df target not reachable for this basis and penalty";
  return rc;
}

namespace {

// ---- binning and bases -----------------------------------------------------

// Design point l of the equal grid on [xmin, xmax] with nb points.
inline double grid_point(double xmin, double xmax, double h, int l, int nb) {
  return (l == nb - 1) ? xmax : xmin + (double)l * h;
}

// Closest design point, ties to the lower one.  An arithmetic estimate of the
// enclosing interval is corrected with exact comparisons against the design
// points, then the two distances decide; the result does not depend on the
// estimate, which may use the reciprocal of h.
inline int bin_of(double x, double xmin, double xmax, double h, int nb, double inv_h) {
  if (x <= xmin) return 0;
  if (x >= xmax) return nb - 1;
  int l = (int)((x - xmin) * inv_h);
  if (l < 0) l = 0;
  if (l > nb - 2) l = nb - 2;
  while (l > 0 && grid_point(xmin, xmax, h, l, nb) > x) --l;
  while (l < nb - 2 && grid_point(xmin, xmax, h, l + 1, nb) <= x) ++l;
  const double dlo = x - grid_point(xmin, xmax, h, l, nb);
  const double dhi = grid_point(xmin, xmax, h, l + 1, nb) - x;
  return (dhi < dlo) ? l + 1 : l;
}

// Nonzero B-spline values at z (de Boor's triangular scheme).  Returns the
// index of the first nonzero basis function; vals gets degree+1 values.
int bspline_band(double z, const std::vector<double>& t, int deg, int d, double* vals) {
  // knot interval mu with t[mu] <= z < t[mu+1], kept inside [deg, d-1]
  const double h = t[deg + 1] - t[deg];
  int mu = deg + (int)std::floor((z - t[deg]) / h);
  if (mu < deg) mu = deg;
  if (mu > d - 1) mu = d - 1;
  while (mu > deg && t[mu] > z) --mu;
  while (mu < d - 1 && t[mu + 1] <= z) ++mu;
  double N[kMaxBand + 1], left[kMaxBand + 1], right[kMaxBand + 1];
  N[0] = 1.0;
  for (int j = 1; j <= deg; ++j) {
    left[j] = z - t[mu + 1 - j];
    right[j] = t[mu + j] - z;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      const double temp = N[r] / (right[r + 1] + left[j - r]);
      N[r] = saved + right[r + 1] * temp;
      saved = left[j - r] * temp;
    }
    N[j] = saved;
  }
  for (int j = 0; j <= deg; ++j) vals[j] = N[j];
  return mu - deg;
}

void set_error(std::string* err, const std::string& msg) {
  if (err->empty()) *err = msg;
}

}  // namespace

int bins_for(int32_t n_bins, int64_t n) {
  if (n_bins > 0) return n_bins;
  // largest b with b^e <= n (e = 2 or 4), in exact integer arithmetic
  const int e = (n_bins == -2) ? 4 : 2;
  auto pow_le = [&](int64_t b) {
    __int128 v = 1;
    for (int i = 0; i < e; ++i) v *= b;
    return v <= (__int128)n;
  };
  int64_t b = (int64_t)std::floor(std::pow((double)n, 1.0 / (double)e));
  while (b > 1 && !pow_le(b)) --b;
  while (pow_le(b + 1)) ++b;
  return (int)std::max<int64_t>(2, std::min<int64_t>(b, 65535));
}

int bin_one_feature(const double* x, int64_t n, int nb, uint16_t* ind, double* z, std::string* err) {
  if (!x || !ind || n < 1) { *err = "null pointer or n < 1"; return CWB_E_INVALID_ARG; }
  if (nb < 2 || nb > 65535) { *err = "n_bins must be 2..65535"; return CWB_E_INVALID_ARG; }
  double xmin = x[0], xmax = x[0];
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(x[i])) { *err = "non-finite x"; return CWB_E_INVALID_ARG; }
    xmin = std::min(xmin, x[i]);
    xmax = std::max(xmax, x[i]);
  }
  if (!(xmax > xmin)) { *err = "constant feature"; return CWB_E_INVALID_ARG; }
  const double h = (xmax - xmin) / (double)(nb - 1);
  for (int64_t i = 0; i < n; ++i) ind[i] = (uint16_t)bin_of(x[i], xmin, xmax, h, nb, 1.0 / h);
  if (z)
    for (int l = 0; l < nb; ++l) z[l] = grid_point(xmin, xmax, h, l, nb);
  return CWB_OK;
}

int validate_problem(const cwb_problem* pr, std::string* err) {
  if (!pr) { *err = "null problem"; return CWB_E_INVALID_ARG; }
  if (pr->n < 2) { *err = "n must be >= 2"; return CWB_E_INVALID_ARG; }
  if (pr->p < 1) { *err = "p must be >= 1"; return CWB_E_INVALID_ARG; }
  if (!pr->x || !pr->y || !pr->specs) { *err = "null x, y or specs"; return CWB_E_INVALID_ARG; }
  if (pr->ldx != 0 && pr->ldx < pr->n) { *err = "ldx must be 0 or at least n"; return CWB_E_INVALID_ARG; }
  if (!(pr->nu > 0.0) || !std::isfinite(pr->nu)) { *err = "nu must be > 0"; return CWB_E_INVALID_ARG; }
  if (pr->M < 1) { *err = "M must be >= 1"; return CWB_E_INVALID_ARG; }
  if (pr->loss != CWB_L2 && pr->loss != CWB_BINOMIAL) { *err = "unknown loss"; return CWB_E_INVALID_ARG; }
  if (pr->variant < CWB_CWB || pr->variant > CWB_HCWB) { *err = "unknown variant"; return CWB_E_INVALID_ARG; }
  if (!(pr->gamma >= 0.0) || !std::isfinite(pr->gamma)) { *err = "gamma must be >= 0"; return CWB_E_INVALID_ARG; }
  if (pr->patience < 0) { *err = "patience must be >= 0"; return CWB_E_INVALID_ARG; }
  if (pr->n > ((int64_t)1 << 40)) { *err = "n too large"; return CWB_E_UNSUPPORTED; }
  for (int64_t i = 0; i < pr->n; ++i) {
    const double v = pr->y[i];
    if (!std::isfinite(v)) { *err = "non-finite y"; return CWB_E_INVALID_ARG; }
    if (pr->loss == CWB_BINOMIAL && v != 0.0 && v != 1.0) { *err = "binomial y must be 0/1"; return CWB_E_INVALID_ARG; }
  }
  if (pr->variant == CWB_HCWB && !pr->val_mask) { *err = "HCWB needs a validation mask"; return CWB_E_INVALID_ARG; }
  if (pr->val_mask) {
    int64_t nv = 0;
    for (int64_t i = 0; i < pr->n; ++i) nv += pr->val_mask[i] ? 1 : 0;
    if (nv == 0 || nv == pr->n) { *err = "empty training or validation split"; return CWB_E_INVALID_ARG; }
  }
  for (int j = 0; j < pr->p; ++j) {
    const cwb_learner_spec& s = pr->specs[j];
    if (s.kind == CWB_RIDGE_CAT || s.kind == CWB_BINARY_CAT) {
      if (s.n_levels < 1 || s.n_levels > kMaxD) { *err = "level count must be 1..64"; return CWB_E_INVALID_ARG; }
      if (s.kind == CWB_BINARY_CAT) continue;  // unpenalised: df and lambda unused
    } else if (s.kind == CWB_PSPLINE) {
      if (s.degree < 1 || s.degree > 3) { *err = "P-spline degree must be 1..3"; return CWB_E_UNSUPPORTED; }
      if (s.n_interior_knots < 0) { *err = "negative knot count"; return CWB_E_INVALID_ARG; }
      const int d = s.n_interior_knots + s.degree + 1;
      if (d > kMaxD) { *err = "basis larger than 64"; return CWB_E_UNSUPPORTED; }
      if (s.penalty_order < 0 || s.penalty_order >= d) { *err = "bad penalty order"; return CWB_E_INVALID_ARG; }
      if (s.n_bins == 0 && s.degree != 3) { *err = "unbinned learners must be cubic"; return CWB_E_UNSUPPORTED; }
      if (s.n_bins != -1 && s.n_bins != -2 && s.n_bins != 0 && (s.n_bins < 2 || s.n_bins > 65535)) {
        *err = "n_bins must be 2..65535 (or 0: unbinned, -1: floor(sqrt(n)), -2: floor(n^(1/4)))";
        return CWB_E_INVALID_ARG;
      }
      if (s.df > 0.0 && (s.df <= (double)s.penalty_order || s.df >= (double)d)) {
        *err = "P-spline df must lie between the penalty order and the basis size";
        return CWB_E_INVALID_ARG;
      }
    } else {
      *err = "unknown learner kind";
      return CWB_E_INVALID_ARG;
    }
    if (s.df <= 0.0 && !(s.lambda >= 0.0)) { *err = "lambda must be >= 0"; return CWB_E_INVALID_ARG; }
  }
  int n_unb = 0;
  for (int j = 0; j < pr->p; ++j)
    n_unb += (pr->specs[j].kind == CWB_PSPLINE && pr->specs[j].n_bins == 0) ? 1 : 0;
  if (n_unb > 0 && n_unb < pr->p) {
    *err = "a fit's learners must be all binned or all unbinned P-splines";
    return CWB_E_UNSUPPORTED;
  }
  return CWB_OK;
}

namespace {

// The four nonzero cubic B-spline values on an interval of equally spaced
// knots, at position t in [0, 1] inside it (the uniform cubic segments).
void uniform_cubic(double t, double* b) {
  const double s = 1.0 - t, t2 = t * t, t3 = t2 * t;
  b[0] = s * s * s / 6.0;
  b[1] = (3.0 * t3 - 6.0 * t2 + 4.0) / 6.0;
  b[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) / 6.0;
  b[3] = t3 / 6.0;
}

}  // namespace

namespace {

// Knots and the banded basis at the design points of a binned P-spline
// learner (Sec. 2.2, Sec. 3.1.1), from its range and design-point count.
void pspline_design(const cwb_learner_spec& s, HostLearner& L) {
  const int deg = s.degree;
  const int nint = s.n_interior_knots;
  const int nk = nint + 2 + 2 * deg;
  const int d = nk - deg - 1;
  L.d = d;
  L.band = deg + 1;
  std::vector<double> t(nk);
  const double hk = (L.xmax - L.xmin) / (double)(nint + 1);
  for (int q = 0; q < nk; ++q) t[q] = L.xmin + (double)(q - deg) * hk;
  const double h = (L.xmax - L.xmin) / (double)(L.nb - 1);
  L.bstart.resize(L.nb);
  L.bval.assign((size_t)L.nb * kMaxBand, 0.0);
  for (int l = 0; l < L.nb; ++l) {
    const double z = grid_point(L.xmin, L.xmax, h, l, L.nb);
    L.bstart[l] = bspline_band(z, t, deg, d, &L.bval[(size_t)l * kMaxBand]);
  }
}

// Identity reduced design of a categorical learner (the levels are the bins).
void categorical_design(HostLearner& L, int c) {
  L.nb = c;
  L.band = 1;
  L.d = c;
  L.bstart.resize(c);
  L.bval.assign((size_t)c * kMaxBand, 0.0);
  for (int l = 0; l < c; ++l) {
    L.bstart[l] = l;
    L.bval[(size_t)l * kMaxBand] = 1.0;
  }
}

// Support ranges, Gram matrices over the training rows and over all rows,
// smoothing parameters and the inverses of G + lambda D (alg::learner_solve,
// the routine the device setup pass runs).  Binned learners take their Grams
// from the bin counts (binMatMat, Algorithm 1); unbinned ones bring them in
// G_unb.  Without `solves` only the support ranges and the count bound are
// set, and the Gram and inverse are zero placeholders of the right size.
int learner_algebra(const cwb_learner_spec& s, int64_t n, HostLearner& L,
                    const std::vector<double>& cnt_t, const std::vector<double>& cnt_a,
                    const std::vector<double>* G_unb, int j, std::string* err, bool solves = true) {
  const int d = L.d;
  // the largest bin count over all rows bounds every histogram sum of the
  // learner (32-bit histogram accumulation)
  L.cnt_max = 0;
  for (double c : cnt_a) L.cnt_max = std::max(L.cnt_max, (int64_t)c);
  // support ranges: design points whose band covers basis index q
  L.jr.assign((size_t)2 * d, 0);
  for (int q = 0; q < d; ++q) {
    int lo = L.nb, hi = -1;
    for (int l = 0; l < L.nb; ++l)
      if (L.bstart[l] <= q && q < L.bstart[l] + L.band) {
        lo = std::min(lo, l);
        hi = std::max(hi, l);
      }
    L.jr[2 * q] = lo;
    L.jr[2 * q + 1] = hi;
  }
  for (int set = 0; set < 2; ++set) {
    const std::vector<double>& cnt = set == 0 ? cnt_t : cnt_a;
    L.gram[set].assign((size_t)d * d, 0.0);
    L.ainv[set].assign((size_t)d * d, 0.0);
    L.lambda[set] = 0.0;
    if (!solves) continue;  // placeholders: the device setup pass fills them in
    std::vector<double> scr((size_t)alg::solve_scratch(d));
    double lam = 0.0;
    int rc;
    if (G_unb) {
      // unbinned: the Gram matrix comes in; lambda and the inverse as for
      // binned learners
      L.gram[set] = G_unb[set];
      double* D = scr.data();
      double* A = D + (size_t)d * d;
      double* rest = A + (size_t)d * d;
      alg::penalty(alg::Serial(), d, s.penalty_order, D, rest);
      lam = s.lambda;
      rc = (s.df > 0.0) ? alg::lambda_for_df(alg::Serial(), d, L.gram[set].data(), D, s.df, &lam, rest) : 0;
      if (!rc) {
        for (size_t i = 0; i < (size_t)d * d; ++i) A[i] = L.gram[set][i] + lam * D[i];
        rc = alg::spd_inverse(alg::Serial(), d, A, L.ainv[set].data(), rest) ? 0 : -5;
      }
    } else {
      rc = alg::learner_solve(alg::Serial(), s.kind, d, L.nb, L.band, L.bstart.data(),
                              L.bval.data(), kMaxBand, cnt.data(), s.penalty_order, s.df, s.lambda, L.gram[set].data(),
                              L.ainv[set].data(), &lam, scr.data());
    }
    if (rc) {
      *err = (rc == -1 ? std::string("df target not reachable for this basis and penalty")
                       : std::string("penalised Gram matrix is singular or degenerate")) +
             " (feature " + std::to_string(j) + ")";
      return rc == -1 ? CWB_E_INVALID_ARG : CWB_E_NUMERIC;
    }
    L.lambda[set] = lam;
  }
  return CWB_OK;
}

// Runs fn(j) for j in [0, p) on up to 32 threads; the first failing feature
// (lowest j) decides the status.
template <class Fn>
int for_features(int p, std::string* err, Fn fn) {
  std::vector<std::string> ferr(p);
  std::vector<int> frc(p, 0);
  std::atomic<int> next(0);
  auto worker = [&]() {
    for (;;) {
      const int j = next.fetch_add(1);
      if (j >= p) break;
      frc[j] = fn(j, &ferr[j]);
    }
  };
  unsigned nth = std::thread::hardware_concurrency();
  if (nth == 0) nth = 4;
  nth = std::min<unsigned>(nth, 32);
  nth = std::min<unsigned>(nth, (unsigned)p);
  std::vector<std::thread> pool;
  for (unsigned i = 1; i < nth; ++i) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  for (int j = 0; j < p; ++j)
    if (frc[j]) {
      set_error(err, ferr[j]);
      return frc[j];
    }
  return CWB_OK;
}

void learner_sizes(HostFit* hf) {
  hf->nb_max = 0;
  hf->d_max = 0;
  hf->sum_d = 0;
  for (int j = 0; j < hf->p; ++j) {
    hf->nb_max = std::max(hf->nb_max, hf->L[j].nb);
    hf->d_max = std::max(hf->d_max, hf->L[j].d);
    hf->sum_d += hf->L[j].d;
  }
}

}  // namespace

int prepare_host_fit(const cwb_problem* pr, HostFit* hf, std::string* err,
                     const std::vector<int64_t>* order) {
  int rc = validate_problem(pr, err);
  if (rc) return rc;
  const int64_t n = pr->n;
  const int p = pr->p;
  hf->n = n;
  hf->p = p;
  hf->n_pad = (n + 63) / 64 * 64;
  hf->loss = pr->loss;
  hf->variant = pr->variant;
  hf->M = pr->M;
  hf->nu = pr->nu;
  hf->gamma = pr->gamma;
  hf->patience = pr->patience;

  // Training rows first, then validation rows (stable), or the given order
  // (every row a training row).
  hf->perm.resize(n);
  int64_t nt = 0;
  if (order) {
    hf->perm = *order;
    nt = n;
  } else {
    for (int64_t i = 0; i < n; ++i)
      if (!pr->val_mask || !pr->val_mask[i]) hf->perm[nt++] = i;
    int64_t pos = nt;
    for (int64_t i = 0; i < n; ++i)
      if (pr->val_mask && pr->val_mask[i]) hf->perm[pos++] = i;
  }
  hf->n_train = nt;

  hf->y.assign(hf->n_pad, 0.0f);
  double ysum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double v = pr->y[hf->perm[i]];
    hf->y[i] = (float)v;
    if (i < nt) ysum += v;
  }
  const double ybar = ysum / (double)nt;
  hf->f0 = (pr->loss == CWB_L2) ? ybar : std::log(ybar / (1.0 - ybar));
  if (!std::isfinite(hf->f0)) {
    *err = "training labels are all equal (binomial intercept not finite)";
    return CWB_E_NUMERIC;
  }
  hf->unbinned = pr->specs[0].kind == CWB_PSPLINE && pr->specs[0].n_bins == 0;
  hf->L.assign(p, HostLearner());
  for (int j = 0; j < p; ++j) {
    const cwb_learner_spec& s = pr->specs[j];
    HostLearner& L = hf->L[j];
    L.kind = s.kind;
    L.degree = s.degree;
    L.n_int = s.n_interior_knots;
    if (s.kind != CWB_PSPLINE) {
      L.nb = L.d = s.n_levels;
      L.band = 1;
    } else if (hf->unbinned) {
      L.nb = L.d = s.n_interior_knots + 4;
      L.band = 1;
    } else {
      L.nb = bins_for(s.n_bins, n);
      L.d = s.n_interior_knots + s.degree + 1;
      L.band = s.degree + 1;
    }
  }
  return CWB_OK;
}

int build_host_fit(const cwb_problem* pr, HostFit* hf, std::string* err,
                   const std::vector<int64_t>* order) {
  int rc = prepare_host_fit(pr, hf, err, order);
  const bool permuted = pr->val_mask != nullptr || order != nullptr;
  if (rc) return rc;
  const int64_t n = pr->n;
  const int p = pr->p;
  const int64_t nt = hf->n_train;
  if (hf->unbinned)
    hf->XU.resize((size_t)p * hf->n_pad);
  else
    hf->X.resize((size_t)p * hf->n_pad);
  rc = for_features(p, err, [&](int j, std::string* ferr) -> int {
    const cwb_learner_spec& s = pr->specs[j];
    const double* xj = pr->x + (size_t)j * (size_t)(pr->ldx ? pr->ldx : n);
    HostLearner& L = hf->L[j];
    uint16_t* Xj = hf->unbinned ? nullptr : hf->X.data() + (size_t)j * hf->n_pad;
    uint32_t* XUj = hf->unbinned ? hf->XU.data() + (size_t)j * hf->n_pad : nullptr;
    for (int64_t i = n; i < hf->n_pad; ++i) {  // padding rows: index 0
      if (Xj) Xj[i] = 0;
      if (XUj) XUj[i] = 0;
    }
    if (s.kind != CWB_PSPLINE) {
      const int c = s.n_levels;
      for (int64_t i = 0; i < n; ++i) {
        const double v = xj[hf->perm[i]];
        if (!(v >= 0.0) || v >= (double)c || v != std::floor(v)) {
          *ferr = "level code out of range in feature " + std::to_string(j);
          return CWB_E_INVALID_ARG;
        }
        Xj[i] = (uint16_t)v;
      }
      categorical_design(L, c);
    } else {
      double xmin = xj[0], xmax = xj[0];
      for (int64_t i = 0; i < n; ++i) {
        const double v = xj[i];
        if (!std::isfinite(v)) { *ferr = "non-finite x"; return CWB_E_INVALID_ARG; }
        xmin = std::min(xmin, v);
        xmax = std::max(xmax, v);
      }
      if (!(xmax > xmin)) {
        *ferr = "constant feature " + std::to_string(j);
        return CWB_E_INVALID_ARG;
      }
      L.xmin = xmin == 0.0 ? 0.0 : xmin;  // one zero for both signs
      L.xmax = xmax == 0.0 ? 0.0 : xmax;
      xmin = L.xmin;
      xmax = L.xmax;
      if (hf->unbinned) {
        // unbinned cubic P-spline: knot-interval codes and an identity
        // reduced design (its "bins" are the basis functions)
        const int nint = s.n_interior_knots;
        const double hk = (xmax - xmin) / (double)(nint + 1);
        for (int64_t i = 0; i < n; ++i) {
          const double u = (xj[hf->perm[i]] - xmin) / hk;
          int iv = (int)std::floor(u);
          iv = std::max(0, std::min(nint, iv));
          const double tt = std::max(0.0, std::min(1.0, u - (double)iv));
          XUj[i] = ((uint32_t)iv << 24) | (uint32_t)std::llround(tt * (double)kUnbFracMax);
        }
        categorical_design(L, nint + 4);
      } else {
        if (L.nb > kMaxBins) {
          *ferr = "more than 8192 bins per learner is not supported";
          return CWB_E_UNSUPPORTED;
        }
        const double h = (xmax - xmin) / (double)(L.nb - 1);
        const double inv_h = 1.0 / h;
        if (permuted) {
          for (int64_t i = 0; i < n; ++i)
            Xj[i] = (uint16_t)bin_of(xj[hf->perm[i]], xmin, xmax, h, L.nb, inv_h);
        } else {  // identity row order
          for (int64_t i = 0; i < n; ++i) Xj[i] = (uint16_t)bin_of(xj[i], xmin, xmax, h, L.nb, inv_h);
        }
        pspline_design(s, L);
      }
    }
    // Gram matrices over the training rows and over all rows: from the bin
    // counts (binMatMat, Algorithm 1), or row by row for unbinned learners
    // (with the basis at the stored interval positions)
    const int d = L.d;
    std::vector<double> cnt_t, cnt_a, G_unb[2];
    if (hf->unbinned) {
      for (int set = 0; set < 2; ++set) G_unb[set].assign((size_t)d * d, 0.0);
      for (int64_t i = 0; i < n; ++i) {
        const uint32_t code = XUj[i];
        const int b0 = (int)(code >> 24);
        double bv[4];
        uniform_cubic((double)(code & kUnbFracMax) / (double)kUnbFracMax, bv);
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) {
            const double v = bv[a] * bv[b];
            G_unb[1][(size_t)(b0 + a) * d + (b0 + b)] += v;
            if (i < nt) G_unb[0][(size_t)(b0 + a) * d + (b0 + b)] += v;
          }
      }
    } else {
      std::vector<int64_t> ct(L.nb, 0), ca(L.nb, 0);
      for (int64_t i = 0; i < nt; ++i) ct[Xj[i]] += 1;
      for (int64_t i = nt; i < n; ++i) ca[Xj[i]] += 1;
      cnt_t.resize(L.nb);
      cnt_a.resize(L.nb);
      for (int l = 0; l < L.nb; ++l) {
        cnt_t[l] = (double)ct[l];
        cnt_a[l] = (double)(ct[l] + ca[l]);
      }
    }
    return learner_algebra(s, n, L, cnt_t, cnt_a, hf->unbinned ? G_unb : nullptr, j, ferr);
  });
  if (rc) return rc;
  learner_sizes(hf);
  return CWB_OK;
}

int finish_host_fit(const cwb_problem* pr, HostFit* hf, const double* xrange,
                    const uint32_t* counts, int64_t counts_stride, std::string* err,
                    bool device_solves) {
  const int p = pr->p;
  const int64_t n = pr->n;
  int rc = for_features(p, err, [&](int j, std::string* ferr) -> int {
    const cwb_learner_spec& s = pr->specs[j];
    HostLearner& L = hf->L[j];
    if (s.kind != CWB_PSPLINE) {
      categorical_design(L, s.n_levels);
    } else {
      L.xmin = xrange[2 * j];
      L.xmax = xrange[2 * j + 1];
      if (L.nb > kMaxBins) {
        *ferr = "more than 8192 bins per learner is not supported";
        return CWB_E_UNSUPPORTED;
      }
      pspline_design(s, L);
    }
    const uint32_t* c = counts + (size_t)j * counts_stride;
    std::vector<double> cnt_t(L.nb), cnt_a(L.nb);
    for (int l = 0; l < L.nb; ++l) {
      cnt_t[l] = (double)c[l];
      cnt_a[l] = (double)c[counts_stride / 2 + l];
    }
    L.solve_on_device = device_solves && L.d <= kDeviceSolveMaxD;
    return learner_algebra(s, n, L, cnt_t, cnt_a, nullptr, j, ferr, !L.solve_on_device);
  });
  if (rc) return rc;
  learner_sizes(hf);
  return CWB_OK;
}

}  // namespace cwb

namespace cwb {

int cv_host_fits(const cwb_problem* pr, int K, const int32_t* fold, HostFit* full,
                 std::vector<HostFit>* folds, std::string* err) {
  cwb_problem all = *pr;
  all.val_mask = nullptr;
  // rows grouped by fold (stable): each fold's held-out rows form one block
  const int64_t n = pr->n;
  std::vector<int64_t> order;
  order.reserve(n);
  for (int k = 0; k < K; ++k)
    for (int64_t i = 0; i < n; ++i)
      if (fold[i] == k) order.push_back(i);
  if ((int64_t)order.size() != n) {
    *err = "fold id out of range";
    return CWB_E_INVALID_ARG;
  }
  int rc = build_host_fit(&all, full, err, &order);
  if (rc) return rc;
  if (full->unbinned) {
    *err = "cross-validation covers binned learners";
    return CWB_E_UNSUPPORTED;
  }
  const int p = pr->p;
  std::vector<int64_t> rows(K, 0);
  std::vector<double> ysum(K, 0.0);
  double ytot = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    rows[fold[i]] += 1;
    ysum[fold[i]] += pr->y[i];
    ytot += pr->y[i];
  }
  folds->assign(K, HostFit());
  for (int k = 0; k < K; ++k) {
    HostFit& h = (*folds)[k];
    h.n = n;
    h.n_pad = full->n_pad;
    h.n_train = n - rows[k];
    h.p = p;
    h.loss = full->loss;
    h.variant = full->variant;
    h.M = full->M;
    h.patience = full->patience;
    h.nu = full->nu;
    h.gamma = full->gamma;
    h.nb_max = full->nb_max;
    h.d_max = full->d_max;
    h.sum_d = full->sum_d;
    h.unbinned = false;
    h.perm = full->perm;  // the fold-grouped row order
    h.y = full->y;
    // loss-optimal constant over the fold's training rows (every other fold)
    const double ybar = (ytot - ysum[k]) / (double)h.n_train;
    h.f0 = (pr->loss == CWB_L2) ? ybar : std::log(ybar / (1.0 - ybar));
    if (!std::isfinite(h.f0)) {
      *err = "training labels of fold " + std::to_string(k) + " are all equal";
      return CWB_E_NUMERIC;
    }
    h.L.assign(p, HostLearner());
  }
  // per feature: bin counts of each fold in one pass, then each fold's
  // training counts (all rows but its own) and its learner tables
  return for_features(p, err, [&](int j, std::string* ferr) -> int {
    const HostLearner& Lf = full->L[j];
    const uint16_t* Xj = full->X.data() + (size_t)j * full->n_pad;
    std::vector<int64_t> c((size_t)K * Lf.nb, 0);
    for (int64_t i = 0; i < n; ++i) c[(size_t)fold[full->perm[i]] * Lf.nb + Xj[i]] += 1;
    std::vector<double> cnt_a(Lf.nb, 0.0), cnt_t(Lf.nb);
    for (int k = 0; k < K; ++k)
      for (int l = 0; l < Lf.nb; ++l) cnt_a[l] += (double)c[(size_t)k * Lf.nb + l];
    for (int k = 0; k < K; ++k) {
      for (int l = 0; l < Lf.nb; ++l) cnt_t[l] = cnt_a[l] - (double)c[(size_t)k * Lf.nb + l];
      HostLearner& L = (*folds)[k].L[j];
      L = Lf;  // the design at the shared design points
      const int r = learner_algebra(pr->specs[j], n, L, cnt_t, cnt_a, nullptr, j, ferr);
      if (r) return r;
    }
    return CWB_OK;
  });
}

}  // namespace cwb
