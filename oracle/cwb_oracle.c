/*
 * cwb_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of componentwise gradient boosting
 * (CWB), accelerated CWB (ACWB) and hybrid CWB (HCWB) on binned and unbinned
 * features, written from "Accelerated Componentwise Gradient Boosting using
 * Efficient Data Representation and Momentum-based Optimization" (Schalk,
 * Bischl, Ruegamer, arXiv 2110.03513).  It exists to check the HIP library;
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header or table with the library.
 *
 * Every floating-point quantity is IEEE double.  Build with
 * -ffp-contract=off so that the binning distances are not fused.
 * OpenMP (optional) parallelises over base learners only; each learner is
 * handled entirely by one thread, so results do not depend on the thread
 * count.
 *
 * Readings of points the paper leaves open (each is repeated where used):
 *  - L2 loss is 1/2 (y-f)^2, so the pseudo-residual is y - f.
 *  - Binomial loss uses y in {0,1}, f = log-odds: L = log(1+e^f) - y f.
 *  - Binning ties go to the lower design point.
 *  - Cubic P-spline knots are equally spaced on [min, max] with the boundary
 *    extended by `degree` knots on each side.
 *  - df means trace of the hat matrix (df_1).
 *  - SSE in the selection step is the unpenalised residual sum of squares at
 *    the penalised estimate.
 *  - argmin ties go to the lowest learner index.
 *  - aggregated coefficients include the learning rate.
 *  - the ACWB correction residual uses the previous iteration's correction
 *    fit; ACWB follows the algorithm box (g from f and h of the previous
 *    iteration); the step size called beta in the prose is nu.
 *  - HCWB keeps a separate patience counter compared against pat_0; the
 *    switch to CWB on all rows is permanent.
 *  - A categorical feature in the binary representation (Appendix A.3.2)
 *    stands for one unpenalised learner per class, ordered by class inside
 *    the feature; a class with no fitted rows has no least-squares estimate
 *    and is never selected.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_NUMERIC -5

enum { ORC_L2 = 0, ORC_BINOMIAL = 1 };
enum { ORC_CWB = 0, ORC_ACWB = 1, ORC_HCWB = 2 };
enum { ORC_PSPLINE = 0, ORC_RIDGE = 1, ORC_BINARY = 2 };

static char g_err[256];
const char* orc_last_error(void) { return g_err; }
static int fail(int code, const char* msg) {
#pragma omp critical(orc_err)
  {
    strncpy(g_err, msg, sizeof(g_err) - 1);
    g_err[sizeof(g_err) - 1] = 0;
  }
  return code;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra (row-major d x d).                             */
/* ------------------------------------------------------------------------ */

/* Cholesky A = L L^T, L lower triangular.  Returns 0, or -1 if A is not
 * positive definite. */
static int cholesky(int d, const double* A, double* L) {
  memset(L, 0, sizeof(double) * (size_t)d * d);
  for (int j = 0; j < d; ++j) {
    double s = A[j * d + j];
    for (int k = 0; k < j; ++k) s -= L[j * d + k] * L[j * d + k];
    if (!(s > 0.0)) return -1;
    double ljj = sqrt(s);
    L[j * d + j] = ljj;
    for (int i = j + 1; i < d; ++i) {
      double t = A[i * d + j];
      for (int k = 0; k < j; ++k) t -= L[i * d + k] * L[j * d + k];
      L[i * d + j] = t / ljj;
    }
  }
  return 0;
}

/* Solve L L^T x = b. */
static void chol_solve(int d, const double* L, const double* b, double* x) {
  double y[64];
  for (int i = 0; i < d; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= L[i * d + k] * y[k];
    y[i] = t / L[i * d + i];
  }
  for (int i = d - 1; i >= 0; --i) {
    double t = y[i];
    for (int k = i + 1; k < d; ++k) t -= L[k * d + i] * x[k];
    x[i] = t / L[i * d + i];
  }
}

/* ------------------------------------------------------------------------ */
/* Binning (Section 3.1.1, "Discretizing numerical features").              */
/* ------------------------------------------------------------------------ */

/* Equally spaced design points z_l = min + l (max-min)/(nb-1), l = 0..nb-1,
 * with the last point set to max exactly. */
void orc_grid(double xmin, double xmax, int nb, double* z) {
  double h = (xmax - xmin) / (double)(nb - 1);
  for (int l = 0; l < nb; ++l) z[l] = xmin + (double)l * h;
  z[nb - 1] = xmax;
}

/* Index of the closest design point; a value exactly half-way between two
 * points belongs to the lower one (the interval of point l is closed on
 * the right at the midpoint to point l+1). */
int orc_nearest(double x, const double* z, int nb) {
  if (x <= z[0]) return 0;
  if (x >= z[nb - 1]) return nb - 1;
  int lo = 0, hi = nb - 1; /* invariant: z[lo] <= x < z[hi] */
  while (hi - lo > 1) {
    int mid = lo + (hi - lo) / 2;
    if (z[mid] <= x) lo = mid; else hi = mid;
  }
  double dlo = x - z[lo];
  double dhi = z[hi] - x;
  return (dhi < dlo) ? hi : lo;
}

/* Bin a whole feature: design points and index vector. */
void orc_bin_feature(const double* x, int64_t n, int nb, double* z_out,
                     int32_t* ind_out) {
  double xmin = x[0], xmax = x[0];
  for (int64_t i = 1; i < n; ++i) {
    if (x[i] < xmin) xmin = x[i];
    if (x[i] > xmax) xmax = x[i];
  }
  orc_grid(xmin, xmax, nb, z_out);
  for (int64_t i = 0; i < n; ++i) ind_out[i] = orc_nearest(x[i], z_out, nb);
}

/* ------------------------------------------------------------------------ */
/* B-spline basis (Section 2.2, P-splines) by the Cox-de Boor recursion.     */
/* ------------------------------------------------------------------------ */

/* Knots: n_int interior knots equally spaced inside (xmin, xmax), the two
 * boundary knots, and `degree` further equally spaced knots beyond each
 * boundary.  Total n_int + 2 + 2*degree knots, n_int + degree + 1 bases. */
int orc_knots(double xmin, double xmax, int n_int, int degree, double* t) {
  int nk = n_int + 2 + 2 * degree;
  double h = (xmax - xmin) / (double)(n_int + 1);
  for (int j = 0; j < nk; ++j) t[j] = xmin + (double)(j - degree) * h;
  return nk;
}

/* All B-spline basis functions of the given degree at x. */
void orc_bspline(double x, const double* t, int nk, int degree, double* out) {
  double B[128];
  int m = nk - 1;
  for (int j = 0; j < m; ++j) B[j] = (t[j] <= x && x < t[j + 1]) ? 1.0 : 0.0;
  for (int q = 1; q <= degree; ++q) {
    for (int j = 0; j < m - q; ++j) {
      double a = 0.0, b = 0.0;
      if (t[j + q] != t[j]) a = (x - t[j]) / (t[j + q] - t[j]) * B[j];
      if (t[j + q + 1] != t[j + 1])
        b = (t[j + q + 1] - x) / (t[j + q + 1] - t[j + 1]) * B[j + 1];
      B[j] = a + b;
    }
  }
  int d = nk - degree - 1;
  for (int j = 0; j < d; ++j) out[j] = B[j];
}

/* Difference penalty D = Delta^T Delta, Delta the (d-ord) x d matrix of
 * ord-th order differences (Appendix A.2); ord = 0 gives the ridge identity. */
void orc_penalty(int d, int ord, double* D) {
  memset(D, 0, sizeof(double) * (size_t)d * d);
  if (ord == 0) {
    for (int i = 0; i < d; ++i) D[i * d + i] = 1.0;
    return;
  }
  /* Build Delta row by row: the ord-th difference of the unit vectors. */
  int rows = d - ord;
  double* Dl = (double*)calloc((size_t)rows * d, sizeof(double));
  for (int r = 0; r < rows; ++r) {
    double c[16] = {0};
    c[0] = 1.0; /* coefficients of (E - 1)^ord, E the shift */
    for (int o = 0; o < ord; ++o) {
      for (int k = o + 1; k >= 1; --k) c[k] = c[k - 1] - c[k];
      c[0] = -c[0];
    }
    /* c[k] is the coefficient on element r + k (sign convention (-1)^(ord-k) binom) */
    for (int k = 0; k <= ord; ++k) Dl[r * d + r + k] = c[k];
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = 0.0;
      for (int r = 0; r < rows; ++r) s += Dl[r * d + i] * Dl[r * d + j];
      D[i * d + j] = s;
    }
  free(Dl);
}

/* ------------------------------------------------------------------------ */
/* Degrees of freedom and the smoothing parameter (Appendix A.2).            */
/* ------------------------------------------------------------------------ */

/* df_1(lambda) = trace((G + lambda D)^-1 G), computed from its definition. */
int orc_df(int d, const double* G, const double* D, double lambda, double* df) {
  double* A = (double*)malloc(sizeof(double) * d * d);
  double* L = (double*)malloc(sizeof(double) * d * d);
  for (int i = 0; i < d * d; ++i) A[i] = G[i] + lambda * D[i];
  int rc = cholesky(d, A, L);
  if (rc == 0) {
    double col[64], sol[64], tr = 0.0;
    for (int j = 0; j < d; ++j) {
      for (int i = 0; i < d; ++i) col[i] = G[i * d + j];
      chol_solve(d, L, col, sol);
      tr += sol[j];
    }
    *df = tr;
  }
  free(A);
  free(L);
  return rc == 0 ? ORC_OK : ORC_E_NUMERIC;
}

/* lambda >= 0 with df_1(lambda) = target, by bisection in log(lambda).
 * df_1 decreases monotonically in lambda. */
int orc_lambda_for_df(int d, const double* G, const double* D, double target,
                      double* lambda_out) {
  double trG = 0.0, trD = 0.0;
  for (int i = 0; i < d; ++i) { trG += G[i * d + i]; trD += D[i * d + i]; }
  if (!(trG > 0.0) || !(trD > 0.0)) return fail(ORC_E_NUMERIC, "degenerate Gram or penalty");
  double s = trG / trD;
  double lo = 1e-10 * s, hi = 1e10 * s, v;
  int k;
  for (k = 0; k < 40; ++k) {
    if (orc_df(d, G, D, lo, &v) != ORC_OK) return fail(ORC_E_NUMERIC, "df: not positive definite");
    if (v > target) break;
    lo *= 1e-3;
  }
  if (k == 40) return fail(ORC_E_ARG, "df target not reachable (too large)");
  for (k = 0; k < 40; ++k) {
    if (orc_df(d, G, D, hi, &v) != ORC_OK) return fail(ORC_E_NUMERIC, "df: not positive definite");
    if (v < target) break;
    hi *= 1e3;
  }
  if (k == 40) return fail(ORC_E_ARG, "df target not reachable (too small)");
  for (k = 0; k < 400 && hi / lo > 1.0 + 1e-15; ++k) {
    double mid = sqrt(lo * hi);
    orc_df(d, G, D, mid, &v);
    if (v > target) lo = mid; else hi = mid;
  }
  *lambda_out = sqrt(lo * hi);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Losses (Section 2.1 and 2.3).                                              */
/* ------------------------------------------------------------------------ */

static double loss_value(int loss, double y, double f) {
  if (loss == ORC_L2) return 0.5 * (y - f) * (y - f);
  /* log(1 + e^f) - y f, evaluated without overflow */
  double sp = (f > 0.0) ? f + log1p(exp(-f)) : log1p(exp(f));
  return sp - y * f;
}

/* Pseudo-residual: minus the derivative of the loss in f. */
static double pseudo_residual(int loss, double y, double f) {
  if (loss == ORC_L2) return y - f;
  double p = 1.0 / (1.0 + exp(-f));
  return y - p;
}

double orc_loss(int loss, double y, double f) { return loss_value(loss, y, f); }
double orc_pseudo_residual(int loss, double y, double f) { return pseudo_residual(loss, y, f); }

/* Loss-optimal constant argmin_c R_emp(c) over the training rows (val[i] == 0,
 * or all rows if val is NULL): the mean for L2, the log-odds of the mean for
 * the binomial loss. */
static double loss_optimal_constant(int loss, const double* y, int64_t n, const uint8_t* val) {
  double s = 0.0;
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i)
    if (!val || !val[i]) { s += y[i]; ++c; }
  double ybar = s / (double)c;
  if (loss == ORC_L2) return ybar;
  return log(ybar / (1.0 - ybar));
}

/* Empirical risk (mean loss) over the training rows (want = 0) or the
 * validation rows (want = 1); without a mask every row is a training row. */
static double empirical_risk(int loss, const double* y, const double* f, int64_t n,
                             const uint8_t* val, int want) {
  double s = 0.0;
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i) {
    int is_val = val ? (val[i] != 0) : 0;
    if (is_val == want) { s += loss_value(loss, y[i], f[i]); ++c; }
  }
  return c ? s / (double)c : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Problem and result.                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;
  int32_t p;
  const double* x;          /* column-major n x p: x[j*n + i] */
  const double* y;          /* n */
  const uint8_t* val_mask;  /* NULL, or n bytes: 1 = validation row */
  int32_t loss;
  const int32_t* kind;      /* p: 0 P-spline, 1 ridge categorical, 2 binary categorical */
  const int32_t* n_bins;    /* p: P-spline bins (>= 2) or 0 = unbinned */
  const int32_t* n_levels;  /* p: ridge levels */
  const double* df;         /* p: target df (> 0) or <= 0 to use lambda */
  const double* lambda;     /* p */
  int32_t degree, n_knots, pen_order;
  double nu, gamma;
  int32_t M, variant, patience;
  const int32_t* force_k;     /* NULL or M entries */
  const int32_t* force_kcor;  /* NULL or M entries */
  int32_t force_switch;       /* < 0: decide; else first CWB iteration */
} orc_problem;

typedef struct {
  int32_t* d;             /* p: basis size per learner */
  double* lambda_train;   /* p: lambda for the training-row Gram */
  double* lambda_all;     /* p: lambda for the all-row Gram (HCWB) */
  double* f0;             /* 1 */
  int32_t* k;             /* M */
  double* theta;          /* M x d_max */
  double* sse;            /* M: SSE of the selected learner */
  int32_t* own_k;         /* M: own argmin (differs from k only when forced) */
  double* gap;            /* M: SSE(selected or runner-up) - SSE(best) */
  int32_t* kcor;          /* M (ACWB/HCWB; -1 in CWB iterations) */
  double* thetacor;       /* M x d_max */
  int32_t* own_kcor;      /* M */
  double* gapcor;         /* M */
  double* risk_train;     /* M+1: risk of f^[m] over training rows */
  double* risk_val;       /* M+1: risk of f^[m] over validation rows */
  int32_t* switch_iter;   /* 1: first CWB iteration of HCWB, or -1 */
  int32_t* own_switch;    /* 1: the oracle's own switch decision (forced runs) */
  double* f;              /* n: f^[M] on all rows */
  double* coef_f;         /* sum d: aggregated primary-model coefficients */
  double* coef_h;         /* sum d: aggregated momentum-model coefficients */
  double* rtr;            /* M: r^T r of the signal fitted by the primary learner */
  double* rtr_cor;        /* M: c^T c of the corrected signal (ACWB steps) */
  double* sse_cor;        /* M: SSE of the selected correction learner (ACWB steps) */
  double* seconds;        /* 2 or NULL: wall time of setup and of the M iterations */
} orc_result;

typedef struct {
  int kind, d, nb;     /* nb: bins or levels; 0 = unbinned P-spline */
  int32_t* ind;        /* n (binned or categorical) */
  double* Z;           /* binned: nb x d; unbinned: n x d */
  double* D;           /* d x d */
  double* G[2];        /* Gram: [0] training rows, [1] all rows */
  double* L[2];        /* Cholesky factor of G + lambda D */
  double lambda[2];
  int64_t off;         /* offset in the concatenated coefficient vector */
} feat_t;

static void free_feats(feat_t* F, int p) {
  if (!F) return;
  for (int j = 0; j < p; ++j) {
    free(F[j].ind); free(F[j].Z); free(F[j].D);
    for (int s = 0; s < 2; ++s) { free(F[j].G[s]); free(F[j].L[s]); }
  }
  free(F);
}

/* Gram matrix of one learner over the rows with (mask[i] != 0) == want, or
 * over all rows when all != 0.  Binned learners use binMatMat (Algorithm 1,
 * left): U(:, l) accumulates the basis row of every observation in bin l
 * (weights 1), and G = U Z^b.  Unbinned learners use Z^T Z directly. */
static void gram(const feat_t* F, int64_t n, const uint8_t* mask, int all, double* G) {
  int d = F->d;
  memset(G, 0, sizeof(double) * d * d);
  if (F->nb > 0) {
    double* U = (double*)calloc((size_t)d * F->nb, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
      if (!all && mask && mask[i]) continue;
      int l = F->ind[i];
      const double* zr = F->Z + (size_t)l * d;
      for (int a = 0; a < d; ++a) U[(size_t)a * F->nb + l] += zr[a];
    }
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double s = 0.0;
        for (int l = 0; l < F->nb; ++l) s += U[(size_t)a * F->nb + l] * F->Z[(size_t)l * d + b];
        G[a * d + b] = s;
      }
    free(U);
  } else {
    for (int64_t i = 0; i < n; ++i) {
      if (!all && mask && mask[i]) continue;
      const double* zr = F->Z + (size_t)i * d;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) G[a * d + b] += zr[a] * zr[b];
    }
  }
}

/* Smoothing parameter and Cholesky factor for one Gram set. */
static int prepare_set(feat_t* F, int s, double df_target, double lambda_fixed) {
  int d = F->d;
  if (F->kind == ORC_BINARY) {  /* unpenalised one-column learners: nothing to factor */
    F->lambda[s] = 0.0;
    return ORC_OK;
  }
  double lam = lambda_fixed;
  if (df_target > 0.0) {
    if (F->kind == ORC_RIDGE && df_target >= (double)d) {
      lam = 0.0; /* the dummy basis already has df = number of levels */
    } else {
      int rc = orc_lambda_for_df(d, F->G[s], F->D, df_target, &lam);
      if (rc) return rc;
    }
  }
  F->lambda[s] = lam;
  double* A = (double*)malloc(sizeof(double) * d * d);
  for (int i = 0; i < d * d; ++i) A[i] = F->G[s][i] + lam * F->D[i];
  F->L[s] = (double*)malloc(sizeof(double) * d * d);
  int rc = cholesky(d, A, F->L[s]);
  free(A);
  if (rc) return fail(ORC_E_NUMERIC, "penalised Gram matrix is not positive definite");
  return ORC_OK;
}

/* Sizes needed to allocate a result: max and total basis size. */
int orc_sizes(const orc_problem* pr, int32_t* d_max, int32_t* sum_d) {
  int dm = 0, sd = 0;
  for (int j = 0; j < pr->p; ++j) {
    int d = (pr->kind[j] != ORC_PSPLINE) ? pr->n_levels[j] : pr->n_knots + pr->degree + 1;
    if (d > dm) dm = d;
    sd += d;
  }
  *d_max = dm;
  *sum_d = sd;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* findBestBaselearner (Algorithm A1, inner loop; Algorithm 1, binMatVec).   */
/* ------------------------------------------------------------------------ */

typedef struct {
  int k;          /* selected learner */
  int own;        /* own argmin */
  double rtr;     /* r^T r over the rows fitted */
  double sse;     /* SSE of the selected learner */
  double gap;     /* SSE(selected) - SSE(best) if forced, else SSE(2nd) - SSE(best) */
  double theta[64];
} pick_t;

/* Fit every learner to the signal r over the rows (mask[i] == 0, or all rows
 * if all != 0) with Gram set s, and select the learner of least SSE.  If
 * forced >= 0 that learner is taken instead, and the gap to the best is kept. */
static void find_best(const feat_t* F, int p, int64_t n, const double* r,
                      const uint8_t* mask, int all, int s, int forced, double* sse_all,
                      double* theta_all, int d_max, pick_t* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < p; ++k) {
    const feat_t* Fk = &F[k];
    int d = Fk->d;
    double v[64], th[64];
    memset(v, 0, sizeof(v));
    if (Fk->kind == ORC_BINARY) {
      /* Binary representation (Appendix A.3.2): class l alone is a learner
       * with the indicator column of that class; its least-squares estimate
       * is the mean of r over the class's fitted rows, and its SSE is taken
       * over all fitted rows.  The best class stands for the feature. */
      double best_sse = INFINITY, best_th = 0.0;
      int best_l = -1;
      for (int l = 0; l < d; ++l) {
        double sum = 0.0;
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) {
          if (!all && mask && mask[i]) continue;
          if (Fk->ind[i] == l) { sum += r[i]; ++cnt; }
        }
        if (cnt == 0) continue;
        double t = sum / (double)cnt;
        double e2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
          if (!all && mask && mask[i]) continue;
          double e = r[i] - ((Fk->ind[i] == l) ? t : 0.0);
          e2 += e * e;
        }
        if (e2 < best_sse) { best_sse = e2; best_th = t; best_l = l; }
      }
      sse_all[k] = best_sse;
      for (int a = 0; a < d_max; ++a)
        theta_all[(size_t)k * d_max + a] = (a == best_l) ? best_th : 0.0;
      continue;
    }
    if (Fk->nb > 0) {
      /* binMatVec: u(l) = sum of r over bin l, then v = Z^b^T u. */
      double* u = (double*)calloc((size_t)Fk->nb, sizeof(double));
      for (int64_t i = 0; i < n; ++i) {
        if (!all && mask && mask[i]) continue;
        u[Fk->ind[i]] += r[i];
      }
      for (int l = 0; l < Fk->nb; ++l) {
        const double* zr = Fk->Z + (size_t)l * d;
        for (int a = 0; a < d; ++a) v[a] += zr[a] * u[l];
      }
      free(u);
    } else {
      for (int64_t i = 0; i < n; ++i) {
        if (!all && mask && mask[i]) continue;
        const double* zr = Fk->Z + (size_t)i * d;
        for (int a = 0; a < d; ++a) v[a] += zr[a] * r[i];
      }
    }
    /* Penalised least squares (Appendix A.2): theta = (G + lambda D)^-1 v. */
    chol_solve(d, Fk->L[s], v, th);
    /* SSE_k = sum over rows of (r_i - b_k(x_i, theta))^2 (Algorithm A1). */
    double sse = 0.0;
    if (Fk->nb > 0) {
      double* fit = (double*)malloc(sizeof(double) * Fk->nb);
      for (int l = 0; l < Fk->nb; ++l) {
        const double* zr = Fk->Z + (size_t)l * d;
        double t = 0.0;
        for (int a = 0; a < d; ++a) t += zr[a] * th[a];
        fit[l] = t;
      }
      for (int64_t i = 0; i < n; ++i) {
        if (!all && mask && mask[i]) continue;
        double e = r[i] - fit[Fk->ind[i]];
        sse += e * e;
      }
      free(fit);
    } else {
      for (int64_t i = 0; i < n; ++i) {
        if (!all && mask && mask[i]) continue;
        const double* zr = Fk->Z + (size_t)i * d;
        double t = 0.0;
        for (int a = 0; a < d; ++a) t += zr[a] * th[a];
        double e = r[i] - t;
        sse += e * e;
      }
    }
    sse_all[k] = sse;
    for (int a = 0; a < d_max; ++a) theta_all[(size_t)k * d_max + a] = (a < d) ? th[a] : 0.0;
  }
  int best = 0;
  for (int k = 1; k < p; ++k)
    if (sse_all[k] < sse_all[best]) best = k;
  int second = -1;
  for (int k = 0; k < p; ++k)
    if (k != best && (second < 0 || sse_all[k] < sse_all[second])) second = k;
  out->own = best;
  out->k = (forced >= 0) ? forced : best;
  if (forced >= 0) out->gap = sse_all[forced] - sse_all[best];
  else out->gap = (second >= 0) ? sse_all[second] - sse_all[best] : INFINITY;
  out->sse = sse_all[out->k];
  for (int a = 0; a < d_max; ++a) out->theta[a] = theta_all[(size_t)out->k * d_max + a];
  double rtr = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!all && mask && mask[i]) continue;
    rtr += r[i] * r[i];
  }
  out->rtr = rtr;
}

/* f_i += step * b_k(x_i, theta) on all rows. */
static void add_learner(const feat_t* F, int64_t n, const double* theta, double step, double* f) {
  int d = F->d;
  if (F->nb > 0) {
    double* fit = (double*)malloc(sizeof(double) * F->nb);
    for (int l = 0; l < F->nb; ++l) {
      const double* zr = F->Z + (size_t)l * d;
      double t = 0.0;
      for (int a = 0; a < d; ++a) t += zr[a] * theta[a];
      fit[l] = t;
    }
    for (int64_t i = 0; i < n; ++i) f[i] += step * fit[F->ind[i]];
    free(fit);
  } else {
    for (int64_t i = 0; i < n; ++i) {
      const double* zr = F->Z + (size_t)i * d;
      double t = 0.0;
      for (int a = 0; a < d; ++a) t += zr[a] * theta[a];
      f[i] += step * t;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Setup: binning, bases, penalties, Grams, smoothing parameters.            */
/* ------------------------------------------------------------------------ */

static int setup(const orc_problem* pr, feat_t** out, int need_all_set, orc_result* res) {
  int p = pr->p;
  int64_t n = pr->n;
  feat_t* F = (feat_t*)calloc((size_t)p, sizeof(feat_t));
  int* frc = (int*)calloc((size_t)p, sizeof(int));
  int64_t off = 0;
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int j = 0; j < p; ++j) {
    feat_t* Fj = &F[j];
    const double* xj = pr->x + (size_t)j * n;
    Fj->kind = pr->kind[j];
    if (Fj->kind == ORC_RIDGE || Fj->kind == ORC_BINARY) {
      int c = pr->n_levels[j];
      Fj->d = c;
      Fj->nb = c;
      Fj->ind = (int32_t*)malloc(sizeof(int32_t) * n);
      for (int64_t i = 0; i < n; ++i) Fj->ind[i] = (int32_t)xj[i];
      /* dummy encoding: the reduced design matrix is the identity */
      Fj->Z = (double*)calloc((size_t)c * c, sizeof(double));
      for (int l = 0; l < c; ++l) Fj->Z[(size_t)l * c + l] = 1.0;
      Fj->D = (double*)malloc(sizeof(double) * c * c);
      orc_penalty(c, 0, Fj->D);
    } else {
      double xmin = xj[0], xmax = xj[0];
      for (int64_t i = 1; i < n; ++i) {
        if (xj[i] < xmin) xmin = xj[i];
        if (xj[i] > xmax) xmax = xj[i];
      }
      double t[128];
      int nk = orc_knots(xmin, xmax, pr->n_knots, pr->degree, t);
      int d = nk - pr->degree - 1;
      Fj->d = d;
      Fj->nb = pr->n_bins[j];
      if (Fj->nb > 0) {
        double* z = (double*)malloc(sizeof(double) * Fj->nb);
        Fj->ind = (int32_t*)malloc(sizeof(int32_t) * n);
        orc_bin_feature(xj, n, Fj->nb, z, Fj->ind);
        Fj->Z = (double*)malloc(sizeof(double) * (size_t)Fj->nb * d);
        for (int l = 0; l < Fj->nb; ++l) orc_bspline(z[l], t, nk, pr->degree, Fj->Z + (size_t)l * d);
        free(z);
      } else {
        Fj->Z = (double*)malloc(sizeof(double) * (size_t)n * d);
        for (int64_t i = 0; i < n; ++i) orc_bspline(xj[i], t, nk, pr->degree, Fj->Z + (size_t)i * d);
      }
      Fj->D = (double*)malloc(sizeof(double) * d * d);
      orc_penalty(d, pr->pen_order, Fj->D);
    }
    for (int s = 0; s < 2; ++s) {
      if (s == 1 && !need_all_set) break;
      Fj->G[s] = (double*)malloc(sizeof(double) * Fj->d * Fj->d);
      gram(Fj, n, pr->val_mask, s == 1, Fj->G[s]);
      int rc = prepare_set(Fj, s, pr->df[j], pr->lambda[j]);
      if (rc) { frc[j] = rc; break; }
    }
  }
  for (int j = 0; j < p; ++j)
    if (frc[j]) { err = frc[j]; break; }
  free(frc);
  if (err) { free_feats(F, p); return err; }
  for (int j = 0; j < p; ++j) {
    F[j].off = off;
    off += F[j].d;
    if (res->d) res->d[j] = F[j].d;
    if (res->lambda_train) res->lambda_train[j] = F[j].lambda[0];
    if (res->lambda_all) res->lambda_all[j] = need_all_set ? F[j].lambda[1] : F[j].lambda[0];
  }
  *out = F;
  return ORC_OK;
}

static int validate(const orc_problem* pr) {
  if (pr->n < 2 || pr->p < 1) return fail(ORC_E_ARG, "need n >= 2 and p >= 1");
  if (!pr->x || !pr->y) return fail(ORC_E_ARG, "null data");
  if (pr->M < 1 || !(pr->nu > 0.0)) return fail(ORC_E_ARG, "need M >= 1 and nu > 0");
  if (pr->loss == ORC_BINOMIAL)
    for (int64_t i = 0; i < pr->n; ++i)
      if (pr->y[i] != 0.0 && pr->y[i] != 1.0) return fail(ORC_E_ARG, "binomial y must be 0/1");
  if (pr->variant == ORC_HCWB && !pr->val_mask) return fail(ORC_E_ARG, "HCWB needs a validation mask");
  if (pr->val_mask) {
    int64_t nv = 0;
    for (int64_t i = 0; i < pr->n; ++i) nv += pr->val_mask[i] ? 1 : 0;
    if (nv == 0 || nv == pr->n) return fail(ORC_E_ARG, "empty training or validation split");
  }
  for (int j = 0; j < pr->p; ++j) {
    const double* xj = pr->x + (size_t)j * pr->n;
    if (pr->kind[j] == ORC_RIDGE || pr->kind[j] == ORC_BINARY) {
      if (pr->n_levels[j] < 1 || pr->n_levels[j] > 64) return fail(ORC_E_ARG, "bad level count");
      for (int64_t i = 0; i < pr->n; ++i) {
        double v = xj[i];
        if (!(v >= 0.0) || v >= (double)pr->n_levels[j] || v != floor(v))
          return fail(ORC_E_ARG, "level code out of range");
      }
    } else {
      double mn = xj[0], mx = xj[0];
      for (int64_t i = 1; i < pr->n; ++i) {
        if (xj[i] < mn) mn = xj[i];
        if (xj[i] > mx) mx = xj[i];
      }
      if (!(mx > mn)) return fail(ORC_E_ARG, "constant feature");
      if (pr->n_bins[j] == 1 || pr->n_bins[j] < 0) return fail(ORC_E_ARG, "bad bin count");
      if (pr->degree < 0 || pr->degree > 5 || pr->n_knots < 0 || pr->n_knots + pr->degree + 1 > 64)
        return fail(ORC_E_ARG, "bad spline degree or knot count");
    }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The boosting loops: CWB (Algorithm A1), ACWB (Algorithm 2), HCWB          */
/* (Algorithm 3).                                                             */
/* ------------------------------------------------------------------------ */

int orc_fit(const orc_problem* pr, orc_result* res) {
  int rc = validate(pr);
  if (rc) return rc;
  const int64_t n = pr->n;
  const int p = pr->p;
  const int M = pr->M;
  const int loss = pr->loss;
  const uint8_t* mask = pr->val_mask;
  int32_t d_max, sum_d;
  orc_sizes(pr, &d_max, &sum_d);
  feat_t* F = NULL;
  const double t_start = omp_get_wtime();
  rc = setup(pr, &F, pr->variant == ORC_HCWB, res);
  if (rc) return rc;
  const double t_setup = omp_get_wtime();

  double* f = (double*)malloc(sizeof(double) * n);
  double* h = (double*)malloc(sizeof(double) * n);
  double* g = (double*)malloc(sizeof(double) * n);
  double* r = (double*)malloc(sizeof(double) * n);
  double* c = (double*)malloc(sizeof(double) * n);
  double* sse_all = (double*)malloc(sizeof(double) * p);
  double* theta_all = (double*)malloc(sizeof(double) * (size_t)p * d_max);
  double* th_f = (double*)calloc((size_t)sum_d, sizeof(double));
  double* th_h = (double*)calloc((size_t)sum_d, sizeof(double));

  /* f^[0] = loss-optimal constant over the training rows. */
  double f0 = loss_optimal_constant(loss, pr->y, n, mask);
  if (!isfinite(f0)) { rc = fail(ORC_E_NUMERIC, "non-finite initial constant"); goto done; }
  *res->f0 = f0;
  for (int64_t i = 0; i < n; ++i) { f[i] = f0; h[i] = f0; g[i] = f0; c[i] = 0.0; }

  res->risk_train[0] = empirical_risk(loss, pr->y, f, n, mask, 0);
  res->risk_val[0] = mask ? empirical_risk(loss, pr->y, f, n, mask, 1) : 0.0;
  *res->switch_iter = -1;
  *res->own_switch = -1;

  int counter = 0, switched = 0;
  double rv_prev = res->risk_val[0];
  int prev_kcor = -1;
  double prev_thcor[64];

  for (int m = 1; m <= M; ++m) {
    int mi = m - 1;
    int acwb_step = (pr->variant == ORC_ACWB);
    if (pr->variant == ORC_HCWB) {
      if (!switched) {
        int go = (pr->force_switch >= 0) ? (m >= pr->force_switch) : (counter >= pr->patience);
        if (counter >= pr->patience && *res->own_switch < 0) *res->own_switch = m;
        if (go) { switched = 1; *res->switch_iter = m; }
      }
      acwb_step = !switched;
    }
    int fk = pr->force_k ? pr->force_k[mi] : -1;
    int fkc = pr->force_kcor ? pr->force_kcor[mi] : -1;
    pick_t pk;
    if (!acwb_step) {
      /* CWB step.  HCWB after the switch uses all rows and the all-row Grams. */
      int all = (pr->variant == ORC_HCWB);
      int set = all ? 1 : 0;
      for (int64_t i = 0; i < n; ++i) r[i] = pseudo_residual(loss, pr->y[i], f[i]);
      find_best(F, p, n, r, mask, all, set, fk, sse_all, theta_all, d_max, &pk);
      add_learner(&F[pk.k], n, pk.theta, pr->nu, f);
      for (int a = 0; a < F[pk.k].d; ++a) th_f[F[pk.k].off + a] += pr->nu * pk.theta[a];
      res->kcor[mi] = -1;
      res->own_kcor[mi] = -1;
      res->gapcor[mi] = 0.0;
      res->rtr_cor[mi] = 0.0;
      res->sse_cor[mi] = 0.0;
      for (int a = 0; a < d_max; ++a) res->thetacor[(size_t)mi * d_max + a] = 0.0;
    } else {
      /* ACWB step on the training rows (Algorithm 2). */
      double vt = 2.0 / ((double)m + 1.0);
      for (int64_t i = 0; i < n; ++i) g[i] = (1.0 - vt) * f[i] + vt * h[i];
      for (int64_t i = 0; i < n; ++i) r[i] = pseudo_residual(loss, pr->y[i], g[i]);
      find_best(F, p, n, r, mask, 0, 0, fk, sse_all, theta_all, d_max, &pk);
      for (int64_t i = 0; i < n; ++i) f[i] = g[i];
      add_learner(&F[pk.k], n, pk.theta, pr->nu, f);
      /* error-corrected pseudo-residuals */
      if (m == 1 || prev_kcor < 0) {
        for (int64_t i = 0; i < n; ++i) c[i] = r[i];
      } else {
        double w = (double)m / ((double)m + 1.0);
        /* c - b_cor^[m-1](x) */
        add_learner(&F[prev_kcor], n, prev_thcor, -1.0, c);
        for (int64_t i = 0; i < n; ++i) c[i] = r[i] + w * c[i];
      }
      pick_t pc;
      find_best(F, p, n, c, mask, 0, 0, fkc, sse_all, theta_all, d_max, &pc);
      double eta = pr->gamma * pr->nu / vt;
      add_learner(&F[pc.k], n, pc.theta, eta, h);
      /* parameter bookkeeping of the three models (Section 3.2.1) */
      for (int64_t a = 0; a < sum_d; ++a) th_f[a] = (1.0 - vt) * th_f[a] + vt * th_h[a];
      for (int a = 0; a < F[pk.k].d; ++a) th_f[F[pk.k].off + a] += pr->nu * pk.theta[a];
      for (int a = 0; a < F[pc.k].d; ++a) th_h[F[pc.k].off + a] += eta * pc.theta[a];
      prev_kcor = pc.k;
      memcpy(prev_thcor, pc.theta, sizeof(double) * d_max);
      res->kcor[mi] = pc.k;
      res->own_kcor[mi] = pc.own;
      res->gapcor[mi] = pc.gap;
      res->rtr_cor[mi] = pc.rtr;
      res->sse_cor[mi] = pc.sse;
      for (int a = 0; a < d_max; ++a) res->thetacor[(size_t)mi * d_max + a] = pc.theta[a];
    }
    res->k[mi] = pk.k;
    res->own_k[mi] = pk.own;
    res->gap[mi] = pk.gap;
    res->sse[mi] = pk.sse;
    res->rtr[mi] = pk.rtr;
    for (int a = 0; a < d_max; ++a) res->theta[(size_t)mi * d_max + a] = pk.theta[a];
    res->risk_train[m] = empirical_risk(loss, pr->y, f, n, mask, 0);
    res->risk_val[m] = mask ? empirical_risk(loss, pr->y, f, n, mask, 1) : 0.0;
    if (pr->variant == ORC_HCWB && acwb_step) {
      /* patience: count consecutive rises of the validation risk */
      if (res->risk_val[m] > rv_prev) counter += 1; else counter = 0;
      rv_prev = res->risk_val[m];
    }
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) if (!isfinite(f[i])) { bad = 1; break; }
    if (bad) { rc = fail(ORC_E_NUMERIC, "non-finite model state"); goto done; }
  }
  if (pr->variant == ORC_HCWB && !switched && counter >= pr->patience && *res->own_switch < 0)
    *res->own_switch = M + 1;
  if (res->seconds) {
    res->seconds[0] = t_setup - t_start;
    res->seconds[1] = omp_get_wtime() - t_setup;
  }
  memcpy(res->f, f, sizeof(double) * n);
  memcpy(res->coef_f, th_f, sizeof(double) * sum_d);
  memcpy(res->coef_h, th_h, sizeof(double) * sum_d);

done:
  free(f); free(h); free(g); free(r); free(c);
  free(sse_all); free(theta_all); free(th_f); free(th_h);
  free_feats(F, p);
  return rc;
}
