// algebra.h -- the per-learner FP64 algebra of fit setup, written once for
// the host setup (setup.cpp) and the device setup pass (binning.hip), so that
// both give bitwise the same results: only +, -, *, / and sqrt, each value
// computed by the same sequence of operations on both sides, built without
// contraction (-ffp-contract=off).
//
// For one learner and one row set (training rows, or all rows):
//   G = Z^bT diag(counts) Z^b   binMatMat from the bin counts (Algorithm 1);
//   lambda with tr((G + lambda D)^-1 G) = df   (App. A.2), by Newton's
//       method on lambda inside a sign-change bracket, with df and its
//       derivative from the Demmler-Reinsch eigenvalues (G = L L^T,
//       eigenvalues of L^-1 D L^-T by round-robin Jacobi rotations), or from
//       the hat-matrix trace when G is singular;
//   (G + lambda D)^-1 by Cholesky (Sec. 2.4).
// Matrices are row-major d x d doubles, d <= 64; every routine takes its
// scratch from the caller.
//
// Every routine takes an executor ex.  ex.each(n, f) calls f(0) .. f(n-1)
// and returns once all calls are done: one after another on the host
// (Serial), spread over the lanes of a block on the device (Lanes, with a
// block barrier before and after).  Each f(i) writes its own elements only and
// reads what earlier each() calls wrote, so the element values do not
// depend on how the calls are spread.  Scalars outside each() (sums over a
// diagonal, the rotation angles, the Newton steps) are computed by every
// lane alike from the same shared values.
#pragma once
#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#define CWB_HD __host__ __device__
#else
#define CWB_HD
#endif

namespace cwb {
namespace alg {

struct Serial {
  template <class F>
  CWB_HD void each(int n, F f) const {
    for (int i = 0; i < n; ++i) f(i);
  }
};

#if defined(__HIPCC__)
// The threads of one block (all of them must call every routine alike).
struct Lanes {
  int lane, width;
  template <class F>
  __device__ void each(int n, F f) const {
    __syncthreads();  // every lane's reads of the shared values are done
    for (int i = lane; i < n; i += width) f(i);
    __syncthreads();
  }
};
#endif

CWB_HD inline double dabs(double v) { return v < 0.0 ? -v : v; }
CWB_HD inline double dmax(double a, double b) { return a > b ? a : b; }
CWB_HD inline bool finite(double v) { return v == v && dabs(v) <= 1.7976931348623157e308; }

// Cholesky factor L (lower) of A; false unless A is positive definite.
// Column j: its diagonal by every lane, then its entries below in parallel.
template <class E>
CWB_HD inline bool chol(const E& ex, int d, const double* A, double* L) {
  ex.each(d * d, [&](int i) { L[i] = 0.0; });
  for (int j = 0; j < d; ++j) {
    double s = A[j * d + j];
    for (int k = 0; k < j; ++k) s -= L[j * d + k] * L[j * d + k];
    if (!(s > 0.0) || !finite(s)) return false;
    const double ljj = sqrt(s);
    ex.each(d - j, [&](int r) {
      const int i = j + r;
      if (r == 0) {
        L[j * d + j] = ljj;
        return;
      }
      double t = A[i * d + j];
      for (int k = 0; k < j; ++k) t -= L[i * d + k] * L[j * d + k];
      L[i * d + j] = t / ljj;
    });
  }
  return true;
}

// X = L^-1 for lower-triangular L, one column per call.
template <class E>
CWB_HD inline void tri_inverse(const E& ex, int d, const double* L, double* X) {
  ex.each(d * d, [&](int i) { X[i] = 0.0; });
  ex.each(d, [&](int c) {
    for (int i = c; i < d; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) t -= L[i * d + k] * X[k * d + c];
      X[i * d + c] = t / L[i * d + i];
    }
  });
}

// inv = A^-1 = L^-T L^-1 for symmetric positive definite A; scratch 2 d^2.
template <class E>
CWB_HD inline bool spd_inverse(const E& ex, int d, const double* A, double* inv, double* scr) {
  double* L = scr;
  double* Li = scr + d * d;
  if (!chol(ex, d, A, L)) return false;
  tri_inverse(ex, d, L, Li);
  ex.each(d * d, [&](int e) {
    const int i = e / d, j = e % d;
    if (j > i) return;
    double s = 0.0;
    for (int k = i; k < d; ++k) s += Li[k * d + i] * Li[k * d + j];
    inv[i * d + j] = s;
    inv[j * d + i] = s;
  });
  return true;
}

// Scratch doubles jacobi needs beside S and w: a cosine, a sine and a flag
// per rotation of one round.
CWB_HD inline int jacobi_scratch(int d) { return 3 * ((d + 1) / 2); }

// Eigenvalues w of the symmetric S (overwritten) by Jacobi rotations in
// round-robin order: each sweep is d - 1 (d even; d for odd d, with one
// index idle per round) rounds of disjoint pairs (p, q), which together
// meet every pair once.  A round's rotations touch disjoint rows and
// columns, so they are computed from the matrix at the round's start and
// applied together: all pairs' columns, then all pairs' rows.
template <class E>
CWB_HD inline void jacobi(const E& ex, int d, double* S, double* w, double* rot) {
  const int m = d + (d & 1);  // players of the round robin: a dummy for odd d
  const int np = m / 2;
  double* rc = rot;
  double* rs = rot + np;
  double* rf = rot + 2 * np;  // 1 if the pair rotates this round
  // pair i of round r: m - 1 stays, the others turn around it
  auto pair = [m](int r, int i, int* p, int* q) {
    int a, b;
    if (i == 0) {
      a = m - 1;
      b = r;
    } else {
      a = (r + i) % (m - 1);
      b = (r - i + m - 1) % (m - 1);
    }
    *p = a < b ? a : b;
    *q = a < b ? b : a;
  };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        const double v = S[i * d + j] * S[i * d + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int r = 0; r < m - 1; ++r) {
      ex.each(np, [&](int i) {  // the round's rotations
        int p, q;
        pair(r, i, &p, &q);
        double c = 1.0, sn = 0.0, act = 0.0;
        if (q < d && S[p * d + q] != 0.0) {
          const double apq = S[p * d + q];
          const double app = S[p * d + p], aqq = S[q * d + q];
          const double theta = (aqq - app) / (2.0 * apq);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (dabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sn = t * c;
          act = 1.0;
        }
        rc[i] = c;
        rs[i] = sn;
        rf[i] = act;
      });
      ex.each(np * d, [&](int e) {  // columns p, q of pair i, row k
        const int i = e / d, k = e % d;
        if (rf[i] == 0.0) return;
        int p, q;
        pair(r, i, &p, &q);
        const double c = rc[i], sn = rs[i];
        const double akp = S[k * d + p], akq = S[k * d + q];
        S[k * d + p] = c * akp - sn * akq;
        S[k * d + q] = sn * akp + c * akq;
      });
      ex.each(np * d, [&](int e) {  // rows p, q of pair i, column k
        const int i = e / d, k = e % d;
        if (rf[i] == 0.0) return;
        int p, q;
        pair(r, i, &p, &q);
        const double c = rc[i], sn = rs[i];
        const double apk = S[p * d + k], aqk = S[q * d + k];
        S[p * d + k] = c * apk - sn * aqk;
        S[q * d + k] = sn * apk + c * aqk;
      });
    }
  }
  ex.each(d, [&](int i) { w[i] = S[i * d + i]; });
}

// P = Delta^T Delta for the difference matrix of order `ord` (0: identity);
// scratch d^2 (Delta, differenced one column per call).
template <class E>
CWB_HD inline void penalty(const E& ex, int d, int ord, double* P, double* Dm) {
  ex.each(d, [&](int j) {
    for (int i = 0; i < d; ++i) Dm[i * d + j] = (i == j) ? 1.0 : 0.0;  // Delta^(0) = I
    int rows = d;
    for (int o = 0; o < ord; ++o) {  // Delta^(o+1)[i] = Delta^(o)[i+1] - Delta^(o)[i]
      for (int i = 0; i < rows - 1; ++i) Dm[i * d + j] = Dm[(i + 1) * d + j] - Dm[i * d + j];
      --rows;
    }
  });
  const int rows = d - ord;
  ex.each(d * d, [&](int e) {
    const int i = e / d, j = e % d;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) {
      const double a = Dm[r * d + i];
      if (a == 0.0) continue;
      s += a * Dm[r * d + j];
    }
    P[e] = s;
  });
}

// G = Z^bT diag(cnt) Z^b for a banded reduced design (bstart[l] and `band`
// values per design point, row stride `stride`); the counts as doubles or
// as the device setup pass's 32-bit integers (exact either way).  One row
// of G per call, summed over the design points in order.
template <class E, class C>
CWB_HD inline void gram_from_counts(const E& ex, int d, int nb, int band, const int32_t* bstart,
                                    const double* bval, int stride, const C* cnt, double* G) {
  ex.each(d, [&](int i) {
    for (int j = 0; j < d; ++j) G[i * d + j] = 0.0;
    for (int l = 0; l < nb; ++l) {
      const double cl = (double)cnt[l];
      if (cl == 0.0) continue;
      const int b0 = bstart[l], a = i - b0;
      if (a < 0 || a >= band) continue;
      const double* bv = bval + (int64_t)l * stride;
      for (int b = 0; b < band; ++b) G[i * d + (b0 + b)] += cl * bv[a] * bv[b];
    }
  });
}

// Scratch doubles lambda_for_df needs.
CWB_HD inline int lambda_scratch(int d) { return 8 * d * d + d + jacobi_scratch(d); }

// lambda >= 0 with df(lambda) = tr((G + lambda D)^-1 G) = target.  Newton's
// method on g(lambda) = df(lambda) - target, which decreases monotonically,
// kept inside a bracket [la, lb] with g(la) > 0 > g(lb): the bracket widens
// from trG / trD by factors of 128 (exact), at most 7 times each way (2^49,
// beyond which the rounding noise in the penalty's null-space eigenvalues
// would reach a target below that null space's dimension), and a
// Newton step that would leave it is replaced by the bracket's geometric
// mean.  df and d df / d lambda come from the Demmler-Reinsch eigenvalues w
// when G is positive definite (df = sum 1/(1 + lambda w),
// df' = -sum w/(1 + lambda w)^2), else from A = G + lambda D directly
// (df = tr(A^-1 G), df' = -tr(A^-1 D A^-1 G)).  Returns 0, -1 (target out
// of reach within the bracket) or -5 (degenerate G or D, or A not positive
// definite).
template <class E>
CWB_HD inline int lambda_for_df(const E& ex, int d, const double* G, const double* D,
                                double target, double* lam_out, double* scr) {
  double* L = scr;
  double* Li = scr + d * d;
  double* T = scr + 2 * d * d;
  double* S = scr + 3 * d * d;
  double* A = scr + 4 * d * d;
  double* P = scr + 5 * d * d;   // A^-1 G
  double* Q = scr + 6 * d * d;   // A^-1 D
  double* inv = scr + 7 * d * d;
  double* w = scr + 8 * d * d;
  double* rot = w + d;
  const bool dro = chol(ex, d, G, L);
  if (dro) {
    tri_inverse(ex, d, L, Li);
    ex.each(d * d, [&](int e) {  // T = L^-1 D
      const int i = e / d, j = e % d;
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += Li[i * d + k] * D[k * d + j];
      T[e] = s;
    });
    ex.each(d * d, [&](int e) {  // S = T L^-T
      const int i = e / d, j = e % d;
      double s = 0.0;
      for (int k = 0; k <= j; ++k) s += T[i * d + k] * Li[j * d + k];
      S[e] = s;
    });
    ex.each(d * d, [&](int e) {  // symmetrise
      const int i = e / d, j = e % d;
      if (j <= i) return;
      const double a = 0.5 * (S[i * d + j] + S[j * d + i]);
      S[i * d + j] = a;
      S[j * d + i] = a;
    });
    jacobi(ex, d, S, w, rot);
    ex.each(d, [&](int i) { w[i] = dmax(w[i], 0.0); });
  }
  // g(lambda) and g'(lambda); false if A is not positive definite
  auto eval = [&](double lam, double* g, double* dg) -> bool {
    if (dro) {
      double f = 0.0, fp = 0.0;
      for (int i = 0; i < d; ++i) {
        const double q = 1.0 / (1.0 + lam * w[i]);
        f += q;
        fp -= w[i] * q * q;
      }
      *g = f - target;
      *dg = fp;
      return true;
    }
    ex.each(d * d, [&](int e) { A[e] = G[e] + lam * D[e]; });
    if (!spd_inverse(ex, d, A, inv, T)) return false;  // T, S as its scratch
    ex.each(d * d, [&](int e) {
      const int i = e / d, j = e % d;
      double p = 0.0, q = 0.0;
      for (int k = 0; k < d; ++k) {
        const double a = inv[i * d + k];
        p += a * G[k * d + j];
        q += a * D[k * d + j];
      }
      P[e] = p;
      Q[e] = q;
    });
    double f = 0.0, fp = 0.0;
    for (int i = 0; i < d; ++i) {
      f += P[i * d + i];
      for (int k = 0; k < d; ++k) fp -= Q[i * d + k] * P[k * d + i];
    }
    *g = f - target;
    *dg = fp;
    return true;
  };
  double trG = 0.0, trD = 0.0;
  for (int i = 0; i < d; ++i) {
    trG += G[i * d + i];
    trD += D[i * d + i];
  }
  if (!(trG > 0.0) || !(trD > 0.0)) return -5;
  const double lam0 = trG / trD;
  constexpr double kWiden = 128.0;
  constexpr int kSteps = 7;
  double la = lam0, lb = lam0, g = 0.0, dg = 0.0;
  int i = 0;
  for (; i <= kSteps; ++i, la /= kWiden) {
    if (!eval(la, &g, &dg)) return -5;
    if (g > 0.0) break;
  }
  if (i > kSteps) return -1;
  for (i = 0; i <= kSteps; ++i, lb *= kWiden) {
    if (!eval(lb, &g, &dg)) return -5;
    if (g < 0.0) break;
  }
  if (i > kSteps) return -1;
  double lam = sqrt(la * lb);
  for (int it = 0; it < 200; ++it) {
    if (!eval(lam, &g, &dg)) return -5;
    if (g == 0.0) break;
    if (g > 0.0) la = lam; else lb = lam;
    double ln = (dg < 0.0) ? lam - g / dg : sqrt(la * lb);
    if (!(ln > la && ln < lb)) ln = sqrt(la * lb);
    if (dabs(ln - lam) <= 8.9e-16 * lam) {  // 4 ulp of lambda
      lam = ln;
      break;
    }
    lam = ln;
  }
  *lam_out = lam;
  return 0;
}

// One learner's solve set from its counts: G, lambda and (G + lambda D)^-1.
// kind: 0 P-spline (penalty of order pen_order), 1 ridge categorical
// (D = I), 2 binary categorical (G = diag(counts), no penalty; an empty
// class keeps a zero inverse entry).  df > 0 asks for lambda with that df
// (a ridge learner with df >= d takes lambda = 0), else lambda is `lambda`.
// Scratch: solve_scratch(d) doubles.  Returns 0, -1 or -5 as lambda_for_df
// (-5 too when G + lambda D is not positive definite).
CWB_HD inline int solve_scratch(int d) { return 2 * d * d + lambda_scratch(d); }

template <class E, class C>
CWB_HD inline int learner_solve(const E& ex, int kind, int d, int nb, int band,
                                const int32_t* bstart, const double* bval, int stride,
                                const C* cnt, int pen_order, double df, double lambda, double* G,
                                double* inv, double* lam_out, double* scr) {
  if (kind == 2) {
    ex.each(d * d, [&](int e) {
      const int i = e / d, j = e % d;
      const double ci = (double)cnt[i];
      G[e] = (i == j) ? ci : 0.0;
      inv[e] = (i == j && ci > 0.0) ? 1.0 / ci : 0.0;
    });
    *lam_out = 0.0;
    return 0;
  }
  double* D = scr;
  double* A = scr + d * d;
  double* rest = scr + 2 * d * d;
  gram_from_counts(ex, d, nb, band, bstart, bval, stride, cnt, G);
  penalty(ex, d, kind == 0 ? pen_order : 0, D, rest);
  double lam = lambda;
  if (df > 0.0) {
    if (kind == 1 && df >= (double)d) {
      lam = 0.0;
    } else {
      const int rc = lambda_for_df(ex, d, G, D, df, &lam, rest);
      if (rc) return rc;
    }
  }
  *lam_out = lam;
  ex.each(d * d, [&](int e) { A[e] = G[e] + lam * D[e]; });
  return spd_inverse(ex, d, A, inv, rest) ? 0 : -5;
}

}  // namespace alg
}  // namespace cwb
