"""Literal dense-matrix NumPy/SciPy boosting for tiny inputs.

An independent cross-check of the C oracle: every learner keeps its full
n x d design matrix (the discretised feature's B(x~) for binned learners,
built with scipy's B-spline design matrix), every fit solves the penalised
normal equations with numpy, and every SSE is formed from an explicit
residual vector.  No binMatVec, no cached factorisation, nothing shared with
the oracle's C code.  Only for n * p small.

A categorical feature in the binary representation becomes one learner per
class with that class's indicator column and no penalty (least squares); the
learner sequence is reported by feature, with the coefficient vector over the
feature's classes (one nonzero entry).
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import BSpline
from scipy.optimize import brentq


def knots(xmin, xmax, n_int=20, degree=3):
    h = (xmax - xmin) / (n_int + 1)
    return xmin + (np.arange(n_int + 2 + 2 * degree) - degree) * h


def design_pspline(xv, xmin, xmax, n_int=20, degree=3):
    t = knots(xmin, xmax, n_int, degree)
    return BSpline.design_matrix(np.asarray(xv, float), t, degree, extrapolate=True).toarray()


def discretise(x, nb):
    """Closest of nb equally spaced design points; ties to the lower point."""
    xmin, xmax = x.min(), x.max()
    z = xmin + np.arange(nb) * ((xmax - xmin) / (nb - 1))
    z[-1] = xmax
    dist = np.abs(x[:, None] - z[None, :])
    ind = np.argmin(dist, axis=1)  # first minimum = lower index on ties
    return z, ind


def second_diff_penalty(d, order=2):
    Dl = np.diff(np.eye(d), n=order, axis=0)
    return Dl.T @ Dl


class Learner:
    def __init__(self, Z, D, rows_fit, df, lam=0.0, all_rows=None, feat=0, cls=-1, width=None):
        self.Z = Z
        self.D = D
        self.feat = feat    # feature index
        self.cls = cls      # class of a binary learner, else -1
        self.width = Z.shape[1] if width is None else width  # coefficient length of the feature
        self.lam = {}
        self.lam["train"] = self._lambda(Z[rows_fit], df, lam)
        if all_rows is not None:
            self.lam["all"] = self._lambda(Z, df, lam)

    def _lambda(self, Z, df, lam):
        if df <= 0:
            return lam
        G = Z.T @ Z
        d = G.shape[0]
        if np.allclose(self.D, np.eye(d)) and df >= d:
            return 0.0

        def dfun(loglam):
            return np.trace(np.linalg.solve(G + np.exp(loglam) * self.D, G)) - df

        s = np.log(np.trace(G) / np.trace(self.D))
        return float(np.exp(brentq(dfun, s - 18.0, s + 25.0, xtol=1e-14, rtol=1e-15,
                                   maxiter=500)))

    def fit(self, r, rows, which):
        Z = self.Z[rows]
        A = Z.T @ Z + self.lam[which] * self.D
        if self.cls >= 0 and A[0, 0] == 0.0:  # empty class: no estimate
            return np.zeros(1), np.inf
        theta = np.linalg.solve(A, Z.T @ r[rows])
        resid = r[rows] - Z @ theta
        return theta, float(resid @ resid)


def build(problem, binned=True):
    x = np.asarray(problem["x"], float)
    n, p = x.shape
    vm = problem.get("val_mask")
    train = np.ones(n, bool) if vm is None else (np.asarray(vm) == 0)
    learners = []
    for j in range(p):
        if int(problem["kind"][j]) == 2:
            c = int(problem["n_levels"][j])
            for l in range(c):
                Z = (x[:, j].astype(int) == l).astype(float)[:, None]
                learners.append(Learner(Z, np.zeros((1, 1)), train, 0.0, 0.0, all_rows=True,
                                        feat=j, cls=l, width=c))
            continue
        if int(problem["kind"][j]) == 1:
            c = int(problem["n_levels"][j])
            Z = np.eye(c)[x[:, j].astype(int)]
            D = np.eye(c)
        else:
            xmin, xmax = x[:, j].min(), x[:, j].max()
            nb = int(problem["n_bins"][j])
            if binned and nb > 0:
                z, ind = discretise(x[:, j], nb)
                xv = z[ind]
            else:
                xv = x[:, j]
            Z = design_pspline(xv, xmin, xmax, problem.get("n_knots", 20), problem.get("degree", 3))
            D = second_diff_penalty(Z.shape[1], problem.get("pen_order", 2))
        learners.append(Learner(Z, D, train, float(problem["df"][j]),
                                float(problem.get("lambda", np.zeros(p))[j]),
                                all_rows=True, feat=j))
    return learners, train


def grad(loss, y, f):
    if loss == "l2":
        return y - f
    return y - 1.0 / (1.0 + np.exp(-f))


def risk(loss, y, f):
    if loss == "l2":
        return float(np.mean(0.5 * (y - f) ** 2))
    return float(np.mean(np.logaddexp(0.0, f) - y * f))


def best(learners, r, rows, which):
    sses, thetas = [], []
    for L in learners:
        th, s = L.fit(r, rows, which)
        thetas.append(th)
        sses.append(s)
    k = int(np.argmin(sses))
    return k, thetas[k], np.array(sses)


def by_feature(learners, k, th):
    """Feature index and the coefficient vector over the feature's basis."""
    L = learners[k]
    if L.cls < 0:
        return L.feat, th
    full = np.zeros(L.width)
    full[L.cls] = th[0]
    return L.feat, full


def run(problem, binned=True, f0=None):
    """Dense CWB / ACWB / HCWB.  Returns dict with k, kcor, f, risk traces."""
    loss = problem["loss"]
    y = np.asarray(problem["y"], float)
    n = y.shape[0]
    M = int(problem["M"])
    nu = float(problem["nu"])
    gamma = float(problem.get("gamma", 0.0))
    variant = problem.get("variant", "cwb")
    learners, train = build(problem, binned)
    val = ~train
    allrows = np.ones(n, bool)
    if f0 is None:
        yb = y[train].mean()
        f0 = yb if loss == "l2" else np.log(yb / (1 - yb))
    f = np.full(n, f0)
    h = f.copy()
    c = np.zeros(n)
    ks, kcs, thetas = [], [], []
    rv = [risk(loss, y[val], f[val])] if val.any() else [0.0]
    counter, switched, switch_iter = 0, False, -1
    prev_cor = None
    pat = int(problem.get("patience", 5))
    for m in range(1, M + 1):
        acwb = variant == "acwb"
        if variant == "hcwb":
            if not switched and counter >= pat:
                switched, switch_iter = True, m
            acwb = not switched
        if not acwb:
            rows = allrows if variant == "hcwb" else train
            which = "all" if variant == "hcwb" else "train"
            r = grad(loss, y, f)
            k, th, _ = best(learners, r, rows, which)
            f = f + nu * learners[k].Z @ th
            kf, thf = by_feature(learners, k, th)
            ks.append(kf)
            kcs.append(-1)
            thetas.append(thf)
        else:
            vt = 2.0 / (m + 1)
            g = (1 - vt) * f + vt * h
            r = grad(loss, y, g)
            k, th, _ = best(learners, r, train, "train")
            f = g + nu * learners[k].Z @ th
            if m == 1:
                c = r.copy()
            else:
                kp, thp = prev_cor
                c = r + m / (m + 1) * (c - learners[kp].Z @ thp)
            kc, thc, _ = best(learners, c, train, "train")
            eta = gamma * nu / vt
            h = h + eta * learners[kc].Z @ thc
            prev_cor = (kc, thc)
            kf, thf = by_feature(learners, k, th)
            ks.append(kf)
            kcs.append(by_feature(learners, kc, thc)[0])
            thetas.append(thf)
        if val.any():
            rv.append(risk(loss, y[val], f[val]))
            if variant == "hcwb" and acwb:
                counter = counter + 1 if rv[-1] > rv[-2] else 0
    return {"k": np.array(ks), "kcor": np.array(kcs), "f": f, "theta": thetas,
            "risk_val": np.array(rv), "switch_iter": switch_iter, "f0": f0,
            "learners": learners}
