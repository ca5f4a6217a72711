"""The library's smoothing parameter for a df target (App. A.2), host only,
against NumPy/SciPy: the Demmler-Reinsch eigenvalue form solved by Brent's
method (positive definite Gram), the trace of the hat matrix solved the same
way (singular Gram), and the oracle's bisection."""
import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.optimize import brentq

import oracle
from paper_2110_03513_amd import cwb


def _basis(x, lo, hi, n_int=20, deg=3):
    h = (hi - lo) / (n_int + 1)
    t = lo + h * np.arange(-deg, n_int + deg + 2)
    return BSpline.design_matrix(np.clip(x, lo, hi), t, deg, extrapolate=True).toarray()


def _penalty(d):
    Dd = np.diff(np.eye(d), 2, axis=0)
    return Dd.T @ Dd


def _df_direct(G, D, lam):
    return float(np.trace(np.linalg.solve(G + lam * D, G)))


@pytest.mark.parametrize("target", [2.5, 4.0, 5.0, 10.0, 20.0, 23.5])
def test_lambda_matches_demmler_reinsch(target):
    rng = np.random.default_rng(int(target * 10))
    x = rng.uniform(-1, 2, 3000)
    Z = _basis(x, -1, 2)
    G = Z.T @ Z
    D = _penalty(24)
    L = np.linalg.cholesky(G)
    Li = np.linalg.inv(L)
    w = np.clip(np.linalg.eigvalsh(Li @ D @ Li.T), 0, None)
    lam_np = np.exp(brentq(lambda u: np.sum(1 / (1 + np.exp(u) * w)) - target, -80, 80,
                           xtol=1e-14, rtol=1e-15))
    lam = cwb.lambda_for_df(G, D, target)
    assert abs(lam - lam_np) <= 1e-9 * lam_np
    assert abs(_df_direct(G, D, lam) - target) <= 1e-9
    assert abs(lam - oracle.lambda_for_df(G, D, target)) <= 1e-9 * lam


def test_lambda_with_singular_gram():
    """Eight distinct values: rank(G) = 8 < 24, so the hat-matrix trace is
    used directly; df(lambda) falls from 8 to the penalty's null space (2)."""
    rng = np.random.default_rng(5)
    x = rng.choice(np.linspace(0, 1, 8), 500)
    Z = _basis(x, 0, 1)
    G = Z.T @ Z
    D = _penalty(24)
    assert np.linalg.matrix_rank(G) == 8
    for target in (3.0, 5.0, 7.5):
        lam_np = np.exp(brentq(lambda u: _df_direct(G, D, np.exp(u)) - target, -40, 40,
                               xtol=1e-13, rtol=1e-15))
        lam = cwb.lambda_for_df(G, D, target)
        assert abs(lam - lam_np) <= 1e-8 * lam_np
        assert abs(_df_direct(G, D, lam) - target) <= 1e-8


def test_lambda_errors():
    G = np.eye(4)
    D = _penalty(4)
    for bad in (0.0, 4.0, 7.0):
        with pytest.raises(cwb.CwbError):
            cwb.lambda_for_df(G, D, bad)
    with pytest.raises(cwb.CwbError):  # below the null space of the penalty (dimension 2)
        cwb.lambda_for_df(G, D, 1.5)
