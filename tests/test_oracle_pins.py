"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms, textbook / library routines (scipy B-splines, numpy least squares),
proven invariants, brute force on tiny inputs (tests/brute.py), and special
cases of the algorithms.
"""
import math
import os

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle
from paper_2110_03513_amd import datagen
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- B-spline basis (Section 2.2; P-splines, degree 3, 20 knots) -----------

def test_basis_matches_scipy_and_partition_of_unity():
    rng = np.random.default_rng(0)
    xmin, xmax = -1.3, 2.7
    t = oracle.knots(xmin, xmax, 20, 3)
    assert t.shape == (28,)
    x = np.concatenate([[xmin, xmax], rng.uniform(xmin, xmax, 500)])
    B = oracle.bspline(x, t, 3)
    assert B.shape == (502, 24)
    ref = BSpline.design_matrix(x, t, 3, extrapolate=True).toarray()
    np.testing.assert_allclose(B, ref, atol=1e-14)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert (B >= -1e-300).all()
    assert ((B > 0).sum(axis=1) <= 4).all()


def test_basis_golden_cardinal_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "cubic_bspline_uniform.txt"))
    t = oracle.knots(0.0, 21.0, 20, 3)  # knot spacing exactly 1
    for u, a, b, c, d, den in rows:
        x = 5.0 + u  # interval [t_8, t_9) = [5, 6): bases 5..8 are nonzero
        B = oracle.bspline([x], t, 3)[0]
        np.testing.assert_allclose(B[5:9], np.array([a, b, c, d]) / den, atol=1e-15)
        assert abs(B.sum() - 1.0) < 1e-15
    # endpoints: (1/6, 4/6, 1/6) on the first / last three bases
    B0 = oracle.bspline([0.0], t, 3)[0]
    B1 = oracle.bspline([21.0], t, 3)[0]
    np.testing.assert_allclose(B0[:3], [1 / 6, 4 / 6, 1 / 6], atol=1e-15)
    np.testing.assert_allclose(B1[-3:], [1 / 6, 4 / 6, 1 / 6], atol=1e-15)


# --- Binning (Section 3.1.1) -------------------------------------------------

def test_grid_and_nearest_brute_force():
    rng = np.random.default_rng(1)
    for nb in (2, 3, 17, 100, 1000):
        x = rng.uniform(-3, 5, 3000)
        z, ind = oracle.bin_feature(x, nb)
        assert z[0] == x.min() and z[-1] == x.max()
        assert (np.diff(z) > 0).all()
        dist = np.abs(x[:, None] - z[None, :])
        np.testing.assert_array_equal(ind, np.argmin(dist, axis=1))  # first min = lower


def test_binning_ties_go_to_lower_point():
    # grid 0, 0.25, ..., 1: midpoints are exactly representable
    x = np.array([0.0, 1.0, 0.125, 0.375, 0.625, 0.875, 0.5])
    z, ind = oracle.bin_feature(x, 5)
    np.testing.assert_array_equal(z, [0, 0.25, 0.5, 0.75, 1.0])
    np.testing.assert_array_equal(ind, [0, 4, 0, 1, 2, 3, 2])
    # one ulp either side of a midpoint
    m = 0.375
    x2 = np.array([0.0, 1.0, np.nextafter(m, 0), m, np.nextafter(m, 1)])
    _, ind2 = oracle.bin_feature(x2, 5)
    np.testing.assert_array_equal(ind2[2:], [1, 1, 2])


# --- Penalty, df and lambda (Appendix A.2) ----------------------------------

def test_penalty_is_second_difference():
    for d, o in ((24, 2), (10, 1), (8, 3)):
        Dl = np.diff(np.eye(d), n=o, axis=0)
        np.testing.assert_allclose(oracle.penalty(d, o), Dl.T @ Dl, atol=0)
    np.testing.assert_array_equal(oracle.penalty(5, 0), np.eye(5))


def _binned_gram(n=5000, nb=100, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, n)
    z, ind = oracle.bin_feature(x, nb)
    t = oracle.knots(x.min(), x.max(), 20, 3)
    Zb = oracle.bspline(z, t, 3)
    cnt = np.bincount(ind, minlength=nb)
    return Zb.T @ (cnt[:, None] * Zb)


def test_df_limits_and_root():
    G = _binned_gram()
    D = oracle.penalty(24, 2)
    assert abs(oracle.df_of_lambda(G, D, 0.0) - 24.0) < 1e-8  # rank G
    # lambda -> infinity leaves the 2-dim null space of the 2nd differences;
    # compare with the Demmler-Reinsch eigenvalue form at large lambda
    L = np.linalg.cholesky(G)
    Li = np.linalg.inv(L)
    w = np.linalg.eigvalsh(Li @ D @ Li.T)
    for lam in (1e2, 1e5, 1e8):
        assert abs(oracle.df_of_lambda(G, D, lam) - np.sum(1 / (1 + lam * w))) < 1e-7
    assert int(np.sum(np.abs(w) < 1e-9 * w.max())) == 2  # limit df(inf) = 2
    vals = [oracle.df_of_lambda(G, D, lam) for lam in (1e-3, 1e0, 1e3, 1e6, 1e9)]
    assert all(a > b for a, b in zip(vals, vals[1:])) and 2.0 < vals[-1] < 2.01
    for target in (3.0, 5.0, 10.0):
        lam = oracle.lambda_for_df(G, D, target)
        # independent evaluation: generalized eigenvalues (Demmler-Reinsch form)
        L = np.linalg.cholesky(G)
        Li = np.linalg.inv(L)
        w = np.linalg.eigvalsh(Li @ D @ Li.T)
        df_dr = np.sum(1.0 / (1.0 + lam * w))
        assert abs(df_dr - target) < 1e-8
        assert abs(np.trace(np.linalg.solve(G + lam * D, G)) - target) < 1e-9


# --- Losses -----------------------------------------------------------------

@pytest.mark.parametrize("name", ["l2", "binomial"])
def test_pseudo_residual_is_negative_gradient(name):
    for y in (0.0, 1.0) if name == "binomial" else (-1.3, 0.2, 4.0):
        for f in (-3.0, -0.2, 0.0, 0.7, 5.0):
            h = 1e-5
            num = -(oracle.loss(name, y, f + h) - oracle.loss(name, y, f - h)) / (2 * h)
            assert abs(num - oracle.pseudo_residual(name, y, f)) < 1e-8


def test_binomial_loss_large_margins_finite():
    assert oracle.loss("binomial", 1.0, 800.0) < 1e-300 + 1e-12
    assert abs(oracle.loss("binomial", 0.0, 800.0) - 800.0) < 1e-9


# --- CWB (Algorithm A1) -----------------------------------------------------

def _one_learner(n=300, seed=11, nb=0, loss="l2", M=1, nu=1.0, df=0.0, lam=0.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 2, (n, 1))
    eta = np.sin(3 * x[:, 0])
    if loss == "l2":
        y = eta + rng.normal(0, 0.3, n)
    else:
        y = (rng.random(n) < 1 / (1 + np.exp(-eta))).astype(float)
    return {"x": x, "y": y, "loss": loss, "kind": [0], "n_bins": [nb], "n_levels": [0],
            "df": [df], "lambda": [lam], "nu": nu, "M": M, "variant": "cwb"}


def test_single_step_unpenalised_is_ols():
    pr = _one_learner(M=1, nu=1.0, df=0.0, lam=0.0)
    out = oracle.fit(pr)
    Z = brute.design_pspline(pr["x"][:, 0], pr["x"].min(), pr["x"].max())
    coef, *_ = np.linalg.lstsq(Z, pr["y"], rcond=None)
    np.testing.assert_allclose(out["f"], Z @ coef, atol=1e-9)


@pytest.mark.parametrize("nb", [0, 40])
def test_l2boost_closed_form_single_learner(nb):
    M, nu = 25, 0.3
    pr = _one_learner(M=M, nu=nu, df=4.0, nb=nb)
    out = oracle.fit(pr)
    learners, _ = brute.build(pr, binned=nb > 0)
    Z = learners[0].Z
    lam = learners[0].lam["train"]
    assert abs(lam - out["lambda_train"][0]) < 1e-7 * max(1.0, lam)
    H = Z @ np.linalg.solve(Z.T @ Z + lam * learners[0].D, Z.T)
    y = pr["y"]
    f0 = y.mean()
    n = y.shape[0]
    S = np.linalg.matrix_power(np.eye(n) - nu * H, M)
    f_closed = f0 + (np.eye(n) - S) @ (y - f0)
    np.testing.assert_allclose(out["f"], f_closed, atol=1e-9)


@pytest.mark.parametrize("seed,nbins", [(5, 20), (6, 0), (7, 50)])
def test_l2_training_risk_non_increasing(seed, nbins):
    pr = datagen.tiny_problem(n=600, p=5, seed=seed, n_bins=nbins, M=60, nu=0.5)
    out = oracle.fit(pr)
    rt = out["risk_train"]
    assert (np.diff(rt) <= 1e-12 * rt[0]).all()


@pytest.mark.parametrize("loss,variant", [("l2", "cwb"), ("binomial", "cwb"),
                                          ("l2", "acwb"), ("binomial", "acwb")])
def test_matches_dense_brute_force(loss, variant):
    pr = datagen.tiny_problem(n=300, p=4, seed=21, n_bins=15, M=25, loss=loss,
                              variant=variant, gamma=0.05)
    out = oracle.fit(pr)
    ref = brute.run(pr, binned=True)
    np.testing.assert_array_equal(out["k"], ref["k"])
    if variant == "acwb":
        np.testing.assert_array_equal(out["kcor"], ref["kcor"])
    np.testing.assert_allclose(out["f"], ref["f"], atol=1e-9)
    for m in range(pr["M"]):
        d = ref["theta"][m].shape[0]
        np.testing.assert_allclose(out["theta"][m, :d], ref["theta"][m], atol=1e-8)


def test_unbinned_matches_dense_brute_force():
    pr = datagen.tiny_problem(n=250, p=3, seed=22, n_bins=0, M=15)
    out = oracle.fit(pr)
    ref = brute.run(pr, binned=False)
    np.testing.assert_array_equal(out["k"], ref["k"])
    np.testing.assert_allclose(out["f"], ref["f"], atol=1e-9)


def test_sse_forms_agree():
    """rho^T rho - 2 theta^T v + theta^T G theta equals the direct SSE."""
    pr = datagen.tiny_problem(n=500, p=4, seed=23, n_bins=30, M=1)
    out = oracle.fit(pr)
    learners, _ = brute.build(pr, binned=True)
    y = pr["y"]
    r = y - y.mean()
    k = out["k"][0]
    Z = learners[k].Z
    th = out["theta"][0, :Z.shape[1]]
    v = Z.T @ r
    G = Z.T @ Z
    sse2 = r @ r - 2 * th @ v + th @ G @ th
    assert abs(out["sse"][0] - sse2) < 1e-10 * (r @ r)


def test_lossless_binning_equals_unbinned():
    """Every value on the equal grid => binned CWB is unbinned CWB (Alg 1 identity)."""
    rng = np.random.default_rng(9)
    n, p, nb = 800, 4, 65
    x = rng.integers(0, nb, size=(n, p)).astype(float) / (nb - 1)  # multiples of 1/64
    x[0, :] = 0.0
    x[1, :] = 1.0
    y = np.sin(4 * x[:, 0]) + x[:, 1] ** 2 + rng.normal(0, 0.2, n)
    base = {"x": x, "y": y, "loss": "l2", "kind": np.zeros(p, int), "n_levels": np.zeros(p),
            "df": np.full(p, 5.0), "nu": 0.2, "M": 40, "variant": "cwb"}
    ob = oracle.fit(dict(base, n_bins=np.full(p, nb)))
    ou = oracle.fit(dict(base, n_bins=np.zeros(p, int)))
    np.testing.assert_array_equal(ob["k"], ou["k"])
    np.testing.assert_allclose(ob["lambda_train"], ou["lambda_train"], rtol=1e-9)
    np.testing.assert_allclose(ob["f"], ou["f"], atol=1e-10)
    np.testing.assert_allclose(ob["coef_f"], ou["coef_f"], atol=1e-9)


def test_aggregated_coefficients_reproduce_f():
    """f = f0 + sum_k Z_k theta_hat_k (base-learner additivity, Section 2.3)."""
    for variant in ("cwb", "acwb", "hcwb"):
        pr = datagen.tiny_problem(n=400, p=4, seed=31, n_bins=25, M=30, variant=variant,
                                  gamma=0.05, patience=2)
        out = oracle.fit(pr)
        learners, _ = brute.build(pr, binned=True)
        f = np.full(400, out["f0"])
        off = 0
        for L in learners:
            d = L.Z.shape[1]
            f += L.Z @ out["coef_f"][off:off + d]
            off += d
        np.testing.assert_allclose(out["f"], f, atol=1e-9)


def test_ridge_closed_form():
    """Categorical ridge learner: theta_l = s_l / (n_l + lambda), df = sum n_l/(n_l+lambda)."""
    rng = np.random.default_rng(4)
    n, c = 2000, 7
    codes = rng.integers(0, c, n)
    lev = rng.normal(0, 1, c)
    y = lev[codes] + rng.normal(0, 1, n)
    pr = {"x": codes[:, None].astype(float), "y": y, "loss": "l2", "kind": [1],
          "n_bins": [c], "n_levels": [c], "df": [3.0], "nu": 0.1, "M": 1, "variant": "cwb"}
    out = oracle.fit(pr)
    lam = out["lambda_train"][0]
    cnt = np.bincount(codes, minlength=c)
    assert abs(np.sum(cnt / (cnt + lam)) - 3.0) < 1e-9
    s = np.bincount(codes, weights=y - y.mean(), minlength=c)
    np.testing.assert_allclose(out["theta"][0, :c], s / (cnt + lam), atol=1e-12)


# --- ACWB (Algorithm 2) -----------------------------------------------------

def test_acwb_first_iteration_equals_cwb():
    pr = datagen.tiny_problem(n=500, p=5, seed=41, n_bins=20, M=3)
    o_c = oracle.fit(dict(pr, variant="cwb", M=1))
    o_a = oracle.fit(dict(pr, variant="acwb", gamma=0.2, M=1))
    assert o_a["k"][0] == o_c["k"][0] == o_a["kcor"][0]
    np.testing.assert_allclose(o_a["theta"][0], o_c["theta"][0], atol=1e-13)
    np.testing.assert_allclose(o_a["thetacor"][0], o_a["theta"][0], atol=1e-13)
    np.testing.assert_allclose(o_a["f"], o_c["f"], atol=1e-13)


def test_acwb_momentum_model_from_recurrences():
    """h = f0 + sum_k Z_k theta_h,k with eta_m = gamma nu (m+1)/2 (Section 3.2.1)."""
    pr = datagen.tiny_problem(n=300, p=3, seed=42, n_bins=15, M=12, variant="acwb",
                              gamma=0.1)
    out = oracle.fit(pr)
    learners, _ = brute.build(pr, binned=True)
    h = np.full(300, out["f0"])
    for m in range(1, pr["M"] + 1):
        kc = out["kcor"][m - 1]
        d = learners[kc].Z.shape[1]
        h += pr["gamma"] * pr["nu"] * (m + 1) / 2 * learners[kc].Z @ out["thetacor"][m - 1, :d]
    h2 = np.full(300, out["f0"])
    off = 0
    for L in learners:
        d = L.Z.shape[1]
        h2 += L.Z @ out["coef_h"][off:off + d]
        off += d
    np.testing.assert_allclose(h2, h, atol=1e-9)


# --- HCWB (Algorithm 3) -----------------------------------------------------

def test_hcwb_never_switching_is_acwb_on_train():
    pr = datagen.tiny_problem(n=500, p=4, seed=51, n_bins=20, M=15, variant="hcwb",
                              gamma=0.05)
    oh = oracle.fit(dict(pr, patience=pr["M"]))
    oa = oracle.fit(dict(pr, variant="acwb"))
    assert oh["switch_iter"] == -1
    np.testing.assert_array_equal(oh["k"], oa["k"])
    np.testing.assert_array_equal(oh["kcor"], oa["kcor"])
    np.testing.assert_allclose(oh["f"], oa["f"], atol=1e-13)


def test_hcwb_zero_patience_is_cwb_on_all_rows():
    pr = datagen.tiny_problem(n=400, p=4, seed=52, n_bins=20, M=12, variant="hcwb")
    oh = oracle.fit(dict(pr, patience=0))
    assert oh["switch_iter"] == 1
    train = pr["val_mask"] == 0
    f0 = pr["y"][train].mean()
    ref = brute.run(dict(pr, variant="cwb", val_mask=None), binned=True, f0=f0)
    np.testing.assert_array_equal(oh["k"], ref["k"])
    np.testing.assert_allclose(oh["f"], ref["f"], atol=1e-9)


def test_hcwb_matches_brute_force():
    pr = datagen.tiny_problem(n=400, p=4, seed=53, n_bins=20, M=40, variant="hcwb",
                              gamma=0.5, patience=2, loss="binomial")
    oh = oracle.fit(pr)
    ref = brute.run(pr, binned=True)
    assert oh["switch_iter"] == ref["switch_iter"]
    np.testing.assert_array_equal(oh["k"], ref["k"])
    np.testing.assert_allclose(oh["f"], ref["f"], atol=1e-9)
    np.testing.assert_allclose(oh["risk_val"], ref["risk_val"], atol=1e-12)


def test_hcwb_forced_switch_by_mirrored_validation_labels():
    """Validation targets mirrored around the training mean make the
    validation risk rise at every ACWB step, so the switch comes exactly
    after pat_0 ACWB iterations."""
    rng = np.random.default_rng(54)
    n_half, p = 300, 3
    x1 = rng.uniform(0, 1, (n_half, p))
    y1 = np.sin(5 * x1[:, 0]) + 2 * x1[:, 1] + rng.normal(0, 0.1, n_half)
    x = np.vstack([x1, x1])
    y = np.concatenate([y1, 2 * y1.mean() - y1])
    vm = np.concatenate([np.zeros(n_half), np.ones(n_half)]).astype(np.uint8)
    for pat in (1, 3, 5):
        pr = {"x": x, "y": y, "loss": "l2", "kind": np.zeros(p, int), "n_bins": np.full(p, 30),
              "n_levels": np.zeros(p), "df": np.full(p, 5.0), "nu": 0.1, "M": 12,
              "variant": "hcwb", "gamma": 0.01, "patience": pat, "val_mask": vm}
        out = oracle.fit(pr)
        assert (np.diff(out["risk_val"][:pat + 1]) > 0).all()
        assert out["switch_iter"] == pat + 1
        assert (out["kcor"][pat:] == -1).all() and (out["kcor"][:pat] >= 0).all()


# --- Forcing and determinism ------------------------------------------------

def test_forcing_own_sequence_is_identity_and_gaps_nonnegative():
    pr = datagen.tiny_problem(n=500, p=6, seed=61, n_bins=20, M=30, variant="acwb")
    o1 = oracle.fit(pr)
    o2 = oracle.fit(pr, force_k=o1["k"], force_kcor=o1["kcor"])
    np.testing.assert_array_equal(o2["own_k"], o1["k"])
    assert (o2["gap"] == 0).all() and (o1["gap"] >= 0).all()
    np.testing.assert_array_equal(o2["f"], o1["f"])
    # force a different learner at step 5: gap becomes positive there
    fk = o1["k"].copy()
    fk[5] = (fk[5] + 1) % 6
    o3 = oracle.fit(pr, force_k=fk)
    assert o3["k"][5] == fk[5] and o3["own_k"][5] == o1["k"][5] and o3["gap"][5] > 0


def test_thread_count_does_not_change_results():
    pr = datagen.tiny_problem(n=3000, p=12, seed=62, n_bins=50, M=20, variant="acwb")
    oracle.set_threads(1)
    a = oracle.fit(pr)
    oracle.set_threads(max(2, os.cpu_count() or 2))
    b = oracle.fit(pr)
    np.testing.assert_array_equal(a["k"], b["k"])
    np.testing.assert_array_equal(a["f"], b["f"])
    np.testing.assert_array_equal(a["coef_h"], b["coef_h"])


def test_invalid_inputs_rejected():
    pr = datagen.tiny_problem(n=100, p=2, seed=63, n_bins=10, M=2)
    x = pr["x"].copy()
    x[:, 1] = 0.5
    with pytest.raises(RuntimeError, match="constant"):
        oracle.fit(dict(pr, x=x))
    with pytest.raises(RuntimeError, match="0/1"):
        oracle.fit(dict(pr, loss="binomial"))
    with pytest.raises(RuntimeError, match="validation"):
        oracle.fit(dict(pr, variant="hcwb", val_mask=None))


def test_mixed_numeric_categorical_matches_brute_force():
    pr = datagen.additive_problem(400, 6, seed=71, n_informative=2, loss="binomial",
                                  n_bins=16, M=20, variant="acwb", gamma=0.1, n_normal=2,
                                  n_informative_normal=1, n_cat=2, n_informative_cat=1)
    assert (pr["kind"][-2:] == 1).all()
    out = oracle.fit(pr)
    ref = brute.run(pr, binned=True)
    np.testing.assert_array_equal(out["k"], ref["k"])
    np.testing.assert_array_equal(out["kcor"], ref["kcor"])
    np.testing.assert_allclose(out["f"], ref["f"], atol=1e-9)


def test_config1_scale_run_is_sane():
    pr = datagen.config1(M=60)
    out = oracle.fit(pr)
    rt = out["risk_train"]
    assert (np.diff(rt) <= 0).all()
    # the five informative features are selected first
    assert set(out["k"][:30]) <= set(range(5))
    assert (out["gap"] >= 0).all()


def test_rtr_is_signal_norm():
    """r^T r reported per iteration equals 2 n R_emp(f^[m-1]) for L2."""
    pr = datagen.tiny_problem(n=500, p=3, seed=81, n_bins=20, M=10)
    out = oracle.fit(pr)
    np.testing.assert_allclose(out["rtr"], 2 * 500 * out["risk_train"][:-1], rtol=1e-12)
    assert (out["sse"] <= out["rtr"]).all()


def test_prediction_reproduces_training_fit():
    """The model evaluated at the training rows is the fit's own f when the
    learners see exact values: unbinned splines, lossless binning (every
    value on the equal grid) and categorical levels; values beyond the
    training range are clamped to it."""
    pr = datagen.tiny_problem(n=300, p=3, seed=41, n_bins=0, M=25)
    o = oracle.fit(pr)
    np.testing.assert_allclose(oracle.predict(pr, o, pr["x"]), o["f"], rtol=1e-12, atol=1e-12)
    rng = np.random.default_rng(42)
    nb = 40
    xg = rng.integers(0, nb, size=(500, 2)) / (nb - 1.0)
    xg[0, :], xg[1, :] = 0.0, 1.0
    pb = dict(datagen.tiny_problem(n=500, p=2, seed=43, n_bins=nb, M=20), x=xg)
    ob = oracle.fit(pb)
    np.testing.assert_allclose(oracle.predict(pb, ob, xg), ob["f"], rtol=1e-12, atol=1e-12)
    pc = datagen.additive_problem(400, 2, seed=44, n_informative=0, n_cat=2, n_informative_cat=2,
                                  M=15)
    oc = oracle.fit(pc)
    np.testing.assert_allclose(oracle.predict(pc, oc, pc["x"]), oc["f"], rtol=1e-12, atol=1e-12)
    lo = pr["x"].min(axis=0)
    beyond = np.vstack([lo - 5.0, lo - 0.1])
    np.testing.assert_array_equal(oracle.predict(pr, o, beyond), oracle.predict(pr, o, lo[None, :]).repeat(2))


# --- Binary representation of categorical features (Appendix A.3.2) ---------

@pytest.mark.parametrize("loss,variant,seed", [("l2", "cwb", 81), ("binomial", "acwb", 82),
                                               ("l2", "hcwb", 83), ("binomial", "hcwb", 84)])
def test_binary_categorical_matches_brute_force(loss, variant, seed):
    """One least-squares learner per class, selected among all learners."""
    pr = datagen.additive_problem(400, 5, seed=seed, n_informative=1, loss=loss, n_bins=16,
                                  M=40, variant=variant, gamma=0.5, n_cat=3,
                                  n_informative_cat=3, cat_kind=datagen.BINARY, patience=1)
    out = oracle.fit(pr)
    ref = brute.run(pr, binned=True)
    assert (pr["kind"][-3:] == datagen.BINARY).all()
    assert np.isin(out["k"], [2, 3, 4]).any(), "no binary learner selected"
    np.testing.assert_array_equal(out["k"], ref["k"])
    np.testing.assert_array_equal(out["kcor"], ref["kcor"])
    assert out["switch_iter"] == ref["switch_iter"]
    np.testing.assert_allclose(out["f"], ref["f"], atol=1e-9)
    for m in range(pr["M"]):
        d = ref["theta"][m].shape[0]
        np.testing.assert_allclose(out["theta"][m, :d], ref["theta"][m], atol=1e-9)
        if out["k"][m] >= 2:  # a binary learner moves one class only
            assert np.count_nonzero(out["theta"][m, :d]) <= 1


def test_binary_categorical_selection_order_closed_form():
    """With one categorical feature, L2 and nu = 1, the class learners are
    orthogonal: each step sets the mean residual of the chosen class to zero
    without touching the others, so the classes come in decreasing order of
    s_l^2 / n_l of the initial residual (ties to the lower class), each with
    the class mean as its coefficient, and after one step per class f is the
    vector of class means."""
    rng = np.random.default_rng(85)
    c, n = 7, 700
    codes = rng.integers(0, c, n)
    means = rng.normal(0, 1, c)
    y = means[codes] + rng.normal(0, 0.3, n)
    pr = {"x": codes[:, None].astype(float), "y": y, "loss": "l2", "kind": [2],
          "n_bins": [c], "n_levels": [c], "df": [0.0], "lambda": [0.0], "nu": 1.0, "M": c,
          "variant": "cwb"}
    out = oracle.fit(pr)
    r0 = y - y.mean()
    cnt = np.bincount(codes, minlength=c).astype(float)
    s = np.bincount(codes, weights=r0, minlength=c)
    order = np.argsort(-(s * s / cnt), kind="stable")
    chosen = [int(np.flatnonzero(out["theta"][m, :c])[0]) for m in range(c)]
    assert chosen == list(order)
    for m, l in enumerate(order):
        assert abs(out["theta"][m, l] - s[l] / cnt[l]) < 1e-12
    group_mean = np.bincount(codes, weights=y, minlength=c) / cnt
    np.testing.assert_allclose(out["f"], group_mean[codes], atol=1e-12)


def test_binary_categorical_empty_class_never_selected():
    """A level without rows has no least-squares estimate; it is skipped."""
    rng = np.random.default_rng(86)
    n, c = 300, 6
    codes = rng.integers(0, c - 1, n)  # level c-1 never occurs
    x = np.column_stack([rng.random(n), codes.astype(float)])
    y = np.sin(3 * x[:, 0]) + 0.5 * (codes == 2) + rng.normal(0, 0.2, n)
    pr = {"x": x, "y": y, "loss": "l2", "kind": [0, 2], "n_bins": [20, c],
          "n_levels": [0, c], "df": [5.0, 0.0], "lambda": [0.0, 0.0], "nu": 0.3, "M": 30,
          "variant": "cwb"}
    out = oracle.fit(pr)
    ref = brute.run(pr, binned=True)
    np.testing.assert_array_equal(out["k"], ref["k"])
    np.testing.assert_allclose(out["f"], ref["f"], atol=1e-10)
    assert (out["k"] == 1).any()
    assert (out["theta"][out["k"] == 1, c - 1] == 0).all()


# --- Initial constant (Section 2.3: f^[0] minimises the empirical risk) ------

@pytest.mark.parametrize("loss", ["l2", "binomial"])
@pytest.mark.parametrize("masked", [False, True])
def test_initial_constant_is_stationary(loss, masked):
    """f^[0] is the loss-optimal constant over the training rows, so the
    pseudo-residuals at f^[0] sum to zero there (first-order condition, the
    residual being the negative gradient pinned by finite differences above),
    and the risk rises on either side of it."""
    rng = np.random.default_rng(91 if loss == "l2" else 92)
    n = 700
    pr = _one_learner(n=n, seed=93, nb=30, loss=loss, M=1, nu=0.1, df=4.0)
    if loss == "binomial":  # an unbalanced label mix, away from 1/2
        pr["y"] = (rng.random(n) < 0.23).astype(float)
    if masked:
        pr["val_mask"] = (rng.random(n) < 0.3).astype(np.uint8)
        pr["variant"] = "hcwb"
    train = np.ones(n, bool) if not masked else pr["val_mask"] == 0
    out = oracle.fit(pr)
    f0 = out["f0"]
    r = np.array([oracle.pseudo_residual(loss, yi, f0) for yi in pr["y"][train]])
    assert abs(r.sum()) <= 1e-12 * train.sum()

    def risk(c):
        return sum(oracle.loss(loss, yi, c) for yi in pr["y"][train]) / train.sum()

    for step in (1e-3, 1e-1):
        assert risk(f0 - step) > risk(f0) and risk(f0 + step) > risk(f0)
    assert abs(out["risk_train"][0] - risk(f0)) <= 1e-12 * abs(risk(f0))


def test_correction_criterion_recorded():
    """The correction learner's SSE is its own fit's: c = r in the first ACWB
    iteration, so it equals the primary SSE there; it never exceeds c^T c,
    and forcing the oracle's own correction sequence leaves gaps of zero."""
    pr = datagen.tiny_problem(n=600, p=5, seed=95, n_bins=25, M=25, variant="acwb")
    out = oracle.fit(pr)
    assert out["sse_cor"][0] == out["sse"][0] and out["rtr_cor"][0] == out["rtr"][0]
    assert (out["sse_cor"] <= out["rtr_cor"] * (1 + 1e-12)).all()
    assert (out["gapcor"] >= 0).all()
    again = oracle.fit(pr, force_k=out["k"], force_kcor=out["kcor"])
    assert (again["gapcor"] == 0).all()
    np.testing.assert_array_equal(again["sse_cor"], out["sse_cor"])
    cwb = oracle.fit(dict(pr, variant="cwb"))
    assert (cwb["sse_cor"] == 0).all() and (cwb["kcor"] == -1).all()
