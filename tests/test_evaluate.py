"""CPU: the MISE evaluation (Sec. 4.1) against closed forms, and the
oracle's partial effects against its prediction."""
import numpy as np

import oracle
from paper_2110_03513_amd import datagen, evaluate


def test_simpson_is_exact_for_cubics():
    xs = np.linspace(-1.0, 2.0, 11)
    f = 3 * xs ** 3 - xs ** 2 + 2 * xs - 5
    exact = (3 / 4) * (2 ** 4 - 1) - (1 / 3) * (8 + 1) + (4 - 1) - 5 * 3
    assert abs(evaluate.simpson(f, -1.0, 2.0) - exact) < 1e-12


def test_integrated_squared_error_closed_forms():
    rng = np.random.default_rng(1)
    s = rng.uniform(0.2, 1.7, 5000)
    lo, hi, m = s.min(), s.max(), s.mean()
    truth = np.sin
    # a constant offset is removed by the centring
    assert evaluate.integrated_squared_error(lambda v: np.sin(v) + 3.0, truth, s) < 1e-24
    # a linear error x - c: after centring the difference is x - mean(x),
    # whose square integrates to ((hi - m)^3 - (lo - m)^3) / 3
    got = evaluate.integrated_squared_error(lambda v: np.sin(v) + 2.0 * v - 7.0, truth, s)
    want = 4.0 * ((hi - m) ** 3 - (lo - m) ** 3) / 3.0
    assert abs(got - want) < 1e-9 * want


def test_true_effect_matches_the_generator():
    """The recorded truth reproduces the signal the targets were drawn from:
    with SNR -> infinity the L2 targets are f(x) = sum of the effects."""
    prob = datagen.additive_problem(4000, 6, seed=3, n_informative=3, n_normal=2,
                                    n_informative_normal=1, snr=1e12)
    x = prob["x"]
    eta = sum(datagen.true_effect(prob, j, x[:, j]) for j in range(6))
    np.testing.assert_allclose(prob["y"], eta, atol=1e-9)
    assert (datagen.true_effect(prob, 5, x[:, 5]) == 0).all()


def test_mise_of_the_true_model_is_zero_and_oracle_fit_improves():
    prob = datagen.additive_problem(3000, 6, seed=4, n_informative=4, n_bins=60, M=300, nu=0.3)
    zero = evaluate.mise(prob, lambda j, v: datagen.true_effect(prob, j, v) + 0.25 * j)
    assert zero < 1e-24
    early = oracle.fit(dict(prob, M=10))
    late = oracle.fit(prob)
    m_early = evaluate.mise(prob, lambda j, v: oracle.partial_effect(prob, early, j, v))
    m_late = evaluate.mise(prob, lambda j, v: oracle.partial_effect(prob, late, j, v))
    assert m_late < 0.5 * m_early


def test_oracle_partial_effects_sum_to_prediction():
    prob = datagen.additive_problem(2000, 5, seed=5, n_informative=2, n_bins=40, M=40,
                                    n_cat=2, n_informative_cat=1)
    res = oracle.fit(prob)
    rng = np.random.default_rng(6)
    xn = rng.uniform(0, 1, (500, 5))
    for j in (3, 4):
        xn[:, j] = rng.integers(0, prob["n_levels"][j], 500)
    total = res["f0"] + sum(oracle.partial_effect(prob, res, j, xn[:, j]) for j in range(5))
    np.testing.assert_allclose(total, oracle.predict(prob, res, xn), rtol=1e-12, atol=1e-12)
