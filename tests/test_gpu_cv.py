"""GPU: K-fold cross-validation with the folds sharing one histogram pass.

Each fold is checked against the oracle's fit of the same problem with the
fold as its validation mask (selection sequence, f, coefficients, training
and validation risks), and the cross-validated risk against the oracle's
fold risks weighted by fold size.
"""
import numpy as np
import pytest

import oracle
from paper_2110_03513_amd import cwb, datagen
from tests.parity import compare, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _folds(n, K, seed):
    rng = np.random.default_rng(seed)
    fold = np.arange(n) % K
    rng.shuffle(fold)
    return fold.astype(np.int32)


def _fold_result(f):
    out = f.trace()
    out.update(f.model())
    out["f"] = f.pred()
    return out


@pytest.mark.parametrize("variant,loss,K", [("cwb", "l2", 5), ("acwb", "binomial", 3),
                                            ("cwb", "binomial", 8)])
def test_cv_folds_against_oracle(variant, loss, K):
    prob = datagen.additive_problem(40_000, 9, seed=111, n_informative=4, loss=loss, n_bins=120,
                                    M=80, variant=variant, gamma=0.05, n_cat=2,
                                    n_informative_cat=1)
    fold = _folds(40_000, K, 112)
    _say(f"cv: K={K} variant={variant} loss={loss} n=40000 p=9 M=80")
    cv = cwb.CV(prob, fold)
    cv.run(80)
    cv.sync()
    weighted = np.zeros(81)
    for k in range(K):
        mask = (fold == k).astype(np.uint8)
        pk = dict(prob, val_mask=mask)
        res = _fold_result(cv.folds[k])
        compare(res, pk)
        o = oracle.fit(pk)
        assert rel_err(res["risk_val"], o["risk_val"]) <= 1e-4
        weighted += o["risk_val"] * mask.sum() / mask.size
    assert rel_err(cv.risk(), weighted) <= 1e-4
    cv.close()


def test_cv_resumes_and_predicts():
    """Runs in parts, and fold fits predict at new rows like any fit."""
    prob = datagen.additive_problem(20_000, 6, seed=113, n_informative=3, n_bins=64, M=60)
    fold = _folds(20_000, 4, 114)
    a = cwb.CV(prob, fold)
    a.run(60)
    a.sync()
    b = cwb.CV(prob, fold)
    for part in (7, 33, 20):
        b.run(part)
    b.sync()
    for k in range(4):
        np.testing.assert_array_equal(a.folds[k].trace()["k"], b.folds[k].trace()["k"])
        np.testing.assert_array_equal(a.folds[k].pred(), b.folds[k].pred())
    np.testing.assert_array_equal(a.risk(), b.risk())
    # the folds' shared groups take 32-bit words (every fold's learners)
    assert a.tile()["learners32"] == 4 * 6
    xn = np.random.default_rng(115).uniform(0, 1, (1000, 6))
    o = oracle.fit(dict(prob, val_mask=(fold == 2).astype(np.uint8)))
    assert rel_err(a.folds[2].predict(xn), oracle.predict(prob, o, xn)) <= 1e-4
    a.close()
    b.close()


def test_cv_uneven_folds_ragged_rows_and_categorical_learners():
    """A one-row fold, very uneven folds, a ragged row count, and ridge and
    binary categorical learners beside P-splines, in ACWB with eight folds."""
    n = 10_001
    prob = datagen.additive_problem(n, 7, seed=116, n_informative=2, loss="binomial",
                                    n_bins=50, M=40, variant="acwb", gamma=0.1, n_cat=2,
                                    n_informative_cat=2)
    prob["kind"][-1] = datagen.BINARY
    prob["df"][-1] = 0.0
    rng = np.random.default_rng(117)
    fold = rng.integers(1, 8, n).astype(np.int32)
    fold[5_000] = 0  # fold 0 holds out a single row
    fold[fold == 7] = rng.integers(5, 7, int((fold == 7).sum()))  # and fold 7 keeps few
    fold[:3] = 7
    K = 8
    assert np.bincount(fold, minlength=K).min() >= 1
    _say(f"cv: K={K} fold sizes {np.bincount(fold, minlength=K).tolist()}")
    cv = cwb.CV(prob, fold)
    cv.run(40)
    cv.sync()
    for k in range(K):
        pk = dict(prob, val_mask=(fold == k).astype(np.uint8))
        res = _fold_result(cv.folds[k])
        compare(res, pk)
    cv.close()
