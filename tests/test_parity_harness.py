"""The GPU parity harness itself, on the CPU: with an oracle run standing in
for a GPU result, identical sequences pass with no accepted ties, and a
planted selection mismatch (made by forcing the oracle) fails, whether or
not near-ties are allowed, because its criterion gap is far above the
near-tie bound."""
import numpy as np
import pytest

import oracle
from paper_2110_03513_amd import datagen
from tests.parity import compare, tie_bound


def _as_gpu(o):
    return {k: o[k] for k in ("k", "kcor", "switch_iter", "f", "coef_f", "coef_h", "theta",
                              "risk_train", "risk_val")}


@pytest.mark.parametrize("variant", ["cwb", "acwb"])
def test_identical_sequence_passes_without_ties(variant):
    pr = datagen.tiny_problem(n=800, p=6, seed=101, n_bins=30, M=25, variant=variant)
    d = compare(_as_gpu(oracle.fit(pr)), pr, verbose=False)
    assert d["same_sequence"] and d["ties"] == 0
    assert d["err_f"] == 0.0


@pytest.mark.parametrize("allow", [False, True])
def test_planted_mismatch_fails(allow):
    pr = datagen.tiny_problem(n=800, p=6, seed=102, n_bins=30, M=25, variant="cwb")
    own = oracle.fit(pr)
    fk = own["k"].copy()
    m = 7
    fk[m] = (fk[m] + 1) % 6
    planted = oracle.fit(pr, force_k=fk)
    assert planted["gap"][m] > tie_bound(planted, m)
    with pytest.raises(AssertionError):
        compare(_as_gpu(planted), pr, verbose=False, allow_ties=allow)


def test_planted_correction_mismatch_fails():
    pr = datagen.tiny_problem(n=800, p=6, seed=103, n_bins=30, M=25, variant="acwb")
    own = oracle.fit(pr)
    fkc = own["kcor"].copy()
    m = 9
    fkc[m] = (fkc[m] + 1) % 6
    planted = oracle.fit(pr, force_k=own["k"], force_kcor=fkc)
    assert planted["gapcor"][m] > tie_bound(planted, m, cor=True)
    with pytest.raises(AssertionError, match="correction"):
        compare(_as_gpu(planted), pr, verbose=False)
    with pytest.raises(AssertionError):
        compare(_as_gpu(planted), pr, verbose=False, allow_ties=True)
