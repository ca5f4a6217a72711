"""GPU-vs-oracle comparison used by the GPU parity tests.

The bar: the GPU's selected learner sequence (primary learners, ACWB
correction learners and the HCWB switch iteration) equals the FP64 oracle's
exactly, and predictions f, aggregated coefficients, per-iteration
coefficients and the training-risk trace agree to 1e-4 relative (infinity
norm relative to the oracle's infinity norm).

Any difference in the sequence fails ``compare`` unless the caller passes
``allow_ties=True``.  Then, and only then, a differing iteration may be a
certified near-tie: the oracle is re-run on the GPU's sequence (forced), and
at each differing iteration the oracle's SSE of the GPU's learner may exceed
the best one by at most TIE_REL * |q_best|, where q_best = SSE_best - s^T s
is that fit's own criterion (s = r for the primary learner, s = c for the
correction learner).  TIE_REL = 1e-6 bounds the criterion error of FP32 model
state: the residuals carry a relative rounding error of a few 1e-8 per
element, drifting by a few float ulps over an iteration sequence, and q is a
quadratic form in their bin sums.  A differing HCWB switch is accepted only
if, at the first iteration whose "validation risk rose" decision differs
between the two runs, the oracle's risk change is below 1e-6 relative.  f and
the coefficients are then compared with the forced oracle run.  The number of
accepted ties is returned in the diagnostics.
"""
from __future__ import annotations

import numpy as np

import oracle

TOL = 1e-4
TIE_REL = 1e-6
SWITCH_REL = 1e-6


def rel_err(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den) if a.size else 0.0


def tie_bound(ref: dict, m: int, cor: bool = False) -> float:
    """Near-tie bound at iteration m (0-based) of a forced oracle run: the
    selected learner's SSE minus the gap is the best SSE, and the best
    criterion is that minus the fitted signal's sum of squares."""
    if cor:
        best = ref["sse_cor"][m] - ref["gapcor"][m]
        q_best = best - ref["rtr_cor"][m]
    else:
        best = ref["sse"][m] - ref["gap"][m]
        q_best = best - ref["rtr"][m]
    return TIE_REL * abs(q_best)


def _rises(rv: np.ndarray, upto: int) -> np.ndarray:
    """Patience decisions of HCWB: did the validation risk of f^[m] rise
    against f^[m-1], for m = 1..upto."""
    rv = np.asarray(rv, np.float64)
    return rv[1:upto + 1] > rv[:upto]


def _certify(gpu, prob, ref_free, threads, M, variant):
    """Re-run the oracle on the GPU's sequence and certify every difference
    as a near-tie; returns (forced oracle run, list of ties)."""
    fk = np.asarray(gpu["k"], np.int32)
    fkc = np.asarray(gpu["kcor"], np.int32) if variant != "cwb" else None
    ref = oracle.fit(prob, force_k=fk, force_kcor=fkc,
                     force_switch=gpu["switch_iter"] if variant == "hcwb" else -1,
                     threads=threads)
    ties = []
    for m in np.nonzero(ref["own_k"] != fk)[0]:
        bound = tie_bound(ref, m)
        ties.append(("k", int(m), float(ref["gap"][m]), float(bound)))
        assert ref["gap"][m] <= bound, (
            f"iteration {m + 1}: GPU picked {fk[m]}, oracle {ref['own_k'][m]}, "
            f"SSE gap {ref['gap'][m]:.3e} above the near-tie bound {bound:.3e}")
    if fkc is not None:
        for m in np.nonzero((ref["own_kcor"] != fkc) & (fkc >= 0))[0]:
            bound = tie_bound(ref, m, cor=True)
            ties.append(("kcor", int(m), float(ref["gapcor"][m]), float(bound)))
            assert ref["gapcor"][m] <= bound, (
                f"iteration {m + 1}: GPU correction learner {fkc[m]}, oracle "
                f"{ref['own_kcor'][m]}, gap {ref['gapcor'][m]:.3e} above {bound:.3e}")
    if variant == "hcwb" and ref["own_switch"] != gpu["switch_iter"]:
        sw, own = gpu["switch_iter"], ref["own_switch"]
        last = min(sw if sw > 0 else M + 1, own if own > 0 else M + 1) - 1
        mine = _rises(gpu["risk_val"], last)
        theirs = _rises(ref["risk_val"], last)
        diff = np.nonzero(mine != theirs)[0]
        assert diff.size, f"HCWB switch at {sw} on the GPU, {own} in the oracle, same decisions"
        j = int(diff[0]) + 1  # the deciding iteration
        rv = ref["risk_val"]
        change = abs(rv[j] - rv[j - 1]) / abs(rv[j])
        ties.append(("switch", int(sw), int(own), float(change)))
        assert change < SWITCH_REL, (
            f"HCWB switch at {sw} on the GPU, {own} in the oracle: the decision of iteration "
            f"{j} differs with a relative validation-risk change of {change:.3e}")
    return ref, ties


def compare(gpu: dict, prob: dict, threads: int | None = None, verbose: bool = True,
            allow_ties: bool = False) -> dict:
    """Check a GPU result against the oracle; return diagnostics."""
    M = len(gpu["k"])
    prob = dict(prob, M=M)
    ref = oracle.fit(prob, threads=threads)
    variant = prob.get("variant", "cwb")
    same_k = np.array_equal(ref["k"], gpu["k"])
    same_kc = variant == "cwb" or np.array_equal(ref["kcor"], gpu["kcor"])
    same_sw = variant != "hcwb" or ref["switch_iter"] == gpu["switch_iter"]
    same = same_k and same_kc and same_sw
    ties = []
    if not same:
        if not allow_ties:
            msg = []
            if not same_k:
                m = int(np.nonzero(np.asarray(ref["k"]) != np.asarray(gpu["k"]))[0][0])
                msg.append(f"learner at iteration {m + 1}: GPU {gpu['k'][m]}, oracle {ref['k'][m]} "
                           f"(oracle top-2 SSE gap {ref['gap'][m]:.3e}, criterion bound "
                           f"{tie_bound(ref, m):.3e})")
            if not same_kc:
                m = int(np.nonzero(np.asarray(ref["kcor"]) != np.asarray(gpu["kcor"]))[0][0])
                msg.append(f"correction learner at iteration {m + 1}: GPU {gpu['kcor'][m]}, "
                           f"oracle {ref['kcor'][m]}")
            if not same_sw:
                msg.append(f"HCWB switch: GPU {gpu['switch_iter']}, oracle {ref['switch_iter']}")
            raise AssertionError("selection sequence differs from the oracle: " + "; ".join(msg))
        ref, ties = _certify(gpu, prob, ref, threads, M, variant)
    e_f = rel_err(gpu["f"], ref["f"])
    e_cf = rel_err(gpu["coef_f"], ref["coef_f"])
    e_ch = rel_err(gpu["coef_h"], ref["coef_h"]) if variant != "cwb" else 0.0
    dm = gpu["theta"].shape[1]
    e_th = rel_err(gpu["theta"], ref["theta"][:, :dm])
    e_rt = rel_err(gpu["risk_train"], ref["risk_train"])
    diag = {"same_sequence": same, "ties": len(ties), "tie_list": ties, "err_f": e_f,
            "err_coef_f": e_cf, "err_coef_h": e_ch, "err_theta": e_th, "err_risk": e_rt, "M": M}
    if variant == "hcwb":
        diag["switch_iter"] = int(gpu["switch_iter"])
    if verbose:
        print("parity:", {k: v for k, v in diag.items() if k != "tie_list"}, flush=True)
    assert e_f <= TOL, f"f error {e_f:.3e}"
    assert e_cf <= TOL, f"coef_f error {e_cf:.3e}"
    assert e_ch <= TOL, f"coef_h error {e_ch:.3e}"
    assert e_th <= TOL, f"theta error {e_th:.3e}"
    assert e_rt <= TOL, f"risk error {e_rt:.3e}"
    return diag
