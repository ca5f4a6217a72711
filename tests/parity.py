"""GPU-vs-oracle comparison used by the GPU parity tests.

The bar: the GPU's selected learner sequence equals the FP64 oracle's, and
predictions f, aggregated coefficients and per-iteration coefficients agree
to 1e-4 relative (infinity norm relative to the oracle's infinity norm).

Where the sequences differ, each differing iteration must be a certified
near-tie: running the oracle on the GPU's sequence (forced), the oracle's
SSE of the GPU's learner may exceed its own best by at most
    TIE_REL * |q_best| + TIE_ABS * r^T r,   q_best = SSE_best - r^T r,
the error band of a criterion evaluated from FP32 model state (the FP32
state drifts from the FP64 one by a few float ulps per iteration).  f and
the coefficients are then compared with the forced oracle run.
"""
from __future__ import annotations

import numpy as np

import oracle

TOL = 1e-4
TIE_REL = 2e-5
TIE_ABS = 1e-9


def rel_err(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den) if a.size else 0.0


def _tie_bound(ref, m, cor=False):
    sse = ref["sse"][m] if not cor else None
    if cor:
        # the forced correction fit's SSE is not stored; bound by c^T c scale
        return TIE_ABS * ref["rtr_cor"][m] + TIE_REL * ref["rtr_cor"][m]
    gap = ref["gap"][m]
    best = sse - gap
    q_best = abs(best - ref["rtr"][m])
    return TIE_REL * q_best + TIE_ABS * ref["rtr"][m]


def compare(gpu: dict, prob: dict, threads: int | None = None, verbose: bool = True) -> dict:
    """Check a GPU result against the oracle; return diagnostics."""
    M = len(gpu["k"])
    prob = dict(prob, M=M)
    ref = oracle.fit(prob, threads=threads)
    variant = prob.get("variant", "cwb")
    same = (np.array_equal(ref["k"], gpu["k"]) and
            (variant == "cwb" or np.array_equal(ref["kcor"], gpu["kcor"])) and
            (variant != "hcwb" or ref["switch_iter"] == gpu["switch_iter"]))
    ties = []
    if not same:
        fk = np.asarray(gpu["k"], np.int32)
        fkc = np.asarray(gpu["kcor"], np.int32) if variant != "cwb" else None
        ref = oracle.fit(prob, force_k=fk, force_kcor=fkc,
                         force_switch=gpu["switch_iter"] if variant == "hcwb" else -1,
                         threads=threads)
        for m in np.nonzero(ref["own_k"] != fk)[0]:
            bound = _tie_bound(ref, m)
            ties.append(("k", int(m), float(ref["gap"][m]), float(bound)))
            assert ref["gap"][m] <= bound, (
                f"iteration {m + 1}: GPU picked {fk[m]}, oracle {ref['own_k'][m]}, "
                f"SSE gap {ref['gap'][m]:.3e} above near-tie bound {bound:.3e}")
        if fkc is not None:
            for m in np.nonzero((ref["own_kcor"] != fkc) & (fkc >= 0))[0]:
                bound = _tie_bound(ref, m, cor=True)
                ties.append(("kcor", int(m), float(ref["gapcor"][m]), float(bound)))
                assert ref["gapcor"][m] <= bound, (
                    f"iteration {m + 1}: GPU correction learner {fkc[m]}, oracle "
                    f"{ref['own_kcor'][m]}, gap {ref['gapcor'][m]:.3e} > {bound:.3e}")
        if variant == "hcwb" and ref["own_switch"] != gpu["switch_iter"]:
            sw = gpu["switch_iter"]
            own = ref["own_switch"]
            m0 = min(sw if sw > 0 else M + 1, own if own > 0 else M + 1) - 1
            rv = ref["risk_val"]
            # the decisions that differ must rest on validation-risk changes
            # at rounding level
            lo, hi = max(1, m0 - prob.get("patience", 5)), min(M, m0 + 1)
            d = np.abs(np.diff(rv[lo - 1:hi + 1])) / np.abs(rv[lo:hi + 1])
            ties.append(("switch", int(sw), int(own), float(d.min()) if d.size else 0.0))
            assert d.size and d.min() < 1e-6, (
                f"HCWB switch at {sw} on the GPU, {own} in the oracle, "
                f"smallest relative validation-risk change {d.min():.3e}")
    e_f = rel_err(gpu["f"], ref["f"])
    e_cf = rel_err(gpu["coef_f"], ref["coef_f"])
    e_ch = rel_err(gpu["coef_h"], ref["coef_h"]) if variant != "cwb" else 0.0
    dm = gpu["theta"].shape[1]
    e_th = rel_err(gpu["theta"], ref["theta"][:, :dm])
    e_rt = rel_err(gpu["risk_train"], ref["risk_train"])
    diag = {"same_sequence": same, "ties": ties, "err_f": e_f, "err_coef_f": e_cf,
            "err_coef_h": e_ch, "err_theta": e_th, "err_risk": e_rt, "M": M}
    if verbose:
        print("parity:", {k: (v if k != "ties" else len(v)) for k, v in diag.items()}, flush=True)
    assert e_f <= TOL, f"f error {e_f:.3e}"
    assert e_cf <= TOL, f"coef_f error {e_cf:.3e}"
    assert e_ch <= TOL, f"coef_h error {e_ch:.3e}"
    assert e_th <= TOL, f"theta error {e_th:.3e}"
    assert e_rt <= TOL, f"risk error {e_rt:.3e}"
    if variant == "hcwb" and same:
        assert ref["switch_iter"] == gpu["switch_iter"]
    return diag
