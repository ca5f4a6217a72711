"""Seeded synthetic inputs shaped like the paper's workloads.

This module generates data only: feature matrices, targets, validation
masks and learner specifications.  It holds none of the boosting method's
arithmetic and is the one module that both the HIP library's callers and the
CPU oracle's tests use, so the two always see identical inputs.

The recipe stands in for the paper's simulation study (Section 4.1.1: smooth
additive effects of uniform features plus noise features, Gaussian noise
scaled by a signal-to-noise ratio) and for its real-data tasks (binary
targets, numeric and categorical columns, Section 4.2 / Appendix B.2), whose
datasets are not used.  All draws use NumPy's PCG64 with fixed seeds.

Effects on [0, 1] (each centred to sample mean 0):
  s1 = sin(2 pi u), s2 = u^2, s3 = exp(u), s4 = tanh(4 (u - 1/2)), s5 = cos(3 pi u).
Informative numeric feature j (0-based) contributes a_j * s_{j mod 5}(u) with
a_j = 1 + j/19, where u = x for uniform columns and u = Phi(x) for normal
columns.  L2 targets add N(0, Var(eta)/SNR^2) noise; binomial targets draw
Bernoulli(sigmoid(eta / sd(eta))).
"""
from __future__ import annotations

import math

import numpy as np

PSPLINE, RIDGE, BINARY = 0, 1, 2

# Defaults the paper fixes for the simulation and benchmarks (Section 4):
# cubic P-splines with 20 knots, df = 5, patience 5; gamma recommendations
# 0.0034 (ACWB) and 0.037 (HCWB) from the H3 results.
GAMMA_ACWB = 0.0034
GAMMA_HCWB = 0.037


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _raw_effect(idx: int, u: np.ndarray) -> np.ndarray:
    e = idx % 5
    if e == 0:
        v = np.sin(2.0 * math.pi * u)
    elif e == 1:
        v = u * u
    elif e == 2:
        v = np.exp(u)
    elif e == 3:
        v = np.tanh(4.0 * (u - 0.5))
    else:
        v = np.cos(3.0 * math.pi * u)
    return v


def _effect(idx: int, u: np.ndarray) -> np.ndarray:
    v = _raw_effect(idx, u)
    return v - v.mean()


def true_effect(prob: dict, j: int, x: np.ndarray) -> np.ndarray:
    """The generating effect of numeric column j at values x, on the scale of
    the model (the logit for binomial targets), centred like the generator
    (by its mean over the sample rows); zero for a noise column."""
    x = np.asarray(x, dtype=np.float64)
    t = prob.get("truth", {}).get("numeric", {}).get(j)
    if t is None:
        return np.zeros_like(x)
    idx, amp, transform, center = t
    u = _norm_cdf(x) if transform == "norm_cdf" else x
    return prob["truth"]["scale"] * amp * (_raw_effect(idx, u) - center)


def _norm_cdf(x: np.ndarray) -> np.ndarray:
    from scipy.special import ndtr
    return ndtr(x)


def learner_specs(p: int, n_bins, df: float = 5.0, kinds=None, n_levels=None) -> dict:
    kinds = np.zeros(p, np.int32) if kinds is None else np.asarray(kinds, np.int32)
    n_levels = np.zeros(p, np.int32) if n_levels is None else np.asarray(n_levels, np.int32)
    cat = kinds != PSPLINE
    nb = np.where(cat, n_levels, np.broadcast_to(np.asarray(n_bins), (p,)))
    dfs = np.where(kinds == RIDGE, np.minimum(df, n_levels.astype(np.float64)),
                   np.where(kinds == BINARY, 0.0, df))
    return {
        "kind": kinds, "n_bins": nb.astype(np.int32), "n_levels": n_levels,
        "df": dfs.astype(np.float64), "lambda": np.zeros(p),
        "degree": 3, "n_knots": 20, "pen_order": 2,
    }


def additive_problem(n: int, p: int, *, seed: int, n_informative: int, loss: str = "l2",
                     n_bins=None, M: int = 100, nu: float = 0.1, variant: str = "cwb",
                     gamma: float | None = None, patience: int = 5, val_frac: float = 0.0,
                     snr: float = 1.0, amp_one: bool = False, n_normal: int = 0,
                     n_informative_normal: int = 0, n_cat: int = 0,
                     n_informative_cat: int = 0, df: float = 5.0,
                     cat_kind: int | None = None) -> dict:
    """Numeric columns (uniform, then normal) followed by categorical codes.

    Columns [0, p_num - n_normal) are Uniform[0, 1], the next n_normal are
    N(0, 1), the last n_cat are level codes 0..c_j-1 with c_j ~ U{5..20}.
    The first n_informative uniform columns, the first n_informative_normal
    normal columns and the first n_informative_cat categorical columns carry
    signal.  Categorical columns get ridge learners, or the learners of
    ``cat_kind`` (BINARY: one least-squares learner per class).
    """
    rng = _rng(seed)
    p_num = p - n_cat
    n_unif = p_num - n_normal
    x = np.empty((n, p), dtype=np.float64, order="F")
    eta = np.zeros(n)
    truth = {}
    for j in range(n_unif):
        x[:, j] = rng.random(n)
        if j < n_informative:
            a = 1.0 if amp_one else 1.0 + j / 19.0
            eta += a * _effect(j, x[:, j])
            truth[j] = (j, a, "id", float(_raw_effect(j, x[:, j]).mean()))
    for jj in range(n_normal):
        j = n_unif + jj
        x[:, j] = rng.standard_normal(n)
        if jj < n_informative_normal:
            a = 1.0 + (n_informative + jj) / 19.0
            u = _norm_cdf(x[:, j])
            eta += a * _effect(n_informative + jj, u)
            truth[j] = (n_informative + jj, a, "norm_cdf", float(_raw_effect(n_informative + jj, u).mean()))
    kinds = np.zeros(p, np.int32)
    n_levels = np.zeros(p, np.int32)
    for jj in range(n_cat):
        j = p_num + jj
        c = int(rng.integers(5, 21))
        codes = rng.integers(0, c, size=n)
        x[:, j] = codes
        kinds[j] = RIDGE if cat_kind is None else cat_kind
        n_levels[j] = c
        if jj < n_informative_cat:
            lev = rng.normal(0.0, 0.5, size=c)
            eta += lev[codes] - lev[codes].mean()
    scale = 1.0
    if loss == "l2":
        sd = math.sqrt(max(eta.var(), 1e-300)) / snr
        y = eta + rng.normal(0.0, sd, size=n)
    elif loss == "binomial":
        s = eta.std()
        z = eta / s if s > 0 else eta
        scale = 1.0 / s if s > 0 else 1.0
        prob = 1.0 / (1.0 + np.exp(-z))
        y = (rng.random(n) < prob).astype(np.float64)
    else:
        raise ValueError(loss)
    val_mask = None
    if val_frac > 0.0 or variant == "hcwb":
        frac = val_frac if val_frac > 0.0 else 0.2
        val_mask = (rng.random(n) < frac).astype(np.uint8)
    if n_bins is None:
        n_bins = int(math.floor(math.sqrt(n)))
    if gamma is None:
        gamma = GAMMA_HCWB if variant == "hcwb" else GAMMA_ACWB
    prob = {"x": x, "y": y, "loss": loss, "nu": nu, "M": M, "variant": variant,
            "gamma": gamma, "patience": patience, "val_mask": val_mask,
            "truth": {"scale": scale, "numeric": truth}}
    prob.update(learner_specs(p, n_bins, df=df, kinds=kinds, n_levels=n_levels))
    return prob


def config1(seed: int = 1, M: int = 500) -> dict:
    """Plain CWB, L2: n = 10,000, p = 10 uniform, 5 informative, 100 bins."""
    return additive_problem(10_000, 10, seed=seed, n_informative=5, n_bins=100, M=M,
                            amp_one=True)


def config2(n: int = 1_000_000, p: int = 200, seed: int = 2, M: int = 2000,
            n_bins: int = 1000) -> dict:
    """Headline: plain CWB, L2, n = 1e6, p = 200 (20 informative), 1,000 bins."""
    return additive_problem(n, p, seed=seed, n_informative=min(20, p), n_bins=n_bins, M=M)


def config3(variant: str = "acwb", n: int = 2_000_000, seed: int = 3, M: int = 3000,
            n_num: int = 150, n_cat: int = 10, n_bins: int = 1000) -> dict:
    """ACWB / HCWB, binomial: 75 uniform + 75 normal (15 informative) numeric
    columns and 10 categorical ridge columns (first 3 informative)."""
    n_normal = n_num // 2
    return additive_problem(n, n_num + n_cat, seed=seed, n_informative=8, loss="binomial",
                            n_bins=n_bins, M=M, variant=variant, n_normal=n_normal,
                            n_informative_normal=7, n_cat=n_cat, n_informative_cat=3,
                            val_frac=0.2 if variant == "hcwb" else 0.0)


def config4_specs(count: int = 64, seed0: int = 1000, M: int = 1000,
                  n_range=(5e4, 5e5), p_range=(20, 100)) -> list[dict]:
    """Sizes and settings of the batched-fit workload (no data yet)."""
    out = []
    for i in range(count):
        rng = _rng(seed0 + i)
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        out.append({"seed": seed0 + i, "n": n, "p": p,
                    "loss": "l2" if i % 2 == 0 else "binomial",
                    "variant": "cwb" if i % 4 in (0, 1) else "acwb", "M": M})
    return out


def config4_problem(spec: dict) -> dict:
    return additive_problem(spec["n"], spec["p"], seed=spec["seed"],
                            n_informative=min(5, spec["p"]), loss=spec["loss"],
                            M=spec["M"], variant=spec["variant"])


def config5_stream(count: int = 400, rate: float = 20.0, seed: int = 5000,
                   n_range=(1e4, 2e6), p_range=(10, 300), M_range=(200, 2000)) -> list[dict]:
    """Poisson arrival stream of fit requests (sizes and settings only)."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        r = _rng(seed + 1 + i)
        n = int(round(math.exp(r.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        p = int(round(math.exp(r.uniform(math.log(p_range[0]), math.log(p_range[1])))))
        variant = ("cwb", "acwb", "hcwb")[int(r.integers(0, 3))]
        M = int(r.integers(M_range[0], M_range[1] + 1))
        out.append({"arrival": t, "seed": seed + 1 + i, "n": n, "p": p, "variant": variant,
                    "loss": "l2" if i % 2 == 0 else "binomial", "M": M})
    return out


def config5_problem(spec: dict) -> dict:
    return additive_problem(spec["n"], spec["p"], seed=spec["seed"],
                            n_informative=min(5, spec["p"]), loss=spec["loss"], M=spec["M"],
                            variant=spec["variant"],
                            val_frac=0.2 if spec["variant"] == "hcwb" else 0.0)


class FeaturePool:
    """One column-major Uniform[0, 1] matrix shared by a request stream: a
    request of n rows and p features uses its leading n x p block, a view
    with column stride n_max that the library reads without a copy."""

    def __init__(self, n_max: int, p_max: int, seed: int = 4999):
        rng = _rng(seed)
        self.x = np.empty((n_max, p_max), dtype=np.float64, order="F")
        for j in range(p_max):
            self.x[:, j] = rng.random(n_max)


def config5_problem_pooled(spec: dict, pool: FeaturePool) -> dict:
    """A served request on the pool's leading block: the first min(5, p)
    columns carry the additive signal, targets and validation split are
    drawn from the request's own seed."""
    n, p = spec["n"], spec["p"]
    x = pool.x[:n, :p]
    rng = _rng(spec["seed"])
    eta = np.zeros(n)
    for j in range(min(5, p)):
        eta += (1.0 + j / 19.0) * _effect(j, x[:, j])
    if spec["loss"] == "l2":
        y = eta + rng.normal(0.0, math.sqrt(max(eta.var(), 1e-300)), size=n)
    else:
        s = eta.std()
        z = eta / s if s > 0 else eta
        y = (rng.random(n) < 1.0 / (1.0 + np.exp(-z))).astype(np.float64)
    variant = spec["variant"]
    val_mask = (rng.random(n) < 0.2).astype(np.uint8) if variant == "hcwb" else None
    prob = {"x": x, "y": y, "loss": spec["loss"], "nu": 0.1, "M": spec["M"], "variant": variant,
            "gamma": GAMMA_HCWB if variant == "hcwb" else GAMMA_ACWB, "patience": 5,
            "val_mask": val_mask}
    prob.update(learner_specs(p, int(math.floor(math.sqrt(n)))))
    return prob


def tiny_problem(n: int = 400, p: int = 4, seed: int = 7, n_bins: int = 20, M: int = 20,
                 loss: str = "l2", variant: str = "cwb", **kw) -> dict:
    """Small problem for brute-force checks."""
    return additive_problem(n, p, seed=seed, n_informative=min(3, p), loss=loss,
                            n_bins=n_bins, M=M, variant=variant, **kw)
