"""Benchmark: binned CWB iterations per second at n = 1e6, p = 200 on one MI355X.

One step = one full boosting iteration of the hot path (row pass, histogram
pass over the uint16 bin-index matrix, per-learner FP64 solves and the
selection) on the headline workload: plain CWB, L2 loss, n = 1,000,000 rows,
p = 200 Uniform[0,1] features (20 informative), 1,000 bins, cubic P-splines
with 24 bases, df = 5, nu = 0.1.  Inputs are synthetic (seed 2) and resident
in HBM before timing starts.  Prints one JSON line.

Extra legs (on by default, each a few seconds): the FP64 CPU oracle timed on
the first iterations of the same input (cpu_baseline, and the selection
parity of those iterations), batched fits (many heterogeneous fits per
launch) against a plain loop of the same single fits, and the fit server
under a Poisson request stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("CWB iters/sec at n=1e6,p=200 (HBM GB/s %peak); batched/served fits/s + p99")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hist_c2_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) of the histogram pass's sources: the
    kernel file, the device helpers it includes and the data layout."""
    import hashlib
    h = hashlib.sha256()
    for name in ("hist.hip", "device_common.h", "cwb_internal.h"):
        with open(os.path.join(ROOT, "paper_2110_03513_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def index_read(tile: dict) -> str:
    """How the histogram pass reads the bin indices, from the tile report."""
    bits = tile.get("index_bits", 16)
    return f" (read as a {bits}-bit packed copy)" if bits in (10, 12) else ""


def measured_traffic(tile: dict):
    """HBM bytes per hist launch from the committed rocprofv3 counter summary
    (one entry per profiled tile shape), or None if it is missing, was taken
    on a different kernel source or on no tile shape this run uses."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_source_hash():
        return None
    for entry in t.get("tiles", []):
        want = entry.get("tile", {})
        if all(want.get(k) == tile.get(k) for k in ("threads", "learners", "blocks")):
            return entry.get("hbm_bytes_per_launch")
    return None


def headline(args, torch, cwb, datagen):
    n, p, nb = args.n, args.p, 1000
    log(f"[bench] generating C2 input n={n} p={p}")
    # the workload's fit has M = 2,000 iterations; the timed window is inside
    # it, and the rest runs after it for the selection-parity check
    M = max(args.fit_iters, args.warmup + args.steps + args.profile_iters)
    prob = datagen.config2(n=n, p=p, M=M, n_bins=nb)
    t0 = time.perf_counter()
    fit = cwb.Fit(prob)
    setup_s = time.perf_counter() - t0
    tile = fit.tile()
    log(f"[bench] setup {setup_s:.2f}s (tile {tile}); warmup {args.warmup} iterations")
    fit.run(args.warmup)
    fit.sync()
    # timed region: exactly `steps` iterations, HIP events around every
    # `timing_period`-th histogram-pass launch on the fit's stream
    fit.set_timing(1, args.timing_period)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit.run(args.steps)
    fit.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hist_ms, hist_n = fit.kernel_time("hist")
    # after the timed region: per-kernel durations of the other two kernels
    st_us = sel_us = None
    if args.profile_iters > 0:
        fit.set_timing(6)
        fit.run(args.profile_iters)
        fit.sync()
        ms, cnt = fit.kernel_time("state")
        st_us = ms / max(cnt, 1) * 1e3
        ms, cnt = fit.kernel_time("select")
        sel_us = ms / max(cnt, 1) * 1e3
    fit.set_timing(0)
    left = M - fit.iters_done
    if left > 0:  # the rest of the fit, untimed, for the parity check
        fit.run(left)
        fit.sync()
    tr = fit.trace()
    tr.update(fit.model())
    tr["f"] = fit.pred()
    fit.close()
    per_iter = wall / args.steps
    iters_s = 1.0 / per_iter
    alg_iter_bytes = 2.0 * n * p + 14.0 * n
    hist_bytes = 2.0 * n * p + 4.0 * n
    hist_avg_s = hist_ms / 1e3 / max(hist_n, 1)
    achieved = hist_bytes / hist_avg_s / 1e9
    traffic = measured_traffic(tile)
    return prob, tr, {
        "iters_s": iters_s, "ms_per_step": per_iter * 1e3, "setup_s": setup_s,
        "iter_gbs": alg_iter_bytes * iters_s / 1e9,
        "hist_avg_us": hist_avg_s * 1e6, "state_avg_us": st_us, "select_avg_us": sel_us,
        "hist_launches": hist_n, "hist_timed_every": args.timing_period,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # measured bytes (the packed index copy moves fewer than the
                     # uint16 formulation's algorithmic bytes) over the same time
                     "traffic_gbs": (round(traffic / hist_avg_s / 1e9, 1)
                                     if traffic else None)},
        "alg_iter_bytes": alg_iter_bytes, "hist_bytes_per_launch": hist_bytes, "tile": tile,
    }


def setup_leg(prob, cwb):
    """Fit creation of the headline problem with binning and bin counts on
    host threads and on the GPU, the latter with the learners' Gram, lambda
    and inverse solves on the GPU too (device_s) or on host threads
    (device_host_solves_s); the tile autotuner is off for all three, so that
    only the setup differs; best of two creations each."""
    saved = {k: os.environ.get(k) for k in ("CWB_AUTOTUNE", "CWB_DEVICE_SOLVES")}
    os.environ["CWB_AUTOTUNE"] = "0"
    out = {}
    try:
        for name, setup, solves in (("host", "host", "1"), ("device", "device", "1"),
                                    ("device_host_solves", "device", "0")):
            os.environ["CWB_DEVICE_SOLVES"] = solves
            best = None
            for _ in range(2):
                t0 = time.perf_counter()
                f = cwb.Fit(dict(prob, setup=setup))
                dt = time.perf_counter() - t0
                f.close()
                best = dt if best is None else min(best, dt)
            out[f"{name}_s"] = round(best, 4)
            log(f"[bench] setup {name}: {best:.3f}s")
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    out["speedup"] = round(out["host_s"] / max(out["device_s"], 1e-9), 2)
    out["host_threads"] = os.cpu_count()
    return out


def cv_leg(args, torch, cwb, datagen):
    """Five-fold cross-validation (n = 1e6, p = 50, 1,000 bins, CWB, L2):
    the folds sharing one index matrix and one histogram pass, against the
    same five folds as separate fits (each with its fold as validation
    mask) in one batch.  Iterations per second of all folds together."""
    n, p, K, iters = args.n, 50, 5, args.cv_iters
    prob = datagen.config2(n=n, p=p, M=iters + 10, n_bins=1000)
    rng = np.random.default_rng(7)
    fold = (np.arange(n) % K).astype(np.int32)
    rng.shuffle(fold)
    log(f"[bench] cv: {K} folds, n={n} p={p}, {iters} iterations")
    out = {"folds": K, "n": n, "p": p, "iterations": iters}
    cv = cwb.CV(prob, fold)
    cv.run(5)
    cv.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cv.run(iters)
    cv.sync()
    out["shared_pass_iters_s"] = round(iters / (time.perf_counter() - t0), 2)
    out["cv_risk_last"] = float(cv.risk()[-1])
    out["shared_tile"] = cv.tile()
    cv.close()
    del cv
    fits = [cwb.Fit(dict(prob, val_mask=(fold == k).astype(np.uint8))) for k in range(K)]
    b = cwb.Batch(fits)
    b.run(5)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(iters)
    b.sync()
    out["separate_fits_iters_s"] = round(iters / (time.perf_counter() - t0), 2)
    out["separate_tile"] = b.tile()
    b.close()
    for f in fits:
        f.close()
    out["speedup"] = round(out["shared_pass_iters_s"] / max(out["separate_fits_iters_s"], 1e-9), 3)
    log(f"[bench] cv {out}")
    return out


def mise_leg(cwb, datagen):
    """Partial-effect quality (the MISE of the simulation study) on the
    small additive workload (n = 10,000, p = 10, five informative effects,
    L2, SNR 1), 500 iterations, from the GPU's partial effects."""
    from paper_2110_03513_amd import evaluate
    out = {}
    cases = [("cwb_sqrt_n_bins", dict(variant="cwb", n_bins=100)),
             ("cwb_fourth_root_bins", dict(variant="cwb", n_bins=-2)),
             ("cwb_unbinned", dict(variant="cwb", n_bins=0)),
             ("acwb", dict(variant="acwb", n_bins=100, gamma=datagen.GAMMA_ACWB)),
             ("hcwb", dict(variant="hcwb", n_bins=100, gamma=datagen.GAMMA_HCWB))]
    for name, kw in cases:
        prob = datagen.additive_problem(10_000, 10, seed=1, n_informative=5, M=500, amp_one=True,
                                        **kw)
        f = cwb.Fit(prob)
        f.run(500)
        f.sync()
        out[name] = round(evaluate.mise(prob, lambda j, v: f.partial_effect(j, v)), 6)
        f.close()
    log(f"[bench] mise {out}")
    return out


def unbinned_leg(args, torch, cwb, datagen):
    """The headline workload with unbinned learners (each row's own cubic
    basis, no binning), timed beside the binned path."""
    n, p, M = args.n, args.p, args.unbinned_iters
    log(f"[bench] unbinned: n={n} p={p}, {M} iterations")
    prob = datagen.config2(n=n, p=p, M=M + 10, n_bins=0)
    t0 = time.perf_counter()
    fit = cwb.Fit(prob)
    setup = time.perf_counter() - t0
    del prob
    tile = fit.tile()
    fit.run(10)
    fit.sync()
    fit.set_timing(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit.run(M)
    fit.sync()
    wall = time.perf_counter() - t0
    hist_ms, hist_n = fit.kernel_time("hist")
    fit.close()
    hist_s = hist_ms / 1e3 / max(hist_n, 1)
    alg = 4.0 * n * p + 4.0 * n  # 32-bit knot-interval code per (row, learner) + residuals
    return {"iters_s": round(M / wall, 2), "hist_avg_us": round(hist_s * 1e6, 2),
            "hist_alg_gbs": round(alg / hist_s / 1e9, 1), "iterations": M, "tile": tile,
            "setup_s": round(setup, 2)}


def momentum_legs(args, torch, cwb, datagen):
    """ACWB and HCWB, binomial, at the full n = 2e6 (150 numeric + 10
    categorical learners): iterations per second and the histogram pass's
    algorithmic bandwidth of each phase, and the oracle on a window of the
    first ACWB iterations."""
    out = {}
    for variant in ("acwb", "hcwb"):
        M = args.momentum_iters
        log(f"[bench] {variant}: n=2e6 p=160, {M} iterations")
        prob = datagen.config3(variant, M=M)
        n, p = prob["x"].shape
        n_train = int(n - (prob["val_mask"].sum() if prob.get("val_mask") is not None else 0))
        fit = cwb.Fit(prob)
        tile = fit.tile()
        fit.run(10)
        fit.sync()
        fit.set_timing(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fit.run(M - 10)
        fit.sync()
        wall = time.perf_counter() - t0
        hist_ms, hist_n = fit.kernel_time("hist")
        tr = fit.trace()
        sw = tr["switch_iter"]
        fit.close()
        rec = {"iters_s": round((M - 10) / wall, 2), "iterations": M, "tile": tile}
        if variant == "acwb":
            two = 2.0 * n * p + 8.0 * n  # both signals from one read of the indices
            avg = hist_ms / 1e3 / max(hist_n, 1)
            rec.update({"hist_avg_us": round(avg * 1e6, 2), "hist_alg_gbs": round(two / avg / 1e9, 1),
                        "hist_frac": round(two / avg / 1e9 / HBM_PEAK_GBS, 4)})
            if not args.no_cpu:
                import oracle
                w = args.momentum_oracle_iters
                log(f"[bench] acwb: oracle, first {w} iterations on {oracle.max_threads()} threads")
                o = oracle.fit(dict(prob, M=w))
                rec["oracle_window"] = {
                    "iterations": w, "iters_s": round(w / o["iter_s"], 3),
                    "cores": oracle.max_threads(), "setup_s": round(o["setup_s"], 2),
                    "k_match": int(np.sum(tr["k"][:w] == o["k"])),
                    "kcor_match": int(np.sum(tr["kcor"][:w] == o["kcor"]))}
                del o
        else:
            rec["switch_iter"] = sw
            if sw > 11:  # each phase timed on a fresh fit of the same input
                fit = cwb.Fit(prob)
                phases = {}
                for name, iters, rows, sig in (("acwb_phase", sw - 1, n_train, 2),
                                               ("cwb_phase", M - sw + 1, n, 1)):
                    fit.set_timing(1)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    fit.run(iters)
                    fit.sync()
                    dt = time.perf_counter() - t0
                    ms, cnt = fit.kernel_time("hist")
                    avg = ms / 1e3 / max(cnt, 1)
                    byt = 2.0 * rows * p + 4.0 * sig * rows
                    phases[name] = {"iterations": iters, "iters_s": round(iters / dt, 2),
                                    "hist_avg_us": round(avg * 1e6, 2),
                                    "hist_alg_gbs": round(byt / avg / 1e9, 1),
                                    "hist_frac": round(byt / avg / 1e9 / HBM_PEAK_GBS, 4),
                                    "rows": rows, "signals": sig}
                assert fit.trace()["switch_iter"] == sw
                fit.close()
                rec["phases"] = phases
        del prob
        out[variant] = rec
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_err(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300)) if a.size else 0.0


def parity_summary(gpu, ref, keys=("k",)) -> dict:
    """Selection sequences (exact) and f, coefficients, per-iteration theta
    and risk trace (relative to the oracle's infinity norm) of a GPU fit
    against the oracle's fit of the same input."""
    m = min(len(gpu["k"]), len(ref["k"]))
    eq = np.ones(m, bool)
    for key in keys:
        eq &= np.asarray(gpu[key][:m]) == np.asarray(ref[key][:m])
    first = int(np.argmin(eq)) if not eq.all() else -1
    out = {"iterations_compared": m, "k_match": int(np.sum(eq)), "first_mismatch": first,
           "oracle_gap_at_mismatch": float(ref["gap"][first]) if first >= 0 else None}
    if "f" in gpu and m == len(ref["k"]):
        dm = gpu["theta"].shape[1]
        out.update({"err_f": rel_err(gpu["f"], ref["f"]),
                    "err_coef_f": rel_err(gpu["coef_f"], ref["coef_f"]),
                    "err_theta": rel_err(gpu["theta"][:m], ref["theta"][:m, :dm]),
                    "err_risk": rel_err(gpu["risk_train"][:m + 1], ref["risk_train"][:m + 1])})
        out["within_1e-4"] = bool(first < 0 and max(out["err_f"], out["err_coef_f"],
                                                    out["err_theta"], out["err_risk"]) <= 1e-4)
    return out


def cpu_baseline(args, prob, gpu):
    """The FP64 oracle on the same input: the whole fit (all M iterations) on
    every host core, timed without its setup and compared with the GPU's fit,
    then a short window on one thread."""
    import oracle
    cores = oracle.max_threads()
    M = int(prob["M"])
    log(f"[bench] CPU oracle: the whole {M}-iteration fit on {cores} threads")
    o = oracle.fit(prob)
    par = parity_summary(gpu, o)
    log(f"[bench] parity {par}")
    cb = {"value": round(M / o["iter_s"], 4), "unit": "iters/s", "cores": cores, "kind": "oracle",
          "sample": (f"FP64 C oracle, all {M} iterations of the same n={prob['x'].shape[0]} "
                     f"p={prob['x'].shape[1]} fit ({o['iter_s']:.1f}s; setup excluded, "
                     f"{o['setup_s']:.1f}s)"),
          "cpu_model": cpu_model()}
    del o
    one = None
    k1 = args.cpu_iters_1thread
    if k1 > 0:
        log(f"[bench] CPU oracle: {k1} iterations on one thread")
        oracle.set_threads(1)
        try:
            o1 = oracle.fit(dict(prob, M=k1))
        finally:
            oracle.set_threads(cores)
        one = {"value": round(k1 / o1["iter_s"], 4), "unit": "iters/s", "cores": 1,
               "kind": "oracle",
               "sample": (f"FP64 C oracle on one thread, iterations 1..{k1} of the same input "
                          f"({o1['iter_s']:.1f}s; setup excluded, {o1['setup_s']:.1f}s)"),
               "cpu_model": cpu_model()}
    return cb, par, one


def config1_leg(torch, cwb, datagen):
    """The small parity workload (n = 10,000, p = 10, 100 bins, M = 500): the
    GPU's whole fit (launch-latency bound, not on the roofline) against the
    oracle's whole fit on one thread."""
    import oracle
    prob = datagen.config1(M=500)
    log("[bench] config1: n=10000 p=10, 500 iterations")
    fit = cwb.Fit(prob)
    fit.run(10)
    fit.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit.run(490)
    fit.sync()
    wall = time.perf_counter() - t0
    gpu = fit.trace()
    gpu.update(fit.model())
    gpu["f"] = fit.pred()
    fit.close()
    cores = oracle.max_threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        o = oracle.fit(prob)
        whole = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    return {"iters_s": round(490 / wall, 1), "ms_per_iter": round(wall / 490 * 1e3, 4),
            "oracle_1thread": {"iters_s": round(500 / o["iter_s"], 1),
                               "whole_fit_s": round(whole, 3), "setup_s": round(o["setup_s"], 3)},
            "parity": parity_summary(gpu, o)}


def batched(args, torch, cwb, datagen):
    specs = datagen.config4_specs(count=args.batch_fits, M=args.batch_iters)
    log(f"[bench] batched: {len(specs)} fits, M={args.batch_iters}")
    probs = [datagen.config4_problem(s) for s in specs]
    stream = torch.cuda.Stream()
    t_batch = {}
    hist = None
    for graphs in ("1", "0"):
        os.environ["CWB_GRAPH"] = graphs
        t0 = time.perf_counter()
        fits = [cwb.Fit(p) for p in probs]
        setup = time.perf_counter() - t0
        b = cwb.Batch(fits, stream=stream)
        tile = b.tile()
        if graphs == "0":  # eager launches: time the batched histogram pass
            fits[0].set_timing(1, args.timing_period)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(args.batch_iters)
        b.sync()
        t_batch[graphs] = time.perf_counter() - t0
        if graphs == "0":
            hist = fits[0].kernel_time("hist")
            fits[0].set_timing(0)
        ks = [f.trace()["k"] for f in fits]
        b.close()
        for f in fits:
            f.close()
    os.environ.pop("CWB_GRAPH")
    # the same fits one after another, each alone
    t_loop, same = None, None
    if not args.batch_no_loop:
        fits = [cwb.Fit(p) for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in fits:
            f.run(args.batch_iters)
        for f in fits:
            f.sync()
        t_loop = time.perf_counter() - t0
        same = all(np.array_equal(f.trace()["k"], k) for f, k in zip(fits, ks))
        for f in fits:
            f.close()
    bytes_iter = sum(2.0 * p["x"].shape[0] * p["x"].shape[1] for p in probs)
    # algorithmic bytes of one batched histogram launch (every fit runs all
    # M iterations): each fit's indices once, and its signals (two for ACWB)
    hist_bytes = sum(2.0 * p["x"].shape[0] * p["x"].shape[1] +
                     4.0 * p["x"].shape[0] * (2 if p["variant"] == "acwb" else 1) for p in probs)
    hist_avg = hist[0] / 1e3 / max(hist[1], 1)
    achieved = hist_bytes / hist_avg / 1e9
    tb = t_batch["1"]
    return {"fits": len(probs), "iters": args.batch_iters,
            "fits_per_s": round(len(probs) / tb, 3),
            "fits_per_s_without_graphs": round(len(probs) / t_batch["0"], 3),
            "loop_fits_per_s": round(len(probs) / t_loop, 3) if t_loop else None,
            "speedup_vs_loop": round(t_loop / tb, 3) if t_loop else None,
            "index_gbs": round(bytes_iter * args.batch_iters / tb / 1e9, 1),
            "roofline": {"bound": "hbm", "kernel": "batched histogram pass",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "hist_avg_us": round(hist_avg * 1e6, 2), "launches_timed": hist[1],
                         "bytes_per_launch": hist_bytes},
            "tile": tile,
            "same_selections_as_alone": None if same is None else bool(same),
            "setup_s": round(setup, 2)}


def served(args, torch, cwb, datagen):
    """Poisson request stream through the fit server (each request binned,
    counted and solved on the GPU during its upload), the same stream with
    the setup on host threads, then the stream served one fit at a time
    (max_slots = 1) on the same GPU."""
    from concurrent.futures import ThreadPoolExecutor
    specs = datagen.config5_stream(count=args.serve_requests)
    n_max = max(s["n"] for s in specs)
    p_max = max(s["p"] for s in specs)
    log(f"[bench] served: {len(specs)} requests, feature pool {n_max} x {p_max}")
    pool = datagen.FeaturePool(n_max, p_max)
    # requests whose results are also computed alone (the smallest few)
    sample = sorted(range(len(specs)), key=lambda i: specs[i]["n"] * specs[i]["p"] * specs[i]["M"])[:8]
    index_bytes = sum(2.0 * s["n"] * s["p"] * s["M"] for s in specs)

    def one_stream(max_slots, setup="auto"):
        srv = cwb.Server(arena_bytes=int(args.serve_arena_gb * (1 << 30)), max_slots=max_slots,
                         quantum=args.serve_quantum)
        ex = ThreadPoolExecutor(max_workers=4)
        futs = {}
        ahead = 8
        for i in range(min(ahead, len(specs))):
            futs[i] = ex.submit(datagen.config5_problem_pooled, specs[i], pool)
        tickets = []
        lateness = []
        t0 = time.perf_counter()
        for i, s in enumerate(specs):
            prob = futs.pop(i).result()
            prob["setup"] = setup
            if i + ahead < len(specs):
                futs[i + ahead] = ex.submit(datagen.config5_problem_pooled, specs[i + ahead], pool)
            wait = t0 + s["arrival"] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(prob))
            lateness.append(time.perf_counter() - (t0 + s["arrival"]))
            del prob
        ex.shutdown()
        results = {}
        pending = set(range(len(tickets)))
        last = time.perf_counter()
        while pending:
            for i in list(pending):
                r = srv.poll(tickets[i])
                if r is not None:
                    pending.discard(i)
                    results[i] = r if i in sample else {"status": r["status"], "latency_s": r["latency_s"]}
                    last = time.perf_counter()
            if time.perf_counter() - last > 300:
                raise RuntimeError("served stream made no progress for 300 s")
            time.sleep(0.005)
        st = srv.stats()
        srv.close()
        # latency from the scheduled arrival (submit lateness included)
        lat = np.sort([lateness[i] + results[i]["latency_s"] for i in range(len(tickets))])
        st["arrival_p50_s"] = float(np.percentile(lat, 50))
        st["arrival_p99_s"] = float(np.percentile(lat, 99))
        st["late_submit_s"] = float(max(lateness))
        st["wall_s"] = time.perf_counter() - t0
        st["failed"] = sum(1 for r in results.values() if r["status"] != 0)
        return st, results

    log("[bench] served: continuous batching (setup on the GPU during upload)")
    st, res = one_stream(args.serve_slots)
    st1 = sth = None
    if not args.serve_batched_only:
        log("[bench] served: continuous batching, setup on host threads")
        sth, _ = one_stream(args.serve_slots, "host")
        log("[bench] served: one fit at a time")
        st1, _ = one_stream(1)
    # alone vs in the mix
    bitwise = 0
    worst = 0.0
    for i in sample:
        a = cwb.fit(datagen.config5_problem_pooled(specs[i], pool))
        r = res[i]
        same = np.array_equal(a["k"], r["k"]) and np.array_equal(a["f"], r["f"])
        bitwise += int(same)
        den = max(float(np.max(np.abs(a["f"]))), 1e-30)
        worst = max(worst, float(np.max(np.abs(a["f"] - r["f"]))) / den)
    span = max(s["arrival"] for s in specs)

    def summary(x):
        return {"fits_per_s": round(x["fits_per_s"], 3), "p50_latency_s": round(x["arrival_p50_s"], 4),
                "p99_latency_s": round(x["arrival_p99_s"], 4),
                "p50_from_submit_s": round(x["p50_latency_s"], 4),
                "p99_from_submit_s": round(x["p99_latency_s"], 4),
                "mean_setup_s": round(x["mean_setup_s"], 4), "mean_queue_s": round(x["mean_queue_s"], 4),
                "rounds": x["rounds"], "round_time_share": round(x["round_s"] / max(x["busy_s"], 1e-9), 3),
                "completed": x["completed"],
                "rejected": x["rejected"], "failed": x["failed"],
                "arena_peak_gb": round(x["arena_peak"] / 2**30, 3), "wall_s": round(x["wall_s"], 2),
                "late_submit_s": round(x["late_submit_s"], 3)}

    return {"requests": len(specs), "rate_per_s": 20.0, "arrival_span_s": round(span, 2),
            "max_slots": args.serve_slots, "quantum": args.serve_quantum,
            "arena_gb": args.serve_arena_gb,
            "continuous_batching": summary(st),
            "continuous_host_setup": summary(sth) if sth else None,
            "one_at_a_time": summary(st1) if st1 else None,
            "speedup_fits_per_s": (round(st["fits_per_s"] / max(st1["fits_per_s"], 1e-12), 3)
                                   if st1 else None),
            "index_gbs": round(index_bytes / max(st["wall_s"], 1e-9) / 1e9, 1),
            "alone_vs_mix": {"requests": len(sample), "bitwise_equal": bitwise,
                             "max_rel_err_f": worst}}


def copy_probe(torch, mib):
    """A plain streaming copy of known size (reads and writes `mib` MiB per
    launch), profiled beside the histogram pass so that the HBM byte counters
    can be scaled by what they read for a known amount of traffic."""
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "launches": 5}), flush=True)


def lds_probe(torch, cwb, args):
    """The LDS histogram ceiling: the histogram pass's inner loop (1,024
    threads, 4 learners per group, 8 rows per index load, the headline's 2e8
    atomics over 256 blocks) with its bin indices read from a 512 KiB table
    in L2 instead of HBM, for 4-byte words (the pass's 32-bit groups) and
    8-byte words (int64 groups).  Random bins (uniform over 1,000) and
    bank-conflict-free bins (lane l of a wave always on its own bank, or
    bank pair for 8-byte words)."""
    nb, learners, blocks = 1000, 4, 256
    atomics = float(args.n) * args.p  # one per (row, learner)
    steps = int(round(atomics / (blocks * 1024 * learners * 8)))
    chunks = 1 << 15
    rng = np.random.default_rng(77)
    rand = rng.integers(0, nb, size=chunks * 8, dtype=np.int64)
    lane = np.arange(chunks) % 64
    free8 = (32 * rng.integers(0, nb // 32, size=(chunks, 8)) + (lane % 32)[:, None]).reshape(-1)
    free4 = (64 * rng.integers(0, nb // 64, size=(chunks, 8)) + lane[:, None]).reshape(-1)
    out = {"atomics": blocks * 1024 * learners * 8 * steps, "blocks": blocks, "nb": nb}
    for wb, free in ((4, free4), (8, free8)):
        for name, tab in (("random", rand), ("conflict_free", free)):
            idx = torch.from_numpy(tab.astype(np.int16)).cuda()
            acc = torch.zeros(blocks, dtype=torch.int64, device="cuda")
            for _ in range(3):
                cwb.probe_lds_hist(idx, nb, learners, steps, blocks, acc, word_bytes=wb)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record()
            for _ in range(reps):
                cwb.probe_lds_hist(idx, nb, learners, steps, blocks, acc, word_bytes=wb)
            e1.record()
            torch.cuda.synchronize()
            out[f"{name}_{wb}b_us"] = round(e0.elapsed_time(e1) * 1e3 / reps, 2)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=200)
    ap.add_argument("--fit-iters", type=int, default=2000,
                    help="iterations of the headline fit (the timed window lies inside it; "
                         "the whole fit is compared with the oracle)")
    ap.add_argument("--cpu-iters-1thread", type=int, default=20,
                    help="time the oracle on one thread over this many iterations (0: skip)")
    ap.add_argument("--momentum-oracle-iters", type=int, default=20)
    ap.add_argument("--no-config1", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-mise", action="store_true", help="skip the partial-effect MISE leg")
    ap.add_argument("--no-lds-probe", action="store_true",
                    help="skip the LDS histogram ceiling probe")
    ap.add_argument("--no-cv", action="store_true", help="skip the cross-validation leg")
    ap.add_argument("--cv-iters", type=int, default=200)
    ap.add_argument("--no-setup", action="store_true",
                    help="skip timing fit creation with host vs device binning")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--batch-fits", type=int, default=64)
    ap.add_argument("--batch-iters", type=int, default=1000)
    ap.add_argument("--batch-no-loop", action="store_true",
                    help="skip the plain loop of single fits (profiling runs)")
    ap.add_argument("--timing-period", type=int, default=8,
                    help="time every k-th histogram launch in the timed region")
    ap.add_argument("--unbinned-iters", type=int, default=200)
    ap.add_argument("--no-unbinned", action="store_true")
    ap.add_argument("--momentum-iters", type=int, default=300)
    ap.add_argument("--no-momentum", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-quantum", type=int, default=50)
    ap.add_argument("--serve-batched-only", action="store_true",
                    help="skip serving the stream one fit at a time")
    ap.add_argument("--serve-arena-gb", type=float, default=64.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain streaming copy of this many MiB (counter calibration)")
    ap.add_argument("--tile", default="",
                    help="threads,lds_kib,blocks_per_cu: force one histogram tile shape "
                         "instead of autotuning (used for counter runs)")
    args = ap.parse_args()
    if args.tile:
        nt, kb, bpc = (int(v) for v in args.tile.split(","))
        os.environ.update({"CWB_HIST_NT": str(nt), "CWB_HIST_LDS_KB": str(kb),
                           "CWB_HIST_BPC": str(bpc)})
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus above 1 is not "
                                   "supported (sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)
        return
    from paper_2110_03513_amd import cwb, datagen
    cwb.lib()
    prob, tr, h = headline(args, torch, cwb, datagen)
    out = {
        "metric": METRIC, "value": round(h["iters_s"], 2), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(h["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": (f"binned CWB, L2, n={args.n}, p={args.p}, 1000 bins, cubic "
                                "P-splines d=24 df=5, nu=0.1 (synthetic, seed 2)"),
                   "n": args.n, "p": args.p, "n_bins": 1000, "variant": "cwb", "loss": "l2",
                   "iterations_in_fit": int(prob["M"])},
        "precision": (f"uint16 bin indices{index_read(h['tile'])}; exact fixed-point "
                      "histograms in 32-bit LDS words (int64 where a bin's count needs it); "
                      "fp32 model state; int64 merge; fp64 solves and selection"),
        "hbm_gbs": round(h["iter_gbs"], 1),
        "hbm_frac": round(h["iter_gbs"] / HBM_PEAK_GBS, 4),
        "roofline": h["roofline"],
        "kernels_us": {"hist": round(h["hist_avg_us"], 2),
                       "state": h["state_avg_us"] and round(h["state_avg_us"], 2),
                       "select": h["select_avg_us"] and round(h["select_avg_us"], 2)},
        "setup_s": round(h["setup_s"], 2),
        "hist_tile": h["tile"],
        "hist_timing": {"launches_timed": h["hist_launches"], "every": args.timing_period,
                        "method": "HIP events on the fit's stream around every k-th histogram "
                                  "launch of the timed region"},
    }
    if not args.no_lds_probe:
        lp = lds_probe(torch, cwb, args)
        # the histogram pass against the LDS ceiling of its own atomics: the
        # headline's groups take 4-byte words
        lp["hist_us"] = round(h["hist_avg_us"], 2)
        lp["ceiling_frac"] = round(lp["random_4b_us"] / h["hist_avg_us"], 4)
        out["lds_ceiling"] = lp
    if not args.no_setup:
        out["setup"] = setup_leg(prob, cwb)
    if not args.no_mise:
        out["mise"] = mise_leg(cwb, datagen)
    if not args.no_cv:
        out["cv"] = cv_leg(args, torch, cwb, datagen)
    if not args.no_cpu:
        cb, par, one = cpu_baseline(args, prob, tr)
        out["cpu_baseline"] = cb
        if one:
            out["cpu_baseline_1thread"] = one
        out["parity"] = par
    del prob
    if not args.no_config1 and not args.no_cpu:
        out["config1"] = config1_leg(torch, cwb, datagen)
    if not args.no_unbinned:
        out["unbinned"] = unbinned_leg(args, torch, cwb, datagen)
    if not args.no_momentum:
        out["momentum"] = momentum_legs(args, torch, cwb, datagen)
    if not args.no_batch:
        out["batched"] = batched(args, torch, cwb, datagen)
    if not args.no_serve:
        out["served"] = served(args, torch, cwb, datagen)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
