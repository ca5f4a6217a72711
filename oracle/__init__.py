"""FP64 CPU oracle for binned / unbinned CWB, ACWB and HCWB.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, independent CPU
implementation of the method of arXiv 2110.03513 (Schalk, Bischl, Ruegamer):
componentwise boosting (Algorithm A1 of the appendix), binMatVec / binMatMat
on binned features (Algorithm 1, Section 3.1), Nesterov-accelerated CWB
(Algorithm 2, Section 3.2) and hybrid CWB (Algorithm 3, Section 3.2.3).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library.

The numeric work is in ``cwb_oracle.c`` (C, FP64), called through ctypes.
``build()`` compiles it with gcc.

Problem dictionaries (also accepted by the GPU binding) hold:
  x (n, p) float64, y (n,) float64, loss "l2"|"binomial",
  kind (p,) 0 = P-spline / 1 = ridge categorical / 2 = binary categorical
  (one least-squares learner per class), n_bins (p,), n_levels (p,),
  df (p,), lambda (p,), degree, n_knots, pen_order, nu, gamma, M,
  variant "cwb"|"acwb"|"hcwb", patience, val_mask (n,) uint8 or None.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cwb_oracle.c")
_LIB = os.path.join(_HERE, "libcwb_oracle.so")

LOSSES = {"l2": 0, "binomial": 1}
VARIANTS = {"cwb": 0, "acwb": 1, "hcwb": 2}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP over learners, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", _SRC, "-o", _LIB, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        lib.orc_last_error.restype = C.c_char_p
        lib.orc_nearest.restype = C.c_int
        lib.orc_knots.restype = C.c_int
        lib.orc_df.restype = C.c_int
        lib.orc_lambda_for_df.restype = C.c_int
        lib.orc_loss.restype = C.c_double
        lib.orc_loss.argtypes = [C.c_int, C.c_double, C.c_double]
        lib.orc_pseudo_residual.restype = C.c_double
        lib.orc_pseudo_residual.argtypes = [C.c_int, C.c_double, C.c_double]
        lib.orc_fit.restype = C.c_int
        lib.orc_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


class _Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("p", C.c_int32),
        ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
        ("val_mask", C.POINTER(C.c_uint8)),
        ("loss", C.c_int32),
        ("kind", C.POINTER(C.c_int32)), ("n_bins", C.POINTER(C.c_int32)),
        ("n_levels", C.POINTER(C.c_int32)),
        ("df", C.POINTER(C.c_double)), ("lam", C.POINTER(C.c_double)),
        ("degree", C.c_int32), ("n_knots", C.c_int32), ("pen_order", C.c_int32),
        ("nu", C.c_double), ("gamma", C.c_double),
        ("M", C.c_int32), ("variant", C.c_int32), ("patience", C.c_int32),
        ("force_k", C.POINTER(C.c_int32)), ("force_kcor", C.POINTER(C.c_int32)),
        ("force_switch", C.c_int32),
    ]


class _Result(C.Structure):
    _fields_ = [(name, C.POINTER(t)) for name, t in [
        ("d", C.c_int32), ("lambda_train", C.c_double), ("lambda_all", C.c_double),
        ("f0", C.c_double), ("k", C.c_int32), ("theta", C.c_double), ("sse", C.c_double),
        ("own_k", C.c_int32), ("gap", C.c_double), ("kcor", C.c_int32),
        ("thetacor", C.c_double), ("own_kcor", C.c_int32), ("gapcor", C.c_double),
        ("risk_train", C.c_double), ("risk_val", C.c_double),
        ("switch_iter", C.c_int32), ("own_switch", C.c_int32), ("f", C.c_double),
        ("coef_f", C.c_double), ("coef_h", C.c_double), ("rtr", C.c_double),
        ("rtr_cor", C.c_double), ("sse_cor", C.c_double), ("seconds", C.c_double)]]


def _arr(a, dtype, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if n is not None and a.shape[0] != n:
        raise ValueError("bad length")
    return a


def sizes(problem: dict) -> tuple[int, int]:
    kind = np.asarray(problem["kind"])
    d = np.where(kind != 0, np.asarray(problem["n_levels"]),
                 problem.get("n_knots", 20) + problem.get("degree", 3) + 1)
    return int(d.max()), int(d.sum())


def fit(problem: dict, force_k=None, force_kcor=None, force_switch: int = -1,
        threads: int | None = None) -> dict:
    """Run CWB / ACWB / HCWB in FP64 and return traces and the final model.

    ``force_k`` / ``force_kcor`` make the oracle follow a given selection
    sequence while still recording its own argmin (``own_k``) and the SSE gap
    between the forced and the best learner (``gap``); ``force_switch`` fixes
    the first CWB iteration of HCWB.
    """
    lib = _load()
    if threads is not None:
        lib.orc_set_threads(int(threads))
    x = np.asarray(problem["x"], dtype=np.float64)
    n, p = x.shape
    xc = np.asfortranarray(x)  # column-major: feature j contiguous
    y = _arr(problem["y"], np.float64, n)
    vm = problem.get("val_mask")
    vm = None if vm is None else _arr(vm, np.uint8, n)
    kind = _arr(problem["kind"], np.int32, p)
    nb = _arr(problem["n_bins"], np.int32, p)
    nl = _arr(problem.get("n_levels", np.zeros(p)), np.int32, p)
    df = _arr(problem["df"], np.float64, p)
    lam = _arr(problem.get("lambda", np.zeros(p)), np.float64, p)
    M = int(problem["M"])
    fk = None if force_k is None else _arr(force_k, np.int32, M)
    fkc = None if force_kcor is None else _arr(force_kcor, np.int32, M)
    pr = _Problem(
        n=n, p=p, x=_p(xc.reshape(-1, order="F"), C.c_double), y=_p(y, C.c_double),
        val_mask=_p(vm, C.c_uint8), loss=LOSSES[problem["loss"]],
        kind=_p(kind, C.c_int32), n_bins=_p(nb, C.c_int32), n_levels=_p(nl, C.c_int32),
        df=_p(df, C.c_double), lam=_p(lam, C.c_double),
        degree=int(problem.get("degree", 3)), n_knots=int(problem.get("n_knots", 20)),
        pen_order=int(problem.get("pen_order", 2)),
        nu=float(problem["nu"]), gamma=float(problem.get("gamma", 0.0)), M=M,
        variant=VARIANTS[problem.get("variant", "cwb")],
        patience=int(problem.get("patience", 5)),
        force_k=_p(fk, C.c_int32), force_kcor=_p(fkc, C.c_int32),
        force_switch=int(force_switch))
    d_max, sum_d = sizes(problem)
    out = {
        "d": np.zeros(p, np.int32), "lambda_train": np.zeros(p), "lambda_all": np.zeros(p),
        "f0": np.zeros(1), "k": np.zeros(M, np.int32), "theta": np.zeros((M, d_max)),
        "sse": np.zeros(M), "own_k": np.zeros(M, np.int32), "gap": np.zeros(M),
        "kcor": np.zeros(M, np.int32), "thetacor": np.zeros((M, d_max)),
        "own_kcor": np.zeros(M, np.int32), "gapcor": np.zeros(M),
        "risk_train": np.zeros(M + 1), "risk_val": np.zeros(M + 1),
        "switch_iter": np.zeros(1, np.int32), "own_switch": np.zeros(1, np.int32),
        "f": np.zeros(n), "coef_f": np.zeros(sum_d), "coef_h": np.zeros(sum_d),
        "rtr": np.zeros(M), "rtr_cor": np.zeros(M), "sse_cor": np.zeros(M),
        "seconds": np.zeros(2),
    }
    res = _Result(**{name: _p(out[name], t._type_) for name, t in _Result._fields_})
    rc = lib.orc_fit(C.byref(pr), C.byref(res))
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}: {lib.orc_last_error().decode()}")
    out["f0"] = float(out["f0"][0])
    out["switch_iter"] = int(out["switch_iter"][0])
    out["own_switch"] = int(out["own_switch"][0])
    out["setup_s"], out["iter_s"] = (float(v) for v in out.pop("seconds"))
    return out


# --- building blocks, exposed for the pins ---------------------------------

def grid(xmin: float, xmax: float, nb: int) -> np.ndarray:
    z = np.zeros(nb)
    _load().orc_grid(C.c_double(xmin), C.c_double(xmax), C.c_int(nb), _p(z, C.c_double))
    return z


def bin_feature(x, nb: int):
    x = _arr(x, np.float64)
    z = np.zeros(nb)
    ind = np.zeros(x.shape[0], np.int32)
    _load().orc_bin_feature(_p(x, C.c_double), C.c_int64(x.shape[0]), C.c_int(nb),
                            _p(z, C.c_double), _p(ind, C.c_int32))
    return z, ind


def knots(xmin: float, xmax: float, n_int: int = 20, degree: int = 3) -> np.ndarray:
    t = np.zeros(n_int + 2 + 2 * degree)
    _load().orc_knots(C.c_double(xmin), C.c_double(xmax), C.c_int(n_int), C.c_int(degree),
                      _p(t, C.c_double))
    return t


def bspline(x, t, degree: int = 3) -> np.ndarray:
    """Basis matrix (len(x), len(t) - degree - 1) by the Cox-de Boor recursion."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = _arr(t, np.float64)
    d = t.shape[0] - degree - 1
    out = np.zeros((x.shape[0], d))
    row = np.zeros(d)
    lib = _load()
    for i, xi in enumerate(x):
        lib.orc_bspline(C.c_double(xi), _p(t, C.c_double), C.c_int(t.shape[0]),
                        C.c_int(degree), _p(row, C.c_double))
        out[i] = row
    return out


def penalty(d: int, order: int = 2) -> np.ndarray:
    D = np.zeros((d, d))
    _load().orc_penalty(C.c_int(d), C.c_int(order), _p(D, C.c_double))
    return D


def df_of_lambda(G, D, lam: float) -> float:
    G = _arr(G, np.float64)
    D = _arr(D, np.float64)
    v = C.c_double()
    rc = _load().orc_df(C.c_int(G.shape[0]), _p(G, C.c_double), _p(D, C.c_double),
                        C.c_double(lam), C.byref(v))
    if rc:
        raise RuntimeError("df: matrix not positive definite")
    return v.value


def lambda_for_df(G, D, target: float) -> float:
    G = _arr(G, np.float64)
    D = _arr(D, np.float64)
    v = C.c_double()
    rc = _load().orc_lambda_for_df(C.c_int(G.shape[0]), _p(G, C.c_double), _p(D, C.c_double),
                                   C.c_double(target), C.byref(v))
    if rc:
        raise RuntimeError(_load().orc_last_error().decode())
    return v.value


def loss(name: str, y: float, f: float) -> float:
    return _load().orc_loss(LOSSES[name], y, f)


def pseudo_residual(name: str, y: float, f: float) -> float:
    return _load().orc_pseudo_residual(LOSSES[name], y, f)


def max_threads() -> int:
    return _load().orc_max_threads()


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def predict(problem: dict, result: dict, x_new) -> np.ndarray:
    """The fitted primary model at new feature values (Section 2.3: the
    intercept plus each learner's fitted function): each P-spline learner's
    basis at x by the Cox-de Boor recursion on the knots of its training
    range, with x clamped to that range; a categorical learner adds the
    coefficient of the level.  ``result`` is an oracle fit of ``problem``."""
    x = np.asarray(problem["x"], dtype=np.float64)
    xn = np.atleast_2d(np.asarray(x_new, dtype=np.float64))
    p = x.shape[1]
    kind = _arr(problem["kind"], np.int32, p)
    degree = int(problem.get("degree", 3))
    n_knots = int(problem.get("n_knots", 20))
    f = np.full(xn.shape[0], float(result["f0"]))
    off = 0
    for k in range(p):
        d = int(result["d"][k])
        c = result["coef_f"][off:off + d]
        if kind[k] != 0:
            f += c[xn[:, k].astype(np.int64)]
        else:
            lo, hi = float(x[:, k].min()), float(x[:, k].max())
            t = knots(lo, hi, n_knots, degree)
            f += bspline(np.clip(xn[:, k], lo, hi), t, degree) @ c
        off += d
    return f



def partial_effect(problem: dict, result: dict, k: int, values) -> np.ndarray:
    """Learner k's fitted function alone at the given values: ``predict``
    with the intercept and every other learner's coefficients set to zero."""
    x = np.asarray(problem["x"], dtype=np.float64)
    kind = np.asarray(problem["kind"])
    v = np.asarray(values, dtype=np.float64)
    xn = np.empty((v.shape[0], x.shape[1]))
    for j in range(x.shape[1]):  # any valid value: these learners contribute 0
        xn[:, j] = 0.0 if kind[j] != 0 else x[0, j]
    xn[:, k] = v
    d = np.asarray(result["d"])
    off = int(d[:k].sum())
    coef = np.zeros_like(np.asarray(result["coef_f"], dtype=np.float64))
    coef[off:off + int(d[k])] = result["coef_f"][off:off + int(d[k])]
    return predict(problem, dict(result, f0=0.0, coef_f=coef), xn)
