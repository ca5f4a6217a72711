"""ctypes binding of libcwb.so (the C ABI in include/cwb.h).

Argument marshalling only: every step of a boosting iteration runs in the
library's HIP kernels.  PyTorch provides the device workspace (a uint8 CUDA
tensor) and the stream.  ``lib()`` raises if libcwb.so has not been built;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcwb.so")

CWB_OK, CWB_E_INVALID_ARG, CWB_E_UNSUPPORTED, CWB_E_NO_MEMORY = 0, -1, -2, -3
CWB_E_DEVICE, CWB_E_NUMERIC, CWB_E_AGAIN, CWB_E_STATE = -4, -5, -6, -7
CWB_PSPLINE, CWB_RIDGE_CAT, CWB_BINARY_CAT = 0, 1, 2
LOSSES = {"l2": 0, "binomial": 1}
VARIANTS = {"cwb": 0, "acwb": 1, "hcwb": 2}
SETUPS = {"auto": 0, "host": 1, "device": 2}


class CwbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cwb error {code}: {msg}")
        self.code = code


class cwb_learner_spec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("degree", C.c_int32), ("n_interior_knots", C.c_int32),
                ("penalty_order", C.c_int32), ("df", C.c_double), ("lam", C.c_double),
                ("n_bins", C.c_int32), ("n_levels", C.c_int32)]


class cwb_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("p", C.c_int32), ("x", C.POINTER(C.c_double)),
                ("y", C.POINTER(C.c_double)), ("loss", C.c_int32),
                ("specs", C.POINTER(cwb_learner_spec)), ("nu", C.c_double), ("M", C.c_int32),
                ("variant", C.c_int32), ("gamma", C.c_double), ("patience", C.c_int32),
                ("val_mask", C.POINTER(C.c_uint8)), ("ldx", C.c_int64),
                ("setup", C.c_int32)]


class cwb_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("p", C.c_int32), ("M", C.c_int32), ("d_max", C.c_int32),
                ("sum_d", C.c_int32), ("nb_max", C.c_int32), ("iters_done", C.c_int32),
                ("n_train", C.c_int64), ("f0", C.c_double)]


class cwb_tile(C.Structure):
    _fields_ = [("threads", C.c_int32), ("learners", C.c_int32), ("blocks", C.c_int32),
                ("candidates", C.c_int32), ("learners32", C.c_int32), ("acc32_bits", C.c_int32),
                ("index_bits", C.c_int32), ("tuned_us", C.c_double)]


class cwb_server_cfg(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("quantum", C.c_int32), ("stream", C.c_void_p), ("setup_threads", C.c_int32)]


class cwb_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("M", C.c_int32), ("latency_s", C.c_double),
                ("queue_s", C.c_double), ("intercept", C.c_double)]


class cwb_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("in_flight", C.c_int32), ("queued", C.c_int32), ("fits_per_s", C.c_double),
                ("p50_latency_s", C.c_double), ("p99_latency_s", C.c_double),
                ("arena_in_use", C.c_size_t), ("arena_peak", C.c_size_t),
                ("mean_setup_s", C.c_double), ("mean_queue_s", C.c_double),
                ("round_s", C.c_double), ("busy_s", C.c_double), ("rounds", C.c_int64)]


_P = C.c_void_p
_SIGNATURES = {
    "cwb_version": [C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "cwb_last_error": [],
    "cwb_bin_feature": [_P, C.c_int64, C.c_int32, _P, _P],
    "cwb_lambda_for_df": [C.c_int32, _P, _P, C.c_double, _P],
    "cwb_workspace_bytes": [C.POINTER(cwb_problem), C.POINTER(C.c_size_t)],
    "cwb_fit_create": [C.POINTER(cwb_problem), _P, C.c_size_t, _P, C.POINTER(_P)],
    "cwb_fit_create_noalloc": [C.POINTER(cwb_problem), _P, C.c_size_t, _P, C.POINTER(_P)],
    "cwb_fit_run": [_P, C.c_int32],
    "cwb_fit_sync": [_P],
    "cwb_fit_info": [_P, C.POINTER(cwb_info)],
    "cwb_fit_get_trace": [_P, _P, _P, _P, _P, _P, _P, _P, _P],
    "cwb_fit_get_model": [_P, _P, _P, _P],
    "cwb_fit_get_pred": [_P, _P],
    "cwb_fit_state_bytes": [_P, C.POINTER(C.c_size_t)],
    "cwb_fit_save_state": [_P, _P, C.c_size_t],
    "cwb_fit_load_state": [_P, _P, C.c_size_t],
    "cwb_fit_set_timing": [_P, C.c_int32],
    "cwb_fit_kernel_time": [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "cwb_fit_destroy": [_P],
    "cwb_batch_workspace_bytes": [C.POINTER(_P), C.c_int32, C.POINTER(C.c_size_t)],
    "cwb_batch_create": [C.POINTER(_P), C.c_int32, _P, C.c_size_t, _P, C.POINTER(_P)],
    "cwb_batch_run": [_P, C.c_int32],
    "cwb_batch_sync": [_P],
    "cwb_batch_destroy": [_P],
    "cwb_fit_tile": [_P, C.POINTER(cwb_tile)],
    "cwb_fit_predict": [_P, _P, C.c_int64, C.c_int64, _P],
    "cwb_fit_partial_effect": [_P, C.c_int32, _P, C.c_int64, _P],
    "cwb_fit_set_timing_period": [_P, C.c_int32, C.c_int32],
    "cwb_batch_tile": [_P, C.POINTER(cwb_tile)],
    "cwb_server_create": [C.POINTER(cwb_server_cfg), C.POINTER(_P)],
    "cwb_server_submit": [_P, C.POINTER(cwb_problem), C.POINTER(C.c_uint64)],
    "cwb_server_poll": [_P, C.c_uint64, C.POINTER(cwb_result), _P, _P],
    "cwb_server_stats": [_P, C.POINTER(cwb_stats)],
    "cwb_server_destroy": [_P],
    "cwb_cv_workspace_bytes": [C.POINTER(cwb_problem), C.c_int32, _P, C.POINTER(C.c_size_t)],
    "cwb_cv_create": [C.POINTER(cwb_problem), C.c_int32, _P, _P, C.c_size_t, _P, C.POINTER(_P)],
    "cwb_cv_run": [_P, C.c_int32],
    "cwb_cv_sync": [_P],
    "cwb_cv_fold": [_P, C.c_int32, C.POINTER(_P)],
    "cwb_cv_risk": [_P, _P],
    "cwb_cv_destroy": [_P],
    "cwb_cv_tile": [_P, C.POINTER(cwb_tile)],
    "cwb_probe_lds_hist": [_P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P],
}
_VOID = {"cwb_fit_destroy", "cwb_batch_destroy", "cwb_server_destroy", "cwb_cv_destroy"}

_lib = None


def lib():
    """Load libcwb.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2110_03513_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            if name == "cwb_last_error":
                fn.restype = C.c_char_p
            elif name in _VOID:
                fn.restype = None
            else:
                fn.restype = C.c_int
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc != CWB_OK and rc != CWB_E_AGAIN:
        raise CwbError(rc, lib().cwb_last_error().decode())
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data


class Problem:
    """A cwb_problem plus the NumPy arrays that back its pointers."""

    def __init__(self, prob: dict):
        x = np.asarray(prob["x"], dtype=np.float64)
        n, p = x.shape
        # column-major views with a column stride (e.g. leading rows and
        # columns of a larger column-major matrix) are passed without a copy
        if x.strides[0] == 8 and x.strides[1] % 8 == 0 and x.strides[1] // 8 >= n:
            self.x, ldx = x, x.strides[1] // 8
        else:
            self.x, ldx = np.asfortranarray(x), n
        self.y = np.ascontiguousarray(prob["y"], dtype=np.float64)
        vm = prob.get("val_mask")
        self.vm = None if vm is None else np.ascontiguousarray(vm, dtype=np.uint8)
        kind = np.asarray(prob["kind"])
        specs = (cwb_learner_spec * p)()
        for j in range(p):
            s = specs[j]
            s.kind = int(kind[j])
            s.degree = int(prob.get("degree", 3))
            s.n_interior_knots = int(prob.get("n_knots", 20))
            s.penalty_order = int(prob.get("pen_order", 2))
            s.df = float(prob["df"][j])
            s.lam = float(np.asarray(prob.get("lambda", np.zeros(p)))[j])
            s.n_bins = int(prob["n_bins"][j])
            s.n_levels = int(np.asarray(prob.get("n_levels", np.zeros(p)))[j])
        self.specs = specs
        self.c = cwb_problem(
            n=n, p=p, x=self.x.ctypes.data_as(C.POINTER(C.c_double)),
            y=self.y.ctypes.data_as(C.POINTER(C.c_double)), loss=LOSSES[prob["loss"]],
            specs=C.cast(specs, C.POINTER(cwb_learner_spec)), nu=float(prob["nu"]),
            M=int(prob["M"]), variant=VARIANTS[prob.get("variant", "cwb")],
            gamma=float(prob.get("gamma", 0.0)), patience=int(prob.get("patience", 5)),
            val_mask=None if self.vm is None else self.vm.ctypes.data_as(C.POINTER(C.c_uint8)),
            ldx=ldx, setup=SETUPS[prob.get("setup", "auto")])
        self.n, self.p, self.M = n, p, int(prob["M"])


def bin_feature(x, n_bins: int):
    """Library binning of one feature: (design points, uint16 index vector)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    ind = np.zeros(x.shape[0], np.uint16)
    z = np.zeros(n_bins)
    check(lib().cwb_bin_feature(_ptr(x), x.shape[0], int(n_bins), _ptr(ind), _ptr(z)))
    return z, ind


def lambda_for_df(G, D, df: float) -> float:
    """Library smoothing parameter for a df target (host only)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    out = np.zeros(1)
    check(lib().cwb_lambda_for_df(int(G.shape[0]), _ptr(G), _ptr(D), float(df), _ptr(out)))
    return float(out[0])


def workspace_bytes(prob: dict | Problem) -> int:
    pr = prob if isinstance(prob, Problem) else Problem(prob)
    b = C.c_size_t()
    check(lib().cwb_workspace_bytes(C.byref(pr.c), C.byref(b)))
    return b.value


def probe_lds_hist(idx, nb: int, learners: int, steps: int, blocks: int, out, stream=None,
                   word_bytes: int = 8):
    """Launch the LDS histogram ceiling probe (a measurement utility, not
    part of the method, include/cwb_probe.h) on `stream` (torch's current
    stream by default): `idx` a CUDA uint16-compatible tensor of bins (int16
    storage), `out` a zeroed CUDA int64 tensor of `blocks` entries,
    `word_bytes` the LDS word width (4 or 8)."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    check(lib().cwb_probe_lds_hist(C.c_void_p(idx.data_ptr()), int(idx.numel()), int(nb),
                                   int(learners), int(word_bytes), int(steps), int(blocks),
                                   C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream), s


class Fit:
    """One fit: workspace owned by a torch uint8 tensor on the current device.
    With ``workspace`` (a torch uint8 CUDA tensor of at least
    ``workspace_bytes`` bytes) the fit uses it instead of allocating one; with
    ``noalloc`` it is created by cwb_fit_create_noalloc (histogram partials
    in the library's static array)."""

    def __init__(self, prob: dict, stream=None, device=None, workspace=None, noalloc=False):
        torch = _torch()
        self.problem = Problem(prob)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            if workspace is None:
                nbytes = workspace_bytes(self.problem)
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            else:
                self.ws = workspace
                nbytes = workspace.numel()
            self._sh, self.stream = _stream_handle(stream)
            h = C.c_void_p()
            create = lib().cwb_fit_create_noalloc if noalloc else lib().cwb_fit_create
            check(create(C.byref(self.problem.c), C.c_void_p(self.ws.data_ptr()), nbytes, self._sh,
                         C.byref(h)))
        self.h = h
        info = cwb_info()
        check(lib().cwb_fit_info(self.h, C.byref(info)))
        self.info = info

    def run(self, iters: int):
        check(lib().cwb_fit_run(self.h, int(iters)))

    def sync(self):
        check(lib().cwb_fit_sync(self.h))

    @property
    def iters_done(self) -> int:
        info = cwb_info()
        check(lib().cwb_fit_info(self.h, C.byref(info)))
        return info.iters_done

    def trace(self) -> dict:
        M = self.info.M
        dm = self.info.d_max
        out = {"k": np.zeros(M, np.int32), "theta": np.zeros((M, dm)),
               "kcor": np.zeros(M, np.int32), "thetacor": np.zeros((M, dm)),
               "risk_train": np.zeros(M + 1), "risk_val": np.zeros(M + 1),
               "gap": np.zeros(M), "switch_iter": np.zeros(1, np.int32)}
        check(lib().cwb_fit_get_trace(self.h, *[_ptr(out[k]) for k in
                                               ("k", "theta", "kcor", "thetacor", "risk_train",
                                                "risk_val", "gap", "switch_iter")]))
        m = self.iters_done
        for key in ("k", "theta", "kcor", "thetacor", "gap"):
            out[key] = out[key][:m]
        out["risk_train"] = out["risk_train"][:m + 1]
        out["risk_val"] = out["risk_val"][:m + 1]
        out["switch_iter"] = int(out["switch_iter"][0])
        return out

    def model(self) -> dict:
        sd = self.info.sum_d
        cf = np.zeros(sd)
        ch = np.zeros(sd)
        ic = C.c_double()
        check(lib().cwb_fit_get_model(self.h, C.byref(ic), _ptr(cf), _ptr(ch)))
        return {"f0": ic.value, "coef_f": cf, "coef_h": ch}

    def pred(self) -> np.ndarray:
        out = np.zeros(self.info.n, np.float32)
        check(lib().cwb_fit_get_pred(self.h, _ptr(out)))
        return out

    def predict(self, x_new) -> np.ndarray:
        """The fitted model at new rows (n x p raw feature values), on the GPU."""
        torch = _torch()
        xn = np.atleast_2d(np.asarray(x_new, dtype=np.float64))
        n = xn.shape[0]
        with torch.cuda.device(self.device):
            xd = torch.from_numpy(np.ascontiguousarray(xn.T)).to(self.device)  # (p, n): column-major x
            out = torch.empty(n, dtype=torch.float64, device=self.device)
            torch.cuda.current_stream().synchronize()
            check(lib().cwb_fit_predict(self.h, C.c_void_p(xd.data_ptr()), n, n,
                                        C.c_void_p(out.data_ptr())))
            check(lib().cwb_fit_sync(self.h))
            return out.cpu().numpy()

    def partial_effect(self, k: int, values) -> np.ndarray:
        """Learner k's fitted function (without the intercept) at the given values."""
        torch = _torch()
        v = np.ascontiguousarray(np.asarray(values, dtype=np.float64).ravel())
        with torch.cuda.device(self.device):
            xd = torch.from_numpy(v).to(self.device)
            out = torch.empty(v.shape[0], dtype=torch.float64, device=self.device)
            torch.cuda.current_stream().synchronize()
            check(lib().cwb_fit_partial_effect(self.h, int(k), C.c_void_p(xd.data_ptr()), v.shape[0],
                                               C.c_void_p(out.data_ptr())))
            check(lib().cwb_fit_sync(self.h))
            return out.cpu().numpy()

    def save_state(self) -> bytes:
        n = C.c_size_t()
        check(lib().cwb_fit_state_bytes(self.h, C.byref(n)))
        buf = (C.c_char * n.value)()
        check(lib().cwb_fit_save_state(self.h, buf, n.value))
        return bytes(buf)

    def load_state(self, blob: bytes):
        buf = (C.c_char * len(blob)).from_buffer_copy(blob)
        check(lib().cwb_fit_load_state(self.h, buf, len(blob)))

    def tile(self) -> dict:
        t = cwb_tile()
        check(lib().cwb_fit_tile(self.h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in cwb_tile._fields_}

    def set_timing(self, mask, period: int = 1):
        """mask: bit set 1 = hist, 2 = state, 4 = select (True = all, False =
        off); only every `period`-th iteration is timed."""
        if mask is True:
            mask = 7
        check(lib().cwb_fit_set_timing_period(self.h, int(mask), int(period)))

    def kernel_time(self, name: str):
        ms = C.c_double()
        cnt = C.c_int64()
        check(lib().cwb_fit_kernel_time(self.h, name.encode(), C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    @classmethod
    def _view(cls, handle, owner):
        """A fit owned by another object (a fold of a cross-validation)."""
        f = cls.__new__(cls)
        f.problem = owner.problem
        f.device = owner.device
        f.ws = None
        f._sh, f.stream = owner._sh, owner.stream
        f.h = handle
        f._owner = owner
        info = cwb_info()
        check(lib().cwb_fit_info(f.h, C.byref(info)))
        f.info = info
        return f

    def close(self):
        if getattr(self, "_owner", None) is not None:  # owned elsewhere
            self.h = None
            return
        if getattr(self, "h", None):
            lib().cwb_fit_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many fits advanced together (one launch per kernel per iteration)."""

    def __init__(self, fits: list[Fit], stream=None):
        torch = _torch()
        self.fits = fits
        arr = (C.c_void_p * len(fits))(*[f.h.value for f in fits])
        self._arr = arr
        b = C.c_size_t()
        check(lib().cwb_batch_workspace_bytes(arr, len(fits), C.byref(b)))
        dev = fits[0].device
        self.ws = torch.empty(b.value, dtype=torch.uint8, device=dev)
        self._sh, self.stream = _stream_handle(stream)
        h = C.c_void_p()
        check(lib().cwb_batch_create(arr, len(fits), C.c_void_p(self.ws.data_ptr()), b.value,
                                     self._sh, C.byref(h)))
        self.h = h

    def run(self, iters: int):
        check(lib().cwb_batch_run(self.h, int(iters)))

    def tile(self) -> dict:
        t = cwb_tile()
        check(lib().cwb_batch_tile(self.h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in cwb_tile._fields_}

    def sync(self):
        check(lib().cwb_batch_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().cwb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CV:
    """K-fold cross-validation: the folds share one index matrix and one
    histogram pass per iteration; ``folds[k]`` is fold k's fit."""

    def __init__(self, prob: dict, fold, stream=None, device=None):
        torch = _torch()
        self.problem = Problem(prob)
        self.fold = np.ascontiguousarray(np.asarray(fold, dtype=np.int32))
        self.n_folds = int(self.fold.max()) + 1 if self.fold.size else 0
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            b = C.c_size_t()
            check(lib().cwb_cv_workspace_bytes(C.byref(self.problem.c), self.n_folds,
                                               _ptr(self.fold), C.byref(b)))
            self.ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
            self._sh, self.stream = _stream_handle(stream)
            h = C.c_void_p()
            check(lib().cwb_cv_create(C.byref(self.problem.c), self.n_folds, _ptr(self.fold),
                                      C.c_void_p(self.ws.data_ptr()), b.value, self._sh, C.byref(h)))
        self.h = h
        self.folds = []
        for k in range(self.n_folds):
            fh = C.c_void_p()
            check(lib().cwb_cv_fold(self.h, k, C.byref(fh)))
            self.folds.append(Fit._view(fh, self))

    def run(self, iters: int):
        check(lib().cwb_cv_run(self.h, int(iters)))

    def sync(self):
        check(lib().cwb_cv_sync(self.h))

    def tile(self) -> dict:
        t = cwb_tile()
        check(lib().cwb_cv_tile(self.h, C.byref(t)))
        return {name: getattr(t, name) for name, _ in cwb_tile._fields_}

    def risk(self) -> np.ndarray:
        """Cross-validated risk of iterations 0..done (held-out loss / n)."""
        m = self.folds[0].iters_done
        out = np.zeros(self.folds[0].info.M + 1)
        check(lib().cwb_cv_risk(self.h, _ptr(out)))
        return out[:m + 1]

    def close(self):
        if getattr(self, "h", None):
            for f in self.folds:
                f.close()
            lib().cwb_cv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit(prob: dict, iters: int | None = None, stream=None) -> dict:
    """Create a fit, run it (all M iterations by default) and return traces,
    model and predictions as NumPy arrays."""
    f = Fit(prob, stream=stream)
    f.run(f.info.M if iters is None else iters)
    f.sync()
    out = f.trace()
    out.update(f.model())
    out["f"] = f.pred()
    out["n_train"] = f.info.n_train
    f.close()
    return out


class Server:
    """Continuous-batching fit server: requests are set up on host threads,
    admitted while the device arena (a torch uint8 tensor) holds them, and
    advanced together in rounds of `quantum` iterations on `stream`."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, quantum: int = 50,
                 setup_threads: int = 0, stream=None):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.synchronize()
        cfg = cwb_server_cfg(arena=C.c_void_p(self.arena.data_ptr()), arena_bytes=int(arena_bytes),
                             max_slots=int(max_slots), quantum=int(quantum),
                             stream=C.c_void_p(self.stream.cuda_stream),
                             setup_threads=int(setup_threads))
        h = C.c_void_p()
        check(lib().cwb_server_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self._pending = {}

    def submit(self, prob: dict) -> int:
        pr = Problem(prob)
        t = C.c_uint64()
        check(lib().cwb_server_submit(self.h, C.byref(pr.c), C.byref(t)))
        # the server reads the problem's arrays in place until the result is polled
        self._pending[t.value] = (pr, np.zeros(pr.n, np.float32), np.zeros(pr.M, np.int32))
        return t.value

    def poll(self, ticket: int):
        """None while the request is pending, else a dict with its status,
        latency, intercept, training predictions and selection trace."""
        _, pred, k = self._pending[ticket]
        res = cwb_result()
        rc = lib().cwb_server_poll(self.h, C.c_uint64(ticket), C.byref(res), _ptr(pred), _ptr(k))
        if rc == CWB_E_AGAIN:
            return None
        check(rc)
        del self._pending[ticket]
        out = {"status": res.status, "M": res.M, "latency_s": res.latency_s,
               "queue_s": res.queue_s, "f0": res.intercept}
        if res.status == CWB_OK:
            out["f"] = pred
            out["k"] = k
        else:
            out["error"] = lib().cwb_last_error().decode()
        return out

    def stats(self) -> dict:
        st = cwb_stats()
        check(lib().cwb_server_stats(self.h, C.byref(st)))
        return {name: getattr(st, name) for name, _ in cwb_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().cwb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
