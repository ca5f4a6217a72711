"""Build libcwb.so (gfx950 HIP kernels + host runtime) in-tree with hipcc.

Usage: python -m paper_2110_03513_amd.build [-v] [-i]
  -v  print the commands;  -i  recompile only sources older than their object
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcwb.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]
# Device code: no packed FP32 instructions.
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops"]
# Host-only sources; setup.cpp must not fuse the binning distances.
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]

SOURCES = [
    ("kernels.hip", DEVICE),
    ("hist.hip", DEVICE),
    ("probe.hip", DEVICE),
    ("noalloc.hip", DEVICE),
    # the device binning rule must not fuse its distances either
    ("binning.hip", DEVICE + ["-ffp-contract=off"]),
    ("runtime.cpp", HOST),
    ("server.cpp", HOST + ["-pthread"]),
    ("setup.cpp", HOST + ["-ffp-contract=off", "-pthread"]),
]


def _stale(src, out) -> bool:
    """The object is missing or older than its source or any header here."""
    if not os.path.exists(out):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC)
                                        if h.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "cwb.h"))
    t = os.path.getmtime(out)
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def _compile(src, flags, verbose, incremental=False):
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if incremental and not _stale(src, out):
        return out
    cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (or, with `incremental`, those whose object is
    older than the source or a header) and link libcwb.so."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], verbose, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libcwb.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
