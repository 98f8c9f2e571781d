"""Build the lensfield HIP library for gfx950 (hipcc, in-tree)."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblensfield.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("LF_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled: the compiler must not form v_pk_*_f32.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-but-set-variable", "-fno-fast-math", "-ffp-contract=on"]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", src, "-o", obj] + COMMON + DEVICE
    if src.endswith(".cpp"):
        cmd = ["hipcc", "-c", "-x", "hip", src, "-o", obj] + COMMON + DEVICE
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


PROBE_SRC = os.path.join(HERE, "probe", "lf_rates.hip")
PROBE_LIB = os.path.join(HERE, "liblfrates.so")


def build_probe(verbose: bool = False) -> str:
    """The issue-rate probe used by the benchmark (a separate library: nothing of lensfield uses it)."""
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", PROBE_SRC, "-o", tmp] + COMMON + DEVICE
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (PROBE_SRC, r.stderr[-4000:]))
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print("built", PROBE_LIB)
    return PROBE_LIB


def build(verbose: bool = False) -> str:
    build_probe(verbose)
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
