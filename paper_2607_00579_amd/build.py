"""Build libepo.so for gfx950 in-tree (hipcc, no JIT cache).

    python -m paper_2607_00579_amd.build

Every HIP source is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops) and only the C-ABI symbols
declared in include/epo.h are exported.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(PKG, "libepo.so")
SOURCES = ["edt.hip", "edge_cost.hip", "reduce.hip", "pose.hip", "converge.hip", "refine.hip",
           "sample.hip", "viewgraph.hip", "order.hip",
           "mlp.hip", "plan.hip"]
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", f"-I{INCLUDE}",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libepo.so)")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


# host-code sanitizers: -fsanitize only on the host pass (the device code is
# built as usual), for the C-ABI's host-side validation checks
SANITIZE = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-sanitize-recover=undefined -Xarch_host -fno-omit-frame-pointer").split()
HOST_CHECK_SRC = os.path.join(ROOT, "tests", "abi_host_check.cpp")
HOST_CHECK_DIR = os.path.join(BUILD_DIR, "host_check")
HOST_CHECK_BIN = os.path.join(HOST_CHECK_DIR, "abi_host_check")


def build_host_check(verbose: bool = False) -> str:
    """Every library source and tests/abi_host_check.cpp compiled with
    AddressSanitizer and UndefinedBehaviorSanitizer on the host code, linked
    into one program (runs without a GPU)."""
    os.makedirs(HOST_CHECK_DIR, exist_ok=True)
    flags = [f for f in COMMON if f != "-fvisibility=hidden"] + ["-O1", "-g"] + SANITIZE

    def comp(src):
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = os.path.join(HOST_CHECK_DIR, os.path.splitext(os.path.basename(path))[0] + ".o")
        cmd = [hipcc(), *flags, "-c", path, "-o", obj]
        if path.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {path}:\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES) + 1, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, SOURCES + [HOST_CHECK_SRC]))
    cmd = [hipcc(), f"--offload-arch={ARCH}", *SANITIZE, "-o", HOST_CHECK_BIN, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    if verbose:
        print(f"built {HOST_CHECK_BIN}")
    return HOST_CHECK_BIN


if __name__ == "__main__":
    build(verbose=True)
    if len(sys.argv) > 1 and sys.argv[1] == "host-check":
        build_host_check(verbose=True)
    sys.exit(0)
