"""Build libsgrt.so (the HIP library behind include/sgrt.h) for gfx950 with hipcc.

Every source is compiled in-tree into ``_build/`` and linked into
``paper_2503_16037_amd/libsgrt.so``; ``build(debug=True)`` makes the bounds-checked
``libsgrt_debug.so`` (SG_DEBUG_BOUNDS, objects in ``_build/debug/``).  Packed FP32 instructions are disabled
for all device code; the phase-cell kernel, the graph builder and the host
runtime are compiled without floating-point contraction (their operation order
is part of the definition of lattice ownership and of the coupling ranking).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsgrt.so")
OUT_DEBUG = os.path.join(HERE, "libsgrt_debug.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("SGRT_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
NO_CONTRACT = {"qbuild.hip", "api.cpp", "graph.hip"}
# the phase-cell kernel sees only finite values: without NaN semantics the running maximum of
# the ownership argmax needs no canonicalisation (no effect on any finite result)
EXTRA = {"qbuild.hip": ["-fno-honor-nans"]}


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src: str, debug: bool = False) -> str:
    obj = os.path.join(BUILD, "debug" if debug else "", src + ".o")
    cmd = ["hipcc", *COMMON]
    if debug:
        cmd.append("-DSG_DEBUG_BOUNDS")
    if src in NO_CONTRACT:
        cmd.append("-ffp-contract=off")
    cmd += EXTRA.get(src, [])
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn:
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = True, debug: bool = False) -> str:
    os.makedirs(os.path.join(BUILD, "debug") if debug else BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, debug), srcs))
    out = OUT_DEBUG if debug else OUT
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(debug="--debug" in sys.argv)
