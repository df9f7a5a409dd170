"""Build libpmace.so (HIP, gfx950) in-tree with hipcc.

Launch-shape parameters come from tuned.json beside this file (written by
tune.py) as -D flags; without it the defaults in csrc/pmace_internal.hpp hold."""
from __future__ import annotations

import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmace.so")
DEMO = os.path.join(HERE, "pmace_demo")
TUNED = os.path.join(HERE, "tuned.json")
SOURCES = ["pmace_api.hip", "pmace_kernels.hip", "pmace_simulate.hip"]

# Packed FP32 VALU forms are kept out of the generated code on purpose, and
# floating-point contraction is off: every fused multiply-add is written out in
# the source, so all instantiations of a device function round identically.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def tuned_defines() -> dict:
    if not os.path.exists(TUNED):
        return {}
    with open(TUNED) as f:
        return {k: int(v) for k, v in json.load(f).get("defines", {}).items()}


def build(verbose: bool = False, out: str = LIB, defines: dict | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    d = tuned_defines() if defines is None else defines
    dflags = [f"-D{k}={int(v)}" for k, v in sorted(d.items())]
    cmd = [hipcc, *FLAGS, *dflags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {out}")
    os.replace(out + ".tmp", out)
    return out


def build_demo(verbose: bool = False, lib: str = LIB, out: str = DEMO) -> str:
    """The C++ example that drives the C ABI without Python, linked against
    `lib` (found beside the executable at run time)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "pmace_demo.cpp"), "-L", os.path.dirname(lib), "-l:" + os.path.basename(lib),
           "-Wl,-rpath,$ORIGIN", "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {out}")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_demo(verbose=True))
