"""Build the gfx950 HIP library ``libtpilu.so`` in-tree, and next to it
``libtpilu_jitter.so``: the same sources with ``-DTPILU_JITTER``, which adds a
pseudo-random pause before every publishing store and after every coherent
load (the race check build; only a test loads it, never the product path).

Every HIP unit is compiled with ``-ffp-contract=off``: hipcc contracts a*b-c
into an FMA by default, which would change the bits of every update.

Packed FP32 instructions (v_pk_add_f32 and its kin) are turned off with
``-Xclang -target-feature -Xclang -packed-fp32-ops``.  The feature belongs to
the gfx950 device pass, which honours it (a float2 kernel built with the flag
has no v_pk_ instruction, without it two); hipcc hands the same flag to the
x86 host pass too, which does not know the feature and prints "not a
recognized feature for this target (ignoring feature)" once per unit: that
warning is harmless and is filtered from the build output below.  The path is
FP64 throughout; the flag keeps the compiler from emitting packed FP32 in any
helper code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtpilu.so")
JITTER_LIB = os.path.join(HERE, "libtpilu_jitter.so")
SOURCES = ["k_symbolic.hip", "k_numeric.hip", "k_solve.hip", "k_solve_cu.hip", "k_krylov.hip", "k_adjoint.hip",
           "k_inverse.hip", "k_probe.hip", "tpilu_runtime.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _compile(src: str, build_dir: str, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # the host pass's note about the device-only feature (see the docstring)
    rest = "\n".join(ln for ln in r.stderr.splitlines()
                     if "packed-fp32-ops' is not a recognized feature" not in ln)
    if rest.strip():
        sys.stderr.write(rest + "\n")
    return obj


def _build_one(lib: str, build_dir: str, defines=(), verbose: bool = False) -> str:
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


def build(verbose: bool = False, jitter: bool = True) -> str:
    """Build libtpilu.so and (jitter=True) libtpilu_jitter.so; returns the
    product library's path."""
    _build_one(LIB, os.path.join(HERE, "_build"), (), verbose)
    if jitter:
        _build_one(JITTER_LIB, os.path.join(HERE, "_build_jitter"), ("-DTPILU_JITTER",), verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
