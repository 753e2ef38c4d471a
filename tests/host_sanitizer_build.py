"""Build the host-side sanitizer driver (test infrastructure): the library's
sources with AddressSanitizer and UndefinedBehaviorSanitizer on the host pass
only (the GPU code is the normal build), the driver tests/host_asan_driver.cpp
and the oracle, linked into one executable, tests/_build_asan/host_asan_driver.
__graft_entry__.build() calls build(); tests/test_gpu_host_sanitizer.py runs
the result."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

from paper_0803_0048_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "tests", "_build_asan")
DRIVER = os.path.join(OUT, "host_asan_driver")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
CLANG = os.environ.get("TPILU_CLANG", "/opt/rocm/llvm/bin/clang")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", B.CSRC]
    jobs = [(os.path.join(B.CSRC, s), os.path.join(OUT, os.path.splitext(s)[0] + ".o")) for s in B.SOURCES]
    jobs.append((os.path.join(ROOT, "tests", "host_asan_driver.cpp"), os.path.join(OUT, "driver.o")))

    def one(job):
        src, obj = job
        r = subprocess.run([B.HIPCC, *B.FLAGS, *HOST_SAN, *inc, "-c", src, "-o", obj], capture_output=True,
                           text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, jobs))
    orc = os.path.join(OUT, "oracle.o")
    r = subprocess.run([CLANG, "-x", "c", "-std=c11", "-O2", "-ffp-contract=off", "-c",
                        os.path.join(ROOT, "oracle", "ilu_oracle.c"), "-o", orc], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle object failed:\n{r.stderr}")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(B.HIPCC)))
    link = [CLANG + "++", "-fsanitize=address,undefined", "-o", DRIVER, *objs, orc,
            "-L", os.path.join(rocm, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}", "-lm"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver link failed:\n{r.stderr}")
    for o in objs + [orc]:
        os.remove(o)
    if verbose:
        print("built", DRIVER)
    return DRIVER


if __name__ == "__main__":
    build(verbose=True)
