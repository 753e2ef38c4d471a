"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
the driver built by tests/host_sanitizer_build.py (tests/host_asan_driver.cpp
linked with a copy of the library whose host pass carries both sanitizers,
and with the oracle) runs every entry point on a small problem, checks the
results against the oracle and the error paths, and must exit cleanly with no
sanitizer report.  Leak reports from the HIP runtime's own allocations are
suppressed; any other leak fails the test."""
from __future__ import annotations

import os
import subprocess

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "_build_asan", "host_asan_driver")

pytestmark = pytest.mark.gpu


def test_host_code_under_asan_and_ubsan(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.path.exists(DRIVER), "the host sanitizer driver is not built"
    sup = tmp_path / "lsan.supp"
    sup.write_text("".join(f"leak:{m}\n" for m in ("libamdhip64", "libhsa-runtime64", "libamd_comgr", "libdrm",
                                                  "librocprofiler", "libhsa-amd-aqlprofile")))
    env = dict(os.environ,
               ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={sup}:print_suppressions=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print("[gpu] host sanitizer driver", flush=True)
    r = subprocess.run([DRIVER], capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
    assert "all checks passed" in r.stdout
