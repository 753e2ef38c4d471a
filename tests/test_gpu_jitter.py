"""The race check: the parity cases of tests/jitter_check.py run against the
jitter build (random pauses before every publishing store and after every
coherent load) in a process of their own, and must keep the oracle's bits."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def test_jitter_build_keeps_the_bits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = os.path.join(ROOT, "paper_0803_0048_amd", "libtpilu_jitter.so")
    assert os.path.exists(lib), "libtpilu_jitter.so is not built"
    print("[gpu] jitter check in a child process", flush=True)
    env = dict(os.environ, TPILU_LIBRARY="jitter")
    r = subprocess.run([sys.executable, "-u", "-m", "tests.jitter_check"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-4000:], flush=True)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "jitter build: all cases bitwise" in r.stdout
