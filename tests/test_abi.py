"""CPU checks of the C ABI library: it loads (bound to torch's HIP runtime),
exports every entry point include/tpilu.h declares, and the product path has
no CPU fallback."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpilu.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"TPILU_API\s+[\w\s\*]+?\b(tpilu_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_0803_0048_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_0803_0048_amd import build

        build.build()
    return binding.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("tpilu_symbolic", "tpilu_numeric", "tpilu_apply", "tpilu_gmres"):
        assert core in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol(lib):
    from paper_0803_0048_amd import binding

    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(tpilu_\w+)", out))
    declared = set(_declared())
    assert declared <= exported, declared - exported
    assert exported <= declared, exported - declared  # nothing undeclared leaks out
    assert set(binding.EXPORTED) == declared
    for n in declared:
        getattr(lib, n)


def test_jitter_build_exports_the_same_symbols(lib):
    """The race check build is the same library with pauses compiled in: same
    entry points, and the product path does not load it."""
    from paper_0803_0048_amd import binding, build

    jit = build.JITTER_LIB
    if not os.path.exists(jit):
        pytest.skip("jitter build not present")
    outs = []
    for path in (binding.LIB_PATH, jit):
        out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
        outs.append(set(re.findall(r"\bT\s+(tpilu_\w+)", out)))
    assert outs[0] == outs[1]
    assert os.path.basename(binding.LIB_PATH) == "libtpilu.so"
    assert "libtpilu_jitter.so" not in open("/proc/self/maps").read()


def test_library_binds_to_torch_hip_runtime(lib):
    import torch

    maps = open("/proc/self/maps").read()
    hips = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(hips) == 1, hips
    assert os.path.dirname(torch.__file__) in next(iter(hips))


def test_status_strings(lib):
    assert lib.tpilu_status_string(0) == b"ok"
    assert lib.tpilu_status_string(3) == b"zero pivot"
    assert lib.tpilu_status_string(6) == b"dependency wait timed out"


def test_no_gpu_means_loud_failure(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_0803_0048_amd import binding

    with pytest.raises(RuntimeError):
        binding.context(0)


def test_missing_library_means_loud_failure(monkeypatch, tmp_path):
    from paper_0803_0048_amd import binding

    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        binding.load_library()


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_0803_0048_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "ilu_oracle" not in txt and "liboracle" not in txt, f


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits non-zero
    before touching torch or the library."""
    import sys as _sys

    r = subprocess.run([_sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
