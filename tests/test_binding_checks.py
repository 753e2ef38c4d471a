"""Host-side argument checks of the Python binding (no GPU needed).

Every size the kernels index is checked against the pattern before any C
call: an undersized tensor must raise ValueError instead of reaching a
kernel.  The device check of the binding is relaxed here (tensors live on the
CPU), everything else is the binding's own code.
"""
from __future__ import annotations

import pytest
import torch

from paper_0803_0048_amd import binding as T


class _FakePattern:
    def __init__(self, n=10, nnz_a=30, nnz_f=40):
        self.n, self.nnz_a, self.nnz_f = n, nnz_a, nnz_f
        self.device = torch.device("cpu")
        self.h = None


@pytest.fixture
def pat(monkeypatch):
    real = T._need

    def need_any_device(t, dtype, name, device):
        return real(t, dtype, name, None) if t.device.type == "cuda" else _need_cpu(t, dtype, name)

    def _need_cpu(t, dtype, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    monkeypatch.setattr(T, "_need", need_any_device)

    def no_context(*a, **k):
        raise AssertionError("a C call was reached with invalid arguments")

    monkeypatch.setattr(T, "context", no_context)
    return _FakePattern()


def d(n):
    return torch.zeros(n, dtype=torch.float64)


def test_numeric_out_undersized(pat):
    with pytest.raises(ValueError):
        T.numeric(pat, d(pat.nnz_a), out=d(pat.nnz_f - 1))
    with pytest.raises(ValueError):
        T.numeric(pat, d(pat.nnz_a - 1))


def test_numeric_batched_out_shape(pat):
    with pytest.raises(ValueError):
        T.numeric(pat, torch.zeros(pat.nnz_a, 4, dtype=torch.float64), out=torch.zeros(pat.nnz_f, 3,
                                                                                         dtype=torch.float64))


def test_apply_sizes(pat):
    with pytest.raises(ValueError):
        T.apply(pat, d(pat.nnz_f), d(pat.n - 1))
    with pytest.raises(ValueError):
        T.apply(pat, d(pat.nnz_f - 1), d(pat.n))
    with pytest.raises(ValueError):
        T.apply(pat, d(pat.nnz_f), d(pat.n), out=d(pat.n - 1))
    b = d(pat.n)
    with pytest.raises(ValueError):
        T.apply(pat, d(pat.nnz_f), b, out=b)


def test_inverse_and_apply_inverse_sizes(pat):
    with pytest.raises(ValueError):
        T.inverse(pat, d(pat.nnz_f), out=d(pat.nnz_f - 1))
    with pytest.raises(ValueError):
        T.apply_inverse(pat, d(pat.nnz_f), d(pat.n), out=d(pat.n - 2))
    with pytest.raises(ValueError):
        T.apply_inverse(pat, d(pat.nnz_f - 1), d(pat.n))


def test_krylov_sizes(pat):
    with pytest.raises(ValueError):
        T.gmres(pat, d(pat.nnz_a), d(pat.nnz_f), d(pat.n - 1))
    with pytest.raises(ValueError):
        T.gmres(pat, d(pat.nnz_a - 1), d(pat.nnz_f), d(pat.n))
    with pytest.raises(ValueError):
        T.gmres(pat, d(pat.nnz_a), d(pat.nnz_f), d(pat.n), x0=d(pat.n + 1))
    with pytest.raises(ValueError):
        T.bicgstab(pat, d(pat.nnz_a), d(pat.nnz_f - 1), d(pat.n))
    with pytest.raises(ValueError):
        T.spmv(pat, d(pat.nnz_a), d(pat.n - 1))


def test_dot_lengths(pat):
    with pytest.raises(ValueError):
        T.dot(d(5), d(4))


def test_adjoint_sizes(pat):
    with pytest.raises(ValueError):
        T.apply_adjoint(pat, d(pat.nnz_f), d(pat.n), d(pat.n - 1), d(pat.n))
    with pytest.raises(ValueError):
        T.apply_adjoint(pat, d(pat.nnz_f - 1), d(pat.n), d(pat.n), d(pat.n))
    with pytest.raises(ValueError):
        T.numeric_adjoint(pat, d(pat.nnz_f), d(pat.nnz_f - 1))


def test_batched_graph_sizes(pat):
    B = 3
    a = torch.zeros(pat.nnz_a, B, dtype=torch.float64)
    b = torch.zeros(pat.n, B, dtype=torch.float64)
    with pytest.raises(ValueError):
        T.BatchedGraph(pat, a, b, f_val=torch.zeros(pat.nnz_f, B - 1, dtype=torch.float64))
    with pytest.raises(ValueError):
        T.BatchedGraph(pat, a, b, y=torch.zeros(pat.n - 1, B, dtype=torch.float64))
    with pytest.raises(ValueError):
        T.BatchedGraph(pat, a, torch.zeros(pat.n, B + 1, dtype=torch.float64))
