"""Shared helpers of the test suite (comparison of GPU results with the oracle)."""
from __future__ import annotations

import numpy as np

import workloads as wl


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def as_dict(op: wl.HostOp):
    return op.as_dict()


def assert_same_operator(got: wl.HostOp, want: wl.HostOp, rtol: float = 1e-12,
                         atol: float = 0.0, what: str = ""):
    """Keys bit-exact, coefficients within rtol * max(1, |want|) + atol."""
    g, w = got.as_dict(), want.as_dict()
    missing = set(w) - set(g)
    extra = set(g) - set(w)
    assert not missing and not extra, \
        f"{what}: key sets differ: {len(missing)} missing, {len(extra)} extra " \
        f"(got {len(g)}, want {len(w)})"
    worst = 0.0
    for k, wv in w.items():
        err = abs(g[k] - wv)
        lim = rtol * max(1.0, abs(wv)) + atol
        worst = max(worst, err / max(lim, 1e-300))
        assert err <= lim, f"{what}: key {k}: got {g[k]!r} want {wv!r}"
    return worst


def exact_fraction(got: wl.HostOp, want: wl.HostOp) -> float:
    g, w = got.as_dict(), want.as_dict()
    if not w:
        return 1.0
    return sum(1 for k in w if k in g and g[k] == w[k]) / len(w)


def assert_canonical_unique(op: wl.HostOp):
    keys = op.keys()
    assert len(set(keys)) == len(keys), "duplicate strings"
    assert np.all((op.coef.real != 0) | (op.coef.imag != 0)), "exact zero stored"
