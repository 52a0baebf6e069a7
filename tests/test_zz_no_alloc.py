"""The allocation-free commutator (pauli_commutator_noalloc: scratch in a
static device array instead of a caller workspace) against the workspace
entry point pauli_commutator, through the C ABI: two calls in a row (the
second smaller, so it runs on the first call's leftover scratch), each bit
for bit equal; a call beyond the static scratch is refused with
PAULI_EWORKSPACE and a message."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as wl
from helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(pk, H, O, trunc, cap):
    L = pk._lib.load()
    out = pk.PauliOp(O.n_qubits, cap, O.dtype)
    hs, os_, outs = H.c_struct(), O.c_struct(), out.c_struct()
    keep_s, ts = trunc.c_struct() if trunc is not None else (None, None)
    st = L.pauli_commutator_noalloc(ctypes.byref(hs), ctypes.byref(os_),
                                    ctypes.byref(ts) if ts is not None else None,
                                    ctypes.byref(outs), pk.ops._stream_handle())
    out.size = int(outs.size)
    return st, out


def _same(a, b):
    ha, hb = a.to_host(), b.to_host()
    assert ha.n == hb.n
    # both follow the canonical order: element by element, bit for bit
    assert np.array_equal(ha.x, hb.x) and np.array_equal(ha.z, hb.z)
    assert np.array_equal(ha.coef.view(np.float64), hb.coef.view(np.float64))


@pytest.mark.parametrize("dtype", [0, 1])
def test_noalloc_matches_workspace_entry_point(dtype):
    import paper_2410_09654_amd as pk
    n = 64
    H = pk.PauliOp.from_raw(n, *(lambda h: (h.x, h.z, h.coef))(wl.ising_chain(n)))
    T = pk.Trunc(max_len=12, max_strings=40000)
    for count, seed in ((60000, 21), (7000, 22)):
        say(f"noalloc commutator dtype={dtype} |O|={count}")
        O = pk.PauliOp.from_host(wl.random_local_strings(n, count, 10, seed=seed), dtype=dtype)
        want = pk.commutator(H, O, T)
        st, got = _noalloc(pk, H, O, T, 40000)
        assert st == pk._lib.PAULI_OK, pk._lib.last_error()
        assert got.size == want.size > 0
        _same(got, want)


def test_noalloc_untruncated_and_refusal():
    import paper_2410_09654_amd as pk
    n = 128
    Hh, _ = wl.xxz_random_field(n)
    H = pk.PauliOp.from_raw(n, Hh.x, Hh.z, Hh.coef)
    O = pk.PauliOp.from_host(wl.random_local_strings(n, 3000, 8, seed=23))
    say("noalloc commutator untruncated, two words")
    want = pk.commutator(H, O)
    st, got = _noalloc(pk, H, O, None, want.size)
    assert st == pk._lib.PAULI_OK, pk._lib.last_error()
    _same(got, want)
    # 2^20 strings of length <= 10 with the 509-string chain: far beyond 256 MiB
    say("noalloc commutator beyond the static scratch")
    big = pk.PauliOp.from_host(wl.random_local_strings(n, 1 << 20, 10, seed=24))
    st, _ = _noalloc(pk, H, big, pk.Trunc(max_strings=1000), 1000)
    assert st == pk._lib.PAULI_EWORKSPACE
    assert "static scratch" in pk._lib.last_error()
