"""GPU tests of the rest of the boundary: the Lanczos step with local
re-orthogonalisation (PAULI_REORTH_LOCAL) against the oracle's, the
autocorrelation S(t) computed in the library (pauli_correlator), and the
workspace sizing of pauli_workspace_query (a workspace of the queried size
holds the call)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import assert_same_operator, exact_fraction, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def pk():
    import paper_2410_09654_amd as pk
    pk._lib.load()
    return pk


@pytest.fixture(scope="module")
def ws(pk):
    return pk.Workspace(256 << 20)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def uph(pk, H):
    return pk.PauliOp.from_raw(H.n_qubits, H.x, H.z, H.coef)


def f32(op):
    c = op.coef.astype(np.complex64).astype(np.complex128)
    keep = (c.real != 0) | (c.imag != 0)
    return wl.HostOp(op.n_qubits, op.x[keep], op.z[keep], c[keep])


def test_reorth_noop_untruncated(pk, ws):
    """Config 1 (N = 12, 12 steps, no truncation): the re-orthogonalised
    recursion gives the plain b_n and the oracle's."""
    say("reorth untruncated config 1")
    H, O0, steps = wl.config_lanczos_small()
    want = oracle.lanczos(H, O0, steps, reorth=True)
    got = pk.lanczos(uph(pk, H), pk.PauliOp.from_host(O0, ws=ws), steps, ws=ws, reorth=True)
    plain = pk.lanczos(uph(pk, H), pk.PauliOp.from_host(O0, ws=ws), steps, ws=ws)
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    assert np.max(np.abs(np.array(got) - plain) / np.array(plain)) <= 1e-15


@pytest.mark.parametrize("n,M,steps,prec", [(16, 300, 12, 0), (128, 500, 8, 0),
                                            (128, 500, 8, 1)])
def test_reorth_truncated_vs_oracle(pk, ws, n, M, steps, prec):
    """Truncated re-orthogonalised steps, fed the oracle's own previous
    vectors each step: keys bit-exact, coefficients within 1e-12 (FP64) or
    equal after rounding to FP32 (the precision split), b_n within 1e-12."""
    say(f"reorth truncated n={n} M={M} prec={prec}")
    if n == 16:
        H = wl.ising_chain(n)
        O0 = wl.from_terms(n, [(1.0, [("Z", 8)])])
    else:
        H, _ = wl.xxz_random_field(n)
        O0 = wl.single_site_sum(n, "X", 1.0 / np.sqrt(n))
    t = oracle.Trunc(max_strings=M)
    T = pk.Trunc(max_strings=M)
    dt = pk.PAULI_C64K if prec else pk.PAULI_C128
    conv = f32 if prec else (lambda o: o)
    prev, cur, b_prev = None, conv(O0), 0.0
    Hd = uph(pk, H)
    for step in range(steps):
        want, bw, broke = oracle.lanczos_step(H, prev, cur, b_prev, t, prec, reorth=True)
        pd = pk.PauliOp.from_host(prev, dtype=dt, ws=ws) if prev is not None else None
        got, bg, gbroke = pk.lanczos_step(Hd, pd, pk.PauliOp.from_host(cur, dtype=dt, ws=ws),
                                          b_prev, T, ws=ws, reorth=True)
        assert broke == gbroke
        assert abs(bg - bw) <= 1e-12 * bw, (step, bg, bw)
        if broke:
            break
        g = got.to_host()
        assert_same_operator(g, want, rtol=1e-12 if not prec else 2e-7, what=f"step {step}")
        if prec:
            assert exact_fraction(g, want) == 1.0
        prev, cur, b_prev = cur, want, bw


def test_correlator_in_library(pk, ws):
    """S = <O0, O>/<O0, O0> from the library against the oracle's inner
    product and norm, with a non-normalised O0 of several strings."""
    say("correlator")
    n = 20
    O0 = wl.random_operator(n, 30, seed=3, density=0.2)
    O = wl.random_operator(n, 2000, seed=4, density=0.2)
    # let O contain O0's strings too
    O = wl.HostOp(n, np.concatenate([O.x, O0.x]), np.concatenate([O.z, O0.z]),
                  np.concatenate([O.coef, 0.5 * O0.coef]))
    O = oracle.canonicalize(O)
    want = oracle.inner(O0, O) / oracle.norm2(O0)
    d0, dO = pk.PauliOp.from_host(O0, ws=ws), pk.PauliOp.from_host(O, ws=ws)
    got = pk.correlator(d0, dO, ws=ws)
    assert abs(got - want) <= 1e-15 * abs(want)
    assert abs(pk.correlator(d0, d0, ws=ws) - 1.0) <= 1e-15


def _fits(pk, nbytes, fn):
    """Run fn(ws) with a workspace of exactly nbytes; no retry may happen."""
    ws = pk.Workspace(nbytes)
    before = ws.nbytes
    fn(ws)
    return ws.nbytes == before


def test_workspace_query_is_sufficient(pk):
    """A workspace of the size pauli_workspace_query returns holds the call
    (no PAULI_EWORKSPACE retry), for every kind of call."""
    n = 64
    H = uph(pk, wl.ising_chain(n))
    Oh = wl.random_local_strings(n, 20000, 10, seed=7)
    O = pk.PauliOp.from_host(Oh)
    O2 = pk.PauliOp.from_host(wl.random_local_strings(n, 5000, 10, seed=8))
    O3 = pk.PauliOp.from_host(wl.random_local_strings(n, 1200, 10, seed=10))
    assert H.size * O3.size <= 1 << 18 and H.size > 127
    T = pk.Trunc(max_len=12, max_strings=30000)
    Q = pk
    cases = [
        (Q.PAULI_Q_COMMUTATOR, H, O, None, T, lambda w: pk.commutator(H, O, T, ws=w)),
        (Q.PAULI_Q_MULTIPLY, H, O2, None, None, lambda w: pk.multiply(H, O2, ws=w)),
        (Q.PAULI_Q_ADD, O, O2, None, T, lambda w: pk.add(O, 1.0, O2, 0.5, T, ws=w)),
        (Q.PAULI_Q_TRUNCATE, None, O, None, T, lambda w: pk.truncate(O, T, ws=w)),
        (Q.PAULI_Q_CANONICALIZE, None, O, None, None, lambda w: pk.canonicalize(O, ws=w)),
        (Q.PAULI_Q_LANCZOS, H, O, O2, T,
         lambda w: pk.lanczos_step(H, O2, O, 0.7, T, ws=w)),
        (Q.PAULI_Q_LANCZOS_REORTH, H, O, O2, T,
         lambda w: pk.lanczos_step(H, O2, O, 0.7, T, ws=w, reorth=True)),
        (Q.PAULI_Q_RK4, H, O2, None, pk.Trunc(max_strings=20000),
         lambda w: pk.rk4_step(H, O2, 0.02, pk.Trunc(max_strings=20000), ws=w)),
        (Q.PAULI_Q_REDUCTION, O, O2, None, None, lambda w: pk.inner(O, O2, ws=w)),
        # small calls (at most 2^18 pairs) over 2^10 bins, H indices kept aside
        (Q.PAULI_Q_COMMUTATOR, H, O3, None, None, lambda w: pk.commutator(H, O3, ws=w)),
        (Q.PAULI_Q_MULTIPLY, H, O3, None, None, lambda w: pk.multiply(H, O3, ws=w)),
    ]
    for op, A, B, C, t, fn in cases:
        nbytes, cap = pk.workspace_query(op, A, B, C, t)
        say(f"workspace query op={op}: {nbytes / 2**20:.1f} MiB, out cap {cap}")
        assert _fits(pk, nbytes, fn), op
    H0 = uph(pk, wl.from_terms(24, [(1.0, [("X", 1), ("X", 2)]), (0.5, [("Z", 1)])]))
    Ots = pk.canonicalize_ts1d(pk.PauliOp.from_host(wl.random_local_strings(24, 3000, 6, seed=9)))
    nbytes, _ = pk.workspace_query(Q.PAULI_Q_COMMUTATOR_TS1D, H0, Ots)
    assert _fits(pk, nbytes, lambda w: pk.commutator_ts1d(H0, Ots, ws=w))


def test_small_call_planned_from_sizes(pk, ws):
    """Calls of at most 2^18 possible records are planned from their sizes:
    the host waits for the stream once per call (commutator, Lanczos step with
    its b_n and breakdown test on the device).  A workspace that holds the
    exact layout but not the layout at that bound makes the call read its
    count first (two waits), with the same result bit for bit."""
    import ctypes

    import torch

    from paper_2410_09654_amd import _lib, ops as pops
    n = 64
    H = uph(pk, wl.ising_chain(n))
    O = pk.PauliOp.from_host(wl.random_local_strings(n, 1200, 10, seed=10))
    assert H.size * O.size <= 1 << 18
    want = pk.commutator(H, O, ws=ws)
    assert pk.last_stats()["host_syncs"] == 1
    O2 = pk.PauliOp.from_host(wl.random_local_strings(n, 900, 10, seed=11))
    pk.lanczos_step(H, O2, O, 0.7, pk.Trunc(max_len=12, max_strings=5000), ws=ws)
    assert pk.last_stats()["host_syncs"] == 1
    # the workspace each failed call asks for, until the call runs
    L = _lib.load()
    nbytes, st = 1 << 20, None
    for _ in range(8):
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        wss = _lib.PauliWsC(buf.data_ptr(), nbytes, 0)
        out = pk.PauliOp(n, H.size * O.size)
        hs, os_, outs = H.c_struct(), O.c_struct(), out.c_struct()
        st = L.pauli_commutator(ctypes.byref(hs), ctypes.byref(os_), None, ctypes.byref(outs),
                                ctypes.byref(wss), pops._stream_handle())
        torch.cuda.synchronize()
        if st != _lib.PAULI_EWORKSPACE:
            break
        nbytes = int(wss.required)
    assert st == _lib.PAULI_OK
    assert pk.last_stats()["host_syncs"] == 2
    nbound, _ = pk.workspace_query(pk.PAULI_Q_COMMUTATOR, H, O)
    say(f"exact workspace {nbytes / 2**20:.1f} MiB, at the bound {nbound / 2**20:.1f} MiB")
    assert nbytes < nbound
    out.size = int(outs.size)
    assert out.size == want.size
    m = out.size
    assert torch.equal(out.x[:, :m], want.x[:, :m]) and torch.equal(out.z[:, :m], want.z[:, :m])
    assert torch.equal(out.coef[:m], want.coef[:m])


def test_keep_set_out_of_order_is_refused(pk, ws):
    """A keep set that is not in canonical order is refused with PAULI_EINVAL:
    by a small call planned from its sizes (checked with the output size), a
    call that reads its count first, a direct truncation and a Lanczos step;
    the same strings in canonical order are accepted."""
    from paper_2410_09654_amd import _lib
    n = 64
    H = uph(pk, wl.ising_chain(n))
    good = pk.PauliOp.from_host(wl.random_local_strings(n, 3, 4, seed=1), ws=ws)
    assert good.size == 3
    gx, gz, gc = good.to_numpy()  # the library's canonical order, then reversed
    bad = pk.PauliOp.from_raw(n, gx[::-1], gz[::-1], gc[::-1])
    for count in (500, 20000):
        say(f"keep out of order, |O| = {count}")
        O = pk.PauliOp.from_host(wl.random_local_strings(n, count, 10, seed=count), ws=ws)
        calls = [lambda T: pk.commutator(H, O, T, ws=ws), lambda T: pk.truncate(O, T, ws=ws),
                 lambda T: pk.lanczos_step(H, None, O, 0.0, T, ws=ws)]
        for fn in calls:
            with pytest.raises(pk.PauliError) as e:
                fn(pk.Trunc(max_strings=100, keep=bad))
            assert e.value.status == _lib.PAULI_EINVAL
            fn(pk.Trunc(max_strings=100, keep=good))


@pytest.mark.parametrize("dtype", [0, 1])
def test_checkpoint_resume_is_exact(pk, ws, tmp_path, dtype):
    """Saving the Krylov vectors to .npz and resuming the recursion from them
    gives the same b_n, bit for bit, as the uninterrupted run."""
    say(f"checkpoint resume dtype={dtype}")
    H, O0 = wl.config_lanczos_split()
    if dtype:
        O0 = f32(O0)
    Hd = uph(pk, H)
    T = pk.Trunc(max_strings=5000)
    full = pk.lanczos(Hd, pk.PauliOp.from_host(O0, dtype=dtype, ws=ws), 10, T, ws=ws)
    prev, cur, b = None, pk.PauliOp.from_host(O0, dtype=dtype, ws=ws), 0.0
    bs = []
    for k in range(10):
        if k == 5:  # checkpoint and restore
            prev.save(str(tmp_path / "prev.npz"))
            cur.save(str(tmp_path / "cur.npz"))
            prev = pk.PauliOp.load(str(tmp_path / "prev.npz"))
            cur = pk.PauliOp.load(str(tmp_path / "cur.npz"))
            assert cur.dtype == dtype
        nxt, b, _ = pk.lanczos_step(Hd, prev, cur, b, T, ws=ws)
        bs.append(b)
        prev, cur = cur, nxt
    assert bs == list(full)
