"""GPU parity of the translation-symmetric operators of Alg. 2 (periodic
chain, one representative string per translation orbit) through the C ABI,
against the CPU oracle: representatives, the commutator over translates, the
stabilizer-weighted norm and the Lanczos recursion built on them.  Keys
bit-exact, FP64 coefficients within 1e-12 relative."""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import assert_canonical_unique, assert_same_operator, exact_fraction, gpu_available

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


def up(pk, host, ws, dtype=0):
    return pk.PauliOp.from_host(host, dtype=dtype, ws=ws)


def raw(pk, host):
    return pk.PauliOp.from_raw(host.n_qubits, host.x, host.z, host.coef)


def chain_h0(n):
    """Terms of a chaotic periodic chain plus a longer-range one: H = sum_k T_k(H0)."""
    return wl.from_terms(n, [(1.0, [("Z", 1), ("Z", 2)]), (1.05, [("X", 1)]), (0.5, [("Z", 1)]),
                             (0.3, [("X", 1), ("Y", 3)]), (0.2, [("Y", 1), ("Z", 2), ("X", 4)])])


@pytest.mark.parametrize("n,seed", [(8, 1), (64, 2), (100, 3), (128, 4)])
def test_canonicalize_ts1d(pk, ws, n, seed):
    say(f"ts canonicalize n={n}")
    A = wl.random_operator(n, 800, seed=seed, density=min(1.0, 4.0 / n))
    # add translates of some strings so that orbits collide
    T = oracle.expand_ts(wl.HostOp(n, A.x[:3], A.z[:3], A.coef[:3]))
    B = wl.HostOp(n, np.concatenate([A.x, T.x]), np.concatenate([A.z, T.z]),
                  np.concatenate([A.coef, T.coef]))
    want = oracle.canonicalize_ts(B)
    got = pk.canonicalize_ts1d(raw(pk, B), ws=ws).to_host()
    assert_canonical_unique(got)
    assert_same_operator(got, want, what="ts representatives")


@pytest.mark.parametrize("n,no,seed", [(8, 40, 11), (20, 400, 12), (64, 3000, 13),
                                       (100, 1500, 14), (128, 800, 15)])
def test_commutator_ts1d(pk, ws, n, no, seed):
    say(f"ts commutator n={n} no={no}")
    H0 = chain_h0(n)
    O0 = oracle.canonicalize_ts(wl.random_local_strings(n, no, min(8, n), seed=seed))
    want = oracle.commutator_ts(H0, O0)
    got = pk.commutator_ts1d(raw(pk, H0), up(pk, O0, ws), ws=ws).to_host()
    assert_canonical_unique(got)
    assert_same_operator(got, want, what="ts commutator")
    assert exact_fraction(got, want) == 1.0
    # truncated (top-M with the length cap)
    t = oracle.Trunc(max_len=6, max_strings=max(1, want.n // 3))
    want_t = oracle.truncate(want, t)
    got_t = pk.commutator_ts1d(raw(pk, H0), up(pk, O0, ws),
                               pk.Trunc(max_len=6, max_strings=max(1, want.n // 3)),
                               ws=ws).to_host()
    assert_same_operator(got_t, want_t, what="truncated ts commutator")


def test_norm2_ts1d(pk, ws):
    say("ts norm")
    for n in (8, 64, 100):
        A0 = oracle.canonicalize_ts(wl.from_terms(n, [
            (0.5 + 0.25j, [("Z", 1), ("Z", 2)]), (1.5, [("X", 1)]),
            (0.75, [("X", j) for j in range(1, n + 1, 2)]),
            (-0.4j, [("Z", j) for j in range(1, n + 1)]),
            (0.1, [("Y", j) for j in range(1, n + 1, 4)] if n % 4 == 0 else [("Y", 2)])]))
        R = oracle.canonicalize_ts(wl.random_operator(n, 500, seed=n, density=min(1.0, 4.0 / n)))
        for op in (A0, R):
            want = oracle.norm2_ts(op)
            got = pk.norm2_ts1d(up(pk, op, ws), ws=ws)
            assert abs(got - want) <= 1e-15 * want


def test_lanczos_ts1d_matches_oracle_and_full_chain(pk, ws):
    say("ts lanczos")
    n, steps = 20, 12
    H0 = chain_h0(n)
    Z1 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    t = oracle.Trunc(max_strings=3000)
    want = oracle.lanczos_ts(H0, Z1, steps, t)
    got = pk.lanczos_ts1d(raw(pk, H0), up(pk, Z1, ws), steps, pk.Trunc(max_strings=3000), ws=ws)
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    # untruncated: the same b_n as the plain recursion on the full periodic chain
    n = 10
    H0 = chain_h0(n)
    Z1 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    b_ts = pk.lanczos_ts1d(raw(pk, H0), up(pk, Z1, ws), 8, ws=ws)
    Hf = oracle.expand_ts(H0)
    Of = wl.single_site_sum(n, "Z", 1 / math.sqrt(n))
    b_full = pk.lanczos(raw(pk, Hf), up(pk, Of, ws), 8, ws=ws)
    assert np.allclose(b_ts, b_full, rtol=1e-12, atol=0)


def test_lanczos_ts1d_xx_chain_closed_form(pk, ws):
    """Periodic XX chain, N = 50, O0 = sum_j X_j / sqrt(N): b_n = sqrt(8n)
    (Gaussian autocorrelation exp(-4t^2)) for n <= 24, untruncated."""
    say("ts lanczos XX N=50 closed form")
    n, steps = 50, 24
    H0 = wl.from_terms(n, [(1.0, [("X", 1), ("X", 2)]), (1.0, [("Y", 1), ("Y", 2)])])
    X1 = wl.from_terms(n, [(1.0, [("X", 1)])])
    b = pk.lanczos_ts1d(raw(pk, H0), up(pk, X1, ws), steps, ws=ws)
    assert np.allclose(np.array(b) ** 2, 8.0 * np.arange(1, steps + 1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("name", ["xxx", "chaotic"])
def test_lanczos_ts1d_paper_chains_match_oracle(pk, ws, name):
    """The XXX chain with O0 ~ sum_j X_j Y_j+1 - Y_j X_j+1 and the chaotic
    chain {XX, -1.05 Z, 0.5 X} with O0 ~ sum_j 1.05 X_j X_j+1 + Z_j, N = 50,
    10 steps at M = 2^10."""
    say(f"ts lanczos {name} N=50")
    n = 50
    if name == "xxx":
        h = [(1.0, [(p, 1), (p, 2)]) for p in "XYZ"]
        o = [(1.0, [("X", 1), ("Y", 2)]), (-1.0, [("Y", 1), ("X", 2)])]
    else:
        h = [(1.0, [("X", 1), ("X", 2)]), (-1.05, [("Z", 1)]), (0.5, [("X", 1)])]
        o = [(1.05, [("X", 1), ("X", 2)]), (1.0, [("Z", 1)])]
    H0, O0 = wl.from_terms(n, h), wl.from_terms(n, o)
    O0.coef /= math.sqrt(oracle.norm2_ts(O0))
    want = oracle.lanczos_ts(H0, O0, 10, oracle.Trunc(max_strings=1 << 10))
    got = pk.lanczos_ts1d(raw(pk, H0), up(pk, O0, ws), 10, pk.Trunc(max_strings=1 << 10), ws=ws)
    assert np.allclose(got, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,M", [(20, 0), (64, 500), (100, 300)])
def test_lanczos_step_ts1d_operator(pk, ws, n, M):
    """One fused step O_{n-2}, O_{n-1} -> O_n (representatives, truncated to M
    when M > 0) equals the oracle's step, keys bit-exact; b_n within 1e-12."""
    say(f"ts lanczos step n={n} M={M}")
    H0 = chain_h0(n)
    t = oracle.Trunc(max_strings=M) if M else oracle.NO_TRUNC
    tg = pk.Trunc(max_strings=M) if M else None
    Z1 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    O1, b1, _ = oracle.lanczos_step_ts(H0, None, Z1, 0.0, t)
    O2, b2, _ = oracle.lanczos_step_ts(H0, Z1, O1, b1, t)
    O3, b3, _ = oracle.lanczos_step_ts(H0, O1, O2, b2, t)
    got, bg, broke = pk.lanczos_step(raw(pk, H0), up(pk, O1, ws), up(pk, O2, ws), b2, tg,
                                     ws=ws, ts1d=True)
    assert not broke
    assert abs(bg - b3) <= 1e-12 * b3
    g = got.to_host()
    assert_canonical_unique(g)
    assert_same_operator(g, O3, what="ts lanczos step")


@pytest.mark.parametrize("n", [8, 64, 100])
def test_lanczos_step_ts1d_periodic_strings_in_norm(pk, ws, n):
    """The fused step's norm weights every representative by its stabilizer
    count: O_prev holds strings of period 1, 2 and 4, which reach O'_n
    through -b_prev O_prev; b_n and O_n equal the oracle's step."""
    say(f"ts lanczos step, periodic strings, n={n}")
    H0 = chain_h0(n)
    P = oracle.canonicalize_ts(wl.from_terms(n, [
        (0.6, [("Z", j) for j in range(1, n + 1)]),                 # period 1
        (-0.3j, [("X", j) for j in range(1, n + 1, 2)]),            # period 2
        (0.25, [("Y", j) for j in range(1, n + 1, 4)]),             # period 4
        (0.4, [("X", 1), ("Z", 2)])]))
    C = oracle.canonicalize_ts(wl.random_local_strings(n, 60, min(6, n), seed=n))
    want, bw, _ = oracle.lanczos_step_ts(H0, P, C, 0.7)
    got, bg, broke = pk.lanczos_step(raw(pk, H0), up(pk, P, ws), up(pk, C, ws), 0.7, ws=ws,
                                     ts1d=True)
    assert not broke
    assert abs(bg - bw) <= 1e-12 * bw
    assert_same_operator(got.to_host(), want, what="ts step with periodic strings")


def test_commutator_ts1d_fp32(pk, ws):
    """FP32 coefficients (PAULI_C64K, Kahan sums): the same representatives as
    the FP64 oracle on the FP32-rounded input, values within FP32 rounding."""
    say("ts commutator fp32 n=64")
    n = 64
    H0 = chain_h0(n)
    O0 = oracle.canonicalize_ts(wl.random_local_strings(n, 2000, 8, seed=77))
    O0 = wl.HostOp(n, O0.x, O0.z, O0.coef.astype(np.complex64).astype(np.complex128))
    want = oracle.commutator_ts(H0, O0)
    got = pk.commutator_ts1d(raw(pk, H0), up(pk, O0, ws, dtype=pk.PAULI_C64K), ws=ws).to_host()
    assert_same_operator(got, want, rtol=1e-5, what="fp32 ts commutator")
    n2 = pk.norm2_ts1d(up(pk, O0, ws, dtype=pk.PAULI_C64K), ws=ws)
    assert abs(n2 - oracle.norm2_ts(O0)) <= 1e-12 * n2
