"""GPU parity of the noisy Heisenberg evolution pieces (Heisenberg section):
the depolarizing channel exp(-lambda length), the coefficient lookup behind
the two-point correlators S_{i-j}(t), and the whole noisy RK4 loop on the
next-nearest-neighbour XXZ chain, through the C ABI, against the CPU oracle.
Keys bit-exact, FP64 coefficients within 1e-12 relative."""
import math
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


def up(pk, host, ws, dtype=0):
    return pk.PauliOp.from_host(host, dtype=dtype, ws=ws)


def uph(pk, host):
    return pk.PauliOp.from_raw(host.n_qubits, host.x, host.z, host.coef)


@pytest.mark.parametrize("n,lam,seed", [(40, 0.037, 1), (100, 0.25, 2), (128, 1e-3, 3)])
def test_add_noise(pk, ws, n, lam, seed):
    say(f"add_noise n={n} lam={lam}")
    O = wl.random_operator(n, 3000, seed=seed, density=min(1.0, 8.0 / n))
    want = oracle.add_noise(O, lam)
    got = pk.add_noise(up(pk, O, ws), lam).to_host()
    assert_same_operator(got, want, rtol=0.0, what="noise")
    # FP32: scaled in double, rounded once
    O32 = up(pk, O, ws, dtype=pk.PAULI_C64K)
    c32 = O32.to_host()
    got32 = pk.add_noise(O32, lam).to_host()
    d = {k: v for k, v in zip(c32.keys(), c32.coef)}
    W = O.x.shape[1]
    for k, v in zip(got32.keys(), got32.coef):
        ln = sum(bin(int(k[w]) | int(k[W + w])).count("1") for w in range(W))
        f = math.exp(-lam * ln)
        w = d[k]
        assert v.real == np.float32(w.real * f) and v.imag == np.float32(w.imag * f)


def test_coefficients_lookup(pk, ws):
    say("coefficients lookup")
    for n in (64, 128):
        A = wl.random_operator(n, 4000, seed=n, density=0.1)
        Qa = wl.random_operator(n, 300, seed=n + 1, density=0.1)
        # half present, half (very likely) absent
        Q = wl.HostOp(n, np.concatenate([A.x[::13], Qa.x]), np.concatenate([A.z[::13], Qa.z]),
                      np.ones(len(A.x[::13]) + Qa.n, complex))
        Ad = up(pk, A, ws)
        got = pk.coefficients(Ad, pk.PauliOp.from_raw(n, Q.x, Q.z, Q.coef), ws=ws)
        want = oracle.coefficients(A, Q)
        assert np.array_equal(got, want)
        assert np.count_nonzero(got) >= len(A.x[::13])


def test_noisy_evolution_matches_oracle(pk, ws):
    """XXZnnn N=10, O0 = Z_1, dt = 0.05, 20 steps, M = 300, eps = 0.05."""
    say("noisy evolution N=10")
    n, dt, steps, M, eps = 10, 0.05, 20, 300, 0.05
    H = wl.xxz_nnn(n)
    O0 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    probes = wl.from_terms(n, [(1.0, [("Z", j)]) for j in range(1, n + 1)])
    want_O, want_S, want_P = oracle.evolve_noisy(H, O0, dt, steps, M, eps, probes)
    got_O, got_S, got_P = pk.evolve_noisy(uph(pk, H), up(pk, O0, ws), dt, steps, M, eps,
                                          probes=pk.PauliOp.from_raw(n, probes.x, probes.z,
                                                                     probes.coef), ws=ws)
    g = got_O.to_host()
    assert g.n == want_O.n
    assert_same_operator(g, want_O, what="noisy O(t)")
    assert exact_fraction(g, want_O) > 0.9
    assert np.allclose(got_S, want_S, rtol=1e-12, atol=1e-15)
    assert np.allclose(np.array(got_P), np.array(want_P), rtol=1e-12, atol=1e-15)


def test_noisy_evolution_total_z_invariant(pk, ws):
    """Untruncated, N=10 (at most 4^10 strings): n(t_k) = sum_j S_{1,j}(t_k)
    = exp(-eps k dt)."""
    say("noisy evolution invariant N=10")
    n, dt, steps, eps = 10, 0.1, 8, 0.1
    H = wl.xxz_nnn(n)
    O0 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    probes = wl.from_terms(n, [(1.0, [("Z", j)]) for j in range(1, n + 1)])
    _, S, P = pk.evolve_noisy(uph(pk, H), up(pk, O0, ws), dt, steps, 0, eps,
                              probes=pk.PauliOp.from_raw(n, probes.x, probes.z, probes.coef),
                              ws=ws)
    for k in range(steps + 1):
        assert abs(sum(P[k]) - math.exp(-eps * k * dt)) < 1e-12, k
        assert S[k] == P[k][0]


def test_coefficients_lookup_fp32_operand(pk, ws):
    """An FP32 operand (PAULI_C64K): the looked-up values are its stored
    floats, widened exactly."""
    say("coefficients lookup fp32")
    n = 100
    A = wl.random_operator(n, 3000, seed=5, density=0.1)
    Q = wl.HostOp(n, A.x[::7], A.z[::7], np.ones(len(A.x[::7]), complex))
    A32 = up(pk, A, ws, dtype=pk.PAULI_C64K)
    got = pk.coefficients(A32, pk.PauliOp.from_raw(n, Q.x, Q.z, Q.coef), ws=ws)
    h = A32.to_host()
    d = {k: v for k, v in zip(h.keys(), h.coef)}
    want = np.array([d.get(k, 0j) for k in Q.keys()])
    assert np.array_equal(got, want)
    assert np.array_equal(want, A.coef[::7].astype(np.complex64).astype(np.complex128))


@pytest.mark.parametrize("dtype", [0, 1])
def test_dagger_conjugates_in_place(pk, ws, dtype):
    """pauli_dagger: the same strings in the same order, every coefficient
    conjugated (bit for bit); Tr(B A^dagger)/2^N from the product's identity
    coefficient equals <A, B>."""
    say(f"dagger dtype={dtype}")
    n = 20
    A = wl.random_operator(n, 3000, seed=41, density=0.2)
    B = wl.HostOp(n, A.x[:1500], A.z[:1500], A.coef[1000:2500] * (0.3 - 0.7j))
    if dtype:
        A.coef = A.coef.astype(np.complex64).astype(np.complex128)
    Ad = up(pk, A, ws, dtype=dtype)
    before = Ad.to_host()
    pk.dagger(Ad)
    after = Ad.to_host()
    assert np.array_equal(after.x, before.x) and np.array_equal(after.z, before.z)
    assert np.array_equal(after.coef, np.conj(before.coef))
    if dtype == 0:
        Bd = up(pk, B, ws)
        prod = pk.multiply(Bd, Ad, ws=ws)  # Tr(B A^dagger) = Tr(A^dagger B)
        tr = pk.trace(prod, ws=ws)
        pk.dagger(Ad)  # back to A
        ip = pk.inner(Ad, Bd, ws=ws)
        assert abs(tr - ip) <= 1e-12 * max(1.0, abs(ip))
