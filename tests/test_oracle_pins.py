"""Pins of the CPU oracle against facts that do not come from the oracle:
textbook Pauli matrices, dense 2^N matrices, exactly rounded sums, the paper's
printed worked example, closed forms of Lanczos coefficients and of one
Runge-Kutta step.  CPU only.
"""
import ctypes
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as wl

SIGMA = {
    (0, 0): np.eye(2, dtype=complex),
    (1, 0): np.array([[0, 1], [1, 0]], dtype=complex),
    (0, 1): np.array([[1, 0], [0, -1]], dtype=complex),
    (1, 1): np.array([[0, -1j], [1j, 0]], dtype=complex),
}


def site_bits(key, W, j):
    w, b = divmod(int(j), 64)
    return ((key[w] >> b) & 1, (key[W + w] >> b) & 1)


def dense_string(n, key):
    W = wl.n_words(n)
    m = np.array([[1.0 + 0j]])
    for j in range(n):  # site 1 is the leftmost Kronecker factor
        m = np.kron(m, SIGMA[site_bits(key, W, j)])
    return m


def dense(op: wl.HostOp):
    d = 2 ** op.n_qubits
    m = np.zeros((d, d), complex)
    for k, c in zip(op.keys(), op.coef):
        m += c * dense_string(op.n_qubits, k)
    return m


def sparse_string(n, key):
    W = wl.n_words(n)
    m = sp.identity(1, dtype=complex, format="csr")
    for j in range(n):
        m = sp.kron(m, sp.csr_matrix(SIGMA[site_bits(key, W, j)]), format="csr")
    return m


def sparse_op(op):
    d = 2 ** op.n_qubits
    m = sp.csr_matrix((d, d), dtype=complex)
    for k, c in zip(op.keys(), op.coef):
        m = m + c * sparse_string(op.n_qubits, k)
    return m


# ---------------------------------------------------------------------------
# String algebra
# ---------------------------------------------------------------------------

def test_single_site_table_matches_pauli_matrices():
    for a in SIGMA:
        for b in SIGMA:
            ka, kb = (a[0], a[1]), (b[0], b[1])
            c, k = oracle.string_product(1, ka, kb)
            lhs = SIGMA[a] @ SIGMA[b]
            rhs = (1j ** k) * SIGMA[(c[0], c[1])]
            assert np.allclose(lhs, rhs, atol=0), (a, b, c, k)


def test_named_products():
    X, Y, Z = (1, 0), (1, 1), (0, 1)
    for a, b, c, k in [(X, Y, Z, 1), (Y, Z, X, 1), (Z, X, Y, 1),
                       (Y, X, Z, 3), (Z, Y, X, 3), (X, Z, Y, 3)]:
        assert oracle.string_product(1, a, b) == (c, k)


@pytest.mark.parametrize("n", [3, 5, 70])
def test_string_products_vs_kron(n):
    rng = np.random.default_rng(n)
    A = wl.random_operator(n, 12, seed=n, density=0.6)
    B = wl.random_operator(n, 12, seed=n + 100, density=0.6)
    for ka in A.keys():
        for kb in B.keys():
            kc, k = oracle.string_product(n, ka, kb)
            if n <= 5:
                assert np.allclose(dense_string(n, ka) @ dense_string(n, kb),
                                   (1j ** k) * dense_string(n, kc), atol=0)
            else:  # site-wise check on wide strings: the phase multiplies over sites
                W = wl.n_words(n)
                ph = 0
                for j in rng.permutation(n):
                    a, b = site_bits(ka, W, j), site_bits(kb, W, j)
                    c1, k1 = oracle.string_product(1, a, b)
                    assert site_bits(kc, W, j) == c1
                    ph += k1
                assert ph % 4 == k


# ---------------------------------------------------------------------------
# Operator algebra vs dense matrices
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(2, 1), (4, 2), (5, 3), (6, 4)])
def test_commutator_vs_dense(n, seed):
    H = wl.random_operator(n, 7, seed=seed, density=0.5)
    O = wl.random_operator(n, 9, seed=seed + 50, density=0.7)
    C = oracle.commutator(H, O)
    dH, dO = dense(H), dense(O)
    assert np.abs(dense(C) - (dH @ dO - dO @ dH)).max() < 1e-12
    assert all(abs(c) > 0 for c in C.coef)
    assert len(set(C.keys())) == C.n


@pytest.mark.parametrize("n,seed", [(3, 5), (5, 6)])
def test_product_vs_dense(n, seed):
    A = wl.random_operator(n, 6, seed=seed)
    B = wl.random_operator(n, 5, seed=seed + 1)
    assert np.abs(dense(oracle.product(A, B)) - dense(A) @ dense(B)).max() < 1e-12


@pytest.mark.parametrize("n,seed", [(2, 21), (4, 22), (6, 23)])
def test_trace_vs_dense(n, seed):
    """Tr(O)/2^N from the matrix, for operators with and without the identity."""
    O = wl.random_operator(n, 9, seed=seed, density=0.6)
    assert abs(oracle.trace(O) - np.trace(dense(O)) / 2 ** n) < 1e-13
    I = wl.HostOp(n, np.zeros((1, O.x.shape[1]), np.uint64), np.zeros((1, O.x.shape[1]), np.uint64),
                  np.array([0.25 - 0.5j]))
    OI = oracle.add(O, 1.0, I, 1.0)
    assert abs(oracle.trace(OI) - np.trace(dense(OI)) / 2 ** n) < 1e-13


@pytest.mark.parametrize("n", [4, 6])
def test_moments_vs_dense_matrix_powers(n):
    """mu_k = Tr(H^k)/2^N of the chaotic Ising chain against matrix powers;
    mu_1 = 0 (traceless) and mu_2 = sum of squared coefficients (Hermitian H)."""
    H = wl.ising_chain(n, hx=1.05, hz=0.5)
    mus = oracle.moments(H, 6)
    dH = dense(H)
    P = np.eye(2 ** n, dtype=complex)
    for k in range(1, 7):
        P = P @ dH
        want = np.trace(P) / 2 ** n
        assert abs(mus[k - 1] - want) <= 1e-12 * max(1.0, abs(want)), k
    assert abs(mus[0]) == 0.0
    assert abs(mus[1] - float(np.sum(np.abs(H.coef) ** 2))) < 1e-12


@pytest.mark.parametrize("n,lam,seed", [(2, 0.3, 61), (3, 0.05, 62), (4, 1.1, 63)])
def test_noise_vs_dense_depolarizing_channel(n, lam, seed):
    """Per-string factor exp(-lam * length) equals the product of single-qubit
    depolarizing channels (1-p) M + p/3 (X M X + Y M Y + Z M Z) with
    1 - 4p/3 = exp(-lam), applied to the dense matrix."""
    O = wl.random_operator(n, 12, seed=seed, density=0.7)
    M = dense(O)
    p = 3.0 * (1.0 - math.exp(-lam)) / 4.0
    for q in range(1, n + 1):
        P = [dense(wl.from_terms(n, [(1.0, [(s, q)])])) for s in "XYZ"]
        M = (1 - p) * M + (p / 3) * sum(Pk @ M @ Pk for Pk in P)
    assert np.abs(dense(oracle.add_noise(O, lam)) - M).max() < 1e-13


def test_noisy_evolution_total_z_decays_as_exp():
    """XXZnnn conserves total Z, RK4 stages are commutators and the channel
    scales the weight-1 strings by exp(-eps dt): n(t_k) = sum_j Tr[Z_1(t_k)
    Z_j]/2^N = exp(-eps k dt) exactly (no truncation), while S(t) decays."""
    n, eps, dt, steps = 8, 0.2, 0.1, 10
    H = wl.xxz_nnn(n)
    O0 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    probes = wl.from_terms(n, [(1.0, [("Z", j)]) for j in range(1, n + 1)])
    _, S, P = oracle.evolve_noisy(H, O0, dt, steps, 0, eps, probes)
    for k in range(steps + 1):
        assert abs(sum(P[k]) - math.exp(-eps * k * dt)) < 1e-12, k
        assert abs(S[k] - P[k][0]) < 1e-15
    assert abs(S[-1]) < 0.95 * math.exp(-eps * steps * dt)


# ---------------------------------------------------------------------------
# Translation-symmetric operators (Alg. 2)
# ---------------------------------------------------------------------------
def _bits(op, k):
    W = op.x.shape[1]
    x = sum(int(op.x[k][w]) << (64 * w) for w in range(W))
    z = sum(int(op.z[k][w]) << (64 * w) for w in range(W))
    return x, z


def _rot(v, k, n):
    """site j -> site (j + k) mod n of an n-bit integer"""
    k %= n
    return ((v << k) | (v >> (n - k))) & ((1 << n) - 1) if k else v


def _w2(v):
    return (ctypes.c_uint64 * 2)(v & (2 ** 64 - 1), v >> 64)


@pytest.mark.parametrize("n,seed", [(6, 81), (10, 82), (64, 83), (70, 84)])
def test_ts_representative_brute_force(n, seed):
    """Shiftleft: the same representative for every translate, and it is the
    rotation with the smallest (occupied pattern, x, z) as n-bit numbers."""
    O = wl.random_operator(n, 40, seed=seed, density=min(1.0, 4.0 / n))
    for k in range(O.n):
        x, z = _bits(O, k)
        best = min(((_rot(x, r, n) | _rot(z, r, n)), _rot(x, r, n), _rot(z, r, n))
                   for r in range(n))
        for r in (0, 1, n // 2, n - 1):
            cx, cz = oracle.ts_representative(n, _w2(_rot(x, r, n)), _w2(_rot(z, r, n)))
            got = (int(cx[0]) | int(cx[1]) << 64, int(cz[0]) | int(cz[1]) << 64)
            assert got == (best[1], best[2])
        assert best[0] & 1  # the representative starts on the first site


@pytest.mark.parametrize("n,seed", [(6, 91), (8, 92)])
def test_ts_commutator_expands_to_full_commutator(n, seed):
    """The Alg. 2 commutator of representatives, expanded over translations,
    equals the plain commutator of the expanded operators."""
    H0 = wl.from_terms(n, [(1.0, [("Z", 1), ("Z", 2)]), (1.05, [("X", 1)]), (0.5, [("Z", 1)]),
                           (0.3, [("X", 1), ("Y", 3)])])
    O0 = oracle.canonicalize_ts(wl.random_operator(n, 15, seed=seed, density=0.5))
    want = oracle.commutator(oracle.expand_ts(H0), oracle.expand_ts(O0))
    got = oracle.expand_ts(oracle.commutator_ts(H0, O0))
    gd, wd = got.as_dict(), want.as_dict()
    assert set(gd) == set(wd)
    for k, v in wd.items():
        assert abs(gd[k] - v) <= 1e-12 * max(1.0, abs(v))


def test_ts_norm_is_full_norm_over_n():
    """norm2_ts(A0) = ||sum_k T_k(A0)||^2 / N, strings with a nontrivial
    stabilizer (period 2 and 1) included."""
    n = 8
    A0 = oracle.canonicalize_ts(wl.from_terms(n, [
        (0.5 + 0.25j, [("Z", 1), ("Z", 2)]), (1.5, [("X", 1)]),
        (0.75, [("X", j) for j in range(1, n + 1, 2)]),       # period 2
        (-0.4j, [("Z", j) for j in range(1, n + 1)])]))        # period 1
    assert abs(oracle.norm2_ts(A0) - oracle.norm2(oracle.expand_ts(A0)) / n) < 1e-13


def test_ts_lanczos_equals_full_periodic_lanczos():
    """b_n of the translation-symmetric recursion (O0 = Z_1 as representative)
    equal those of the plain recursion on the periodic chain with
    O0 = sum_j Z_j / sqrt(N) (the norm's factor N drops out of the b_n)."""
    n = 8
    H0 = wl.from_terms(n, [(1.0, [("Z", 1), ("Z", 2)]), (1.05, [("X", 1)]), (0.5, [("Z", 1)])])
    Z1 = wl.from_terms(n, [(1.0, [("Z", 1)])])
    b_ts = oracle.lanczos_ts(H0, Z1, 8)
    Of = wl.single_site_sum(n, "Z", 1 / math.sqrt(n))
    b_full = oracle.lanczos(oracle.expand_ts(H0), Of, 8)
    assert len(b_ts) == len(b_full) == 8
    assert np.allclose(b_ts, b_full, rtol=1e-12, atol=0)


def _xx_periodic_dense(n):
    """sum_j X_j X_j+1 + Y_j Y_j+1 (sites mod n) and sum_j X_j / sqrt(n) as dense matrices."""
    d = 2 ** n

    def site(p, j):
        m = np.array([[1.0 + 0j]])
        for s in range(n):
            m = np.kron(m, p if s == j else np.eye(2))
        return m
    X, Y = SIGMA[(1, 0)], SIGMA[(1, 1)]
    H = np.zeros((d, d), complex)
    for j in range(n):
        H += site(X, j) @ site(X, (j + 1) % n) + site(Y, j) @ site(Y, (j + 1) % n)
    O = sum(site(X, j) for j in range(n)) / math.sqrt(n)
    return H, O


def test_xx_chain_gaussian_lanczos_closed_form():
    """Periodic XX chain with O0 = sum_j X_j / sqrt(N): the infinite-temperature
    autocorrelation of X_j is the Gaussian exp(-4t^2) (a free-fermion result),
    whose Lanczos coefficients are b_n = sqrt(8n) while the operator's support
    fits in the ring.  Checked first by a dense Lanczos recursion (N = 8,
    Tr(A^dag B)/2^N), then on the oracle's translation-symmetric recursion
    (Alg. 2 commutator and stabilizer-weighted norm) at N = 8 and N = 20."""
    n = 8
    H, O = _xx_periodic_dense(n)
    d = 2 ** n
    prev, cur, b_prev, bd = np.zeros_like(O), O, 0.0, []
    for _ in range(4):
        nxt = H @ cur - cur @ H - b_prev * prev
        b = math.sqrt(np.vdot(nxt, nxt).real / d)
        bd.append(b)
        prev, cur, b_prev = cur, nxt / b, b
    assert np.allclose(np.array(bd) ** 2, 8.0 * np.arange(1, 5), rtol=1e-12, atol=0)
    for n, steps in ((8, 4), (20, 10)):
        H0 = wl.from_terms(n, [(1.0, [("X", 1), ("X", 2)]), (1.0, [("Y", 1), ("Y", 2)])])
        X1 = wl.from_terms(n, [(1.0, [("X", 1)])])
        b_ts = oracle.lanczos_ts(H0, X1, steps)
        assert np.allclose(np.array(b_ts) ** 2, 8.0 * np.arange(1, steps + 1), rtol=1e-12, atol=0)


def test_chunked_commutator_equals_commutator():
    """The full-size helper (chunks of O, summed by linearity) gives the same
    strings as the plain commutator and coefficients equal to rounding."""
    H = wl.ising_chain(64)
    O = wl.random_local_strings(64, 6000, 10, seed=12)
    a, b = oracle.commutator(H, O).as_dict(), oracle.commutator_chunked(H, O, threads=4,
                                                                       chunks=7).as_dict()
    assert set(a) == set(b)
    assert max(abs(a[k] - b[k]) / max(1.0, abs(a[k])) for k in a) <= 1e-14


def test_add_norm_inner_vs_dense():
    n = 5
    A = wl.random_operator(n, 20, seed=11)
    B = wl.random_operator(n, 25, seed=12)
    B.coef[:5] = A.coef[:5]
    B.x[:5], B.z[:5] = A.x[:5], A.z[:5]  # force common keys
    B = oracle.canonicalize(B)
    al, be = 0.7 - 0.2j, -1.3 + 0.5j
    S = oracle.add(A, al, B, be)
    assert np.abs(dense(S) - (al * dense(A) + be * dense(B))).max() < 1e-12
    d = 2 ** n
    dA, dB = dense(A), dense(B)
    assert abs(oracle.norm2(A) - np.trace(dA.conj().T @ dA).real / d) < 1e-12
    assert abs(oracle.inner(A, B) - np.trace(dA.conj().T @ dB) / d) < 1e-12


def test_add_exact_cancellation_drops_string():
    n = 4
    A = wl.random_operator(n, 10, seed=3)
    S = oracle.add(A, 1.0, A, -1.0)
    assert S.n == 0


def test_canonicalize_sums_duplicates():
    n = 4
    A = wl.random_operator(n, 10, seed=21)
    dup = wl.HostOp(n, np.concatenate([A.x, A.x[:4]]), np.concatenate([A.z, A.z[:4]]),
                    np.concatenate([A.coef, A.coef[:4] * 2]))
    C = oracle.canonicalize(dup)
    assert C.n == A.n
    assert np.abs(dense(C) - dense(dup)).max() < 1e-12


# ---------------------------------------------------------------------------
# Exact summation (pinned to Python's correctly rounded math.fsum)
# ---------------------------------------------------------------------------

def test_exact_sum_matches_fsum():
    rng = np.random.default_rng(0)
    for trial in range(60):
        n = int(rng.integers(1, 400))
        scale = 10.0 ** rng.integers(-300, 300, size=n)
        v = rng.standard_normal(n) * scale
        if trial % 3 == 0:  # heavy cancellation
            v = np.concatenate([v, -v[: n // 2], rng.standard_normal(3) * 1e-200])
        if trial % 5 == 0:
            v = np.concatenate([v, [5e-324, -5e-324, 2.2250738585072014e-308]])
        assert oracle.exact_sum(v) == math.fsum(v.tolist())
    assert oracle.exact_sum([1.0, 2.0 ** -53, 2.0 ** -53]) == math.fsum([1.0, 2.0 ** -53, 2.0 ** -53])
    assert oracle.exact_sum([]) == 0.0


def test_norm2_is_exactly_rounded_sum_of_weights():
    A = wl.random_operator(6, 300, seed=8)
    m2 = [c.real * c.real + c.imag * c.imag for c in A.coef]
    assert oracle.norm2(A) == math.fsum(m2)


# ---------------------------------------------------------------------------
# Lanczos: the paper's worked example, closed forms, dense recursion
# ---------------------------------------------------------------------------

def load_worked_example():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "worked_example_lanczos.txt")
    steps = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        s, re, im, text = line.split()
        steps.setdefault(int(s), []).append((complex(float(re), float(im)), text))
    return steps


def test_worked_example_verbatim():
    golden = load_worked_example()
    n = 10
    H = wl.xx_plus_zz_defect(n, 4)
    O0 = wl.from_terms(n, [(1.0, [("X", 1)])])
    bs, basis = oracle.lanczos(H, O0, 7, oracle.Trunc(coef_eps=1e-10), keep_basis=True)
    for step in range(1, 8):
        got = {wl.text_of_key(n, k): c for k, c in zip(basis[step - 1].keys(),
                                                       basis[step - 1].coef)}
        want = dict((t, c) for c, t in golden[step])
        assert set(got) == set(want), step
        for t in want:
            assert abs(got[t] - want[t]) < 1e-10, (step, t)
    # b_n of that run: 2, 2, 2, 2 sqrt2, 2 sqrt3, 2 sqrt(25/6)
    expect = [2, 2, 2, 2 * math.sqrt(2), 2 * math.sqrt(3), 2 * math.sqrt(25 / 6)]
    assert np.allclose(bs[:6], expect, rtol=1e-14)


def test_config_small_closed_form_and_dense():
    H, O0, steps = wl.config_lanczos_small()
    bs, basis = oracle.lanczos(H, O0, steps, keep_basis=True)
    assert bs[0] == pytest.approx(2.1, rel=1e-15)          # [H,Z1] = 2*1.05*(-i)Y1
    assert bs[1] == pytest.approx(math.sqrt(5), rel=1e-15)  # O'_2 = -2 X1 Z2 - X1 (up to phase)
    # dense Liouvillian recursion at N = 12 (sparse H, dense operators)
    n = 12
    Hs = sparse_op(H)
    d = 2 ** n
    prev = None
    cur = sparse_op(O0).toarray()
    b_prev = 0.0
    dense_b = []
    for _ in range(steps):
        A = np.asarray(Hs @ cur) - np.asarray(cur @ Hs)
        if prev is not None:
            A = A - b_prev * prev
        b = math.sqrt(np.vdot(A, A).real / d)
        dense_b.append(b)
        prev, cur, b_prev = cur, A / b, b
    assert np.allclose(bs, dense_b, rtol=1e-13, atol=0)
    # Krylov basis orthonormal; coefficients alternate real / imaginary
    for m in range(len(basis)):
        for k in range(m, min(len(basis), m + 3)):
            ip = oracle.inner(basis[m], basis[k])
            assert abs(ip - (1.0 if m == k else 0.0)) < 1e-12
    for m, B in enumerate(basis):
        if m % 2 == 0:
            assert np.all(B.coef.imag == 0)
        else:
            assert np.all(B.coef.real == 0)


def test_dense_lanczos_random_small():
    n = 5
    H = wl.random_operator(n, 10, seed=31, real=True)
    O0 = wl.from_terms(n, [(1.0, [("Z", 2)])])
    bs = oracle.lanczos(H, O0, 8)
    dH = dense(H)
    d = 2 ** n
    prev, cur, b_prev, ref = None, dense(O0), 0.0, []
    for _ in range(len(bs)):
        A = dH @ cur - cur @ dH
        if prev is not None:
            A = A - b_prev * prev
        b = math.sqrt(np.vdot(A, A).real / d)
        ref.append(b)
        prev, cur, b_prev = cur, A / b, b
    assert np.allclose(bs, ref, rtol=1e-11)


def test_reorth_is_a_noop_untruncated():
    """Without truncation the Krylov vectors are orthogonal, so the local
    re-orthogonalisation changes nothing: config 1's b_1..b_12 agree to
    1e-15."""
    H, O0, steps = wl.config_lanczos_small()
    plain = oracle.lanczos(H, O0, steps)
    ro = oracle.lanczos(H, O0, steps, reorth=True)
    assert len(ro) == len(plain)
    assert np.max(np.abs(np.array(ro) - plain) / np.array(plain)) <= 1e-15


def test_reorth_lowers_overlap_when_truncated():
    """With a top-M cut the three-term recursion loses orthogonality to
    O_{n-2} (consecutive vectors share no strings here, so <O_n, O_{n-1}>
    vanishes either way); the re-orthogonalised run keeps |<O_n, O_{n-2}>|
    well below the plain recursion's."""
    n = 10
    H = wl.random_operator(n, 20, seed=51, real=True, density=0.3)
    O0 = wl.from_terms(n, [(1.0, [("Z", 5)])])
    t = oracle.Trunc(max_strings=60)

    def worst(reorth):
        _, basis = oracle.lanczos(H, O0, 14, t, keep_basis=True, reorth=reorth)
        w1 = max(abs(oracle.inner(basis[k], basis[k - 1])) for k in range(1, len(basis)))
        w2 = max(abs(oracle.inner(basis[k], basis[k - 2])) for k in range(2, len(basis)))
        return w1, w2
    p1, p2 = worst(False)
    r1, r2 = worst(True)
    assert p2 > 0.1 and r2 < p2 / 3
    assert r1 <= p1


def _pauli_basis(n):
    """Every string of n sites (x, z in 0..2^n-1), its dense matrix and key."""
    keys, mats = [], []
    for x in range(2 ** n):
        for z in range(2 ** n):
            keys.append((x, z))
            mats.append(dense_string(n, (x, z)))
    return keys, mats


def test_reorth_truncated_lanczos_vs_dense_vector_space():
    """The whole re-orthogonalised, truncated step against an independent
    implementation: operators as coefficient vectors over all 4^n strings,
    the Liouvillian as the matrix Tr(P_i [H, P_j]) / 2^n from dense matrices,
    Gram-Schmidt against the two previous vectors with numpy inner products,
    division by b_n, then the top-M cut by |c| (ties by the smaller key)."""
    n, M, steps = 4, 40, 10
    H = wl.random_operator(n, 9, seed=41, real=True)
    O0 = wl.random_operator(n, 5, seed=42, real=True)
    O0.coef = O0.coef / math.sqrt(float(np.sum(np.abs(O0.coef) ** 2)))
    keys, mats = _pauli_basis(n)
    d = 2 ** n
    dH = dense(H)
    L = np.array([[np.trace(Pi @ (dH @ Pj - Pj @ dH)) / d for Pj in mats] for Pi in mats])
    index = {k: i for i, k in enumerate(keys)}

    def vec(op):
        v = np.zeros(len(keys), complex)
        for k, c in zip(op.keys(), op.coef):
            v[index[k]] = c
        return v

    def trunc(v):
        m2 = v.real * v.real + v.imag * v.imag
        order = sorted((i for i in range(len(v)) if m2[i] > 0),
                       key=lambda i: (-m2[i], keys[i][0], keys[i][1]))
        out = np.zeros_like(v)
        out[order[:M]] = v[order[:M]]
        return out
    prev, cur, b_prev, ref = None, vec(O0), 0.0, []
    for _ in range(steps):
        A = L @ cur
        if prev is not None:
            A = A - b_prev * prev
        coefs = [np.vdot(V, A) / np.vdot(V, V).real for V in (cur, prev) if V is not None]
        for V, a in zip((cur, prev), coefs):
            A = A - a * V
        b = math.sqrt(np.vdot(A, A).real)
        ref.append(b)
        prev, cur, b_prev = cur, trunc(A / b), b
    got = oracle.lanczos(H, O0, steps, oracle.Trunc(max_strings=M), reorth=True)
    assert np.allclose(got, ref, rtol=1e-12, atol=0)
    plain = oracle.lanczos(H, O0, steps, oracle.Trunc(max_strings=M))
    assert not np.allclose(plain, ref, rtol=1e-6, atol=0)  # the flag matters here


@pytest.mark.parametrize("n", [6, 70])
def test_majorana_chain_closed_form(n):
    J, h = 1.0, 0.7
    H = wl.majorana_chain(n, J, h)
    O0 = wl.from_terms(n, [(1.0, [("X", 1)])])
    bs, basis = oracle.lanczos(H, O0, 2 * n + 1, keep_basis=True)
    want = [2 * h if k % 2 == 0 else 2 * J for k in range(2 * n - 1)]
    assert len(bs) == 2 * n  # breakdown reported at step 2N
    assert np.allclose(bs[:-1], want, rtol=1e-14)
    assert bs[-1] < 1e-12
    assert all(B.n == 1 for B in basis)
    # the last basis string of the chain is Y...Y X or Y...Y Z covering all N sites
    last = wl.text_of_key(n, basis[-1].keys()[0])
    assert "1" not in last


def test_conserved_operator_breaks_down():
    H, _ = wl.xxz_random_field(8, 0.5, 0.3, 4)
    O0 = wl.single_site_sum(8, "Z", 1 / math.sqrt(8))
    nxt, b, broke = oracle.lanczos_step(H, None, O0, 0.0)
    assert b == 0.0 and broke and nxt.n == 0
    O0x = wl.single_site_sum(8, "X", 1 / math.sqrt(8))
    _, b, broke = oracle.lanczos_step(H, None, O0x, 0.0)
    assert b > 0.5 and not broke


def test_krylov_dimension_single_site():
    # D = 2: n <= D^2 - D + 1 = 3 ... H = hX, O = Z closes after one step
    h = 0.8
    H = wl.from_terms(1, [(h, [("X", 1)])])
    O0 = wl.from_terms(1, [(1.0, [("Z", 1)])])
    bs = oracle.lanczos(H, O0, 5)
    assert bs[0] == pytest.approx(2 * h, rel=1e-15)
    assert len(bs) == 2 and bs[1] == 0.0


# ---------------------------------------------------------------------------
# Runge-Kutta
# ---------------------------------------------------------------------------

def test_rk4_step_taylor_closed_form_tfim():
    H, O0 = wl.config_rk4_tfim()
    dt = 0.02
    O1 = oracle.rk4_step(H, O0, dt)
    S = oracle.inner(O0, O1)
    b1, b2 = 4.0, 4.0  # 2 hx and 2 J sqrt(4): closed forms for an interior site
    want = 1 - b1 ** 2 * dt ** 2 / 2 + b1 ** 2 * (b1 ** 2 + b2 ** 2) * dt ** 4 / 24
    assert abs(S.real - want) < 1e-14 and abs(S.imag) < 1e-15
    bs = oracle.lanczos(H, O0, 2)
    assert np.allclose(bs, [b1, b2], rtol=1e-15)
    assert O1.n == 50


def dense_rk4(dH, dO, dt):
    L = lambda M: 1j * (dH @ M - M @ dH)
    k1 = L(dO)
    k2 = L(dO + dt / 2 * k1)
    k3 = L(dO + dt / 2 * k2)
    k4 = L(dO + dt * k3)
    return dO + dt / 6 * k1 + dt / 3 * k2 + dt / 3 * k3 + dt / 6 * k4


def test_rk4_vs_dense_and_norm():
    n = 4
    H = wl.random_operator(n, 8, seed=41, real=True)
    O = wl.random_operator(n, 6, seed=42, real=True)
    dt = 0.05
    dH = dense(H)
    dO = dense(O)
    cur = O
    for _ in range(3):
        cur = oracle.rk4_step(H, cur, dt)
        dO = dense_rk4(dH, dO, dt)
    assert np.abs(dense(cur) - dO).max() < 1e-12
    # exact evolution conserves the Frobenius norm; RK4 only to O(dt^5) per step
    n0 = oracle.norm2(O)
    assert abs(oracle.norm2(cur) - n0) < 1e-4 * n0
    d = 2 ** n
    assert abs(oracle.norm2(cur) - np.vdot(dO, dO).real / d) < 1e-12


# ---------------------------------------------------------------------------
# Truncation: defining properties of top-M with keep set and filters
# ---------------------------------------------------------------------------

def key_order(k, W):
    return tuple(reversed(k[:W])) + tuple(reversed(k[W:]))


@pytest.mark.parametrize("seed", range(6))
def test_truncate_properties(seed):
    rng = np.random.default_rng(seed)
    n = 20
    O = wl.random_operator(n, 300, seed=seed + 60, density=0.3)
    # many exact ties: quantise magnitudes
    if seed % 2 == 0:
        O.coef = np.round(O.coef * 2) / 2
        O.coef[O.coef == 0] = 0.5
    keep = wl.HostOp(n, O.x[:3], O.z[:3], O.coef[:3])
    M = int(rng.integers(1, 250))
    L = int(rng.integers(3, 10))
    eps = 0.3 if seed % 3 == 0 else 0.0
    t = oracle.Trunc(max_len=L, coef_eps=eps, max_strings=M, keep=keep)
    out = oracle.truncate(O, t)
    W = 1
    length = lambda k: bin(k[0] | k[1]).count("1")
    m2 = lambda c: c.real * c.real + c.imag * c.imag
    surv = {k: c for k, c in zip(O.keys(), O.coef)
            if length(k) <= L and (eps == 0 or m2(c) >= eps * eps) and c != 0}
    kept = out.as_dict()
    assert set(kept) <= set(surv)
    for k in kept:
        assert kept[k] == surv[k]
    keep_keys = set(keep.keys()) & set(surv)
    assert keep_keys <= set(kept)
    assert len(kept) == len(keep_keys) + min(max(0, M - len(keep_keys)),
                                             len(surv) - len(keep_keys))
    dropped = [k for k in surv if k not in kept]
    for kk in kept:
        if kk in keep_keys:
            continue
        for kd in dropped:
            a, b = m2(kept[kk]), m2(surv[kd])
            assert a > b or (a == b and key_order(kk, W) < key_order(kd, W))


# ---------------------------------------------------------------------------
# Precision split: FP32 products with Kahan-compensated sums
# ---------------------------------------------------------------------------

def test_f32k_equals_f64_when_everything_is_exact():
    """Dyadic coefficients with few bits: FP32 products and sums are exact, so
    the FP32 mode must reproduce the FP64 commutator bit for bit."""
    n = 6
    rng = np.random.default_rng(3)
    H = wl.random_operator(n, 8, seed=71, density=0.5)
    O = wl.random_operator(n, 12, seed=72, density=0.6)
    H.coef = (rng.integers(-8, 9, H.n) + 1j * rng.integers(-8, 9, H.n)) / 4
    O.coef = (rng.integers(-8, 9, O.n) + 1j * rng.integers(-8, 9, O.n)) / 8
    a = oracle.commutator(H, O, oracle.F64)
    b = oracle.commutator(H, O, oracle.F32K)
    assert a.as_dict() == b.as_dict()


def test_kahan_sum_matches_exact_sum():
    """One output string collecting many contributions of very different size:
    the compensated FP32 sum stays within a few FP32 ulps of the exact sum of
    the (FP32-rounded) contributions, where a plain FP32 sum loses everything."""
    n = 20
    k = 200
    rng = np.random.default_rng(5)
    # a_i = X_1 S_i, b_i = Y_1 S_i with distinct S_i on sites 2..n: every pair
    # (a_i, b_i) anticommutes and yields Z_1 (X Y = iZ on site 1)
    S = set()
    while len(S) < k:
        S.add(tuple(int(v) for v in rng.integers(0, 4, n - 1)))
    S = sorted(S)
    def op(first, coefs):
        terms = []
        for s, c in zip(S, coefs):
            f = [(first, 1)] + [("IXZY"[p], j + 2) for j, p in enumerate(s) if p]
            terms.append((c, f))
        return wl.from_terms(n, terms)
    H = op("X", np.ones(k))
    big = np.where(np.arange(k) % 2 == 0, 1.0e7, -1.0e7)
    small = rng.uniform(0.5, 1.5, k)
    O = op("Y", np.where(np.arange(k) < k - 50, big, small))
    C = oracle.commutator(H, O, oracle.F32K).as_dict()
    z1 = (0,) + (1,)  # x word 0, z word 0 of Z_1
    got = C[z1]
    # contribution of pair i: [X S, c Y S] = 2i c Z_1 (only the i = j pairs give Z_1)
    contrib = [2.0 * float(np.float32(c)) for c in O.coef.real]
    exact = math.fsum(contrib)
    assert abs(got.real) == 0.0
    assert abs(got.imag - exact) <= 4 * np.spacing(np.float32(abs(exact))) + 1e-30
    naive = np.float32(0.0)
    for c in contrib:
        naive = np.float32(naive + np.float32(c))
    assert abs(float(naive) - exact) > abs(got.imag - exact)


def test_kahan_fold_hand_derived():
    """The FP32 mode's compensated fold on one string, worked out by hand.

    [X_1 S_i, c_i Y_1 S_i] = 2i c_i Z_1, so the imaginary part of Z_1's
    coefficient sums t_i = 2 c_i in ascending H index, with
    t = (2^-20, -2^24, -1, 2^24) (c_i = t_i / 2, all exact).  Kahan's update
    y = t - comp, u = s + y, comp = (u - s) - y, s = u in FP32 gives:
      t1: y = 2^-20, u = 2^-20, comp = 0, s = 2^-20
      t2: y = -2^24, u = RN(2^-20 - 2^24) = -2^24,
          comp = RN(-2^24 - 2^-20) + 2^24 = 0, s = -2^24
      t3: y = -1, u = RN(-2^24 - 1) = -2^24 (tie to even), comp = 0 + 1 = 1
      t4: y = 2^24 - 1 (exact), u = -1, comp = (2^24 - 1) - (2^24 - 1) = 0
    so the value is (double)s - (double)comp = -1 exactly.  A plain FP32 sum
    gives 0 (the string would be dropped) and an FP64 sum gives the exact
    -1 + 2^-20: the three readings of the fold differ."""
    t = [2.0**-20, -2.0**24, -1.0, 2.0**24]
    H, O = wl.same_key_runs(8, [v / 2 for v in t], seed=9)
    z1 = (0, 1)  # x word 0, z word 0 of Z_1
    got = oracle.commutator(H, O, oracle.F32K).as_dict()[z1]
    assert got == complex(0.0, -1.0)
    exact = oracle.commutator(H, O, oracle.F64).as_dict()[z1]
    assert exact == complex(0.0, -1.0 + 2.0**-20)


def f32_tie_case():
    """A Lanczos step whose two largest quotients tie in FP32 but not in FP64:
    [X_1, c Z_1 Z_j] = -2i c Y_1 Z_j with c = 1 - 2^-24 (j = 2), 1 (j = 3)
    and a small third string (j = 4) that sets b_1."""
    f = np.float32
    ca, cb, c3 = float(np.nextafter(f(1.0), f(0))), 1.0, float(f(0.010598019696772099))
    n = 4
    H = wl.from_terms(n, [(1.0, [("X", 1)])])
    O = wl.from_terms(n, [(ca, [("Z", 1), ("Z", 2)]), (cb, [("Z", 1), ("Z", 3)]),
                          (c3, [("Z", 1), ("Z", 4)])])
    b = math.sqrt(4 * ca * ca + 4 * cb * cb + 4 * c3 * c3)
    return H, O, 2 * ca / b, 2 * cb / b


def test_f32k_lanczos_cut_decided_on_fp64_quotient():
    """FP32 mode keeps the string with the larger FP64 quotient when the two
    quotients round to the same FP32 value (M = 1): the cut is taken before
    the values are rounded for storage.  Rounding first would tie them and
    keep Y_1 Z_2, the smaller key."""
    H, O, qa, qb = f32_tie_case()
    assert qa < qb and float(np.float32(qa)) == float(np.float32(qb))
    got, _, _ = oracle.lanczos_step(H, None, O, 0.0, oracle.Trunc(max_strings=1), oracle.F32K)
    y1z3 = wl.string_bits(4, [("Y", 1), ("Z", 3)])
    assert got.as_dict() == {tuple(y1z3[0]) + tuple(y1z3[1]): complex(0.0, -float(np.float32(qb)))}


def test_f32k_lanczos_within_split_tolerance():
    H, O0, steps = wl.config_lanczos_small()
    b64 = oracle.lanczos(H, O0, steps, prec=oracle.F64)
    b32 = oracle.lanczos(H, O0, steps, prec=oracle.F32K)
    rel = np.abs(np.array(b32) - np.array(b64)) / np.array(b64)
    assert rel.max() < 1e-6


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts), driven through every routine on random one- and
    two-word operators by tests/sanitize_oracle.c."""
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "sanitize_oracle")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(here, "sanitize_oracle.c"),
                           os.path.join(here, "..", "oracle", "pauli_oracle.c"), "-lm"])
    # a preloaded library ahead of the sanitizer runtime is tolerated
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "sanitizer driver ok" in r.stdout


@pytest.mark.parametrize("seed", range(3))
def test_adjoint_is_conjugated_coefficients(seed):
    """Every string of the encoding is Hermitian, so the adjoint of an
    operator is the same strings with conjugated coefficients (what
    pauli_dagger computes): dense(A)^H equals dense of the conjugated
    operator, and Tr(A^H B)/2^N equals the oracle's inner product."""
    n = 3
    A = wl.random_operator(n, 12, seed=seed + 300, density=0.7)
    B = wl.random_operator(n, 10, seed=seed + 310, density=0.7)
    conjA = wl.HostOp(n, A.x, A.z, np.conj(A.coef))
    dA = dense(A)
    assert np.allclose(dA.conj().T, dense(conjA), atol=1e-14)
    got = oracle.inner(A, B)
    want = np.trace(dA.conj().T @ dense(B)) / 2 ** n
    assert abs(got - want) < 1e-13
