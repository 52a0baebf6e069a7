"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *describes* operators: it sets the bits of Pauli strings and
draws seeded coefficients.  It holds none of the method's arithmetic (no
string products, no phases, no sums of coefficients, no truncation), so both
the oracle and the HIP path can take their inputs from here without sharing
any of the computation they are compared on.

Encoding (binary Pauli-string encoding of the paper's Methods section, in the
physical basis): site j (1-based, as in the paper) is bit (j-1) % 64 of word
(j-1) // 64 of two bit-masks x and z; the single-site operator is
I = (x,z) = (0,0), X = (1,0), Z = (0,1), Y = (1,1).  A string of W = ceil(N/64)
words per mask stands for the tensor product of its sites, each Pauli being
the Hermitian matrix (so Y, not iY; the paper's tau_11 = iY differs from this
by a phase that the operator's coefficient absorbs).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PAULI_BITS = {"I": (0, 0), "1": (0, 0), "X": (1, 0), "Z": (0, 1), "Y": (1, 1)}
BITS_PAULI = {(0, 0): "1", (1, 0): "X", (0, 1): "Z", (1, 1): "Y"}


def n_words(n_qubits: int) -> int:
    return (n_qubits + 63) // 64


@dataclasses.dataclass
class HostOp:
    """A sum of Pauli strings on the host: sum_k coef[k] * P(x[k], z[k]).

    x, z: uint64 arrays of shape (n, W), word w holding sites 64w+1..64w+64.
    coef: complex128 array of shape (n,).
    """

    n_qubits: int
    x: np.ndarray
    z: np.ndarray
    coef: np.ndarray

    def __post_init__(self):
        W = n_words(self.n_qubits)
        self.x = np.ascontiguousarray(self.x, dtype=np.uint64).reshape(-1, W)
        self.z = np.ascontiguousarray(self.z, dtype=np.uint64).reshape(-1, W)
        self.coef = np.ascontiguousarray(self.coef, dtype=np.complex128).reshape(-1)
        assert self.x.shape == self.z.shape and self.x.shape[0] == self.coef.shape[0]

    @property
    def n(self) -> int:
        return int(self.coef.shape[0])

    @property
    def W(self) -> int:
        return n_words(self.n_qubits)

    def keys(self):
        """List of hashable keys (x words..., z words...) in storage order."""
        return [tuple(int(v) for v in self.x[k]) + tuple(int(v) for v in self.z[k])
                for k in range(self.n)]

    def as_dict(self):
        return {k: complex(c) for k, c in zip(self.keys(), self.coef)}

    def copy(self) -> "HostOp":
        return HostOp(self.n_qubits, self.x.copy(), self.z.copy(), self.coef.copy())


def empty(n_qubits: int) -> HostOp:
    W = n_words(n_qubits)
    return HostOp(n_qubits, np.zeros((0, W), np.uint64), np.zeros((0, W), np.uint64),
                  np.zeros(0, np.complex128))


def string_bits(n_qubits: int, factors):
    """(x words, z words) of the string with the given (pauli, site) factors.

    Sites are 1-based.  A site may appear at most once.
    """
    W = n_words(n_qubits)
    x = [0] * W
    z = [0] * W
    seen = set()
    for p, site in factors:
        if not (1 <= site <= n_qubits):
            raise ValueError(f"site {site} outside 1..{n_qubits}")
        if site in seen:
            raise ValueError(f"site {site} appears twice")
        seen.add(site)
        bx, bz = PAULI_BITS[p]
        w, b = divmod(site - 1, 64)
        x[w] |= bx << b
        z[w] |= bz << b
    return x, z


def from_terms(n_qubits: int, terms) -> HostOp:
    """Operator from [(coef, [(pauli, site), ...]), ...] with distinct strings."""
    xs, zs, cs = [], [], []
    seen = set()
    for coef, factors in terms:
        x, z = string_bits(n_qubits, factors)
        key = tuple(x) + tuple(z)
        if key in seen:
            raise ValueError("duplicate string in from_terms; terms must be distinct")
        seen.add(key)
        xs.append(x)
        zs.append(z)
        cs.append(coef)
    W = n_words(n_qubits)
    return HostOp(n_qubits, np.array(xs, np.uint64).reshape(-1, W),
                  np.array(zs, np.uint64).reshape(-1, W), np.array(cs, np.complex128))


def string_from_text(text: str):
    """Parse the paper's printed string form, site 1 leftmost, '1' = identity."""
    return [(ch, j + 1) for j, ch in enumerate(text) if ch not in "1I"]


def text_of_key(n_qubits: int, key) -> str:
    W = n_words(n_qubits)
    out = []
    for j in range(n_qubits):
        w, b = divmod(j, 64)
        out.append(BITS_PAULI[((key[w] >> b) & 1, (key[W + w] >> b) & 1)])
    return "".join(out)


# --------------------------------------------------------------------------
# Hamiltonians and initial operators of the workloads
# --------------------------------------------------------------------------

def ising_chain(n: int, hx: float = 1.05, hz: float = 0.5, J: float = 1.0) -> HostOp:
    """Open chain J*sum Z_i Z_{i+1} + hx*sum X_i + hz*sum Z_i (the chaotic Ising
    chain of the Krylov section, in the Z-coupled form).  |H| = 3N - 1."""
    terms = [(J, [("Z", i), ("Z", i + 1)]) for i in range(1, n)]
    terms += [(hx, [("X", i)]) for i in range(1, n + 1)]
    if hz != 0.0:
        terms += [(hz, [("Z", i)]) for i in range(1, n + 1)]
    return from_terms(n, terms)


def xx_plus_zz_defect(n: int = 10, defect_site: int = 4) -> HostOp:
    """Sum_j (X_j X_{j+1} + Z_j Z_{j+1}) + X_defect on an open chain.

    This is the Hamiltonian whose Lanczos run reproduces the printed output of
    the paper's integrability-breaking example (section "Visualizing the
    algebra"); the printout matches XX+ZZ, not the XX+YY listing shown there.
    """
    terms = []
    for j in range(1, n):
        terms.append((1.0, [("X", j), ("X", j + 1)]))
        terms.append((1.0, [("Z", j), ("Z", j + 1)]))
    terms.append((1.0, [("X", defect_site)]))
    return from_terms(n, terms)


def xx_model(n: int, defect_site: int | None = None) -> HostOp:
    """Open XX chain sum_j (X_j X_{j+1} + Y_j Y_{j+1}) (eq. XXmodel)."""
    terms = []
    for j in range(1, n):
        terms.append((1.0, [("X", j), ("X", j + 1)]))
        terms.append((1.0, [("Y", j), ("Y", j + 1)]))
    if defect_site is not None:
        terms.append((1.0, [("X", defect_site)]))
    return from_terms(n, terms)


def majorana_chain(n: int, J: float, h: float) -> HostOp:
    """J*sum X_i X_{i+1} + h*sum Z_i on an open chain (free-fermion chain)."""
    terms = [(J, [("X", i), ("X", i + 1)]) for i in range(1, n)]
    terms += [(h, [("Z", i)]) for i in range(1, n + 1)]
    return from_terms(n, terms)


def tfim_2d(L: int = 8, J: float = 1.0, hx: float = 2.0) -> HostOp:
    """Open LxL transverse-field Ising lattice J*sum_<ij> Z_i Z_j + hx*sum X_i.

    Site (r, c), 1-based, row-major, is qubit (r-1)*L + c.  |H| = 2L(L-1) + L^2.
    """
    def q(r, c):
        return (r - 1) * L + c
    terms = []
    for r in range(1, L + 1):
        for c in range(1, L + 1):
            if c < L:
                terms.append((J, [("Z", q(r, c)), ("Z", q(r, c + 1))]))
            if r < L:
                terms.append((J, [("Z", q(r, c)), ("Z", q(r + 1, c))]))
    for r in range(1, L + 1):
        for c in range(1, L + 1):
            terms.append((hx, [("X", q(r, c))]))
    return from_terms(L * L, terms)


def xxz_random_field(n: int = 128, delta: float = 0.5, field: float = 0.3,
                     seed: int = 4):
    """Open chain sum (XX + YY + delta ZZ) + field * sum r_i Z_i, r_i ~ U[-1,1].

    Returns (H, r).  |H| = 3(N-1) + N.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.uniform(-1.0, 1.0, size=n)
    terms = []
    for j in range(1, n):
        terms.append((1.0, [("X", j), ("X", j + 1)]))
        terms.append((1.0, [("Y", j), ("Y", j + 1)]))
        terms.append((delta, [("Z", j), ("Z", j + 1)]))
    for j in range(1, n + 1):
        terms.append((field * float(r[j - 1]), [("Z", j)]))
    return from_terms(n, terms), r


def xxz_nnn(n: int = 30, delta: float = 2.0, gamma: float = 0.5) -> HostOp:
    """Periodic next-nearest-neighbour XXZ chain of the Heisenberg section:
    sum_i (X_i X_{i+1} + Y_i Y_{i+1} + delta Z_i Z_{i+1})
    + gamma sum_i (X_i X_{i+2} + Y_i Y_{i+2} + delta Z_i Z_{i+2}), sites mod n
    (the printed listing pairs site j with itself; the equation pairs it with
    j+1 and j+2).  |H| = 6n for n >= 5."""
    def s(j):
        return (j - 1) % n + 1
    terms = []
    for j in range(1, n + 1):
        for d, g in ((1, 1.0), (2, gamma)):
            terms.append((g, [("X", j), ("X", s(j + d))]))
            terms.append((g, [("Y", j), ("Y", s(j + d))]))
            terms.append((g * delta, [("Z", j), ("Z", s(j + d))]))
    return from_terms(n, terms)


def config_noisy_xxz():
    """Noisy diffusion run: N=30 periodic XXZnnn (delta=2, gamma=1/2),
    O0 = Z_1, dt=0.05, 200 steps (t=10), M=2^18, eps=0.01, probes Z_1..Z_N."""
    n = 30
    H = xxz_nnn(n)
    O0 = from_terms(n, [(1.0, [("Z", 1)])])
    probes = from_terms(n, [(1.0, [("Z", j)]) for j in range(1, n + 1)])
    return H, O0, probes


def single_site_sum(n: int, pauli: str, coef: float) -> HostOp:
    """coef * sum_i P_i (e.g. sum X_i / sqrt(N))."""
    return from_terms(n, [(coef, [(pauli, i)]) for i in range(1, n + 1)])


def random_local_strings(n_qubits: int, count: int, max_support: int = 10,
                         seed: int = 20241009, coef_dist: str = "normal") -> HostOp:
    """`count` distinct random strings, each with support on <= max_support
    contiguous sites, every site in the window a uniformly drawn X, Y or Z,
    complex coefficients with i.i.d. N(0,1) real and imaginary parts.

    Recipe: length l ~ U{1..max_support}, start ~ U{1..N-l+1}; draws are taken in
    order and repeats of an earlier string are skipped, until `count` distinct
    strings exist.  PCG64 seeded with `seed`.
    """
    W = n_words(n_qubits)
    rng = np.random.Generator(np.random.PCG64(seed))
    max_support = min(max_support, n_qubits)
    rowtype = np.dtype((np.void, 16 * W))
    xs = np.zeros((0, W), np.uint64)
    zs = np.zeros((0, W), np.uint64)
    seen = np.zeros(0, rowtype)  # sorted void view of the rows kept so far
    while xs.shape[0] < count:
        need = count - xs.shape[0]
        batch = max(4096, 2 * need + count // 4)
        length = rng.integers(1, max_support + 1, size=batch)
        start = rng.integers(0, n_qubits - length + 1)  # 0-based first site
        paulis = rng.integers(1, 4, size=(batch, max_support))  # 1=X 2=Z 3=Y
        bx = np.zeros((batch, W), np.uint64)
        bz = np.zeros((batch, W), np.uint64)
        for k in range(max_support):
            active = k < length
            site = start + k
            word = site // 64
            bit = (site % 64).astype(np.uint64)
            px = ((paulis[:, k] & 1) == 1) & active
            pz = ((paulis[:, k] & 2) == 2) & active
            for w in range(W):
                sel = word == w
                bx[:, w] |= np.where(px & sel, np.uint64(1) << bit, np.uint64(0))
                bz[:, w] |= np.where(pz & sel, np.uint64(1) << bit, np.uint64(0))
        rows = np.ascontiguousarray(np.concatenate([bx, bz], axis=1)).view(rowtype).ravel()
        _, first = np.unique(rows, return_index=True)
        first.sort()                                   # first draws within the batch, in order
        fresh = first[~np.isin(rows[first], seen)]     # skip strings drawn in earlier batches
        fresh = fresh[:need]
        xs = np.concatenate([xs, bx[fresh]])
        zs = np.concatenate([zs, bz[fresh]])
        seen = np.sort(np.concatenate([seen, rows[fresh]]))
    coef = rng.standard_normal(count) + 1j * rng.standard_normal(count)
    if coef_dist != "normal":
        raise ValueError(coef_dist)
    return HostOp(n_qubits, xs[:count], zs[:count], coef)


def cancelling_values(k: int, seed: int) -> np.ndarray:
    """k signed powers of two in seeded random order: k//4 large values
    +-2^20..2^24 each paired with its negative, the rest small values
    +-2^-24..2^-1 (their sum is the exact total)."""
    rng = np.random.default_rng(seed)
    nb = k // 4
    big = np.ldexp(rng.choice([-1.0, 1.0], nb), rng.integers(20, 25, nb))
    small = np.ldexp(rng.choice([-1.0, 1.0], k - 2 * nb), rng.integers(-24, 0, k - 2 * nb))
    vals = np.concatenate([big, -big, small])
    return vals[rng.permutation(k)]


def same_key_runs(n_qubits: int, coefs, seed: int = 5):
    """H = [X_1 S_1, ..., X_1 S_k] (coefficient 1) and O = [Y_1 S_1, c_1, ...,
    Y_1 S_k, c_k] with k distinct seeded strings S_i on sites 2..n_qubits:
    pair (i, i) is the only one of H_i with O_i that lands on Z_1, so the
    coefficient of Z_1 in [H, O] collects k contributions, one per H index."""
    k = len(coefs)
    rng = np.random.default_rng(seed)
    S = set()
    while len(S) < k:
        S.add(tuple(int(v) for v in rng.integers(0, 4, n_qubits - 1)))
    S = sorted(S)

    def op(first, cs):
        return from_terms(n_qubits, [(c, [(first, 1)] + [("IXZY"[p], j + 2)
                                                         for j, p in enumerate(s) if p])
                                     for s, c in zip(S, cs)])
    return op("X", np.ones(k)), op("Y", np.asarray(coefs, np.complex128))


def random_operator(n_qubits: int, count: int, seed: int, density: float = 0.5,
                    real: bool = False) -> HostOp:
    """`count` distinct strings with every site independently non-identity with
    probability `density` (uniform over X, Y, Z), N(0,1) coefficients."""
    W = n_words(n_qubits)
    rng = np.random.Generator(np.random.PCG64(seed))
    keys = {}
    order = []
    limit = 4 ** n_qubits - 1 if n_qubits < 32 else None
    if limit is not None:
        count = min(count, limit)
    while len(order) < count:
        x = [0] * W
        z = [0] * W
        for j in range(n_qubits):
            if rng.random() < density:
                p = int(rng.integers(1, 4))
                w, b = divmod(j, 64)
                x[w] |= (p & 1) << b
                z[w] |= ((p >> 1) & 1) << b
        k = tuple(x) + tuple(z)
        if all(v == 0 for v in k) or k in keys:
            continue
        keys[k] = True
        order.append(k)
    xs = np.array([k[:W] for k in order], np.uint64).reshape(-1, W)
    zs = np.array([k[W:] for k in order], np.uint64).reshape(-1, W)
    if real:
        coef = rng.standard_normal(len(order)).astype(np.complex128)
    else:
        coef = rng.standard_normal(len(order)) + 1j * rng.standard_normal(len(order))
    return HostOp(n_qubits, xs, zs, coef)


# --------------------------------------------------------------------------
# Named workloads (sizes of the benchmarked configurations)
# --------------------------------------------------------------------------

def config_lanczos_small():
    """Open chain N=12, H = sum ZZ + 1.05 sum X + 0.5 sum Z, O0 = Z_1,
    12 untruncated FP64 Lanczos steps."""
    n = 12
    return ising_chain(n), from_terms(n, [(1.0, [("Z", 1)])]), 12


def config_commutator_bench(count: int = 1 << 20, seed: int = 20241009):
    """N=64 chain with the same H (191 strings); O = 2^20 random local strings
    (support <= 10 contiguous sites); truncation to length <= 12, top 2^20."""
    n = 64
    return ising_chain(n), random_local_strings(n, count, 10, seed)


def config_rk4_tfim():
    """8x8 open TFIM (J=1, hx=2), O0 = Z at site (4,4) = qubit 28, dt=0.02,
    200 steps, M=2^22, length <= 16, keep = {O0}."""
    H = tfim_2d(8, 1.0, 2.0)
    O0 = from_terms(64, [(1.0, [("Z", 3 * 8 + 4)])])
    return H, O0


def config_lanczos_split(literal_o0: bool = False):
    """N=128 chain sum(XX+YY+0.5ZZ) + 0.3 sum r_i Z_i; O0 = sum X_i/sqrt(N)
    (sum Z_i/sqrt(N) when literal_o0, which commutes with H)."""
    n = 128
    H, _ = xxz_random_field(n, 0.5, 0.3, 4)
    O0 = single_site_sum(n, "Z" if literal_o0 else "X", 1.0 / math.sqrt(n))
    return H, O0


def surrogate_couplings(n_runs: int, seed: int):
    """(hx, hz) draws hx ~ U[0.5,1.5], hz ~ U[0,1] for the b_n surrogate data."""
    rng = np.random.Generator(np.random.PCG64(seed))
    hx = rng.uniform(0.5, 1.5, size=n_runs)
    hz = rng.uniform(0.0, 1.0, size=n_runs)
    return hx, hz
