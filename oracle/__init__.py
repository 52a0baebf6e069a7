"""CPU oracle for the Pauli-string operator algebra (test infrastructure).

Only the tests, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  It wraps `liboracle.so`, a plain C
implementation (see pauli_oracle.c) that shares no code with the HIP path,
plus `mlp`, a float64 NumPy reference of the b_n surrogate network.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from workloads import HostOp, n_words

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "pauli_oracle.c")

OR_OK, OR_EINVAL, OR_ENOMEM, OR_BREAKDOWN = 0, 1, 2, 4
F64, F32K = 0, 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp, _SRC, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _OrOp(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n", ctypes.c_int64),
                ("x", ctypes.POINTER(ctypes.c_uint64)), ("z", ctypes.POINTER(ctypes.c_uint64)),
                ("re", ctypes.POINTER(ctypes.c_double)), ("im", ctypes.POINTER(ctypes.c_double))]


class _OrTrunc(ctypes.Structure):
    _fields_ = [("max_len", ctypes.c_int32), ("coef_eps", ctypes.c_double),
                ("max_strings", ctypes.c_int64), ("keep", ctypes.POINTER(_OrOp))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or \
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        L.or_free.argtypes = [P(_OrOp)]
        L.or_string_product.argtypes = [ctypes.c_int] + [P(ctypes.c_uint64)] * 6 + [P(ctypes.c_int)]
        L.or_canonicalize.argtypes = [P(_OrOp), P(_OrOp)]
        L.or_commutator.argtypes = [P(_OrOp), P(_OrOp), ctypes.c_int, P(_OrOp)]
        L.or_product.argtypes = [P(_OrOp), P(_OrOp), P(_OrOp)]
        L.or_add.argtypes = [P(_OrOp), ctypes.c_double, ctypes.c_double, P(_OrOp),
                             ctypes.c_double, ctypes.c_double, P(_OrOp)]
        L.or_truncate.argtypes = [P(_OrOp), P(_OrTrunc), P(_OrOp)]
        L.or_divide.argtypes = [P(_OrOp), ctypes.c_double, P(_OrOp)]
        L.or_add_noise.argtypes = [P(_OrOp), ctypes.c_double, P(_OrOp)]
        U2 = ctypes.c_uint64 * 2
        L.or_ts_canonical.argtypes = [ctypes.c_int, U2, U2, U2, U2]
        L.or_ts_canonical.restype = ctypes.c_int
        L.or_ts_translate.argtypes = [ctypes.c_int, U2, U2, ctypes.c_int, U2, U2]
        L.or_ts_translate.restype = None
        L.or_commutator_ts.argtypes = [P(_OrOp), P(_OrOp), P(_OrOp)]
        L.or_norm2_ts.argtypes = [P(_OrOp)]
        L.or_norm2_ts.restype = ctypes.c_double
        L.or_norm2.argtypes = [P(_OrOp)]
        L.or_norm2.restype = ctypes.c_double
        L.or_inner.argtypes = [P(_OrOp), P(_OrOp), P(ctypes.c_double), P(ctypes.c_double)]
        L.or_exact_sum.argtypes = [P(ctypes.c_double), ctypes.c_int64]
        L.or_exact_sum.restype = ctypes.c_double
        L.or_lanczos_step.argtypes = [P(_OrOp), P(_OrOp), P(_OrOp), ctypes.c_double,
                                      P(_OrTrunc), ctypes.c_int, P(_OrOp), P(ctypes.c_double)]
        L.or_lanczos_step_reorth.argtypes = L.or_lanczos_step.argtypes
        L.or_lanczos_step_ts.argtypes = [P(_OrOp), P(_OrOp), P(_OrOp), ctypes.c_double,
                                         P(_OrTrunc), P(_OrOp), P(ctypes.c_double)]
        L.or_rk4_step.argtypes = [P(_OrOp), P(_OrOp), ctypes.c_double, P(_OrTrunc), P(_OrOp)]
        _lib = L
    return _lib


class _Marshalled:
    """Keeps the numpy buffers of an or_op alive while C reads them."""

    def __init__(self, op: HostOp):
        n = op.n
        x = np.zeros((max(n, 1), 2), np.uint64)
        z = np.zeros((max(n, 1), 2), np.uint64)
        W = op.W
        x[:n, :W] = op.x
        z[:n, :W] = op.z
        re = np.ascontiguousarray(op.coef.real if n else np.zeros(1))
        im = np.ascontiguousarray(op.coef.imag if n else np.zeros(1))
        self._keep = (x, z, re, im)
        P = ctypes.POINTER
        self.s = _OrOp(op.n_qubits, n, x.ctypes.data_as(P(ctypes.c_uint64)),
                       z.ctypes.data_as(P(ctypes.c_uint64)),
                       re.ctypes.data_as(P(ctypes.c_double)),
                       im.ctypes.data_as(P(ctypes.c_double)))


def _take(out: _OrOp, n_qubits: int) -> HostOp:
    n = out.n
    W = n_words(n_qubits)
    if n > 0:
        x = np.ctypeslib.as_array(out.x, shape=(n, 2))[:, :W].copy()
        z = np.ctypeslib.as_array(out.z, shape=(n, 2))[:, :W].copy()
        re = np.ctypeslib.as_array(out.re, shape=(n,)).copy()
        im = np.ctypeslib.as_array(out.im, shape=(n,)).copy()
    else:
        x = np.zeros((0, W), np.uint64)
        z = np.zeros((0, W), np.uint64)
        re = im = np.zeros(0)
    lib().or_free(ctypes.byref(out))
    return HostOp(n_qubits, x, z, re + 1j * im)


def _check(rc):
    if rc not in (OR_OK, OR_BREAKDOWN):
        raise RuntimeError(f"oracle error {rc}")
    return rc


class Trunc:
    def __init__(self, max_len=0, coef_eps=0.0, max_strings=0, keep: HostOp | None = None):
        self.max_len, self.coef_eps, self.max_strings, self.keep = \
            int(max_len), float(coef_eps), int(max_strings), keep

    def marshal(self):
        km = _Marshalled(self.keep) if self.keep is not None else None
        kp = ctypes.pointer(km.s) if km is not None else ctypes.POINTER(_OrOp)()
        return km, _OrTrunc(self.max_len, self.coef_eps, self.max_strings, kp)


NO_TRUNC = Trunc()


def string_product(n_qubits, a_key, b_key):
    """(c_key, k) with P_a P_b = i^k P_c; keys are (x words..., z words...)."""
    W = n_words(n_qubits)
    arr = lambda v: (ctypes.c_uint64 * 2)(*(list(v) + [0] * (2 - len(v))))
    ax, az = arr(a_key[:W]), arr(a_key[W:])
    bx, bz = arr(b_key[:W]), arr(b_key[W:])
    cx, cz = (ctypes.c_uint64 * 2)(), (ctypes.c_uint64 * 2)()
    k = ctypes.c_int()
    lib().or_string_product(n_qubits, ax, az, bx, bz, cx, cz, ctypes.byref(k))
    return tuple(cx[:W]) + tuple(cz[:W]), k.value


def canonicalize(op: HostOp) -> HostOp:
    a, out = _Marshalled(op), _OrOp()
    _check(lib().or_canonicalize(ctypes.byref(a.s), ctypes.byref(out)))
    return _take(out, op.n_qubits)


def commutator(H: HostOp, O: HostOp, prec: int = F64) -> HostOp:
    h, o, out = _Marshalled(H), _Marshalled(O), _OrOp()
    _check(lib().or_commutator(ctypes.byref(h.s), ctypes.byref(o.s), prec, ctypes.byref(out)))
    return _take(out, O.n_qubits)


def commutator_chunked(H: HostOp, O: HostOp, threads: int = 16, chunks: int | None = None,
                       prec: int = F64) -> HostOp:
    """[H, O] for large O by linearity, [H, sum_k O_k] = sum_k [H, O_k]: the
    plain oracle commutator of each chunk of O (in threads; the C oracle
    runs without the GIL), then every string's chunk values added in FP64 in
    chunk order and exact zeros dropped.  Not the canonical summation order
    (each string's contributions in ascending H index), so it agrees with
    `commutator` to rounding only: for full-size checks at the 1e-12
    tolerance and for timing the oracle on all host cores."""
    from concurrent.futures import ThreadPoolExecutor
    k = max(1, int(chunks or threads))
    bounds = np.linspace(0, O.n, k + 1).astype(np.int64)
    parts = [HostOp(O.n_qubits, O.x[a:b], O.z[a:b], O.coef[a:b])
             for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    with ThreadPoolExecutor(max_workers=max(1, int(threads))) as ex:
        res = list(ex.map(lambda p: commutator(H, p, prec), parts))
    x = np.concatenate([r.x for r in res])
    z = np.concatenate([r.z for r in res])
    c = np.concatenate([r.coef for r in res])
    if len(c) == 0:
        return HostOp(O.n_qubits, x, z, c)
    W = n_words(O.n_qubits)
    # stable sort by key keeps the chunk order inside every string's run
    order = np.lexsort([z[:, w] for w in range(W)] + [x[:, w] for w in range(W)])
    x, z, c = x[order], z[order], c[order]
    head = np.ones(len(c), bool)
    head[1:] = np.any(x[1:] != x[:-1], axis=1) | np.any(z[1:] != z[:-1], axis=1)
    starts = np.nonzero(head)[0]
    ends = np.append(starts[1:], len(c))
    tot = c[starts].copy()
    for j in range(1, int((ends - starts).max())):  # sequential adds in chunk order
        m = starts + j < ends
        tot[m] = tot[m] + c[starts[m] + j]
    keep = (tot.real != 0) | (tot.imag != 0)
    return HostOp(O.n_qubits, x[starts][keep], z[starts][keep], tot[keep])


def product(A: HostOp, B: HostOp) -> HostOp:
    a, b, out = _Marshalled(A), _Marshalled(B), _OrOp()
    _check(lib().or_product(ctypes.byref(a.s), ctypes.byref(b.s), ctypes.byref(out)))
    return _take(out, A.n_qubits)


def trace(O: HostOp) -> complex:
    """Tr(O)/2^N: every Pauli string but the identity is traceless, so this is
    the identity string's coefficient (0 when O has none)."""
    if O.n == 0:
        return 0j
    ident = np.all(O.x == 0, axis=1) & np.all(O.z == 0, axis=1)
    idx = np.nonzero(ident)[0]
    return complex(O.coef[idx[0]]) if len(idx) else 0j


def moments(H: HostOp, kmax: int) -> list:
    """mu_k = Tr(H^k)/2^N, k = 1..kmax (the spectral moments of the
    Conclusion), from the powers H^k = H H^(k-1) by exact string products."""
    mus, cur = [], H
    for k in range(1, kmax + 1):
        if k > 1:
            cur = product(H, cur)
        mus.append(trace(cur))
    return mus


def add(A: HostOp, alpha: complex, B: HostOp, beta: complex) -> HostOp:
    a, b, out = _Marshalled(A), _Marshalled(B), _OrOp()
    alpha, beta = complex(alpha), complex(beta)
    _check(lib().or_add(ctypes.byref(a.s), alpha.real, alpha.imag, ctypes.byref(b.s),
                        beta.real, beta.imag, ctypes.byref(out)))
    return _take(out, A.n_qubits)


def truncate(O: HostOp, t: Trunc) -> HostOp:
    o, out = _Marshalled(O), _OrOp()
    km, ts = t.marshal()
    _check(lib().or_truncate(ctypes.byref(o.s), ctypes.byref(ts), ctypes.byref(out)))
    del km
    return _take(out, O.n_qubits)


def divide(O: HostOp, b: float) -> HostOp:
    o, out = _Marshalled(O), _OrOp()
    _check(lib().or_divide(ctypes.byref(o.s), float(b), ctypes.byref(out)))
    return _take(out, O.n_qubits)


def add_noise(O: HostOp, lam: float) -> HostOp:
    """Depolarizing noise: every coefficient times exp(-lam * length)."""
    o, out = _Marshalled(O), _OrOp()
    _check(lib().or_add_noise(ctypes.byref(o.s), float(lam), ctypes.byref(out)))
    return _take(out, O.n_qubits)


def coefficients(O: HostOp, Q: HostOp) -> np.ndarray:
    """O's coefficient of each string of Q (0 where O lacks it)."""
    d = O.as_dict()
    return np.array([d.get(k, 0j) for k in Q.keys()], dtype=complex)


def evolve_noisy(H: HostOp, O0: HostOp, dt: float, steps: int, max_strings: int,
                 noise: float, probes: HostOp | None = None, max_len: int = 0):
    """The noisy Heisenberg loop of the Heisenberg section: per step an RK4
    step with stages truncated to max_strings (O0 kept), the depolarizing
    channel exp(-noise dt length), and a trim to max_strings (O0 kept).
    Returns (O(t_steps), S[k] = <O0, O(t_k)>/<O0, O0>, P[k] = coefficients of
    the probe strings in O(t_k)), k = 0..steps."""
    t = Trunc(max_len=max_len, max_strings=max_strings, keep=O0)
    n0 = norm2(O0)
    S, P, cur = [], [], O0

    def record(op):
        S.append(inner(O0, op) / n0)
        if probes is not None:
            P.append(coefficients(op, probes))

    record(cur)
    for _ in range(steps):
        cur = truncate(add_noise(rk4_step(H, cur, dt, t), noise * dt), t)
        record(cur)
    return cur, S, P


# ---------------------------------------------------------------------------
# Translation-symmetric operators on a periodic chain (Alg. 2): an operator
# sum_k T_k(A0) is held as A0, one representative string per orbit.
# ---------------------------------------------------------------------------
def _words2(op: HostOp, k: int):
    W = op.x.shape[1]
    x = (ctypes.c_uint64 * 2)(*(list(int(v) for v in op.x[k]) + [0] * (2 - W)))
    z = (ctypes.c_uint64 * 2)(*(list(int(v) for v in op.z[k]) + [0] * (2 - W)))
    return x, z


def _from_dict(n_qubits: int, d: dict) -> HostOp:
    W = n_words(n_qubits)
    items = [(k, c) for k, c in d.items() if c != 0]
    x = np.array([k[:W] for k, _ in items], np.uint64).reshape(-1, W)
    z = np.array([k[W:] for k, _ in items], np.uint64).reshape(-1, W)
    return canonicalize(HostOp(n_qubits, x, z, np.array([c for _, c in items], complex)))


def ts_representative(n_qubits: int, x2, z2):
    """Shiftleft of Alg. 2: the orbit representative of one string."""
    cx, cz = (ctypes.c_uint64 * 2)(), (ctypes.c_uint64 * 2)()
    lib().or_ts_canonical(n_qubits, x2, z2, cx, cz)
    return cx, cz


def canonicalize_ts(op: HostOp) -> HostOp:
    """Every string replaced by its orbit representative, duplicates summed."""
    W, d = n_words(op.n_qubits), {}
    for k in range(op.n):
        cx, cz = ts_representative(op.n_qubits, *_words2(op, k))
        key = tuple(int(cx[w]) for w in range(W)) + tuple(int(cz[w]) for w in range(W))
        d[key] = d.get(key, 0) + complex(op.coef[k])
    return _from_dict(op.n_qubits, d)


def expand_ts(op: HostOp) -> HostOp:
    """The full operator sum_k T_k(op) on the periodic chain."""
    N, W, d = op.n_qubits, n_words(op.n_qubits), {}
    for k in range(op.n):
        x2, z2 = _words2(op, k)
        for s in range(N):
            ox, oz = (ctypes.c_uint64 * 2)(), (ctypes.c_uint64 * 2)()
            lib().or_ts_translate(N, x2, z2, s, ox, oz)
            key = tuple(int(ox[w]) for w in range(W)) + tuple(int(oz[w]) for w in range(W))
            d[key] = d.get(key, 0) + complex(op.coef[k])
    return _from_dict(N, d)


def commutator_ts(H0: HostOp, O0: HostOp) -> HostOp:
    """Representatives of [sum_k T_k(H0), sum_k T_k(O0)] (O0 representatives)."""
    h, o, out = _Marshalled(H0), _Marshalled(O0), _OrOp()
    _check(lib().or_commutator_ts(ctypes.byref(h.s), ctypes.byref(o.s), ctypes.byref(out)))
    return _take(out, O0.n_qubits)


def norm2_ts(O0: HostOp) -> float:
    """||sum_k T_k(O0)||^2 / N (O0 representatives)."""
    o = _Marshalled(O0)
    r = lib().or_norm2_ts(ctypes.byref(o.s))
    if r < 0:
        raise RuntimeError("oracle error")
    return r


def lanczos_step_ts(H0: HostOp, O_prev: HostOp | None, O_cur: HostOp, b_prev: float,
                    t: Trunc = NO_TRUNC):
    """One Lanczos step on translation-symmetric operators (Krylov section with
    the Alg. 2 commutator and the stabilizer-weighted norm), with the rules of
    lanczos_step: O_n = trunc(O'_n / b_n), breakdown when
    b_n <= 1e-13 max(1, b_{n-1}).  Returns (O_next, b_n, breakdown)."""
    h, c = _Marshalled(H0), _Marshalled(O_cur)
    p = _Marshalled(O_prev) if O_prev is not None else None
    pp = ctypes.byref(p.s) if p is not None else ctypes.POINTER(_OrOp)()
    km, ts = t.marshal()
    out, b = _OrOp(), ctypes.c_double()
    rc = _check(lib().or_lanczos_step_ts(ctypes.byref(h.s), pp, ctypes.byref(c.s), float(b_prev),
                                         ctypes.byref(ts), ctypes.byref(out), ctypes.byref(b)))
    del km
    return _take(out, O_cur.n_qubits), b.value, rc == OR_BREAKDOWN


def lanczos_ts(H0: HostOp, O0: HostOp, steps: int, t: Trunc | None = None) -> list:
    """b_1..b_steps of the translation-symmetric recursion (stops early at
    breakdown).  O0 holds representatives with norm2_ts(O0) = 1; the b_n are
    those of the plain recursion on sum_k T_k(H0) and sum_k T_k(O0)/sqrt(N)."""
    bs, prev, cur, b_prev = [], None, O0, 0.0
    for _ in range(steps):
        nxt, b, broke = lanczos_step_ts(H0, prev, cur, b_prev, t if t is not None else NO_TRUNC)
        bs.append(b)
        if broke:
            break
        prev, cur, b_prev = cur, nxt, b
    return bs


def norm2(O: HostOp) -> float:
    o = _Marshalled(O)
    return lib().or_norm2(ctypes.byref(o.s))


def inner(A: HostOp, B: HostOp) -> complex:
    a, b = _Marshalled(A), _Marshalled(B)
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().or_inner(ctypes.byref(a.s), ctypes.byref(b.s), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def exact_sum(values) -> float:
    v = np.ascontiguousarray(values, dtype=np.float64)
    return lib().or_exact_sum(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), v.size)


def lanczos_step(H: HostOp, O_prev: HostOp | None, O_cur: HostOp, b_prev: float,
                 t: Trunc = NO_TRUNC, prec: int = F64, reorth: bool = False):
    """Returns (O_next, b_n, breakdown).  reorth: local re-orthogonalisation
    of O'_n against O_cur and O_prev before b_n is taken."""
    h, c = _Marshalled(H), _Marshalled(O_cur)
    p = _Marshalled(O_prev) if O_prev is not None else None
    pp = ctypes.byref(p.s) if p is not None else ctypes.POINTER(_OrOp)()
    km, ts = t.marshal()
    out, b = _OrOp(), ctypes.c_double()
    fn = lib().or_lanczos_step_reorth if reorth else lib().or_lanczos_step
    rc = _check(fn(ctypes.byref(h.s), pp, ctypes.byref(c.s), float(b_prev),
                   ctypes.byref(ts), prec, ctypes.byref(out), ctypes.byref(b)))
    del km
    return _take(out, O_cur.n_qubits), b.value, rc == OR_BREAKDOWN


def lanczos(H: HostOp, O0: HostOp, steps: int, t: Trunc = NO_TRUNC, prec: int = F64,
            keep_basis: bool = False, reorth: bool = False):
    """b_1..b_steps (stops early at breakdown) and, optionally, the basis."""
    bs, basis = [], [O0]
    prev, cur, b_prev = None, O0, 0.0
    for _ in range(steps):
        nxt, b, broke = lanczos_step(H, prev, cur, b_prev, t, prec, reorth)
        bs.append(b)
        if broke:
            break
        prev, cur, b_prev = cur, nxt, b
        if keep_basis:
            basis.append(cur)
    return (bs, basis) if keep_basis else bs


def rk4_step(H: HostOp, O: HostOp, dt: float, t: Trunc = NO_TRUNC) -> HostOp:
    h, o = _Marshalled(H), _Marshalled(O)
    km, ts = t.marshal()
    out = _OrOp()
    _check(lib().or_rk4_step(ctypes.byref(h.s), ctypes.byref(o.s), float(dt), ctypes.byref(ts),
                             ctypes.byref(out)))
    del km
    return _take(out, O.n_qubits)
