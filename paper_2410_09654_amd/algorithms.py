"""Drivers of the two iterative methods on device operators.

Both loops only sequence calls of the C ABI: every operator update runs in
the HIP library.
"""
from __future__ import annotations

from . import ops
from .ops import PauliOp, Trunc, Workspace


def lanczos(H: PauliOp, O0: PauliOp, steps: int, trunc: Trunc | None = None,
            ws: Workspace | None = None, keep_basis: bool = False, reorth: bool = False):
    """Liouvillian Lanczos recursion (Krylov section): b_1..b_steps, stopping
    at breakdown.  O0 must have unit norm.  reorth: local
    re-orthogonalisation at every step (PAULI_REORTH_LOCAL)."""
    ws = ws or ops.default_workspace(O0.device)
    bs, basis = [], [O0]
    prev, cur, b_prev = None, O0, 0.0
    for _ in range(steps):
        nxt, b, broke = ops.lanczos_step(H, prev, cur, b_prev, trunc, ws=ws, reorth=reorth)
        bs.append(b)
        if broke:
            break
        prev, cur, b_prev = cur, nxt, b
        if keep_basis:
            basis.append(cur)
    return (bs, basis) if keep_basis else bs


def evolve(H: PauliOp, O0: PauliOp, dt: float, steps: int, trunc: Trunc | None = None,
           ws: Workspace | None = None, observe=None):
    """Heisenberg evolution dO/dt = i[H, O] by classical RK4 steps.

    Returns (O(t_steps), [S(t_0), ..., S(t_steps)]) with the autocorrelation
    S(t) = <O0, O(t)> / <O0, O0> (the correlator of the Heisenberg section).
    """
    ws = ws or ops.default_workspace(O0.device)
    S = [ops.correlator(O0, O0, ws=ws)]
    cur = O0
    for _ in range(steps):
        cur = ops.rk4_step(H, cur, dt, trunc, ws=ws)
        S.append(ops.correlator(O0, cur, ws=ws))
        if observe is not None:
            observe(cur)
    return cur, S


def moments(H: PauliOp, kmax: int, trunc: Trunc | None = None, ws: Workspace | None = None):
    """Moments mu_k = Tr(H^k)/2^N for k = 1..kmax (the spectral moments the
    Conclusion proposes): H^k = H H^(k-1) by string products, mu_k = the
    identity coefficient of H^k.  Exact without truncation; with `trunc`
    every power is truncated before the next product."""
    ws = ws or ops.default_workspace(H.device)
    mus, cur = [], H
    for k in range(1, kmax + 1):
        if k > 1:
            cur = ops.multiply(H, cur, trunc, ws=ws)
        mus.append(ops.trace(cur, ws=ws))
    return mus


def evolve_noisy(H: PauliOp, O0: PauliOp, dt: float, steps: int, max_strings: int,
                 noise: float, probes: PauliOp | None = None, max_len: int = 0,
                 ws: Workspace | None = None, observe=None):
    """Noisy Heisenberg evolution as the Heisenberg section runs it: per step
    one RK4 step with its stages truncated to `max_strings` (O0 kept), the
    depolarizing channel exp(-noise dt length), and a trim to `max_strings`
    (O0 kept).  Returns (O(t_steps), S, P): S[k] = Tr(O(t_k) O0^dagger) /
    Tr(O0 O0^dagger) for k = 0..steps, and, when `probes` is given, P[k] =
    the coefficients in O(t_k) of the probe strings (with O0 = Z_i and probes
    Z_j: the two-point correlators S_{i-j}(t_k)).  `observe(k, O(t_k))`, if
    given, is called after every step."""
    ws = ws or ops.default_workspace(O0.device)
    tr = Trunc(max_len=max_len, max_strings=max_strings, keep=O0)
    S, P = [], []
    cur = O0

    def record(op):
        S.append(ops.correlator(O0, op, ws=ws))
        if probes is not None:
            P.append(ops.coefficients(op, probes, ws=ws))

    record(cur)
    for _ in range(steps):
        cur = ops.rk4_step(H, cur, dt, tr, ws=ws)
        ops.add_noise(cur, noise * dt)
        cur = ops.truncate(cur, tr, ws=ws)
        record(cur)
        if observe is not None:
            observe(len(S) - 1, cur)
    return cur, S, P


def lanczos_ts1d(H0: PauliOp, O0: PauliOp, steps: int, trunc: Trunc | None = None,
                 ws: Workspace | None = None, observe=None):
    """Lanczos recursion on translation-symmetric operators of the periodic
    chain (Krylov section with the Alg. 2 commutator), one fused
    pauli_lanczos_step_ts1d call per step: O'_n = [H, O_{n-1}] - b_{n-1} O_{n-2},
    b_n = sqrt(norm2_ts1d(O'_n)), O_n = trunc(O'_n / b_n), stopping at
    breakdown.  O0 holds representatives with norm2_ts1d(O0) = 1.  Same b_n as
    the plain recursion on the full operators.  `observe(n, O_n)`, if given,
    is called after every step that did not break down."""
    ws = ws or ops.default_workspace(O0.device)
    bs, prev, cur, b_prev = [], None, O0, 0.0
    for _ in range(steps):
        nxt, b, broke = ops.lanczos_step(H0, prev, cur, b_prev, trunc, ws=ws, ts1d=True)
        bs.append(b)
        if broke:
            break
        prev, cur, b_prev = cur, nxt, b
        if observe is not None:
            observe(len(bs), cur)
    return bs
