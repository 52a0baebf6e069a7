"""The RK4 and precision-split workloads at their full parameters, through the
C ABI: element-wise against the oracle over the first steps (before the
string budget binds, where the oracle still finishes in seconds), then
properties that hold at any size once the budget binds.

  * RK4: 8x8 open TFIM (J = 1, h_x = 2), O0 = Z(4,4), dt = 0.02,
    M = 2^22, length <= 16, O0 kept.
  * Lanczos precision split: N = 128 XXZ(0.5) + 0.3 r_i Z_i, O0 = sum X_i /
    sqrt(N), M = 2^23, FP64 and FP32 + Kahan.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import assert_same_operator, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def pk():
    import paper_2410_09654_amd as pk
    pk._lib.load()
    return pk


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def f32(op):
    return wl.HostOp(op.n_qubits, op.x, op.z,
                     op.coef.astype(np.complex64).astype(np.complex128))


def test_rk4_tfim_full_parameters(pk):
    import torch
    H, O0 = wl.config_rk4_tfim()
    M, L, dt = 1 << 22, 16, 0.02
    ws = pk.Workspace(1 << 30)
    Hd = pk.PauliOp.from_raw(64, H.x, H.z, H.coef)
    Od = pk.PauliOp.from_host(O0, ws=ws)
    tg = pk.Trunc(max_len=L, max_strings=M, keep=Od)
    th = oracle.Trunc(max_len=L, max_strings=M, keep=O0)
    cur_h, cur_d = O0, Od
    for k in range(3):  # 50, 4100, 354934 strings: the budget does not bind yet
        say(f"rk4 TFIM full parameters: step {k + 1} against the oracle")
        cur_h = oracle.rk4_step(H, cur_h, dt, th)
        cur_d = pk.rk4_step(Hd, cur_d, dt, tg, ws=ws)
        assert_same_operator(cur_d.to_host(), cur_h, what=f"rk4 step {k + 1}")
    for k in range(3, 6):  # the budget binds from step 4 on
        say(f"rk4 TFIM full parameters: step {k + 1}, properties")
        cur_d = pk.rk4_step(Hd, cur_d, dt, tg, ws=ws)
        h = cur_d.to_host()
        assert h.n == M
        # i[H, O] of Hermitian strings with real coefficients is real: every
        # coefficient stays exactly real
        assert np.all(h.coef.imag == 0.0)
        assert np.all(np.bitwise_count(h.x[:, 0] | h.z[:, 0]) <= L)
        o = np.lexsort((h.z[:, 0], h.x[:, 0]))
        sx, sz = h.x[o, 0], h.z[o, 0]
        assert np.all((sx[1:] != sx[:-1]) | (sz[1:] != sz[:-1]))  # unique strings
        assert np.any((h.x[:, 0] == O0.x[0, 0]) & (h.z[:, 0] == O0.z[0, 0]))  # O0 kept
    del ws, Od, cur_d
    torch.cuda.empty_cache()


def test_lanczos_precision_split_full_parameters(pk):
    import torch
    H, O0 = wl.config_lanczos_split()
    M, steps = 1 << 23, 4
    ws = pk.Workspace(1 << 30)
    Hd = pk.PauliOp.from_raw(128, H.x, H.z, H.coef)
    say("precision split full parameters: 4 steps, FP64 and FP32 + Kahan, against the oracle")
    want64 = oracle.lanczos(H, O0, steps, oracle.Trunc(max_strings=M))
    want32 = oracle.lanczos(H, f32(O0), steps, oracle.Trunc(max_strings=M), prec=oracle.F32K)
    got64 = pk.lanczos(Hd, pk.PauliOp.from_host(O0, ws=ws), steps, pk.Trunc(max_strings=M),
                       ws=ws)
    got32 = pk.lanczos(Hd, pk.PauliOp.from_host(f32(O0), dtype=pk.PAULI_C64K, ws=ws), steps,
                       pk.Trunc(max_strings=M), ws=ws)
    assert np.allclose(got64, want64, rtol=1e-12, atol=0)
    assert np.allclose(got32, want32, rtol=1e-12, atol=0)
    assert np.max(np.abs(np.array(got32) - np.array(got64)) / np.array(got64)) < 1e-6
    del ws
    torch.cuda.empty_cache()


def test_noisy_xxz_full_parameters(pk):
    """Noisy diffusion on the periodic XXZnnn chain (N = 30, delta = 2,
    gamma = 1/2), O0 = Z_1, dt = 0.05, M = 2^18 with O0 kept, eps = 0.01:
    two steps element-wise against the oracle (the second already trims to
    M at every stage), with S(t) and the 30 correlators S_{1-j}(t)."""
    import torch
    H, O0, probes = wl.config_noisy_xxz()
    n, dt, M, eps = H.n_qubits, 0.05, 1 << 18, 0.01
    say("noisy XXZnnn full parameters: 2 steps against the oracle")
    want_O, want_S, want_P = oracle.evolve_noisy(H, O0, dt, 2, M, eps, probes)
    ws = pk.Workspace(1 << 30)
    got_O, got_S, got_P = pk.evolve_noisy(
        pk.PauliOp.from_raw(n, H.x, H.z, H.coef), pk.PauliOp.from_host(O0, ws=ws), dt, 2, M,
        eps, probes=pk.PauliOp.from_raw(n, probes.x, probes.z, probes.coef), ws=ws)
    g = got_O.to_host()
    assert g.n == want_O.n == M
    assert_same_operator(g, want_O, what="noisy O(2 dt)")
    assert np.allclose(got_S, want_S, rtol=1e-12, atol=1e-15)
    assert np.allclose(np.array(got_P), np.array(want_P), rtol=1e-12, atol=1e-15)
    del ws, got_O
    torch.cuda.empty_cache()


def test_rk4_tfim_trajectory_single_steps_with_budget_binding(pk):
    """The RK4 workload with the string budget binding: along the oracle's
    own trajectory (8x8 TFIM, O0 = Z(4,4), dt = 0.02, length <= 16, O0 kept,
    M = 2^12, which binds from step 2), every step is taken on the GPU from
    the oracle's previous state and compared element-wise, through step 12."""
    H, O0 = wl.config_rk4_tfim()
    M, L, dt = 1 << 12, 16, 0.02
    ws = pk.Workspace(256 << 20)
    Hd = pk.PauliOp.from_raw(64, H.x, H.z, H.coef)
    Od0 = pk.PauliOp.from_host(O0, ws=ws)
    tg = pk.Trunc(max_len=L, max_strings=M, keep=Od0)
    th = oracle.Trunc(max_len=L, max_strings=M, keep=O0)
    cur = O0
    for k in range(12):
        say(f"rk4 TFIM trajectory, M = 2^12: step {k + 1}")
        want = oracle.rk4_step(H, cur, dt, th)
        got = pk.rk4_step(Hd, pk.PauliOp.from_host(cur, ws=ws), dt, tg, ws=ws).to_host()
        assert want.n == (M if k >= 1 else want.n)
        assert_same_operator(got, want, what=f"rk4 step {k + 1}")
        cur = want


@pytest.mark.parametrize("prec", [0, 1])
def test_lanczos_split_trajectory_single_steps_with_budget_binding(pk, prec):
    """The precision-split workload with the budget binding: along the
    oracle's trajectory (N = 128 XXZ(0.5) + 0.3 r_i Z_i, O0 = sum X_i/sqrt N,
    M = 2^12, binding from step 4), each Lanczos step on the GPU from the
    oracle's O_{n-2}, O_{n-1} and b_{n-1}, FP64 (1e-12) and FP32 + Kahan
    (keys and stored FP32 values bit-exact), through step 14."""
    H, O0 = wl.config_lanczos_split()
    M = 1 << 12
    ws = pk.Workspace(256 << 20)
    Hd = pk.PauliOp.from_raw(128, H.x, H.z, H.coef)
    dt = pk.PAULI_C64K if prec else pk.PAULI_C128
    th, tg = oracle.Trunc(max_strings=M), pk.Trunc(max_strings=M)
    prev, cur, b_prev = None, (f32(O0) if prec else O0), 0.0
    for k in range(14):
        say(f"precision split trajectory, M = 2^12, prec {prec}: step {k + 1}")
        want, bw, broke = oracle.lanczos_step(H, prev, cur, b_prev, th, prec)
        pd = pk.PauliOp.from_host(prev, dtype=dt, ws=ws) if prev is not None else None
        got, bg, gbroke = pk.lanczos_step(Hd, pd, pk.PauliOp.from_host(cur, dtype=dt, ws=ws),
                                          b_prev, tg, ws=ws)
        assert not broke and not gbroke
        assert abs(bg - bw) <= 1e-12 * bw
        g = got.to_host()
        if k >= 3:
            assert want.n == M
        assert_same_operator(g, want, rtol=1e-12 if not prec else 0.0,
                             what=f"lanczos step {k + 1}")
        prev, cur, b_prev = cur, want, bw
