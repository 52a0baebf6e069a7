"""GPU parity of the precision split (PAULI_C64K: FP32 coefficients and
products, Kahan-compensated sums, FP64 recombination, norms and b_n) against
the oracle's FP32 mode, and its error against the FP64 path.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import assert_same_operator, exact_fraction, gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

C64K = 1


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


def f32(op: wl.HostOp) -> wl.HostOp:
    """The operator with FP32-rounded coefficients (exact zeros dropped)."""
    c = op.coef.astype(np.complex64).astype(np.complex128)
    keep = (c.real != 0) | (c.imag != 0)
    return wl.HostOp(op.n_qubits, op.x[keep], op.z[keep], c[keep])


def uph(pk, H):
    return pk.PauliOp.from_raw(H.n_qubits, H.x, H.z, H.coef)


@pytest.mark.parametrize("n,nh,no,seed", [(16, 30, 3000, 1), (64, 191, 2500, 2),
                                          (128, 60, 1200, 3)])
def test_commutator_f32k(pk, ws, n, nh, no, seed):
    say(f"f32k commutator n={n}")
    H = wl.random_operator(n, nh, seed=seed, density=min(1.0, 3.0 / n + 0.05))
    O = f32(wl.random_operator(n, no, seed=seed + 9, density=min(1.0, 6.0 / n + 0.05)))
    want = f32(oracle.commutator(H, O, oracle.F32K))
    Od = pk.PauliOp.from_host(O, dtype=C64K, ws=ws)
    got = pk.commutator(uph(pk, H), Od, ws=ws).to_host()
    assert_same_operator(got, want, rtol=2e-7, what="f32k commutator")
    assert exact_fraction(got, want) == 1.0


def test_add_f32k(pk, ws):
    say("f32k add")
    n = 64
    A = f32(wl.random_operator(n, 3000, seed=4, density=0.2))
    B = f32(wl.random_operator(n, 2000, seed=5, density=0.2))
    al, be = 1.0, -0.37
    want = f32(oracle.add(A, al, B, be))
    got = pk.add(pk.PauliOp.from_host(A, dtype=C64K, ws=ws), al,
                 pk.PauliOp.from_host(B, dtype=C64K, ws=ws), be, ws=ws).to_host()
    assert_same_operator(got, want, rtol=2e-7, what="f32k add")
    assert exact_fraction(got, want) == 1.0


def test_lanczos_f32k_small(pk, ws):
    say("f32k lanczos N=12")
    H, O0, steps = wl.config_lanczos_small()
    want32 = oracle.lanczos(H, O0, steps, prec=oracle.F32K)
    want64 = oracle.lanczos(H, O0, steps, prec=oracle.F64)
    got = pk.lanczos(uph(pk, H), pk.PauliOp.from_host(O0, dtype=C64K, ws=ws), steps, ws=ws)
    assert np.allclose(got, want32, rtol=1e-13, atol=0)
    rel = np.abs(np.array(got) - np.array(want64)) / np.array(want64)
    assert rel.max() < 1e-6


def test_lanczos_f32k_two_words_truncated(pk, ws):
    """N=128 XXZ chain with random field (two words per mask), truncated: the
    FP32 mode follows the oracle's FP32 mode step for step, and stays within
    1e-6 of the FP64 run."""
    say("f32k lanczos N=128 truncated")
    H, O0 = wl.config_lanczos_split()
    M, steps = 3000, 6
    t = oracle.Trunc(max_strings=M)
    want32 = oracle.lanczos(H, f32(O0), steps, t, prec=oracle.F32K)
    Hd = uph(pk, H)
    got32 = pk.lanczos(Hd, pk.PauliOp.from_host(f32(O0), dtype=C64K, ws=ws), steps,
                       pk.Trunc(max_strings=M), ws=ws)
    got64 = pk.lanczos(Hd, pk.PauliOp.from_host(O0, ws=ws), steps, pk.Trunc(max_strings=M),
                       ws=ws)
    assert np.allclose(got32, want32, rtol=1e-12, atol=0)
    rel = np.abs(np.array(got32) - np.array(got64)) / np.array(got64)
    assert rel.max() < 1e-6, rel


def test_kahan_fold_hand_derived_gpu(pk, ws):
    """The compensated FP32 fold on the GPU: Z_1 collects the contributions
    2 c_i = (2^-20, -2^24, -1, 2^24) in ascending H index; Kahan's fold gives
    exactly -1 (a plain FP32 sum gives 0, an FP64 sum -1 + 2^-20)."""
    say("f32k kahan fold, hand-derived")
    t = [2.0**-20, -2.0**24, -1.0, 2.0**24]
    H, O = wl.same_key_runs(8, [v / 2 for v in t], seed=9)
    got = pk.commutator(uph(pk, H), pk.PauliOp.from_raw(8, O.x, O.z, O.coef, dtype=C64K),
                        ws=ws).to_host().as_dict()
    assert got[(0, 1)] == complex(0.0, -1.0)


@pytest.mark.parametrize("n,k,seed", [(20, 200, 2), (128, 1000, 0)])
def test_kahan_long_runs_bit_exact(pk, ws, n, k, seed):
    """Long cancelling runs into one string (k contributions of widely
    different size): the GPU's FP32 fold equals the oracle's FP32 mode bit
    for bit, on an instance where the compensated fold, a plain FP32 sum and
    an FP64 sum of the same contributions round to three different FP32
    values."""
    say(f"f32k kahan long runs n={n} k={k}")
    coefs = wl.cancelling_values(k, seed) / 2
    H, O = wl.same_key_runs(n, coefs, seed=seed)
    want = oracle.commutator(H, O, oracle.F32K)
    z1 = (0,) * H.W + (1,) + (0,) * (H.W - 1)
    wv = want.as_dict()[z1].imag
    contrib = [np.float32(2 * c) for c in coefs]
    plain = np.float32(0)
    for v in contrib:
        plain = np.float32(plain + v)
    f64 = math.fsum(float(v) for v in contrib)
    assert len({float(np.float32(wv)), float(plain), float(np.float32(f64))}) == 3
    got = pk.commutator(uph(pk, H), pk.PauliOp.from_raw(n, O.x, O.z, O.coef, dtype=C64K),
                        ws=ws).to_host()
    assert exact_fraction(got, f32(want)) == 1.0
    assert got.as_dict()[z1] == complex(0.0, float(np.float32(wv)))


def test_lanczos_f32k_cut_on_fp64_quotient_gpu(pk, ws):
    """The FP32 Lanczos step decides the top-M cut on the FP64 quotient: of
    two quotients that tie in FP32 it keeps the larger FP64 one, as the
    oracle does (M = 1)."""
    import math as _m
    f = np.float32
    ca, cb, c3 = float(np.nextafter(f(1.0), f(0))), 1.0, float(f(0.010598019696772099))
    H = wl.from_terms(4, [(1.0, [("X", 1)])])
    O = wl.from_terms(4, [(ca, [("Z", 1), ("Z", 2)]), (cb, [("Z", 1), ("Z", 3)]),
                          (c3, [("Z", 1), ("Z", 4)])])
    b = _m.sqrt(4 * ca * ca + 4 * cb * cb + 4 * c3 * c3)
    assert float(f(2 * ca / b)) == float(f(2 * cb / b))
    want, _, _ = oracle.lanczos_step(H, None, O, 0.0, oracle.Trunc(max_strings=1), oracle.F32K)
    got, _, _ = pk.lanczos_step(uph(pk, H), None, pk.PauliOp.from_host(O, dtype=C64K, ws=ws),
                                0.0, pk.Trunc(max_strings=1), ws=ws)
    assert got.to_host().as_dict() == want.as_dict()
