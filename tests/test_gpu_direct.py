"""Linear combinations of canonical operators, merged straight from their
sorted runs (no emission of records): against the oracle, and bit for bit
against the emission path, which the same call takes when a term is handed
over out of canonical order."""
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
    return pk.Workspace(512 << 20)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def random_words_op(n, count, seed, share=None, nshare=0):
    """`count` distinct random strings (uniform mask words) with N(0,1)
    complex coefficients; the first `nshare` strings copied from `share`."""
    rng = np.random.default_rng(seed)
    W = n // 64
    x = rng.integers(0, 2**63, size=(count, W), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(count, W), dtype=np.uint64)
    z = rng.integers(0, 2**63, size=(count, W), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(count, W), dtype=np.uint64)
    c = rng.standard_normal(count) + 1j * rng.standard_normal(count)
    if share is not None and nshare:
        x[:nshare], z[:nshare] = share.x[:nshare], share.z[:nshare]
    _, first = np.unique(np.concatenate([x, z], 1), axis=0, return_index=True)
    first = np.sort(first)
    return wl.HostOp(n, x[first], z[first], c[first])


def shuffled(pk, host, seed, dtype=0):
    """The strings of `host` uploaded in a random order (not canonical)."""
    p = np.random.default_rng(seed).permutation(host.n)
    return pk.PauliOp.from_raw(host.n_qubits, host.x[p], host.z[p], host.coef[p], dtype=dtype)


@pytest.mark.parametrize("n,count", [(64, 40_000), (128, 30_000), (64, 2_000_000)])
def test_add_direct_vs_oracle_and_emission(pk, ws, n, count):
    say(f"direct add n={n} count={count}")
    A = random_words_op(n, count, seed=n + count)
    B = random_words_op(n, count, seed=n + count + 1, share=A, nshare=count // 4)
    al, be = 0.7 - 0.25j, -1.5 + 0.5j
    want = oracle.add(A, al, B, be)
    Ad, Bd = pk.PauliOp.from_host(A, ws=ws), pk.PauliOp.from_host(B, ws=ws)
    got = pk.add(Ad, al, Bd, be, ws=ws)
    st = pk.last_stats()
    # the direct path: one pass, about one bucket per 730 records
    assert st["passes"] == 1 and st["buckets"] <= (A.n + B.n) // 256, st
    gh = got.to_host()
    assert_same_operator(gh, want, what="direct add")
    assert exact_fraction(gh, want) == 1.0
    # B out of canonical order: the emission path, the same bits
    alt = pk.add(Ad, al, shuffled(pk, B, 3), be, ws=ws)
    assert np.array_equal(alt.x[:, :alt.size].cpu().numpy(), got.x[:, :got.size].cpu().numpy())
    assert np.array_equal(alt.z[:, :alt.size].cpu().numpy(), got.z[:, :got.size].cpu().numpy())
    assert np.array_equal(alt.coef[:alt.size].cpu().numpy(), got.coef[:got.size].cpu().numpy())


@pytest.mark.parametrize("n,dtype", [(64, 0), (128, 0), (64, 1), (128, 1)])
def test_truncate_direct_matches_emission(pk, ws, n, dtype):
    """Length cap, |c| cutoff, keep set and top-M on a canonical operator
    (direct) and on the same strings out of order (emission): identical
    outputs; FP64 also against the oracle."""
    say(f"direct truncate n={n} dtype={dtype}")
    O = random_words_op(n, 60_000, seed=17 + n)
    if dtype == 1:
        O.coef = O.coef.astype(np.complex64).astype(np.complex128)
    keep = oracle.canonicalize(wl.HostOp(n, O.x[10:14], O.z[10:14], O.coef[10:14]))
    kd = pk.PauliOp.from_host(keep, ws=ws)
    L = n * 3 // 4
    for M, eps, max_len in ((1000, 0.0, 0), (25_000, 0.3, L), (59_000, 0.0, L)):
        tr = pk.Trunc(max_len, eps, M, kd)
        got = pk.truncate(pk.PauliOp.from_host(O, dtype=dtype, ws=ws), tr, ws=ws)
        alt = pk.truncate(shuffled(pk, O, M, dtype=dtype), tr, ws=ws)
        assert got.size == alt.size
        for a, b in ((got.x, alt.x), (got.z, alt.z)):
            assert np.array_equal(a[:, :got.size].cpu().numpy(), b[:, :alt.size].cpu().numpy())
        assert np.array_equal(got.coef[:got.size].cpu().numpy(), alt.coef[:alt.size].cpu().numpy())
        if dtype == 0:
            want = oracle.truncate(O, oracle.Trunc(max_len, eps, M, keep))
            assert_same_operator(got.to_host(), want, rtol=0.0, what=f"truncate M={M}")


def test_rk4_final_sum_of_five_terms(pk, ws):
    """The RK4 step's last call adds five canonical operators (O and the four
    stage commutators) with truncation: one RK4 step from a 3000-string
    operator against the oracle's step."""
    say("direct rk4 five-term sum")
    H = wl.tfim_2d(4, 1.0, 2.0)
    O = wl.random_operator(16, 3000, seed=9, density=0.3, real=True)
    t = oracle.Trunc(max_len=8, max_strings=2500, keep=None)
    want = oracle.rk4_step(H, O, 0.05, t)
    Hd = pk.PauliOp.from_raw(16, H.x, H.z, H.coef)
    got = pk.rk4_step(Hd, pk.PauliOp.from_host(O, ws=ws), 0.05, pk.Trunc(max_len=8,
                                                                         max_strings=2500), ws=ws)
    assert_same_operator(got.to_host(), want, what="rk4 step")


@pytest.mark.parametrize("prefix_bits,background", [(10, 20_000), (14, 300_000)])
def test_crowded_hash_range_falls_back_to_emission(pk, ws, prefix_bits, background):
    """3000 strings whose order keys share their top bits on a background of
    ordinary ones: the direct merge's bucket overflows and the call is redone
    by emission.  With 10 shared bits and 20000 others (a small call planned
    from its sizes) the 2^10-bin count overflows too and the call is redone
    with the count read first, over 2^14 bins; with 14 shared bits and 300000
    others the scatter launched beside the count read stands down (a 2^14 bin
    above the merge capacity) and the host plans passes over 2^15 bins.
    Truncation (canonical and shuffled input) and canonicalisation of a list
    with repeats, against the oracle."""
    import torch
    say(f"crowded hash range: {prefix_bits} shared bits, {background} others")
    n, k = 64, 3000
    rng = np.random.default_rng(99)
    w = rng.integers(0, 2**63, size=(k, 2), dtype=np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, size=(k, 2), dtype=np.uint64)
    prefix = {10: 0x2A7, 14: 0x29C3}[prefix_bits]
    w[:, 0] = (np.uint64(prefix) << np.uint64(64 - prefix_bits)) | \
        (w[:, 0] >> np.uint64(prefix_bits))
    keys = torch.from_numpy(w.view(np.int64)).cuda()
    cx, cz = pk.strings_from_order_keys(n, keys)
    cx = cx.cpu().numpy().view(np.uint64).T.copy()
    cz = cz.cpu().numpy().view(np.uint64).T.copy()
    bg = random_words_op(n, background, seed=5)
    x = np.concatenate([cx, bg.x])
    z = np.concatenate([cz, bg.z])
    _, first = np.unique(np.concatenate([x, z], 1), axis=0, return_index=True)
    first = np.sort(first)
    c = rng.standard_normal(len(x)) + 1j * rng.standard_normal(len(x))
    O = wl.HostOp(n, x[first], z[first], c[first])
    assert O.n > background + 2000
    for M in (0, 5000):
        want = oracle.truncate(O, oracle.Trunc(max_strings=M))
        got = pk.truncate(pk.PauliOp.from_host(O, ws=ws), pk.Trunc(max_strings=M), ws=ws)
        assert_same_operator(got.to_host(), want, rtol=0.0, what=f"canonical M={M}")
        got = pk.truncate(shuffled(pk, O, M), pk.Trunc(max_strings=M), ws=ws)
        # the count was read before the records that went to a bucket
        assert pk.last_stats()["host_syncs"] >= 2
        assert_same_operator(got.to_host(), want, rtol=0.0, what=f"shuffled M={M}")
    # a list with repeats of the crowded strings, summed in input order
    rep = rng.integers(0, k, size=1500)
    L = wl.HostOp(n, np.concatenate([O.x, cx[rep]]), np.concatenate([O.z, cz[rep]]),
                  np.concatenate([O.coef, -0.5 * c[rep]]))
    want = oracle.canonicalize(L)
    got = pk.canonicalize(pk.PauliOp.from_raw(n, L.x, L.z, L.coef), ws=ws)
    assert_same_operator(got.to_host(), want, what="canonicalize crowded list")


@pytest.mark.parametrize("n,count,dtype", [(64, 1, 0), (64, 7, 0), (64, 900, 0), (64, 1500, 1),
                                           (128, 3000, 0), (64, 70_000, 1), (128, 200_000, 0)])
def test_direct_sizes_match_emission(pk, ws, n, count, dtype):
    """From one string to 2^F buckets of every size class (F = 0 through 9):
    a three-term sum with truncation, canonical terms (direct) against the
    same terms out of order (emission), bit for bit."""
    say(f"direct sizes n={n} count={count} dtype={dtype}")
    A = random_words_op(n, count, seed=count + n)
    B = random_words_op(n, count, seed=count + n + 1, share=A, nshare=count // 2)
    if dtype:
        for X in (A, B):
            X.coef = X.coef.astype(np.complex64).astype(np.complex128)
    Ad = pk.PauliOp.from_host(A, dtype=dtype, ws=ws)
    Bd = pk.PauliOp.from_host(B, dtype=dtype, ws=ws)
    T = pk.Trunc(n * 3 // 4, 0.1, max(1, count // 3))
    got = pk.add(Ad, 0.5 + 0.25j, Bd, -1.0, T, ws=ws)
    alt = pk.add(shuffled(pk, A, 1, dtype), 0.5 + 0.25j, shuffled(pk, B, 2, dtype), -1.0, T,
                 ws=ws)
    assert got.size == alt.size
    for a, b in ((got.x, alt.x), (got.z, alt.z)):
        assert np.array_equal(a[:, :got.size].cpu().numpy(), b[:, :alt.size].cpu().numpy())
    assert np.array_equal(got.coef[:got.size].cpu().numpy(), alt.coef[:alt.size].cpu().numpy())
    if dtype == 0:
        want = oracle.truncate(oracle.add(A, 0.5 + 0.25j, B, -1.0),
                               oracle.Trunc(n * 3 // 4, 0.1, max(1, count // 3)))
        assert_same_operator(got.to_host(), want, what="direct sizes")
