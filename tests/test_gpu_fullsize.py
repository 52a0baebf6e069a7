"""Parity at the benchmark's full size, in the launch configuration the
benchmark times: the N = 64 chaotic Ising chain (|H| = 191) against 2^20
random local strings (support <= 10, seed 20241009), one commutator call with
a 1 GiB workspace, length <= 12, top 2^20.

test_commutator_full_size checks, quickly:
  * the set of output strings of the length-capped commutator equals the set
    of distinct anticommuting products of length <= 12, computed on the host
    by XOR and popcount of the keys (the string algebra of Alg. 1);
  * 256 sampled output coefficients against the oracle, each computed from
    the O strings that can reach it (b = h P_c for every H string h);
  * the top-2^20 call returns exactly the 2^20 largest |c| of that result.
test_commutator_full_size_every_string_vs_oracle compares every output
string with the oracle's whole commutator (chunks of O on the host cores,
added by linearity) and the top-2^20 cut with the oracle's truncation.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as wl
from helpers import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

MAX_LEN, M = 12, 1 << 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sorted_keys(x, z):
    order = np.lexsort((z, x))
    return x[order], z[order], order


def test_commutator_full_size():
    import torch
    import paper_2410_09654_amd as pk
    pk._lib.load()
    say("full-size commutator N=64 |H|=191 |O|=2^20")
    H, O = wl.config_commutator_bench()
    assert H.x.shape[1] == 1 and O.n == 1 << 20
    ws = pk.Workspace(1 << 30)
    Hd = pk.PauliOp.from_raw(64, H.x, H.z, H.coef)
    Od = pk.PauliOp.from_host(O, ws=ws)
    full = pk.commutator(Hd, Od, pk.Trunc(max_len=MAX_LEN), ws=ws).to_host()
    st_full = pk.last_stats()
    out = pk.PauliOp(64, M + 16)
    top = pk.commutator(Hd, Od, pk.Trunc(max_len=MAX_LEN, max_strings=M), out=out,
                        ws=ws).to_host()
    st_top = pk.last_stats()
    say(f"  emitted {st_full['emitted']}, unique {full.n}, output {top.n}")

    # key set: distinct anticommuting products of length <= MAX_LEN
    ox, oz = O.x[:, 0], O.z[:, 0]
    xs, zs = [], []
    for h in range(H.n):
        hx, hz = H.x[h, 0], H.z[h, 0]
        anti = (np.bitwise_count((hx & oz) ^ (hz & ox)) & 1).astype(bool)
        cx, cz = ox[anti] ^ hx, oz[anti] ^ hz
        short = np.bitwise_count(cx | cz) <= MAX_LEN
        xs.append(cx[short])
        zs.append(cz[short])
    cx, cz = np.concatenate(xs), np.concatenate(zs)
    assert len(cx) == st_full["emitted"] == st_top["emitted"]
    sx, sz, _ = _sorted_keys(cx, cz)
    first = np.ones(len(sx), bool)
    first[1:] = (sx[1:] != sx[:-1]) | (sz[1:] != sz[:-1])
    ux, uz = sx[first], sz[first]
    gx, gz, gorder = _sorted_keys(full.x[:, 0], full.z[:, 0])
    assert len(gx) == len(ux)
    assert np.array_equal(gx, ux) and np.array_equal(gz, uz)
    del xs, zs, cx, cz, sx, sz, first

    # sampled coefficients from the oracle
    rng = np.random.default_rng(7)
    pick = rng.choice(full.n, size=256, replace=False)
    okey = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(ox, oz))}
    need = set()
    for j in pick:
        px, pz = int(full.x[j, 0]), int(full.z[j, 0])
        for h in range(H.n):
            i = okey.get((px ^ int(H.x[h, 0]), pz ^ int(H.z[h, 0])))
            if i is not None:
                need.add(i)
    idx = np.array(sorted(need))
    Osub = wl.HostOp(64, O.x[idx], O.z[idx], O.coef[idx])
    want = oracle.commutator(H, Osub).as_dict()
    worst = 0.0
    for j in pick:
        k = (int(full.x[j, 0]), int(full.z[j, 0]))
        g, w = complex(full.coef[j]), want[k]
        worst = max(worst, abs(g - w) / abs(w))
        assert abs(g - w) <= 1e-12 * abs(w), (k, g, w)
    say(f"  256 sampled coefficients, worst relative difference {worst:.2e}")

    # top-M: the M largest |c|^2 of the length-capped result (no ties expected
    # among random coefficients; asserted below)
    m2 = full.coef.real * full.coef.real + full.coef.imag * full.coef.imag
    kth = np.partition(m2, full.n - M)[full.n - M]
    assert np.count_nonzero(m2 == kth) == 1
    sel = np.nonzero(m2 >= kth)[0]
    assert len(sel) == M == top.n
    tx, tz, torder = _sorted_keys(top.x[:, 0], top.z[:, 0])
    wx, wz, worder = _sorted_keys(full.x[sel, 0], full.z[sel, 0])
    assert np.array_equal(tx, wx) and np.array_equal(tz, wz)
    assert np.array_equal(top.coef[torder], full.coef[sel][worder])
    del ws, Od, out
    torch.cuda.empty_cache()


def _by_key(op):
    o = np.lexsort((op.z[:, 0], op.x[:, 0]))
    return op.x[o, 0], op.z[o, 0], op.coef[o]


def test_commutator_full_size_every_string_vs_oracle():
    """The whole benchmark call against the oracle, string by string: the
    oracle's commutator of all 2^20 strings (chunks of O on the host cores,
    added by linearity), length-capped, then the oracle's own top-2^20 cut.
    Keys bit-exact; coefficients within 1e-12 of max(1, |c|)."""
    import os
    import time
    import torch
    import paper_2410_09654_amd as pk
    pk._lib.load()
    H, O = wl.config_commutator_bench()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    say(f"full-size commutator vs the chunked oracle on {threads} threads")
    t0 = time.time()
    ref = oracle.commutator_chunked(H, O, threads=threads, chunks=4 * threads)
    ref_cap = oracle.truncate(ref, oracle.Trunc(max_len=MAX_LEN))
    say(f"  oracle: {ref.n} strings, {ref_cap.n} of length <= {MAX_LEN}, "
        f"{time.time() - t0:.1f} s")
    ws = pk.Workspace(1 << 30)
    Hd = pk.PauliOp.from_raw(64, H.x, H.z, H.coef)
    Od = pk.PauliOp.from_host(O, ws=ws)
    full = pk.commutator(Hd, Od, pk.Trunc(max_len=MAX_LEN), ws=ws).to_host()
    for got, want, what in ((full, ref_cap, "length-capped"),):
        gx, gz, gc = _by_key(got)
        wx, wz, wc = _by_key(want)
        assert len(gx) == len(wx), what
        assert np.array_equal(gx, wx) and np.array_equal(gz, wz), what
        err = np.abs(gc - wc) / np.maximum(1.0, np.abs(wc))
        say(f"  {what}: {len(gx)} strings, worst coefficient difference {err.max():.2e}")
        assert err.max() <= 1e-12, what
    del full
    t0 = time.time()
    ref_top = oracle.truncate(ref, oracle.Trunc(max_len=MAX_LEN, max_strings=M))
    say(f"  oracle top-2^20: {time.time() - t0:.1f} s")
    out = pk.PauliOp(64, M + 16)
    top = pk.commutator(Hd, Od, pk.Trunc(max_len=MAX_LEN, max_strings=M), out=out,
                        ws=ws).to_host()
    gx, gz, gc = _by_key(top)
    wx, wz, wc = _by_key(ref_top)
    assert len(gx) == len(wx) == M
    assert np.array_equal(gx, wx) and np.array_equal(gz, wz)
    assert (np.abs(gc - wc) / np.maximum(1.0, np.abs(wc))).max() <= 1e-12
    del ws, Od, out
    torch.cuda.empty_cache()
