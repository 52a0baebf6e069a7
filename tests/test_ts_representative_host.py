"""The library's orbit-representative search (Alg. 2, Shiftleft), compiled for
the host from its device source, against a brute-force minimum over all
rotations: random strings of every density, periodic strings, the identity,
one and two words.  The search prunes the rotations it tries (only occupied
sites, and for longer one-word strings only those after a longest empty run),
so this checks that the pruning never drops the minimum or changes which
rotation wins a tie (the smallest).  CPU only; needs g++."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2410_09654_amd", "csrc", "device_common.hpp")


@pytest.fixture(scope="module")
def rep():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    text = open(SRC).read()
    a = text.index("// v rotated so that site j of the result")
    b = text.index("// Number of non-identity sites of a raw key.")
    cpp = ("#include <stdint.h>\n#define DEV static inline\n#define __popcll __builtin_popcountll\n"
           + text[a:b] +
           'extern "C" int rep1(uint64_t* k, int n) { return ts_representative<1>(k, n); }\n'
           'extern "C" int rep2(uint64_t* k, int n) { return ts_representative<2>(k, n); }\n')
    d = tempfile.mkdtemp()
    src, lib = os.path.join(d, "rep.cpp"), os.path.join(d, "rep.so")
    open(src, "w").write(cpp)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", lib, src])
    L = ctypes.CDLL(lib)
    L.rep1.argtypes = L.rep2.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    yield L
    shutil.rmtree(d, ignore_errors=True)


def rot(v, r, n):
    """site j of the result = site (j + r) mod n of v"""
    return ((v >> r) | (v << (n - r))) & ((1 << n) - 1) if r else v


def brute(x, z, n):
    best = None
    for r in range(n):
        cand = (rot(x | z, r, n), rot(x, r, n), rot(z, r, n), r)
        if best is None or cand < best:
            best = cand
    return best[1], best[2], best[3]


def strings(n, rng):
    out = [(0, 0)]
    for dens in (0.05, 0.3, 0.6, 0.9, 1.0):
        for _ in range(60):
            x = z = 0
            for j in range(n):
                if rng.random() < dens:
                    p = int(rng.integers(1, 4))
                    x |= (p & 1) << j
                    z |= (p >> 1) << j
            out.append((x, z))
    for d in [d for d in range(1, n + 1) if n % d == 0]:  # periodic strings
        for _ in range(4):
            x = z = 0
            for j in range(d):
                p = int(rng.integers(0, 4))
                x |= (p & 1) << j
                z |= (p >> 1) << j
            X = sum(x << (d * q) for q in range(n // d))
            Z = sum(z << (d * q) for q in range(n // d))
            out.append((X, Z))
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 13, 31, 32, 33, 50, 63, 64])
def test_one_word_representative_is_brute_force_minimum(rep, n):
    rng = np.random.default_rng(1000 + n)
    m64 = (1 << 64) - 1
    for x, z in strings(n, rng):
        for r0 in (0, 1 % n, n // 2):
            xs, zs = rot(x, r0, n), rot(z, r0, n)
            k = (ctypes.c_uint64 * 2)(xs & m64, zs & m64)
            r = rep.rep1(k, n)
            bx, bz, br = brute(xs, zs, n)
            assert (int(k[0]), int(k[1]), r) == (bx, bz, br), (n, xs, zs)


@pytest.mark.parametrize("n", [65, 100, 128])
def test_two_word_representative_is_brute_force_minimum(rep, n):
    rng = np.random.default_rng(2000 + n)
    m64 = (1 << 64) - 1
    for x, z in strings(n, rng)[::3]:
        k = (ctypes.c_uint64 * 4)(x & m64, x >> 64, z & m64, z >> 64)
        r = rep.rep2(k, n)
        bx, bz, br = brute(x, z, n)
        got = (int(k[0]) | int(k[1]) << 64, int(k[2]) | int(k[3]) << 64, r)
        assert got == (bx, bz, br), (n, x, z)
