"""CPU checks of the boundary: the HIP library loads and exports every entry
point that include/pauli.h declares; host-side marshalling is consistent."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pauli.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pauli_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["pauli_commutator", "pauli_add", "pauli_truncate", "pauli_rk4_step",
                 "pauli_lanczos_step", "pauli_norm2", "pauli_inner", "pauli_canonicalize"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2410_09654_amd import _lib
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_strerror_and_profile_calls_run_on_host():
    from paper_2410_09654_amd import _lib
    L = _lib.load()
    assert L.pauli_strerror(0) == b"ok"
    assert b"workspace" in L.pauli_strerror(3)
    L.pauli_profile_enable(0)
    assert L.pauli_profile_read(None, 0) >= 1


def test_struct_layout_matches_header():
    from paper_2410_09654_amd._lib import PauliOpC, PauliTruncC, PauliWsC
    assert ctypes.sizeof(PauliOpC) == 4 + 4 + 8 + 8 + 8 * 3
    assert PauliOpC.x.offset == 24
    assert ctypes.sizeof(PauliTruncC) == 32
    assert ctypes.sizeof(PauliWsC) == 24


def test_invalid_arguments_rejected_without_gpu_work():
    """Argument validation happens on the host before any HIP call."""
    from paper_2410_09654_amd import _lib
    L = _lib.load()
    op = _lib.PauliOpC(200, 0, 0, 0, None, None, None)  # 200 qubits: unsupported
    ws = _lib.PauliWsC(None, 0, 0)
    rc = L.pauli_commutator(ctypes.byref(op), ctypes.byref(op), None, ctypes.byref(op),
                            ctypes.byref(ws), None)
    assert rc == _lib.PAULI_EINVAL
    bad_dtype = _lib.PauliOpC(10, 7, 0, 0, None, None, None)
    rc = L.pauli_truncate(ctypes.byref(bad_dtype), None, ctypes.byref(bad_dtype),
                          ctypes.byref(ws), None)
    assert rc == _lib.PAULI_EINVAL
    rc = L.pauli_lanczos_step(ctypes.byref(op), None, ctypes.byref(op), 0.0, None, 1,
                              ctypes.byref(op), None, ctypes.byref(ws), None)
    assert rc == _lib.PAULI_EINVAL


def test_invalid_arguments_of_the_other_entry_points():
    """The product, trace, noise, lookup and translation-symmetric entry points
    also reject bad arguments on the host, before any HIP call."""
    from paper_2410_09654_amd import _lib
    L = _lib.load()
    ws = _lib.PauliWsC(None, 0, 0)
    bad = _lib.PauliOpC(200, 0, 0, 0, None, None, None)   # 200 qubits: unsupported
    a10 = _lib.PauliOpC(10, 0, 0, 0, None, None, None)    # empty, valid
    a12 = _lib.PauliOpC(12, 0, 0, 0, None, None, None)
    r = ctypes.byref
    d2 = (ctypes.c_double * 2)()
    assert L.pauli_multiply(r(bad), r(a10), None, r(a10), r(ws), None) == _lib.PAULI_EINVAL
    assert L.pauli_multiply(r(a10), r(a12), None, r(a12), r(ws), None) == _lib.PAULI_EINVAL
    assert L.pauli_trace(r(bad), d2, r(ws), None) == _lib.PAULI_EINVAL
    assert L.pauli_add_noise(r(a10), -1.0, None) == _lib.PAULI_EINVAL
    assert L.pauli_add_noise(r(a10), float("nan"), None) == _lib.PAULI_EINVAL
    assert L.pauli_coefficients(r(a10), r(a12), d2, r(ws), None) == _lib.PAULI_EINVAL
    assert L.pauli_commutator_ts1d(r(a10), r(a12), None, r(a12), r(ws), None) == _lib.PAULI_EINVAL
    assert L.pauli_canonicalize_ts1d(r(bad), r(a10), r(ws), None) == _lib.PAULI_EINVAL
    assert L.pauli_norm2_ts1d(r(a10), None, r(ws), None) == _lib.PAULI_EINVAL
    b = ctypes.c_double()
    assert L.pauli_lanczos_step_ts1d(r(a10), None, None, 0.0, None, r(a10), r(b), r(ws),
                                     None) == _lib.PAULI_EINVAL
    assert L.pauli_lanczos_step_ts1d(r(a10), None, r(a12), 0.0, None, r(a12), r(b), r(ws),
                                     None) == _lib.PAULI_EINVAL


def _query(L, _lib, op, sizes, n=64, dtype=0, trunc=None):
    ops = [(_lib.PauliOpC(n, dtype, s, s, None, None, None) if s is not None else None)
           for s in sizes]
    nb, cap = ctypes.c_size_t(0), ctypes.c_int64(0)
    rc = L.pauli_workspace_query(op, *[ctypes.byref(o) if o is not None else None for o in ops],
                                 ctypes.byref(trunc) if trunc is not None else None,
                                 ctypes.byref(nb), ctypes.byref(cap))
    return rc, nb.value, cap.value


def test_workspace_query_runs_on_host():
    """pauli_workspace_query reads sizes only: it runs without a GPU, grows
    with the operands, bounds the output by the top-M budget and rejects
    unknown calls."""
    from paper_2410_09654_amd import _lib
    L = _lib.load()
    for op in range(12):
        rc, nb, cap = _query(L, _lib, op, [191, 1 << 14, 1 << 10])
        assert rc == _lib.PAULI_OK and nb >= 1 << 20, (op, rc)
    _, small, _ = _query(L, _lib, _lib.PAULI_Q_COMMUTATOR, [191, 1 << 12, None])
    _, big, cap = _query(L, _lib, _lib.PAULI_Q_COMMUTATOR, [191, 1 << 16, None])
    assert big > small and cap == 191 << 16
    t = _lib.PauliTruncC(0, 0.0, 1000, None)
    _, _, cap = _query(L, _lib, _lib.PAULI_Q_COMMUTATOR, [191, 1 << 16, None], trunc=t)
    assert cap == 1000
    _, _, cap = _query(L, _lib, _lib.PAULI_Q_ADD, [300, 500, None])
    assert cap == 800
    assert _query(L, _lib, 99, [1, 1, None])[0] == _lib.PAULI_EINVAL
    assert _query(L, _lib, _lib.PAULI_Q_COMMUTATOR, [None, 5, None])[0] == _lib.PAULI_EINVAL


def test_lanczos_rejects_unknown_flags():
    from paper_2410_09654_amd import _lib
    L = _lib.load()
    op = _lib.PauliOpC(10, 0, 0, 0, None, None, None)
    ws = _lib.PauliWsC(None, 0, 0)
    b = ctypes.c_double()
    rc = L.pauli_lanczos_step(ctypes.byref(op), None, ctypes.byref(op), 0.0, None, 2,
                              ctypes.byref(op), ctypes.byref(b), ctypes.byref(ws), None)
    assert rc == _lib.PAULI_EINVAL
