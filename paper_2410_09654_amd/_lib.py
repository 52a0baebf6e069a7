"""ctypes declarations of the C ABI in include/pauli.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpauli.so")

PAULI_OK, PAULI_EINVAL, PAULI_ECAPACITY, PAULI_EWORKSPACE, PAULI_BREAKDOWN, PAULI_EHIP, \
    PAULI_EINTERNAL = range(7)
PAULI_C128, PAULI_C64K = 0, 1
PAULI_REORTH_LOCAL = 1
(PAULI_Q_COMMUTATOR, PAULI_Q_MULTIPLY, PAULI_Q_ADD, PAULI_Q_TRUNCATE, PAULI_Q_CANONICALIZE,
 PAULI_Q_LANCZOS, PAULI_Q_LANCZOS_REORTH, PAULI_Q_RK4, PAULI_Q_COMMUTATOR_TS1D,
 PAULI_Q_CANONICALIZE_TS1D, PAULI_Q_LANCZOS_TS1D, PAULI_Q_REDUCTION) = range(12)

EXPORTS = ["pauli_commutator", "pauli_multiply", "pauli_trace", "pauli_add", "pauli_truncate",
           "pauli_canonicalize", "pauli_divide", "pauli_add_noise", "pauli_dagger", "pauli_coefficients",
           "pauli_commutator_ts1d", "pauli_canonicalize_ts1d", "pauli_norm2_ts1d",
           "pauli_lanczos_step_ts1d",
           "pauli_rk4_step", "pauli_lanczos_step", "pauli_norm2", "pauli_inner",
           "pauli_correlator", "pauli_workspace_query", "pauli_commutator_noalloc",
           "pauli_read_totals",
           "pauli_strerror", "pauli_last_error", "pauli_profile_enable", "pauli_profile_only", "pauli_profile_read",
           "pauli_last_stats", "pauli_order_keys", "pauli_strings_from_order_keys",
           "pauli_mlp_num_params", "pauli_mlp_sync", "pauli_mlp_forward",
           "pauli_mlp_loss_grad", "pauli_mlp_adam", "pauli_gemm_bf16", "pauli_mlp_train"]


class PauliOpC(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("size", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("z", ctypes.c_void_p), ("coef", ctypes.c_void_p)]


class PauliTruncC(ctypes.Structure):
    _fields_ = [("max_len", ctypes.c_int32), ("coef_eps", ctypes.c_double),
                ("max_strings", ctypes.c_int64), ("keep", ctypes.POINTER(PauliOpC))]


class PauliWsC(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("bytes", ctypes.c_size_t),
                ("required", ctypes.c_size_t)]


class PauliStatsC(ctypes.Structure):
    _fields_ = [("emitted", ctypes.c_int64), ("unique", ctypes.c_int64),
                ("survivors", ctypes.c_int64), ("output", ctypes.c_int64),
                ("passes", ctypes.c_int32), ("buckets", ctypes.c_int32),
                ("host_syncs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PauliTotalsC(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("inputs", ctypes.c_int64),
                ("emitted", ctypes.c_int64), ("unique", ctypes.c_int64),
                ("output", ctypes.c_int64), ("alg_bytes", ctypes.c_double)]


class PauliError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: status {status} ({strerror(status)}) {detail}".strip())


_lib = None


def load():
    """Load libpauli.so.  Raises if it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with "
                          "`python -m paper_2410_09654_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    op, tr, ws = P(PauliOpC), P(PauliTruncC), P(PauliWsC)
    vp, d = ctypes.c_void_p, ctypes.c_double
    L.pauli_commutator.argtypes = [op, op, tr, op, ws, vp]
    L.pauli_multiply.argtypes = [op, op, tr, op, ws, vp]
    L.pauli_commutator_noalloc.argtypes = [op, op, tr, op, vp]
    L.pauli_trace.argtypes = [op, P(d), ws, vp]
    L.pauli_add_noise.argtypes = [op, d, vp]
    L.pauli_dagger.argtypes = [op, vp]
    L.pauli_divide.argtypes = [op, d, op, ws, vp]
    L.pauli_commutator_ts1d.argtypes = [op, op, tr, op, ws, vp]
    L.pauli_canonicalize_ts1d.argtypes = [op, op, ws, vp]
    L.pauli_norm2_ts1d.argtypes = [op, P(d), ws, vp]
    L.pauli_lanczos_step_ts1d.argtypes = [op, op, op, d, tr, op, P(d), ws, vp]
    L.pauli_coefficients.argtypes = [op, op, P(d), ws, vp]
    L.pauli_add.argtypes = [op, d, d, op, d, d, tr, op, ws, vp]
    L.pauli_truncate.argtypes = [op, tr, op, ws, vp]
    L.pauli_canonicalize.argtypes = [op, op, ws, vp]
    L.pauli_rk4_step.argtypes = [op, op, d, tr, op, ws, vp]
    L.pauli_lanczos_step.argtypes = [op, op, op, d, tr, ctypes.c_uint32, op, P(d), ws, vp]
    L.pauli_norm2.argtypes = [op, P(d), ws, vp]
    L.pauli_inner.argtypes = [op, op, P(d), ws, vp]
    L.pauli_correlator.argtypes = [op, op, P(d), ws, vp]
    L.pauli_workspace_query.argtypes = [ctypes.c_int, op, op, op, tr, P(ctypes.c_size_t),
                                        P(ctypes.c_int64)]
    L.pauli_strerror.argtypes = [ctypes.c_int]
    L.pauli_strerror.restype = ctypes.c_char_p
    L.pauli_last_error.argtypes = []
    L.pauli_last_error.restype = ctypes.c_char_p
    L.pauli_profile_enable.argtypes = [ctypes.c_int]
    L.pauli_profile_only.argtypes = [ctypes.c_char_p]
    L.pauli_profile_read.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.pauli_profile_read.restype = ctypes.c_size_t
    L.pauli_last_stats.argtypes = [P(PauliStatsC)]
    L.pauli_last_stats.restype = None
    L.pauli_read_totals.argtypes = [P(PauliTotalsC), ctypes.c_int]
    L.pauli_read_totals.restype = None
    L.pauli_order_keys.argtypes = [P(PauliOpC), ctypes.c_void_p, ctypes.c_void_p]
    L.pauli_strings_from_order_keys.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_int64, ctypes.c_void_p]
    for name in EXPORTS:
        if name in ("pauli_strerror", "pauli_last_error", "pauli_profile_read",
                    "pauli_last_stats", "pauli_read_totals"):
            continue
        if name == "pauli_mlp_num_params":
            L[name].restype = ctypes.c_int64
            continue
        L[name].restype = (None if name in ("pauli_profile_enable", "pauli_profile_only")
                            else ctypes.c_int)
    _lib = L
    return L


def strerror(status: int) -> str:
    try:
        return load().pauli_strerror(status).decode()
    except ImportError:
        return str(status)


def last_error() -> str:
    return load().pauli_last_error().decode()
