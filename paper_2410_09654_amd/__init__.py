"""MI355X-native Pauli-string operator engine (HIP for gfx950).

The hot path (commutator [H, O] on binary-encoded Pauli strings, duplicate
merge, truncation, and the Lanczos / Runge-Kutta steps built on them) runs in
libpauli.so behind the C ABI of include/pauli.h; this package is its thin
Python binding over torch device memory.
"""
from ._lib import PAULI_C128, PAULI_C64K, PauliError
from .ops import (PauliOp, Trunc, Workspace, add, add_noise, canonicalize, canonicalize_ts1d,
                  coefficients, commutator, commutator_ts1d, inner, lanczos_step, last_stats,
                  multiply, norm2, norm2_ts1d, order_keys, profile_enable, profile_read,
                  rk4_step, strings_from_order_keys, trace, truncate)
from .algorithms import evolve, evolve_noisy, lanczos, lanczos_ts1d, moments

__all__ = ["PAULI_C128", "PAULI_C64K", "PauliError", "PauliOp", "Trunc", "Workspace", "add",
           "canonicalize", "commutator", "inner", "lanczos_step", "norm2", "rk4_step",
           "truncate", "lanczos", "evolve", "profile_enable", "profile_read", "last_stats",
           "order_keys", "strings_from_order_keys", "multiply", "trace", "moments",
           "add_noise", "coefficients", "evolve_noisy", "commutator_ts1d",
           "canonicalize_ts1d", "norm2_ts1d", "lanczos_ts1d"]
