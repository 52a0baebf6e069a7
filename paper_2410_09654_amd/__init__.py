"""MI355X-native Pauli-string operator engine (HIP for gfx950).

The hot path (commutator [H, O] on binary-encoded Pauli strings, duplicate
merge, truncation, and the Lanczos / Runge-Kutta steps built on them) runs in
libpauli.so behind the C ABI of include/pauli.h; this package is its thin
Python binding over torch device memory.
"""
from ._lib import (PAULI_C128, PAULI_C64K, PAULI_Q_ADD, PAULI_Q_CANONICALIZE,
                   PAULI_Q_CANONICALIZE_TS1D, PAULI_Q_COMMUTATOR, PAULI_Q_COMMUTATOR_TS1D,
                   PAULI_Q_LANCZOS, PAULI_Q_LANCZOS_REORTH, PAULI_Q_LANCZOS_TS1D,
                   PAULI_Q_MULTIPLY, PAULI_Q_REDUCTION, PAULI_Q_RK4, PAULI_Q_TRUNCATE,
                   PAULI_REORTH_LOCAL, PauliError)
from .ops import (PauliOp, Trunc, Workspace, add, add_noise, canonicalize, canonicalize_ts1d,
                  coefficients, commutator, commutator_ts1d, correlator, dagger, divide, inner,
                  lanczos_step,
                  last_stats, read_totals, workspace_query,
                  multiply, norm2, norm2_ts1d, order_keys, profile_enable, profile_read,
                  rk4_step, strings_from_order_keys, trace, truncate)
from .algorithms import evolve, evolve_noisy, lanczos, lanczos_ts1d, moments

__all__ = ["PAULI_C128", "PAULI_C64K", "PauliError", "PauliOp", "Trunc", "Workspace", "add",
           "canonicalize", "commutator", "inner", "lanczos_step", "norm2", "rk4_step",
           "truncate", "lanczos", "evolve", "profile_enable", "profile_read", "last_stats",
           "order_keys", "strings_from_order_keys", "multiply", "trace", "moments",
           "add_noise", "dagger", "divide", "coefficients", "evolve_noisy", "commutator_ts1d",
           "canonicalize_ts1d", "norm2_ts1d", "lanczos_ts1d", "correlator",
           "workspace_query", "read_totals", "PAULI_REORTH_LOCAL", "PAULI_Q_COMMUTATOR", "PAULI_Q_MULTIPLY",
           "PAULI_Q_ADD", "PAULI_Q_TRUNCATE", "PAULI_Q_CANONICALIZE", "PAULI_Q_LANCZOS",
           "PAULI_Q_LANCZOS_REORTH", "PAULI_Q_RK4", "PAULI_Q_COMMUTATOR_TS1D",
           "PAULI_Q_CANONICALIZE_TS1D", "PAULI_Q_LANCZOS_TS1D", "PAULI_Q_REDUCTION"]
