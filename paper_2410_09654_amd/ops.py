"""Device operators and the operations of the C ABI, over torch device memory.

Every step of the computation runs in the HIP library (libpauli.so); this
module only allocates torch tensors, fills the ABI structs with their
pointers and the current HIP stream, and retries a call when the library
reports that an output or the workspace was too small.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import (PAULI_BREAKDOWN, PAULI_C64K, PAULI_C128, PAULI_ECAPACITY, PAULI_EWORKSPACE,
                   PAULI_OK, PauliError, PauliOpC, PauliTruncC, PauliWsC)


def _words(n_qubits: int) -> int:
    return (n_qubits + 63) // 64


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class PauliOp:
    """A sum of Pauli strings held in device memory in the library's layout.

    x, z: int64 tensors [W, capacity] (bit patterns of the uint64 masks);
    coef: float64 [capacity, 2] (PAULI_C128) or float32 [capacity, 2]
    (PAULI_C64K).  Only the first `size` rows are meaningful.
    """

    def __init__(self, n_qubits: int, capacity: int, dtype: int = PAULI_C128,
                 device: str | torch.device = "cuda"):
        self.n_qubits = int(n_qubits)
        self.dtype = int(dtype)
        self.capacity = max(int(capacity), 1)
        W = _words(n_qubits)
        # rows at and above `size` are never read: no fill kernels
        self.x = torch.empty((W, self.capacity), dtype=torch.int64, device=device)
        self.z = torch.empty((W, self.capacity), dtype=torch.int64, device=device)
        ft = torch.float64 if self.dtype == PAULI_C128 else torch.float32
        self.coef = torch.empty((self.capacity, 2), dtype=ft, device=device)
        self.size = 0

    @property
    def W(self):
        return _words(self.n_qubits)

    @property
    def device(self):
        return self.x.device

    def c_struct(self) -> PauliOpC:
        return PauliOpC(self.n_qubits, self.dtype, self.size, self.capacity,
                        self.x.data_ptr(), self.z.data_ptr(), self.coef.data_ptr())

    def __len__(self):
        return self.size

    # -- host transfer ---------------------------------------------------------
    @classmethod
    def from_raw(cls, n_qubits, x: np.ndarray, z: np.ndarray, coef: np.ndarray,
                 dtype: int = PAULI_C128, device="cuda") -> "PauliOp":
        """Upload (n, W) uint64 masks and complex coefficients without any
        canonicalisation (the rows must be distinct strings)."""
        n = int(coef.shape[0])
        op = cls(n_qubits, max(n, 1), dtype, device)
        if n:
            xs = np.ascontiguousarray(np.asarray(x, np.uint64).reshape(n, -1).T).view(np.int64)
            zs = np.ascontiguousarray(np.asarray(z, np.uint64).reshape(n, -1).T).view(np.int64)
            op.x[:, :n] = torch.from_numpy(xs).to(device)
            op.z[:, :n] = torch.from_numpy(zs).to(device)
            c = np.stack([np.real(coef), np.imag(coef)], axis=1)
            op.coef[:n] = torch.from_numpy(c).to(device=device, dtype=op.coef.dtype)
        op.size = n
        return op

    @classmethod
    def from_host(cls, host, dtype: int = PAULI_C128, device="cuda", ws=None) -> "PauliOp":
        """Upload a workloads.HostOp and bring it to canonical form on the GPU."""
        raw = cls.from_raw(host.n_qubits, host.x, host.z, host.coef, dtype, device)
        return canonicalize(raw, ws=ws)

    @classmethod
    def from_terms(cls, n_qubits: int, terms, dtype: int = PAULI_C128, device="cuda",
                   ws=None) -> "PauliOp":
        """Operator from terms (coef, "XZ", [i, j]): letters X, Y, Z (I or 1 for the
        identity) on the given 1-based sites; strings that repeat are summed in
        the order given.  Canonical on return."""
        W = _words(n_qubits)
        terms = list(terms)
        x = np.zeros((len(terms), W), np.uint64)
        z = np.zeros((len(terms), W), np.uint64)
        coef = np.zeros(len(terms), np.complex128)
        bits = {"X": (1, 0), "Y": (1, 1), "Z": (0, 1), "I": (0, 0), "1": (0, 0)}
        for k, (c, letters, sites) in enumerate(terms):
            if len(letters) != len(sites):
                raise ValueError(f"term {k}: {len(letters)} letters for {len(sites)} sites")
            coef[k] = c
            for ch, site in zip(letters, sites):
                if not 1 <= int(site) <= n_qubits or ch not in bits:
                    raise ValueError(f"term {k}: bad factor {ch}{site}")
                w, b = divmod(int(site) - 1, 64)
                bx, bz = bits[ch]
                if (x[k, w] >> np.uint64(b)) & np.uint64(1) or (z[k, w] >> np.uint64(b)) & np.uint64(1):
                    raise ValueError(f"term {k}: site {site} given twice")
                x[k, w] |= np.uint64(bx) << np.uint64(b)
                z[k, w] |= np.uint64(bz) << np.uint64(b)
        raw = cls.from_raw(n_qubits, x, z, coef, dtype, device)
        return canonicalize(raw, ws=ws)

    def to_strings(self):
        """The operator as lines "(re + im im) XYZ1...": site 1 leftmost, 1 for the
        identity, in storage order."""
        x, z, c = self.to_numpy()
        letters = {(0, 0): "1", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}
        lines = []
        for k in range(len(c)):
            text = "".join(
                letters[(int(x[k, j // 64] >> np.uint64(j % 64)) & 1,
                         int(z[k, j // 64] >> np.uint64(j % 64)) & 1)]
                for j in range(self.n_qubits))
            sign = "-" if np.signbit(c[k].imag) else "+"
            # a zero real part prints as 0, whatever its sign bit
            lines.append(f"({c[k].real + 0.0:.10g} {sign} {abs(c[k].imag):.10g}im) {text}")
        return lines

    def to_numpy(self):
        n = self.size
        x = self.x[:, :n].cpu().numpy().view(np.uint64).T.copy()
        z = self.z[:, :n].cpu().numpy().view(np.uint64).T.copy()
        c = self.coef[:n].cpu().to(torch.float64).numpy()
        return x, z, c[:, 0] + 1j * c[:, 1]

    def to_host(self):
        from workloads import HostOp
        x, z, c = self.to_numpy()
        return HostOp(self.n_qubits, x, z, c)

    # -- checkpoints -------------------------------------------------------------
    def save(self, path: str):
        """Checkpoint: the operator's rows as stored (word-major masks, coefficients
        in their own precision, the library's order) in one .npz file."""
        n = self.size
        np.savez(path, n_qubits=np.int64(self.n_qubits), dtype=np.int64(self.dtype),
                 x=self.x[:, :n].cpu().numpy().view(np.uint64),
                 z=self.z[:, :n].cpu().numpy().view(np.uint64),
                 coef=self.coef[:n].cpu().numpy())

    @classmethod
    def load(cls, path: str, device="cuda") -> "PauliOp":
        """An operator saved by `save`, restored row for row (no recomputation)."""
        with np.load(path, allow_pickle=False) as f:
            n_qubits, dtype = int(f["n_qubits"]), int(f["dtype"])
            x, z, coef = f["x"], f["z"], f["coef"]
        n = coef.shape[0]
        op = cls(n_qubits, max(n, 1), dtype, device)
        if n:
            op.x[:, :n] = torch.from_numpy(np.ascontiguousarray(x).view(np.int64)).to(device)
            op.z[:, :n] = torch.from_numpy(np.ascontiguousarray(z).view(np.int64)).to(device)
            op.coef[:n] = torch.from_numpy(np.ascontiguousarray(coef)).to(device)
        op.size = n
        return op


class Trunc:
    """Truncation parameters (see pauli_trunc in include/pauli.h)."""

    def __init__(self, max_len: int = 0, coef_eps: float = 0.0, max_strings: int = 0,
                 keep: PauliOp | None = None):
        self.max_len, self.coef_eps, self.max_strings, self.keep = \
            int(max_len), float(coef_eps), int(max_strings), keep

    def c_struct(self):
        keep_s = self.keep.c_struct() if self.keep is not None else None
        kp = ctypes.pointer(keep_s) if keep_s is not None else ctypes.POINTER(PauliOpC)()
        return keep_s, PauliTruncC(self.max_len, self.coef_eps, self.max_strings, kp)

    def bound(self):
        """Upper bound of the output size, or None."""
        if self.max_strings > 0:
            return self.max_strings + (self.keep.size if self.keep is not None else 0)
        return None


class Workspace:
    """Grow-only device scratch handed to the library."""

    def __init__(self, nbytes: int = 64 << 20, device="cuda"):
        self.device = device
        self.buf = torch.empty(max(int(nbytes), 1 << 20), dtype=torch.uint8, device=device)

    def c_struct(self) -> PauliWsC:
        return PauliWsC(self.buf.data_ptr(), self.buf.numel(), 0)

    def grow(self, required: int):
        n = max(int(required), int(self.buf.numel() * 1.5))
        del self.buf
        self.buf = torch.empty(n, dtype=torch.uint8, device=self.device)

    @property
    def nbytes(self):
        return self.buf.numel()


_default_ws = {}


def default_workspace(device="cuda") -> Workspace:
    key = str(torch.device(device))
    if key not in _default_ws:
        _default_ws[key] = Workspace(device=device)
    return _default_ws[key]


def _call(name, fn, ws: Workspace, out: PauliOp | None, max_retry: int = 8):
    """Run fn(ws_struct) -> status with workspace / capacity retries.

    fn returns (status, out_struct or None)."""
    for _ in range(max_retry):
        wss = ws.c_struct()
        status, outs = fn(wss)
        if status == PAULI_EWORKSPACE:
            ws.grow(wss.required)
            continue
        if status == PAULI_ECAPACITY and out is not None and outs is not None:
            need = int(outs.size)
            out.__init__(out.n_qubits, max(need, 1), out.dtype, out.device)
            continue
        if status not in (PAULI_OK, PAULI_BREAKDOWN):
            raise PauliError(status, name, _lib.last_error())
        if out is not None and outs is not None:
            out.size = int(outs.size)
        return status
    raise PauliError(status, name, "retries exhausted")


def _out_like(n_qubits, guess, dtype, device):
    return PauliOp(n_qubits, max(int(guess), 1), dtype, device)


def commutator(H: PauliOp, O: PauliOp, trunc: Trunc | None = None, out: PauliOp | None = None,
               ws: Workspace | None = None) -> PauliOp:
    """[H, O] (then truncated), on the GPU."""
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    if out is None:
        b = trunc.bound() if trunc else None
        guess = b if b is not None else min(H.size * O.size, 16 * O.size + 1024)
        out = _out_like(O.n_qubits, guess, O.dtype, O.device)
    hs, os_ = H.c_struct(), O.c_struct()
    keep_s, ts = trunc.c_struct() if trunc else (None, None)

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_commutator(ctypes.byref(hs), ctypes.byref(os_),
                                ctypes.byref(ts) if ts is not None else None,
                                ctypes.byref(outs), ctypes.byref(wss), _stream_handle())
        return st, outs

    _call("pauli_commutator", fn, ws, out)
    return out


def multiply(A: PauliOp, B: PauliOp, trunc: Trunc | None = None, out: PauliOp | None = None,
             ws: Workspace | None = None) -> PauliOp:
    """A B (then truncated), on the GPU: every pair of strings, no filter."""
    L = _lib.load()
    ws = ws or default_workspace(B.device)
    if out is None:
        b = trunc.bound() if trunc else None
        guess = b if b is not None else min(A.size * B.size, 16 * B.size + 1024)
        out = _out_like(B.n_qubits, guess, B.dtype, B.device)
    As, Bs = A.c_struct(), B.c_struct()
    keep_s, ts = trunc.c_struct() if trunc else (None, None)

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_multiply(ctypes.byref(As), ctypes.byref(Bs),
                              ctypes.byref(ts) if ts is not None else None,
                              ctypes.byref(outs), ctypes.byref(wss), _stream_handle())
        return st, outs

    _call("pauli_multiply", fn, ws, out)
    return out


def commutator_ts1d(H0: PauliOp, O: PauliOp, trunc: Trunc | None = None,
                    out: PauliOp | None = None, ws: Workspace | None = None) -> PauliOp:
    """Translation-symmetric [H, O] on the periodic chain (Alg. 2): O and the
    result hold one representative string per translation orbit."""
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    if out is None:
        b = trunc.bound() if trunc else None
        guess = b if b is not None else min(H0.size * O.n_qubits * O.size, 16 * O.size + 1024)
        out = _out_like(O.n_qubits, guess, O.dtype, O.device)
    hs, os_ = H0.c_struct(), O.c_struct()
    keep_s, ts = trunc.c_struct() if trunc else (None, None)

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_commutator_ts1d(ctypes.byref(hs), ctypes.byref(os_),
                                     ctypes.byref(ts) if ts is not None else None,
                                     ctypes.byref(outs), ctypes.byref(wss), _stream_handle())
        return st, outs

    _call("pauli_commutator_ts1d", fn, ws, out)
    return out


def canonicalize_ts1d(A: PauliOp, ws: Workspace | None = None) -> PauliOp:
    """Every string replaced by its translation-orbit representative,
    duplicates summed in input order."""
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    out = _out_like(A.n_qubits, max(A.size, 1), A.dtype, A.device)
    As = A.c_struct()

    def fn(wss):
        outs = out.c_struct()
        return L.pauli_canonicalize_ts1d(ctypes.byref(As), ctypes.byref(outs),
                                         ctypes.byref(wss), _stream_handle()), outs

    _call("pauli_canonicalize_ts1d", fn, ws, out)
    return out


def norm2_ts1d(A: PauliOp, ws: Workspace | None = None) -> float:
    """||sum_k T_k(A)||^2 / N for representatives A."""
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    As = A.c_struct()
    r = ctypes.c_double()

    def fn(wss):
        return L.pauli_norm2_ts1d(ctypes.byref(As), ctypes.byref(r), ctypes.byref(wss),
                                  _stream_handle()), None

    _call("pauli_norm2_ts1d", fn, ws, None)
    return r.value


def trace(A: PauliOp, ws: Workspace | None = None) -> complex:
    """Tr(A)/2^N: the coefficient of the identity string."""
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    As = A.c_struct()
    r = (ctypes.c_double * 2)()

    def fn(wss):
        return L.pauli_trace(ctypes.byref(As), r, ctypes.byref(wss), _stream_handle()), None

    _call("pauli_trace", fn, ws, None)
    return complex(r[0], r[1])


def add_noise(A: PauliOp, lam: float) -> PauliOp:
    """Depolarizing noise in place: c *= exp(-lam * length); returns A."""
    L = _lib.load()
    As = A.c_struct()
    st = L.pauli_add_noise(ctypes.byref(As), float(lam), _stream_handle())
    if st != PAULI_OK:
        raise PauliError(st, "pauli_add_noise", _lib.last_error())
    return A


def dagger(A: PauliOp) -> PauliOp:
    """A <- A^dagger in place (conjugated coefficients: every string is
    Hermitian); returns A."""
    L = _lib.load()
    As = A.c_struct()
    st = L.pauli_dagger(ctypes.byref(As), _stream_handle())
    if st != PAULI_OK:
        raise PauliError(st, "pauli_dagger", _lib.last_error())
    return A


def coefficients(A: PauliOp, Q: PauliOp, ws: Workspace | None = None) -> np.ndarray:
    """complex128 [Q.size]: A's coefficient of each string of Q (0 if absent)."""
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    As, Qs = A.c_struct(), Q.c_struct()
    r = (ctypes.c_double * (2 * max(Q.size, 1)))()

    def fn(wss):
        return L.pauli_coefficients(ctypes.byref(As), ctypes.byref(Qs), r, ctypes.byref(wss),
                                    _stream_handle()), None

    _call("pauli_coefficients", fn, ws, None)
    v = np.frombuffer(r, dtype=np.float64)[:2 * Q.size]
    return v[0::2] + 1j * v[1::2]


def add(A: PauliOp, alpha: complex, B: PauliOp, beta: complex, trunc: Trunc | None = None,
        out: PauliOp | None = None, ws: Workspace | None = None) -> PauliOp:
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    alpha, beta = complex(alpha), complex(beta)
    if out is None:
        b = trunc.bound() if trunc else None
        guess = min(b, A.size + B.size) if b is not None else A.size + B.size
        out = _out_like(A.n_qubits, guess, A.dtype, A.device)
    As, Bs = A.c_struct(), B.c_struct()
    keep_s, ts = trunc.c_struct() if trunc else (None, None)

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_add(ctypes.byref(As), alpha.real, alpha.imag, ctypes.byref(Bs), beta.real,
                         beta.imag, ctypes.byref(ts) if ts is not None else None,
                         ctypes.byref(outs), ctypes.byref(wss), _stream_handle())
        return st, outs

    _call("pauli_add", fn, ws, out)
    return out


def truncate(O: PauliOp, trunc: Trunc, out: PauliOp | None = None,
             ws: Workspace | None = None) -> PauliOp:
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    if out is None:
        b = trunc.bound()
        out = _out_like(O.n_qubits, min(b, O.size) if b else O.size, O.dtype, O.device)
    Os = O.c_struct()
    keep_s, ts = trunc.c_struct()

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_truncate(ctypes.byref(Os), ctypes.byref(ts), ctypes.byref(outs),
                              ctypes.byref(wss), _stream_handle())
        return st, outs

    _call("pauli_truncate", fn, ws, out)
    return out


def divide(O: PauliOp, b: float, out: PauliOp | None = None,
           ws: Workspace | None = None) -> PauliOp:
    """O / b for a finite real b != 0 (IEEE division of each part, exact zeros
    dropped), canonical."""
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    if out is None:
        out = _out_like(O.n_qubits, O.size, O.dtype, O.device)
    Os = O.c_struct()

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_divide(ctypes.byref(Os), float(b), ctypes.byref(outs), ctypes.byref(wss),
                            _stream_handle())
        return st, outs

    _call("pauli_divide", fn, ws, out)
    return out


def canonicalize(O: PauliOp, out: PauliOp | None = None, ws: Workspace | None = None) -> PauliOp:
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    if out is None:
        out = _out_like(O.n_qubits, O.size, O.dtype, O.device)
    Os = O.c_struct()

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_canonicalize(ctypes.byref(Os), ctypes.byref(outs), ctypes.byref(wss),
                                  _stream_handle())
        return st, outs

    _call("pauli_canonicalize", fn, ws, out)
    return out


def lanczos_step(H: PauliOp, O_prev: PauliOp | None, O_cur: PauliOp, b_prev: float,
                 trunc: Trunc | None = None, out: PauliOp | None = None,
                 ws: Workspace | None = None, ts1d: bool = False, reorth: bool = False):
    """(O_next, b_n, breakdown) of one Liouvillian Lanczos step on the GPU;
    ts1d: H holds H0 and the operators orbit representatives of the periodic
    chain (translation-symmetric step, Alg. 2); reorth: local
    re-orthogonalisation against O_cur and O_prev (PAULI_REORTH_LOCAL)."""
    if ts1d and reorth:
        raise ValueError("re-orthogonalisation is not offered for translation-symmetric steps")
    L = _lib.load()
    ws = ws or default_workspace(O_cur.device)
    if out is None:
        b = trunc.bound() if trunc else None
        guess = b if b is not None else min(H.size * O_cur.size + (O_prev.size if O_prev else 0),
                                            16 * O_cur.size + 1024)
        out = _out_like(O_cur.n_qubits, guess, O_cur.dtype, O_cur.device)
    hs, cs = H.c_struct(), O_cur.c_struct()
    ps = O_prev.c_struct() if O_prev is not None else None
    keep_s, ts = trunc.c_struct() if trunc else (None, None)
    bval = ctypes.c_double(0.0)

    def fn(wss):
        outs = out.c_struct()
        pp = ctypes.byref(ps) if ps is not None else None
        tp = ctypes.byref(ts) if ts is not None else None
        if ts1d:
            st = L.pauli_lanczos_step_ts1d(ctypes.byref(hs), pp, ctypes.byref(cs), float(b_prev),
                                           tp, ctypes.byref(outs), ctypes.byref(bval),
                                           ctypes.byref(wss), _stream_handle())
        else:
            st = L.pauli_lanczos_step(ctypes.byref(hs), pp, ctypes.byref(cs), float(b_prev), tp,
                                      _lib.PAULI_REORTH_LOCAL if reorth else 0,
                                      ctypes.byref(outs), ctypes.byref(bval),
                                      ctypes.byref(wss), _stream_handle())
        return st, outs

    st = _call("pauli_lanczos_step_ts1d" if ts1d else "pauli_lanczos_step", fn, ws, out)
    return out, bval.value, st == PAULI_BREAKDOWN


def rk4_step(H: PauliOp, O: PauliOp, dt: float, trunc: Trunc | None = None,
             out: PauliOp | None = None, ws: Workspace | None = None) -> PauliOp:
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    if out is None:
        b = trunc.bound() if trunc else None
        guess = b if b is not None else 64 * O.size + 1024
        out = _out_like(O.n_qubits, guess, O.dtype, O.device)
    hs, os_ = H.c_struct(), O.c_struct()
    keep_s, ts = trunc.c_struct() if trunc else (None, None)

    def fn(wss):
        outs = out.c_struct()
        st = L.pauli_rk4_step(ctypes.byref(hs), ctypes.byref(os_), float(dt),
                              ctypes.byref(ts) if ts is not None else None, ctypes.byref(outs),
                              ctypes.byref(wss), _stream_handle())
        return st, outs

    _call("pauli_rk4_step", fn, ws, out)
    return out


def norm2(A: PauliOp, ws: Workspace | None = None) -> float:
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    As = A.c_struct()
    r = ctypes.c_double()

    def fn(wss):
        return L.pauli_norm2(ctypes.byref(As), ctypes.byref(r), ctypes.byref(wss),
                             _stream_handle()), None

    _call("pauli_norm2", fn, ws, None)
    return r.value


def inner(A: PauliOp, B: PauliOp, ws: Workspace | None = None) -> complex:
    """<A, B> = Tr(A^dagger B)/2^N; B must be canonical."""
    L = _lib.load()
    ws = ws or default_workspace(A.device)
    As, Bs = A.c_struct(), B.c_struct()
    r = (ctypes.c_double * 2)()

    def fn(wss):
        return L.pauli_inner(ctypes.byref(As), ctypes.byref(Bs), r, ctypes.byref(wss),
                             _stream_handle()), None

    _call("pauli_inner", fn, ws, None)
    return complex(r[0], r[1])


def order_keys(A: PauliOp) -> torch.Tensor:
    """[A.size, 2W] int64 order keys: ascending (word 0 first, unsigned) is the
    canonical storage order."""
    L = _lib.load()
    keys = torch.empty((max(A.size, 1), 2 * A.W), dtype=torch.int64, device=A.device)
    As = A.c_struct()
    st = L.pauli_order_keys(ctypes.byref(As), keys.data_ptr(), _stream_handle())
    if st != PAULI_OK:
        raise PauliError(st, "pauli_order_keys", _lib.last_error())
    return keys[:A.size]


def strings_from_order_keys(n_qubits: int, keys: torch.Tensor):
    """(x, z) int64 [W, n] of the strings with the given [n, 2W] order keys."""
    L = _lib.load()
    keys = keys.contiguous()
    n = keys.shape[0]
    W = (n_qubits + 63) // 64
    x = torch.zeros((W, max(n, 1)), dtype=torch.int64, device=keys.device)
    z = torch.zeros_like(x)
    st = L.pauli_strings_from_order_keys(n_qubits, keys.data_ptr(), n, x.data_ptr(), z.data_ptr(),
                                         x.shape[1], _stream_handle())
    if st != PAULI_OK:
        raise PauliError(st, "pauli_strings_from_order_keys", _lib.last_error())
    return x[:, :n], z[:, :n]


# -- kernel timing -------------------------------------------------------------

def profile_enable(on: bool = True, only=None):
    """Start (or stop) per-kernel event timing and clear the log.  `only`: the
    kernel names to time (each costs two event records per launch); None
    times every kernel."""
    L = _lib.load()
    L.pauli_profile_only(",".join(only).encode() if only else None)
    L.pauli_profile_enable(1 if on else 0)


def profile_read() -> dict:
    L = _lib.load()
    n = L.pauli_profile_read(None, 0)
    buf = ctypes.create_string_buffer(n + 1)
    L.pauli_profile_read(buf, n + 1)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def correlator(O0: PauliOp, O: PauliOp, ws: Workspace | None = None) -> complex:
    """S = <O0, O> / <O0, O0> (pauli_correlator; O0 canonical)."""
    L = _lib.load()
    ws = ws or default_workspace(O.device)
    a, b = O0.c_struct(), O.c_struct()
    res = (ctypes.c_double * 2)()
    _call("pauli_correlator",
          lambda wss: (L.pauli_correlator(ctypes.byref(a), ctypes.byref(b), res,
                                          ctypes.byref(wss), _stream_handle()), None), ws, None)
    return complex(res[0], res[1])


def workspace_query(op: int, A: PauliOp | None, B: PauliOp | None, C: PauliOp | None = None,
                    trunc: Trunc | None = None):
    """(workspace bytes, output capacity) that pauli_workspace_query gives
    for call `op` (one of the PAULI_Q_* codes) on these operands."""
    L = _lib.load()
    structs = [o.c_struct() if o is not None else None for o in (A, B, C)]
    keep_s, ts = trunc.c_struct() if trunc else (None, None)
    nb, cap = ctypes.c_size_t(0), ctypes.c_int64(0)
    st = L.pauli_workspace_query(int(op), *[ctypes.byref(x) if x is not None else None
                                            for x in structs],
                                 ctypes.byref(ts) if ts is not None else None,
                                 ctypes.byref(nb), ctypes.byref(cap))
    if st != PAULI_OK:
        raise PauliError(st, "pauli_workspace_query", _lib.last_error())
    return int(nb.value), int(cap.value)


def read_totals(reset: bool = False) -> dict:
    """Totals over every engine pass since the last reset (pauli_read_totals)."""
    t = _lib.PauliTotalsC()
    _lib.load().pauli_read_totals(ctypes.byref(t), 1 if reset else 0)
    return {k: getattr(t, k) for k, _ in _lib.PauliTotalsC._fields_}


def last_stats() -> dict:
    """Counters of the last engine pass on this thread (see pauli_stats)."""
    st = _lib.PauliStatsC()
    _lib.load().pauli_last_stats(ctypes.byref(st))
    return {k: getattr(st, k) for k, _ in _lib.PauliStatsC._fields_}
