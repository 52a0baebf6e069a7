"""Learned continuation of Lanczos coefficients.

A small network (16 -> 256 -> 256 -> 16, GELU) reads a window of 16
consecutive Lanczos coefficients b_n, scaled by the window mean, and predicts
the next 16.  It is trained on the GPU by the library's own BF16 matrix-core
forward and backward kernels (pauli_mlp_*) on b_n sequences that the Lanczos
recursion of this library computed, and the plain truncated recursion remains
its fallback and the reference for its error.  The paper notes that a few Lanczos
coefficients can suffice to estimate long-time dynamics; this component
extrapolates the sequence beyond the computed depth.

This module only marshals tensors and sequences C-ABI calls; every matrix
product, activation, loss, gradient and optimizer update runs in libpauli.so.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import PAULI_OK, PauliError
from .ops import Workspace, _stream_handle, default_workspace

WIN, HID, OUT = 16, 256, 16


class PauliMlpC(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("params", ctypes.c_void_p),
                ("params_bf16", ctypes.c_void_p), ("grads", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p)]


def _check(status, name):
    if status != PAULI_OK:
        raise PauliError(status, name, _lib.last_error())


def _setup(L):
    if getattr(L, "_mlp_ready", False):
        return
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.pauli_mlp_num_params.restype = ctypes.c_int64
    L.pauli_mlp_sync.argtypes = [P(PauliMlpC), vp]
    L.pauli_mlp_forward.argtypes = [P(PauliMlpC), vp, ctypes.c_int64, vp, P(_lib.PauliWsC), vp]
    L.pauli_mlp_loss_grad.argtypes = [P(PauliMlpC), vp, vp, vp, ctypes.c_int64,
                                      P(ctypes.c_double), vp, P(_lib.PauliWsC), vp]
    L.pauli_mlp_adam.argtypes = [P(PauliMlpC), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int64, vp]
    L.pauli_gemm_bf16.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                  vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    d = ctypes.c_double
    L.pauli_mlp_train.argtypes = [P(PauliMlpC), vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int64,
                                  ctypes.c_int32, d, d, d, d, ctypes.c_int64, vp,
                                  P(_lib.PauliWsC), vp]
    for f in ("pauli_mlp_sync", "pauli_mlp_forward", "pauli_mlp_loss_grad", "pauli_mlp_adam",
              "pauli_gemm_bf16", "pauli_mlp_train"):
        L[f].restype = ctypes.c_int
    L._mlp_ready = True


def lib():
    L = _lib.load()
    _setup(L)
    return L


def param_offsets():
    o = {}
    off = 0
    for name, n in (("W1", HID * WIN), ("b1", HID), ("W2", HID * HID), ("b2", HID),
                    ("W3", OUT * HID), ("b3", OUT)):
        o[name] = (off, n)
        off += n
    return o, off


class BnSurrogate:
    """Parameters, gradients and Adam state of the network in device memory."""

    def __init__(self, seed: int = 0, device="cuda", ws: Workspace | None = None):
        L = lib()
        self.n = int(L.pauli_mlp_num_params())
        offs, total = param_offsets()
        assert total == self.n
        self.device = device
        self.ws = ws or default_workspace(device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        p = torch.zeros(self.n, dtype=torch.float32)
        # uniform initialisation with bound 1/sqrt(fan_in) for weights and biases
        for name, (o, n) in offs.items():
            fan_in = {"W1": WIN, "b1": WIN, "W2": HID, "b2": HID, "W3": HID, "b3": HID}[name]
            bound = 1.0 / math.sqrt(fan_in)
            p[o:o + n] = (torch.rand(n, generator=g) * 2 - 1) * bound
        self.params = p.to(device)
        self.params_bf16 = torch.zeros(self.n, dtype=torch.int16, device=device)
        self.grads = torch.zeros(self.n, dtype=torch.float32, device=device)
        self.adam_m = torch.zeros(self.n, dtype=torch.float32, device=device)
        self.adam_v = torch.zeros(self.n, dtype=torch.float32, device=device)
        self.t = 0
        _check(L.pauli_mlp_sync(ctypes.byref(self.c_struct()), _stream_handle()), "pauli_mlp_sync")

    def c_struct(self):
        return PauliMlpC(WIN, HID, OUT, self.params.data_ptr(), self.params_bf16.data_ptr(),
                         self.grads.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr())

    def _ws_call(self, fn, name):
        for _ in range(4):
            wss = self.ws.c_struct()
            st = fn(wss)
            if st == _lib.PAULI_EWORKSPACE:
                self.ws.grow(wss.required)
                continue
            _check(st, name)
            return
        raise PauliError(st, name, "workspace retries exhausted")

    @staticmethod
    def _pad(x: torch.Tensor, fill=0.0):
        B = x.shape[0]
        Bp = max(32, (B + 31) // 32 * 32)
        if Bp == B:
            return x.contiguous(), B
        pad = torch.full((Bp - B,) + tuple(x.shape[1:]), fill, dtype=x.dtype, device=x.device)
        return torch.cat([x, pad]).contiguous(), B

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: [B, 16] float32 (device) -> [B, 16]."""
        L = lib()
        xp, B = self._pad(x.to(self.device, torch.float32))
        y = torch.empty_like(xp)
        net = self.c_struct()
        self._ws_call(lambda wss: L.pauli_mlp_forward(ctypes.byref(net), xp.data_ptr(),
                                                      xp.shape[0], y.data_ptr(),
                                                      ctypes.byref(wss), _stream_handle()),
                      "pauli_mlp_forward")
        return y[:B]

    def loss_grad(self, x, t, mask, want_acts=False):
        """Masked MSE and parameter gradients (into self.grads)."""
        L = lib()
        xp, B = self._pad(x.to(self.device, torch.float32))
        tp, _ = self._pad(t.to(self.device, torch.float32))
        mp, _ = self._pad(mask.to(self.device, torch.float32))
        Bp = xp.shape[0]
        acts = torch.empty(Bp * 2112, dtype=torch.float32, device=self.device) if want_acts else None
        loss = ctypes.c_double()
        net = self.c_struct()
        self._ws_call(lambda wss: L.pauli_mlp_loss_grad(
            ctypes.byref(net), xp.data_ptr(), tp.data_ptr(), mp.data_ptr(), Bp,
            ctypes.byref(loss), acts.data_ptr() if acts is not None else None,
            ctypes.byref(wss), _stream_handle()), "pauli_mlp_loss_grad")
        if want_acts:
            return loss.value, acts, Bp
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        net = self.c_struct()
        _check(lib().pauli_mlp_adam(ctypes.byref(net), lr, beta1, beta2, eps, self.t,
                                    _stream_handle()), "pauli_mlp_adam")

    @staticmethod
    def epoch_orders(n, epochs, seed=0):
        """The minibatch order of every epoch: seeded permutations of 0..n-1."""
        g = torch.Generator(device="cpu").manual_seed(seed)
        return torch.stack([torch.randperm(n, generator=g) for _ in range(epochs)])

    def train(self, x, t, mask, epochs=200, batch=512, lr=1e-3, seed=0, log_every=0,
              beta1=0.9, beta2=0.999, eps=1e-8):
        """Minibatch Adam with the fused step kernels (pauli_mlp_train: one
        library call for the whole run); returns the per-epoch mean training
        loss (minibatch losses weighted by their rows)."""
        L = lib()
        n = int(x.shape[0])
        xs = x.to(self.device, torch.float32).contiguous()
        ts = t.to(self.device, torch.float32).contiguous()
        ms = mask.to(self.device, torch.float32).contiguous()
        order = self.epoch_orders(n, epochs, seed).to(self.device, torch.int32).contiguous()
        spe = (n + batch - 1) // batch
        losses = torch.zeros(max(epochs * spe, 1), dtype=torch.float64, device=self.device)
        net = self.c_struct()
        self._ws_call(lambda wss: L.pauli_mlp_train(
            ctypes.byref(net), xs.data_ptr(), ts.data_ptr(), ms.data_ptr(), n, order.data_ptr(),
            epochs, batch, lr, beta1, beta2, eps, self.t, losses.data_ptr(), ctypes.byref(wss),
            _stream_handle()), "pauli_mlp_train")
        self.t += epochs * spe
        rows = np.array([min(batch, n - k * batch) for k in range(spe)], dtype=np.float64)
        lv = losses.cpu().numpy()[:epochs * spe].reshape(epochs, spe)
        hist = [float((lv[e] * rows).sum() / n) for e in range(epochs)]
        if log_every:
            for e in range(0, epochs, log_every):
                print(f"epoch {e} loss {hist[e]:.3e}", flush=True)
        return hist

    def train_layers(self, x, t, mask, epochs=200, batch=512, lr=1e-3, seed=0, log_every=0):
        """The same minibatch Adam sequenced from Python, one layer-by-layer
        loss/gradient call and one Adam call per minibatch (same epoch
        orders as `train`); returns the per-epoch mean training loss."""
        n = x.shape[0]
        orders = self.epoch_orders(n, epochs, seed)
        hist = []
        for ep in range(epochs):
            perm = orders[ep]
            tot, cnt = 0.0, 0
            for s in range(0, n, batch):
                idx = perm[s:s + batch].to(x.device)
                loss = self.loss_grad(x[idx], t[idx], mask[idx])
                self.adam(lr)
                tot += loss * len(idx)
                cnt += len(idx)
            hist.append(tot / cnt)
            if log_every and ep % log_every == 0:
                print(f"epoch {ep} loss {hist[-1]:.3e}", flush=True)
        return hist


def gemm_bf16(A: torch.Tensor, B: torch.Tensor, transA=False, transB=False) -> torch.Tensor:
    """C = op(A) op(B) on the matrix cores; A, B int16 tensors holding bf16."""
    L = lib()
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(L.pauli_gemm_bf16(A.data_ptr(), A.shape[1], int(transA), B.data_ptr(), B.shape[1],
                             int(transB), C.data_ptr(), N, M, N, K, _stream_handle()),
           "pauli_gemm_bf16")
    return C


# ---------------------------------------------------------------------------
# Windows, prediction, baselines
# ---------------------------------------------------------------------------

def make_windows(bseq: np.ndarray, n_avail: int):
    """Training windows from b_n tables [runs, >= n_avail]: input b_k..b_{k+15},
    target b_{k+16}..b_{k+31}, supervised only where the index is < n_avail;
    everything is divided by the input window's mean.

    The training runs should reach at least the depth the network is asked to
    predict (for continuing b_1..b_30 to b_46: runs of 46 steps), so that
    every output slot is trained on windows from the same stretch of the
    sequence it later extends."""
    xs, ts, ms = [], [], []
    for run in bseq:
        for k in range(0, n_avail - WIN):
            inp = run[k:k + WIN]
            s = inp.mean()
            tgt = np.zeros(OUT)
            msk = np.zeros(OUT)
            for j in range(OUT):
                if k + WIN + j < n_avail:
                    tgt[j] = run[k + WIN + j] / s
                    msk[j] = 1.0
            xs.append(inp / s)
            ts.append(tgt)
            ms.append(msk)
    f = lambda a: torch.tensor(np.array(a), dtype=torch.float32)
    return f(xs), f(ts), f(ms)


def predict_continuation(net: BnSurrogate, b_known: np.ndarray, n_known: int, n_total: int,
                         n_slots: int = OUT):
    """Extend b_1..b_{n_known} to n_total by repeated network passes, using the
    first n_slots output slots of each pass (one pass when n_total - n_known
    <= n_slots)."""
    seqs = [list(r[:n_known]) for r in b_known]
    while len(seqs[0]) < n_total:
        x = np.array([s[-WIN:] for s in seqs])
        sc = x.mean(axis=1, keepdims=True)
        y = net.forward(torch.tensor(x / sc, dtype=torch.float32, device=net.device))
        y = y.cpu().numpy().astype(np.float64) * sc
        take = min(n_slots, n_total - len(seqs[0]))
        for s, row in zip(seqs, y):
            s.extend(row[:take].tolist())
    return np.array([s[n_known:n_total] for s in seqs])


def baseline_constant(b_known: np.ndarray, n_known: int, n_total: int):
    return np.repeat(b_known[:, n_known - 1:n_known], n_total - n_known, axis=1)


def baseline_linear(b_known: np.ndarray, n_known: int, n_total: int):
    """Least-squares line through the last 16 coefficients, extrapolated."""
    n = np.arange(n_known - WIN + 1, n_known + 1)
    out = []
    for r in b_known:
        a, c = np.polyfit(n, r[n_known - WIN:n_known], 1)
        out.append(a * np.arange(n_known + 1, n_total + 1) + c)
    return np.array(out)
