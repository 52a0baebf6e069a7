"""Float64 NumPy reference of the b_n continuation network (test infrastructure).

16 -> 256 -> 256 -> 16 with GELU(x) = x (1 + erf(x / sqrt 2)) / 2 on the
hidden layers, masked mean-squared error, analytic backward pass and Adam.
Parameters use the flat layout W1[256][16], b1[256], W2[256][256], b2[256],
W3[16][256], b3[16].  `bf16` rounds float32 values to bfloat16 (round to
nearest even), the operand precision of the GPU's matrix products.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

WIN, HID, OUT = 16, 256, 16
SHAPES = [("W1", (HID, WIN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (OUT, HID)), ("b3", (OUT,))]


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (nearest even) via float32, returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(p, x):
    w = unpack(p)
    z1 = x @ w["W1"].T + w["b1"]
    y1 = gelu(z1)
    z2 = y1 @ w["W2"].T + w["b2"]
    y2 = gelu(z2)
    y = y2 @ w["W3"].T + w["b3"]
    return {"z1": z1, "y1": y1, "z2": z2, "y2": y2, "y": y}


def loss_and_grad(p, x, t, mask):
    """Masked MSE sum(mask (y - t)^2) / sum(mask) and its gradient (flat)."""
    w = unpack(p)
    f = forward(p, x)
    cnt = mask.sum()
    loss = float((mask * (f["y"] - t) ** 2).sum() / cnt)
    dy = 2.0 * mask * (f["y"] - t) / cnt
    g = {"W3": dy.T @ f["y2"], "b3": dy.sum(0)}
    dz2 = (dy @ w["W3"]) * gelu_grad(f["z2"])
    g["W2"] = dz2.T @ f["y1"]
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ w["W2"]) * gelu_grad(f["z1"])
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
