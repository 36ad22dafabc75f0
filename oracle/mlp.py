"""FP64 oracle of the learned coefficient surrogate (TEST INFRASTRUCTURE
ONLY: used by tests, never by the product).

The network: din -> hidden -> hidden -> hidden -> dout, tanh hidden layers,
linear output, mean-squared-error loss.  Forward and backward are the
textbook chain rule written out in FP64 with numpy matrix products as the
only library primitive.  With ``bf16=True`` the values the GPU stores in
BF16 (weights, hidden activations, the loss gradient and the back-propagated
pre-activation gradients) are rounded to BF16 at the same points, so the GPU
(FP32 accumulation) can be compared with it operand for operand.
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Values are first rounded to float32, as on the GPU."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(p: np.ndarray, din: int, hidden: int, dout: int) -> dict:
    shapes = [("W1", (din, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
              ("W3", (hidden, hidden)), ("b3", (hidden,)), ("W4", (hidden, dout)), ("b4", (dout,))]
    out, o = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([d[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")])


def forward(p: np.ndarray, X: np.ndarray, din: int, hidden: int, dout: int, bf16_round: bool = True):
    """Returns (Y, [H1, H2, H3])."""
    P = unpack(p, din, hidden, dout)
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    W = {k: (r(P[k]) if k.startswith("W") else P[k]) for k in P}
    X = np.asarray(X, dtype=np.float64)
    H1 = r(np.tanh(X @ W["W1"] + W["b1"]))
    H2 = r(np.tanh(H1 @ W["W2"] + W["b2"]))
    H3 = r(np.tanh(H2 @ W["W3"] + W["b3"]))
    Y = H3 @ W["W4"] + W["b4"]
    return Y, [H1, H2, H3]


def loss_and_grad_out(Y: np.ndarray, T: np.ndarray, bf16_round: bool = True):
    D = Y - np.asarray(T, dtype=np.float64)
    n = D.size
    dY = 2.0 * D / n
    return float(np.mean(D * D)), (bf16(dY) if bf16_round else dY)


def backward(p: np.ndarray, X: np.ndarray, Hs, dY: np.ndarray, din: int, hidden: int, dout: int,
             bf16_round: bool = True) -> np.ndarray:
    """Gradient of the loss w.r.t. every parameter (flat, same layout)."""
    P = unpack(p, din, hidden, dout)
    r = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    W = {k: r(P[k]) for k in ("W1", "W2", "W3", "W4")}
    X = np.asarray(X, dtype=np.float64)
    H1, H2, H3 = Hs
    g = {}
    g["W4"] = H3.T @ dY
    g["b4"] = dY.sum(axis=0)
    dZ3 = r((dY @ W["W4"].T) * (1.0 - H3 * H3))
    g["W3"] = H2.T @ dZ3
    g["b3"] = dZ3.sum(axis=0)
    dZ2 = r((dZ3 @ W["W3"].T) * (1.0 - H2 * H2))
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = r((dZ2 @ W["W2"].T) * (1.0 - H1 * H1))
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def loss(p, X, T, din, hidden, dout, bf16_round=False) -> float:
    Y, _ = forward(p, X, din, hidden, dout, bf16_round)
    return float(np.mean((Y - T) ** 2))


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Kingma & Ba's Adam with bias correction; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
