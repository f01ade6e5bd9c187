"""FP64 reference of the far-sidelobe network (test infrastructure only).

Network: x (5) -> [Linear, SiLU] x hidden -> Linear -> y (3).  Parameters are
one flat array: for each linear map l, W_l (rows = outputs, row-major) then
b_l.  The products use the BF16-rounded weights (the GPU's storage format);
everything else is float64.  Loss: mean of the squared errors over all n x 3
outputs.  Adam: bias-corrected, eps added to sqrt(v_hat).

Pins (tests/test_oracle_mlp.py): central finite differences of the loss
against the analytic gradient, the SiLU derivative, Adam's first step from
zero moments, and the bf16 rounding rule on exact cases.
"""
from __future__ import annotations

import numpy as np

N_IN, N_OUT = 5, 3


def bf16_round(a) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def dims(width: int, hidden: int):
    return [N_IN] + [width] * hidden + [N_OUT]


def layout(width: int, hidden: int):
    """[(w_offset, rows, cols, b_offset)] per linear map."""
    d = dims(width, hidden)
    out, o = [], 0
    for l in range(hidden + 1):
        rows, cols = d[l + 1], d[l]
        out.append((o, rows, cols, o + rows * cols))
        o += rows * cols + rows
    return out, o


def unpack(params, width: int, hidden: int, round_weights: bool = True):
    lay, total = layout(width, hidden)
    p = np.asarray(params, dtype=np.float64)
    assert p.size == total
    Ws, bs = [], []
    for wo, r, c, bo in lay:
        W = p[wo:wo + r * c].reshape(r, c)
        Ws.append(bf16_round(W) if round_weights else W)
        bs.append(p[bo:bo + r])
    return Ws, bs


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, width: int, hidden: int, round_weights: bool = True):
    Ws, bs = unpack(params, width, hidden, round_weights)
    a = np.asarray(x, dtype=np.float64)
    zs, acts = [], [a]
    for l in range(hidden):
        z = a @ Ws[l].T + bs[l]
        a = silu(z)
        zs.append(z)
        acts.append(a)
    y = a @ Ws[hidden].T + bs[hidden]
    return y, (zs, acts, Ws)


def loss_and_grad(params, x, t, width: int, hidden: int, round_weights: bool = True):
    """MSE loss and its gradient with respect to the (unrounded) parameters,
    treating the bf16 rounding of the weights as the identity (straight through)."""
    y, (zs, acts, Ws) = forward(params, x, width, hidden, round_weights)
    n = y.shape[0]
    e = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(e * e))
    lay, total = layout(width, hidden)
    g = np.zeros(total)
    dz = 2.0 * e / e.size
    for l in range(hidden, -1, -1):
        wo, r, c, bo = lay[l]
        g[wo:wo + r * c] = (dz.T @ acts[l]).ravel()
        g[bo:bo + r] = dz.sum(0)
        if l > 0:
            dz = (dz @ Ws[l]) * silu_grad(zs[l - 1])
    del n
    return loss, g


def adam_step(params, m, v, grad, step: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
