"""Host-side preparation of a detector's beam for the convolution kernels.

The kernels take the detector row already folded into the beamsor
(Sec. 4.1: D(chi) Lambda(chi) = D(0), so D(0) B is constant over the sky).
With the Mueller field stored as M[..., out, in] over (T, Q, U, V) -- the
paper's element B_XY (input X, output Y) at M[Y, X] -- and
D(0) = (s/2) [1 + eps, 1 - eps, 0, 0]:

    bI = (s/2)[(1+eps) M[T,T] + (1-eps) M[Q,T]]
    bQ = (s/2)[(1+eps) M[T,Q] + (1-eps) M[Q,Q]]
    bU = (s/2)[(1+eps) M[T,U] + (1-eps) M[Q,U]]
    bT = M[T,T]                        (the normalising scalar beam, Sec. 3)
    bV = (s/2)[(1+eps) M[T,V] + (1-eps) M[Q,V]]   (the V column; zero for most beams)
"""
from __future__ import annotations

import numpy as np


def fold_detector(M: np.ndarray, eps: float, s: float):
    """M: (n, n, 4, 4) Mueller field -> (bI, bQ, bU, bT), each (n, n) float64."""
    M = np.asarray(M, dtype=np.float64)
    if M.ndim != 4 or M.shape[2:] != (4, 4) or M.shape[0] != M.shape[1]:
        raise ValueError("Mueller field must be (n, n, 4, 4)")
    a, b = 0.5 * s * (1.0 + eps), 0.5 * s * (1.0 - eps)
    bI = a * M[:, :, 0, 0] + b * M[:, :, 1, 0]
    bQ = a * M[:, :, 0, 1] + b * M[:, :, 1, 1]
    bU = a * M[:, :, 0, 2] + b * M[:, :, 1, 2]
    return bI, bQ, bU, M[:, :, 0, 0].copy()


def fold_detector_maps(M: np.ndarray, eps: float, s: float):
    """M: (npix, 4, 4) Mueller maps (HEALPix) -> (bI, bQ, bU, bT, bV), each (npix,) float64."""
    M = np.asarray(M, dtype=np.float64)
    if M.ndim != 3 or M.shape[1:] != (4, 4):
        raise ValueError("Mueller maps must be (npix, 4, 4)")
    a, b = 0.5 * s * (1.0 + eps), 0.5 * s * (1.0 - eps)
    return tuple(a * M[:, 0, k] + b * M[:, 1, k] for k in range(3)) + (M[:, 0, 0].copy(), a * M[:, 0, 3] + b * M[:, 1, 3])


def fold_v(M: np.ndarray, eps: float, s: float):
    """The V-column channel bV of a (n, n, 4, 4) Mueller field, or None when it is zero."""
    M = np.asarray(M, dtype=np.float64)
    a, b = 0.5 * s * (1.0 + eps), 0.5 * s * (1.0 - eps)
    bV = a * M[:, :, 0, 3] + b * M[:, :, 1, 3]
    return None if not np.any(bV) else bV


def fold_elements(elements: dict, n: int, eps: float, s: float):
    """Same as fold_detector for a sparse {(out, in): (n, n)} Mueller field."""
    z = np.zeros((n, n))
    g = lambda o, i: np.asarray(elements.get((o, i), z), dtype=np.float64)  # noqa: E731
    a, b = 0.5 * s * (1.0 + eps), 0.5 * s * (1.0 - eps)
    return (a * g(0, 0) + b * g(1, 0), a * g(0, 1) + b * g(1, 1), a * g(0, 2) + b * g(1, 2), g(0, 0).copy())


def grid_solid_angle(bT: np.ndarray, half_span_tan: float, rho_max: float | None = None) -> float:
    """Omega~ = integral of B_TT over the sphere, by the node rule on the tangent
    grid with the gnomonic Jacobian (1 + u^2 + v^2)^(-3/2); optionally only
    nodes within rho_max of the centre."""
    n = bT.shape[0]
    T = float(half_span_tan)
    ax = -T + np.arange(n) * (2.0 * T / (n - 1))
    v, u = np.meshgrid(ax, ax, indexing="ij")
    r2 = u * u + v * v
    w = (1.0 + r2) ** -1.5
    if rho_max is not None:
        w = w * (np.arctan(np.sqrt(r2)) <= rho_max)
    h = 2.0 * T / (n - 1)
    return float(np.sum(bT * w) * h * h)


def scalar_weights(bI, bQ, bU, bT, rtol: float = 1e-12):
    """(wI, wQ, wU) if every channel is a constant multiple of bT, else None."""
    bT = np.asarray(bT, dtype=np.float64)
    k = np.unravel_index(np.argmax(np.abs(bT)), bT.shape)
    if bT[k] == 0.0:
        return None
    scale = np.abs(bT).max()
    out = []
    for b in (bI, bQ, bU):
        b = np.asarray(b, dtype=np.float64)
        w = b[k] / bT[k]
        if np.abs(b - w * bT).max() > rtol * max(scale * abs(w), scale):
            return None
        out.append(float(w))
    return tuple(out)
