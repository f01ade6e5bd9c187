"""Binned map-making from TOD: test infrastructure, like the rest of `oracle/`.

The paper hands the TOD to a map-making code (Sec. 5.1) and validates with maps
made from them (Sec. 6); it does not spell the estimator out.  This is the
standard binned estimator for a polarisation-sensitive detector seen through an
ideal beam at its boresight: the sample t of a detector with response s and
cross-polar leakage eps, at position angle chi_t = psi_t + zeta (plus 2 phi_t
behind an ideal half-wave plate at phi_t), measures

    d_t = w_t . (I, Q, U)_p,   w_t = (s/2) ((1 + eps), (1 - eps) cos 2chi_t, (1 - eps) sin 2chi_t)

(the one-pixel form of the detector row D of Sec. 4.1 with Lambda(chi)), p
being the RING pixel that holds the boresight.  Per pixel the maps solve
(sum_t w_t w_t^T) m = sum_t w_t d_t.  rcond = smallest / largest eigenvalue of
that 3 x 3 matrix; pixels below `rcond_min` get the intensity-only solution
I = sum w_0 d / sum w_0^2 with Q = U = 0; unobserved pixels are zero.

Plain numpy: np.add.at for the sums, numpy.linalg for the solves.
"""
from __future__ import annotations

import numpy as np

from . import ang2pix


def weights(psi, zeta: float, eps: float, s: float, hwp=None) -> np.ndarray:
    """(n, 3) pointing weights w_t."""
    a = 2.0 * (np.asarray(psi, dtype=np.float64) + zeta)
    if hwp is not None:
        a = a + 4.0 * np.asarray(hwp, dtype=np.float64)
    return 0.5 * s * np.stack([np.full(a.shape, 1.0 + eps), (1.0 - eps) * np.cos(a), (1.0 - eps) * np.sin(a)], 1)


def bin_tod(nside: int, theta, phi, psi, tod, zeta: float, eps: float, s: float, hwp=None):
    """Per-pixel sums of one detector's samples: (ata (npix, 3, 3), atd (npix, 3), hits (npix,))."""
    npix = 12 * nside * nside
    pix = ang2pix(nside, theta, phi)
    w = weights(psi, zeta, eps, s, hwp)
    d = np.asarray(tod, dtype=np.float64)
    ata = np.zeros((npix, 3, 3))
    atd = np.zeros((npix, 3))
    hits = np.zeros(npix)
    np.add.at(ata, pix, w[:, :, None] * w[:, None, :])
    np.add.at(atd, pix, w * d[:, None])
    np.add.at(hits, pix, 1.0)
    return ata, atd, hits


def solve(ata, atd, hits, rcond_min: float = 1e-6):
    """(I, Q, U, rcond) maps from the per-pixel sums."""
    npix = hits.size
    I, Q, U, rc = (np.zeros(npix) for _ in range(4))
    seen = hits > 0
    ev = np.linalg.eigvalsh(ata[seen])
    rc[seen] = np.where(ev[:, 2] > 0, ev[:, 0] / np.where(ev[:, 2] > 0, ev[:, 2], 1.0), 0.0)
    full = seen & (rc >= rcond_min)
    if full.any():
        m = np.linalg.solve(ata[full], atd[full][:, :, None])[:, :, 0]
        I[full], Q[full], U[full] = m[:, 0], m[:, 1], m[:, 2]
    part = seen & ~full
    I[part] = atd[part, 0] / ata[part, 0, 0]
    return I, Q, U, rc
