"""Beam fixtures: Mueller-matrix beam fields ("beamsors") on tangent-plane grids.

A grid of n x n nodes (n odd, so the beam centre is a node) spans
u, v in [-T, T] with T = tan(half_span); node (iu, iv) sits at
u = -T + iu h, v = -T + iv h, h = 2T / (n - 1), stored row-major [iv][iu].
A node's angular offset from the boresight is rho = atan(sqrt(u^2 + v^2))
and its azimuth sigma = atan2(v, u) (gnomonic projection of the antenna
frame).

A beamsor is a field of 4x4 Mueller matrices M[out][in] over (T, Q, U, V);
the paper's element B_XY (input X, output Y) sits at M[Y][X].  Only
non-zero elements are stored.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

STOKES = {"T": 0, "Q": 1, "U": 2, "V": 3}
FWHM_TO_SIGMA = 1.0 / np.sqrt(8.0 * np.log(2.0))


def tangent_grid(n: int, half_span_rad: float):
    """Node coordinates: returns (T, u[iv, iu], v[iv, iu], rho, sigma)."""
    if n < 3 or n % 2 == 0:
        raise ValueError("grid size must be odd and >= 3")
    T = float(np.tan(half_span_rad))
    ax = -T + np.arange(n) * (2.0 * T / (n - 1))
    v, u = np.meshgrid(ax, ax, indexing="ij")
    rho = np.arctan(np.hypot(u, v))
    sig = np.arctan2(v, u)
    return T, u, v, rho, sig


def elliptical_gaussian(rho, sig, fwhm_rad: float, ellipticity: float = 0.0, orient_rad: float = 0.0):
    """Peak-normalised elliptical Gaussian.

    sigma_maj * sigma_min = sigma^2 (sigma from the FWHM) and
    e = (sigma_maj - sigma_min) / (sigma_maj + sigma_min); the major axis
    lies at ``orient_rad`` from the u axis.
    """
    s0 = fwhm_rad * FWHM_TO_SIGMA
    r = np.sqrt((1.0 + ellipticity) / (1.0 - ellipticity))
    smaj, smin = s0 * r, s0 / r
    x = rho * np.cos(sig - orient_rad)
    y = rho * np.sin(sig - orient_rad)
    return np.exp(-0.5 * ((x / smaj) ** 2 + (y / smin) ** 2))


def ring_lobe(rho, radius_rad: float, fwhm_rad: float, amp: float):
    """Axisymmetric ring: amp * exp(-(rho - R)^2 / (2 w^2)), w from the ring FWHM."""
    w = fwhm_rad * FWHM_TO_SIGMA
    return amp * np.exp(-0.5 * ((rho - radius_rad) / w) ** 2)


@dataclass
class Beamsor:
    n: int
    half_span_tan: float
    elements: dict = field(default_factory=dict)  # (out, in) -> (n, n) float64

    def get(self, out: int, inp: int) -> np.ndarray:
        e = self.elements.get((out, inp))
        return np.zeros((self.n, self.n)) if e is None else e

    def dense(self) -> np.ndarray:
        """(n, n, 4, 4) float64 array M[iv, iu, out, in]."""
        d = np.zeros((self.n, self.n, 4, 4))
        for (o, i), g in self.elements.items():
            d[:, :, o, i] = g
        return d


def ideal_beamsor(b: np.ndarray, half_span_tan: float) -> Beamsor:
    """b (x) identity: co-polar response b on every Stokes parameter."""
    n = b.shape[0]
    return Beamsor(n, half_span_tan, {(k, k): b.copy() for k in range(4)})


def with_qu_leakage(bs: Beamsor, b: np.ndarray, frac: float) -> Beamsor:
    """Add symmetric Q<->U leakage of ``frac`` times b (B_QU and B_UQ)."""
    el = dict(bs.elements)
    el[(STOKES["U"], STOKES["Q"])] = frac * b
    el[(STOKES["Q"], STOKES["U"])] = frac * b
    return Beamsor(bs.n, bs.half_span_tan, el)


def delta_beamsor(n: int, half_span_tan: float) -> Beamsor:
    """Only the centre node is non-zero (= 1) on the diagonal."""
    b = np.zeros((n, n))
    b[n // 2, n // 2] = 1.0
    return ideal_beamsor(b, half_span_tan)


@dataclass
class DetectorParams:
    zeta: float = 0.0      # polarisation angle w.r.t. theta'_0 (rad)
    eps: float = 0.0       # 1 - eps = polarisation efficiency
    s: float = 1.0         # responsivity


def healpix_beam_map(nside: int, fwhm_rad: float, ellipticity: float = 0.0, orient_rad: float = 0.0,
                     rho_max_rad: float | None = None) -> np.ndarray:
    """Elliptical Gaussian (peak 1) sampled at the pixel centres of a RING map
    whose north pole is the boresight: theta = rho, phi = sigma.  Zero beyond
    rho_max when given (only the cap needs computing)."""
    from .rings import pixel_centres

    th, ph = pixel_centres(nside)
    out = np.zeros(th.size)
    keep = np.ones(th.size, dtype=bool) if rho_max_rad is None else th <= rho_max_rad
    out[keep] = elliptical_gaussian(th[keep], ph[keep], fwhm_rad, ellipticity, orient_rad)
    return out
