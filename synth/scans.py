"""Pointing-stream fixtures (theta = colatitude, phi = longitude, psi; radians).

These only generate inputs: the convolution takes pointing as given.
"""
from __future__ import annotations

import numpy as np

from .rings import pixel_centres

SIDEREAL_DAY_S = 86164.0905


def radec_sweep(n: int, rng: np.random.Generator, dec_max_deg: float = 60.0):
    """RA sweeps linearly over 360 deg across the stream; Dec ~ U[-dmax, dmax]; psi ~ U[0, 2pi)."""
    phi = 2.0 * np.pi * np.arange(n) / n
    dec = np.deg2rad(rng.uniform(-dec_max_deg, dec_max_deg, n))
    psi = rng.uniform(0.0, 2.0 * np.pi, n)
    return 0.5 * np.pi - dec, phi, psi


def uniform_sphere(n: int, rng: np.random.Generator):
    """Isotropic directions with uniform psi."""
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    psi = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.arccos(z), phi, psi


def ces(n: int, lat_rad: float, el_deg: float = 45.0, az_step_deg: float = 0.01,
        sweep_deg: float = 720.0, rate_hz: float = 100.0, start: int = 0,
        boresight_deg=None, boresight_period: int = 100_000, lst0: float = 0.0):
    """Constant-elevation scan: azimuth in triangle sweeps of ``sweep_deg``.

    Azimuth advances ``az_step_deg`` per sample, local sidereal time at the
    sidereal rate for ``rate_hz`` sampling.  psi = parallactic angle +
    boresight angle; the boresight angle cycles through ``boresight_deg``
    every ``boresight_period`` samples (None: 0).
    """
    t = np.arange(start, start + n, dtype=np.float64)
    half = sweep_deg / az_step_deg
    ph = np.mod(t, 2.0 * half)
    az = np.deg2rad(np.where(ph < half, ph, 2.0 * half - ph) * az_step_deg)
    el = np.deg2rad(el_deg)
    lst = lst0 + 2.0 * np.pi * (t / rate_hz) / SIDEREAL_DAY_S
    sl, cl = np.sin(lat_rad), np.cos(lat_rad)
    se, ce = np.sin(el), np.cos(el)
    sin_dec = se * sl + ce * cl * np.cos(az)
    dec = np.arcsin(np.clip(sin_dec, -1.0, 1.0))
    ha = np.arctan2(-np.sin(az) * ce, se * cl - ce * sl * np.cos(az))
    ra = np.mod(lst - ha, 2.0 * np.pi)
    q = np.arctan2(np.sin(ha), np.tan(lat_rad) * np.cos(dec) - np.sin(dec) * np.cos(ha))
    bs = np.zeros(n)
    if boresight_deg is not None:
        steps = np.asarray(boresight_deg, dtype=np.float64)
        bs = np.deg2rad(steps[(t.astype(np.int64) // boresight_period) % len(steps)])
    return 0.5 * np.pi - dec, ra, np.mod(q + bs, 2.0 * np.pi)


def _basis(theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    p = np.stack([st * cp, st * sp, ct], -1)
    th = np.stack([ct * cp, ct * sp, -st], -1)
    ph = np.stack([-sp, cp, np.zeros_like(theta)], -1)
    return p, th, ph


def offset_pointing(theta, phi, psi, dx: float, dy: float):
    """Pointing of a detector offset by (dx, dy) radians in the boresight focal plane.

    The offset is taken along the boresight's rotated basis (dx along
    theta', dy along phi'); the detector's own psi is the boresight frame
    carried to the detector direction along the connecting great circle.
    """
    p, th, ph = _basis(theta, phi)
    c, s = np.cos(psi)[:, None], np.sin(psi)[:, None]
    thp = c * th + s * ph
    php = -s * th + c * ph
    r = np.hypot(dx, dy)
    if r == 0.0:
        return theta.copy(), phi.copy(), psi.copy()
    a = np.arctan2(dy, dx)
    d = np.cos(r) * p + np.sin(r) * (np.cos(a) * thp + np.sin(a) * php)
    # carry thp from p to d by the minimal rotation (axis p x d)
    axis = np.cross(p, d)
    cz = np.sum(p * d, -1, keepdims=True)
    t = thp + np.cross(axis, thp) + np.cross(axis, np.cross(axis, thp)) / (1.0 + cz)
    th_d = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    ph_d = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2.0 * np.pi)
    _, thd, phd = _basis(th_d, ph_d)
    psi_d = np.arctan2(np.sum(t * phd, -1), np.sum(t * thd, -1))
    return th_d, ph_d, np.mod(psi_d, 2.0 * np.pi)


def hex_focal_plane(n_sites: int, pitch_rad: float):
    """First ``n_sites`` points of a hexagonal lattice, nearest the centre first."""
    pts = []
    R = int(np.ceil(np.sqrt(n_sites))) + 2
    for i in range(-R, R + 1):
        for j in range(-R, R + 1):
            x = (i + 0.5 * j) * pitch_rad
            y = j * np.sqrt(3.0) / 2.0 * pitch_rad
            pts.append((np.hypot(x, y), x, y))
    pts.sort()
    return np.array([(x, y) for _, x, y in pts[:n_sites]])


def pixel_centre_scan(nside: int, psis_deg=(0.0, 45.0, 90.0)):
    """Every pixel centre visited once per psi (the paper's benchmark pattern)."""
    th, ph = pixel_centres(nside)
    k = len(psis_deg)
    theta = np.tile(th, k)
    phi = np.tile(ph, k)
    psi = np.repeat(np.deg2rad(np.asarray(psis_deg, dtype=np.float64)), th.size)
    return theta, phi, psi
