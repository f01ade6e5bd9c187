"""HEALPix RING-scheme ring table for the input generators.

The generators need pixel-centre positions to synthesise maps and to aim
pointings at pixel centres.  They carry this small table of their own so
that the input module shares no code with either the oracle or the GPU
library.  Geometry follows Gorski et al. 2005 (ApJ 622, 759): 12 N^2
equal-area pixels on 4N-1 iso-latitude rings; polar-cap ring i (< N) holds
4i pixels at z = 1 - i^2/(3N^2); equatorial ring i (N..3N) holds 4N pixels
at z = 4/3 - 2i/(3N), its first pixel half a step from phi = 0 on rings
with odd (i - N) offset parity; the southern cap mirrors the northern one.
"""
from __future__ import annotations

import numpy as np


def ring_table(nside: int):
    """Return per-ring arrays for rings 1..4N-1 (north to south).

    z, sin_theta : cos and sin of the ring colatitude (sin computed from
                   1 - z and 1 + z separately so polar rings keep precision)
    npix         : pixels on the ring
    first        : RING index of the ring's first pixel
    phi0         : longitude of the first pixel (later pixels step by 2 pi / npix)
    """
    N = int(nside)
    i = np.arange(1, 4 * N, dtype=np.int64)
    npix_tot = 12 * N * N
    north = i < N
    south = i > 3 * N
    i_s = 4 * N - i
    one_minus_z = np.empty(i.shape, dtype=np.float64)
    one_plus_z = np.empty(i.shape, dtype=np.float64)
    z = np.empty(i.shape, dtype=np.float64)
    eq = ~(north | south)
    # polar caps: 1 -+ z = i^2 / (3 N^2)
    one_minus_z[north] = i[north].astype(np.float64) ** 2 / (3.0 * N * N)
    z[north] = 1.0 - one_minus_z[north]
    one_plus_z[north] = 1.0 + z[north]
    one_plus_z[south] = i_s[south].astype(np.float64) ** 2 / (3.0 * N * N)
    z[south] = one_plus_z[south] - 1.0
    one_minus_z[south] = 1.0 - z[south]
    z[eq] = 4.0 / 3.0 - 2.0 * i[eq].astype(np.float64) / (3.0 * N)
    one_minus_z[eq] = 1.0 - z[eq]
    one_plus_z[eq] = 1.0 + z[eq]
    sin_theta = np.sqrt(one_minus_z * one_plus_z)

    npix = np.where(north, 4 * i, np.where(south, 4 * i_s, 4 * N))
    first = np.empty(i.shape, dtype=np.int64)
    first[north] = 2 * i[north] * (i[north] - 1)
    first[eq] = 2 * N * (N - 1) + (i[eq] - N) * 4 * N
    first[south] = npix_tot - 2 * i_s[south] * (i_s[south] + 1)

    phi0 = np.empty(i.shape, dtype=np.float64)
    phi0[north] = np.pi / (4.0 * i[north])
    phi0[south] = np.pi / (4.0 * i_s[south])
    shifted = ((i[eq] - N + 1) % 2) == 1
    phi0[eq] = np.where(shifted, np.pi / (4.0 * N), 0.0)
    return z, sin_theta, npix, first, phi0


def pixel_centres(nside: int):
    """(theta, phi) of every pixel in RING order, float64."""
    z, st, npix, first, phi0 = ring_table(nside)
    n_tot = 12 * nside * nside
    theta = np.empty(n_tot)
    phi = np.empty(n_tot)
    ring_theta = np.arctan2(st, z)
    for r in range(len(z)):
        n = int(npix[r])
        sl = slice(int(first[r]), int(first[r]) + n)
        theta[sl] = ring_theta[r]
        phi[sl] = phi0[r] + 2.0 * np.pi * np.arange(n) / n
    return theta, phi
