"""Pins of the oracle's HEALPix beam-map interpolation and its resampling onto
the gnomonic grid (beamsor maps re-pixelated by interpolation, Sec. 4.2).

Interpolation: pixel centres give the pixel values; constants are exact;
along a ring it is linear in phi between neighbouring centres; a map that is
constant on every ring with value theta_i reproduces theta itself between the
first and last rings (the theta weighting is linear); above the first ring
the pole takes the mean of the first ring; a smooth beam converges as the
square of the pixel size.  Resampling: node (u, v) reads theta = rho =
atan(|(u, v)|), phi = sigma = atan2(v, u), checked on maps equal to the
antenna-frame direction cosines.
"""
import numpy as np

import oracle

D2R = np.pi / 180


def test_centres_constants_and_phi_linearity():
    rng = np.random.default_rng(1)
    for N in (1, 4, 16):
        npix = 12 * N * N
        m = rng.standard_normal(npix)
        th, ph = oracle.pix2ang(N, np.arange(npix))
        assert np.abs(oracle.healpix_interp(N, m, th, ph) - m).max() < 1e-13
        assert np.abs(oracle.healpix_interp(N, m, th, ph + 2 * np.pi) - m).max() < 1e-12
        c = np.full(npix, -1.25)
        th2, ph2 = np.arccos(rng.uniform(-1, 1, 500)), rng.uniform(-7, 7, 500)
        assert np.abs(oracle.healpix_interp(N, c, th2, ph2) + 1.25).max() < 1e-15
    # along ring i: values a + b j (no wrap between j and j + 1) -> midpoints give a + b (j + 1/2)
    N = 8
    npix = 12 * N * N
    for ring in (3, 8, 12, 20, 29):
        thr, cnt, first = oracle.ring(N, ring)
        m = np.zeros(npix)
        m[first:first + cnt] = 0.5 + 0.25 * np.arange(cnt)
        th, ph = oracle.pix2ang(N, np.arange(first, first + cnt))
        mid = 0.5 * (ph[:-1] + ph[1:])
        got = oracle.healpix_interp(N, m, np.full(mid.size, thr), mid)
        assert np.abs(got - (0.5 + 0.25 * (np.arange(cnt - 1) + 0.5))).max() < 1e-12


def test_theta_weighting_and_poles():
    N = 8
    npix = 12 * N * N
    rings = np.arange(1, 4 * N)
    thr = np.array([oracle.ring(N, int(i))[0] for i in rings])
    m = np.zeros(npix)
    for i, t in zip(rings, thr):
        _, cnt, first = oracle.ring(N, int(i))
        m[first:first + cnt] = t
    rng = np.random.default_rng(2)
    th = rng.uniform(thr[0], thr[-1], 2000)
    ph = rng.uniform(0, 2 * np.pi, th.size)
    assert np.abs(oracle.healpix_interp(N, m, th, ph) - th).max() < 1e-13
    # north pole: the mean of the first ring's four pixels, linear in theta down to ring 1
    m2 = rng.standard_normal(npix)
    pole = m2[:4].mean()
    assert abs(oracle.healpix_interp(N, m2, 0.0, 1.3)[()] - pole) < 1e-14
    t = 0.4 * thr[0]
    on_ring = oracle.healpix_interp(N, m2, thr[0], 2.0)[()]
    assert abs(oracle.healpix_interp(N, m2, t, 2.0)[()] - (0.6 * pole + 0.4 * on_ring)) < 1e-14
    # south pole likewise
    south = m2[-4:].mean()
    assert abs(oracle.healpix_interp(N, m2, np.pi, 0.2)[()] - south) < 1e-14


def test_smooth_beam_converges_quadratically():
    """A circular Gaussian (FWHM 1.5 deg) sampled at pixel centres: the error
    of the interpolated beam within 2 deg of the pole drops about 4x per nside
    doubling."""
    sig = 1.5 * D2R / np.sqrt(8 * np.log(2))
    rng = np.random.default_rng(3)
    th = np.sqrt(rng.uniform(0, (2 * D2R) ** 2, 3000))
    ph = rng.uniform(0, 2 * np.pi, th.size)
    errs = []
    for N in (128, 256, 512):
        npix = 12 * N * N
        # only the polar cap matters; fill the map from the closed form at the centres
        pix = np.arange(2 * (4 * N // 3) * (4 * N // 3 - 1))
        tc, _ = oracle.pix2ang(N, pix)
        m = np.zeros(npix)
        m[pix] = np.exp(-0.5 * (tc / sig) ** 2)
        got = oracle.healpix_interp(N, m, th, ph)
        errs.append(np.abs(got - np.exp(-0.5 * (th / sig) ** 2)).max())
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3, errs
    assert errs[2] < 1.5e-2   # h^2 |f"| / 8 ~ (0.115 / 0.64)^2 / 8 = 4e-3 at nside 512, more at the pole


def test_grid_orientation():
    """Maps equal to sin(theta) cos(phi) and sin(theta) sin(phi) (the antenna
    frame's x' and y' direction cosines) resample to u / sqrt(1 + u^2 + v^2)
    and v / sqrt(1 + u^2 + v^2) at the nodes, to the interpolation error."""
    N = 256
    npix = 12 * N * N
    pix = np.arange(2 * 40 * 39)
    th, ph = oracle.pix2ang(N, pix)
    mx, my = np.zeros(npix), np.zeros(npix)
    mx[pix] = np.sin(th) * np.cos(ph)
    my[pix] = np.sin(th) * np.sin(ph)
    T, n = np.tan(3 * D2R), 31
    ax = -T + np.arange(n) * (2 * T / (n - 1))
    v, u = np.meshgrid(ax, ax, indexing="ij")
    r = np.sqrt(1 + u * u + v * v)
    gx, gy = oracle.healpix_to_grid(N, mx, T, n), oracle.healpix_to_grid(N, my, T, n)
    # near the pole ring i has 4i pixels: linear-in-phi error ~ theta_1 (pi/2)^2 / 8 ~ 8e-4 on ring 1
    assert np.abs(gx - u / r).max() < 2e-3 and np.abs(gy - v / r).max() < 2e-3
    far = np.hypot(u, v) > 2 * D2R   # the phi error falls as 1 / theta away from the pole
    assert np.abs(gx - u / r)[far].max() < 1e-4 and np.abs(gy - v / r)[far].max() < 1e-4
    assert gx[n // 2, -1] > 0 > gx[n // 2, 0] and gy[-1, n // 2] > 0 > gy[0, n // 2]
