"""Pins of the oracle's HEALPix ang2pix and binned map-maker.

ang2pix (Gorski et al. 2005, Sec. 4): every pixel centre maps to its own
pixel; small offsets from a centre stay in the pixel; HEALPix pixels have
equal areas, so uniform directions fill them evenly (chi-square).
Map-maker: the closed-form inversion of three samples at psi = 0, 45, 90 deg
(the paper's scanning pattern of Sec. 6); exact recovery of any I, Q, U from
model-consistent samples at random angles; a plate at phi equals a position
angle rotated by 2 phi; one angle per pixel falls back to intensity only; and
end to end through the convolution oracle, an unpolarised sky seen through a
circular ideal beam at pixel centres gives Q = U = 0 (no temperature to
polarisation leakage, Sec. 6).
"""
import numpy as np

import oracle
from oracle import maps as M
from synth import beams as B
from synth import sky as SK

D2R = np.pi / 180


def test_ang2pix_centres_round_trip():
    for nside in (1, 2, 4, 8, 16, 64):
        pix = np.arange(12 * nside * nside)
        th, ph = oracle.pix2ang(nside, pix)
        assert np.array_equal(oracle.ang2pix(nside, th, ph), pix)
        # the same directions with phi shifted by whole turns
        assert np.array_equal(oracle.ang2pix(nside, th, ph - 2 * np.pi), pix)
        assert np.array_equal(oracle.ang2pix(nside, th, ph + 4 * np.pi), pix)


def test_ang2pix_small_offsets_stay_in_the_pixel():
    rng = np.random.default_rng(1)
    for nside in (1, 4, 32, 256):
        npix = 12 * nside * nside
        pix = rng.integers(0, npix, 4000)
        th, ph = oracle.pix2ang(nside, pix)
        scale = np.sqrt(4 * np.pi / npix)
        r = 0.1 * scale * np.sqrt(rng.uniform(0, 1, pix.size))
        a = rng.uniform(0, 2 * np.pi, pix.size)
        # offset along the local (theta, phi) axes, exact on the sphere via vectors
        p = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
        et = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], 1)
        ef = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], 1)
        q = (np.cos(r)[:, None] * p + np.sin(r)[:, None] * (np.cos(a)[:, None] * et + np.sin(a)[:, None] * ef))
        th2, ph2 = np.arccos(np.clip(q[:, 2], -1, 1)), np.arctan2(q[:, 1], q[:, 0])
        assert np.array_equal(oracle.ang2pix(nside, th2, ph2), pix), nside


def test_ang2pix_equal_areas():
    rng = np.random.default_rng(2)
    nside, n = 4, 2_000_000
    th, ph = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n)
    counts = np.bincount(oracle.ang2pix(nside, th, ph), minlength=192)
    e = n / 192
    chi2 = ((counts - e) ** 2 / e).sum()
    assert chi2 < 191 + 6 * np.sqrt(2 * 191), chi2       # 191 degrees of freedom


def _centres_three_angles(nside):
    npix = 12 * nside * nside
    th, ph = oracle.pix2ang(nside, np.arange(npix))
    psi = np.repeat(np.deg2rad([0.0, 45.0, 90.0]), npix)
    return np.tile(th, 3), np.tile(ph, 3), psi


def test_three_angle_closed_form():
    """eps = 0, s = 1: d0 = (I + Q)/2, d45 = (I + U)/2, d90 = (I - Q)/2, so
    I = d0 + d90, Q = d0 - d90, U = 2 d45 - d0 - d90."""
    nside = 4
    rng = np.random.default_rng(3)
    d = rng.standard_normal(3 * 192)
    th, ph, psi = _centres_three_angles(nside)
    I, Q, U, rc = M.solve(*M.bin_tod(nside, th, ph, psi, d, 0.0, 0.0, 1.0))
    d0, d45, d90 = d[:192], d[192:384], d[384:]
    for got, want in [(I, d0 + d90), (Q, d0 - d90), (U, 2 * d45 - d0 - d90)]:
        assert np.abs(got - want).max() < 1e-13
    # eigenvalues of 1/4 [[3,1,1],[1,2,0],[1,0,1]]: rcond 3 - 2 sqrt(2)
    assert np.allclose(rc, 3 - 2 * np.sqrt(2), rtol=1e-12)


def test_exact_recovery_with_detectors_and_plate():
    """Samples that follow the measurement model exactly (several detectors,
    random angles, a plate on one) give back the input maps."""
    nside = 8
    npix = 12 * nside * nside
    rng = np.random.default_rng(4)
    m = rng.standard_normal((3, npix))
    ata, atd, hits = np.zeros((npix, 3, 3)), np.zeros((npix, 3)), np.zeros(npix)
    for zeta, eps, s, plate in [(0.0, 0.01, 1.0, False), (-np.pi / 2, 0.02, 0.9, False), (0.7, 0.0, 1.1, True)]:
        n = 8 * npix
        pix = rng.integers(0, npix, n)
        th, ph = oracle.pix2ang(nside, pix)
        psi = rng.uniform(0, 2 * np.pi, n)
        hw = rng.uniform(0, np.pi, n) if plate else None
        a = 2 * (psi + zeta) + (4 * hw if plate else 0.0)
        d = 0.5 * s * ((1 + eps) * m[0, pix] + (1 - eps) * (np.cos(a) * m[1, pix] + np.sin(a) * m[2, pix]))
        x = M.bin_tod(nside, th, ph, psi, d, zeta, eps, s, hw)
        ata += x[0]
        atd += x[1]
        hits += x[2]
    I, Q, U, rc = M.solve(ata, atd, hits)
    ok = rc >= 1e-6
    assert ok.mean() > 0.99
    for k, got in enumerate((I, Q, U)):
        assert np.abs(got[ok] - m[k, ok]).max() < 1e-11


def test_plate_is_a_rotated_angle_and_single_angle_falls_back():
    nside = 4
    rng = np.random.default_rng(5)
    th, ph, psi = _centres_three_angles(nside)
    d = rng.standard_normal(psi.size)
    hw = rng.uniform(0, np.pi, psi.size)
    a = M.solve(*M.bin_tod(nside, th, ph, psi, d, 0.3, 0.01, 1.0, hw))
    b = M.solve(*M.bin_tod(nside, th, ph, psi + 2 * hw, d, 0.3, 0.01, 1.0))
    for x, y in zip(a, b):   # random plate angles leave some pixels badly conditioned: relative bound
        assert np.abs(x - y).max() <= 1e-11 * max(np.abs(y).max(), 1.0)
    # one angle per pixel: rank one, intensity-only solution d / w0
    I, Q, U, rc = M.solve(*M.bin_tod(nside, th[:192], ph[:192], psi[:192], d[:192], 0.0, 0.1, 2.0))
    assert np.all(rc < 1e-12) and not Q.any() and not U.any()
    assert np.abs(I - d[:192] / 1.1).max() < 1e-14


def test_unpolarised_sky_no_leakage_exact_and_interpolated():
    """TOD from the convolution oracle for an I-only sky at every pixel centre
    at psi = 0, 45, 90 deg.  With a beam flat over the disc (bilinear
    interpolation reproduces it exactly at any rotation) the three samples of a
    pixel are equal and the maps have Q = U = 0 to rounding.  With a circular
    Gaussian on the square grid, bilinear interpolation is only four-fold
    symmetric: the 45 deg sample differs at the interpolation-error level, and
    so does the leakage (bounded here)."""
    nside = 8
    I = SK.make_sky(nside, 3 * nside - 1, 2.0, seed=6)[0]
    zero = np.zeros_like(I)
    Tn, u, v, rho, sig = B.tangent_grid(61, 12 * D2R)
    th, ph, psi = _centres_three_angles(nside)
    for flat, bound in [(True, 1e-13), (False, 1e-3)]:
        g = np.ones_like(rho) if flat else B.elliptical_gaussian(rho, sig, 6 * D2R, 0.0, 0.0)
        bs = B.ideal_beamsor(g, Tn)
        d = oracle.tod(nside, I, zero, zero, bs.dense(), Tn, 0.0, 0.0, 1.0, 0.0, 10 * D2R, oracle.NORM_PER_SAMPLE,
                       1.0, th, ph, psi)
        mI, mQ, mU, rc = M.solve(*M.bin_tod(nside, th, ph, psi, d, 0.0, 0.0, 1.0))
        top = np.abs(mI).max()
        assert np.abs(mQ).max() <= bound * top and np.abs(mU).max() <= bound * top, flat
        if flat:
            assert np.abs(mI - 2.0 * d[:768]).max() <= 1e-13 * top   # w_0 = s (1 + eps) / 2 = 1/2
