"""Pins of the antenna-frame trigonometry (the paper's Appendix A) by independent routes."""
import numpy as np
import pytest

import oracle
from oracle import brute


def _wrap(a):
    return np.mod(a + np.pi, 2 * np.pi) - np.pi


def _random_pairs(rng, n, rmax):
    t0 = np.arccos(rng.uniform(-0.98, 0.98, n))
    f0 = rng.uniform(0, 2 * np.pi, n)
    psi = rng.uniform(0, 2 * np.pi, n)
    zeta = rng.uniform(-np.pi, np.pi, n)
    # offset direction at distance r, azimuth a around the pointing
    r = rng.uniform(1e-4, rmax, n)
    a = rng.uniform(0, 2 * np.pi, n)
    out = []
    for k in range(n):
        p, th, ph = brute.sky_basis(t0[k], f0[k])
        d = np.cos(r[k]) * p + np.sin(r[k]) * (np.cos(a[k]) * th + np.sin(a[k]) * ph)
        out.append((t0[k], f0[k], psi[k], zeta[k], np.arccos(np.clip(d[2], -1, 1)), np.arctan2(d[1], d[0])))
    return out


def test_rho_sigma_match_vector_route():
    rng = np.random.default_rng(1)
    for t0, f0, psi, zeta, t, f in _random_pairs(rng, 300, np.deg2rad(25)):
        rho, sig, chi = oracle.appA(t0, f0, psi, zeta, t, f)
        r2, s2, *_ = brute.antenna_coords(t0, f0, psi, np.array(t), np.array(f))
        assert abs(rho - r2) < 1e-14
        assert abs(_wrap(sig - s2)) < 1e-9


def test_rho_full_precision_at_small_separations():
    """rho of a direction placed at a known distance r from the pointing, for r
    from 1e-7 rad to 1 deg: absolute error a few units of 1e-16, where an
    arccosine of the cosine would be off by ~1e-16 / r."""
    rng = np.random.default_rng(7)
    for r in 10.0 ** np.arange(-7.0, -1.7, 0.5):
        t0, f0, a = rng.uniform(0.6, 2.5), rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)
        p, th, ph = brute.sky_basis(t0, f0)
        d = np.cos(r) * p + np.sin(r) * (np.cos(a) * th + np.sin(a) * ph)
        t, f = np.arctan2(np.hypot(d[0], d[1]), d[2]), np.arctan2(d[1], d[0])
        rho, _, _ = oracle.appA(t0, f0, 0.3, 0.0, t, f)
        assert abs(rho - r) < 2e-15, (r, rho - r)


def test_chi_matches_ludwig3_vector_route():
    rng = np.random.default_rng(2)
    for t0, f0, psi, zeta, t, f in _random_pairs(rng, 300, np.deg2rad(25)):
        _, _, chi = oracle.appA(t0, f0, psi, zeta, t, f)
        c2 = brute.chi_ludwig3(t0, f0, psi, zeta, np.array(t), np.array(f))
        # only 2 chi enters the Stokes rotation
        assert abs(_wrap(2 * (chi - c2))) < 1e-9


def test_chi_boresight_limit():
    """As the pixel approaches the boresight chi -> psi + zeta (the detector's own angle)."""
    for psi, zeta in [(0.3, 0.0), (1.2, -0.7), (2.9, 1.1)]:
        for r in (1e-3, 1e-5, 1e-7):
            t0, f0 = 1.1, 0.4
            p, th, ph = brute.sky_basis(t0, f0)
            d = np.cos(r) * p + np.sin(r) * (np.cos(0.9) * th + np.sin(0.9) * ph)
            t, f = np.arccos(d[2]), np.arctan2(d[1], d[0])
            _, _, chi = oracle.appA(t0, f0, psi, zeta, t, f)
            assert abs(_wrap(2 * (chi - psi - zeta))) < 10 * r + 1e-8


def test_chi_along_meridian_and_equator():
    """Parallel transport along a meridian or the equator keeps the angle to theta_hat."""
    # pixel due south on the same meridian, psi = 0, zeta = 0: chi = 0
    _, sig, chi = oracle.appA(0.8, 1.0, 0.0, 0.0, 0.9, 1.0)
    assert abs(_wrap(2 * chi)) < 1e-12 and abs(_wrap(sig)) < 1e-12
    # pixel due east along the equator: chi = psi + zeta, sigma = pi/2 - psi
    psi, zeta = 0.4, 0.25
    _, sig, chi = oracle.appA(np.pi / 2, 0.0, psi, zeta, np.pi / 2, 0.05)
    assert abs(_wrap(2 * (chi - psi - zeta))) < 1e-12
    assert abs(_wrap(sig - (np.pi / 2 - psi))) < 1e-12


def test_printed_rho_hat_is_not_unit_and_fixed_one_is_derivative():
    rho, sig = 0.3, 1.1
    tp, fp, p = np.eye(3)
    k = lambda r: np.sin(r) * np.cos(sig) * tp + np.sin(r) * np.sin(sig) * fp + np.cos(r) * p  # noqa: E731
    printed = np.cos(rho) * np.cos(sig) * tp + np.sin(rho) * np.sin(sig) * fp - np.sin(rho) * p
    fixed = np.cos(rho) * np.cos(sig) * tp + np.cos(rho) * np.sin(sig) * fp - np.sin(rho) * p
    assert abs(np.linalg.norm(printed) - 1) > 1e-2
    assert abs(np.linalg.norm(fixed) - 1) < 1e-15
    num = (k(rho + 1e-6) - k(rho - 1e-6)) / 2e-6
    assert np.abs(num - fixed).max() < 1e-9


@pytest.mark.parametrize("zeta", [0.0, 0.6, -1.3])
def test_ludwig3_equals_great_circle_transport(zeta):
    """Ludwig-3 co-polar vector = boresight co-polar vector carried along the great
    circle to the pixel.  In antenna coordinates with n = (x', y', z') and
    w = x' cos zeta + y' sin zeta this is (cos zeta - x' w/(1+z'), sin zeta - y' w/(1+z'), -w)."""
    rng = np.random.default_rng(3)
    for t0, f0, psi, _, t, f in _random_pairs(rng, 200, np.deg2rad(30)):
        p0, th0, ph0 = brute.sky_basis(t0, f0)
        tp = np.cos(psi) * th0 + np.sin(psi) * ph0
        fp = -np.sin(psi) * th0 + np.cos(psi) * ph0
        _, _, x, y, z = brute.antenna_coords(t0, f0, psi, np.array(t), np.array(f))
        w = x * np.cos(zeta) + y * np.sin(zeta)
        e = (np.cos(zeta) - x * w / (1 + z)) * tp + (np.sin(zeta) - y * w / (1 + z)) * fp - w * p0
        _, tht, pht = brute.sky_basis(t, f)
        chi_t = np.arctan2(e @ pht, e @ tht)
        chi_l = brute.chi_ludwig3(t0, f0, psi, zeta, np.array(t), np.array(f))
        assert abs(_wrap(chi_t - chi_l)) < 1e-10
