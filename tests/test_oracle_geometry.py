"""Pins of the oracle's HEALPix geometry and disc selection (CPU only)."""
import os

import numpy as np
import pytest

import oracle
from synth.rings import pixel_centres, ring_table

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_published_centres_nside1_nside2():
    rows = np.loadtxt(os.path.join(GOLD, "healpix_small.txt"))
    for nside, pix, zn, zd, fn, fd in rows:
        z, s, phi = oracle.pix2zphi(int(nside), int(pix))
        assert abs(z[0] - zn / zd) < 1e-15
        assert abs(phi[0] - np.pi * fn / fd) < 1e-14
        assert abs(s[0] - np.sqrt(1 - (zn / zd) ** 2)) < 1e-15


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 64, 1024, 8192])
def test_ring_tiling(nside):
    """Rings tile the pixel index range without gaps: sum of ring sizes is 12 N^2."""
    first_expected = 0
    step = max(1, (4 * nside - 1) // 97)
    rings = sorted(set(list(range(1, 4 * nside, step)) + [1, nside - 1 if nside > 1 else 1, nside, 2 * nside,
                                                          3 * nside, 4 * nside - 1]))
    total = 0
    for i in range(1, 4 * nside):
        cnt = 4 * min(i, nside, 4 * nside - i)
        total += cnt
    assert total == 12 * nside * nside
    for i in rings:
        th, cnt, first = oracle.ring(nside, i)
        assert cnt == 4 * min(i, nside, 4 * nside - i)
        # first pixel index = pixels in all earlier rings
        earlier = sum(4 * min(k, nside, 4 * nside - k) for k in range(1, i))
        assert first == earlier
    del first_expected


@pytest.mark.parametrize("nside", [1, 2, 8, 64])
def test_matches_independent_ring_table(nside):
    """Oracle pixel formula vs the generators' separate ring table, every pixel."""
    th, ph = pixel_centres(nside)
    t2, p2 = oracle.pix2ang(nside, np.arange(12 * nside * nside))
    assert np.abs(th - t2).max() < 1e-14
    d = np.mod(ph - p2 + np.pi, 2 * np.pi) - np.pi
    assert np.abs(d).max() < 1e-13


def test_equal_area_ring_z():
    """Equal-area property: the cap above the boundary between two rings holds an
    integer number of pixels' worth of area.  For polar rings the mean z of a
    ring pair brackets the cap boundary z_b with area 2 pi (1 - z_b) = 4 pi k / (12 N^2)."""
    N = 16
    z, st, npix, first, phi0 = ring_table(N)
    # pixels north of ring i (inclusive) for i < N: 2 i (i + 1); the boundary below
    # ring i is where 1 - z_b = 2 i (i + 1) * 2 / (12 N^2); centres sit inside.
    for i in range(1, N):
        omz_b = 2 * i * (i + 1) * 2.0 / (12 * N * N)
        assert 1 - z[i - 1] < omz_b < 1 - z[i]


@pytest.mark.parametrize("nside", [16, 32])
def test_disc_vs_all_pixel_scan(nside):
    rng = np.random.default_rng(7)
    th, ph = pixel_centres(nside)
    n = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    cases = [(0.0, 0.0, 0.3), (np.pi, 1.0, 0.2), (0.05, 2.0, 0.2), (np.pi / 2, 0.0, 0.1)]
    for _ in range(12):
        cases.append((np.arccos(rng.uniform(-1, 1)), rng.uniform(0, 2 * np.pi), rng.uniform(0.02, 0.6)))
    for t0, f0, r in cases:
        p = np.array([np.sin(t0) * np.cos(f0), np.sin(t0) * np.sin(f0), np.cos(t0)])
        want = np.nonzero(n @ p >= np.cos(r))[0]
        got = oracle.disc(nside, t0, f0, r)
        assert np.array_equal(got, want)


def _read_range():
    path = os.path.join(GOLD, "disc_count_range_nside128.txt")
    return {round(r, 1): (int(lo), int(alo), int(hi), int(ahi)) for r, lo, alo, hi, ahi in np.loadtxt(path)}


def test_paper_table1_disc_sizes_within_range():
    """Every pixel count printed in the paper's benchmark table lies within the
    range of centre-inside disc sizes over all NSIDE-128 pixel-centre pointings."""
    table = np.loadtxt(os.path.join(GOLD, "table1_disc_pixels.txt"))
    rng_ = _read_range()
    for rho, pixels, _ in table:
        lo, _, hi, _ = rng_[round(rho, 1)]
        assert lo <= pixels <= hi, (rho, pixels, lo, hi)


def test_disc_range_file_reproduces():
    """Re-derive the stored extremes at their arg-pixels with the current oracle."""
    rng_ = _read_range()
    for rho in (5.0, 10.0):
        lo, alo, hi, ahi = rng_[rho]
        t, p = oracle.pix2ang(128, [alo, ahi])
        c = oracle.disc_counts(128, t, p, np.deg2rad(rho))
        assert c[0] == lo and c[1] == hi
