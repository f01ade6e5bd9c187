"""Pins of the seeded input generators (they feed both the oracle and the GPU path)."""
import numpy as np
from scipy.special import sph_harm_y

from synth import beams as B
from synth import scans as S
from synth import workloads as W
from synth.rings import pixel_centres
from synth.sky import alm2map, alm_index, gaussian_alm, power_law_cl


def test_alm2map_matches_direct_harmonic_sums():
    for nside, lmax in [(4, 11), (8, 30)]:
        rng = np.random.default_rng(nside)
        alm = gaussian_alm(lmax, power_law_cl(lmax, 2.0), rng)
        m = alm2map(alm, lmax, nside)
        th, ph = pixel_centres(nside)
        ref = np.zeros_like(m)
        for l in range(lmax + 1):
            for mm in range(l + 1):
                ref += (alm[alm_index(lmax, l, mm)] * sph_harm_y(l, mm, th, ph)).real * (1 if mm == 0 else 2)
        assert np.abs(m - ref).max() < 1e-12 * np.abs(ref).max()


def test_alm2map_high_m_underflow_is_handled():
    """Large lmax on a coarse map: the scaled recurrences keep every ring finite and
    reproduce direct sums of the few modes that matter on polar rings."""
    nside, lmax = 4, 600
    alm = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=complex)
    alm[alm_index(lmax, 500, 480)] = 1.0 + 0.5j
    m = alm2map(alm, lmax, nside)
    th, ph = pixel_centres(nside)
    ref = 2 * (alm[alm_index(lmax, 500, 480)] * sph_harm_y(500, 480, th, ph)).real
    assert np.all(np.isfinite(m))
    assert np.abs(m - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_grid_and_beams():
    T, u, v, rho, sig = B.tangent_grid(11, np.deg2rad(3.0))
    assert abs(T - np.tan(np.deg2rad(3.0))) < 1e-16
    assert u[5, 5] == 0.0 and v[5, 5] == 0.0 and u[0, 0] == -T and v[-1, 0] == T
    g = B.elliptical_gaussian(rho, sig, np.deg2rad(2.0), 0.1, 0.3)
    assert g[5, 5] == 1.0
    # FWHM along the major axis is wider than along the minor axis
    r = np.deg2rad(1.0)
    maj = B.elliptical_gaussian(np.array(r), np.array(0.3), np.deg2rad(2.0), 0.1, 0.3)
    mnr = B.elliptical_gaussian(np.array(r), np.array(0.3 + np.pi / 2), np.deg2rad(2.0), 0.1, 0.3)
    assert maj > 0.5 > mnr


def test_offset_pointing_distance_and_frame():
    rng = np.random.default_rng(0)
    th, ph, ps = S.uniform_sphere(200, rng)
    th = np.clip(th, 0.2, np.pi - 0.2)
    dx, dy = np.deg2rad(0.5), np.deg2rad(-0.3)
    t2, p2, s2 = S.offset_pointing(th, ph, ps, dx, dy)
    c = np.sin(th) * np.sin(t2) * np.cos(ph - p2) + np.cos(th) * np.cos(t2)
    assert np.abs(np.arccos(np.clip(c, -1, 1)) - np.hypot(dx, dy)).max() < 1e-9
    assert np.abs(np.mod(s2 - ps + np.pi, 2 * np.pi) - np.pi).max() < 0.05


def test_workload_shapes_small():
    w = W.c1(n_samples=1000)
    assert w.nside == 64 and len(w.detectors) == 1 and w.detectors[0].n == 1000
    assert w.sky[0].size == 12 * 64 * 64
    assert w.detectors[0].beam.n == 101
    th = w.detectors[0].theta
    assert np.all((th >= np.deg2rad(30) - 1e-12) & (th <= np.deg2rad(150) + 1e-12))


def test_spin2_synthesis_matches_goldberg():
    """One E mode and one B mode synthesised by the generator equal the closed-form
    spin-2 harmonics (Goldberg et al. 1967, 50-digit arithmetic) at pixel centres:
    Q + iU = -sum_{m=+-m0} (a^E + i a^B)_lm _2Y_lm with a_{l,-m} = (-1)^m a*_lm."""
    from test_oracle_spectra import goldberg

    from synth import sky
    from synth.rings import pixel_centres

    lmax, nside = 5, 4
    th, ph = pixel_centres(nside)
    pick = np.arange(0, 12 * nside * nside, 7)
    for (l, m, e_mode) in ((3, 2, True), (4, 1, False), (2, 0, True), (5, 5, False)):
        a = np.zeros(sky.alm_size(lmax), dtype=np.complex128)
        a[sky.alm_index(lmax, l, m)] = 0.6 - 0.8j if m else 0.7
        z = np.zeros_like(a)
        Q, U = sky.alm2map_spin2(a if e_mode else z, z if e_mode else a, lmax, nside)
        c = a[sky.alm_index(lmax, l, m)]
        for p in pick:
            P = 0j
            for mm in ((m,) if m == 0 else (m, -m)):
                cc = c if mm >= 0 else (-1) ** m * np.conj(c)
                ae, ab = (cc, 0) if e_mode else (0, cc)
                P -= (ae + 1j * ab) * goldberg(2, l, mm, th[p]) * np.exp(1j * mm * ph[p])
            assert abs(Q[p] - P.real) < 1e-12 and abs(U[p] - P.imag) < 1e-12, (l, m, p)


def test_teb_sky_has_the_recipe_correlations():
    from synth import sky

    lmax = 40
    cl = sky.cmb_like_cl(lmax)
    (I, Q, U), (aT, aE, aB) = sky.make_teb_sky(16, lmax, cl, seed=3)
    assert np.all(aB == 0) and np.all(np.isfinite(Q))
    ell = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    sel = ell >= 20
    r = np.sum((aT * np.conj(aE)).real[sel]) / np.sqrt(np.sum(np.abs(aT[sel]) ** 2) * np.sum(np.abs(aE[sel]) ** 2))
    assert 0.2 < r < 0.4          # recipe: correlation 0.3
