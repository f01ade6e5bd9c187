"""Whole-path pins of the FP64 oracle: closed forms, special cases, invariants, brute force."""
import numpy as np
import pytest
from scipy.special import sph_harm_y, eval_legendre

import oracle
from oracle import brute
from synth import beams as B
from synth.rings import pixel_centres, ring_table
from synth.sky import alm2map, alm_index, gaussian_alm, power_law_cl

D2R = np.pi / 180


def _lambda(x):
    return brute.lambda_mat(x)


def _D(chi, eps, s):
    return 0.5 * s * np.array([1 + eps, (1 - eps) * np.cos(2 * chi), (1 - eps) * np.sin(2 * chi), 0.0])


def test_detector_row_absorbs_rotation():
    """D(chi) Lambda(chi) = D(0) for every chi (Sec. 4.1 algebra)."""
    for chi in np.linspace(-3, 3, 13):
        for eps, s in [(0.0, 1.0), (0.2, 1.7)]:
            assert np.abs(_D(chi, eps, s) @ _lambda(chi) - _D(0.0, eps, s)).max() < 1e-15


def _sky(nside, seed, lmax=None):
    rng = np.random.default_rng(seed)
    lmax = lmax or 3 * nside - 1
    return [alm2map(gaussian_alm(lmax, power_law_cl(lmax, 2.0) * a * a, rng), lmax, nside) for a in (1, .1, .1)]


def _gauss_bs(n, span_deg, fwhm_deg, e=0.0, o=0.0, leak=0.0):
    T, u, v, rho, sig = B.tangent_grid(n, span_deg * D2R)
    g = B.elliptical_gaussian(rho, sig, fwhm_deg * D2R, e, o)
    bs = B.ideal_beamsor(g, T)
    if leak:
        bs = B.with_qu_leakage(bs, g, leak)
    return bs


def test_delta_beam_reproduces_boresight_pixel():
    nside = 32
    I, Q, U = _sky(nside, 11)
    # grid spacing and disc radius both far below the pixel size (~0.03 rad)
    bs = B.delta_beamsor(41, 0.01)
    pix = np.array([0, 5, 77, 3000, 6143, 12287, 6000])
    th, ph = oracle.pix2ang(nside, pix)
    rng = np.random.default_rng(0)
    psi = rng.uniform(0, 2 * np.pi, pix.size)
    for zeta, eps, s in [(0.0, 0.0, 1.0), (0.7, 0.1, 2.0)]:
        d = oracle.tod(nside, I, Q, U, bs.dense(), bs.half_span_tan, zeta, eps, s, 0.0,
                       np.arctan(bs.half_span_tan), oracle.NORM_PER_SAMPLE, 1.0, th, ph, psi)
        want = 0.5 * s * ((1 + eps) * I[pix] + (1 - eps) * (Q[pix] * np.cos(2 * (psi + zeta))
                                                             + U[pix] * np.sin(2 * (psi + zeta))))
        assert np.abs(d - want).max() < 1e-13


def test_uniform_sky_per_sample_is_exact_and_fixed_is_nearly_constant():
    nside = 64
    one = np.ones(12 * nside * nside)
    zero = np.zeros_like(one)
    bs = _gauss_bs(101, 4.5, 1.5)
    rng = np.random.default_rng(5)
    th, ph = np.arccos(rng.uniform(-1, 1, 40)), rng.uniform(0, 2 * np.pi, 40)
    psi = rng.uniform(0, 2 * np.pi, 40)
    d = oracle.tod(nside, one, zero, zero, bs.dense(), bs.half_span_tan, 0.3, 0.0, 2.0, 0.0, 4.5 * D2R,
                   oracle.NORM_PER_SAMPLE, 1.0, th, ph, psi)
    assert np.abs(d - 1.0).max() < 1e-14
    # FIXED: N = dOmega / Omega~ with Omega~ the quadrature of B_TT on the tangent grid
    T, u, v, rho, sig = B.tangent_grid(101, 4.5 * D2R)
    h = 2 * T / 100
    jac = (1 + u * u + v * v) ** -1.5
    om = np.sum(bs.get(0, 0) * jac * (rho <= 4.5 * D2R)) * h * h
    dOm = 4 * np.pi / (12 * nside * nside)
    d2 = oracle.tod(nside, one, zero, zero, bs.dense(), bs.half_span_tan, 0.3, 0.0, 2.0, 0.0, 4.5 * D2R,
                    oracle.NORM_FIXED, dOm / om, th, ph, psi)
    assert np.abs(d2 - 1.0).max() < 1e-2
    assert d2.std() < 5e-3


def test_psi_plus_pi_invariance_point_symmetric_beam():
    nside = 64
    I, Q, U = _sky(nside, 3)
    bs = _gauss_bs(101, 4.5, 1.5, e=0.2, o=0.4, leak=0.01)
    rng = np.random.default_rng(9)
    th, ph = np.arccos(rng.uniform(-1, 1, 30)), rng.uniform(0, 2 * np.pi, 30)
    psi = rng.uniform(0, 2 * np.pi, 30)
    args = (bs.dense(), bs.half_span_tan, 0.4, 0.05, 1.0, 0.0, 4.5 * D2R, oracle.NORM_PER_SAMPLE, 1.0, th, ph)
    d1 = oracle.tod(nside, I, Q, U, *args, psi)
    d2 = oracle.tod(nside, I, Q, U, *args, psi + np.pi)
    assert np.abs(d1 - d2).max() < 1e-12 * np.abs(d1).max()
    # a non-symmetric beam does change: the invariance is not vacuous
    g = bs.get(0, 0) * (1 + 0.5 * np.linspace(-1, 1, 101)[None, :])
    bs2 = B.ideal_beamsor(g, bs.half_span_tan)
    a = (bs2.dense(), bs2.half_span_tan, 0.4, 0.05, 1.0, 0.0, 4.5 * D2R, oracle.NORM_PER_SAMPLE, 1.0, th, ph)
    assert np.abs(oracle.tod(nside, I, Q, U, *a, psi) - oracle.tod(nside, I, Q, U, *a, psi + np.pi)).max() > 1e-4


def test_temperature_only_sky_has_no_polarised_response():
    """Ideal beamsor, I-only sky: the TOD does not depend on the detector angle
    and the Stokes pickup has Q = U = 0 exactly (no T to P leakage)."""
    nside = 32
    I, _, _ = _sky(nside, 4)
    z = np.zeros_like(I)
    bs = _gauss_bs(61, 6.0, 3.0, e=0.1)
    rng = np.random.default_rng(2)
    th, ph, psi = np.arccos(rng.uniform(-1, 1, 10)), rng.uniform(0, 6, 10), rng.uniform(0, 6, 10)
    common = (bs.dense(), bs.half_span_tan)
    tail = (0.0, 6 * D2R, oracle.NORM_PER_SAMPLE, 1.0, th, ph, psi)
    a = oracle.tod(nside, I, z, z, *common, 0.0, 0.0, 1.0, *tail)
    b = oracle.tod(nside, I, z, z, *common, 1.1, 0.0, 1.0, *tail)
    assert np.abs(a - b).max() < 1e-14
    st = oracle.tod(nside, I, z, z, *common, 0.0, 0.0, 1.0, *tail, out_mode=oracle.OUT_STOKES)
    assert np.all(st[:, 1:] == 0.0)


def test_stokes_pickup_reassembles_tod():
    """Ideal beamsor: d(zeta) = (s/2)[(1+eps) P_I + (1-eps)(cos 2zeta P_Q + sin 2zeta P_U)]
    with P the Stokes pickup of the zeta = 0 frame (chi is additive in zeta)."""
    nside = 32
    I, Q, U = _sky(nside, 8)
    bs = _gauss_bs(61, 6.0, 3.0, e=0.15, o=1.0)
    rng = np.random.default_rng(4)
    th, ph, psi = np.arccos(rng.uniform(-1, 1, 12)), rng.uniform(0, 6, 12), rng.uniform(0, 6, 12)
    c = (bs.dense(), bs.half_span_tan)
    P = oracle.tod(nside, I, Q, U, *c, 0.0, 0.0, 1.0, 0.0, 6 * D2R, oracle.NORM_FIXED, 1.0, th, ph, psi,
                   out_mode=oracle.OUT_STOKES)
    for zeta, eps, s in [(0.0, 0.0, 2.0), (0.8, 0.3, 1.5), (-1.9, 0.01, 1.0)]:
        d = oracle.tod(nside, I, Q, U, *c, zeta, eps, s, 0.0, 6 * D2R, oracle.NORM_FIXED, 1.0, th, ph, psi)
        want = 0.5 * s * ((1 + eps) * P[:, 0] + (1 - eps) * (np.cos(2 * zeta) * P[:, 1] + np.sin(2 * zeta) * P[:, 2]))
        assert np.abs(d - want).max() < 1e-12 * np.abs(d).max()


def test_quarter_turn_symmetry():
    """Rotating sky and pointing by pi/2 about the pole permutes every ring
    (j -> j + n_ring/4) and leaves the TOD unchanged."""
    nside = 32
    I, Q, U = _sky(nside, 6)
    z, st, npix, first, phi0 = ring_table(nside)
    perm = np.empty(12 * nside * nside, dtype=np.int64)
    for r in range(len(z)):
        n, f = int(npix[r]), int(first[r])
        j = np.arange(n)
        perm[f + (j + n // 4) % n] = f + j
    # rotated map: value at rotated pixel = value at original pixel
    rot = [m[perm] for m in (I, Q, U)]
    bs = _gauss_bs(61, 8.0, 4.0, e=0.2, o=0.3, leak=0.02)
    rng = np.random.default_rng(12)
    th, ph, psi = np.arccos(rng.uniform(-1, 1, 15)), rng.uniform(0, 6, 15), rng.uniform(0, 6, 15)
    c = (bs.dense(), bs.half_span_tan, 0.3, 0.05, 1.0, 0.0, 8 * D2R, oracle.NORM_PER_SAMPLE, 1.0)
    d1 = oracle.tod(nside, I, Q, U, *c, th, ph, psi)
    d2 = oracle.tod(nside, *rot, *c, th, ph + np.pi / 2, psi)
    assert np.abs(d1 - d2).max() < 1e-12 * np.abs(d1).max()


def test_linearity_and_annulus_partition():
    nside = 32
    S1, S2 = _sky(nside, 1), _sky(nside, 2)
    bs = _gauss_bs(81, 10.0, 3.0, e=0.1, leak=0.01)
    rng = np.random.default_rng(3)
    th, ph, psi = np.arccos(rng.uniform(-1, 1, 10)), rng.uniform(0, 6, 10), rng.uniform(0, 6, 10)
    c = (bs.dense(), bs.half_span_tan, 0.2, 0.02, 1.3)
    run = lambda S, rmin, rmax, mode=oracle.OUT_TOD: oracle.tod(  # noqa: E731
        nside, *S, *c, rmin, rmax, oracle.NORM_FIXED, 0.7, th, ph, psi, out_mode=mode)
    a, b = 0.7, -1.9
    mix = [a * x + b * y for x, y in zip(S1, S2)]
    lhs, rhs = run(mix, 0.0, 10 * D2R), a * run(S1, 0.0, 10 * D2R) + b * run(S2, 0.0, 10 * D2R)
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(lhs).max()
    for mode in (oracle.OUT_TOD, oracle.OUT_STOKES):
        full = run(S1, 0.0, 10 * D2R, mode)
        part = run(S1, 0.0, 4 * D2R, mode) + run(S1, 4 * D2R, 10 * D2R, mode)
        assert np.abs(full - part).max() < 1e-13 * np.abs(full).max()


@pytest.mark.parametrize("nside", [4, 8])
def test_matches_brute_force_twin(nside):
    """App.-A oracle vs the main-text vector twin scanning every pixel; a random
    full 4x4 beamsor exercises every Mueller element."""
    rng = np.random.default_rng(nside)
    th_pix, ph_pix = pixel_centres(nside)
    I, Q, U = rng.standard_normal((3, th_pix.size))
    T, u, v, rho, sig = B.tangent_grid(41, 40 * D2R)
    bs = rng.standard_normal((41, 41, 4, 4)) * np.exp(-rho / 0.3)[..., None, None]
    bs[..., 0, 0] = np.abs(bs[..., 0, 0]) + 0.1
    th, ph, psi = np.arccos(rng.uniform(-1, 1, 8)), rng.uniform(0, 6.3, 8), rng.uniform(0, 6.3, 8)
    th[0] = 0.0  # boresight on the pole
    for nm in (oracle.NORM_FIXED, oracle.NORM_PER_SAMPLE):
        for om in (oracle.OUT_TOD, oracle.OUT_STOKES):
            for rmin in (0.0, 12 * D2R):
                args = (I, Q, U, bs, T, 0.4, 0.07, 1.3, rmin, 40 * D2R, nm, 0.9, th, ph, psi, om)
                a = oracle.tod(nside, *args)
                b = brute.tod(th_pix, ph_pix, *args)
                assert np.abs(a - b).max() < 1e-11 * max(1.0, np.abs(a).max())


def test_bilinear_function_is_reproduced_exactly():
    """A beam that is a bilinear function of (u, v) is interpolated exactly; a
    single bright pixel then reads b(u_k, v_k) with (u_k, v_k) = (x'/z', y'/z')."""
    nside = 32
    npix = 12 * nside * nside
    T, u, v, rho, sig = B.tangent_grid(21, 10 * D2R)
    f = lambda uu, vv: 1.0 + 3.0 * uu - 2.0 * vv + 5.0 * uu * vv  # noqa: E731
    bs = B.ideal_beamsor(f(u, v), T)
    rng = np.random.default_rng(1)
    for _ in range(10):
        k = int(rng.integers(0, npix))
        I = np.zeros(npix)
        I[k] = 1.0
        tk, pk = oracle.pix2ang(nside, k)
        t0 = float(np.clip(tk[0] + rng.uniform(-0.05, 0.05), 0.01, 3.13))
        f0, ps0 = pk[0] + rng.uniform(-0.05, 0.05), rng.uniform(0, 6.28)
        d = oracle.tod(nside, I, 0 * I, 0 * I, bs.dense(), T, 0.0, 0.0, 2.0, 0.0, 10 * D2R, oracle.NORM_FIXED, 1.0,
                       [t0], [f0], [ps0])
        _, _, x, y, z = brute.antenna_coords(t0, f0, ps0, tk, pk)
        assert abs(d[0] - f(x[0] / z[0], y[0] / z[0])) < 1e-12


def _beam_legendre(profile, rmax, lmax):
    """B_l = int b P_l(cos r) sin r dr / int b sin r dr (Gauss-Legendre in r)."""
    x, w = np.polynomial.legendre.leggauss(400)
    r = 0.5 * rmax * (x + 1)
    wr = 0.5 * rmax * w * np.sin(r) * profile(r)
    return np.array([np.sum(wr * eval_legendre(l, np.cos(r))) for l in range(lmax + 1)]) / np.sum(wr)


def test_harmonic_smoothing_convergence():
    """Axisymmetric Gaussian beam on a band-limited I sky: the pixel-space sum
    converges to sum_lm a_lm B_l Y_lm(p0).  The error falls with the sky
    resolution, and at fixed sky it falls as h^2 with the beam-grid spacing h
    (bilinear interpolation); B_l is close to exp(-l(l+1) sigma^2 / 2)."""
    lmax = 16
    rng = np.random.default_rng(2024)
    alm = gaussian_alm(lmax, np.ones(lmax + 1), rng)
    sig = 8 * D2R * B.FWHM_TO_SIGMA
    rmax = 25 * D2R
    Bl = _beam_legendre(lambda r: np.exp(-0.5 * (r / sig) ** 2), rmax, lmax)
    ell = np.arange(lmax + 1)
    assert np.abs(Bl - np.exp(-0.5 * ell * (ell + 1) * sig * sig)).max() < 5e-3
    th = np.arccos(rng.uniform(-1, 1, 16))
    ph = rng.uniform(0, 2 * np.pi, 16)
    ref = np.zeros(16)
    for l in range(lmax + 1):
        for m in range(l + 1):
            a = alm[alm_index(lmax, l, m)]
            ref += (a * Bl[l] * sph_harm_y(l, m, th, ph)).real * (1 if m == 0 else 2)

    def err(n, nside):
        T, u, v, rho, sg = B.tangent_grid(n, rmax)
        bs = B.ideal_beamsor(np.exp(-0.5 * (rho / sig) ** 2), T)
        I = alm2map(alm, lmax, nside)
        z = np.zeros_like(I)
        d = oracle.tod(nside, I, z, z, bs.dense(), T, 0.0, 0.0, 2.0, 0.0, rmax, oracle.NORM_PER_SAMPLE, 1.0,
                       th, ph, np.zeros(16))
        return np.abs(d - ref).max() / np.abs(ref).max()

    by_sky = [err(1201, ns) for ns in (8, 16, 32, 64)]
    assert by_sky[1] < by_sky[0] / 10 and by_sky[2] < by_sky[1] / 10 and by_sky[3] < by_sky[2], by_sky
    assert by_sky[-1] < 1.5e-5, by_sky
    by_grid = [err(n, 64) for n in (301, 601)] + [by_sky[-1]]
    for a, b in zip(by_grid, by_grid[1:]):
        assert 3.0 < a / b < 5.0, by_grid
