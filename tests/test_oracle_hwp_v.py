"""Pins of the oracle's circular-polarisation (V) and half-wave-plate terms.

The plate enters as a modulated beamsor B . H(phi_t) with H(phi) = Lambda(phi)
diag(1, 1, -1, -1) Lambda(-phi) (Sec. 4.1's Lambda; an ideal half-wave plate
at angle phi); V is the fourth Stokes component of the discrete sum (Sec. 4.2,
indices T, Q, U, V).  The checks below use closed forms and identities that
follow from the algebra, each through a route other than the oracle's own
matrix products: delta beams (one pixel), the equivalence of a plate at phi
with a detector rotated by 2 phi for ideal beamsors, the period pi/2 in phi,
and the linearity of the V pickup.
"""
import numpy as np

import oracle
from synth import beams as B
from synth import sky as SK

D2R = np.pi / 180


def _sky(nside, seed):
    I, Q, U = SK.make_sky(nside, 3 * nside - 1, 2.0, seed=seed)
    rng = np.random.default_rng(seed + 1)
    V = 0.05 * rng.standard_normal(I.size)
    return I, Q, U, V


def test_delta_beam_plate_and_v_closed_forms():
    """One pixel, boresight on its centre (chi = psi + zeta), a beam that is flat
    over the (sub-pixel) disc so the rounding of rho near zero does not enter:
    d = s/2 [(1+eps)(I + sign beta V) + (1-eps)(cos(2chi + 4phi) Q + sin(2chi + 4phi) U)]
    with sign = +1 without a plate and -1 with one (the plate flips V)."""
    nside = 16
    I, Q, U, V = _sky(nside, 3)
    pix = np.array([5, 300, 1500, 3071])
    th, ph = oracle.pix2ang(nside, pix)
    rng = np.random.default_rng(7)
    ps = rng.uniform(0, 2 * np.pi, pix.size)
    hw = rng.uniform(0, 2 * np.pi, pix.size)
    beta = 0.2
    bs = B.ideal_beamsor(np.ones((41, 41)), 0.005)
    M = bs.dense().copy()
    M[:, :, 0, 3] = beta                            # V -> T leakage
    T = bs.half_span_tan
    for zeta, eps, s in [(0.0, 0.0, 1.0), (0.4, 0.1, 2.0), (-1.1, -0.05, 0.7)]:
        chi = ps + zeta
        args = (nside, I, Q, U, M, T, zeta, eps, s, 0.0, np.arctan(0.005), oracle.NORM_FIXED, 1.0, th, ph, ps)
        got0 = oracle.tod(*args, V=V)
        want0 = 0.5 * s * ((1 + eps) * (I[pix] + beta * V[pix]) +
                           (1 - eps) * (np.cos(2 * chi) * Q[pix] + np.sin(2 * chi) * U[pix]))
        assert np.abs(got0 - want0).max() < 1e-11
        got1 = oracle.tod(*args, V=V, hwp=hw)
        a = 2 * chi + 4 * hw
        want1 = 0.5 * s * ((1 + eps) * (I[pix] - beta * V[pix]) +
                           (1 - eps) * (np.cos(a) * Q[pix] + np.sin(a) * U[pix]))
        assert np.abs(got1 - want1).max() < 1e-11


def test_plate_equals_rotated_detector_for_ideal_beams():
    """For b x identity beamsors the TOD depends on zeta only through chi in D,
    and Lambda(chi) H(phi) Lambda(-chi) = H(chi + phi): a plate at a constant
    angle phi gives the TOD of a plate-less detector at zeta + 2 phi (any disc)."""
    nside = 16
    I, Q, U, _ = _sky(nside, 5)
    Tn, u, v, rho, sig = B.tangent_grid(61, 8 * D2R)
    g = B.elliptical_gaussian(rho, sig, 3 * D2R, 0.1, 0.3)
    M = B.ideal_beamsor(g, Tn).dense()
    rng = np.random.default_rng(2)
    n = 9
    th, ph, ps = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    for zeta, phi, eps in [(0.0, 0.3, 0.0), (0.7, -1.2, 0.05), (-0.4, 2.5, -0.1)]:
        with_plate = oracle.tod(nside, I, Q, U, M, Tn, zeta, eps, 1.3, 0.0, 7 * D2R, oracle.NORM_PER_SAMPLE, 1.0,
                                th, ph, ps, hwp=np.full(n, phi))
        rotated = oracle.tod(nside, I, Q, U, M, Tn, zeta + 2 * phi, eps, 1.3, 0.0, 7 * D2R, oracle.NORM_PER_SAMPLE,
                             1.0, th, ph, ps)
        assert np.abs(with_plate - rotated).max() <= 1e-12 * np.abs(rotated).max()


def test_plate_period_and_stokes_output():
    """H(phi + pi/2) = H(phi) for any beamsor (here with cross-polar leakage),
    in TOD and Stokes outputs."""
    nside = 16
    I, Q, U, V = _sky(nside, 9)
    Tn, u, v, rho, sig = B.tangent_grid(51, 6 * D2R)
    g = B.elliptical_gaussian(rho, sig, 2.5 * D2R)
    M = B.with_qu_leakage(B.ideal_beamsor(g, Tn), g, 0.03).dense().copy()
    M[:, :, 1, 3] = 0.01 * g                        # V -> Q leakage
    rng = np.random.default_rng(4)
    n = 6
    th, ph, ps = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    hw = rng.uniform(0, np.pi, n)
    for mode in (oracle.OUT_TOD, oracle.OUT_STOKES):
        a = oracle.tod(nside, I, Q, U, M, Tn, 0.2, 0.02, 1.0, 0.0, 5 * D2R, oracle.NORM_FIXED, 1e-3, th, ph, ps,
                       mode, V=V, hwp=hw)
        b = oracle.tod(nside, I, Q, U, M, Tn, 0.2, 0.02, 1.0, 0.0, 5 * D2R, oracle.NORM_FIXED, 1e-3, th, ph, ps,
                       mode, V=V, hwp=hw + np.pi / 2)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
        c = oracle.tod(nside, I, Q, U, M, Tn, 0.2, 0.02, 1.0, 0.0, 5 * D2R, oracle.NORM_FIXED, 1e-3, th, ph, ps,
                       mode, V=V, hwp=hw + 0.3)
        assert np.abs(a - c).max() > 1e-6 * np.abs(a).max()   # the plate angle matters


def test_v_pickup_is_linear_in_the_leakage():
    """A V -> T column beta b adds beta times the intensity-only TOD of the V map
    (D's V entry is zero and Lambda leaves T and V alone)."""
    nside = 16
    I, Q, U, V = _sky(nside, 13)
    Tn, u, v, rho, sig = B.tangent_grid(51, 6 * D2R)
    g = B.elliptical_gaussian(rho, sig, 2.5 * D2R)
    ideal = B.ideal_beamsor(g, Tn).dense()
    leak = ideal.copy()
    beta = 0.3
    leak[:, :, 0, 3] = beta * g
    rng = np.random.default_rng(8)
    n = 7
    th, ph, ps = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    common = (Tn, 0.5, 0.1, 1.7, 0.0, 5 * D2R, oracle.NORM_FIXED, 1e-3, th, ph, ps)
    d_leak = oracle.tod(nside, I, Q, U, leak, *common, V=V)
    d_ideal = oracle.tod(nside, I, Q, U, ideal, *common, V=V)          # V unseen without leakage
    d_ideal_nov = oracle.tod(nside, I, Q, U, ideal, *common)
    zero = np.zeros_like(I)
    d_vmap = oracle.tod(nside, V, zero, zero, ideal, *common)           # V map read as intensity
    assert np.abs(d_ideal - d_ideal_nov).max() == 0.0
    assert np.abs(d_leak - (d_ideal + beta * d_vmap)).max() <= 1e-12 * np.abs(d_leak).max()
