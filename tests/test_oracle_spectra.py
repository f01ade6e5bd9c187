"""Pins of the spectrum oracle (`oracle/spectra.py`) against things other than itself:
a library routine (scipy's spherical harmonics), Goldberg's closed form of the
spin-weighted harmonics evaluated in 50-digit arithmetic, exact Gauss-Legendre
quadrature of band-limited fields built from those independent routines,
Parseval's identity, parity under theta -> pi - theta, and the pixel quadrature
of the HEALPix grid at low l."""
import mpmath as mp
import numpy as np
import pytest
from scipy.special import sph_harm_y

from oracle import pix2ang
from oracle import spectra as S

mp.mp.dps = 50


def goldberg(s: int, l: int, m: int, theta: float) -> float:
    """_sY_lm(theta, 0) from the explicit sum of Goldberg et al. (1967)."""
    if l < abs(s) or l < abs(m):
        return 0.0
    th = mp.mpf(theta)
    pre = (-1) ** m * mp.sqrt(mp.factorial(l + m) * mp.factorial(l - m) * (2 * l + 1)
                              / (4 * mp.pi * mp.factorial(l + s) * mp.factorial(l - s)))
    tot = mp.mpf(0)
    for r in range(0, l - s + 1):
        k = r + s - m
        if 0 <= k <= l + s:
            tot += mp.binomial(l - s, r) * mp.binomial(l + s, k) * (-1) ** (l - r - s) * mp.cot(th / 2) ** (2 * r + s - m)
    return float(pre * mp.sin(th / 2) ** (2 * l) * tot)


def test_lambda_matches_scipy():
    rng = np.random.default_rng(0)
    th = np.concatenate([rng.uniform(0.01, np.pi - 0.01, 40), [0.02, np.pi / 2, np.pi - 0.02]])
    lmax = 40
    for m in (0, 1, 2, 7, 23, 40):
        lam = S.lambda_block(m, lmax, np.cos(th), np.sin(th))
        for l in range(m, lmax + 1):
            want = sph_harm_y(l, m, th, 0.0).real
            assert np.allclose(lam[l - m], want, rtol=1e-11, atol=1e-13), (l, m)


def test_spin2_matches_goldberg():
    th = np.array([0.13, 0.9, 1.7, 2.95])
    lmax = 10
    for m in range(0, lmax + 1):
        lam = S.lambda_block(m, lmax, np.cos(th), np.sin(th))
        W, X = S.spin2_block(m, lmax, np.cos(th), np.sin(th), lam)
        for l in range(max(m, 2), lmax + 1):
            for k, t in enumerate(th):
                p, q = goldberg(2, l, m, t), goldberg(-2, l, m, t)
                assert abs(W[l - m, k] - 0.5 * (p + q)) < 1e-12, (l, m, t)
                assert abs(X[l - m, k] - 0.5 * (p - q)) < 1e-12, (l, m, t)
        assert np.all(W[: max(0, 2 - m)] == 0) and np.all(X[: max(0, 2 - m)] == 0)


def test_lambda_survives_underflow_of_the_start():
    """lambda_mm = c_m sin^m theta is below the FP64 range here (~1e-384); the
    carried exponent must bring the recurrence back to the values a 50-digit run
    of the plain recurrence (no scaling: mpmath has no exponent limit) reaches."""
    m, lmax, th = 1200, 2700, 0.5
    lam = S.lambda_block(m, lmax, np.array([np.cos(th)]), np.array([np.sin(th)]))[:, 0]
    z, s = mp.cos(mp.mpf(th)), mp.sin(mp.mpf(th))
    v = 1 / mp.sqrt(4 * mp.pi)
    for k in range(1, m + 1):
        v = -mp.sqrt(mp.mpf(2 * k + 1) / (2 * k)) * s * v
    vals = {m: v}
    vp, v = v, mp.sqrt(2 * m + 3) * z * v
    vals[m + 1] = v
    for l in range(m + 2, lmax + 1):
        a = mp.sqrt(mp.mpf(4 * l * l - 1) / (l * l - m * m))
        b = mp.sqrt(mp.mpf((l - 1) ** 2 - m * m) / (4 * (l - 1) ** 2 - 1))
        vp, v = v, a * (z * v - b * vp)
        vals[l] = v
    assert abs(vals[m]) < mp.mpf(10) ** -380
    hit = 0
    for l in range(m, lmax + 1):
        want = vals[l]
        if abs(want) > mp.mpf(10) ** -290:       # inside FP64's normal range
            hit += 1
            assert abs(lam[l - m] - float(want)) <= 1e-11 * abs(float(want)), l
        elif abs(want) < mp.mpf(10) ** -330:
            assert lam[l - m] == 0.0
    assert hit > 100 and abs(float(vals[lmax])) > 1e-3


def test_parity_under_reflection():
    th = np.array([0.3, 1.1, 1.4])
    lmax = 30
    for m in (0, 1, 5, 18):
        lam_n = S.lambda_block(m, lmax, np.cos(th), np.sin(th))
        lam_s = S.lambda_block(m, lmax, -np.cos(th), np.sin(th))
        Wn, Xn = S.spin2_block(m, lmax, np.cos(th), np.sin(th), lam_n)
        Ws, Xs = S.spin2_block(m, lmax, -np.cos(th), np.sin(th), lam_s)
        for l in range(m, lmax + 1):
            sg = (-1.0) ** (l + m)
            assert np.allclose(lam_s[l - m], sg * lam_n[l - m], atol=1e-13)
            assert np.allclose(Ws[l - m], sg * Wn[l - m], atol=1e-13)
            assert np.allclose(Xs[l - m], -sg * Xn[l - m], atol=1e-13)


def _random_alm(rng, lmax, lmin=0):
    a = np.zeros(S.alm_size(lmax), dtype=np.complex128)
    for m in range(lmax + 1):
        for l in range(max(m, lmin), lmax + 1):
            a[S.alm_index(lmax, l, m)] = rng.normal() + (1j * rng.normal() if m > 0 else 0.0)
    return a


def _synth_gauss(rings, lmax, aT, aE, aB):
    """Band-limited T, Q, U on the ring grid from scipy's Y_lm and Goldberg's _{+-2}Y_lm
    (independent of the oracle).  Q + iU = -sum_{l, m=-l..l} (a^E + i a^B)_lm _2Y_lm,
    with a_{l,-m} = (-1)^m a*_lm."""
    nr = len(rings["z"])
    n = int(rings["count"][0])
    th = np.arctan2(rings["s"], rings["z"])
    T = np.zeros(nr * n)
    P = np.zeros(nr * n, dtype=np.complex128)
    for r in range(nr):
        ph = rings["phi0"][r] + 2 * np.pi * np.arange(n) / n
        sl = slice(r * n, (r + 1) * n)
        for l in range(lmax + 1):
            for m in range(0, l + 1):
                y = sph_harm_y(l, m, th[r], ph)
                a = aT[S.alm_index(lmax, l, m)]
                T[sl] += (a * y).real * (1.0 if m == 0 else 2.0)
                if l < 2:
                    continue
                for mm in ((m,) if m == 0 else (m, -m)):
                    ae, ab = aE[S.alm_index(lmax, l, m)], aB[S.alm_index(lmax, l, m)]
                    if mm < 0:
                        ae, ab = (-1) ** m * np.conj(ae), (-1) ** m * np.conj(ab)
                    P[sl] -= (ae + 1j * ab) * goldberg(2, l, mm, th[r]) * np.exp(1j * mm * ph)
    return T, P.real.copy(), P.imag.copy()


def test_exact_quadrature_recovers_alm_and_parseval():
    rng = np.random.default_rng(1)
    lmax = 6
    rings = S.gauss_rings(lmax + 2, 2 * lmax + 4, phi0=0.37)
    aT, aE, aB = _random_alm(rng, lmax), _random_alm(rng, lmax, 2), _random_alm(rng, lmax, 2)
    T, Q, U = _synth_gauss(rings, lmax, aT, aE, aB)
    gT, gE, gB = S.map2alm(T, Q, U, rings, lmax)
    assert np.abs(gT - aT).max() < 1e-12
    assert np.abs(gE - aE).max() < 1e-12
    assert np.abs(gB - aB).max() < 1e-12
    w = np.repeat(rings["weight"], rings["count"])
    cl = [S.alm2cl(a, b, lmax) for a, b in ((gT, gT), (gE, gE), (gB, gB))]
    l = np.arange(lmax + 1)
    assert abs(np.sum(w * T * T) - np.sum((2 * l + 1) * cl[0])) < 1e-11 * np.sum(w * T * T)
    assert abs(np.sum(w * (Q * Q + U * U)) - np.sum((2 * l + 1) * (cl[1] + cl[2]))) < 1e-11 * np.sum(w * (Q * Q + U * U))


def test_pure_e_and_pure_b_do_not_mix():
    """A single E mode gives no B and vice versa (the sign and factor of i in the
    E/B definitions), on the exact grid."""
    lmax = 5
    rings = S.gauss_rings(lmax + 2, 2 * lmax + 3, phi0=0.0)
    z = np.zeros(S.alm_size(lmax), dtype=np.complex128)
    for (l, m) in ((2, 0), (3, 2), (5, 5)):
        one = z.copy()
        one[S.alm_index(lmax, l, m)] = 1.0 if m == 0 else 0.6 - 0.8j
        for e_mode in (True, False):
            T, Q, U = _synth_gauss(rings, lmax, z, one if e_mode else z, z if e_mode else one)
            _, gE, gB = S.map2alm(T, Q, U, rings, lmax)
            want, other = (gE, gB) if e_mode else (gB, gE)
            assert np.abs(want - one).max() < 1e-12 and np.abs(other).max() < 1e-12


def test_healpix_rings_and_low_l_quadrature():
    nside, lmax = 16, 4
    R = S.healpix_rings(nside)
    assert R["count"].sum() == 12 * nside * nside
    assert np.all(R["first"][1:] == np.cumsum(R["count"])[:-1])
    assert np.allclose(R["z"] ** 2 + R["s"] ** 2, 1.0)
    rng = np.random.default_rng(2)
    aT = _random_alm(rng, lmax)
    th, ph = pix2ang(nside, np.arange(12 * nside * nside))
    T = np.zeros(th.size)
    for l in range(lmax + 1):
        for m in range(l + 1):
            T += (aT[S.alm_index(lmax, l, m)] * sph_harm_y(l, m, th, ph)).real * (1.0 if m == 0 else 2.0)
    gT, _, _ = S.map2alm(T, None, None, R, lmax)
    # one pass of pixel quadrature: error well below a percent at l << nside
    assert np.abs(gT - aT).max() < 3e-3 * np.abs(aT).max()


def test_anafast_orders_spectra():
    nside, lmax = 8, 10
    rng = np.random.default_rng(3)
    T, Q, U = rng.normal(size=(3, 12 * nside * nside))
    cl = S.anafast(nside, lmax, T, Q, U)
    R = S.healpix_rings(nside)
    aT, aE, aB = S.map2alm(T, Q, U, R, lmax)
    assert np.allclose(cl[3], S.alm2cl(aT, aE, lmax)) and np.allclose(cl[4], S.alm2cl(aE, aB, lmax))
    assert np.allclose(cl[1], S.alm2cl(aE, aE, lmax)) and np.all(cl[:3] >= 0)
    assert np.allclose(cl[1:3, :2], 0.0)          # no spin-2 power below l = 2


def test_gauss_beam_window_against_quadrature():
    """b_l of a normalised circular Gaussian by Legendre quadrature of its profile
    agrees with exp(-l(l+1) sigma^2 / 2) to O(sigma^2)."""
    fwhm = np.deg2rad(1.5)
    sig = fwhm / np.sqrt(8 * np.log(2))
    x, w = np.polynomial.legendre.leggauss(4000)
    th = np.arccos(x)
    prof = np.exp(-0.5 * (th / sig) ** 2)
    from scipy.special import eval_legendre
    b0 = np.sum(w * prof)
    bl = S.gauss_beam_window(fwhm, 300)
    for l in (10, 100, 200, 300):
        got = np.sum(w * prof * eval_legendre(l, x)) / b0
        assert abs(got - bl[l]) < 2e-3, l
    assert np.all(S.gauss_beam_window(fwhm, 300, spin=2)[2:] >= bl[2:])


def test_alm2map_single_modes_match_closed_forms():
    """Synthesis of one mode equals scipy's Y_lm (spin 0) and Goldberg's _2Y_lm
    (spin 2) at HEALPix pixel centres."""
    nside, lmax = 4, 5
    R = S.healpix_rings(nside)
    th, ph = pix2ang(nside, np.arange(12 * nside * nside))
    pick = np.arange(0, th.size, 5)
    z = np.zeros(S.alm_size(lmax), dtype=np.complex128)
    for (l, m) in ((3, 2), (5, 0), (4, 4)):
        one = z.copy()
        one[S.alm_index(lmax, l, m)] = 0.6 - 0.8j if m else 0.9
        T, _, _ = S.alm2map(one, None, None, R, lmax)
        want = (one[S.alm_index(lmax, l, m)] * sph_harm_y(l, m, th, ph)).real * (1.0 if m == 0 else 2.0)
        assert np.abs(T - want).max() < 1e-13
        for e_mode in (True, False):
            _, Q, U = S.alm2map(z, one if e_mode else z, z if e_mode else one, R, lmax)
            c = one[S.alm_index(lmax, l, m)]
            for p in pick:
                P = 0j
                for mm in ((m,) if m == 0 else (m, -m)):
                    cc = c if mm >= 0 else (-1) ** m * np.conj(c)
                    ae, ab = (cc, 0) if e_mode else (0, cc)
                    P -= (ae + 1j * ab) * goldberg(2, l, mm, th[p]) * np.exp(1j * mm * ph[p])
                assert abs(Q[p] - P.real) < 1e-12 and abs(U[p] - P.imag) < 1e-12


def test_alm2map_inverts_exact_quadrature():
    rng = np.random.default_rng(4)
    lmax = 8
    rings = S.gauss_rings(lmax + 2, 2 * lmax + 3, phi0=0.21)
    a = [_random_alm(rng, lmax), _random_alm(rng, lmax, 2), _random_alm(rng, lmax, 2)]
    maps = S.alm2map(*a, rings, lmax)
    back = S.map2alm(*maps, rings, lmax)
    for x, y in zip(a, back):
        assert np.abs(x - y).max() < 1e-12


def test_iterations_shrink_the_quadrature_error():
    """On HEALPix pixels one pass of quadrature errs at ~1e-2 here (l up to 1.25
    nside); the Jacobi steps contract the error geometrically, by a factor of the
    order of the quadrature error itself (at least ten per step)."""
    nside, lmax = 16, 20
    R = S.healpix_rings(nside)
    rng = np.random.default_rng(5)
    a = [_random_alm(rng, lmax), _random_alm(rng, lmax, 2), _random_alm(rng, lmax, 2)]
    maps = S.alm2map(*a, R, lmax)
    errs = []
    for it in (0, 1, 3):
        got = S.map2alm_iter(*maps, R, lmax, it)
        errs.append(max(np.abs(x - y).max() for x, y in zip(a, got)) / np.abs(a[0]).max())
    assert errs[0] < 2e-2 and errs[1] < 0.1 * errs[0] and errs[2] < 1e-3 * errs[0]
