"""Spherical-harmonic analysis of I, Q, U maps and their angular power spectra:
test infrastructure, like the rest of `oracle/`.  Nothing outside `tests/`,
the smoke check and the benchmark's CPU leg may import it.

The paper sends its maps to an external spectrum estimator (Sec. 6.2) and
compares the beam-corrected spectra with those of the input maps.  This is
that estimator, written from the standard definitions:

  Y_lm(theta, phi) = lambda_lm(theta) e^{i m phi}: orthonormal spherical
      harmonics with the Condon-Shortley phase;
  _{+-2}Y_lm = (W_lm(theta) +- X_lm(theta)) e^{i m phi}: spin-weighted
      harmonics in the convention of Goldberg et al. (1967, J. Math. Phys. 8,
      2155), W and X real;
  a^T_lm = sum_p w_p T_p Y*_lm(p),
  a^{+-2}_lm = sum_p w_p (Q +- iU)_p _{+-2}Y*_lm(p),
  a^E = -(a^2 + a^-2) / 2,  a^B = i (a^2 - a^-2) / 2
      (Zaldarriaga & Seljak 1997, PRD 55, 1830; the HEALPix convention of
      Gorski et al. 2005), so that Q + iU = -sum (a^E + i a^B) _2Y_lm;
  C^XY_l = (2l + 1)^-1 sum_{m=-l..l} a^X_lm a^Y*_lm (real part),
      using a_{l,-m} = (-1)^m a*_lm for real maps.

w_p is the quadrature weight of pixel p: 4 pi / Npix on the HEALPix grid,
Gauss-Legendre weights on the grids the pins use.  `map2alm` is one pass of
that quadrature; `map2alm_iter` refines it by Jacobi steps through the
synthesis `alm2map` (the scheme of HEALPix's anafast with iterations).

Steps, in the order the sums are written: the Fourier sum along each
iso-latitude ring (a library FFT, then the ring's phase offset), then the sum
over rings with lambda_lm from the three-term recurrence in l, and W, X from
lambda_lm and lambda_{l-1,m} by the spin-raising identities (Kamionkowski,
Kosowsky & Stebbins 1997, PRD 55, 7368).  lambda_mm is carried as a mantissa
and a power-of-two exponent so that sin^m(theta) does not underflow before
the recurrence lifts it back (Press et al., Numerical Recipes, Sec. 6.7).
"""
from __future__ import annotations

import numpy as np

from . import _lib

SCALE = 256                      # exponent step of the carried recurrence
_UP = 2.0 ** SCALE
_DOWN = 2.0 ** -SCALE

SPECTRA = ("TT", "EE", "BB", "TE", "EB", "TB")


def alm_size(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(lmax: int, l, m):
    """m-major packing: all l = m..lmax of m = 0, then of m = 1, ..."""
    return m * (2 * lmax + 1 - m) // 2 + l


def healpix_rings(nside: int) -> dict:
    """Ring table of the RING scheme (rings 1..4N-1): cos and sin of the
    colatitude, longitude of the first pixel, pixel count, first pixel index,
    and the weight of every pixel (4 pi / Npix)."""
    import ctypes

    N = int(nside)
    nr = 4 * N - 1
    z, s, phi0 = (np.empty(nr) for _ in range(3))
    count = np.empty(nr, dtype=np.int64)
    first = np.empty(nr, dtype=np.int64)
    th = ctypes.c_double()
    cnt, fst = ctypes.c_int64(), ctypes.c_int64()
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    for r in range(nr):
        _lib().orc_ring(N, r + 1, ctypes.byref(th), ctypes.byref(cnt), ctypes.byref(fst))
        _lib().orc_pix2zphi(N, fst.value, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        z[r], s[r], phi0[r] = a.value, b.value, c.value
        count[r], first[r] = cnt.value, fst.value
    w = np.full(nr, 4.0 * np.pi / (12.0 * N * N))
    return {"z": z, "s": s, "phi0": phi0, "count": count, "first": first, "weight": w}


def gauss_rings(nlat: int, nlon: int, phi0: float = 0.0) -> dict:
    """Gauss-Legendre rings in cos(theta) with nlon equally spaced pixels each:
    exact quadrature for band-limited products of degree < 2 nlat in cos(theta)
    and < nlon in phi."""
    x, wx = np.polynomial.legendre.leggauss(nlat)
    z = x[::-1].copy()
    return {"z": z, "s": np.sqrt((1.0 - z) * (1.0 + z)), "phi0": np.full(nlat, float(phi0)),
            "count": np.full(nlat, nlon, dtype=np.int64), "first": np.arange(nlat, dtype=np.int64) * nlon,
            "weight": wx[::-1] * 2.0 * np.pi / nlon}


def ring_fourier(m_map, rings: dict, mmax: int) -> np.ndarray:
    """F[r, m] = sum_j x_{r,j} exp(-i m phi_{r,j}), phi_{r,j} = phi0_r + 2 pi j / n_r,
    for m = 0..mmax (the ring's DFT read at m mod n_r, times exp(-i m phi0_r))."""
    x = np.asarray(m_map, dtype=np.float64)
    nr = len(rings["z"])
    F = np.empty((nr, mmax + 1), dtype=np.complex128)
    m = np.arange(mmax + 1)
    for r in range(nr):
        n, f = int(rings["count"][r]), int(rings["first"][r])
        X = np.fft.fft(x[f:f + n])
        F[r] = np.exp(-1j * m * rings["phi0"][r]) * X[m % n]
    return F


def lambda_block(m: int, lmax: int, z, s) -> np.ndarray:
    """lambda_lm at every ring for l = m..lmax (rows l - m)."""
    z = np.asarray(z, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros((lmax - m + 1, z.size))
    if m > lmax:
        return out
    # lambda_mm = (-1)^m c_m s^m with c_0 = 1 / sqrt(4 pi), c_k / c_{k-1} = sqrt((2k + 1) / (2k))
    v = np.full(z.size, 1.0 / np.sqrt(4.0 * np.pi))
    e = np.zeros(z.size, dtype=np.int64)
    for k in range(1, m + 1):
        v = -np.sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * v
        small = np.abs(v) < _DOWN
        v = np.where(small, v * _UP, v)
        e = e - small
    out[0] = np.ldexp(v, SCALE * e)
    if lmax == m:
        return out
    v_prev, v = v, np.sqrt(2.0 * m + 3.0) * z * v
    out[1] = np.ldexp(v, SCALE * e)
    for l in range(m + 2, lmax + 1):
        a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
        v_prev, v = v, a * (z * v - b * v_prev)
        big = np.abs(v) > _UP
        v = np.where(big, v * _DOWN, v)
        v_prev = np.where(big, v_prev * _DOWN, v_prev)
        e = e + big
        out[l - m] = np.ldexp(v, SCALE * e)
    return out


def spin2_block(m: int, lmax: int, z, s, lam: np.ndarray):
    """W_lm and X_lm (rows l - m) from lambda_lm and lambda_{l-1,m}:

      W = n_l [ -((l - m^2) / s^2 + l (l - 1) / 2) lambda_l + (l + m) c_lm (z / s^2) lambda_{l-1} ]
      X = n_l (m / s^2) [ -(l - 1) z lambda_l + (l + m) c_lm lambda_{l-1} ]

    with n_l = 2 sqrt((l - 2)! / (l + 2)!) and c_lm = sqrt((2l + 1)(l - m) / ((2l - 1)(l + m)))
    (the ratio of the normalisations of lambda_lm and lambda_{l-1,m}); zero for l < 2."""
    z = np.asarray(z, dtype=np.float64)
    s2 = np.asarray(s, dtype=np.float64) ** 2
    W = np.zeros_like(lam)
    X = np.zeros_like(lam)
    for l in range(max(m, 2), lmax + 1):
        lam_l = lam[l - m]
        lam_p = lam[l - m - 1] if l > m else np.zeros_like(lam_l)
        c = np.sqrt((2.0 * l + 1.0) * (l - m) / ((2.0 * l - 1.0) * (l + m))) if l > m else 0.0
        n_l = 2.0 / np.sqrt((l - 1.0) * l * (l + 1.0) * (l + 2.0))
        W[l - m] = n_l * (-((l - m * m) / s2 + l * (l - 1.0) / 2.0) * lam_l + (l + m) * c * z / s2 * lam_p)
        X[l - m] = n_l * (m / s2) * (-(l - 1.0) * z * lam_l + (l + m) * c * lam_p)
    return W, X


def map2alm(T, Q, U, rings: dict, lmax: int, mmax: int | None = None, ms=None):
    """a^T, a^E, a^B (complex, m-major packing of `alm_index`).  Q and U may be
    None (a^E, a^B then None).  `ms` restricts the work to those m (other
    entries stay zero)."""
    mmax = lmax if mmax is None else mmax
    pol = Q is not None
    w = rings["weight"]
    FT = ring_fourier(T, rings, mmax) * w[:, None]
    if pol:
        FQ = ring_fourier(Q, rings, mmax) * w[:, None]
        FU = ring_fourier(U, rings, mmax) * w[:, None]
    n = alm_size(lmax)
    aT = np.zeros(n, dtype=np.complex128)
    aE = np.zeros(n, dtype=np.complex128) if pol else None
    aB = np.zeros(n, dtype=np.complex128) if pol else None
    for m in (range(mmax + 1) if ms is None else ms):
        lam = lambda_block(m, lmax, rings["z"], rings["s"])
        k = alm_index(lmax, np.arange(m, lmax + 1), m)
        aT[k] = lam @ FT[:, m]
        if pol:
            W, X = spin2_block(m, lmax, rings["z"], rings["s"], lam)
            aE[k] = -(W @ FQ[:, m] + 1j * (X @ FU[:, m]))
            aB[k] = -(W @ FU[:, m] - 1j * (X @ FQ[:, m]))
    return aT, aE, aB


def alm2map(aT, aE, aB, rings: dict, lmax: int, mmax: int | None = None):
    """Maps at the ring pixels from a^T (and a^E, a^B): the sums the analysis
    inverts, written out,

      T = sum_{l, m=-l..l} a^T_lm Y_lm,
      Q + iU = -sum_{l, m=-l..l} (a^E + i a^B)_lm _2Y_lm,

    i.e. with a_{l,-m} = (-1)^m a*_lm, per ring x(phi) = G_0 + 2 Re sum_{m>0} G_m e^{i m phi},
      G^T_m = sum_l a^T_lm lambda_lm,  G^Q_m = -sum_l (a^E W + i a^B X)_lm,
      G^U_m = -sum_l (a^B W - i a^E X)_lm.
    Returns (T, Q, U) (Q, U None without a^E)."""
    mmax = lmax if mmax is None else mmax
    pol = aE is not None
    nr = len(rings["z"])
    GT = np.zeros((nr, mmax + 1), dtype=np.complex128)
    GQ = np.zeros_like(GT) if pol else None
    GU = np.zeros_like(GT) if pol else None
    for m in range(mmax + 1):
        lam = lambda_block(m, lmax, rings["z"], rings["s"])
        k = alm_index(lmax, np.arange(m, lmax + 1), m)
        GT[:, m] = aT[k] @ lam
        if pol:
            W, X = spin2_block(m, lmax, rings["z"], rings["s"], lam)
            GQ[:, m] = -(aE[k] @ W + 1j * (aB[k] @ X))
            GU[:, m] = -(aB[k] @ W - 1j * (aE[k] @ X))
    npix = int(rings["count"].sum())
    outs = []
    for G in (GT, GQ, GU):
        if G is None:
            outs.append(None)
            continue
        x = np.empty(npix)
        m = np.arange(mmax + 1)
        c = np.where(m == 0, 1.0, 2.0)
        for r in range(nr):
            n, f = int(rings["count"][r]), int(rings["first"][r])
            phi = rings["phi0"][r] + 2.0 * np.pi * np.arange(n) / n
            x[f:f + n] = ((c * G[r]) @ np.exp(1j * np.outer(m, phi))).real
        outs.append(x)
    return tuple(outs)


def map2alm_iter(T, Q, U, rings: dict, lmax: int, iterations: int):
    """Pixel quadrature refined by `iterations` Jacobi steps:
    a <- map2alm(m), then a <- a + map2alm(m - alm2map(a)) (the scheme of
    HEALPix's anafast with iter > 0)."""
    a = list(map2alm(T, Q, U, rings, lmax))
    maps = [T, Q, U]
    for _ in range(iterations):
        syn = alm2map(*a, rings, lmax)
        res = [None if m is None else m - s for m, s in zip(maps, syn)]
        d = map2alm(*res, rings, lmax)
        a = [None if x is None else x + y for x, y in zip(a, d)]
    return tuple(a)


def alm2cl(a, b, lmax: int) -> np.ndarray:
    """C_l = (2l + 1)^-1 [Re(a_l0 b*_l0) + 2 sum_{m>0} Re(a_lm b*_lm)]."""
    cl = np.zeros(lmax + 1)
    for l in range(lmax + 1):
        m = np.arange(l + 1)
        p = (a[alm_index(lmax, l, m)] * np.conj(b[alm_index(lmax, l, m)])).real
        cl[l] = (p[0] + 2.0 * p[1:].sum()) / (2.0 * l + 1.0)
    return cl


def anafast(nside: int, lmax: int, T, Q, U, iterations: int = 0) -> np.ndarray:
    """(6, lmax + 1) spectra TT, EE, BB, TE, EB, TB of RING maps."""
    aT, aE, aB = map2alm_iter(T, Q, U, healpix_rings(nside), lmax, iterations)
    pairs = ((aT, aT), (aE, aE), (aB, aB), (aT, aE), (aE, aB), (aT, aB))
    return np.stack([alm2cl(a, b, lmax) for a, b in pairs])


def gauss_beam_window(fwhm_rad: float, lmax: int, spin: int = 0) -> np.ndarray:
    """Transfer function b_l of a circular Gaussian beam: exp(-(l(l+1) - s^2) sigma^2 / 2)
    (s = 0 for temperature, 2 for the E and B spin-2 fields; Challinor et al. 2000)."""
    sig = fwhm_rad / np.sqrt(8.0 * np.log(2.0))
    l = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * (l * (l + 1.0) - spin * spin) * sig * sig)
