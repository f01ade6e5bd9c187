"""Seeded Gaussian skies on the HEALPix RING grid.

A sky is drawn as complex Gaussian a_lm with variance C_l and synthesised
onto pixel centres.  Power spectra follow the workload recipes:
C_l = (l + 1)^-p for l <= lmax (p = 2 or 3), with Q and U drawn as two
further independent realisations at amplitude ``pol_frac`` of I.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from .rings import ring_table


def alm_size(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(lmax: int, l, m):
    """m-major packing used throughout the generators."""
    return m * (lmax + 1) - m * (m - 1) // 2 + (l - m)


def gaussian_alm(lmax: int, cl: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Complex a_lm, m >= 0, with <|a_lm|^2> = C_l (a_l0 real)."""
    out = np.zeros(alm_size(lmax), dtype=np.complex128)
    for m in range(lmax + 1):
        ls = np.arange(m, lmax + 1)
        k = alm_index(lmax, ls, m)
        sd = np.sqrt(cl[ls])
        if m == 0:
            out[k] = rng.standard_normal(len(ls)) * sd
        else:
            out[k] = (rng.standard_normal(len(ls)) + 1j * rng.standard_normal(len(ls))) * sd / np.sqrt(2.0)
    return out


def alm2map(alm: np.ndarray, lmax: int, nside: int) -> np.ndarray:
    """T(pixel) = sum_{l,m} a_lm Y_lm at every RING pixel centre (float64)."""
    z, st, npix, first, phi0 = ring_table(nside)
    nring = len(z)
    N = nside
    # ring pairs: north ring r (1..2N) with mirror 4N - r
    npair = 2 * N
    zn = np.ascontiguousarray(z[:npair])
    sn = np.ascontiguousarray(st[:npair])
    are = np.ascontiguousarray(alm.real)
    aim = np.ascontiguousarray(alm.imag)
    shape = (npair, lmax + 1)
    FNr, FNi, FSr, FSi = (np.empty(shape) for _ in range(4))
    dp = ctypes.POINTER(ctypes.c_double)
    P = lambda a: a.ctypes.data_as(dp)  # noqa: E731
    _native.lib().synth_ring_coeffs(lmax, P(are), P(aim), npair, P(zn), P(sn), P(FNr), P(FNi), P(FSr), P(FSi))
    F = np.empty((nring, lmax + 1), dtype=np.complex128)
    F[:npair] = FNr + 1j * FNi
    south = 4 * N - np.arange(1, npair)  # ring numbers 4N-1 .. 2N+1 mirror rings 1 .. 2N-1
    F[south - 1] = (FSr + 1j * FSi)[: npair - 1]
    out = np.empty(12 * N * N)
    m = np.arange(lmax + 1)
    wm = np.where(m == 0, 1.0, 2.0)
    for r in range(nring):
        n = int(npix[r])
        G = F[r] * wm * np.exp(1j * m * phi0[r])
        H = np.zeros(n, dtype=np.complex128)
        np.add.at(H, m % n, G)
        vals = (np.fft.ifft(H) * n).real
        out[int(first[r]): int(first[r]) + n] = vals
    return out


def power_law_cl(lmax: int, power: float, amp: float = 1.0) -> np.ndarray:
    ell = np.arange(lmax + 1, dtype=np.float64)
    return amp * (ell + 1.0) ** (-power)


def make_sky(nside: int, lmax: int, power: float, seed: int, pol_frac: float = 0.1, return_alm: bool = False):
    """I, Q, U maps (float64, RING) from three independent seeded realisations."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cl = power_law_cl(lmax, power)
    maps, alms = [], []
    for amp in (1.0, pol_frac, pol_frac):
        a = gaussian_alm(lmax, cl * amp * amp, rng)
        alms.append(a)
        maps.append(alm2map(a, lmax, nside))
    if return_alm:
        return maps, alms
    return maps
