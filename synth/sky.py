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


def _rings_to_map(FN, FS, lmax: int, nside: int) -> np.ndarray:
    """Real map from per-ring coefficients F_m (m >= 0) of the north ring of each
    pair and of its mirror: x(phi) = F_0 + 2 Re sum_{m>0} F_m e^{i m phi}."""
    z, st, npix, first, phi0 = ring_table(nside)
    nring = len(z)
    N = nside
    npair = 2 * N
    F = np.empty((nring, lmax + 1), dtype=np.complex128)
    F[:npair] = FN
    south = 4 * N - np.arange(1, npair)  # ring numbers 4N-1 .. 2N+1 mirror rings 1 .. 2N-1
    F[south - 1] = FS[: npair - 1]
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


def _pairs(nside: int):
    z, st, _, _, _ = ring_table(nside)
    npair = 2 * nside          # ring pairs: north ring r (1..2N) with mirror 4N - r
    return npair, np.ascontiguousarray(z[:npair]), np.ascontiguousarray(st[:npair])


def alm2map(alm: np.ndarray, lmax: int, nside: int) -> np.ndarray:
    """T(pixel) = sum_{l,m} a_lm Y_lm at every RING pixel centre (float64)."""
    npair, zn, sn = _pairs(nside)
    are = np.ascontiguousarray(alm.real)
    aim = np.ascontiguousarray(alm.imag)
    shape = (npair, lmax + 1)
    FNr, FNi, FSr, FSi = (np.empty(shape) for _ in range(4))
    dp = ctypes.POINTER(ctypes.c_double)
    P = lambda a: a.ctypes.data_as(dp)  # noqa: E731
    _native.lib().synth_ring_coeffs(lmax, P(are), P(aim), npair, P(zn), P(sn), P(FNr), P(FNi), P(FSr), P(FSi))
    return _rings_to_map(FNr + 1j * FNi, FSr + 1j * FSi, lmax, nside)


def alm2map_spin2(alm_e: np.ndarray, alm_b: np.ndarray, lmax: int, nside: int):
    """(Q, U) at every RING pixel centre from E and B expansions (float64), with
    Q + iU = -sum (a^E + i a^B)_lm _2Y_lm (Zaldarriaga & Seljak 1997, HEALPix signs)."""
    npair, zn, sn = _pairs(nside)
    ins = [np.ascontiguousarray(x) for x in (alm_e.real, alm_e.imag, alm_b.real, alm_b.imag)]
    outs = [np.empty((npair, lmax + 1)) for _ in range(8)]
    dp = ctypes.POINTER(ctypes.c_double)
    P = lambda a: a.ctypes.data_as(dp)  # noqa: E731
    _native.lib().synth_ring_coeffs_spin2(lmax, *(P(x) for x in ins), npair, P(zn), P(sn), *(P(x) for x in outs))
    QNr, QNi, UNr, UNi, QSr, QSi, USr, USi = outs
    Q = _rings_to_map(QNr + 1j * QNi, QSr + 1j * QSi, lmax, nside)
    U = _rings_to_map(UNr + 1j * UNi, USr + 1j * USi, lmax, nside)
    return Q, U


def cmb_like_cl(lmax: int) -> dict:
    """A CMB-like recipe of our own (no Boltzmann code here): C^TT = (l+1)^-2,
    C^EE = 0.05 C^TT (l / (l + 50))^2 (polarisation grows from large to small
    scales), C^TE = 0.3 sqrt(C^TT C^EE), C^BB = 0 (no primordial or lensing B);
    monopole and dipole zeroed."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    tt = (ell + 1.0) ** -2.0
    ee = 0.05 * tt * (ell / (ell + 50.0)) ** 2
    te = 0.3 * np.sqrt(tt * ee)
    for c in (tt, ee, te):
        c[:2] = 0.0
    return {"TT": tt, "EE": ee, "TE": te, "BB": np.zeros(lmax + 1)}


def make_teb_sky(nside: int, lmax: int, cl: dict, seed: int):
    """(I, Q, U) maps and (a^T, a^E, a^B) of one Gaussian realisation with
    correlated T and E: a^T = sqrt(TT) g1, a^E = (TE / TT) a^T + sqrt(EE - TE^2/TT) g2,
    a^B = sqrt(BB) g3 (g unit complex Gaussians, a_l0 real)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tt, ee, te, bb = cl["TT"], cl["EE"], cl["TE"], cl["BB"]
    g1 = gaussian_alm(lmax, np.ones(lmax + 1), rng)
    g2 = gaussian_alm(lmax, np.ones(lmax + 1), rng)
    g3 = gaussian_alm(lmax, np.ones(lmax + 1), rng)
    ell = np.arange(lmax + 1)
    lidx = np.concatenate([ell[m:] for m in range(lmax + 1)])     # l of every packed entry
    safe = np.where(tt > 0, tt, 1.0)
    aT = np.sqrt(tt)[lidx] * g1
    aE = (te / safe)[lidx] * aT + np.sqrt(np.maximum(ee - te * te / safe, 0.0))[lidx] * g2
    aB = np.sqrt(bb)[lidx] * g3
    I = alm2map(aT, lmax, nside)
    Q, U = alm2map_spin2(aE, aB, lmax, nside)
    return (I, Q, U), (aT, aE, aB)


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
