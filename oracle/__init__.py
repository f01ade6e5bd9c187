"""Plain FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it,
and it shares no code with the GPU path: its HEALPix geometry, its
antenna-frame trigonometry (the paper's Appendix A) and its literal 4x4
Mueller products live in ``pisco_oracle.c``; ``brute.py`` is a numpy twin
following the paper's main-text vector definitions for tiny maps; ``mlp.py``
is the FP64 reference for the sidelobe network.

Every function that has no pin says so; see ``tests/test_oracle_*.py`` for
the pins (paper table values, closed forms, invariants, brute force).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pisco_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_h = None

NORM_FIXED = 0
NORM_PER_SAMPLE = 1
OUT_TOD = 0
OUT_STOKES = 1


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               _SRC, "-o", _LIB, "-lm"])
    return _LIB


def _lib():
    global _h
    if _h is None:
        if not os.path.exists(_LIB):
            build(force=True)
        h = ctypes.CDLL(_LIB)
        i64, dbl, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        h.orc_pix2zphi.argtypes = [i64, i64, dp, dp, dp]
        h.orc_pix2ang.argtypes = [i64, i64, dp, dp]
        h.orc_ring.argtypes = [i64, i64, dp, lp, lp]
        h.orc_appA.argtypes = [dbl, dbl, dbl, dbl, dbl, dbl, dp, dp, dp]
        h.orc_tod.argtypes = [i64, dp, dp, dp, i32, dbl, dp, dbl, dbl, dbl, dbl, dbl, i32, dbl,
                              i64, dp, dp, dp, i32, dp, i32]
        h.orc_tod.restype = i32
        h.orc_tod_iquv.argtypes = [i64, dp, dp, dp, dp, i32, dbl, dp, dbl, dbl, dbl, dbl, dbl, i32, dbl,
                                   i64, dp, dp, dp, dp, i32, dp, i32]
        h.orc_tod_iquv.restype = i32
        h.orc_disc.argtypes = [i64, dbl, dbl, dbl, lp, i64]
        h.orc_disc.restype = i64
        h.orc_disc_counts.argtypes = [i64, i64, dp, dp, dbl, lp, i32]
        h.orc_max_threads.restype = i32
        h.orc_ang2pix.argtypes = [i64, i64, dp, dp, lp]
        h.orc_healpix_interp.argtypes = [i64, dp, dbl, dbl]
        h.orc_healpix_interp.restype = dbl
        h.orc_healpix_to_grid.argtypes = [i64, dp, dbl, i32, dp]
        _h = h
    return _h


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def max_threads() -> int:
    return int(_lib().orc_max_threads())


def pix2ang(nside: int, pix):
    """(theta, phi) of RING pixels (Gorski et al. 2005 closed forms)."""
    pix = np.atleast_1d(np.asarray(pix, dtype=np.int64))
    th = np.empty(pix.shape)
    ph = np.empty(pix.shape)
    a, b = ctypes.c_double(), ctypes.c_double()
    for k, p in enumerate(pix.ravel()):
        _lib().orc_pix2ang(nside, int(p), ctypes.byref(a), ctypes.byref(b))
        th.flat[k], ph.flat[k] = a.value, b.value
    return th, ph


def ang2pix(nside: int, theta, phi) -> np.ndarray:
    """RING pixels containing the directions (theta, phi) (Gorski et al. 2005, Sec. 4)."""
    th, ph = _f64(theta).ravel(), _f64(phi).ravel()
    if th.shape != ph.shape:
        raise ValueError("theta and phi differ in length")
    out = np.empty(th.size, dtype=np.int64)
    _lib().orc_ang2pix(nside, th.size, _dp(th), _dp(ph), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def healpix_interp(nside: int, m, theta, phi) -> np.ndarray:
    """A RING map read at (theta, phi) by bilinear interpolation on the sphere
    (two bracketing rings, two bracketing pixels on each; poles = mean of the
    first / last ring)."""
    m = _f64(m)
    if m.size != 12 * nside * nside:
        raise ValueError("map size does not match nside")
    th, ph = np.broadcast_arrays(_f64(theta), _f64(phi))
    out = np.empty(th.shape)
    for k, (a, b) in enumerate(zip(th.ravel(), ph.ravel())):
        out.flat[k] = _lib().orc_healpix_interp(nside, _dp(m), float(a), float(b))
    return out


def healpix_to_grid(nside: int, m, half_span_tan: float, n: int) -> np.ndarray:
    """(n, n) gnomonic grid ([v][u] over [-T, T]^2) read from a map whose north
    pole is the boresight (theta = rho, phi = sigma)."""
    m = _f64(m)
    if m.size != 12 * nside * nside:
        raise ValueError("map size does not match nside")
    out = np.empty((n, n))
    _lib().orc_healpix_to_grid(nside, _dp(m), float(half_span_tan), int(n), _dp(out))
    return out


def pix2zphi(nside: int, pix):
    pix = np.atleast_1d(np.asarray(pix, dtype=np.int64))
    z = np.empty(pix.shape)
    s = np.empty(pix.shape)
    ph = np.empty(pix.shape)
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    for k, p in enumerate(pix.ravel()):
        _lib().orc_pix2zphi(nside, int(p), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        z.flat[k], s.flat[k], ph.flat[k] = a.value, b.value, c.value
    return z, s, ph


def ring(nside: int, i: int):
    """(theta, count, first pixel) of ring i = 1..4N-1."""
    th = ctypes.c_double()
    cnt, first = ctypes.c_int64(), ctypes.c_int64()
    _lib().orc_ring(nside, i, ctypes.byref(th), ctypes.byref(cnt), ctypes.byref(first))
    return th.value, cnt.value, first.value


def appA(theta0, phi0, psi0, zeta, theta, phi):
    """Appendix A: (rho, sigma, chi) of direction (theta, phi) for pointing (theta0, phi0, psi0)."""
    r, s, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _lib().orc_appA(theta0, phi0, psi0, zeta, theta, phi, ctypes.byref(r), ctypes.byref(s), ctypes.byref(c))
    return r.value, s.value, c.value


def disc(nside: int, theta0: float, phi0: float, rho: float) -> np.ndarray:
    """Ascending RING indices of pixels with centres within rho (inclusive)."""
    n = _lib().orc_disc(nside, theta0, phi0, rho, None, 0)
    out = np.empty(n, dtype=np.int64)
    _lib().orc_disc(nside, theta0, phi0, rho, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n)
    return out


def disc_counts(nside: int, theta, phi, rho: float, nthreads: int = 0) -> np.ndarray:
    th, ph = _f64(theta), _f64(phi)
    out = np.empty(th.size, dtype=np.int64)
    _lib().orc_disc_counts(nside, th.size, _dp(th), _dp(ph), rho,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nthreads)
    return out


def tod(nside: int, I, Q, U, beamsor, half_span_tan: float, zeta: float, eps: float, s: float,
        rho_min: float, rho_max: float, norm_mode: int, norm_scale: float,
        theta, phi, psi, out_mode: int = OUT_TOD, nthreads: int = 0, V=None, hwp=None) -> np.ndarray:
    """FP64 convolution of one detector's stream.

    beamsor : (n, n, 4, 4) Mueller field M[iv, iu, out, in] over u, v in [-T, T]
    V       : optional V map (zero when None)
    hwp     : optional per-sample half-wave-plate angle (radians); the beamsor
              of sample t becomes M . H(hwp[t])
    returns (nsamp,) for OUT_TOD or (nsamp, 3) for OUT_STOKES.
    """
    I, Q, U = _f64(I), _f64(Q), _f64(U)
    Vv = None if V is None else _f64(V)
    g = _f64(beamsor)
    n = g.shape[0]
    if g.shape != (n, n, 4, 4):
        raise ValueError("beamsor must be (n, n, 4, 4)")
    th, ph, ps = _f64(theta), _f64(phi), _f64(psi)
    m = th.size
    hw = None if hwp is None else _f64(hwp)
    if hw is not None and hw.size != m:
        raise ValueError("hwp must have one angle per sample")
    if Vv is not None and Vv.size != I.size:
        raise ValueError("V must match I")
    width = 3 if out_mode == OUT_STOKES else 1
    out = np.empty(m * width)
    null = ctypes.POINTER(ctypes.c_double)()
    rc = _lib().orc_tod_iquv(nside, _dp(I), _dp(Q), _dp(U), null if Vv is None else _dp(Vv), n, half_span_tan,
                             _dp(g), zeta, eps, s, rho_min, rho_max, norm_mode, norm_scale, m, _dp(th), _dp(ph),
                             _dp(ps), null if hw is None else _dp(hw), out_mode, _dp(out), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out.reshape(m, 3) if width == 3 else out


def tod_detector(nside: int, sky, d, out_mode: int = OUT_TOD, idx=None, nthreads: int = 0) -> np.ndarray:
    """Convenience: run a ``synth.workloads.Detector`` (optionally a subset of samples)."""
    sel = slice(None) if idx is None else idx
    return tod(nside, sky[0], sky[1], sky[2], d.beam.dense(), d.beam.half_span_tan, d.det.zeta, d.det.eps,
               d.det.s, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale,
               d.theta[sel], d.phi[sel], d.psi[sel], out_mode, nthreads)
