"""Seeded synthetic workloads shaped like the paper's and the benchmark recipes.

Every workload is fully determined by its name and seed.  Arrays are
float64 on the host; callers cast to the precision they run in.

  c1  nside 64 sky, C_l=(l+1)^-2, l<=191; 101^2 grid over +-4.5 deg, Gaussian
      FWHM 1.5 deg with 1% Q<->U leakage; RA sweep, Dec ~ U[-60,60] deg,
      psi ~ U[0,2pi); 1e5 samples; disc 4.5 deg; FP64.
  c2  nside 512 sky, l<=1535; 201^2 grid over +-2 deg, elliptical Gaussian
      FWHM 0.5 deg, e = 5%; CES at 45 deg elevation, 0.01 deg/sample;
      1e7 samples; disc 2 deg.
  c3  nside 1024 sky, l<=3071; 64 detectors (32 pairs at zeta, zeta-90,
      zeta alternating 0/45 deg) on a 0.7 deg-pitch hexagonal focal plane;
      each its own 201^2 elliptical beam (FWHM U[0.4,0.6], e U[0,0.1],
      orientation U[0,pi)), eps = 1e-3; n_d ~ U[1e5,1e6] samples from a random
      start of a CES scan with boresight steps of 15 deg; disc 2 deg.
  c4  nside 256 sky, C_l=(l+1)^-3, l<=767; 401^2 grid over +-20 deg, Gaussian
      FWHM 1 deg + 1e-4 ring at 10 deg (FWHM 2 deg); disc 20 deg, main disc
      5 deg; isotropic pointings (train and held-out streams seeded apart).
  c5  nside 2048 sky, l<=4095; 256 detectors, elliptical FWHM 0.25 deg on a
      151^2 grid over +-1.5 deg (main disc 1.5 deg) plus a shared 401^2 ring
      grid over +-20 deg; CES with boresight rotation, 390625 samples each.
  P   the paper's benchmark shape: nside 128 sky, every pixel centre at
      psi in {0, 45, 90} deg for a pair at zeta {0, -90} deg; Gaussian FWHM
      1.5 deg on a grid of ~0.1 deg spacing over +-rho_max.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

from . import beams as B
from . import scans as S
from .sky import make_sky

SEED_BASE = 1908056620
NORM_FIXED = 0
NORM_PER_SAMPLE = 1


@dataclass
class Detector:
    beam: B.Beamsor
    det: B.DetectorParams
    rho_min: float
    rho_max: float
    norm_mode: int
    norm_scale: float
    theta: np.ndarray
    phi: np.ndarray
    psi: np.ndarray

    @property
    def n(self) -> int:
        return int(self.theta.size)


@dataclass
class Workload:
    name: str
    nside: int
    sky: tuple            # (I, Q, U) float64 RING maps
    detectors: list = field(default_factory=list)
    meta: dict = field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return sum(d.n for d in self.detectors)


def _rng(idx: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([SEED_BASE + idx, stream]))


def _deg(x):
    return np.deg2rad(x)


def _per_detector(make, n_det: int) -> list:
    """[make(k) for k in range(n_det)] on a thread pool: every detector is built
    from its own index alone, so the arrays equal a plain loop's (numpy releases
    the interpreter lock in its array kernels)."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(make, range(n_det)))


def sky_for(nside: int, lmax: int, power: float, idx: int):
    return tuple(make_sky(nside, lmax, power, seed=SEED_BASE + idx))


def c1(n_samples: int = 100_000, sky=None) -> Workload:
    rng = _rng(1, 1)
    nside, lmax = 64, 191
    sky = sky if sky is not None else sky_for(nside, lmax, 2.0, 1)
    T, u, v, rho, sig = B.tangent_grid(101, _deg(4.5))
    g = B.elliptical_gaussian(rho, sig, _deg(1.5))
    bs = B.with_qu_leakage(B.ideal_beamsor(g, T), g, 0.01)
    th, ph, ps = S.radec_sweep(n_samples, rng)
    d = Detector(bs, B.DetectorParams(0.0, 0.0, 1.0), 0.0, _deg(4.5), NORM_PER_SAMPLE, 1.0, th, ph, ps)
    return Workload("c1", nside, sky, [d], {"precision": "f64", "lmax": lmax})


def c2(n_samples: int = 10_000_000, sky=None) -> Workload:
    rng = _rng(2, 1)
    nside, lmax = 512, 1535
    sky = sky if sky is not None else sky_for(nside, lmax, 2.0, 2)
    T, u, v, rho, sig = B.tangent_grid(201, _deg(2.0))
    g = B.elliptical_gaussian(rho, sig, _deg(0.5), 0.05, rng.uniform(0, np.pi))
    lat = _deg(rng.uniform(-45.0, 45.0))
    th, ph, ps = S.ces(n_samples, lat, lst0=rng.uniform(0, 2 * np.pi))
    d = Detector(B.ideal_beamsor(g, T), B.DetectorParams(0.0, 0.0, 1.0), 0.0, _deg(2.0),
                 NORM_PER_SAMPLE, 1.0, th, ph, ps)
    return Workload("c2", nside, sky, [d], {"precision": "f32", "lmax": lmax, "lat": lat})


def c3(count_scale: float = 1.0, n_det: int = 64, sky=None, max_per_det=None) -> Workload:
    """``count_scale`` shrinks every detector's sample count (parity subsets)."""
    rng = _rng(3, 1)
    nside, lmax = 1024, 3071
    sky = sky if sky is not None else sky_for(nside, lmax, 2.0, 3)
    lat = _deg(rng.uniform(-45.0, 45.0))
    lst0 = rng.uniform(0, 2 * np.pi)
    counts = rng.integers(100_000, 1_000_001, size=64)
    starts = rng.integers(0, 2_000_000, size=64)
    fwhm = rng.uniform(0.4, 0.6, size=64)
    ell = rng.uniform(0.0, 0.1, size=64)
    orient = rng.uniform(0.0, np.pi, size=64)
    sites = S.hex_focal_plane(32, _deg(0.7))
    T, u, v, rho, sig = B.tangent_grid(201, _deg(2.0))
    def one(k):
        pair = k // 2
        zeta = _deg(0.0 if pair % 2 == 0 else 45.0) - (_deg(90.0) if k % 2 else 0.0)
        n = max(1, int(round(counts[k] * count_scale)))
        if max_per_det is not None:
            n = min(n, int(max_per_det))
        th, ph, ps = S.ces(n, lat, start=int(starts[k]), boresight_deg=np.arange(-45, 46, 15), lst0=lst0)
        dx, dy = sites[pair]
        th, ph, ps = S.offset_pointing(th, ph, ps, dx, dy)
        g = B.elliptical_gaussian(rho, sig, _deg(fwhm[k]), ell[k], orient[k])
        return Detector(B.ideal_beamsor(g, T), B.DetectorParams(zeta, 1e-3, 1.0), 0.0, _deg(2.0),
                        NORM_PER_SAMPLE, 1.0, th, ph, ps)

    dets = _per_detector(one, n_det)
    return Workload("c3", nside, sky, dets, {"precision": "f32", "lmax": lmax, "lat": lat})


def sidelobe_beam(n: int, half_span_deg: float, main_fwhm_deg: float, ellipticity: float = 0.0,
                  orient: float = 0.0, ring: bool = True):
    T, u, v, rho, sig = B.tangent_grid(n, _deg(half_span_deg))
    g = B.elliptical_gaussian(rho, sig, _deg(main_fwhm_deg), ellipticity, orient)
    if ring:
        g = g + B.ring_lobe(rho, _deg(10.0), _deg(2.0), 1e-4)
    return T, g


def analytic_solid_angle(main_fwhm_deg: float, ring: bool = True) -> float:
    """Small-angle solid angle of the fixture beam (an input constant for FIXED normalisation)."""
    s0 = _deg(main_fwhm_deg) * B.FWHM_TO_SIGMA
    om = 2.0 * np.pi * s0 * s0
    if ring:
        w = _deg(2.0) * B.FWHM_TO_SIGMA
        om += 1e-4 * 2.0 * np.pi * np.sin(_deg(10.0)) * w * np.sqrt(2.0 * np.pi)
    return om


def c4(n_samples: int = 1_000_000, stream: int = 1, sky=None) -> Workload:
    """stream 1 = training pointings, stream 2 = held-out pointings."""
    rng = _rng(4, stream)
    nside, lmax = 256, 767
    sky = sky if sky is not None else sky_for(nside, lmax, 3.0, 4)
    T, g = sidelobe_beam(401, 20.0, 1.0)
    th, ph, ps = S.uniform_sphere(n_samples, rng)
    dOm = 4.0 * np.pi / (12 * nside * nside)
    norm = dOm / analytic_solid_angle(1.0)
    d = Detector(B.ideal_beamsor(g, T), B.DetectorParams(0.0, 0.0, 1.0), 0.0, _deg(20.0), NORM_FIXED, norm, th, ph, ps)
    return Workload("c4", nside, sky, [d], {"precision": "f32", "lmax": lmax, "r_main": _deg(5.0)})


def c5(n_det: int = 256, per_det: int = 390_625, sky=None) -> Workload:
    rng = _rng(5, 1)
    nside, lmax = 2048, 4095
    sky = sky if sky is not None else sky_for(nside, lmax, 2.0, 5)
    lat = _deg(rng.uniform(-45.0, 45.0))
    lst0 = rng.uniform(0, 2 * np.pi)
    starts = rng.integers(0, 4_000_000, size=256)
    ell = rng.uniform(0.0, 0.1, size=256)
    orient = rng.uniform(0.0, np.pi, size=256)
    sites = S.hex_focal_plane(128, _deg(0.35))
    T, u, v, rho, sig = B.tangent_grid(151, _deg(1.5))
    dOm = 4.0 * np.pi / (12 * nside * nside)
    norm = dOm / analytic_solid_angle(0.25)
    def one(k):
        pair = k // 2
        zeta = _deg(0.0 if pair % 2 == 0 else 45.0) - (_deg(90.0) if k % 2 else 0.0)
        th, ph, ps = S.ces(per_det, lat, start=int(starts[k]), boresight_deg=np.arange(-45, 46, 15), lst0=lst0)
        dx, dy = sites[pair]
        th, ph, ps = S.offset_pointing(th, ph, ps, dx, dy)
        g = B.elliptical_gaussian(rho, sig, _deg(0.25), ell[k], orient[k])
        return Detector(B.ideal_beamsor(g, T), B.DetectorParams(zeta, 0.0, 1.0), 0.0, _deg(1.5),
                        NORM_FIXED, norm, th, ph, ps)

    dets = _per_detector(one, n_det)
    return Workload("c5", nside, sky, dets, {"precision": "f32", "lmax": lmax, "lat": lat,
                                              "ring_grid": (401, 20.0), "r_main": _deg(1.5)})


def paper_shape(rho_max_deg: float = 5.0, nside: int = 128, sky=None, spacing_deg: float = 0.1) -> Workload:
    nside = int(nside)
    lmax = 3 * nside - 1
    sky = sky if sky is not None else sky_for(nside, lmax, 2.0, 6)
    n = 2 * int(np.ceil(rho_max_deg / spacing_deg)) + 1
    T, u, v, rho, sig = B.tangent_grid(n, _deg(rho_max_deg))
    g = B.elliptical_gaussian(rho, sig, _deg(1.5))
    th, ph, ps = S.pixel_centre_scan(nside)
    dets = []
    for zeta in (0.0, -90.0):
        dets.append(Detector(B.ideal_beamsor(g, T), B.DetectorParams(_deg(zeta), 0.0, 1.0), 0.0, _deg(rho_max_deg),
                             NORM_PER_SAMPLE, 1.0, th, ph, ps))
    return Workload("P", nside, sky, dets, {"precision": "f32", "lmax": lmax})
