"""Binned map-making on the GPU (pisco_map_accumulate / pisco_map_solve)
against the oracle's binned estimator: per-pixel sums (hits exactly), rcond
and maps, for FP32 and FP64 TOD, several detectors and a half-wave plate; the
paper's whole-sky pattern (every pixel centre at psi = 0, 45, 90 deg) through
the GPU convolution; non-finite samples; argument errors; and eight detectors
of the nside-1024 benchmark workload binned at nside 1024."""
import numpy as np
import pytest

import oracle
from oracle import maps as OM
from synth import beams as B
from synth import workloads as W

from gpu_helpers import cached_workload, load_workload, rel_err, say

pytestmark = pytest.mark.gpu
D2R = np.pi / 180


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture()
def conv(torch):
    from paper_1908_05662_amd.api import Convolver

    c = Convolver(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _oracle_sums(nside, dets):
    npix = 12 * nside * nside
    ata, atd, hits = np.zeros((npix, 3, 3)), np.zeros((npix, 3)), np.zeros(npix)
    for th, ph, ps, d, zeta, eps, s, hw in dets:
        x = OM.bin_tod(nside, th, ph, ps, d, zeta, eps, s, hw)
        ata += x[0]
        atd += x[1]
        hits += x[2]
    return ata, atd, hits


def _gpu_sums(mm):
    a = mm.accum.view(mm.npix, 10).cpu().numpy()
    ata = np.empty((mm.npix, 3, 3))
    for k, (i, j) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        ata[:, i, j] = ata[:, j, i] = a[:, k]
    return ata, a[:, 6:9], a[:, 9]


def _random_dets(rng, nside, n, tod_dtype):
    out = []
    for zeta, eps, s, plate in [(0.0, 0.01, 1.0, False), (-np.pi / 2, 0.02, 0.9, False), (0.7, 0.0, 1.1, True)]:
        th, ph = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(-7, 7, n)
        ps = rng.uniform(0, 2 * np.pi, n)
        d = rng.standard_normal(n).astype(tod_dtype).astype(np.float64)
        hw = rng.uniform(0, np.pi, n) if plate else None
        out.append((th, ph, ps, d, zeta, eps, s, hw))
    return out


@pytest.mark.parametrize("tod_dtype", [np.float64, np.float32])
def test_map_parity_random_pointing(conv, torch, tod_dtype):
    from paper_1908_05662_amd.api import MapMaker

    say(f"case: binned maps vs oracle, nside 16, 3 detectors (one with a plate), TOD {np.dtype(tod_dtype).name}")
    nside = 16
    rng = np.random.default_rng(11)
    dets = _random_dets(rng, nside, 30_000, tod_dtype)
    mm = MapMaker(conv, nside)
    for th, ph, ps, d, zeta, eps, s, hw in dets:
        mm.add(th, ph, ps, torch.from_numpy(d.astype(tod_dtype)).cuda(), zeta, eps, s, hw)
    maps, rc = mm.solve(1e-6)
    ata, atd, hits = _oracle_sums(nside, dets)
    g_ata, g_atd, g_hits = _gpu_sums(mm)
    assert np.array_equal(g_hits, hits)                       # the same pixel for every sample
    assert rel_err(g_ata.reshape(-1), ata.reshape(-1)) <= 1e-13
    assert rel_err(g_atd.reshape(-1), atd.reshape(-1)) <= 1e-13
    I, Q, U, orc = OM.solve(ata, atd, hits, 1e-6)
    got = maps.cpu().numpy()
    ok = orc >= 1e-6
    assert ok.mean() > 0.9
    assert np.array_equal(rc.cpu().numpy() >= 1e-6, ok)
    assert np.abs(rc.cpu().numpy() - orc).max() <= 1e-12
    for k, want in enumerate((I, Q, U)):
        e = rel_err(got[k], want)
        say(f"  map {'IQU'[k]}: max rel err {e:.3e}")
        assert e <= 1e-10


def test_paper_pattern_through_the_convolution(conv, torch):
    """Every nside-16 pixel centre at psi = 0, 45, 90 deg; an unpolarised sky
    seen through a beam flat over a 10 deg disc (FP64): the GPU TOD binned on
    the GPU give Q = U = 0 to rounding, and the maps equal the oracle's maps of
    the same TOD; a polarised sky comes back through the same chain as the
    oracle's chain does."""
    from paper_1908_05662_amd.api import MapMaker
    from synth.sky import make_sky
    from synth.workloads import Detector, Workload

    say("case: paper pattern, nside 16, flat beam, I-only and polarised skies")
    nside = 16
    npix = 12 * nside * nside
    th, ph = oracle.pix2ang(nside, np.arange(npix))
    th3, ph3 = np.tile(th, 3), np.tile(ph, 3)
    psi = np.repeat(np.deg2rad([0.0, 45.0, 90.0]), npix)
    Tn, u, v, rho, sig = B.tangent_grid(61, 12 * D2R)
    bs = B.ideal_beamsor(np.ones_like(rho), Tn)
    I, Q, U = make_sky(nside, 3 * nside - 1, 2.0, seed=8)
    for pol in (False, True):
        sky = (I, Q if pol else 0 * Q, U if pol else 0 * U)
        det = Detector(bs, B.DetectorParams(0.0, 0.0, 1.0), 0.0, 10 * D2R, W.NORM_PER_SAMPLE, 1.0, th3, ph3, psi)
        w = Workload("pattern", nside, sky, [det])
        load_workload(conv, w, np.float64)
        tod = conv.convolve(0)
        mm = MapMaker(conv, nside)
        mm.add(th3, ph3, psi, tod, 0.0, 0.0, 1.0)
        maps, rc = mm.solve()
        got = maps.cpu().numpy()
        want = OM.solve(*OM.bin_tod(nside, th3, ph3, psi, tod.cpu().numpy(), 0.0, 0.0, 1.0))
        for k in range(3):
            assert np.abs(got[k] - want[k]).max() <= 1e-11 * np.abs(want[0]).max()
        if not pol:
            top = np.abs(got[0]).max()
            assert np.abs(got[1]).max() <= 1e-12 * top and np.abs(got[2]).max() <= 1e-12 * top


def test_nonfinite_samples_are_skipped_and_errors(conv, torch):
    from paper_1908_05662_amd import PiscoError
    from paper_1908_05662_amd.api import MapMaker

    say("case: non-finite samples, empty calls, argument errors")
    nside = 8
    rng = np.random.default_rng(12)
    n = 5000
    th, ph, ps = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 7, n), rng.uniform(0, 7, n)
    d = rng.standard_normal(n)
    a = MapMaker(conv, nside).add(th, ph, ps, d, 0.2, 0.0, 1.0)
    th2, d2, ps2 = th.copy(), d.copy(), ps.copy()
    th2[::7] = np.nan
    d2[3::11] = np.inf
    ps2[5::13] = -np.inf
    b = MapMaker(conv, nside).add(th2, ph, ps2, d2, 0.2, 0.0, 1.0)
    keep = np.isfinite(th2) & np.isfinite(d2) & np.isfinite(ps2)
    c = MapMaker(conv, nside).add(th[keep], ph[keep], ps[keep], d[keep], 0.2, 0.0, 1.0)
    assert rel_err(b.accum.cpu().numpy(), c.accum.cpu().numpy()) <= 1e-13
    assert not np.array_equal(a.accum.cpu().numpy(), b.accum.cpu().numpy())
    e = MapMaker(conv, nside).add(th[:0], ph[:0], ps[:0], d[:0])
    assert not e.accum.any().item()
    lib = conv._lib
    assert lib.pisco_map_solve(conv._h, 3, a.accum.data_ptr(), 1e-6, a.accum.data_ptr(), None, None) != 0
    assert lib.pisco_map_solve(conv._h, nside, a.accum.data_ptr(), 2.0, a.accum.data_ptr(), None, None) != 0
    assert lib.pisco_map_solve(conv._h, nside, None, 1e-6, a.accum.data_ptr(), None, None) != 0
    with pytest.raises(PiscoError):
        conv._check(lib.pisco_map_accumulate(conv._h, 16, 10, None, None, None, None, None, 0, 0.0, 0.0, 1.0,
                                             a.accum.data_ptr(), None))
    with pytest.raises(PiscoError):
        MapMaker(conv, nside).add(th, ph, ps, d, 0.2, float("nan"), 1.0)


def test_runs_of_equal_pixels_with_gaps(conv, torch):
    """Samples in runs of 1 to 20 equal directions (runs cross wave
    boundaries), some of them non-finite: the wave-level run sums give the
    oracle's per-pixel sums (hits exactly)."""
    from paper_1908_05662_amd.api import MapMaker

    say("case: runs of equal pixels with non-finite samples inside")
    nside = 32
    rng = np.random.default_rng(13)
    reps = rng.integers(1, 21, 4000)
    th = np.repeat(np.arccos(rng.uniform(-1, 1, reps.size)), reps)
    ph = np.repeat(rng.uniform(0, 2 * np.pi, reps.size), reps)
    n = th.size
    ps = rng.uniform(0, 2 * np.pi, n)
    d = rng.standard_normal(n)
    d[rng.uniform(size=n) < 0.05] = np.nan
    th[rng.uniform(size=n) < 0.02] = np.inf
    keep = np.isfinite(th) & np.isfinite(d)
    mm = MapMaker(conv, nside).add(th, ph, ps, d, 0.4, 0.01, 1.2)
    ata, atd, hits = _oracle_sums(nside, [(th[keep], ph[keep], ps[keep], d[keep], 0.4, 0.01, 1.2, None)])
    g_ata, g_atd, g_hits = _gpu_sums(mm)
    assert np.array_equal(g_hits, hits)
    assert rel_err(g_ata.reshape(-1), ata.reshape(-1)) <= 1e-13
    assert rel_err(g_atd.reshape(-1), atd.reshape(-1)) <= 1e-13


def test_benchmark_detectors_binned_at_nside_1024(conv, torch):
    """Eight detectors of the nside-1024 benchmark workload (their GPU TOD),
    binned at nside 1024: every pixel's sums and maps against the oracle."""
    from paper_1908_05662_amd.api import MapMaker

    say("case: 8 detectors of the nside-1024 workload binned at nside 1024")
    import copy

    w = copy.copy(cached_workload("c3"))
    w.detectors = w.detectors[:8]
    load_workload(conv, w, np.float32)
    tod = conv.convolve(-1).cpu().numpy()
    mm = MapMaker(conv, 1024)
    off = 0
    dets = []
    for d in w.detectors:
        t = tod[off:off + d.n]
        mm.add(d.theta, d.phi, d.psi, torch.from_numpy(t).cuda(), d.det.zeta, d.det.eps, d.det.s)
        dets.append((d.theta, d.phi, d.psi, t.astype(np.float64), d.det.zeta, d.det.eps, d.det.s, None))
        off += d.n
    maps, rc = mm.solve(1e-3)
    ata, atd, hits = _oracle_sums(1024, dets)
    g_ata, g_atd, g_hits = _gpu_sums(mm)
    say(f"  {int((hits > 0).sum())} pixels hit by {off} samples")
    assert np.array_equal(g_hits, hits)
    assert rel_err(g_atd.reshape(-1), atd.reshape(-1)) <= 1e-12
    I, Q, U, orc = OM.solve(ata, atd, hits, 1e-3)
    got = maps.cpu().numpy()
    agree = (rc.cpu().numpy() >= 1e-3) == (orc >= 1e-3)
    assert agree.mean() > 0.9999
    for k, want in enumerate((I, Q, U)):
        e = np.abs(got[k][agree] - want[agree]).max() / np.abs(want[agree]).max()
        say(f"  map {'IQU'[k]}: max rel err {e:.3e}")
        assert e <= 1e-9


@pytest.mark.parametrize("stokes", [0, 1, 2])
def test_point_source_flux_preserved(conv, torch, stokes):
    """The paper's point-source validation (Sec. 6): one non-zero pixel (I, Q
    or U) at 45 deg declination on an nside-256 sky, a 1.5 deg Gaussian beam
    given as an nside-1024 HEALPix map (4:1), every map pixel within 6 deg of
    the source observed at its centre at psi = 0, 45, 90 deg; GPU TOD binned on
    the GPU.  The source's flux in its own Stokes map is preserved to 0.2% (the
    figure the paper reports) and the other two maps stay below 0.2% of it."""
    from paper_1908_05662_amd.api import MapMaker

    say(f"case: point source, Stokes {'IQU'[stokes]}, sky nside 256, beam map nside 1024")
    nside, nsb = 256, 1024
    npix = 12 * nside * nside
    src = int(oracle.ang2pix(nside, np.array([np.pi / 4]), np.array([1.0]))[0])
    sky = [np.zeros(npix) for _ in range(3)]
    sky[stokes][src] = 1.0
    ths, phs = oracle.pix2ang(nside, np.array([src]))
    th, ph = oracle.pix2ang(nside, np.arange(npix))
    near = np.arccos(np.clip(np.cos(th) * np.cos(ths) + np.sin(th) * np.sin(ths) * np.cos(ph - phs), -1, 1)) < 6 * D2R
    pix = np.nonzero(near)[0]
    th3, ph3 = np.tile(th[pix], 3), np.tile(ph[pix], 3)
    psi = np.repeat(np.deg2rad([0.0, 45.0, 90.0]), pix.size)
    bmap = B.healpix_beam_map(nsb, 1.5 * D2R, rho_max_rad=7 * D2R)
    conv.set_sky(nside, *(torch.from_numpy(m).cuda() for m in sky), dtype=torch.float64)
    conv.set_beam_healpix_scalar(0, nsb, 201, np.tan(5 * D2R), bmap, 0.5, 0.5, 0.0, 1.0, dtype=torch.float64)
    conv.set_detector(0, 0.0, 0.0, 5 * D2R, W.NORM_PER_SAMPLE, 1.0)
    conv.set_pointing(0, *(torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (th3, ph3, psi)))
    tod = conv.convolve(0)
    mm = MapMaker(conv, nside).add(th3, ph3, psi, tod, 0.0, 0.0, 1.0)
    maps, rc = mm.solve()
    m = maps.cpu().numpy()[:, pix]
    flux = m.sum(axis=1)
    say(f"  flux I, Q, U: {flux[0]:.6f} {flux[1]:.6f} {flux[2]:.6f}")
    assert abs(flux[stokes] - 1.0) < 2e-3
    for k in range(3):
        if k != stokes:
            assert abs(flux[k]) < 2e-3
