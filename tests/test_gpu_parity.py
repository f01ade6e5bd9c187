"""GPU parity of the HIP convolution against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle
from synth import beams as B
from synth import scans as S
from synth import workloads as W
from synth.workloads import Detector, Workload

from gpu_helpers import load_workload, oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu
D2R = np.pi / 180
F64_TOL = 1e-12
F32_TOL = 1e-6


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


ALGOS = [0, 1, 2]       # pixel-parallel, sample-parallel tile path, tile path on the matrix cores
BEAMS = ["full", "auto"]  # four-channel grid, one-grid (scalar) form


def test_c1_fp64_full_stream(conv, torch):
    """nside-64 FP64 workload at full size: 1e5 samples, FP64 kernel, every sample vs the oracle."""
    say("case: c1 fp64 1e5 samples")
    w = W.c1()
    load_workload(conv, w, np.float64)
    got = conv.convolve(0).cpu().numpy()
    want = oracle_detector(w, 0, slice(None), np.float64)
    e = rel_err(got, want)
    say(f"c1 fp64 max rel err {e:.3e}")
    assert e <= F64_TOL


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("beam", BEAMS)
def test_c1_fp32_mixed(conv, torch, algo, beam):
    say(f"case: c1 fp32 2e4 samples algo {algo} beam {beam}")
    w = W.c1(n_samples=20000)
    conv.set_launch(algorithm=algo)
    load_workload(conv, w, np.float32, beam=beam)
    got = conv.convolve(0).cpu().numpy()
    want = oracle_detector(w, 0, slice(None), np.float32)
    e = rel_err(got, want)
    say(f"c1 fp32 max rel err {e:.3e}")
    assert e <= F32_TOL


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("beam", BEAMS)
def test_c2_fp32_sampled(conv, torch, algo, beam):
    """Precision workload shape (nside 512, 201^2 elliptical beam, CES) on 2e5 samples;
    the oracle checks an evenly spread subset."""
    say(f"case: c2 fp32 2e5 samples, 1500 checked, algo {algo} beam {beam}")
    w = W.c2(n_samples=200_000)
    conv.set_launch(algorithm=algo)
    load_workload(conv, w, np.float32, beam=beam)
    got = conv.convolve(0).cpu().numpy()
    idx = np.linspace(0, w.detectors[0].n - 1, 1500).astype(np.int64)
    want = oracle_detector(w, 0, idx, np.float32)
    e = rel_err(got[idx], want)
    say(f"c2 fp32 max rel err {e:.3e}")
    assert e <= F32_TOL


def _small_workload(nside, dets, seed=0):
    from synth.sky import make_sky

    sky = tuple(make_sky(nside, 3 * nside - 1, 2.0, seed=seed))
    return Workload("edge", nside, sky, dets)


def _det(bs, th, ph, ps, zeta=0.3, eps=0.02, s=1.1, rmin=0.0, rmax=0.1, norm=W.NORM_PER_SAMPLE, scale=1.0):
    return Detector(bs, B.DetectorParams(zeta, eps, s), rmin, rmax, norm, scale, np.asarray(th, float),
                    np.asarray(ph, float), np.asarray(ps, float))


def _gauss(n, span_deg, fwhm_deg, e=0.1, o=0.5, leak=0.01):
    T, u, v, rho, sig = B.tangent_grid(n, span_deg * D2R)
    g = B.elliptical_gaussian(rho, sig, fwhm_deg * D2R, e, o)
    return B.with_qu_leakage(B.ideal_beamsor(g, T), g, leak)


@pytest.mark.parametrize("dtype,tol,algo", [(np.float64, F64_TOL, 0), (np.float32, F32_TOL, 0),
                                            (np.float32, F32_TOL, 1), (np.float32, F32_TOL, 2)])
def test_edge_geometry(conv, torch, dtype, tol, algo):
    """Poles inside the disc, boresight exactly on a pole, longitude wrap-around,
    negative / >2pi longitudes, full rings, coarse maps with wide discs."""
    say(f"case: edge geometry {np.dtype(dtype).name} algo {algo}")
    conv.set_launch(algorithm=algo)
    rng = np.random.default_rng(4)
    th = np.concatenate([[0.0, np.pi, 1e-9, np.pi - 1e-9, 0.05, np.pi - 0.05, 1.0, 2.0],
                         np.arccos(rng.uniform(-1, 1, 24))])
    ph = np.concatenate([[0.0, 1.0, 2 * np.pi - 1e-12, -0.3, 7.0, -12.0, 2 * np.pi, 1e-13],
                         rng.uniform(-10, 10, 24)])
    ps = rng.uniform(-7, 7, th.size)
    for nside, span, fwhm, rmax in [(1, 60.0, 40.0, 59.0), (2, 50.0, 30.0, 50.0), (8, 20.0, 8.0, 20.0),
                                    (32, 10.0, 3.0, 10.0)]:
        bs = _gauss(81, span, fwhm)
        w = _small_workload(nside, [_det(bs, th, ph, ps, rmax=rmax * D2R)], seed=nside)
        load_workload(conv, w, dtype)
        got = conv.convolve(0).cpu().numpy()
        want = oracle_detector(w, 0, slice(None), dtype)
        e = rel_err(got, want)
        say(f"  nside {nside}: max rel err {e:.3e}")
        assert e <= tol, (nside, e)


def _pole_crossing_scan(n):
    """Slow scans that pass over both poles and across phi = 0: consecutive
    samples overlap (tile path) while the discs contain a pole or wrap."""
    s = np.linspace(-1, 1, n // 2)
    th1, ph1 = np.abs(0.3 * s) + 1e-12, np.where(s < 0, 0.7, 0.7 + np.pi)
    th2, ph2 = np.pi - np.abs(0.3 * s), np.where(s < 0, 2 * np.pi - 1e-9, np.pi - 1e-9)
    th = np.concatenate([th1, th2])
    ph = np.concatenate([ph1, ph2])
    ps = np.linspace(0, 3, th.size)
    return th, ph, ps


@pytest.mark.parametrize("dtype,tol,algo,scan", [(np.float64, F64_TOL, 0, "random"), (np.float32, F32_TOL, 0, "random"),
                                                 (np.float32, F32_TOL, 1, "random"), (np.float32, F32_TOL, 1, "poles"),
                                                 (np.float32, F32_TOL, 2, "random"), (np.float32, F32_TOL, 2, "poles"),
                                                 (np.float64, F64_TOL, 0, "poles")])
def test_annulus_stokes_fixed(conv, torch, dtype, tol, algo, scan):
    """Annulus selection, the Stokes-pickup output and FIXED normalisation; the
    disc = inner disc + annulus partition holds on the GPU too."""
    say(f"case: annulus/stokes {np.dtype(dtype).name} algo {algo} scan {scan}")
    conv.set_launch(algorithm=algo)
    rng = np.random.default_rng(5)
    n = 200
    th, ph, ps = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 2 * np.pi, n), rng.uniform(0, 2 * np.pi, n)
    th[:3] = [0.0, 0.02, np.pi]
    if scan == "poles":
        th, ph, ps = _pole_crossing_scan(256)
    T, u, v, rho, sig = B.tangent_grid(161, 20 * D2R)
    g = B.elliptical_gaussian(rho, sig, 2 * D2R) + B.ring_lobe(rho, 10 * D2R, 2 * D2R, 1e-2)
    bs = B.ideal_beamsor(g, T)
    nside = 32
    dets = [_det(bs, th, ph, ps, zeta=0.0, eps=0.0, s=1.0, rmin=r0, rmax=r1, norm=W.NORM_FIXED, scale=1e-3)
            for r0, r1 in [(0.0, 20 * D2R), (0.0, 5 * D2R), (5 * D2R, 20 * D2R)]]
    w = _small_workload(nside, dets, seed=7)
    load_workload(conv, w, dtype)
    for mode in (oracle.OUT_TOD, oracle.OUT_STOKES):
        outs = []
        for k in range(3):
            if mode == oracle.OUT_TOD and k == 0:
                # pixel counts are integers.  The pixel path decides membership in
                # FP64 like the oracle: exact.  The tile path decides it in FP32 on
                # differences from the tile centre: a pixel within ~1e-7 of the
                # disc edge may flip, so at most a rare +-1.
                cnt = conv.convolve(k, out_mode=2).cpu().numpy().astype(np.int64)
                want_cnt = np.array([oracle.disc(nside, a, b, 20 * D2R).size for a, b in zip(th, ph)])
                if algo == 0:
                    assert np.array_equal(cnt, want_cnt)
                else:
                    d = np.abs(cnt - want_cnt)
                    assert d.max() <= 1 and (d > 0).mean() <= 0.01
            got = conv.convolve(k, out_mode=mode).cpu().numpy()
            want = oracle_detector(w, k, slice(None), dtype, out_mode=mode)
            e = rel_err(got, want)
            say(f"  det {k} mode {mode}: max rel err {e:.3e}")
            assert e <= tol
            outs.append(got.astype(np.float64))
        assert rel_err(outs[1] + outs[2], outs[0]) <= 10 * tol


def test_delta_and_uniform_closed_forms(conv, torch):
    say("case: delta beam and uniform sky")
    nside = 64
    pix = np.array([0, 7, 1000, 24575, 30000, 49151])
    th, ph = oracle.pix2ang(nside, pix)
    rng = np.random.default_rng(1)
    ps = rng.uniform(0, 2 * np.pi, pix.size)
    bs = B.delta_beamsor(41, 0.005)
    w = _small_workload(nside, [_det(bs, th, ph, ps, zeta=0.4, eps=0.1, s=2.0, rmax=np.arctan(0.005))], seed=3)
    load_workload(conv, w, np.float64)
    got = conv.convolve(0).cpu().numpy()
    I, Q, U = (m[pix] for m in w.sky)
    want = 0.5 * 2.0 * (1.1 * I + 0.9 * (Q * np.cos(2 * (ps + 0.4)) + U * np.sin(2 * (ps + 0.4))))
    # pixel-centre pointings land within ~1e-16 rad of the centre node: f ~ 1e-12
    assert np.abs(got - want).max() < 1e-11
    one = np.ones(12 * nside * nside)
    w2 = Workload("u", nside, (one, 0 * one, 0 * one),
                  [_det(_gauss(101, 4.5, 1.5, leak=0.0), np.arccos(rng.uniform(-1, 1, 500)),
                        rng.uniform(0, 6.3, 500), rng.uniform(0, 6.3, 500), eps=0.0, s=2.0, rmax=4.5 * D2R)])
    for dtype, tol in [(np.float64, 1e-14), (np.float32, 2e-7)]:
        load_workload(conv, w2, dtype)
        got = conv.convolve(0).cpu().numpy()
        assert np.abs(got - 1.0).max() < tol, dtype


@pytest.mark.parametrize("algo", ALGOS)
def test_psi_plus_pi_and_determinism(conv, torch, algo):
    say(f"case: psi+pi, determinism, launch shapes, algo {algo}")
    w = W.c2(n_samples=4000)
    d = w.detectors[0]
    conv.set_launch(algorithm=algo)
    load_workload(conv, w, np.float32)
    a = conv.convolve(0).cpu().numpy()
    b = conv.convolve(0).cpu().numpy()
    assert np.array_equal(a, b)
    for shape in [(64, 1, 1, 1, 64), (192, 2, 3, 8, 128), (256, 8, 1, 1, 128), (64, 4, 2, 8, 256)]:
        spt, wpg, gpc, xq, ch = shape
        conv.set_launch(samples_per_tile=spt, waves_per_group=wpg, groups_per_cu=gpc, xcd_queues=xq, chunk=ch)
        c = conv.convolve(0).cpu().numpy()
        assert np.array_equal(a, c), shape
    if algo == 0:
        conv.set_launch(samples_per_tile=7)
        assert np.array_equal(a, conv.convolve(0).cpu().numpy())
    conv.set_pointing(0, *(torch.from_numpy(x).cuda() for x in (d.theta, d.phi, d.psi + np.pi)))
    e = conv.convolve(0).cpu().numpy()
    assert rel_err(e, a) <= 2e-6


def test_empty_and_invalid_inputs(conv, torch):
    from paper_1908_05662_amd import PiscoError

    say("case: empty and invalid inputs")
    w = W.c1(n_samples=10)
    load_workload(conv, w, np.float64)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    conv.set_pointing(0, e, e, e)
    assert conv.output_samples(0) == 0
    out = conv.convolve(0)
    assert out.numel() == 0
    bad = torch.tensor([np.nan], dtype=torch.float64, device="cuda")
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(PiscoError):
        conv.set_pointing(0, bad, one, one)
    with pytest.raises(PiscoError):
        conv.set_pointing(0, one + 4.0, one, one)  # theta > pi
    with pytest.raises(PiscoError):
        conv.set_detector(0, 0.0, 0.0, 2.0, 0, 1.0)  # rho_max >= pi/2
    with pytest.raises(PiscoError):
        conv.set_sky(3, one, one, one)  # nside not a power of two
    # a failed call leaves the previous state usable
    assert conv.output_samples(0) == 0


@pytest.mark.parametrize("algo", ALGOS)
def test_batched_graph_replay_matches_per_detector(conv, torch, algo):
    """All detectors in one persistent launch, captured once and replayed; every
    replay (with eager launches in between) equals the per-detector launches."""
    say(f"case: batched graph replay algo {algo}")
    conv.set_launch(algorithm=algo)
    rng = np.random.default_rng(8)
    nside = 64
    dets = []
    for k in range(6):
        n = int(rng.integers(1, 3000))
        if k % 2:
            th, ph, ps = np.arccos(rng.uniform(-1, 1, n)), rng.uniform(0, 6.3, n), rng.uniform(0, 6.3, n)
        else:  # a slow great-circle-ish sweep: coherent tiles
            s0 = rng.uniform(0, 6.3)
            th = 1.0 + 0.4 * np.sin(np.linspace(0, 2, n) + s0)
            ph, ps = np.linspace(s0, s0 + 1.5, n), np.linspace(0, 4, n)
        dets.append(_det(_gauss(61, 3.0 + k * 0.3, 1.0 + 0.1 * k, e=0.05 * k, o=k), th, ph, ps,
                         zeta=0.3 * k, rmax=(3.0 + 0.3 * k) * D2R))
    w = _small_workload(nside, dets, seed=11)
    load_workload(conv, w, np.float32)
    ref = np.concatenate([conv.convolve(k).cpu().numpy() for k in range(6)])
    s = torch.cuda.Stream()
    out = torch.empty(conv.output_samples(-1), dtype=torch.float32, device="cuda")
    for rep in range(4):
        with torch.cuda.stream(s):
            out.fill_(np.nan)
            conv.convolve(-1, out=out, stream=s)
        s.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
        _ = conv.convolve(2).cpu()  # eager work between replays
    idx = np.arange(0, len(dets[3].theta), 97)
    off = sum(len(d.theta) for d in dets[:3])
    want = oracle_detector(w, 3, idx, np.float32)
    assert rel_err(ref[off + idx], want) <= F32_TOL


@pytest.mark.parametrize("nside,rmax_deg,step_deg", [(64, 10.0, 0.3), (256, 5.0, 0.05), (512, 2.0, 0.01),
                                                     (128, 30.0, 0.5)])
def test_tile_counts_on_coherent_scans(conv, torch, nside, rmax_deg, step_deg):
    """The tile path walks each ring over the hull of its lanes' own disc
    intervals (narrower than the union cap): on coherent CES tiles at several
    radii and latitudes its pair counts match the FP64 disc sizes (the FP32
    membership test may flip a pixel within ~1e-7 of an edge: at most a rare
    +-1), and the TOD matches the oracle."""
    say(f"case: tile counts on coherent scans, nside {nside}, disc {rmax_deg} deg, step {step_deg} deg")
    conv.set_launch(algorithm=1)
    parts = [S.ces(3000, lat, el_deg=el, az_step_deg=step_deg, sweep_deg=360.0 * step_deg / 0.01 / 4)
             for lat, el in [(-0.4, 45.0), (0.2, 30.0), (-1.1, 60.0), (0.9, 50.0)]]
    th, ph, ps = (np.concatenate(x) for x in zip(*parts))
    rmax = rmax_deg * D2R
    bs = _gauss(101, rmax_deg, rmax_deg / 3, leak=0.0)
    w = _small_workload(nside, [_det(bs, th, ph, ps, rmax=rmax)], seed=nside + 3)
    load_workload(conv, w, np.float32)
    cnt = conv.convolve(0, out_mode=2).cpu().numpy().astype(np.int64)
    idx = np.linspace(0, th.size - 1, 150).astype(int)
    want_cnt = np.array([oracle.disc(nside, th[i], ph[i], rmax).size for i in idx])
    d = np.abs(cnt[idx] - want_cnt)
    say(f"  counts: max |diff| {d.max()}, {int((d > 0).sum())} of {idx.size} differ")
    assert d.max() <= 1 and (d > 0).mean() <= 0.02
    got = conv.convolve(0).cpu().numpy()
    want = oracle_detector(w, 0, idx, np.float32)
    e = rel_err(got[idx], want)
    say(f"  TOD: max rel err {e:.3e}")
    assert e <= F32_TOL


@pytest.mark.parametrize("n,algo,beam", [(3, 0, "auto"), (3, 1, "auto"), (3, 2, "auto"), (4095, 0, "auto"),
                                         (4095, 1, "auto"), (4095, 2, "auto"), (3, 1, "full"), (4095, 0, "full"),
                                         (4095, 1, "full")])
def test_grid_size_limits(conv, torch, n, algo, beam):
    """Beams at the smallest and the largest grid the ABI accepts (n = 3 and 4095).
    One-grid: the padded record array of the largest holds 4096^2 records in row
    pairs, so record indices reach 2^24; four-channel: node byte offsets reach
    268 MB.  Every FP32 path, against the oracle."""
    say(f"case: grid size {n} x {n}, algo {algo}, beam {beam}")
    from synth.sky import make_sky

    span = 3.0 if n == 3 else 2.5
    T, u, v, rho, sig = B.tangent_grid(n, span * D2R)
    g = B.elliptical_gaussian(rho, sig, 1.5 * D2R, 0.05, 0.4)
    bs = B.ideal_beamsor(g, T)
    if beam == "full":
        bs = B.with_qu_leakage(bs, g, 0.01)
    m = 256
    t = np.linspace(0.0, 1.0, m)
    th, ph, ps = 1.0 + 0.05 * t, 2.0 + 0.1 * t, 0.7 + 0.3 * t
    det = Detector(bs, B.DetectorParams(0.2, 0.01, 1.0), 0.0, 2.0 * D2R, W.NORM_PER_SAMPLE, 1.0, th, ph, ps)
    w = Workload("grid-limits", 128, tuple(make_sky(128, 383, 2.0, seed=13)), [det])
    conv.set_launch(algorithm=algo, coherence=0.5)
    load_workload(conv, w, np.float32, beam=beam)
    got = conv.convolve(0).cpu().numpy()
    want = oracle_detector(w, 0, slice(None), np.float32)
    e = rel_err(got, want)
    say(f"  max rel err {e:.3e}")
    assert e <= F32_TOL


@pytest.mark.parametrize("algo", [0, 1])
def test_max_nside_sky(conv, torch, algo):
    """The largest sky the ABI accepts (nside 8192, 805M pixels, 12.9 GB on the
    device): zero maps with a smooth I, Q, U on the rings within 4 deg of a
    128-sample scan (2 deg disc, ~2.4e5 pixels per sample), against the oracle
    on the same (FP32-rounded) maps."""
    import gc

    from synth.rings import ring_table

    say(f"case: nside 8192 sky, algo {algo}")
    N = 8192
    npix = 12 * N * N
    th0 = 1.0
    z, st, nring, first, phi0 = ring_table(N)
    rth = np.arctan2(st, z)
    maps = [np.zeros(npix, dtype=np.float32) for _ in range(3)]
    for r in np.nonzero(np.abs(rth - th0) < 4.0 * D2R)[0]:
        n = int(nring[r])
        ph = phi0[r] + 2.0 * np.pi * np.arange(n) / n
        sl = slice(int(first[r]), int(first[r]) + n)
        t = rth[r]
        maps[0][sl] = 1.0 + np.sin(40.0 * t) * np.cos(30.0 * ph) + 0.3 * np.cos(70.0 * ph + 5.0 * t)
        maps[1][sl] = 0.1 * np.cos(50.0 * t + 20.0 * ph)
        maps[2][sl] = 0.1 * np.sin(35.0 * t - 45.0 * ph)
    T, u, v, rho, sig = B.tangent_grid(201, 2.2 * D2R)
    bs = B.ideal_beamsor(B.elliptical_gaussian(rho, sig, 1.0 * D2R, 0.05, 0.3), T)
    m = 128
    s = np.linspace(0.0, 1.0, m)
    th, ph, ps = th0 + 0.002 * s, 2.0 + 0.02 * s, 0.4 + 0.5 * s
    det = Detector(bs, B.DetectorParams(0.2, 0.01, 1.0), 0.0, 2.0 * D2R, W.NORM_PER_SAMPLE, 1.0, th, ph, ps)
    w = Workload("max-nside", N, tuple(maps), [det])
    try:
        conv.set_launch(algorithm=algo, coherence=0.5)
        load_workload(conv, w, np.float32)
        got = conv.convolve(0).cpu().numpy()
        want = oracle_detector(w, 0, slice(None), np.float32)
        e = rel_err(got, want)
        say(f"  max rel err {e:.3e}")
        assert e <= F32_TOL
    finally:
        del w, maps
        gc.collect()


@pytest.mark.parametrize("algo", [0, 1, 2])
def test_discs_with_zero_or_one_pixel(conv, torch, algo):
    """Degenerate discs: radius 0.2 deg on an nside-64 sky (pixels ~0.9 deg apart)
    along a slow scan, so most samples see no pixel centre (per-sample
    normalisation by an empty sum: the TOD is 0) or exactly one (the TOD is that
    pixel's term, normalised); the GPU must give 0 exactly where the oracle does
    and match it elsewhere."""
    say(f"case: discs of zero or one pixel, algo {algo}")
    from synth.sky import make_sky

    T, u, v, rho, sig = B.tangent_grid(41, 0.5 * D2R)
    bs = B.ideal_beamsor(B.elliptical_gaussian(rho, sig, 0.3 * D2R, 0.05, 0.3), T)
    m = 512
    s = np.linspace(0.0, 1.0, m)
    th, ph, ps = 1.0 + 0.3 * s, 2.0 + 0.05 * s, 0.4 + 2.0 * s
    det = Detector(bs, B.DetectorParams(0.2, 0.01, 1.0), 0.0, 0.2 * D2R, W.NORM_PER_SAMPLE, 1.0, th, ph, ps)
    w = Workload("tiny-discs", 64, tuple(make_sky(64, 191, 2.0, seed=17)), [det])
    conv.set_launch(algorithm=algo, coherence=0.5)
    load_workload(conv, w, np.float32)
    got = conv.convolve(0).cpu().numpy()
    from paper_1908_05662_amd import OUT_COUNT

    cnt = conv.convolve(0, out_mode=OUT_COUNT).cpu().numpy()
    want = oracle_detector(w, 0, slice(None), np.float32)
    empty = want == 0.0
    say(f"  {int(empty.sum())} empty discs, {int((cnt == 1).sum())} with one pixel, of {m}")
    assert empty.sum() >= m // 4 and (cnt == 1).sum() >= m // 8, "the scan must produce both degenerate cases"
    assert np.all(got[empty] == 0.0)
    e = rel_err(got[~empty], want[~empty])
    say(f"  max rel err {e:.3e}")
    assert e <= F32_TOL


@pytest.mark.parametrize("eps", [1.0, -1.0])
@pytest.mark.parametrize("algo,beam", [(0, "auto"), (1, "auto"), (0, "full"), (1, "full")])
def test_polarisation_efficiency_extremes(conv, torch, eps, algo, beam):
    """Detector polarisation efficiency at its extremes: eps = 1 cancels the
    polarised response (the TOD sees I only), eps = -1 the total-intensity one
    (Q and U only); the folded channels then have zero weights, in the one-grid
    and the four-channel forms alike."""
    say(f"case: eps {eps}, algo {algo}, beam {beam}")
    from synth.sky import make_sky

    T, u, v, rho, sig = B.tangent_grid(101, 2.5 * D2R)
    g = B.elliptical_gaussian(rho, sig, 1.0 * D2R, 0.05, 0.3)
    bs = B.ideal_beamsor(g, T)
    if beam == "full":
        bs = B.with_qu_leakage(bs, g, 0.01)
    m = 256
    s = np.linspace(0.0, 1.0, m)
    th, ph, ps = 0.8 + 0.01 * s, 1.0 + 0.05 * s, 0.3 + 2.0 * s
    det = Detector(bs, B.DetectorParams(0.35, eps, 1.0), 0.0, 2.0 * D2R, W.NORM_PER_SAMPLE, 1.0, th, ph, ps)
    w = Workload("eps-extremes", 128, tuple(make_sky(128, 383, 2.0, seed=19)), [det])
    conv.set_launch(algorithm=algo, coherence=0.5)
    load_workload(conv, w, np.float32, beam=beam)
    got = conv.convolve(0).cpu().numpy()
    want = oracle_detector(w, 0, slice(None), np.float32)
    e = rel_err(got, want)
    say(f"  max rel err {e:.3e}")
    assert e <= F32_TOL
