"""The nside-2048 full-scale workload at its real shapes: sky of 50.3 M pixels
(l <= 4095), 151^2 elliptical main beams with disc 1.5 deg, and the shared
401^2 ring grid over +-20 deg for the annulus (1.5, 20] deg.  Sixteen of the
256 detectors (390,625 CES samples each, 6.25e6 in all) run in one batched
launch; sampled outputs are checked against the oracle, and the fused
sidelobe epilogue is checked on detector slices of the batched TOD."""
import numpy as np
import pytest

import oracle
from synth import beams as B
from synth import workloads as W

from gpu_helpers import load_workload, oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu
F32_TOL = 1e-6
N_DET = 16


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture(scope="module")
def workload():
    say("case: full-scale workload, 16 detectors, nside 2048 sky synthesis")
    return W.c5(n_det=N_DET)


def test_full_scale_main_and_annulus_parity(torch, workload):
    from paper_1908_05662_amd.api import Convolver

    w = workload
    conv = Convolver(0)
    try:
        say("case: full-scale batched main-beam TOD, sampled outputs vs oracle")
        load_workload(conv, w, np.float32)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            tod = conv.convolve(-1, stream=stream)
        stream.synchronize()
        got = tod.cpu().numpy()
        offs = np.cumsum([0] + [d.n for d in w.detectors])
        worst = 0.0
        rng = np.random.default_rng(2048)
        for k in range(N_DET):
            d = w.detectors[k]
            # group boundaries (64-sample tiles), the stream's ends and middle, and seeded positions
            j = np.unique(np.concatenate([[0, 1, 63, 64, 127, 128, d.n // 3, d.n // 2, d.n - 65, d.n - 64, d.n - 1],
                                          rng.integers(0, d.n, 5)]))
            want = oracle_detector(w, k, j, np.float32)
            worst = max(worst, rel_err(got[offs[k] + j], want))
        say(f"  main: max rel err {worst:.3e} ({N_DET} detectors x up to 16 samples)")
        assert worst <= F32_TOL

        say("case: full-scale annulus (1.5, 20] deg on the ring grid, STOKES, vs oracle")
        T, g = W.sidelobe_beam(401, 20.0, 0.25)
        r_main = w.meta["r_main"]
        d0 = w.detectors[0]
        k = N_DET
        conv.set_beam_scalar(k, 401, T, g, 0.5, 0.5, 0.0, 1.0, dtype=torch.float32)
        conv.set_detector(k, 0.0, r_main, np.deg2rad(20.0), W.NORM_FIXED, d0.norm_scale)
        sel = slice(1000, 1000 + 320)  # 5 groups of 64 consecutive scan samples
        th, ph, ps = (np.ascontiguousarray(x[sel]) for x in (d0.theta, d0.phi, d0.psi))
        conv.set_pointing(k, *(torch.from_numpy(x).cuda() for x in (th, ph, ps)))
        p = conv.convolve(k, out_mode=oracle.OUT_STOKES).cpu().numpy()
        jj = np.array([0, 1, 2, 63, 64, 65, 100, 127, 128, 150, 191, 192, 200, 230, 255, 256, 257, 290, 318, 319])
        sky = [m.astype(np.float32).astype(np.float64) for m in w.sky]
        dense = B.ideal_beamsor(g.astype(np.float32).astype(np.float64), T).dense()
        want = oracle.tod(w.nside, *sky, dense, T, 0.0, 0.0, 1.0, r_main, np.deg2rad(20.0), W.NORM_FIXED,
                          d0.norm_scale, th[jj], ph[jj], ps[jj], oracle.OUT_STOKES)
        e = rel_err(p[jj], want)
        say(f"  annulus: max rel err {e:.3e} ({len(jj)} samples)")
        assert e <= F32_TOL
    finally:
        torch.cuda.synchronize()
        conv.close()


def test_full_scale_epilogue_on_detector_slices(torch, workload):
    """The fused network epilogue applied per detector on slices of the batched
    TOD equals forward + combination computed from the features."""
    from paper_1908_05662_amd.api import Convolver, Mlp
    from paper_1908_05662_amd.surrogate import detector_coef

    say("case: full-scale epilogue on detector slices")
    w = workload
    conv = Convolver(0)
    try:
        load_workload(conv, w, np.float32)
        net = Mlp(conv, 512, 10, 4096, 3)
        tod = torch.zeros(w.n_samples, dtype=torch.float32, device="cuda")
        offs = np.cumsum([0] + [d.n for d in w.detectors])
        mean, std = [0.1, -0.2, 0.05], [1.5, 0.7, 0.9]
        for k in (0, 5, 15):
            d = w.detectors[k]
            coef = detector_coef(d.det.zeta, d.det.eps, d.det.s)
            net.apply(k, mean, std, coef, tod[offs[k]:offs[k + 1]])
            x = net.features(k)[:4096]
            y = net.forward(x).double().cpu().numpy()
            want = sum(coef[c] * (mean[c] + std[c] * y[:, c]) for c in range(3))
            got = tod[offs[k]:offs[k] + 4096].double().cpu().numpy()
            e = float(np.abs(got - want).max() / np.abs(want).max())
            say(f"  detector {k}: max rel diff {e:.3e}")
            assert e < 1e-6
        assert float(tod[offs[1]:offs[5]].abs().max()) == 0.0  # untouched detectors stay zero
        net.close()
    finally:
        torch.cuda.synchronize()
        conv.close()
