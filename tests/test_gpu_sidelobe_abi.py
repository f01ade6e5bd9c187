"""The far-sidelobe lifecycle behind the C ABI (pisco_sidelobe_train / enable /
share / history): state rules, the TOD with the network enabled, the
rotation of the network's pickups by each detector's angle, and the batched
graph launch with enabled detectors.  A short training run (the network's
accuracy on the full workload is judged in test_gpu_surrogate.py)."""
import numpy as np
import pytest

from synth import workloads as W

from gpu_helpers import say

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


def _setup(conv, torch, n=20_000):
    """nside-256 smooth sky, the 401^2 far-sidelobe beam over +-20 deg (main disc
    5 deg); detector 0 the full 20 deg disc at zeta = 0; held-out pointings."""
    from paper_1908_05662_amd.surrogate import spatial_order

    w = W.c4(n, stream=2)
    d = w.detectors[0]
    o = spatial_order(d.theta, d.phi)
    pts = [torch.from_numpy(np.ascontiguousarray(x[o])).cuda() for x in (d.theta, d.phi, d.psi)]
    T, g = W.sidelobe_beam(401, 20.0, 1.0)
    conv.set_sky(w.nside, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in w.sky), dtype=torch.float32)
    conv.set_beam_scalar(0, 401, T, torch.from_numpy(g.astype(np.float32)).cuda(), 0.5, 0.5, 0.0, 1.0,
                         dtype=torch.float32)
    conv.set_detector(0, 0.0, 0.0, 20 * D2R, W.NORM_FIXED, d.norm_scale)
    conv.set_pointing(0, *pts)
    return w, d, pts


def test_state_rules(conv, torch):
    from paper_1908_05662_amd import PiscoError

    say("case: sidelobe state rules (untrained, per-sample norm, radii, dropped on parameter change)")
    w, d, pts = _setup(conv, torch)
    with pytest.raises(PiscoError, match="ESTATE"):
        conv.sidelobe_enable(0, True)
    with pytest.raises(PiscoError, match="EINVAL"):
        conv.sidelobe_train(0, 25 * D2R, 16384, 1, 1)          # r_main beyond the disc
    conv.set_detector(1, 0.0, 0.0, 20 * D2R, W.NORM_PER_SAMPLE, 1.0)
    conv.share_beam(1, 0)
    with pytest.raises(PiscoError, match="EINVAL"):
        conv.sidelobe_train(1, 5 * D2R, 16384, 1, 1)           # per-sample normalisation: no split
    conv.sidelobe_options(batch=8192)
    with pytest.raises(PiscoError, match="EINVAL"):
        conv.sidelobe_train(0, 5 * D2R, 4096, 1, 1)            # fewer samples than one batch
    hist = conv.sidelobe_train(0, 5 * D2R, 16384, 3, 2)
    say(f"  loss history {hist}")
    assert len(hist) == 2 and all(np.isfinite(hist))
    conv.sidelobe_enable(0, True)
    conv.set_detector(0, 0.0, 0.0, 20 * D2R, W.NORM_FIXED, d.norm_scale)  # the disc changed: network dropped
    assert conv.sidelobe_history(0) == []
    with pytest.raises(PiscoError, match="ESTATE"):
        conv.sidelobe_enable(0, True)


def test_enabled_tod_and_angle_rotation(conv, torch):
    """Detectors sharing one network at zeta = 0, 45, 90 deg give the network's
    three pickup channels; a detector at 22.5 deg must then see their rotation by
    45 deg, and disabling restores the exact TOD bit for bit."""
    say("case: enabled TOD = exact main disc + network pickups turned by each detector's angle")
    w, d, pts = _setup(conv, torch)
    exact_full = conv.convolve(0).clone()
    conv.sidelobe_train(0, 5 * D2R, 32768, 5, 3)
    zetas = [0.0, 45.0, 90.0, 22.5]
    wI, wQ = 0.5, 0.5
    for k, z in enumerate(zetas, start=1):
        conv.share_beam(k, 0)
        conv.set_detector(k, z * D2R, 0.0, 5 * D2R, W.NORM_FIXED, d.norm_scale)
        conv.set_pointing(k, *pts)
    main = [conv.convolve(k).double() for k in range(1, 5)]
    for k in range(1, 5):
        conv.sidelobe_share(k, 0)
        conv.sidelobe_enable(k, True)
    side = [conv.convolve(k).double() - main[k - 1] for k in range(1, 5)]
    pI = (side[0] + side[2]) / (2 * wI)
    pQ = (side[0] - side[2]) / (2 * wQ)
    pU = (side[1] - wI * pI) / wQ
    c, s = np.cos(2 * 22.5 * D2R), np.sin(2 * 22.5 * D2R)
    want = wI * pI + wQ * (c * pQ + s * pU)
    scale = float(torch.sqrt(torch.mean(side[3] ** 2)))
    e = float((side[3] - want).abs().max()) / scale
    say(f"  rotation consistency: max |diff| / rms(sidelobe) {e:.2e}")
    assert scale > 0 and e < 1e-3
    # the enabled TOD of the trained detector itself, and its exact TOD back when disabled
    conv.sidelobe_enable(0, True)
    on = conv.convolve(0).double()
    assert float((on - main[0] - side[0]).abs().max()) <= 1e-6 * float(main[0].abs().max())
    conv.sidelobe_enable(0, False)
    assert torch.equal(conv.convolve(0), exact_full)


def test_batched_graph_with_enabled_detectors(conv, torch):
    say("case: batched graph launch with surrogate-enabled detectors equals single-detector launches")
    w, d, pts = _setup(conv, torch)
    conv.sidelobe_train(0, 5 * D2R, 16384, 7, 1)
    for k in (1, 2):
        conv.share_beam(k, 0)
        conv.set_detector(k, [30.0, -60.0][k - 1] * D2R, 0.0, 20 * D2R, W.NORM_FIXED, d.norm_scale)
        conv.set_pointing(k, *pts)
        conv.sidelobe_share(k, 0)
    conv.sidelobe_enable(0, True)
    conv.sidelobe_enable(2, True)      # detector 1 stays exact
    single = torch.cat([conv.convolve(k) for k in range(3)])
    stream = torch.cuda.Stream()
    out = torch.empty(single.numel(), dtype=torch.float32, device="cuda")
    for _ in range(3):                 # capture, then two replays
        out.zero_()
        with torch.cuda.stream(stream):
            conv.convolve(-1, out=out, stream=stream)
        stream.synchronize()
        assert torch.equal(out, single)
