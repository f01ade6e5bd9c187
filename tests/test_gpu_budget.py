"""The device-memory budget (pisco_set_memory_budget): pointing and plate-angle
streams that do not fit stay on the host and are convolved in blocks of
samples, as are launches whose output staging does not fit.  Blocks start at
multiples of 64 samples, so in the given processing order the results equal
the resident path's bit for bit; sampled outputs also match the oracle."""
import numpy as np
import pytest

from synth import workloads as W

from gpu_helpers import oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu
F32_TOL = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.fixture(scope="module")
def work():
    w = W.c2(n_samples=100_000)
    w.detectors.append(W.c2(n_samples=37_001, sky=w.sky).detectors[0])   # ragged second detector
    return w


def _ctx(torch, w, budget_extra=None, host_pointing=False, plate=None):
    from paper_1908_05662_amd.api import Convolver

    conv = Convolver(0)
    conv.set_ordering("given")
    conv.set_sky(w.nside, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in w.sky), dtype=torch.float32)
    for k, d in enumerate(w.detectors):
        conv.set_beamsor(k, d.beam.dense(), d.beam.half_span_tan, d.det.eps, d.det.s, dtype=torch.float32)
        conv.set_detector(k, d.det.zeta, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale)
    base = conv.memory_in_use()
    if budget_extra is not None:
        conv.set_memory_budget(base + budget_extra)
    for k, d in enumerate(w.detectors):
        arrs = [np.ascontiguousarray(x) for x in (d.theta, d.phi, d.psi)]
        conv.set_pointing(k, *(arrs if host_pointing else [torch.from_numpy(a).cuda() for a in arrs]))
        if plate is not None:
            conv.set_hwp(k, plate[k])
    return conv, base


def test_host_pointing_streams_in_blocks(torch, work):
    say("case: pointing over the budget stays on the host; TOD and Stokes in blocks equal the resident path")
    w = work
    ref, _ = _ctx(torch, w)
    tod_ref = ref.convolve(-1).cpu()
    sto_ref = ref.convolve(0, out_mode=1).cpu()
    ref.close()
    conv, used = _ctx(torch, w, budget_extra=600_000, host_pointing=True)
    assert conv.memory_in_use() == used      # both streams stayed on the host
    for dev_out in (True, False):
        out = torch.empty(tod_ref.numel(), dtype=torch.float32, device="cuda" if dev_out else "cpu")
        got = conv.convolve(-1, out=out).cpu()
        assert torch.equal(got, tod_ref), f"device output {dev_out}"
    sto = conv.convolve(0, out_mode=1, out=torch.empty(sto_ref.shape, dtype=torch.float32)).cpu()
    assert torch.equal(sto, sto_ref)
    assert conv.memory_in_use() <= used + 600_000
    conv.close()
    d = w.detectors[1]
    idx = np.unique(np.concatenate([np.linspace(0, d.n - 1, 200).astype(np.int64), [63, 64, d.n - 1]]))
    e = rel_err(tod_ref.numpy()[w.detectors[0].n + idx], oracle_detector(w, 1, idx, np.float32))
    say(f"  ragged detector vs oracle: {e:.3e}")
    assert e <= F32_TOL


def test_plate_angles_on_the_host(torch, work):
    say("case: plate angles over the budget stay on the host; blocks equal the resident path")
    w = work
    plate = [2 * np.pi * 2.0 * np.arange(d.n) / 100.0 for d in w.detectors]
    ref, _ = _ctx(torch, w, plate=plate)
    want = ref.convolve(-1).cpu()
    ref.close()
    conv, _ = _ctx(torch, w, budget_extra=2_600_000, plate=plate)   # device pointing fits, plate angles do not
    got = conv.convolve(-1).cpu()
    conv.close()
    assert torch.equal(got, want)


def test_output_staging_over_budget(torch, work):
    say("case: device pointing within the budget, host output staging over it")
    w = work
    ref, _ = _ctx(torch, w)
    want = ref.convolve(-1).cpu()
    ref.close()
    conv, _ = _ctx(torch, w)
    conv.set_memory_budget(conv.memory_in_use() + 200_000)
    got = conv.convolve(-1, out=torch.empty(want.numel(), dtype=torch.float32)).cpu()
    conv.close()
    assert torch.equal(got, want)


def test_budget_too_small_for_a_block(torch, work):
    from paper_1908_05662_amd import PiscoError

    say("case: budget below one 64-sample block gives ENOMEM")
    conv, _ = _ctx(torch, work, budget_extra=1000, host_pointing=True)
    with pytest.raises(PiscoError, match="ENOMEM"):
        conv.convolve(-1)
    conv.close()


def test_surrogate_enabled_in_blocks(torch):
    say("case: a surrogate-enabled detector streamed in blocks equals the resident path")
    from paper_1908_05662_amd.api import Convolver

    D2R = np.pi / 180
    w = W.c4(30_000, stream=2)
    d = w.detectors[0]
    T, g = W.sidelobe_beam(401, 20.0, 1.0)
    outs = []
    for budget in (None, 400_000):
        conv = Convolver(0)
        conv.set_ordering("given")
        conv.set_sky(w.nside, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in w.sky), dtype=torch.float32)
        conv.set_beam_scalar(0, 401, T, torch.from_numpy(g.astype(np.float32)).cuda(), 0.5, 0.5, 0.0, 1.0)
        conv.set_detector(0, 0.3, 0.0, 20 * D2R, W.NORM_FIXED, d.norm_scale)
        conv.sidelobe_train(0, 5 * D2R, 16384, 11, 1)
        conv.sidelobe_enable(0, True)
        if budget is not None:
            conv.set_memory_budget(conv.memory_in_use() + budget)
        conv.set_pointing(0, d.theta, d.phi, d.psi)
        outs.append(conv.convolve(0, out=torch.empty(d.n, dtype=torch.float32)).clone())
        conv.close()
    assert torch.equal(outs[0], outs[1])
