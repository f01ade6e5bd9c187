"""The allocation-free entry point pisco_convolve_static against pisco_convolve
(same context, given processing order): bit-identical outputs on two calls in
a row, the second with a smaller stream, for TOD and Stokes pickups; no
device memory is allocated by the calls; the size limit is enforced."""
import ctypes

import numpy as np
import pytest

from synth import workloads as W

from gpu_helpers import load_workload, oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu
F32_TOL = 1e-6
MAX_SAMPLES = 4_194_304


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


def test_static_entry_matches_convolve(torch):
    from paper_1908_05662_amd import OUT_STOKES, OUT_TOD
    from paper_1908_05662_amd.api import Convolver

    say("case: allocation-free convolve vs pisco_convolve, 100,000 then 30,001 samples, TOD and Stokes")
    w = W.c2(n_samples=100_000)
    w.detectors.append(W.c2(n_samples=20_000, sky=w.sky).detectors[0])
    conv = Convolver(0)
    conv.set_ordering("given")
    load_workload(conv, w, np.float32)
    d = w.detectors[0]
    stream = torch.cuda.Stream()
    for n in (100_000, 30_001):
        keep = [torch.from_numpy(np.ascontiguousarray(x[:n])).cuda() for x in (d.theta, d.phi, d.psi)]
        conv.set_pointing(0, *keep)
        torch.cuda.synchronize()
        before = conv.memory_in_use()
        got = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        with torch.cuda.stream(stream):
            conv.convolve_static(0, OUT_TOD, out=got, stream=stream)
        sto = torch.full((n, 3), float("nan"), dtype=torch.float32, device="cuda")
        with torch.cuda.stream(stream):
            conv.convolve_static(0, OUT_STOKES, out=sto, stream=stream)
        stream.synchronize()
        assert conv.memory_in_use() == before
        want = conv.convolve(0)
        want_s = conv.convolve(0, out_mode=OUT_STOKES)
        torch.cuda.synchronize()
        say(f"  n {n}: TOD equal {torch.equal(got, want)}, Stokes equal {torch.equal(sto, want_s)}")
        assert torch.equal(got, want) and torch.equal(sto, want_s)
        idx = np.array([0, 63, 64, n // 2, n - 1])
        sub = W.Workload("c2", w.nside, w.sky, [d])
        e = rel_err(got.cpu().numpy()[idx], oracle_detector(sub, 0, idx, np.float32))
        say(f"  n {n}: sampled oracle rel err {e:.3e}")
        assert e <= F32_TOL
    # another detector of the same context (its own beam and stream)
    got1 = conv.convolve_static(1)
    torch.cuda.synchronize()
    assert torch.equal(got1, conv.convolve(1))
    conv.close()


def test_static_entry_size_limit(torch):
    from paper_1908_05662_amd import PiscoError
    from paper_1908_05662_amd.api import Convolver

    say("case: allocation-free convolve rejects streams beyond its static plan")
    w = W.c2(n_samples=1000)
    conv = Convolver(0)
    load_workload(conv, w, np.float32)
    n = MAX_SAMPLES + 1
    th = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    ph = torch.zeros(n, dtype=torch.float64, device="cuda")
    conv.set_pointing(0, th, ph, ph)
    with pytest.raises(PiscoError, match="EINVAL"):
        conv.convolve_static(0)
    conv.close()
