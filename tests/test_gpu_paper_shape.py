"""The paper's whole-sky benchmark pattern (Sec. 5.3, Table 1): a detector pair
at zeta 0 and -90 deg pointed at every nside-128 pixel centre at psi 0, 45,
90 deg (1,179,648 samples), Gaussian FWHM 1.5 deg, per-sample normalisation,
disc radii 5 and 30 deg; sampled outputs of the batched launch vs the oracle."""
import numpy as np
import pytest

from synth import workloads as W

from gpu_helpers import load_workload, oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


@pytest.mark.parametrize("rho", [5.0, 30.0])
def test_paper_shape_parity(torch, rho):
    from paper_1908_05662_amd.api import Convolver

    say(f"case: paper benchmark pattern, rho_max {rho} deg, 1,179,648 samples")
    w = W.paper_shape(rho, nside=128)
    conv = Convolver(0)
    try:
        load_workload(conv, w, np.float32)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            got = conv.convolve(-1, stream=stream)
        stream.synchronize()
        got = got.cpu().numpy()
        off = 0
        for k, d in enumerate(w.detectors):
            j = np.unique(np.concatenate([np.linspace(0, d.n - 1, 24).astype(int), [0, 1, 4, 196607, 196608]]))
            want = oracle_detector(w, k, j, np.float32)
            e = rel_err(got[off + j], want)
            say(f"  detector {k}: max rel err {e:.3e}")
            assert e <= 1e-6
            off += d.n
    finally:
        torch.cuda.synchronize()
        conv.close()
