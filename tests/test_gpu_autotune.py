"""Launch-shape autotuner: it searches real launches, applies the best shape,
caches it, and the tuned launch computes the same TOD."""
import numpy as np
import pytest

from synth import workloads as W

from gpu_helpers import load_workload, oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    return t


def test_autotune_search_cache_and_parity(torch, tmp_path):
    from paper_1908_05662_amd.api import Convolver
    from paper_1908_05662_amd.autotune import tune

    say("case: autotune on the nside-512 CES workload, 4e5 samples, batched graph launch")
    w = W.c2(n_samples=400_000)
    conv = Convolver(0)
    try:
        load_workload(conv, w, np.float32)
        default = conv.get_launch()
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            ref = conv.convolve(-1, stream=stream).clone()
        stream.synchronize()
        cache = str(tmp_path / "t.tune.json")
        rec = tune(conv, -1, subsample=0.5, reps=2, cache=cache, max_passes=1, log=say)
        say(f"  tuned {rec['launch']}: {rec['ms']:.3f} ms vs default {rec['default_ms']:.3f} ms, "
            f"{len(rec['trials'])} trials")
        assert not rec["cached"]
        assert conv.get_launch() == rec["launch"]
        assert rec["ms"] <= rec["default_ms"]
        assert all(t["ms"] is None or t["ms"] > 0 for t in rec["trials"])
        # the full streams are restored after the subsampled search
        assert conv.output_samples(-1) == w.n_samples
        with torch.cuda.stream(stream):
            got = conv.convolve(-1, stream=stream).clone()
        stream.synchronize()
        idx = np.linspace(0, w.n_samples - 1, 40).astype(int)
        want = oracle_detector(w, 0, idx, np.float32)
        assert rel_err(got.cpu().numpy()[idx], want) <= 1e-6
        assert rel_err(got.cpu().numpy(), ref.cpu().numpy()) <= 2e-6
        # second call: same signature -> cached shape, no search
        conv.set_launch(**default)
        rec2 = tune(conv, -1, subsample=0.5, reps=2, cache=cache, max_passes=1)
        assert rec2["cached"] and rec2["launch"] == rec["launch"] and conv.get_launch() == rec["launch"]
    finally:
        torch.cuda.synchronize()
        conv.close()
