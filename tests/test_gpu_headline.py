"""Full-size parity of the benchmark launches against the FP64 oracle.

* The nside-1024 batched workload exactly as the benchmark times it: all 64
  detectors (31.2M samples, each its own 201^2 elliptical beam, disc 2 deg,
  per-sample normalisation) in one graph-replayed launch with the default
  launch shape (the shape the tuner keeps for this workload).  For every
  detector, at least 16 samples are compared element by element with the
  oracle: tile boundaries (t = 63, 64, 127, 128), the ragged last group, spread
  samples, and samples of groups the tile classification sends to the pixel
  path (found on the host from the same coherence rule).
* The precision workload's whole 1e7-sample stream (nside 512), 10,000 samples
  spread over the full stream.
* The far-sidelobe workload's held-out stream (1e6 isotropic pointings, nside
  256): the 5 deg main-disc TOD and the full 20 deg disc TOD.

Tolerance: 1e-6 relative to the largest oracle value of the compared samples
(the FP32 path against the FP64 oracle on the same FP32-rounded inputs).
"""
import numpy as np
import pytest

from synth import workloads as W

from gpu_helpers import cached_workload, coherence_chords, load_workload, oracle_detector, rel_err, say

pytestmark = pytest.mark.gpu
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


def _headline_samples(d, rng, coherence):
    """At least 16 sample indices of detector d: group boundaries, the ragged
    tail, spread samples, and first/last samples of up to three groups that
    the coherence rule sends to the pixel path.  Returns (idx, pixel-path idx)."""
    n = d.n
    fixed = [0, 1, 62, 63, 64, 65, 127, 128, n // 4, n // 2, (3 * n) // 4, n - 65, n - 64, n - 2, n - 1,
             ((n - 1) // 64) * 64]
    chord, lim = coherence_chords(d, coherence)
    far = np.nonzero(chord > 1.05 * lim)[0]
    pix = []
    for g in rng.permutation(far)[:3]:
        pix += [64 * int(g), min(n - 1, 64 * int(g) + 63)]
    idx = np.unique(np.clip(np.array(fixed + pix + list(rng.integers(0, n, 4))), 0, n - 1))
    return idx, np.array(sorted(set(pix)), dtype=np.int64)


def test_c3_full_batched_launch_vs_oracle(conv, torch):
    say("case: nside-1024 benchmark workload, 64 detectors, one graph-replayed launch, sampled vs oracle")
    w = cached_workload("c3")
    load_workload(conv, w, np.float32)
    launch = conv.get_launch()
    say(f"  launch {launch}")
    stream = torch.cuda.Stream()
    out = torch.empty(w.n_samples, dtype=torch.float32, device="cuda")
    with torch.cuda.stream(stream):
        conv.convolve(-1, out=out, stream=stream)   # captures the graph
    stream.synchronize()
    first = out.clone()
    with torch.cuda.stream(stream):
        conv.convolve(-1, out=out, stream=stream)   # replays it
    stream.synchronize()
    assert torch.equal(first, out), "graph replay is not bitwise reproducible"
    got = out.cpu().numpy()
    offs = np.cumsum([0] + [d.n for d in w.detectors])
    rng = np.random.default_rng(1908)
    worst, n_checked, n_pix = 0.0, 0, 0
    for k, d in enumerate(w.detectors):
        idx, pix = _headline_samples(d, rng, launch["coherence"])
        want = oracle_detector(w, k, idx, np.float32)
        e = rel_err(got[offs[k] + idx], want)
        worst = max(worst, e)
        n_checked += idx.size
        n_pix += pix.size
        assert idx.size >= 16
        assert e <= F32_TOL, f"detector {k}: max rel err {e:.3e} (samples {idx.tolist()})"
    say(f"  {n_checked} samples of 64 detectors ({n_pix} from pixel-path groups): max rel err {worst:.3e}")
    assert n_pix > 0, "the workload should hold some groups the tile path leaves to the pixel path"


def test_c2_full_stream_spread_samples(conv, torch):
    say("case: nside-512 precision workload, the whole 1e7-sample stream, 10,000 spread samples vs oracle")
    w = W.c2()
    d = w.detectors[0]
    load_workload(conv, w, np.float32)
    got = conv.convolve(0).cpu().numpy()
    idx = np.unique(np.concatenate([np.linspace(0, d.n - 1, 10_001).astype(np.int64), [63, 64, 65, 127, 128],
                                    np.arange(d.n - 11, d.n)]))
    want = oracle_detector(w, 0, idx, np.float32)
    e = rel_err(got[idx], want)
    say(f"  {idx.size} samples of {d.n}: max rel err {e:.3e}")
    assert idx.size >= 10_000
    assert e <= F32_TOL


def test_c4_main_and_full_disc_vs_oracle(conv, torch):
    say("case: far-sidelobe workload, 1e6 held-out pointings, main 5 deg disc and full 20 deg disc vs oracle")
    from paper_1908_05662_amd.surrogate import spatial_order

    w = W.c4(1_000_000, stream=2)
    d = w.detectors[0]
    o = spatial_order(d.theta, d.phi)
    d.theta, d.phi, d.psi = d.theta[o], d.phi[o], d.psi[o]
    r_main = w.meta["r_main"]
    load_workload(conv, w, np.float32)
    idx = np.unique(np.concatenate([np.linspace(0, d.n - 1, 40).astype(np.int64), [63, 64, 999_999]]))
    full = conv.convolve(0).cpu().numpy()
    want = oracle_detector(w, 0, idx, np.float32)
    e_full = rel_err(full[idx], want)
    conv.set_detector(0, d.det.zeta, 0.0, r_main, d.norm_mode, d.norm_scale)
    main = conv.convolve(0).cpu().numpy()
    want_m = oracle_detector(w, 0, idx, np.float32, rho_max=r_main)
    e_main = rel_err(main[idx], want_m)
    say(f"  {idx.size} samples: full disc max rel err {e_full:.3e}, main disc {e_main:.3e}")
    assert e_full <= F32_TOL and e_main <= F32_TOL
