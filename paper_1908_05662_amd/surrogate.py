"""Far-sidelobe surrogate: exact main beam + a network for the far sidelobe.

For a detector whose folded beam channels are proportional to one scalar beam
b (an ideal beamsor, Eqs. 19-20 with D(chi)Lambda(chi) = D(0)), the TOD over
the disc rho <= r_full splits exactly into the main disc (rho <= r_main) and
the annulus (r_main < rho <= r_full):

    d = d_main + sum_c coef[c] P[c],
    coef = (s/2) ((1 + eps), (1 - eps) cos 2 zeta, (1 - eps) sin 2 zeta),

with P the annulus' Stokes pickup N sum b Lambda(-chi) S in the zeta = 0
frame (the convolver's STOKES output).  P depends on the pointing only, so a
network trained on exact pickups of one pointing set predicts it for any
other; the exact annulus convolution stays available as fallback and as the
judge of the network's error.

Training and the surrogate TOD run in the library (pisco_sidelobe_train /
pisco_sidelobe_enable: targets from the convolution kernels; features,
standardisation, shuffling, Adam steps, inference and the TOD epilogue on the
device).  This module only sets up workloads and measures them.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import _lib as L
from .api import Convolver, Mlp


def _hilbert_index(n: int, x, y):
    """Position along a Hilbert curve of an n x n grid (n a power of two) of the
    integer cells (x, y), vectorised (the standard quadrant-rotation recursion)."""
    x = np.asarray(x, dtype=np.int64).copy()
    y = np.asarray(y, dtype=np.int64).copy()
    d = np.zeros_like(x)
    s = n // 2
    while s > 0:
        rx = ((x & s) > 0).astype(np.int64)
        ry = ((y & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        low = ry == 0
        flip = low & (rx == 1)
        x = np.where(flip, s - 1 - x, x)
        y = np.where(flip, s - 1 - y, y)
        x, y = np.where(low, y, x), np.where(low, x, y)
        s //= 2
    return d


def spatial_order(theta, phi) -> np.ndarray:
    """Permutation that puts nearby pointings next to each other: Hilbert order
    on the equal-area (phi, z) square.  Samples are independent, so any order
    gives the same per-sample result; this one lets 64 consecutive samples
    share one compact disc union (the tile kernels)."""
    n = 1 << 16
    f = np.mod(np.asarray(phi, dtype=np.float64), 2 * np.pi) / (2 * np.pi)
    z = (np.cos(np.asarray(theta, dtype=np.float64)) + 1.0) * 0.5
    qx = np.clip((f * n).astype(np.int64), 0, n - 1)
    qy = np.clip((z * n).astype(np.int64), 0, n - 1)
    return np.argsort(_hilbert_index(n, qx, qy), kind="stable")


def detector_coef(zeta: float, eps: float, s: float):
    """Weights of (P_I, P_Q, P_U) in the detector's TOD (detector row of Eq. 20, rotated by zeta)."""
    return (0.5 * s * (1 + eps), 0.5 * s * (1 - eps) * math.cos(2 * zeta), 0.5 * s * (1 - eps) * math.sin(2 * zeta))


# dense BF16 matrix-core peak of the MI355X (no sparsity)
BF16_PEAK_TFLOPS = 2500.0


def network_flops_per_sample(width: int = 256, hidden: int = 4) -> int:
    """Multiply-adds x 2 of one forward pass: 5 -> width, (hidden - 1) x width^2, width -> 3."""
    return 2 * (5 * width + (hidden - 1) * width * width + width * 3)


def rms(x) -> float:
    import torch

    x = x.double() if isinstance(x, torch.Tensor) else torch.as_tensor(x, dtype=torch.float64)
    return float(torch.sqrt(torch.mean(x * x)))


def time_call(fn, reps: int = 5) -> float:
    """Mean seconds per call on the current stream, HIP events, one warm-up."""
    import torch

    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def network_rate(conv: Convolver, det: int, width: int, hidden: int, reps: int = 5) -> dict:
    """Time of the fused network epilogue alone (features, every layer and the TOD
    sum) over detector `det`'s pointing, for a network of this shape (the cost
    does not depend on the weights)."""
    import torch

    n = conv.output_samples(det)
    net = Mlp(conv, width, hidden, 64, 0)
    tod = torch.zeros(n, dtype=torch.float32, device=conv.torch_device)
    t = time_call(lambda: net.apply(det, [0.0] * 3, [1.0] * 3, [1.0, 0.0, 0.0], tod), reps)
    net.close()
    flops = n * network_flops_per_sample(width, hidden)
    return {"samples_per_s": n / t, "ms": t * 1e3, "flops_per_sample": flops / n,
            "achieved_tflops": flops / t / 1e12, "peak_tflops": BF16_PEAK_TFLOPS,
            "frac": flops / t / 1e12 / BF16_PEAK_TFLOPS}


def experiment(conv: Convolver, nside: int, sky, beam, half_span_tan: float, det_params, norm_scale: float,
               r_main: float, r_full: float, test, n_train: int = 1_000_000, epochs: int = 40, batch: int = 8192,
               lr: float = 2e-3, lr_end: float = 2e-5, width: int = 256, hidden: int = 4, seed: int = 1) -> dict:
    """Train the library's far-sidelobe network of a detector and judge it.

    sky: (I, Q, U) float32 RING maps; beam: n x n scalar beam (float32) with
    det_params = (zeta, eps, s) and FIXED normalisation norm_scale; test:
    (theta, phi, psi) float64 held-out pointings.  The library draws n_train
    training pointings itself and trains on their exact annulus pickups
    (pisco_sidelobe_train).  Detector slots: 0 the detector (disc r_full; its
    network stands in for (r_main, r_full] once enabled), 1 the exact main disc,
    2 the exact annulus pickup at zeta = 0.  Errors are relative to RMS(d_main).
    """
    import torch

    zeta, eps, s = det_params
    conv.set_sky(nside, *(torch.as_tensor(np.asarray(m, dtype=np.float32)).cuda() for m in sky),
                 dtype=torch.float32)
    b = torch.as_tensor(np.asarray(beam, dtype=np.float32)).cuda()
    wI, wQ = 0.5 * s * (1 + eps), 0.5 * s * (1 - eps)
    conv.set_beam_scalar(0, b.shape[0], half_span_tan, b, wI, wQ, 0.0, 1.0, dtype=torch.float32)
    for k in (1, 2):
        conv.share_beam(k, 0)
    for k, (z, r0, r1) in enumerate([(zeta, 0.0, r_full), (zeta, 0.0, r_main), (0.0, r_main, r_full)]):
        conv.set_detector(k, z, r0, r1, L.NORM_FIXED, norm_scale)
    keep = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in test]
    for k in range(3):
        conv.set_pointing(k, *keep)
    conv.sidelobe_options(width=width, hidden_layers=hidden, batch=batch, lr=lr, lr_end=lr_end)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = conv.sidelobe_train(0, r_main, n_train, seed, epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    # held-out judgement by the exact path
    conv.sidelobe_enable(0, False)
    d_full = conv.convolve(0).double()
    d_main = conv.convolve(1).double()
    p_ann = conv.convolve(2, out_mode=L.OUT_STOKES).double()
    conv.sidelobe_enable(0, True)
    d_sur = conv.convolve(0).double()
    cvec = torch.tensor(detector_coef(zeta, eps, s), dtype=torch.float64, device=d_main.device)
    d_sl = p_ann @ cvec
    d_sl_hat = d_sur - d_main
    ref = rms(d_main)
    res = {
        "sidelobe_error": rms(d_sl_hat - d_sl) / ref,
        "main_only_error": rms(d_sl) / ref,
        "split_identity_error": rms(d_main + d_sl - d_full) / rms(d_full),
        "train_samples": int(n_train), "test_samples": int(d_main.numel()), "epochs": epochs,
        "loss_first_last": [hist[0], hist[-1]], "final_loss": hist[-1], "train_s": t_train,
    }

    # rates over the held-out pointings: exact disc, exact main disc, main disc + network
    n = d_main.numel()
    out = torch.empty(n, dtype=torch.float32, device=d_main.device)
    conv.sidelobe_enable(0, False)
    t_full = time_call(lambda: conv.convolve(0, out=out))
    t_main = time_call(lambda: conv.convolve(1, out=out))
    conv.sidelobe_enable(0, True)
    t_sur = time_call(lambda: conv.convolve(0, out=out))
    res.update({"samples_per_s_exact": n / t_full, "samples_per_s_main_only": n / t_main,
                "samples_per_s_surrogate": n / t_sur, "speedup": t_full / t_sur,
                "network": network_rate(conv, 1, width, hidden)})
    conv.sidelobe_enable(0, False)
    del keep
    return res
