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

Everything runs on the device through the C ABI (targets: the convolution
kernels; features, training, inference and the TOD epilogue: the network
kernels).  torch only holds buffers and shuffles training rows.
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


class SidelobeModel:
    """Network mapping (unit vector, sin psi, cos psi) to the annulus pickup P [3],
    with the standardisation of the targets it was trained on."""

    def __init__(self, conv: Convolver, width: int = 256, hidden: int = 4, max_batch: int = 16384, seed: int = 1):
        self.conv = conv
        self.net = Mlp(conv, width, hidden, max_batch, seed)
        self.mean = np.zeros(3, dtype=np.float32)
        self.std = np.ones(3, dtype=np.float32)

    def close(self):
        self.net.close()

    def targets(self, annulus_det: int):
        """Exact pickups P [n, 3] of a detector slot set to the annulus (STOKES output)."""
        return self.conv.convolve(annulus_det, out_mode=L.OUT_STOKES)

    def features(self, det: int):
        return self.net.features(det)

    def fit(self, x, p, epochs: int = 40, batch: int = 8192, lr: float = 2e-3, lr_end: float = 2e-5,
            seed: int = 0, log=None):
        """Adam on the mean squared error of standardised targets, cosine-decayed
        learning rate, reshuffled every epoch.  x [n, 5], p [n, 3] device tensors."""
        import torch

        if batch % 64 or batch > self.net.max_batch:
            raise ValueError("batch must be a multiple of 64 and at most max_batch")
        n = (x.shape[0] // batch) * batch
        if n == 0:
            raise ValueError("fewer samples than one batch")
        pm = p.double().mean(0)
        ps = p.double().std(0).clamp_min(1e-300)
        self.mean = pm.float().cpu().numpy()
        self.std = ps.float().cpu().numpy()
        t = ((p.double() - pm) / ps).float()
        g = torch.Generator(device=x.device)
        g.manual_seed(seed)
        steps = n // batch
        total = epochs * steps
        k = 0
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(x.shape[0], device=x.device, generator=g)[:n]
            xs, ts = x[perm].contiguous(), t[perm].contiguous()
            acc = torch.zeros((), dtype=torch.float64, device=x.device)
            for i in range(steps):
                cur = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * k / max(1, total - 1)))
                acc += self.net.train_step(xs[i * batch:(i + 1) * batch], ts[i * batch:(i + 1) * batch],
                                           lr=cur).double()[0]
                k += 1
            hist.append(acc.item() / steps)
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.4e}")
        return hist

    def predict(self, x):
        """P [n, 3] for features x [n, 5] (chunked by max_batch)."""
        import torch

        outs = []
        for b in range(0, x.shape[0], self.net.max_batch):
            outs.append(self.net.forward(x[b:b + self.net.max_batch]))
        y = torch.cat(outs) if outs else torch.empty((0, 3), dtype=torch.float32, device=x.device)
        dev = y.device
        return y * torch.from_numpy(self.std).to(dev) + torch.from_numpy(self.mean).to(dev)

    def apply(self, det: int, coef, tod, stream=None, conv=None):
        """tod += sum_c coef[c] P_hat[c] for detector slot det's pointing (one fused launch)."""
        return self.net.apply(det, self.mean, self.std, coef, tod, stream, conv)


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


def experiment(conv: Convolver, nside: int, sky, beam, half_span_tan: float, det_params, norm_scale: float,
               r_main: float, r_full: float, train, test, epochs: int = 40, batch: int = 8192,
               lr: float = 2e-3, width: int = 256, hidden: int = 4, seed: int = 1, log=None) -> dict:
    """Train on exact annulus pickups of the `train` pointings, judge on `test`.

    sky: (I, Q, U) float32 RING maps; beam: n x n scalar beam (float32) with
    det_params = (zeta, eps, s); train/test: (theta, phi, psi) float64 arrays
    (put in spatial order by the caller or not, results are per sample).
    Detector slots: 0 main/train, 1 annulus/train, 2 main/test, 3 annulus/test,
    4 full disc/test.  Returns errors relative to RMS(d_main) and rates.
    """
    import torch

    zeta, eps, s = det_params
    say = log or (lambda m: None)
    conv.set_sky(nside, *(torch.as_tensor(np.asarray(m, dtype=np.float32)).cuda() for m in sky),
                 dtype=torch.float32)
    b = torch.as_tensor(np.asarray(beam, dtype=np.float32)).cuda()
    wI, wQ = 0.5 * s * (1 + eps), 0.5 * s * (1 - eps)
    conv.set_beam_scalar(0, b.shape[0], half_span_tan, b, wI, wQ, 0.0, 1.0, dtype=torch.float32)
    for k in range(1, 5):
        conv.share_beam(k, 0)
    # annulus slots use zeta = 0: P is the zeta = 0 frame pickup
    for k, (z, r0, r1) in enumerate([(zeta, 0.0, r_main), (0.0, r_main, r_full), (zeta, 0.0, r_main),
                                     (0.0, r_main, r_full), (zeta, 0.0, r_full)]):
        conv.set_detector(k, z, r0, r1, L.NORM_FIXED, norm_scale)
    keep = []
    for k, pts in enumerate([train, train, test, test, test]):
        arrs = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in pts]
        conv.set_pointing(k, *arrs)
        keep.append(arrs)
    coef = detector_coef(zeta, eps, s)
    cvec = torch.tensor(coef, dtype=torch.float64, device="cuda")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model = SidelobeModel(conv, width, hidden, max(batch, 16384), seed)
    p_train = model.targets(1)
    x_train = model.features(1)
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    say(f"targets: {p_train.shape[0]} samples in {t_targets:.2f} s")

    t0 = time.perf_counter()
    hist = model.fit(x_train, p_train, epochs=epochs, batch=batch, lr=lr, seed=seed, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del x_train, p_train

    # held-out judgement by the exact path
    p_test = model.targets(3).double()
    d_main = conv.convolve(2).double()
    d_full = conv.convolve(4).double()
    d_sl = p_test @ cvec
    p_hat = model.predict(model.features(3)).double()
    d_sl_hat = p_hat @ cvec
    tod = conv.convolve(2)
    model.apply(2, coef, tod)
    ref = rms(d_main)
    res = {
        "sidelobe_error": rms(d_sl_hat - d_sl) / ref,
        "main_only_error": rms(d_sl) / ref,
        "split_identity_error": rms(d_main + d_sl - d_full) / rms(d_full),
        "apply_vs_predict": rms(tod.double() - d_main - d_sl_hat) / ref,
        "channel_rel_rms": [rms(p_hat[:, c] - p_test[:, c]) / max(rms(p_test[:, c] - p_test[:, c].mean()), 1e-300)
                            for c in range(3)],
        "train_samples": int(train[0].size), "test_samples": int(test[0].size),
        "epochs": epochs, "final_loss": hist[-1], "targets_s": t_targets, "train_s": t_train,
    }

    # rates: exact full disc vs exact main disc + network, on the test pointings
    out_full = torch.empty(int(test[0].size), dtype=torch.float32, device="cuda")
    out_main = torch.empty_like(out_full)
    t_full = time_call(lambda: conv.convolve(4, out=out_full))
    t_main = time_call(lambda: conv.convolve(2, out=out_main))
    t_sur = time_call(lambda: model.apply(2, coef, conv.convolve(2, out=out_main)))
    t_net = time_call(lambda: model.apply(2, coef, out_main))
    n = test[0].size
    flops = n * network_flops_per_sample(width, hidden)
    res.update({"samples_per_s_exact": n / t_full, "samples_per_s_main_only": n / t_main,
                "samples_per_s_surrogate": n / t_sur, "speedup": t_full / t_sur,
                "network": {"samples_per_s": n / t_net, "ms": t_net * 1e3, "flops_per_sample": flops / n,
                            "achieved_tflops": flops / t_net / 1e12, "peak_tflops": BF16_PEAK_TFLOPS,
                            "frac": flops / t_net / 1e12 / BF16_PEAK_TFLOPS}})
    model.close()
    del keep
    return res
