"""Throughput of the batched exact convolution on one MI355X.

Workload: the nside-1024 batched-detector recipe (64 detectors, each with its
own 201^2 elliptical beam, CES pointing with boresight rotation, 1e5..1e6
samples per detector, disc radius 2 deg), synthetic and seeded.  One step is
one convolution of every detector's full stream in a single persistent,
graph-replayed launch; inputs are resident in HBM before timing starts.

Prints one JSON line with samples/s (value), beam-pixel MACs/s, the roofline
of the convolution kernel (HIP events on its launch stream) and the FP64
oracle timed on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per (sample, disc pixel) pair of each tile-path loop variant,
# counted from its source (FMA = 2; add, multiply, fract, floor and reciprocal 1;
# compares, selects, conversions to integers and address arithmetic 0):
#  membership 1 - n.p 6; n.theta'_0 and n.phi'_0 12; 1/z' and 1/(1+z') as
#  series in omega, to the second and first power 5 (third and second: 9; one
#  reciprocal of z'(1+z') and the two products: 6); grid coordinates 4; cell
#  fractions 2;
#  q = (n.theta'_0) / (1 + z') 1; one-grid bilinear cell polynomial 6; times
#  the beam value 1 and the per-step sum 1; the sum of eight terms added in
#  FP64 0.25 per sum; the normaliser of a per-sample-normalised launch (its
#  masked add 1 + 0.25).  The position-angle part:
#  one-grid TOD without a plate (the quadratic-form records, in gnomonic
#  coordinates about the tile centre): n.theta'_0 and n.phi'_0 over n_z 8
#  instead of 12 (the scale 1/(1 - t) has the same series and reciprocal counts),
#  the first two tile-frame components of theta'_0 carried to the pixel 8, the
#  quadratic form 8 -> 50.25, 51.5 with the normaliser;
#  otherwise theta'_0 carried to the pixel 6, its projections on the pixel's
#  theta/phi 10, and for one-grid TOD with a plate the turn by 2 phi_t 6 and the
#  cos^2 form 5 (-> 66.5 with the normaliser); four-channel beams: floors and
#  fractions 4 instead of 2, four bilinear channels 36 instead of 6, cos 2gamma
#  and sin 2gamma 4 and the contraction with the Stokes rotation 12 -> 102.5
#  with the normaliser.
#  Matrix-core variant (algorithm 2): eight 16x16x4 FP32 MFMAs per 16 pixels x
#  16 samples give the pixel-linear quantities (64 matrix flops per pair);
#  vector ALU 44 (one-grid) / 81 (four-channel).
#  Pixel path (FP32 incoherent groups), four-channel beam: 155; one-grid: 125.
FLOPS_PER_PAIR = {(1, "scalar", 2, True): (51.5, 0), (1, "scalar", 2, False): (50.25, 0),
                  (1, "scalar", 1, True): (55.5, 0), (1, "scalar", 1, False): (54.25, 0),
                  (1, "scalar", 0, True): (52.5, 0), (1, "scalar", 0, False): (51.25, 0),
                  (1, "full", 2, True): (102.5, 0), (1, "full", 2, False): (101.25, 0),
                  (1, "full", 1, True): (106.5, 0), (1, "full", 0, True): (103.5, 0),
                  (2, "scalar"): (44, 64), (2, "full"): (81, 64), (0, "scalar"): (125, 0), (0, "full"): (155, 0)}


def flops_per_pair(algorithm, kind, rho_max, per_sample):
    """(vector, matrix) flops per pair of the loop a launch runs: the series
    order follows the disc (omega = 1 - cos rho_max <= 1e-3: second order, <= 4e-3:
    third, else the reciprocal; quadratic-form tiles also need their union radius
    within 3.6 deg for the second order, which every tile of coherence 0.5 on a
    2 deg disc meets)."""
    if algorithm != 1:
        return FLOPS_PER_PAIR[(algorithm, kind)]
    om = 2.0 * np.sin(0.5 * rho_max) ** 2
    sc = 2 if om <= 1e-3 else (1 if om <= 4e-3 else 0)
    return FLOPS_PER_PAIR.get((1, kind, sc, per_sample), FLOPS_PER_PAIR[(1, kind, sc, True)])


# FP32 vector peak of one MI355X (published): 256 CUs x 4 SIMDs x 32 FMA per
# SIMD per clock x 2 flops x 2.4 GHz = 157.3 TFLOP/s.  The build never emits
# packed FP32, but gfx950 issues plain v_fma_f32, v_add_f32 and v_mul_f32 faster
# than one wave64 instruction per four clocks (a probe of independent chains:
# 1.27x, 1.54x and 1.54x that rate), so the published figure is the ceiling of
# this loop too.  FP64 vector: 78.6 TFLOP/s (16 FMA per SIMD per clock).
ALU_PEAK_TFLOPS = 256 * 4 * 32 * 2.4e9 * 2 / 1e12
FP64_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# HBM3E bandwidth of one MI355X (published)
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_counters(launch):
    """The committed rocprofv3 counter record of the dominant kernel for this
    launch shape (HBM bytes per launch, and for the default shape the texture
    path and L1 counters), or None once a source they depend on (the kernel, the
    plan builder that orders its tiles) or the launch shape differs from the one
    the counters were taken with."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_conv_c3.json")
    try:
        rec = json.load(open(path))
        same = all(hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest() == h
                   for f, h in rec["sources_sha256"].items())
        if not same:
            return None
        for r in rec["records"]:
            if all(launch.get(k) == v for k, v in r["launch"].items()):
                return r
    except (OSError, KeyError, ValueError, AttributeError, TypeError):
        return None
    return None


def measured_traffic(launch):
    """HBM bytes per launch of the dominant kernel (see measured_counters)."""
    r = measured_counters(launch)
    return None if r is None else r.get("traffic_bytes_per_launch")


def gather_roofline(launch, pairs, k_ms):
    """The beam gathers of the one-grid tile loop (one 16-byte cell record per
    pair, from L1/L2): their rate, and from the committed counter runs how busy
    the texture path that serves them was and how many L1 lines a 64-lane gather
    touched.  None without a matching counter record."""
    r = measured_counters(launch)
    p = None if r is None else r.get("pipeline")
    if p is None:
        return None
    return {"unit": "GB/s", "bytes_per_pair": 16, "achieved": pairs * 16 / (k_ms / 1e3) / 1e9,
            "binding": "texture-data path of the L1 (beam-record gathers)",
            "td_busy": p["td_busy"], "ta_busy": p["ta_busy"], "l1_lines_per_gather": p["l1_lines_per_gather"],
            "l1_miss_frac": p["l1_miss_frac"]}


def load(conv, w, torch):
    from paper_1908_05662_amd.beamsor import fold_elements, scalar_weights

    conv.set_sky(w.nside, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in w.sky), dtype=torch.float32)
    keep, kinds = [], set()
    for k, d in enumerate(w.detectors):
        bI, bQ, bU, bT = fold_elements(d.beam.elements, d.beam.n, d.det.eps, d.det.s)
        wts = scalar_weights(bI, bQ, bU, bT)
        if wts is not None:
            conv.set_beam_scalar(k, d.beam.n, d.beam.half_span_tan, bT, *wts, 1.0, dtype=torch.float32)
            kinds.add("scalar")
        else:
            conv.set_beam(k, d.beam.n, d.beam.half_span_tan, bI, bQ, bU, bT, dtype=torch.float32)
            kinds.add("full")
        conv.set_detector(k, d.det.zeta, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale)
        arrs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (d.theta, d.phi, d.psi)]
        conv.set_pointing(k, *arrs)
        keep.append(arrs)
    assert len(kinds) == 1
    return keep, kinds.pop()


def cpu_baseline(w, got, seconds):
    """FP64 oracle on an evenly spread sample of every detector's stream; only
    the oracle calls are timed (inputs are prepared beforehand)."""
    import oracle

    offs = np.cumsum([0] + [d.n for d in w.detectors])
    sky = [m.astype(np.float32).astype(np.float64) for m in w.sky]
    beams = [d.beam.dense().astype(np.float32).astype(np.float64) for d in w.detectors]

    def run(per_det):
        tot_s, errs, dt = 0, [], 0.0
        for k, d in enumerate(w.detectors):
            idx = np.linspace(0, d.n - 1, per_det).astype(np.int64)
            th, ph, ps = d.theta[idx], d.phi[idx], d.psi[idx]
            t = time.perf_counter()
            want = oracle.tod(w.nside, *sky, beams[k], d.beam.half_span_tan, d.det.zeta, d.det.eps, d.det.s,
                              d.rho_min, d.rho_max, d.norm_mode, d.norm_scale, th, ph, ps)
            dt += time.perf_counter() - t
            g = got[offs[k] + idx].astype(np.float64)
            errs.append((np.abs(g - want).max(), np.abs(want).max()))
            tot_s += idx.size
        return tot_s, errs, dt

    n_cal, _, dt_cal = run(max(2, oracle.max_threads()))
    per_sample = dt_cal / n_cal
    per_det = int(max(2, min(4000, seconds / max(per_sample, 1e-7) / len(w.detectors))))
    n, errs, dt = run(per_det)
    err = max(e for e, _ in errs) / max(m for _, m in errs)
    return n, dt, err, per_det


def host_info():
    """Logical CPUs and model name of this host (nproc, lscpu)."""
    import subprocess

    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def valu_probe():
    """Issue rates of the vector ALU on this device from the probe program built
    beside the library (wave64 instructions/s and their ratio to one per four
    clocks per SIMD), or None without it."""
    import subprocess

    exe = os.path.join(ROOT, "paper_1908_05662_amd", "valu_probe")
    try:
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120).stdout
        return json.loads(out.strip().splitlines()[-1])
    except (OSError, ValueError, IndexError, subprocess.SubprocessError):
        return None


def load_any(conv, w, dtype, torch, dets=None):
    """Sky, beams (one-grid form when the folded channels allow it), detector
    parameters and device pointing of workload w in precision dtype."""
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    conv.set_sky(w.nside, *(torch.from_numpy(np.asarray(m, dtype=dtype)).cuda() for m in w.sky), dtype=tdt)
    keep = []
    for k in (range(len(w.detectors)) if dets is None else dets):
        d = w.detectors[k]
        conv.set_beamsor(k, d.beam.dense(), d.beam.half_span_tan, d.det.eps, d.det.s, dtype=tdt)
        conv.set_detector(k, d.det.zeta, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale)
        arrs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (d.theta, d.phi, d.psi)]
        conv.set_pointing(k, *arrs)
        keep.append(arrs)
    return keep


def oracle_samples(w, k, idx, dtype, out_mode=0, rho_min=None, rho_max=None, beam=None, zeta=None):
    """The FP64 oracle on detector k's samples idx, the sky and beam rounded as the GPU holds them."""
    import oracle

    d = w.detectors[k]
    sky = [np.asarray(m, dtype=dtype).astype(np.float64) for m in w.sky]
    M = d.beam.dense() if beam is None else beam
    M = np.asarray(M, dtype=dtype).astype(np.float64)
    return oracle.tod(w.nside, *sky, M, d.beam.half_span_tan, d.det.zeta if zeta is None else zeta, d.det.eps,
                      d.det.s, d.rho_min if rho_min is None else rho_min, d.rho_max if rho_max is None else rho_max,
                      d.norm_mode, d.norm_scale, d.theta[idx], d.phi[idx], d.psi[idx], out_mode)


def rel_inf(got, want):
    got, want = np.asarray(got, dtype=np.float64), np.asarray(want, dtype=np.float64)
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


def parity_leg():
    """Relative TOD error of the GPU against the FP64 oracle, per workload recipe,
    ||d_gpu - d_oracle||_inf / ||d_oracle||_inf over the compared samples (the
    nside-1024 batched recipe is checked inside the headline run, the nside-2048
    one inside the full-scale leg)."""
    import torch

    from paper_1908_05662_amd import OUT_STOKES
    from paper_1908_05662_amd.api import Convolver
    from paper_1908_05662_amd.surrogate import spatial_order
    from synth import workloads as W

    res = {}
    t0 = time.perf_counter()
    # nside 64, FP64 kernel, the whole 1e5-sample stream
    w = W.c1()
    conv = Convolver(0)
    keep = load_any(conv, w, np.float64, torch)
    got = conv.convolve(0).cpu().numpy()
    conv.close()
    res["c1_nside64_fp64"] = {"max_rel_err": rel_inf(got, oracle_samples(w, 0, slice(None), np.float64)),
                              "samples": int(got.size), "of": int(got.size), "tolerance": 1e-12,
                              "path": "FP64 pixel path"}
    # nside 512, FP32 tile path, the whole 1e7-sample stream; 10,000 samples spread over it
    w = W.c2()
    d = w.detectors[0]
    conv = Convolver(0)
    keep = load_any(conv, w, np.float32, torch)
    got = conv.convolve(0).cpu().numpy()
    conv.close()
    idx = np.unique(np.concatenate([np.linspace(0, d.n - 1, 10_001).astype(np.int64), [63, 64, d.n - 1]]))
    res["c2_nside512_fp32"] = {"max_rel_err": rel_inf(got[idx], oracle_samples(w, 0, idx, np.float32)),
                               "samples": int(idx.size), "of": int(d.n), "tolerance": 1e-6,
                               "path": "FP32 tile path (pixel path for incoherent groups)"}
    # nside 256 far-sidelobe recipe, 1e6 held-out isotropic pointings in spatial order:
    # the 20 deg disc, the 5 deg main disc and the (5, 20] deg annulus pickups
    w = W.c4(1_000_000, stream=2)
    d = w.detectors[0]
    o = spatial_order(d.theta, d.phi)
    d.theta, d.phi, d.psi = d.theta[o], d.phi[o], d.psi[o]
    r_main = w.meta["r_main"]
    conv = Convolver(0)
    keep = load_any(conv, w, np.float32, torch)
    idx = np.unique(np.concatenate([np.linspace(0, d.n - 1, 400).astype(np.int64), [63, 64]]))
    full = conv.convolve(0).cpu().numpy()[idx]
    conv.set_detector(0, d.det.zeta, 0.0, r_main, d.norm_mode, d.norm_scale)
    main = conv.convolve(0).cpu().numpy()[idx]
    conv.set_detector(0, 0.0, r_main, d.rho_max, d.norm_mode, d.norm_scale)
    ann = conv.convolve(0, out_mode=OUT_STOKES).cpu().numpy()[idx]
    conv.close()
    del keep
    e_full = rel_inf(full, oracle_samples(w, 0, idx, np.float32))
    e_main = rel_inf(main, oracle_samples(w, 0, idx, np.float32, rho_max=r_main))
    e_ann = rel_inf(ann, oracle_samples(w, 0, idx, np.float32, out_mode=OUT_STOKES, rho_min=r_main, zeta=0.0))
    res["c4_nside256_fp32"] = {"max_rel_err": max(e_full, e_main, e_ann), "full_disc": e_full, "main_disc": e_main,
                               "annulus_stokes": e_ann, "samples": int(idx.size), "of": int(d.n),
                               "tolerance": 1e-6, "path": "FP32 tile path"}
    log(f"parity: " + ", ".join(f"{k} {v['max_rel_err']:.2e}" for k, v in res.items()) +
        f" ({time.perf_counter() - t0:.1f}s)")
    return res


def full_beam_leg(conv, w, stream, out, steps, warmup, torch, pairs):
    """The benchmark workload with four-channel beams: every beamsor gains a
    four-lobed cross-polar leakage B_QU = B_UQ = 0.01 b cos 2 sigma, so the folded
    channels are no longer multiples of one grid and each pair reads the four
    bilinear channels.  Timed like the headline; the one-grid beams return after."""
    from paper_1908_05662_amd import OUT_TOD
    from synth import beams as B

    T, u, v, rho, sig = B.tangent_grid(w.detectors[0].beam.n, np.deg2rad(2.0))
    lobes = np.cos(2.0 * sig)
    for k, d in enumerate(w.detectors):
        g = d.beam.get(0, 0)
        el = dict(d.beam.elements)
        el[(1, 2)] = 0.01 * g * lobes
        el[(2, 1)] = 0.01 * g * lobes
        kind = conv.set_beamsor(k, B.Beamsor(d.beam.n, d.beam.half_span_tan, el).dense(), d.beam.half_span_tan,
                                d.det.eps, d.det.s, dtype=torch.float32)
        assert kind == "full"
    conv.set_timing(True)
    for _ in range(max(warmup, 1)):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    conv.kernel_time(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = conv.kernel_time(reset=True)
    k_ms = kms / max(launches, 1)
    got = out.cpu().numpy()
    # sampled parity of the four-channel path
    offs = np.cumsum([0] + [d.n for d in w.detectors])
    errs = []
    for k in range(0, len(w.detectors), 8):
        d = w.detectors[k]
        el = dict(d.beam.elements)
        el[(1, 2)] = 0.01 * d.beam.get(0, 0) * lobes
        el[(2, 1)] = 0.01 * d.beam.get(0, 0) * lobes
        idx = np.array([0, 63, 64, d.n // 2, d.n - 1])
        want = oracle_samples(w, k, idx, np.float32, beam=B.Beamsor(d.beam.n, d.beam.half_span_tan, el).dense())
        errs.append(rel_inf(got[offs[k] + idx], want))
    for k, d in enumerate(w.detectors):   # back to the one-grid beams
        conv.set_beamsor(k, d.beam.dense(), d.beam.half_span_tan, d.det.eps, d.det.s, dtype=torch.float32)
    fpp, _ = flops_per_pair(1, "full", w.detectors[0].rho_max, True)
    achieved = fpp * pairs / (k_ms / 1e3) / 1e12
    n = conv.output_samples(-1)
    log(f"four-channel beams: {wall * 1e3 / steps:.2f} ms/step, kernel {k_ms:.2f} ms, frac {achieved / ALU_PEAK_TFLOPS:.3f}")
    return {"workload": "the benchmark workload with four-channel beams (cross-polar leakage 0.01 b cos 2 sigma "
                        "in B_QU and B_UQ)", "ms_per_step": wall * 1e3 / steps, "kernel_ms": k_ms,
            "samples_per_s": n / (wall / steps), "macs_per_s": pairs / (wall / steps),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / ALU_PEAK_TFLOPS, "flops_per_pair": fpp},
            "parity_max_rel_err": max(errs), "parity_samples": 5 * len(errs)}


def network_leg(torch):
    """Training-step and fused-inference rates of the sidelobe network for both
    sizes the bench uses (4 x 256 on the nside-256 workload, 10 x 512 at full
    scale): one Adam step on a batch of 8192 (forward, loss, backward, fixed-order
    gradient sums, Adam; three times the forward flops), and the fused TOD
    epilogue over 1e6 pointings (features, every layer, the TOD sum), HIP
    events.  Against the dense BF16 matrix-core peak."""
    from paper_1908_05662_amd import surrogate as SG
    from paper_1908_05662_amd.api import Convolver, Mlp
    from synth import workloads as W

    conv = Convolver(0)
    w = W.c4(1_000_000, stream=2)
    d = w.detectors[0]
    T, g = W.sidelobe_beam(401, 20.0, 1.0)
    conv.set_sky(w.nside, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in w.sky), dtype=torch.float32)
    conv.set_beam_scalar(0, 401, T, torch.from_numpy(g.astype(np.float32)).cuda(), 0.5, 0.5, 0.0, 1.0,
                         dtype=torch.float32)
    conv.set_detector(0, 0.0, 0.0, np.deg2rad(5.0), W.NORM_FIXED, d.norm_scale)
    conv.set_pointing(0, *(torch.from_numpy(v).cuda() for v in (d.theta, d.phi, d.psi)))
    res = {}
    gen = torch.Generator(device="cuda").manual_seed(5)
    for (H, L) in ((256, 4), (512, 10)):
        batch = 8192
        m = Mlp(conv, H, L, max_batch=batch, seed=1)
        x = torch.randn(batch, 5, device="cuda", generator=gen)
        t = torch.randn(batch, 3, device="cuda", generator=gen)
        t_step = SG.time_call(lambda: m.train_step(x, t, lr=1e-4), reps=50)
        m.close()
        fwd = SG.network_flops_per_sample(H, L)
        inf = SG.network_rate(conv, 0, H, L)
        res[f"{L}x{H}"] = {
            "train_step_ms": t_step * 1e3, "train_batch": batch,
            "train_tflops": 3 * fwd * batch / t_step / 1e12,
            "train_frac": 3 * fwd * batch / t_step / 1e12 / SG.BF16_PEAK_TFLOPS,
            "infer_ms_per_1e6": inf["ms"] * 1e6 / d.n, "infer_tflops": inf["achieved_tflops"],
            "infer_frac": inf["frac"], "flops_per_sample": fwd}
        log(f"network {L}x{H}: train step {t_step * 1e3:.3f} ms ({res[f'{L}x{H}']['train_tflops']:.1f} TFLOP/s), "
            f"inference {inf['ms']:.3f} ms per {d.n} ({inf['achieved_tflops']:.1f} TFLOP/s, frac {inf['frac']:.3f})")
    conv.close()
    res["peak_tflops"] = SG.BF16_PEAK_TFLOPS
    res["note"] = "training counts 3x the forward flops per sample; inference is the fused TOD epilogue"
    return res


def surrogate_leg(epochs):
    """Exact main beam + the library-trained far-sidelobe network against the
    exact 20 deg disc on the nside-256 far-sidelobe workload: the library draws
    1e6 training pointings uniform on the sphere and trains on their exact
    annulus pickups; 1e6 held-out pointings (put in spatial order) judge it
    against the exact annulus convolution."""
    from paper_1908_05662_amd import surrogate as SG
    from paper_1908_05662_amd.api import Convolver
    from synth import workloads as W

    wte = W.c4(1_000_000, stream=2)
    d = wte.detectors[0]
    o = SG.spatial_order(d.theta, d.phi)
    T, g = W.sidelobe_beam(401, 20.0, 1.0)
    conv = Convolver(0)
    r = SG.experiment(conv, wte.nside, wte.sky, g, T, (d.det.zeta, d.det.eps, d.det.s), d.norm_scale,
                      wte.meta["r_main"], d.rho_max, (d.theta[o], d.phi[o], d.psi[o]), n_train=1_000_000,
                      epochs=epochs)
    conv.close()
    r["workload"] = ("nside-256 smooth sky, 401^2 beam over +-20 deg (1 deg Gaussian + -40 dB ring at 10 deg), "
                     "main disc 5 deg, annulus (5, 20] deg; network 5 -> 4 x 256 SiLU -> 3, BF16 weights, trained "
                     "by the library (pisco_sidelobe_train) on 1e6 drawn pointings")
    r["error_unit"] = "RMS(d_sl_hat - d_sl) / RMS(d_main) on held-out samples"
    log(f"surrogate: sidelobe error {r['sidelobe_error']:.3e} (main only {r['main_only_error']:.3e}), "
        f"{r['samples_per_s_surrogate']:.4g} vs exact {r['samples_per_s_exact']:.4g} samples/s, "
        f"training {r['train_s']:.1f}s")
    return r


# Wall times of the paper's whole-sky benchmark (Sec. 5.3, Table 1): one PSB (2
# detectors, Gaussian FWHM 1.5 deg) at every nside-128 pixel centre and psi in
# {0, 45, 90} deg, 1,179,648 samples, on one GTX 1080, including the assembly
# of the beam interpolation grid and host-device copies.  Context, not a target.
PAPER_TABLE1 = [(5.0, 374, 1471.41), (7.5, 832, 3135.19), (10.0, 1506, 5560.25), (15.0, 3360, 12719.56),
                (20.0, 5938, 23190.68), (25.0, 9218, 39447.70), (30.0, 13174, 53800.74)]


def paper_shape_leg():
    """The paper's benchmark workload on this GPU: the same sample pattern and disc
    radii (synthetic nside-128 sky, 0.1 deg tangent grid over +-rho_max, per-sample
    normalisation).  Timed kernel-only (inputs resident) in the given sample order,
    which the library processes in its own spatial order (the given ring order puts
    ~29 deg between the ends of a 64-sample group), and again with that ordering
    switched off (such groups then run on the pixel path); in Hilbert order supplied
    by the caller; and end to end from host arrays in the given order (pointing and
    beam upload, plan, convolution, TOD download)."""
    import torch

    from paper_1908_05662_amd import OUT_COUNT, OUT_TOD
    from paper_1908_05662_amd.api import Convolver
    from paper_1908_05662_amd.surrogate import spatial_order
    from synth import workloads as W

    sky = W.sky_for(128, 383, 2.0, 6)
    from synth import beams as B

    beam_map = B.healpix_beam_map(512, np.deg2rad(1.5), rho_max_rad=np.deg2rad(40.0)).astype(np.float32)
    rows = []
    conv = Convolver(0)
    conv.set_sky(128, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in sky), dtype=torch.float32)
    stream = torch.cuda.Stream()

    def run(out):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
        stream.synchronize()

    def kernel_time(out, reps=3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            a.record(stream)
            for _ in range(reps):
                conv.convolve(-1, OUT_TOD, out=out, stream=stream)
            b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / reps / 1e3

    for rho, n_pix, paper_ms in PAPER_TABLE1:
        w = W.paper_shape(rho, nside=128, sky=sky)
        n = w.n_samples
        out = torch.empty(n, dtype=torch.float32, device="cuda")

        def upload(order=None):
            for k, d in enumerate(w.detectors):
                conv.set_beamsor(k, d.beam.dense(), d.beam.half_span_tan, d.det.eps, d.det.s, dtype=torch.float32)
                conv.set_detector(k, d.det.zeta, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale)
                pts = (d.theta, d.phi, d.psi) if order is None else (d.theta[order], d.phi[order], d.psi[order])
                conv.set_pointing(k, *pts)   # host arrays: copied

        upload()
        run(out)                       # plan, graph
        t0 = time.perf_counter()
        upload()
        run(out)
        host = out.cpu().numpy()
        t_e2e = time.perf_counter() - t0
        # the same, with each detector's beam given as the paper gives it: a HEALPix map of nside 512
        # (host array), resampled by the library onto the same grid
        d0 = w.detectors[0]
        n_grid, T_grid = d0.beam.n, d0.beam.half_span_tan

        def upload_hpx():
            for k, d in enumerate(w.detectors):
                conv.set_beam_healpix_scalar(k, 512, n_grid, T_grid, beam_map, 0.5 * d.det.s * (1 + d.det.eps),
                                             0.5 * d.det.s * (1 - d.det.eps), 0.0, 1.0, dtype=torch.float32)
                conv.set_detector(k, d.det.zeta, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale)
                conv.set_pointing(k, d.theta, d.phi, d.psi)

        upload_hpx()
        run(out)
        t0 = time.perf_counter()
        upload_hpx()
        run(out)
        _ = out.cpu().numpy()
        t_e2e_hpx = time.perf_counter() - t0
        pairs = float(conv.convolve(-1, OUT_COUNT).double().sum())
        t_given = kernel_time(out)               # given order; the library processes it in spatial order
        conv.set_ordering("given")
        run(out)
        t_given_raw = kernel_time(out)           # given order processed as given
        conv.set_ordering("auto")
        del host
        # the same samples in Hilbert order
        order = spatial_order(w.detectors[0].theta, w.detectors[0].phi)
        upload(order)
        run(out)
        t_hil = kernel_time(out)
        rows.append({"rho_max_deg": rho, "pixels_max_paper": n_pix, "pairs_per_sample": pairs / n,
                     "kernel_ms_given_order": t_given * 1e3, "kernel_ms_given_order_unsorted": t_given_raw * 1e3,
                     "kernel_ms_hilbert_order": t_hil * 1e3,
                     "end_to_end_ms_given_order": t_e2e * 1e3, "paper_ms": paper_ms,
                     "end_to_end_ms_healpix_beam_nside512": t_e2e_hpx * 1e3,
                     "speedup_end_to_end": paper_ms / (t_e2e * 1e3),
                     "pairs_per_s_hilbert_order": pairs / t_hil})
        log(f"paper shape rho {rho}: kernel {t_given * 1e3:.2f} ms given order ({t_given_raw * 1e3:.2f} ms processed "
            f"unsorted), {t_hil * 1e3:.2f} ms Hilbert "
            f"order; end to end {t_e2e * 1e3:.1f} ms, {t_e2e_hpx * 1e3:.1f} ms from a HEALPix beam map (paper "
            f"{paper_ms} ms on a GTX 1080)")
    conv.close()
    return {"workload": "the paper's whole-sky benchmark pattern: 2 detectors x 3 psi x 196,608 nside-128 pixel "
                        "centres = 1,179,648 samples, Gaussian FWHM 1.5 deg, per-sample normalisation",
            "paper_hardware": "1x NVIDIA GTX 1080, wall time incl. beam-grid assembly and host-device copies",
            "rows": rows}


def ideal_cmb_leg():
    """The paper's whole-sky ideal CMB run (Sec. 6.2) in its own configuration,
    wall time of one simulation from host arrays: an nside-512 I, Q, U sky (a
    CMB-like E-only realisation, synthesised beforehand: the sky generator is not
    part of the pipeline, as the paper's synfast step is not), the 1.5 deg
    Gaussian as an nside-2048 HEALPix beam map (resampled by the library), one
    detector at every nside-128 pixel centre and psi = 0, 45, 90 deg (589,824
    samples, FP32 convolution), binned nside-128 maps and the six spectra to
    lmax 383 with three Jacobi steps (FP64)."""
    import torch

    from paper_1908_05662_amd.api import Convolver, MapMaker, Spectra
    from synth import beams as B
    from synth import scans as SC
    from synth import sky as SK
    from synth import workloads as W

    d2r = np.pi / 180.0
    cl = SK.cmb_like_cl(1535)
    (I, Q, U), _ = SK.make_teb_sky(512, 1535, cl, seed=W.SEED_BASE + 63)
    bmap = B.healpix_beam_map(2048, 1.5 * d2r, rho_max_rad=6.0 * d2r).astype(np.float32)
    th, ph, psi = SC.pixel_centre_scan(128)
    conv = Convolver(0)
    marks = {}

    def run():
        t0 = time.perf_counter()
        conv.set_sky(512, *(torch.from_numpy(m.astype(np.float32)).cuda() for m in (I, Q, U)), dtype=torch.float32)
        conv.set_beam_healpix_scalar(0, 2048, 201, np.tan(5.0 * d2r), bmap, 0.5, 0.5, 0.0, 1.0, dtype=torch.float32)
        conv.set_detector(0, 0.0, 0.0, 5.0 * d2r, W.NORM_PER_SAMPLE, 1.0)
        conv.set_pointing(0, th, ph, psi)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tod = conv.convolve(0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        maps, rc = MapMaker(conv, 128).add(th, ph, psi, tod, 0.0, 0.0, 1.0).solve()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out = Spectra(conv, 128, 383).anafast(maps[0], maps[1], maps[2], iterations=3).cpu().numpy()
        t4 = time.perf_counter()
        marks.update(inputs=t1 - t0, convolve=t2 - t1, maps=t3 - t2, spectra=t4 - t3, total=t4 - t0)
        return out

    run()
    out = run()
    conv.close()
    log(f"ideal CMB (paper configuration): {marks['total'] * 1e3:.1f} ms per simulation (paper: under 25 s)")
    return {"workload": "the paper's whole-sky ideal CMB run: nside-512 sky, nside-2048 HEALPix beam map "
                        "(1.5 deg Gaussian), 589,824 pixel-centre samples, nside-128 maps, spectra to lmax 383 "
                        "with 3 Jacobi steps",
            "ms_total": marks["total"] * 1e3, "ms_inputs_and_beam_resampling": marks["inputs"] * 1e3,
            "ms_convolve": marks["convolve"] * 1e3, "ms_maps": marks["maps"] * 1e3,
            "ms_spectra": marks["spectra"] * 1e3, "paper": "under 25 s on one GTX 1080",
            "bb_over_ee_max_l2_200": float(np.max(out[2, 2:201] / np.maximum(out[1, 2:201], 1e-300)))}


def plate_leg(conv, w, stream, out, steps, warmup, plain_kernel_ms, torch):
    """The benchmark workload with a rotating ideal half-wave plate on every
    detector (2 Hz at the scan's 100 Hz sampling, seeded phase per detector):
    every pair then takes its angle as 2 chi + 4 phi_t and flips the U row.
    Timed like the headline; the plates are removed afterwards."""
    from paper_1908_05662_amd import OUT_TOD

    rng = np.random.default_rng(20)
    keep = []
    for k, d in enumerate(w.detectors):
        phi = 2.0 * np.pi * 2.0 / 100.0 * np.arange(d.n) + rng.uniform(0.0, 2.0 * np.pi)
        t = torch.from_numpy(phi).cuda()
        conv.set_hwp(k, t)
        keep.append(t)
    for _ in range(max(warmup, 1)):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    conv.kernel_time(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = conv.kernel_time(reset=True)
    k_ms = kms / max(launches, 1)
    for k in range(len(w.detectors)):
        conv.set_hwp(k, None)
    n = conv.output_samples(-1)
    log(f"plate: {wall * 1e3 / steps:.2f} ms/step, kernel {k_ms:.2f} ms ({plain_kernel_ms / k_ms:.3f}x the plain rate)")
    return {"workload": "the benchmark workload with an ideal half-wave plate on every detector, 2 Hz at 100 Hz "
                        "sampling", "ms_per_step": wall * 1e3 / steps, "kernel_ms": k_ms,
            "samples_per_s": n / (wall / steps), "rate_vs_plain": plain_kernel_ms / k_ms}


def map_leg(w, keep, out, stream, torch, nside_map=1024, reps=3):
    """Binned maps of the benchmark TOD: every detector's samples accumulated
    into nside-1024 per-pixel sums (one launch per detector), then the
    per-pixel solve; HIP events on the launch stream.  HBM bytes counted: per
    sample 24 B of pointing and 4 B of TOD read; per pixel the 80-byte sums
    zeroed and read by the solve, and 32 B of maps and rcond written; per hit
    pixel the sums read and written once by the accumulation (its updates
    staying in cache)."""
    from paper_1908_05662_amd.api import MapMaker

    mm = MapMaker(keep["conv"], nside_map)
    offs = np.cumsum([0] + [d.n for d in w.detectors])

    def run():
        mm.clear()
        for k, d in enumerate(w.detectors):
            th, ph, ps = keep["pointing"][k]
            mm.add(th, ph, ps, out[offs[k]:offs[k + 1]], d.det.zeta, d.det.eps, d.det.s, stream=None)
        return mm.solve(1e-3)

    with torch.cuda.stream(stream):
        run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        with torch.cuda.stream(stream):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            maps, rc = run()
            b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    t = min(times)
    n = int(offs[-1])
    npix = 12 * nside_map * nside_map
    hit = int((mm.hits() > 0).sum().item())
    good = int((rc >= 1e-3).sum().item())
    nbytes = 28.0 * n + 80.0 * npix + 160.0 * hit + 80.0 * npix + 32.0 * npix
    log(f"maps: {t * 1e3:.2f} ms for {n} samples into nside {nside_map} ({hit} pixels hit, {good} solved for I, Q, U)")
    keep["maps"] = maps
    return {"workload": f"the benchmark TOD ({len(w.detectors)} detectors) binned into nside-{nside_map} I, Q, U maps",
            "ms": t * 1e3, "samples_per_s": n / t, "pixels_hit": hit, "pixels_iqu": good,
            "hbm_bytes": nbytes, "achieved_gbs": nbytes / t / 1e9, "peak_gbs": HBM_PEAK_GBS,
            "frac": nbytes / t / 1e9 / HBM_PEAK_GBS}


SHT_FLOPS_PER_ITEM = 33   # per (l, m, ring pair): recurrence 4; lambda scaling 2; T 4; W 6, X 5; E 6, B 6


def spectra_leg(conv, maps, torch, lmax=3071, reps=5):
    """Spectra of the map leg's nside-1024 I, Q, U maps (the validation step the
    maps go through): harmonic analysis to lmax 3071 and the six spectra, FP64,
    HIP events on the current stream; also the synthesis (alm2map) and the
    analysis refined by three Jacobi steps.  The roofline of the analysis
    (`roofline`) counts the work the a_lm kernel executes: its VALU wave
    instructions per analysis from the committed counter run (valid while the
    kernel source is the one counted), against one FP64 wave64 instruction per
    four clocks per SIMD.  `dense_equivalent_tflops` (33 flops for every
    (l, m, ring pair) of the triangle, skipped polar pairs included) is a rate
    for comparison only."""
    from paper_1908_05662_amd.api import Spectra

    nside = int(round(np.sqrt(maps.shape[1] / 12)))
    sp = Spectra(conv, nside, lmax)
    T, Q, U = maps[0], maps[1], maps[2]
    sp.anafast(T, Q, U)
    torch.cuda.synchronize()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps / 1e3

    t_alm = timed(lambda: sp.map2alm(T, Q, U))
    t_all = timed(lambda: sp.anafast(T, Q, U))
    aT, aE, aB = (x.clone() for x in sp.map2alm(T, Q, U))
    t_syn = timed(lambda: sp.alm2map(aT, aE, aB))
    t_it3 = timed(lambda: sp.anafast(T, Q, U, iterations=3))
    cl = sp.anafast(T, Q, U).cpu().numpy()
    items = sum((lmax - m + 1) * 2 * nside for m in range(lmax + 1))
    dense = SHT_FLOPS_PER_ITEM * items / t_alm / 1e12
    roof = None
    rec = counted_instructions("spectra_counters.json")
    if rec is not None and rec.get("nside") == nside and rec.get("lmax") == lmax:
        issue = rec["alm_kernel_valu_wave_instructions"] / (rec["alm_kernel_ms"] * 1e-3)
        roof = {"bound": "alu (fp64)", "achieved": issue, "unit": "wave64 VALU instructions/s",
                "peak": FP64_ISSUE_PEAK, "frac": issue / FP64_ISSUE_PEAK,
                "counted_ms": rec["alm_kernel_ms"], "instructions": rec["alm_kernel_valu_wave_instructions"]}
    log(f"spectra: nside {nside} lmax {lmax}: map2alm {t_alm * 1e3:.2f} ms, anafast {t_all * 1e3:.2f} ms "
        f"({dense:.1f} TFLOP/s dense-equivalent), alm2map {t_syn * 1e3:.2f} ms, anafast with 3 iterations "
        f"{t_it3 * 1e3:.2f} ms")
    return {"workload": f"the map leg's nside-{nside} I, Q, U maps: harmonic analysis to lmax {lmax} and the six "
                        "spectra TT, EE, BB, TE, EB, TB (FP64)",
            "ms_map2alm": t_alm * 1e3, "ms_anafast": t_all * 1e3, "ms_alm2map": t_syn * 1e3,
            "ms_anafast_3_iterations": t_it3 * 1e3, "items": items,
            "dense_equivalent_tflops": dense, "roofline": roof, "finite": bool(np.all(np.isfinite(cl)))}


def counted_instructions(name):
    """A committed counter record from profiles/ if the kernel source it names is
    unchanged since the counters were taken, else None."""
    import hashlib

    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        sha = hashlib.sha256(open(os.path.join(ROOT, rec["source"]), "rb").read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    return rec if sha == rec.get("source_sha256") else None


# FP64 VALU issue peak: one wave64 instruction per four clocks per SIMD at 2.4 GHz
FP64_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def full_scale_leg(epochs, n_train, width, hidden, lr):
    """The nside-2048 full-scale workload on one GPU: 256 detectors x 390,625 CES
    samples (1e8), each its own 151^2 elliptical main beam (disc 1.5 deg), plus
    the shared -40 dB ring at 10 deg on a 401^2 grid over +-20 deg for the
    annulus (1.5, 20] deg.  The library trains one network on the ring grid's
    annulus (pisco_sidelobe_train on a slot without pointing) and every detector
    uses it (pisco_sidelobe_share / pisco_sidelobe_enable): one batched graph
    launch runs the exact main beams and adds the network.  Against the exact
    form (exact main beams + exact annulus): the annulus is timed on 1024 samples
    of every detector (four runs of 256 consecutive samples, 262,144 in all, also
    the held-out set) and its rate extrapolated to the whole job."""
    import torch

    from paper_1908_05662_amd import OUT_STOKES, OUT_TOD
    from paper_1908_05662_amd import surrogate as SG
    from paper_1908_05662_amd.api import Convolver
    from synth import workloads as W

    t0 = time.perf_counter()
    w = W.c5()
    n = w.n_samples
    log(f"full scale: {len(w.detectors)} detectors, {n} samples, nside {w.nside}, setup {time.perf_counter() - t0:.1f}s")
    r_main = w.meta["r_main"]
    d0 = w.detectors[0]
    norm = d0.norm_scale
    stream = torch.cuda.Stream()
    cm = Convolver(0)
    keep, kind = load(cm, w, torch)
    out = torch.empty(n, dtype=torch.float32, device="cuda")

    def timed_launch():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            cm.convolve(-1, OUT_TOD, out=out, stream=stream)     # capture or warm-up
        stream.synchronize()
        with torch.cuda.stream(stream):
            a.record(stream)
            cm.convolve(-1, OUT_TOD, out=out, stream=stream)
            b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / 1e3

    # exact main beams over the whole job
    t_main = timed_launch()
    d_main_all = out.clone()
    log(f"main exact: {t_main:.3f} s for {n} samples")

    # one network for the shared ring grid's annulus, trained by the library
    R = len(w.detectors)
    T, g = W.sidelobe_beam(401, 20.0, 0.25)
    cm.set_beam_scalar(R, 401, T, torch.from_numpy(g.astype(np.float32)).cuda(), 0.5, 0.5, 0.0, 1.0,
                       dtype=torch.float32)
    cm.set_detector(R, 0.0, 0.0, np.deg2rad(20.0), W.NORM_FIXED, norm)
    cm.sidelobe_options(width=width, hidden_layers=hidden, batch=8192, lr=lr, lr_end=2e-5)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = cm.sidelobe_train(R, r_main, n_train, 1, epochs)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"library training (targets included): {n_train} samples, {epochs} epochs in {t_train:.1f} s, "
        f"loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    for k in range(R):
        cm.sidelobe_share(k, R)
        cm.sidelobe_enable(k, True)
    # surrogate form over the whole job: exact main beams + the network, one graph launch
    t_sur = timed_launch()
    d_sur_all = out.clone()

    # held-out judgement: exact annulus pickups (zeta = 0) of 262,144 scan samples
    offs = np.cumsum([0] + [d.n for d in w.detectors])
    idx, det_of = [], []
    for k, d in enumerate(w.detectors):
        for q in range(4):
            s0 = (q * d.n) // 4
            idx.append(offs[k] + s0 + np.arange(256))
            det_of.append(np.full(256, k))
    idx = np.concatenate(idx)
    det_of = np.concatenate(det_of)
    all_th = np.concatenate([d.theta for d in w.detectors])
    all_ph = np.concatenate([d.phi for d in w.detectors])
    all_ps = np.concatenate([d.psi for d in w.detectors])
    held = [torch.from_numpy(np.ascontiguousarray(x[idx])).cuda() for x in (all_th, all_ph, all_ps)]
    A = R + 1
    cm.share_beam(A, R)
    cm.set_detector(A, 0.0, r_main, np.deg2rad(20.0), W.NORM_FIXED, norm)
    cm.set_pointing(A, *held)
    p_held = cm.convolve(A, OUT_STOKES).double()
    coef = np.array([SG.detector_coef(d.det.zeta, d.det.eps, d.det.s) for d in w.detectors])
    cvec = torch.from_numpy(coef[det_of]).cuda()
    d_sl = (p_held * cvec).sum(1)
    sel = torch.from_numpy(idx).cuda()
    d_main = d_main_all[sel].double()
    d_sl_hat = d_sur_all[sel].double() - d_main
    ref = SG.rms(d_main)
    err = SG.rms(d_sl_hat - d_sl) / ref
    err0 = SG.rms(d_sl) / ref
    # exact annulus rate on the held-out runs
    ann_out = torch.empty(idx.size, dtype=torch.float32, device="cuda")
    t_ann = SG.time_call(lambda: cm.convolve(A, OUT_TOD, out=ann_out), reps=2)
    per_sample_ann = t_ann / idx.size
    log(f"full scale: sidelobe error {err:.3e} (main only {err0:.3e})")

    # sampled parity of this recipe against the oracle: main beams and annulus pickups
    main_np = d_main_all.cpu().numpy()
    e_main = 0.0
    n_main = 0
    for k in range(0, R, 8):
        d = w.detectors[k]
        j = np.unique(np.array([0, 1, 63, 64, 127, 128, d.n // 2, d.n - 1]))
        e_main = max(e_main, rel_inf(main_np[offs[k] + j], oracle_samples(w, k, j, np.float32)))
        n_main += j.size
    jj = np.arange(0, idx.size, idx.size // 32)[:32]
    ring = B_ideal(g, T)
    import oracle

    sky = [np.asarray(m, dtype=np.float32).astype(np.float64) for m in w.sky]
    want = oracle.tod(w.nside, *sky, ring, T, 0.0, 0.0, 1.0, r_main, np.deg2rad(20.0), W.NORM_FIXED, norm,
                      all_th[idx[jj]], all_ph[idx[jj]], all_ps[idx[jj]], OUT_STOKES)
    e_ann = rel_inf(p_held.cpu().numpy()[jj], want)
    parity = {"max_rel_err": max(e_main, e_ann), "main_beams": e_main, "annulus_stokes": e_ann,
              "samples": int(n_main + jj.size), "of": int(n), "tolerance": 1e-6,
              "path": "FP32 tile path"}

    t_exact = t_main + per_sample_ann * n
    res = {
        "workload": "nside-2048 sky (l <= 4095), 256 detectors x 390,625 CES samples, 151^2 elliptical main beams "
                    "(disc 1.5 deg) + shared 401^2 ring grid over +-20 deg (annulus (1.5, 20] deg)",
        "samples": n,
        "main_exact_s": t_main,
        "main_exact_samples_per_s": n / t_main,
        "surrogate_s": t_sur,
        "samples_per_s_surrogate": n / t_sur,
        "annulus_exact_samples_per_s": 1.0 / per_sample_ann,
        "annulus_timed_samples": int(idx.size),
        "exact_s_extrapolated": t_exact,
        "samples_per_s_exact_extrapolated": n / t_exact,
        "speedup": t_exact / t_sur,
        "sidelobe_error": err,
        "main_only_error": err0,
        "error_unit": "RMS(d_sl_hat - d_sl) / RMS(d_main) on the 262,144 held-out scan samples",
        "network": f"5 -> {hidden} x {width} SiLU -> 3, BF16 weights, trained by the library on {n_train} drawn "
                   f"pointings, {epochs} epochs",
        "network_flops_per_sample": SG.network_flops_per_sample(width, hidden),
        "train_samples": n_train, "epochs": epochs, "lr": lr, "final_loss": hist[-1],
        "train_s_with_targets": t_train,
        "parity": parity,
    }
    cm.close()
    del keep, held
    return res


def B_ideal(g, T):
    """Dense ideal beamsor of a scalar grid, FP32-rounded like the device copy."""
    from synth import beams as B

    return B.ideal_beamsor(np.asarray(g, dtype=np.float32).astype(np.float64), T).dense()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy (for HBM counter scaling under rocprofv3)")
    ap.add_argument("--launch", type=str, default="", help="key=value,... fields of pisco_launch")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the far-sidelobe surrogate leg")
    ap.add_argument("--no-paper-shape", action="store_true", help="skip the paper's benchmark-pattern leg")
    ap.add_argument("--no-plate", action="store_true", help="skip the half-wave-plate leg")
    ap.add_argument("--no-full-beam", action="store_true", help="skip the four-channel-beam leg")
    ap.add_argument("--no-network", action="store_true", help="skip the sidelobe-network rate leg")
    ap.add_argument("--no-maps", action="store_true", help="skip the map-making leg (and the spectra leg)")
    ap.add_argument("--no-spectra", action="store_true", help="skip the power-spectrum leg")
    ap.add_argument("--no-ideal-cmb", action="store_true", help="skip the paper's whole-sky ideal CMB run")
    ap.add_argument("--no-parity", action="store_true", help="skip the per-recipe parity leg")
    ap.add_argument("--no-full-scale", action="store_true",
                    help="skip the nside-2048, 1e8-sample surrogate-vs-exact leg")
    ap.add_argument("--full-scale-train", type=int, default=6_000_000)
    ap.add_argument("--full-scale-epochs", type=int, default=120)
    ap.add_argument("--full-scale-net", type=str, default="512x10",
                    help="network width x hidden layers for the full-scale leg")
    ap.add_argument("--full-scale-lr", type=float, default=7e-4)
    ap.add_argument("--tune", choices=("auto", "off", "force"), default="auto",
                    help="launch-shape autotuning: auto = use the cached shape or search once, force = search again")
    ap.add_argument("--surrogate-epochs", type=int, default=40)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the path is data-parallel over "
              "detectors and sample ranges and needs no collective, see the sharding notes.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1908_05662_amd import OUT_COUNT, OUT_TOD
    from paper_1908_05662_amd.api import Convolver
    from synth import workloads as W

    probe = valu_probe()
    if probe:
        log("vector ALU issue (x one wave64 instruction per 4 clocks per SIMD): " +
            ", ".join(f"{k} {v[1]:.2f}" for k, v in probe.items() if isinstance(v, list)))
    t0 = time.perf_counter()
    w = W.c3()
    log(f"workload c3: {len(w.detectors)} detectors, {w.n_samples} samples, setup {time.perf_counter() - t0:.1f}s")
    conv = Convolver(0)
    keep, kind = load(conv, w, torch)
    tuned = None
    if args.tune != "off":
        from paper_1908_05662_amd.autotune import tune

        cache = os.path.join(ROOT, "paper_1908_05662_amd", "launch.tune.json")
        tuned = tune(conv, -1, subsample=0.25, cache=cache, force=(args.tune == "force"), extra_key="batched-1024",
                     log=log)
        log(f"autotune: {tuned['launch']} ({tuned['speedup']:.3f}x over the default on the subsample, "
            f"{'cached' if tuned['cached'] else 'searched'} in {tuned['seconds']:.1f}s)")
    if args.launch:
        kv = dict(x.split("=") for x in args.launch.split(","))
        conv.set_launch(**{k: (float(v) if k == "coherence" else int(v)) for k, v in kv.items()})
    launch = conv.get_launch()
    per_sample = any(d.norm_mode == W.NORM_PER_SAMPLE for d in w.detectors)
    fpp, mfma_per_pair = flops_per_pair(launch["algorithm"], kind, w.detectors[0].rho_max, per_sample)
    n = conv.output_samples(-1)
    stream = torch.cuda.Stream()
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    cnt = torch.empty(n, dtype=torch.float32, device="cuda")
    with torch.cuda.stream(stream):
        conv.convolve(-1, OUT_COUNT, out=cnt, stream=stream)
    stream.synchronize()
    pairs = int(cnt.double().sum().item())
    del cnt
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"pairs {pairs} ({pairs / n:.1f} per sample)")

    conv.set_timing(True)
    for _ in range(args.warmup):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    conv.kernel_time(reset=True)
    t = time.perf_counter()
    for i in range(args.steps):
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    kms, launches = conv.kernel_time()
    ms_step = wall * 1e3 / args.steps
    k_ms = kms / max(launches, 1)
    value = n / (ms_step / 1e3)
    achieved = fpp * pairs / (k_ms / 1e3) / 1e12
    got = out.cpu().numpy()
    log(f"{ms_step:.2f} ms/step, kernel {k_ms:.2f} ms, {value:.4g} samples/s, {pairs / (k_ms / 1e3):.4g} pairs/s, "
        f"roofline frac {achieved / ALU_PEAK_TFLOPS:.3f} ({fpp} flops/pair)")

    cpu = None
    parity = {}
    if not args.no_cpu_baseline:
        import oracle

        ns, dt, err, per_det = cpu_baseline(w, got, args.cpu_seconds)
        frac = ns / n
        cpu = {"value": ns / dt, "unit": "samples/s", "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"{per_det} evenly spaced samples per detector x {len(w.detectors)} detectors "
                         f"({ns} samples, {frac * pairs:.3g} pairs est.) of the same workload, FP64, {dt:.1f}s",
               "macs_per_s": frac * pairs / dt, "threads": oracle.max_threads(), **host_info()}
        parity["c3_nside1024_fp32"] = {"max_rel_err": err, "samples": int(ns), "of": int(n), "tolerance": 1e-6,
                                       "path": "FP32 tile path + pixel path, the timed batched launch"}
        log(f"cpu oracle {ns / dt:.4g} samples/s on {oracle.max_threads()} threads; parity max rel err {err:.3e}")

    # the same job with the pointing handed over as host arrays: upload, plan and convolution
    t = time.perf_counter()
    for k, d in enumerate(w.detectors):
        conv.set_pointing(k, *(np.ascontiguousarray(x) for x in (d.theta, d.phi, d.psi)))
    t_up = time.perf_counter() - t
    with torch.cuda.stream(stream):
        conv.convolve(-1, OUT_TOD, out=out, stream=stream)
    stream.synchronize()
    t_all = time.perf_counter() - t
    pcie = {"workload": "the benchmark job with the pointing given as host arrays (pageable): upload of "
                        f"{24 * n / 1e9:.2f} GB, plan, one convolution", "ms": t_all * 1e3, "upload_ms": t_up * 1e3,
            "samples_per_s": n / t_all}
    log(f"pointing upload included: {t_all * 1e3:.1f} ms ({t_up * 1e3:.1f} ms upload)")
    for k, d in enumerate(w.detectors):   # the resident device pointing again
        conv.set_pointing(k, *keep[k])

    plate = None
    if not args.no_plate:
        plate = plate_leg(conv, w, stream, out, args.steps, args.warmup, k_ms, torch)
    full_beam = None
    if not args.no_full_beam:
        full_beam = full_beam_leg(conv, w, stream, out, args.steps, args.warmup, torch, pairs)
    maps = spectra = None
    if not args.no_maps:
        with torch.cuda.stream(stream):
            conv.convolve(-1, OUT_TOD, out=out, stream=stream)
        stream.synchronize()
        mk = {"conv": conv, "pointing": keep}
        maps = map_leg(w, mk, out, stream, torch)
        if not args.no_spectra:
            spectra = spectra_leg(conv, mk["maps"], torch)
        del mk

    rec = {
        "metric": "TOD samples/s + beam-pixel MACs/s at nside 1024; surrogate vs exact at fixed error",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 geometry set-up)",
        "data": "synthetic",
        "config": {"workload": "nside-1024 batched detectors: 64 dets, 201^2 elliptical beams, CES scan, "
                               "disc 2 deg", "samples": n, "pairs": pairs,
                   "launch": launch, "beam": kind},
        "macs_per_s": pairs / (ms_step / 1e3),
        "kernel_ms": k_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / ALU_PEAK_TFLOPS, "traffic": measured_traffic(launch),
                     "flops_per_pair": fpp,
                     "gather": gather_roofline(launch, pairs, k_ms) if kind == "scalar" else None,
                     "matrix_tflops": mfma_per_pair * pairs / (k_ms / 1e3) / 1e12,
                     "valu_issue_probe": probe},
        "cpu_baseline": cpu,
        "autotune": None if tuned is None else {k: tuned[k] for k in ("launch", "ms", "default_ms", "speedup",
                                                                        "cached", "seconds", "subsample")},
        "pointing_upload_included": pcie,
        "parity": parity,
        "plate": plate,
        "full_beam": full_beam,
        "maps": maps,
        "spectra": spectra,
    }
    conv.close()
    del keep, out
    torch.cuda.empty_cache()
    if not args.no_parity:
        parity.update(parity_leg())
    if not args.no_surrogate:
        rec["surrogate"] = surrogate_leg(args.surrogate_epochs)
    if not args.no_network:
        torch.cuda.empty_cache()
        rec["network"] = network_leg(torch)
    if not args.no_paper_shape:
        torch.cuda.empty_cache()
        rec["paper_shape"] = paper_shape_leg()
    if not args.no_ideal_cmb:
        torch.cuda.empty_cache()
        rec["ideal_cmb"] = ideal_cmb_leg()
    if not args.no_full_scale:
        torch.cuda.empty_cache()
        width, hidden = (int(v) for v in args.full_scale_net.split("x"))
        rec["full_scale"] = full_scale_leg(args.full_scale_epochs, args.full_scale_train, width, hidden,
                                           args.full_scale_lr)
        parity["c5_nside2048_fp32"] = rec["full_scale"]["parity"]
    if parity:
        parity["metric"] = "max |d_gpu - d_oracle| / max |d_oracle| over the compared samples (FP64 oracle)"
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
