"""Shared glue for the GPU tests: load a synthetic workload into the convolver
and evaluate the oracle on the same (precision-rounded) inputs."""
from __future__ import annotations

import numpy as np

import oracle


def rounded(x, dtype):
    return np.asarray(x, dtype=dtype).astype(np.float64)


def load_workload(conv, w, dtype, dets=None, device_pointing=True, beam="auto"):
    """Upload sky, beams, detector parameters and pointing; returns the detector ids used.
    beam: "auto" (one-grid form when the folded channels are proportional) or "full"."""
    import torch

    tdt = torch.float64 if dtype == np.float64 else torch.float32
    conv.set_sky(w.nside, *(torch.from_numpy(np.asarray(m, dtype=dtype)).cuda() for m in w.sky), dtype=tdt)
    ids = list(range(len(w.detectors))) if dets is None else list(dets)
    for k in ids:
        d = w.detectors[k]
        conv.set_beamsor(k, d.beam.dense(), d.beam.half_span_tan, d.det.eps, d.det.s, dtype=tdt,
                         allow_scalar=(beam == "auto"))
        conv.set_detector(k, d.det.zeta, d.rho_min, d.rho_max, d.norm_mode, d.norm_scale)
        arrs = [torch.from_numpy(np.ascontiguousarray(x)) for x in (d.theta, d.phi, d.psi)]
        if device_pointing:
            arrs = [a.cuda() for a in arrs]
        conv.set_pointing(k, *arrs)
    return ids


def oracle_detector(w, k, idx, dtype, out_mode=oracle.OUT_TOD, rho_min=None, rho_max=None):
    """Oracle on detector k's samples idx, with the sky and beam rounded like the GPU copy."""
    d = w.detectors[k]
    sky = [rounded(m, dtype) for m in w.sky]
    M = d.beam.dense()
    if dtype == np.float32:
        M = rounded(M, np.float32)
    return oracle.tod(w.nside, *sky, M, d.beam.half_span_tan, d.det.zeta, d.det.eps, d.det.s,
                      d.rho_min if rho_min is None else rho_min, d.rho_max if rho_max is None else rho_max,
                      d.norm_mode, d.norm_scale, d.theta[idx], d.phi[idx], d.psi[idx], out_mode)


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


def say(msg):
    print(msg, flush=True)


_WORKLOADS = {}


def cached_workload(name, **kw):
    """A synthetic workload built once per test process (the nside-1024 recipe takes
    about half a minute to synthesise); callers must not modify what they get."""
    from synth import workloads as W

    key = (name, tuple(sorted(kw.items())))
    if key not in _WORKLOADS:
        _WORKLOADS[key] = getattr(W, name)(**kw)
    return _WORKLOADS[key]


def coherence_chords(d, frac, group=64):
    """Per group of `group` consecutive samples: the largest chord from the
    group's normalised mean direction, and the limit frac * rho_max below which
    the tile path takes the group (FP64 on the host).  Returns (chord, limit)."""
    st = np.sin(d.theta)
    p = np.stack([st * np.cos(d.phi), st * np.sin(d.phi), np.cos(d.theta)], 1)
    nfull = d.n // group
    chords = []
    if nfull:
        q = p[:nfull * group].reshape(nfull, group, 3)
        c = q.sum(1)
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        chords.append(np.linalg.norm(q - c[:, None, :], axis=2).max(1))
    if d.n % group:
        q = p[nfull * group:]
        c = q.sum(0)
        c /= np.linalg.norm(c)
        chords.append(np.array([np.linalg.norm(q - c, axis=1).max()]))
    return np.concatenate(chords), frac * d.rho_max
