"""Launch-shape autotuner for the convolution (tile size, disc-chunk size,
workgroup shape, occupancy, queue split, coherence threshold).

It times real launches through the C ABI on the inputs already loaded in a
convolver, on a prefix of every detector's pointing stream (scan order keeps
the prefix representative), and searches the shape by coordinate descent:
each field in turn is swept with the others held, a value kept only when it
beats the current best by more than `accept` (2%: run-to-run timing noise is
about 1%, so near-ties keep the starting shape), until a full pass gains under
`min_gain`.  Results are cached per device and workload
signature in a JSON file, so a later run with the same signature applies the
tuned shape without searching.
"""
from __future__ import annotations

import json
import os
import time

from . import _lib as L

# search space, in sweep order; fields marked tile-only do not affect the pixel path
SPACE = [
    # the matrix-core tile variant is not searched: on gfx950 it takes about
    # twice as long as the vector tile kernel on every workload measured
    ("algorithm", (L.ALGO_TILE, L.ALGO_PIXEL)),
    ("chunk", (64, 128, 256)),
    ("waves_per_group", (2, 4, 8)),
    ("groups_per_cu", (1, 2, 3, 4)),
    ("xcd_queues", (8, 1)),
    ("coherence", (0.25, 0.5, 1.0)),
    ("samples_per_tile", (32, 64, 128)),
]
TILE_ONLY = {"chunk", "coherence"}


def _key(conv, det: int, pairs_per_sample: float, extra: str) -> str:
    import torch

    p = torch.cuda.get_device_properties(conv.device)
    arch = getattr(p, "gcnArchName", p.name)
    return (f"{arch}|cu{p.multi_processor_count}|nside{conv.nside}|{str(conv.dtype).replace('torch.', '')}|"
            f"det{det}|n{conv.output_samples(det)}|pps{pairs_per_sample:.3g}|{extra}")


class _Prefix:
    """Point every device-resident detector stream at its first `frac` samples
    (at least 64) for the duration of a with-block."""

    def __init__(self, conv, frac: float):
        self.conv, self.frac, self.saved = conv, frac, {}

    def __enter__(self):
        self.saved_hwp = {}
        if self.frac < 1.0:
            for det, ts in list(self.conv._keep.items()):
                n = ts[0].numel()
                m = min(n, max(64, int(round(n * self.frac))))
                self.saved[det] = ts
                self.conv.set_pointing(det, *(t[:m] for t in ts))
                hw = self.conv._keep_hwp.get(det)
                if hw is not None:
                    self.saved_hwp[det] = hw
                    self.conv.set_hwp(det, hw[:m])
        return self

    def __exit__(self, *exc):
        for det, ts in self.saved.items():
            self.conv.set_pointing(det, *ts)
        for det, hw in self.saved_hwp.items():
            self.conv.set_hwp(det, hw)
        return False


def _time_shape(conv, det, shape, out, stream, reps):
    """Median ms per convolve for one shape, or None if the shape is rejected."""
    import torch

    try:
        conv.set_launch(**shape)
    except L.PiscoError:
        return None
    with torch.cuda.stream(stream):
        conv.convolve(det, L.OUT_TOD, out=out, stream=stream)      # plan + graph build, warm caches
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            a.record(stream)
            conv.convolve(det, L.OUT_TOD, out=out, stream=stream)
            b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(conv, det: int = -1, subsample: float = 0.25, reps: int = 3, cache: str | None = None,
         force: bool = False, extra_key: str = "", max_passes: int = 2, min_gain: float = 0.01,
         accept: float = 0.02, log=None) -> dict:
    """Pick and apply the fastest launch shape for the loaded inputs.

    Returns {"launch", "ms", "default_ms", "speedup", "trials", "cached", "key", "seconds"}
    where ms are per convolve of the subsampled streams."""
    import torch

    say = log or (lambda m: None)
    t_start = time.perf_counter()
    stream = torch.cuda.Stream()
    start = conv.get_launch()

    with _Prefix(conv, subsample):
        n = conv.output_samples(det)
        cnt = torch.empty(n, dtype=conv.dtype, device=conv.torch_device)
        with torch.cuda.stream(stream):
            conv.convolve(det, L.OUT_COUNT, out=cnt, stream=stream)
        stream.synchronize()
        pps = float(cnt.double().sum().item()) / max(n, 1)
        del cnt
        key = _key(conv, det, pps, f"sub{subsample:g}|{extra_key}")

        table = {}
        if cache and os.path.exists(cache):
            try:
                table = json.load(open(cache))
            except (OSError, ValueError):
                table = {}
        if not force and key in table:
            rec = dict(table[key])
            conv.set_launch(**rec["launch"])
            rec.update(cached=True, key=key, seconds=time.perf_counter() - t_start)
            say(f"autotune: cached shape for {key}")
            return rec

        out = torch.empty(n, dtype=conv.dtype, device=conv.torch_device)
        trials = []

        def run(shape):
            ms = _time_shape(conv, det, shape, out, stream, reps)
            trials.append({"launch": dict(shape), "ms": ms})
            say(f"autotune: {shape} -> {ms}")
            return ms

        best = dict(start)
        best_ms = run(best)
        default_ms = best_ms
        for _ in range(max_passes):
            pass_start = best_ms
            for field, values in SPACE:
                if field in TILE_ONLY and best["algorithm"] == L.ALGO_PIXEL:
                    continue
                for v in values:
                    if v == best[field]:
                        continue
                    cand = dict(best)
                    cand[field] = v
                    ms = run(cand)
                    if ms is not None and ms < best_ms * (1.0 - accept):
                        best, best_ms = cand, ms
            if best_ms > pass_start * (1.0 - min_gain):
                break

    # The queue split is settled on the whole streams, where the per-die
    # queues cost less than on a prefix (on the nside-1024 benchmark 6% slower
    # on a 25% prefix, under 1% in full; on small or gather-bound streams they
    # stay much slower).  Within `accept` of the shared queue they are taken,
    # as they read a fraction of the bytes from memory.
    queues = None
    if best["algorithm"] != L.ALGO_PIXEL and subsample < 1.0:
        n_full = conv.output_samples(det)
        out_full = torch.empty(n_full, dtype=conv.dtype, device=conv.torch_device)
        per_die = dict(best, xcd_queues=8)
        shared = dict(best, xcd_queues=1)
        ms8 = _time_shape(conv, det, per_die, out_full, stream, reps)
        ms1 = _time_shape(conv, det, shared, out_full, stream, reps)
        trials.append({"launch": per_die, "ms": ms8, "full": True})
        trials.append({"launch": shared, "ms": ms1, "full": True})
        say(f"autotune: whole streams, eight queues {ms8} ms, one queue {ms1} ms")
        if ms8 is not None and ms1 is not None:
            best = shared if ms1 < ms8 * (1.0 - accept) else per_die
            queues = {"eight_ms": ms8, "one_ms": ms1}
        del out_full

    conv.set_launch(**best)
    rec = {"launch": best, "ms": best_ms, "default_ms": default_ms, "speedup": default_ms / best_ms,
           "trials": trials, "subsample": subsample, "pairs_per_sample": pps, "queues_full": queues}
    if cache:
        table[key] = rec
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1)
        os.replace(tmp, cache)
    rec.update(cached=False, key=key, seconds=time.perf_counter() - t_start)
    return rec
