"""Python binding of the C ABI: torch tensors in, torch tensors out.

PyTorch only provides device memory and streams here; every step of the
convolution runs in the HIP kernels of libpisco.so.  Names follow the C ABI
(include/pisco.h) without the ``pisco_`` prefix.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from .beamsor import fold_detector, fold_detector_maps, fold_v, scalar_weights


def _torch():
    import torch

    return torch


class Convolver:
    """One context on one GPU (``pisco_create``)."""

    def __init__(self, device: int = 0):
        self._lib = L.load()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the convolver has no CPU path")
        self.device = int(device)
        self.torch_device = torch.device("cuda", self.device)
        h = ctypes.c_void_p()
        st = self._lib.pisco_create(self.device, ctypes.byref(h))
        if st != L.OK:
            raise L.PiscoError(st, "pisco_create failed (device must be gfx950)")
        self._h = h
        self._keep = {}      # borrowed device pointing tensors, per detector
        self._keep_hwp = {}  # borrowed device plate-angle tensors, per detector
        self.dtype = None    # torch dtype of the sky
        self._sizes = {}

    # -- plumbing ---------------------------------------------------------
    def _check(self, st: int):
        if st != L.OK:
            raise L.PiscoError(st, self._lib.pisco_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pisco_destroy(self._h)
            self._h = None
            self._keep.clear()
            self._keep_hwp.clear()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _as_tensor(self, x, dtype):
        torch = _torch()
        if isinstance(x, np.ndarray):
            x = torch.from_numpy(np.ascontiguousarray(x))
        return x.to(dtype=dtype).contiguous()

    def _mem(self, t):
        return L.DEVICE if t.is_cuda else L.HOST

    @staticmethod
    def _code(dtype):
        torch = _torch()
        return L.F64 if dtype == torch.float64 else L.F32

    # -- C ABI ------------------------------------------------------------
    def set_sky(self, nside: int, I, Q, U, dtype=None, V=None):
        """Stokes maps in RING order; V (circular polarisation) is optional."""
        torch = _torch()
        dtype = dtype or torch.float32
        ts = [self._as_tensor(m, dtype) for m in ((I, Q, U) if V is None else (I, Q, U, V))]
        mems = {self._mem(t) for t in ts}
        if len(mems) != 1:
            raise ValueError("the maps must all live on the host or all on the device")
        if V is None:
            self._check(self._lib.pisco_set_sky(self._h, int(nside), *(t.data_ptr() for t in ts),
                                                self._code(dtype), mems.pop()))
        else:
            self._check(self._lib.pisco_set_sky_iquv(self._h, int(nside), *(t.data_ptr() for t in ts),
                                                     self._code(dtype), mems.pop()))
        self.dtype = dtype
        self.nside = int(nside)

    def set_beam(self, det: int, n: int, half_span_tan: float, bI, bQ, bU, bT, dtype=None, bV=None):
        """Four-channel beam (bI, bQ, bU, bT); bV couples the sky's V (optional)."""
        dtype = dtype or self.dtype or _torch().float32
        chans = (bI, bQ, bU, bT) if bV is None else (bI, bQ, bU, bV, bT)
        ts = [self._as_tensor(b, dtype).reshape(-1) for b in chans]
        mems = {self._mem(t) for t in ts}
        if len(mems) != 1:
            raise ValueError("beam channels must all live on the host or all on the device")
        if bV is None:
            self._check(self._lib.pisco_set_beam(self._h, int(det), int(n), float(half_span_tan),
                                                 *(t.data_ptr() for t in ts), self._code(dtype), mems.pop()))
        else:
            self._check(self._lib.pisco_set_beam_v(self._h, int(det), int(n), float(half_span_tan),
                                                   *(t.data_ptr() for t in ts), self._code(dtype), mems.pop()))

    def set_beam_scalar(self, det: int, n: int, half_span_tan: float, b, wI: float, wQ: float, wU: float,
                        wT: float = 1.0, dtype=None, wV: float = 0.0):
        dtype = dtype or self.dtype or _torch().float32
        t = self._as_tensor(b, dtype).reshape(-1)
        if wV:
            self._check(self._lib.pisco_set_beam_scalar_v(self._h, int(det), int(n), float(half_span_tan),
                                                          t.data_ptr(), float(wI), float(wQ), float(wU), float(wV),
                                                          float(wT), self._code(dtype), self._mem(t)))
            return
        self._check(self._lib.pisco_set_beam_scalar(self._h, int(det), int(n), float(half_span_tan), t.data_ptr(),
                                                    float(wI), float(wQ), float(wU), float(wT), self._code(dtype),
                                                    self._mem(t)))

    def set_beam_healpix(self, det: int, nside_beam: int, n: int, half_span_tan: float, bI, bQ, bU, bT, dtype=None):
        """Four-channel beam given as HEALPix maps (boresight at the north pole),
        resampled by the library onto the n x n grid over +-half_span_tan."""
        dtype = dtype or self.dtype or _torch().float32
        ts = [self._as_tensor(b, dtype).reshape(-1) for b in (bI, bQ, bU, bT)]
        mems = {self._mem(t) for t in ts}
        if len(mems) != 1:
            raise ValueError("beam maps must all live on the host or all on the device")
        self._check(self._lib.pisco_set_beam_healpix(self._h, int(det), int(nside_beam), *(t.data_ptr() for t in ts),
                                                     int(n), float(half_span_tan), self._code(dtype), mems.pop()))

    def set_beam_healpix_scalar(self, det: int, nside_beam: int, n: int, half_span_tan: float, b, wI: float,
                                wQ: float, wU: float, wT: float = 1.0, dtype=None):
        dtype = dtype or self.dtype or _torch().float32
        t = self._as_tensor(b, dtype).reshape(-1)
        self._check(self._lib.pisco_set_beam_healpix_scalar(self._h, int(det), int(nside_beam), t.data_ptr(),
                                                            float(wI), float(wQ), float(wU), float(wT), int(n),
                                                            float(half_span_tan), self._code(dtype), self._mem(t)))

    def set_beamsor_healpix(self, det: int, nside_beam: int, mueller_maps: np.ndarray, half_span_tan: float, n: int,
                            eps: float, s: float, dtype=None, allow_scalar: bool = True):
        """Fold (npix, 4, 4) Mueller maps with the detector row and upload them
        as HEALPix beam maps; the one-map form when every folded channel is a
        constant multiple of B_TT.  A V column is not taken on this route."""
        bI, bQ, bU, bT, bV = fold_detector_maps(mueller_maps, eps, s)
        if np.any(bV):
            raise ValueError("HEALPix beam maps with a V column: resample them onto a grid and use set_beam")
        if allow_scalar:
            w = scalar_weights(bI, bQ, bU, bT)
            if w is not None:
                self.set_beam_healpix_scalar(det, nside_beam, n, half_span_tan, bT, *w, 1.0, dtype=dtype)
                return "scalar"
        self.set_beam_healpix(det, nside_beam, n, half_span_tan, bI, bQ, bU, bT, dtype)
        return "full"

    def set_beamsor(self, det: int, mueller: np.ndarray, half_span_tan: float, eps: float, s: float, dtype=None,
                    allow_scalar: bool = True):
        """Fold a (n, n, 4, 4) Mueller field with the detector row and upload it;
        uses the one-grid form when every folded channel is a constant multiple
        of B_TT (to 1e-12 relative)."""
        bI, bQ, bU, bT = fold_detector(mueller, eps, s)
        bV = fold_v(mueller, eps, s)
        if allow_scalar:
            w = scalar_weights(bI, bQ, bU, bT)
            wv = None if bV is None else scalar_weights(bV, bV, bV, bT)
            if w is not None and (bV is None or wv is not None):
                self.set_beam_scalar(det, bT.shape[0], half_span_tan, bT, *w, 1.0, dtype=dtype,
                                     wV=0.0 if wv is None else wv[0])
                return "scalar"
        self.set_beam(det, bI.shape[0], half_span_tan, bI, bQ, bU, bT, dtype, bV=bV)
        return "full"

    def set_hwp(self, det: int, angle=None):
        """Per-sample half-wave-plate angle (rad) for detector `det`; None removes the plate."""
        torch = _torch()
        if angle is None:
            self._check(self._lib.pisco_set_hwp(self._h, int(det), 0, None, L.HOST))
            self._keep_hwp.pop(det, None)
            return
        t = self._as_tensor(angle, torch.float64).reshape(-1)
        self._check(self._lib.pisco_set_hwp(self._h, int(det), t.numel(), t.data_ptr(), self._mem(t)))
        if t.is_cuda:
            self._keep_hwp[det] = t     # borrowed by the library
        else:
            self._keep_hwp.pop(det, None)

    def share_beam(self, det: int, src: int):
        self._check(self._lib.pisco_share_beam(self._h, int(det), int(src)))

    def set_detector(self, det: int, zeta: float, rho_min: float, rho_max: float, norm_mode: int,
                     norm_scale: float = 1.0):
        self._check(self._lib.pisco_set_detector(self._h, int(det), float(zeta), float(rho_min), float(rho_max),
                                                 int(norm_mode), float(norm_scale)))

    def set_pointing(self, det: int, theta, phi, psi):
        torch = _torch()
        ts = [self._as_tensor(x, torch.float64).reshape(-1) for x in (theta, phi, psi)]
        n = ts[0].numel()
        if any(t.numel() != n for t in ts):
            raise ValueError("theta, phi, psi must have equal length")
        mems = {self._mem(t) for t in ts}
        if len(mems) != 1:
            raise ValueError("pointing arrays must all live on the host or all on the device")
        mem = mems.pop()
        self._check(self._lib.pisco_set_pointing(self._h, int(det), n, *(t.data_ptr() for t in ts), mem))
        if mem == L.DEVICE:
            self._keep[det] = ts       # borrowed by the library
        else:
            self._keep.pop(det, None)

    def output_samples(self, det: int = -1) -> int:
        return int(self._lib.pisco_output_samples(self._h, int(det)))

    def convolve(self, det: int = -1, out_mode: int = L.OUT_TOD, out=None, stream=None):
        """Run on the current (or given) torch stream; returns the device output tensor."""
        torch = _torch()
        n = self.output_samples(det)
        shape = (n, 3) if out_mode == L.OUT_STOKES else (n,)
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.torch_device)
        if tuple(out.shape) != shape or out.dtype != self.dtype or not out.is_contiguous() or \
                (out.is_cuda and out.device != self.torch_device):
            raise ValueError(f"out must be a contiguous {self.dtype} tensor of shape {shape} on the host or "
                             f"{self.torch_device}")
        if not out.is_cuda:   # host output: the library synchronises and copies
            self._check(self._lib.pisco_convolve(self._h, int(det), int(out_mode), out.data_ptr(), L.HOST, None))
            return out
        s = stream if stream is not None else torch.cuda.current_stream(self.torch_device)
        self._check(self._lib.pisco_convolve(self._h, int(det), int(out_mode), out.data_ptr(), L.DEVICE,
                                             ctypes.c_void_p(s.cuda_stream)))
        return out

    def convolve_static(self, det: int, out_mode: int = L.OUT_TOD, out=None, stream=None):
        """pisco_convolve_static: one detector, device output, no allocation by the
        library (the output tensor is allocated here when not given)."""
        torch = _torch()
        n = self.output_samples(det)
        shape = (n, 3) if out_mode == L.OUT_STOKES else (n,)
        if out is None:
            out = torch.empty(shape, dtype=self.dtype, device=self.torch_device)
        if tuple(out.shape) != shape or out.dtype != self.dtype or not out.is_contiguous() or \
                not out.is_cuda or out.device != self.torch_device:
            raise ValueError(f"out must be a contiguous {self.dtype} tensor of shape {shape} on {self.torch_device}")
        s = stream if stream is not None else torch.cuda.current_stream(self.torch_device)
        self._check(self._lib.pisco_convolve_static(self._h, int(det), int(out_mode), out.data_ptr(),
                                                    ctypes.c_void_p(s.cuda_stream)))
        return out

    def set_launch(self, **kw):
        """Update fields of the launch shape (see pisco_launch); returns the new shape."""
        cur = self.get_launch()
        cur.update(kw)
        l = L.Launch(**cur)
        self._check(self._lib.pisco_set_launch(self._h, ctypes.byref(l)))
        return self.get_launch()

    def set_ordering(self, mode: str = "auto"):
        """Processing order of each detector's samples: "given", "auto" (spatial
        order for streams whose given order is incoherent) or "spatial"."""
        code = {"given": 0, "auto": 1, "spatial": 2}[mode]
        self._check(self._lib.pisco_set_ordering(self._h, code))

    def get_launch(self) -> dict:
        l = L.Launch()
        self._check(self._lib.pisco_get_launch(self._h, ctypes.byref(l)))
        return l.as_dict()

    def set_memory_budget(self, nbytes: int):
        """Cap the device memory this context allocates (0: no cap); streams that do
        not fit are convolved in blocks of samples (``pisco_set_memory_budget``)."""
        self._check(self._lib.pisco_set_memory_budget(self._h, int(nbytes)))

    def memory_in_use(self) -> int:
        return int(self._lib.pisco_memory_in_use(self._h))

    def sidelobe_options(self, width: int = 256, hidden_layers: int = 4, batch: int = 8192, lr: float = 2e-3,
                         lr_end: float = 2e-5, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        """Network and optimiser of later ``sidelobe_train`` runs."""
        o = L.SidelobeOpts(int(width), int(hidden_layers), int(batch), float(lr), float(lr_end), float(beta1),
                           float(beta2), float(eps))
        self._check(self._lib.pisco_sidelobe_set_options(self._h, ctypes.byref(o)))

    def sidelobe_train(self, det: int, r_main: float, n_train: int, seed: int = 1, epochs: int = 40):
        """Train detector `det`'s far-sidelobe network on exact annulus pickups
        (r_main, rho_max] of n_train library-drawn pointings; returns the per-epoch
        mean training losses."""
        self._check(self._lib.pisco_sidelobe_train(self._h, int(det), float(r_main), int(n_train),
                                                   ctypes.c_uint64(seed), int(epochs)))
        return self.sidelobe_history(det)

    def sidelobe_enable(self, det: int, on: bool = True):
        """TOD of `det` = exact main disc + the trained network (on) or the exact disc (off)."""
        self._check(self._lib.pisco_sidelobe_enable(self._h, int(det), int(bool(on))))

    def sidelobe_share(self, det: int, src: int):
        """Detector `det` uses the network trained for `src` (its own beam, weights and zeta)."""
        self._check(self._lib.pisco_sidelobe_share(self._h, int(det), int(src)))

    def sidelobe_history(self, det: int):
        n = int(self._lib.pisco_sidelobe_history(self._h, int(det), None, 0))
        if n <= 0:
            return []
        buf = (ctypes.c_double * n)()
        self._lib.pisco_sidelobe_history(self._h, int(det), buf, n)
        return list(buf)

    def set_timing(self, on: bool = True):
        self._check(self._lib.pisco_set_timing(self._h, int(bool(on))))

    def kernel_time(self, reset: bool = False):
        ms, k = ctypes.c_double(), ctypes.c_int64()
        self._check(self._lib.pisco_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(k), int(reset)))
        return ms.value, k.value


class Mlp:
    """Far-sidelobe network on the convolver's device (``pisco_mlp_*``)."""

    def __init__(self, conv: Convolver, width: int = 256, hidden_layers: int = 4, max_batch: int = 16384,
                 seed: int = 0):
        self.conv = conv
        self._lib = conv._lib
        h = ctypes.c_void_p()
        conv._check(self._lib.pisco_mlp_create(conv._h, int(width), int(hidden_layers), int(max_batch),
                                               ctypes.c_uint64(seed), ctypes.byref(h)))
        self._h = h
        self.width, self.hidden, self.max_batch = int(width), int(hidden_layers), int(max_batch)
        self.n_params = int(self._lib.pisco_mlp_param_count(h))
        torch = _torch()
        dev = conv.torch_device
        self._loss = torch.zeros(1, dtype=torch.float32, device=dev)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pisco_mlp_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.conv.torch_device)
        return ctypes.c_void_p(s.cuda_stream)

    def layout(self, layer: int):
        wo, bo = ctypes.c_int64(), ctypes.c_int64()
        r, c = ctypes.c_int32(), ctypes.c_int32()
        self.conv._check(self._lib.pisco_mlp_layout(self._h, int(layer), ctypes.byref(wo), ctypes.byref(bo),
                                                    ctypes.byref(r), ctypes.byref(c)))
        return wo.value, bo.value, r.value, c.value

    def get_params(self):
        torch = _torch()
        out = torch.empty(self.n_params, dtype=torch.float32)
        self.conv._check(self._lib.pisco_mlp_get_params(self._h, out.data_ptr(), L.HOST))
        return out

    def set_params(self, params):
        torch = _torch()
        t = self.conv._as_tensor(params, torch.float32).reshape(-1)
        if t.numel() != self.n_params:
            raise ValueError("wrong parameter count")
        self.conv._check(self._lib.pisco_mlp_set_params(self._h, t.data_ptr(), self.conv._mem(t)))

    def _rows(self, x, cols, name, batch=False):
        """A contiguous float32 device copy (or view) of x with shape (n, cols); with
        batch, n must be a multiple of 64 in [64, max_batch].  The caller keeps
        the returned tensor alive until the library call has been queued."""
        torch = _torch()
        if not torch.is_tensor(x) or x.dtype != torch.float32 or x.device != self.conv.torch_device \
                or x.dim() != 2 or x.shape[1] != cols:
            raise ValueError(f"{name} must be a float32 tensor of shape (n, {cols}) on {self.conv.torch_device}")
        n = x.shape[0]
        if batch and (n < 64 or n > self.max_batch or n % 64):
            raise ValueError(f"{name}: batch of {n} rows must be a multiple of 64 in [64, {self.max_batch}]")
        return x.contiguous()

    def forward(self, x, stream=None):
        torch = _torch()
        xc = self._rows(x, 5, "x")
        y = torch.empty((xc.shape[0], 3), dtype=torch.float32, device=xc.device)
        self.conv._check(self._lib.pisco_mlp_forward(self._h, xc.data_ptr(), xc.shape[0], y.data_ptr(),
                                                     self._stream(stream)))
        return y

    def gradient(self, x, t, stream=None):
        torch = _torch()
        xc = self._rows(x, 5, "x", batch=True)
        tc = self._rows(t, 3, "targets", batch=True)
        if tc.shape[0] != xc.shape[0]:
            raise ValueError("x and targets must have the same number of rows")
        g = torch.empty(self.n_params, dtype=torch.float32, device=xc.device)
        self.conv._check(self._lib.pisco_mlp_gradient(self._h, xc.data_ptr(), tc.data_ptr(), xc.shape[0],
                                                      g.data_ptr(), self._loss.data_ptr(), self._stream(stream)))
        return self._loss.clone(), g

    def train_step(self, x, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        """One Adam step; returns the (device) loss tensor of the batch before the update."""
        xc = self._rows(x, 5, "x", batch=True)
        tc = self._rows(t, 3, "targets", batch=True)
        if tc.shape[0] != xc.shape[0]:
            raise ValueError("x and targets must have the same number of rows")
        self.conv._check(self._lib.pisco_mlp_train_step(self._h, xc.data_ptr(), tc.data_ptr(), xc.shape[0],
                                                        float(lr), float(beta1), float(beta2), float(eps),
                                                        self._loss.data_ptr(), self._stream(stream)))
        return self._loss

    def features(self, det: int, stream=None, conv=None):
        """Features of detector `det` of `conv` (default: the network's convolver)."""
        torch = _torch()
        cv = conv or self.conv
        n = cv.output_samples(det)
        x = torch.empty((n, 5), dtype=torch.float32, device=cv.torch_device)
        cv._check(self._lib.pisco_sidelobe_features(cv._h, int(det), x.data_ptr(), self._stream(stream)))
        return x

    def apply(self, det: int, mean, std, coef, tod, stream=None, conv=None):
        """tod += sum_c coef[c] (mean[c] + std[c] y[c]) over detector `det` of
        `conv` (default: the network's convolver; any convolver on the same device)."""
        cv = conv or self.conv
        m = (ctypes.c_float * 3)(*[float(v) for v in mean])
        s = (ctypes.c_float * 3)(*[float(v) for v in std])
        c = (ctypes.c_double * 3)(*[float(v) for v in coef])
        if tod.numel() != cv.output_samples(det) or not tod.is_cuda or tod.dtype != _torch().float32:
            raise ValueError("tod must be a float32 device tensor with one value per sample of the detector")
        cv._check(self._lib.pisco_sidelobe_apply(cv._h, self._h, int(det), m, s, c, tod.data_ptr(),
                                                 self._stream(stream)))
        return tod


class MapMaker:
    """Binned (I, Q, U) maps of nside `nside` from TOD on the convolver's device
    (``pisco_map_accumulate`` / ``pisco_map_solve``); the per-pixel sums live in
    one device float64 tensor of 10 values per pixel."""

    def __init__(self, conv: Convolver, nside: int):
        torch = _torch()
        self.conv, self.nside = conv, int(nside)
        self.npix = 12 * self.nside * self.nside
        self._lib = conv._lib
        self.accum = torch.zeros(self.npix * 10, dtype=torch.float64, device=conv.torch_device)

    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.conv.torch_device)
        return ctypes.c_void_p(s.cuda_stream)

    def clear(self):
        self.accum.zero_()

    def add(self, theta, phi, psi, tod, zeta: float = 0.0, eps: float = 0.0, s: float = 1.0, hwp=None, stream=None):
        """Add one detector's samples (device tensors, or arrays copied to the device)."""
        torch = _torch()
        dev = self.conv.torch_device
        th, ph, ps = (self.conv._as_tensor(x, torch.float64).to(dev) for x in (theta, phi, psi))
        d = tod if (torch.is_tensor(tod) and tod.dtype in (torch.float32, torch.float64)) else \
            self.conv._as_tensor(tod, torch.float64)
        d = d.to(dev).contiguous()
        hw = None if hwp is None else self.conv._as_tensor(hwp, torch.float64).to(dev)
        n = th.numel()
        if ph.numel() != n or ps.numel() != n or d.numel() != n or (hw is not None and hw.numel() != n):
            raise ValueError("theta, phi, psi, tod (and hwp) must have one value per sample")
        code = L.F64 if d.dtype == torch.float64 else L.F32
        self.conv._check(self._lib.pisco_map_accumulate(
            self.conv._h, self.nside, n, th.data_ptr(), ph.data_ptr(), ps.data_ptr(),
            None if hw is None else hw.data_ptr(), d.data_ptr(), code, float(zeta), float(eps), float(s),
            self.accum.data_ptr(), self._stream(stream)))
        if stream is not None:   # the inputs must outlive the queued work
            stream.synchronize()
        return self

    def solve(self, rcond_min: float = 1e-6, stream=None):
        """(maps [3, npix] as I, Q, U rows; rcond [npix]) float64 device tensors."""
        torch = _torch()
        maps = torch.empty((3, self.npix), dtype=torch.float64, device=self.conv.torch_device)
        rc = torch.empty(self.npix, dtype=torch.float64, device=self.conv.torch_device)
        self.conv._check(self._lib.pisco_map_solve(self.conv._h, self.nside, self.accum.data_ptr(), float(rcond_min),
                                                   maps.data_ptr(), rc.data_ptr(), self._stream(stream)))
        return maps, rc

    def hits(self):
        return self.accum.view(self.npix, 10)[:, 9]

class Spectra:
    """Spherical-harmonic analysis of HEALPix maps and their angular power
    spectra on the convolver's device (``pisco_map2alm``, ``pisco_alm2cl``,
    ``pisco_anafast``), FP64.  a_lm are complex128 device tensors in the
    m-major packing index(l, m) = m (2 lmax + 1 - m) / 2 + l; spectra come in the
    order TT, EE, BB, TE, EB, TB."""

    NAMES = ("TT", "EE", "BB", "TE", "EB", "TB")

    def __init__(self, conv: Convolver, nside: int, lmax: int | None = None, pol: bool = True):
        torch = _torch()
        self.conv, self.nside = conv, int(nside)
        self.lmax = 3 * self.nside - 1 if lmax is None else int(lmax)
        self.pol = bool(pol)
        self._lib = conv._lib
        nbytes = self._lib.pisco_map2alm_workspace_bytes(self.nside, self.lmax, int(self.pol))
        if nbytes < 0:
            raise ValueError("nside must be a power of two in [1, 1024] and lmax in [0, 4 nside]")
        dev = conv.torch_device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        n = int(self._lib.pisco_alm_size(self.lmax))
        self.alm = [torch.empty(n, dtype=torch.complex128, device=dev) for _ in range(3 if self.pol else 1)]

    def _stream(self, stream):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.conv.torch_device)
        return ctypes.c_void_p(s.cuda_stream)

    def _maps(self, T, Q, U):
        torch = _torch()
        dev = self.conv.torch_device
        npix = 12 * self.nside * self.nside
        ms = [self.conv._as_tensor(x, torch.float64).to(dev).contiguous() for x in (T, Q, U) if x is not None]
        if (Q is None) != (U is None) or (Q is not None and not self.pol) or any(m.numel() != npix for m in ms):
            raise ValueError(f"expected T (and Q, U if polarised) RING maps of {npix} pixels")
        return ms + [None] * (3 - len(ms))

    def _ptrs(self, maps):
        pol = maps[1] is not None
        mp = [None if m is None else m.data_ptr() for m in maps]
        ap = [self.alm[0].data_ptr()] + ([a.data_ptr() for a in self.alm[1:]] if pol else [None, None])
        return mp, ap

    def map2alm(self, T, Q=None, U=None, iterations: int = 0, stream=None):
        """(a^T, a^E, a^B) complex128 device tensors (a^E, a^B None without Q, U); the
        tensors are this object's buffers, overwritten by the next call.
        `iterations` Jacobi steps refine the pixel quadrature."""
        maps = self._maps(T, Q, U)
        mp, ap = self._ptrs(maps)
        self.conv._check(self._lib.pisco_map2alm(self.conv._h, self.nside, self.lmax, int(iterations), *mp, *ap,
                                                 self.workspace.data_ptr(), self.workspace.numel(),
                                                 self._stream(stream)))
        if stream is not None:
            stream.synchronize()
        return tuple(self.alm) if maps[1] is not None else (self.alm[0], None, None)

    def alm2map(self, aT, aE=None, aB=None, stream=None):
        """(T, Q, U) float64 device maps from complex128 a_lm tensors of this
        object's lmax (Q, U None without a^E, a^B)."""
        torch = _torch()
        n = int(self._lib.pisco_alm_size(self.lmax))
        al = [aT, aE, aB]
        if (aE is None) != (aB is None) or (aE is not None and not self.pol) or any(
                a is not None and (a.dtype != torch.complex128 or a.numel() != n or not a.is_cuda) for a in al):
            raise ValueError(f"a_lm must be complex128 device tensors of {n} values (a^E and a^B together)")
        pol = aE is not None
        npix = 12 * self.nside * self.nside
        maps = [torch.empty(npix, dtype=torch.float64, device=self.conv.torch_device) for _ in range(3 if pol else 1)]
        al = [a.contiguous() for a in al if a is not None]
        ap = [a.data_ptr() for a in al] + [None] * (3 - len(al))
        mp = [m.data_ptr() for m in maps] + [None] * (3 - len(maps))
        self.conv._check(self._lib.pisco_alm2map(self.conv._h, self.nside, self.lmax, *ap, *mp,
                                                 self.workspace.data_ptr(), self.workspace.numel(),
                                                 self._stream(stream)))
        if stream is not None:
            stream.synchronize()
        return tuple(maps) if pol else (maps[0], None, None)

    def anafast(self, T, Q=None, U=None, iterations: int = 0, stream=None):
        """[6, lmax + 1] float64 device tensor (TT, EE, BB, TE, EB, TB), or [1, lmax + 1] for T only."""
        torch = _torch()
        maps = self._maps(T, Q, U)
        mp, ap = self._ptrs(maps)
        cl = torch.empty((6 if maps[1] is not None else 1, self.lmax + 1), dtype=torch.float64,
                         device=self.conv.torch_device)
        self.conv._check(self._lib.pisco_anafast(self.conv._h, self.nside, self.lmax, int(iterations), *mp, *ap,
                                                 self.workspace.data_ptr(), self.workspace.numel(), cl.data_ptr(),
                                                 self._stream(stream)))
        if stream is not None:
            stream.synchronize()
        return cl

    def alm2cl(self, x, y=None, stream=None):
        """C_l of two a_lm tensors of this object's lmax (y = x for an auto-spectrum)."""
        torch = _torch()
        y = x if y is None else y
        n = int(self._lib.pisco_alm_size(self.lmax))
        if x.dtype != torch.complex128 or y.dtype != torch.complex128 or x.numel() != n or y.numel() != n \
                or not x.is_cuda or not y.is_cuda:
            raise ValueError(f"a_lm must be complex128 device tensors of {n} values")
        cl = torch.empty(self.lmax + 1, dtype=torch.float64, device=self.conv.torch_device)
        self.conv._check(self._lib.pisco_alm2cl(self.conv._h, self.lmax, x.contiguous().data_ptr(),
                                                y.contiguous().data_ptr(), cl.data_ptr(), self._stream(stream)))
        if stream is not None:
            stream.synchronize()
        return cl
