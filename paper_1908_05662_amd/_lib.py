"""ctypes view of the C ABI in include/pisco.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpisco.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED = range(6)
F32, F64 = 0, 1
HOST, DEVICE = 0, 1
NORM_FIXED, NORM_PER_SAMPLE = 0, 1
OUT_TOD, OUT_STOKES, OUT_COUNT = 0, 1, 2
ALGO_PIXEL, ALGO_TILE, ALGO_TILE_MX = 0, 1, 2


class Launch(ctypes.Structure):
    """Mirror of pisco_launch."""
    _fields_ = [("algorithm", ctypes.c_int32), ("samples_per_tile", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32),
                ("xcd_queues", ctypes.c_int32), ("chunk", ctypes.c_int32), ("coherence", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

class SidelobeOpts(ctypes.Structure):
    """Mirror of pisco_sidelobe_opts."""
    _fields_ = [("width", ctypes.c_int32), ("hidden_layers", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("lr_end", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_STATUS = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE",
           EUNSUPPORTED: "EUNSUPPORTED"}

# (name, restype, argtypes) for every exported symbol of include/pisco.h
_vp, _i32, _i64, _dbl, _cp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_char_p
_ip = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = [
    ("pisco_abi_version", ctypes.c_int, []),
    ("pisco_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_vp)]),
    ("pisco_destroy", None, [_vp]),
    ("pisco_last_error", _cp, [_vp]),
    ("pisco_set_sky", ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int]),
    ("pisco_set_beam", ctypes.c_int, [_vp, _i32, _i32, _dbl, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int]),
    ("pisco_set_beam_scalar", ctypes.c_int, [_vp, _i32, _i32, _dbl, _vp, _dbl, _dbl, _dbl, _dbl, ctypes.c_int,
                                             ctypes.c_int]),
    ("pisco_share_beam", ctypes.c_int, [_vp, _i32, _i32]),
    ("pisco_set_beam_healpix", ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _i32, _dbl, ctypes.c_int,
                                              ctypes.c_int]),
    ("pisco_set_beam_healpix_scalar", ctypes.c_int, [_vp, _i32, _i64, _vp, _dbl, _dbl, _dbl, _dbl, _i32, _dbl,
                                                     ctypes.c_int, ctypes.c_int]),
    ("pisco_set_sky_iquv", ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int]),
    ("pisco_set_beam_v", ctypes.c_int, [_vp, _i32, _i32, _dbl, _vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                        ctypes.c_int]),
    ("pisco_set_beam_scalar_v", ctypes.c_int, [_vp, _i32, _i32, _dbl, _vp, _dbl, _dbl, _dbl, _dbl, _dbl,
                                               ctypes.c_int, ctypes.c_int]),
    ("pisco_set_hwp", ctypes.c_int, [_vp, _i32, _i64, _vp, ctypes.c_int]),
    ("pisco_set_detector", ctypes.c_int, [_vp, _i32, _dbl, _dbl, _dbl, ctypes.c_int, _dbl]),
    ("pisco_set_pointing", ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _vp, ctypes.c_int]),
    ("pisco_convolve", ctypes.c_int, [_vp, _i32, ctypes.c_int, _vp, ctypes.c_int, _vp]),
    ("pisco_output_samples", _i64, [_vp, _i32]),
    ("pisco_convolve_static", ctypes.c_int, [_vp, _i32, ctypes.c_int, _vp, _vp]),
    ("pisco_set_launch", ctypes.c_int, [_vp, ctypes.c_void_p]),
    ("pisco_set_ordering", ctypes.c_int, [_vp, _i32]),
    ("pisco_get_launch", ctypes.c_int, [_vp, ctypes.c_void_p]),
    ("pisco_set_timing", ctypes.c_int, [_vp, ctypes.c_int]),
    ("pisco_kernel_time", ctypes.c_int, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_i64), ctypes.c_int]),
    ("pisco_mlp_create", ctypes.c_int, [_vp, _i32, _i32, _i32, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    ("pisco_mlp_destroy", None, [_vp]),
    ("pisco_mlp_param_count", _i64, [_vp]),
    ("pisco_mlp_layout", ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i64), _ip, _ip]),
    ("pisco_mlp_set_params", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("pisco_mlp_get_params", ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    ("pisco_mlp_forward", ctypes.c_int, [_vp, _vp, _i64, _vp, _vp]),
    ("pisco_mlp_gradient", ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    ("pisco_mlp_train_step", ctypes.c_int, [_vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float, _vp, _vp]),
    ("pisco_sidelobe_features", ctypes.c_int, [_vp, _i32, _vp, _vp]),
    ("pisco_sidelobe_apply", ctypes.c_int, [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_dbl), _vp, _vp]),
    ("pisco_sidelobe_set_options", ctypes.c_int, [_vp, ctypes.c_void_p]),
    ("pisco_sidelobe_train", ctypes.c_int, [_vp, _i32, _dbl, _i64, ctypes.c_uint64, _i32]),
    ("pisco_sidelobe_enable", ctypes.c_int, [_vp, _i32, ctypes.c_int]),
    ("pisco_sidelobe_share", ctypes.c_int, [_vp, _i32, _i32]),
    ("pisco_sidelobe_history", _i32, [_vp, _i32, ctypes.POINTER(_dbl), _i32]),
    ("pisco_set_memory_budget", ctypes.c_int, [_vp, _i64]),
    ("pisco_memory_in_use", _i64, [_vp]),
    ("pisco_map_accumulate", ctypes.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, _dbl, _dbl, _dbl,
                                            _vp, _vp]),
    ("pisco_map_solve", ctypes.c_int, [_vp, _i64, _vp, _dbl, _vp, _vp, _vp]),
    ("pisco_alm_size", _i64, [_i32]),
    ("pisco_map2alm_workspace_bytes", _i64, [_i64, _i32, _i32]),
    ("pisco_map2alm", ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    ("pisco_alm2map", ctypes.c_int, [_vp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    ("pisco_alm2cl", ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp]),
    ("pisco_anafast", ctypes.c_int, [_vp, _i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp]),
]

_lib = None


class PiscoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libpisco.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
