"""MI355X-native pixel-space polarised beam convolution (PISCO's hot path).

The convolution, batching and sidelobe-network kernels are hand-written HIP
for gfx950 in ``csrc/`` behind the C ABI of ``include/pisco.h``; this
package is the thin Python binding (``Convolver``) plus host-side beam
preparation.  There is no CPU fallback: without ``libpisco.so`` and a
gfx950 device every call raises.
"""
from ._lib import (DEVICE, F32, F64, HOST, NORM_FIXED, NORM_PER_SAMPLE, OUT_COUNT, OUT_STOKES,  # noqa: F401
                   OUT_TOD, PiscoError)
from .beamsor import fold_detector, fold_elements, grid_solid_angle  # noqa: F401


def __getattr__(name):
    if name == "Convolver":
        from .api import Convolver

        return Convolver
    raise AttributeError(name)
