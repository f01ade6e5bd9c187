"""Loader for the generators' small C helper (built by ``__graft_entry__.build``)."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alm2ring.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_handle = None


def build(force: bool = True) -> str:
    """Compile the helper with gcc + OpenMP (portable -O3, no -march=native)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB, "-lm"])
    return _LIB


def lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB):
            build(force=True)
        h = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        h.synth_ring_coeffs.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        h.synth_ring_coeffs.restype = None
        h.synth_ring_coeffs_spin2.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_int, dp, dp] + [dp] * 8
        h.synth_ring_coeffs_spin2.restype = None
        _handle = h
    return _handle
