"""ctypes access to oracle/liboracle.so (built on first use)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.ora_solid_S.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, _D, _D]
        L.ora_green_periodic.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_int, _D]
        L.ora_lower_gamma_half.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.ora_direct.argtypes = [ctypes.c_int64, _D, _D, _D, _D]
        L.ora_direct_at.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int64), _D, _D]
        L.ora_ewald.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, _D]
        L.ora_near.argtypes = [ctypes.c_int64, _D, _D, _I, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, ctypes.c_int, _D, _D]
        _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def iptr(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def set_threads(n: int | None):
    if n is not None:
        os.environ["OMP_NUM_THREADS"] = str(n)
