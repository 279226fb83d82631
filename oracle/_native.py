"""Oracle: loader of the textbook FP64 FFT (test infrastructure only).

Builds ``fft64.c`` with gcc into ``_fft64.so`` next to it when that library is
missing, and exposes the 1-D and 2-D transforms on numpy ``complex128`` arrays.
Only tests, the smoke check and the benchmark's CPU-baseline leg use this.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fft64.c")
_LIB = os.path.join(_HERE, "_fft64.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle FFT with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_fft1.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
            lib.oracle_fft1.restype = ctypes.c_int
            lib.oracle_fft2.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int, ctypes.c_int]
            lib.oracle_fft2.restype = ctypes.c_int
            lib.oracle_twiddle.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
            lib.oracle_twiddle.restype = None
            lib.oracle_max_threads.argtypes = []
            lib.oracle_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def fft1(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Unnormalised 1-D DFT (sign -1 forward, +1 inverse) of a power-of-two vector."""
    a = np.array(x, dtype=np.complex128, copy=True, order="C").reshape(-1)
    rc = _load().oracle_fft1(a.ctypes.data, a.size, int(bool(inverse)))
    if rc != 0:
        raise ValueError("oracle FFT length must be a power of two, got %d" % a.size)
    return a


def fft2(x: np.ndarray, inverse: bool = False, threads: int = 0) -> np.ndarray:
    """Unnormalised 2-D DFT of a row-major [ny][nx] power-of-two array."""
    a = np.array(x, dtype=np.complex128, copy=True, order="C")
    if a.ndim != 2:
        raise ValueError("fft2 expects a 2-D array")
    rc = _load().oracle_fft2(a.ctypes.data, a.shape[0], a.shape[1], int(bool(inverse)),
                             int(threads))
    if rc != 0:
        raise ValueError("oracle FFT sizes must be powers of two, got %s" % (a.shape,))
    return a


def twiddle(k: int, m: int) -> complex:
    out = np.zeros(2, dtype=np.float64)
    _load().oracle_twiddle(int(k), int(m), out.ctypes.data)
    return complex(out[0], out[1])


def max_threads() -> int:
    return int(_load().oracle_max_threads())
