"""Seeded synthetic inputs (SplitMix64 counter generator + Box-Muller).

Shared by the tests, the bench and the oracle side.  Holds random-number
generation only: no FFT, Poisson or power-spectrum arithmetic lives here.
The generator definition is in ``synth.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile libsynth.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.synth_sm64_raw.restype = u64
        lib.synth_sm64_raw.argtypes = [u64, u64]
        lib.synth_u64.restype = u64
        lib.synth_u64.argtypes = [u64, u64, u64]
        for name in ("synth_uniform_f64", "synth_normal_f64", "synth_normal_f32"):
            getattr(lib, name).restype = None
            getattr(lib, name).argtypes = [u64, u64, u64, i64, vp]
        lib.synth_choice.restype = None
        lib.synth_choice.argtypes = [u64, u64, i64, i64, vp]
        _lib = lib
    return _lib


def sm64_raw(state: int, i: int) -> int:
    """Output i of the raw SplitMix64 generator started from `state`."""
    return int(_load().synth_sm64_raw(state, i))


def u64(seed: int, stream: int, i: int) -> int:
    return int(_load().synth_u64(seed, stream, i))


def uniform(seed: int, n: int, stream: int = 0, offset: int = 0) -> np.ndarray:
    out = np.empty(int(n), dtype=np.float64)
    _load().synth_uniform_f64(seed, stream, offset, out.size, out.ctypes.data)
    return out


def normal(seed: int, n: int, stream: int = 0, offset: int = 0, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) values; float32 output is the float64 value rounded once."""
    if np.dtype(dtype) == np.float32:
        out = np.empty(int(n), dtype=np.float32)
        _load().synth_normal_f32(seed, stream, offset, out.size, out.ctypes.data)
    else:
        out = np.empty(int(n), dtype=np.float64)
        _load().synth_normal_f64(seed, stream, offset, out.size, out.ctypes.data)
    return out


def choice(seed: int, n: int, m: int, stream: int = 0) -> np.ndarray:
    """n integers uniform in [0, m)."""
    out = np.empty(int(n), dtype=np.int64)
    _load().synth_choice(seed, stream, out.size, int(m), out.ctypes.data)
    return out


def white_field(seed: int, shape, ncomp: int = 1, complex_values: bool = False,
                stream: int = 0) -> np.ndarray:
    """Dense AoS field of i.i.d. N(0,1) float32 values in memory order.

    shape is (N0, N1, N2) with N0 fastest; the returned array has C shape
    (N2, N1, N0, ncomp[, 2]) with the component (and re/im) innermost.
    Value i of the flat memory order is normal(seed, stream, i).
    """
    n0, n1, n2 = (int(s) for s in shape)
    inner = ncomp * (2 if complex_values else 1)
    flat = normal(seed, n0 * n1 * n2 * inner, stream=stream, dtype=np.float32)
    arr = flat.reshape(n2, n1, n0, ncomp, 2) if complex_values else flat.reshape(n2, n1, n0, ncomp)
    return arr
