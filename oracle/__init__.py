"""FP64 CPU oracle for the lf2 3-D FFT / Poisson / power-spectrum path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``; never by the GPU library.  It shares
no code with the HIP path.  The arithmetic lives in ``lf2_oracle.c``; this
module marshals numpy arrays.

Array conventions (lattice N0 x N1 x N2, dimension 0 fastest, paper
section 3.4): real fields are numpy arrays of C shape (N2, N1, N0); complex
fields are complex128 arrays of shape (N2, N1, N0) or, for r2c half
spectra, (N2, N1, N0//2+1).  Multi-component (AoS) fields carry a trailing
component axis; the functions here act on one component at a time.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lf2_oracle.c")
_LIB = os.path.join(_HERE, "liblf2_oracle.so")
_lib = None

FORWARD = -1
BACKWARD = +1


def build() -> str:
    """Compile liblf2_oracle.so (FP64, -ffp-contract=off, OpenMP over lines)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                           "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        sig = {
            "orc_num_threads": (ci, []),
            "orc_set_num_threads": (None, [ci]),
            "orc_dft1d": (None, [i64, vp, vp, ci]),
            "orc_fft1d": (None, [i64, vp, ci]),
            "orc_c2c3d": (None, [vp, vp, vp, ci]),
            "orc_r2c3d": (None, [vp, vp, vp]),
            "orc_c2r3d": (None, [vp, vp, vp]),
            "orc_dft3d_at": (None, [vp, vp, ci, vp, ci, vp]),
            "orc_lcm3": (i64, [vp]),
            "orc_poisson": (None, [vp, cd, ci, vp, vp]),
            "orc_pk_bin": (i64, [i64, i64, i64]),
            "orc_pk_qmax": (i64, [vp]),
            "orc_power_spectrum": (None, [vp, ci, vp, i64, cd, vp, vp, vp]),
            "orc_grf": (cd, [vp, cd, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _dims(shape3):
    return np.ascontiguousarray(np.asarray(shape3, dtype=np.int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def dft1d(x, sign=FORWARD):
    """Direct O(n^2) definition of the 1-D DFT."""
    x = _c128(x)
    out = np.empty_like(x)
    _load().orc_dft1d(x.size, x.ctypes.data, out.ctypes.data, sign)
    return out


def fft1d(x, sign=FORWARD):
    """Mixed-radix (2, 3, 5, then any prime) decimation-in-time 1-D FFT."""
    y = _c128(x).copy()
    _load().orc_fft1d(y.size, y.ctypes.data, sign)
    return y


def shape_of(a, half=False):
    """(N0, N1, N2) of a (N2, N1, N0[h]) array; half spectra need N0 given."""
    n2, n1, n0 = a.shape[:3]
    return (n0, n1, n2)


def c2c(f, sign=FORWARD):
    """Unnormalised 3-D c2c of complex f with C shape (N2, N1, N0)."""
    f = _c128(f)
    n = _dims(shape_of(f))
    out = np.empty_like(f)
    _load().orc_c2c3d(n.ctypes.data, f.ctypes.data, out.ctypes.data, sign)
    return out


def r2c(f):
    """Forward r2c of real f (N2, N1, N0) -> complex (N2, N1, N0//2+1)."""
    f = _f64(f)
    n2, n1, n0 = f.shape
    n = _dims((n0, n1, n2))
    out = np.empty((n2, n1, n0 // 2 + 1), dtype=np.complex128)
    _load().orc_r2c3d(n.ctypes.data, f.ctypes.data, out.ctypes.data)
    return out


def c2r(F, n0):
    """Unnormalised c2r of a half spectrum (N2, N1, n0//2+1) -> real (N2, N1, n0)."""
    F = _c128(F)
    n2, n1, nh = F.shape
    assert nh == n0 // 2 + 1
    n = _dims((n0, n1, n2))
    out = np.empty((n2, n1, n0), dtype=np.float64)
    _load().orc_c2r3d(n.ctypes.data, F.ctypes.data, out.ctypes.data)
    return out


def dft3d_at(f, k, sign=FORWARD):
    """One mode F(k) of the 3-D DFT of f (real or complex, C shape (N2,N1,N0))."""
    is_c = np.iscomplexobj(f)
    f = _c128(f) if is_c else _f64(f)
    n = _dims(shape_of(f))
    kk = _dims(k)
    res = np.empty(2, dtype=np.float64)
    _load().orc_dft3d_at(n.ctypes.data, f.ctypes.data, int(is_c), kk.ctypes.data, sign,
                         res.ctypes.data)
    return complex(res[0], res[1])


def lcm3(shape3) -> int:
    return int(_load().orc_lcm3(_dims(shape3).ctypes.data))


K2_CONTINUOUS = 0
K2_DISCRETE = 1


def poisson(rho, dx=1.0, k2mode=K2_CONTINUOUS):
    """Periodic solution of laplacian(phi) = rho with the zero mode removed."""
    rho = _f64(rho)
    n = _dims(shape_of(rho))
    phi = np.empty_like(rho)
    _load().orc_poisson(n.ctypes.data, float(dx), int(k2mode), rho.ctypes.data, phi.ctypes.data)
    return phi


def pk_bin(q, qmax, nbins) -> int:
    return int(_load().orc_pk_bin(int(q), int(qmax), int(nbins)))


def pk_qmax(shape3) -> int:
    return int(_load().orc_pk_qmax(_dims(shape3).ctypes.data))


def power_spectrum(F, shape3, nbins, dx=1.0, half=True):
    """(pk, kmean, count) of a half (r2c) or full (c2c) spectrum."""
    F = _c128(F)
    n = _dims(shape3)
    pk = np.zeros(nbins)
    km = np.zeros(nbins)
    ct = np.zeros(nbins)
    _load().orc_power_spectrum(n.ctypes.data, int(bool(half)), F.ctypes.data, int(nbins),
                               float(dx), pk.ctypes.data, km.ctypes.data, ct.ctypes.data)
    return pk, km, ct


def grf(shape3, alpha, u):
    """Fixed-amplitude Gaussian random field; returns (field, scale).

    u: uniform [0,1) draws, one per full-lattice flat index (N0 fastest).
    """
    n0, n1, n2 = (int(s) for s in shape3)
    u = _f64(u)
    assert u.size == n0 * n1 * n2
    out = np.empty((n2, n1, n0), dtype=np.float64)
    scale = _load().orc_grf(_dims(shape3).ctypes.data, float(alpha), u.ctypes.data,
                            out.ctypes.data)
    return out, float(scale)


def to_paper_layout(F, kind):
    """A natural spectrum (C shape (N2, N1, Nk[, ncomp]), k_x fastest) in the
    k-space order of the paper's distributed transform (section 3.6): for
    r2c the dimensions run (k_x, k_z, k_y), k_x fastest -> C shape
    (N1, N2, Nh); for c2c (k_z, k_x, k_y), k_z fastest -> C shape
    (N1, N0, N2).  A trailing component axis stays innermost."""
    F = np.asarray(F)
    rest = tuple(range(3, F.ndim))
    if kind == "r2c":
        return np.ascontiguousarray(np.transpose(F, (1, 0, 2) + rest))
    if kind == "c2c":
        return np.ascontiguousarray(np.transpose(F, (1, 2, 0) + rest))
    raise ValueError(kind)
