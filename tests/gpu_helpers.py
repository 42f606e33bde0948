"""Shared helpers of the GPU parity tests (inputs, oracle calls, metrics)."""
from __future__ import annotations

import math

import numpy as np

import oracle
import synth


def tol(shape) -> float:
    """rel-L2 gate 1e-5 * log2(N), N = total lattice points."""
    N = int(np.prod(shape))
    return 1e-5 * math.log2(max(N, 2))


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def rel_max(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    mb = np.abs(b).max()
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0))


def real_field(shape, seed, ncomp=1, halo=0):
    """(dense float32 (N2,N1,N0,ncomp), halo-padded float32 with NaN halos)."""
    n0, n1, n2 = shape
    dense = synth.white_field(seed, shape, ncomp)
    if halo == 0:
        return dense, dense
    h = halo
    pad = np.full((n2 + 2 * h, n1 + 2 * h, n0 + 2 * h, ncomp), np.nan, dtype=np.float32)
    pad[h:h + n2, h:h + n1, h:h + n0] = dense
    return dense, pad


def complex_field(shape, seed, ncomp=1):
    n0, n1, n2 = shape
    a = synth.white_field(seed, shape, ncomp, complex_values=True)
    return (a[..., 0] + 1j * a[..., 1]).astype(np.complex64)


def grf_field(shape, alpha, seed):
    """Fixed-amplitude GRF from the oracle: (float32 field, float64 field, scale)."""
    n0, n1, n2 = shape
    u = synth.uniform(seed, n0 * n1 * n2)
    f64, scale = oracle.grf(shape, alpha, u)
    f32 = f64.astype(np.float32)
    return f32, f32.astype(np.float64), scale


def assert_close(got, ref, shape, what: str = "") -> tuple[float, float]:
    """Gate a GPU result against the oracle on rel-L2 AND on max error.

    Both must be within 1e-5 * log2(N).  The max gate (max|a - b| / max|b|)
    catches a localized fault that the L2 norm dilutes: at 512^3 one fully
    wrong mode of a half spectrum moves rel-L2 by only ~1e-4."""
    t = tol(shape)
    e, em = rel_l2(got, ref), rel_max(got, ref)
    if what:
        print(f"  [{what}] rel-L2 {e:.3e} max {em:.3e} tol {t:.2e}", flush=True)
    assert e <= t, f"{what}: rel-L2 {e:.3e} above {t:.3e}"
    assert em <= t, f"{what}: max error {em:.3e} above {t:.3e}"
    return e, em
