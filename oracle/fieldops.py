"""FP64 reference of the field operations of the paper's second benchmark
(section 4.2): the periodic halo update of a field with halo width h
(section 3.3.1, the halo layout of section 3.4) and the first-order spatial
derivative of every component stored in another field.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy on the
definitions; it shares no code with the GPU library.

Arrays use the C shape (N2 + 2h, N1 + 2h, N0 + 2h, ncomp): dimension 0
(x) fastest, components innermost.
"""
from __future__ import annotations

import numpy as np


def interior(padded, h):
    """The N2 x N1 x N0 interior of a halo-padded array."""
    if h == 0:
        return padded
    return padded[h:-h, h:-h, h:-h]


def halo_fill(padded, h):
    """Periodic halo update: every halo site takes the value of the interior
    site at its coordinates taken modulo the lattice extent (section 3.3.1:
    halo sites hold copies of the neighbouring sites, which on a periodic
    lattice held by one process are the sites across the boundary)."""
    out = np.array(padded, copy=True)
    n2, n1, n0 = (s - 2 * h for s in padded.shape[:3])
    z = (np.arange(n2 + 2 * h) - h) % n2 + h
    y = (np.arange(n1 + 2 * h) - h) % n1 + h
    x = (np.arange(n0 + 2 * h) - h) % n0 + h
    src = np.asarray(padded)
    out[...] = src[z][:, y][:, :, x]
    return out


def gradient(field, dx=1.0):
    """First-order forward difference of every component along each axis:
    out[z, y, x, 3 c + i] = (f(x + e_i) - f(x))_c / dx on the periodic lattice
    (dense field of C shape (N2, N1, N0, ncomp)); i = 0, 1, 2 for x, y, z."""
    f = np.asarray(field, dtype=np.float64)
    n2, n1, n0, nc = f.shape
    out = np.empty((n2, n1, n0, 3 * nc), dtype=np.float64)
    for i, axis in enumerate((2, 1, 0)):  # x, y, z are C axes 2, 1, 0
        d = (np.roll(f, -1, axis=axis) - f) / dx
        out[..., i::3] = d
    return out
