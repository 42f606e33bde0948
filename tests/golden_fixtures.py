"""Readers of the fixtures under tests/golden/ (values fixed by hand-derived
closed forms; each file states its derivation and the section it follows)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def spectrum(name, shape):
    """The full complex spectrum of a DFT fixture, C shape (N2, N1, N0)."""
    rows = np.loadtxt(os.path.join(GOLDEN, name), comments="#")
    n0, n1, n2 = shape
    F = np.full((n2, n1, n0), np.nan + 0j)
    for k0, k1, k2, re, im in rows:
        F[int(k2), int(k1), int(k0)] = re + 1j * im
    assert not np.isnan(F.real).any(), f"{name} does not cover every mode"
    return F


def ramp_2x2x2():
    """f(n0, n1, n2) = n0 + 2 n1 + 4 n2 and its spectrum."""
    n = np.arange(2)
    f = n[None, None, :] + 2 * n[None, :, None] + 4 * n[:, None, None]
    return f.astype(np.float64), spectrum("dft_ramp_2x2x2.txt", (2, 2, 2))


def line_4x2x2():
    """x = (1, 2, 3, 4) along dimension 0 at n1 = n2 = 0, and its spectrum."""
    f = np.zeros((2, 2, 4))
    f[0, 0, :] = [1.0, 2.0, 3.0, 4.0]
    return f, spectrum("dft_line_4x2x2.txt", (4, 2, 2))


def poisson_cos_8x4x4():
    """rho = cos(2 pi n0 / 8) on 8 x 4 x 4 and the cases (dx, k2mode, A) of
    phi = A rho."""
    n0 = np.arange(8)
    rho = np.broadcast_to(np.cos(2 * np.pi * n0 / 8)[None, None, :], (4, 4, 8)).copy()
    rows = np.loadtxt(os.path.join(GOLDEN, "poisson_cos_8x4x4.txt"), comments="#")
    return rho, [(float(dx), int(m), float(a)) for dx, m, a in rows]
