"""Pins of the paper-layout permutation (section 3.6): element by element,
the k-space site (k_x, k_y, k_z) lands where the stated dimension order puts
it."""
import numpy as np

import oracle


def test_r2c_paper_order_brute():
    nh, n1, n2 = 5, 4, 3
    F = np.arange(n2 * n1 * nh).reshape(n2, n1, nh)  # F[kz, ky, kx]
    P = oracle.to_paper_layout(F, "r2c")
    # dimensions (k_x, k_z, k_y) with k_x fastest: flat = kx + nh (kz + n2 ky)
    flat = P.ravel()
    for kz in range(n2):
        for ky in range(n1):
            for kx in range(nh):
                assert flat[kx + nh * (kz + n2 * ky)] == F[kz, ky, kx]


def test_c2c_paper_order_brute():
    n0, n1, n2 = 4, 3, 5
    F = np.arange(n2 * n1 * n0).reshape(n2, n1, n0)
    P = oracle.to_paper_layout(F, "c2c")
    # dimensions (k_z, k_x, k_y) with k_z fastest: flat = kz + n2 (kx + n0 ky)
    flat = P.ravel()
    for kz in range(n2):
        for ky in range(n1):
            for kx in range(n0):
                assert flat[kz + n2 * (kx + n0 * ky)] == F[kz, ky, kx]


def test_components_stay_innermost():
    F = np.arange(2 * 3 * 4 * 2).reshape(2, 3, 4, 2)
    P = oracle.to_paper_layout(F, "r2c")
    assert P.shape == (3, 2, 4, 2)
    assert np.array_equal(P[1, 0, 2], F[0, 1, 2])
