"""Pins of the field-operation oracle (paper section 4.2): halo fill and the
first-order derivative against facts independent of its code."""
import numpy as np
import pytest

from oracle import fieldops


def padded_random(shape, h, nc, seed):
    n0, n1, n2 = shape
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n2 + 2 * h, n1 + 2 * h, n0 + 2 * h, nc))


@pytest.mark.parametrize("shape,h", [((4, 5, 6), 1), ((8, 3, 2), 2), ((3, 3, 3), 1)])
def test_halo_fill_brute(shape, h):
    """Site by site: each padded site equals the interior site at its wrapped
    coordinates; the interior is untouched."""
    a = padded_random(shape, h, 2, 1)
    b = fieldops.halo_fill(a, h)
    n0, n1, n2 = shape
    for z in range(n2 + 2 * h):
        for y in range(n1 + 2 * h):
            for x in range(n0 + 2 * h):
                src = a[h + (z - h) % n2, h + (y - h) % n1, h + (x - h) % n0]
                assert np.array_equal(b[z, y, x], src)
    assert np.array_equal(fieldops.interior(b, h), fieldops.interior(a, h))


def test_halo_fill_corner_example():
    """A 2 x 2 x 2 lattice with h = 1: the halo corner (0, 0, 0) copies the
    interior site (1, 1, 1) of the far corner."""
    a = np.zeros((4, 4, 4, 1))
    a[2, 2, 2, 0] = 7.0  # interior site z = y = x = 1 (0-based interior)
    b = fieldops.halo_fill(a, 1)
    assert b[0, 0, 0, 0] == 7.0
    assert b[3, 3, 3, 0] == 0.0  # wraps to interior (0, 0, 0)


def test_gradient_constant_and_linear_periodic():
    n = (8, 6, 4)
    f = np.full((n[2], n[1], n[0], 2), 3.5)
    assert np.all(fieldops.gradient(f) == 0.0)
    # a ramp in x wraps once: forward difference 1 everywhere but the last
    # column, where it is -(N0 - 1)
    x = np.arange(n[0], dtype=np.float64)
    g = np.broadcast_to(x, (n[2], n[1], n[0]))[..., None]
    d = fieldops.gradient(g, dx=0.5)
    assert np.all(d[..., :-1, 0] == 2.0)
    assert np.all(d[..., -1, 0] == -(n[0] - 1) / 0.5)
    assert np.all(d[..., 1] == 0.0) and np.all(d[..., 2] == 0.0)


def test_gradient_plane_wave_closed_form():
    """f = exp(2 pi i m.x / N): (f(x + e_i) - f(x)) = f (exp(2 pi i m_i / N_i) - 1)."""
    n0, n1, n2 = 8, 10, 6
    m = (1, 3, 2)
    z, y, x = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    ph = 2 * np.pi * (m[0] * x / n0 + m[1] * y / n1 + m[2] * z / n2)
    f = np.stack([np.cos(ph), np.sin(ph)], axis=-1)
    d = fieldops.gradient(f, dx=1.0)
    for i, (mi, ni) in enumerate(zip(m, (n0, n1, n2))):
        w = np.exp(2j * np.pi * mi / ni) - 1.0
        expect = np.exp(1j * ph) * w
        got = d[..., i] + 1j * d[..., 3 + i]  # component 0 = cos, 1 = sin
        assert np.allclose(got, expect, atol=1e-13)


def test_gradient_component_order():
    n = (4, 4, 4)
    f = np.zeros((4, 4, 4, 2))
    f[0, 0, 1, 1] = 1.0  # component 1 at x = 1
    d = fieldops.gradient(f)
    # x-derivative of component 1 at x = 0 is +1, stored at 3 * 1 + 0
    assert d[0, 0, 0, 3] == 1.0 and d[0, 0, 1, 3] == -1.0
    assert np.count_nonzero(d[..., :3]) == 0
