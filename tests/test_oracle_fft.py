"""Pins of the FP64 oracle's transforms against facts independent of it.

Each check is something the oracle's code does not restate: the O(N^2)
definition evaluated by brute force in numpy, an independent library FFT
(numpy's pocketfft), closed forms (plane waves, shift theorem), Parseval,
Hermitian symmetry and the exact round trip.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

TINY = [(4, 6, 10), (6, 10, 12), (8, 8, 8), (16, 1, 1), (1, 1, 16), (2, 3, 5), (10, 4, 6)]


def brute_dft3(f, sign=-1):
    """Definition of the 3-D DFT as an explicit matrix product (numpy)."""
    n2, n1, n0 = f.shape
    xs = np.stack(np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij"),
                  -1).reshape(-1, 3)
    ph = (np.outer(xs[:, 0], xs[:, 0]) % n2) / n2 + (np.outer(xs[:, 1], xs[:, 1]) % n1) / n1 \
        + (np.outer(xs[:, 2], xs[:, 2]) % n0) / n0
    M = np.exp(sign * 2j * np.pi * ph)
    return (M @ f.reshape(-1).astype(np.complex128)).reshape(f.shape)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 9, 12, 15, 16, 24, 25, 30, 32, 48, 49, 60, 64,
                               96, 128, 160, 192, 7, 11, 14])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_vs_direct_definition(n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    j = np.arange(n)
    direct = np.exp(sign * 2j * np.pi * ((np.outer(j, j) % n) / n)) @ x
    assert rel(oracle.fft1d(x, sign), direct) < 1e-13
    assert rel(oracle.dft1d(x, sign), direct) < 1e-13


@pytest.mark.parametrize("shape", TINY)
@pytest.mark.parametrize("sign", [-1, 1])
def test_c2c3d_vs_brute(shape, sign):
    n0, n1, n2 = shape
    rng = np.random.default_rng(sum(shape))
    f = rng.standard_normal((n2, n1, n0)) + 1j * rng.standard_normal((n2, n1, n0))
    assert rel(oracle.c2c(f, sign), brute_dft3(f, sign)) < 1e-13


@pytest.mark.parametrize("shape", [s for s in TINY if s[0] % 2 == 0])
def test_r2c3d_vs_brute(shape):
    n0, n1, n2 = shape
    f = np.random.default_rng(7).standard_normal((n2, n1, n0))
    F = oracle.r2c(f)
    assert F.shape == (n2, n1, n0 // 2 + 1)
    assert rel(F, brute_dft3(f)[:, :, : n0 // 2 + 1]) < 1e-13


@pytest.mark.parametrize("shape", [(32, 32, 32), (96, 20, 12), (160, 6, 10), (24, 40, 18), (64, 48, 30)])
def test_against_numpy_pocketfft(shape):
    """Independent library FFT (numpy's pocketfft), test-side only."""
    n0, n1, n2 = shape
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n2, n1, n0))
    assert rel(oracle.r2c(f), np.fft.rfftn(f)) < 1e-13
    z = f + 1j * rng.standard_normal(f.shape)
    assert rel(oracle.c2c(z, -1), np.fft.fftn(z)) < 1e-13
    assert rel(oracle.c2c(z, +1), np.fft.ifftn(z) * z.size) < 1e-13
    H = oracle.r2c(f)
    assert rel(oracle.c2r(H, n0), np.fft.irfftn(H, s=f.shape, axes=(0, 1, 2)) * f.size) < 1e-13


@pytest.mark.parametrize("shape", [(32, 32, 32), (12, 10, 6), (96, 64, 32)])
def test_round_trip_exact(shape):
    n0, n1, n2 = shape
    f = synth.normal(11, n0 * n1 * n2).reshape(n2, n1, n0)
    back = oracle.c2r(oracle.r2c(f), n0) / f.size
    assert np.abs(back - f).max() / np.abs(f).max() < 1e-14
    z = f + 1j * synth.normal(12, f.size).reshape(f.shape)
    back = oracle.c2c(oracle.c2c(z, -1), +1) / z.size
    assert np.abs(back - z).max() / np.abs(z).max() < 1e-14


def half_weights(n0, nh):
    w = np.full(nh, 2.0)
    w[0] = 1.0
    if n0 % 2 == 0:
        w[n0 // 2] = 1.0
    return w


@pytest.mark.parametrize("shape", [(32, 32, 32), (20, 12, 6), (64, 96, 10)])
def test_parseval(shape):
    n0, n1, n2 = shape
    f = synth.normal(5, n0 * n1 * n2).reshape(n2, n1, n0)
    F = oracle.r2c(f)
    w = half_weights(n0, n0 // 2 + 1)
    lhs = np.sum(f * f)
    rhs = np.sum(w[None, None, :] * np.abs(F) ** 2) / f.size
    assert abs(lhs - rhs) / lhs < 1e-13


@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 10, 6), (8, 6, 10)])
def test_hermitian_planes(shape):
    """On the k_x = 0 and k_x = N0/2 planes F(-k) = conj F(k); self-conjugate modes are real."""
    n0, n1, n2 = shape
    f = synth.normal(9, n0 * n1 * n2).reshape(n2, n1, n0)
    F = oracle.r2c(f)
    for kx in (0, n0 // 2):
        P = F[:, :, kx]
        Pm = P[(-np.arange(n2)) % n2][:, (-np.arange(n1)) % n1]
        assert np.abs(P - np.conj(Pm)).max() < 1e-12
        for kz in {0, n2 // 2} if n2 % 2 == 0 else {0}:
            for ky in {0, n1 // 2} if n1 % 2 == 0 else {0}:
                assert abs(P[kz, ky].imag) < 1e-12


@pytest.mark.parametrize("m", [(1, 0, 0), (3, 2, 1), (0, 0, 5), (4, 3, 2), (8, 0, 0), (8, 6, 5)])
def test_plane_wave_delta(m):
    """cos(2 pi m.x/N) transforms to N/2 at +m and -m (N if m is self-conjugate), 0 elsewhere."""
    n0, n1, n2 = 16, 12, 10
    z, y, x = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    f = np.cos(2 * np.pi * (m[0] * x / n0 + m[1] * y / n1 + m[2] * z / n2))
    N = f.size
    F = oracle.c2c(f.astype(np.complex128), -1)
    mm = tuple((-np.array(m)) % np.array([n0, n1, n2]))
    expect = np.zeros_like(F)
    selfconj = mm == tuple(m)
    expect[m[2], m[1], m[0]] = N if selfconj else N / 2
    expect[mm[2], mm[1], mm[0]] = N if selfconj else N / 2
    assert np.abs(F - expect).max() < 1e-10 * N
    H = oracle.r2c(f)
    assert np.abs(H - expect[:, :, : n0 // 2 + 1]).max() < 1e-10 * N


@pytest.mark.parametrize("axis_shift", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 3, 1)])
def test_shift_theorem(axis_shift):
    """Translating f by s multiplies F(k) by exp(-2 pi i k.s / N)."""
    n0, n1, n2 = 12, 10, 8
    rng = np.random.default_rng(1)
    f = rng.standard_normal((n2, n1, n0)) + 1j * rng.standard_normal((n2, n1, n0))
    sx, sy, sz = axis_shift
    g = np.roll(f, shift=(sz, sy, sx), axis=(0, 1, 2))  # g(x) = f(x - s)
    kz, ky, kx = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    phase = np.exp(-2j * np.pi * (kx * sx / n0 + ky * sy / n1 + kz * sz / n2))
    assert rel(oracle.c2c(g, -1), oracle.c2c(f, -1) * phase) < 1e-13


def test_linearity():
    n = (10, 6, 4)
    rng = np.random.default_rng(2)
    a = rng.standard_normal((4, 6, 10))
    b = rng.standard_normal((4, 6, 10))
    assert rel(oracle.r2c(2.5 * a - 0.75 * b), 2.5 * oracle.r2c(a) - 0.75 * oracle.r2c(b)) < 1e-14


@pytest.mark.parametrize("shape", [(4, 3, 2), (6, 4, 3), (8, 2, 5)])
def test_c2r_reprojection_non_hermitian(shape):
    """c2r of an arbitrary half spectrum equals sum_k c(k_x) Re(G_k e^{+ik.x}) term by term."""
    n0, n1, n2 = shape
    nh = n0 // 2 + 1
    rng = np.random.default_rng(4)
    G = rng.standard_normal((n2, n1, nh)) + 1j * rng.standard_normal((n2, n1, nh))
    out = oracle.c2r(G, n0)
    ref = np.zeros((n2, n1, n0))
    for z, y, x in itertools.product(range(n2), range(n1), range(n0)):
        s = 0.0
        for kz, ky, kx in itertools.product(range(n2), range(n1), range(nh)):
            c = 1.0 if kx in (0, n0 // 2) else 2.0
            ph = 2 * np.pi * (kx * x / n0 + ky * y / n1 + kz * z / n2)
            s += c * (G[kz, ky, kx] * np.exp(1j * ph)).real
        ref[z, y, x] = s
    assert np.abs(out - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("k", [(0, 0, 0), (3, 5, 7), (31, 1, 16), (17, 30, 2)])
def test_dft3d_at_matches_full(k):
    n0, n1, n2 = 32, 32, 32
    f = synth.normal(1, n0 * n1 * n2).reshape(n2, n1, n0)
    full = oracle.c2c(f.astype(np.complex128), -1)
    v = oracle.dft3d_at(f, k)
    assert abs(v - full[k[2], k[1], k[0]]) < 1e-11 * np.abs(full).max()
    z = f + 1j * f[::-1]
    fullz = oracle.c2c(z, +1)
    assert abs(oracle.dft3d_at(z, k, +1) - fullz[k[2], k[1], k[0]]) < 1e-11 * np.abs(fullz).max()
