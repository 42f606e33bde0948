"""Pins of the oracle's Poisson solve and power-spectrum binning.

Poisson: closed-form solution of a sinusoidal source, and the 7-point
discrete Laplacian of the discrete-k^2 solution returning the source.
P(k): shell counts by brute-force enumeration, the sum rule, plane-wave
spectra, the deterministic spectrum of a fixed-amplitude random field and
the white-noise normalisation.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def grid(n0, n1, n2):
    z, y, x = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    return x, y, z


@pytest.mark.parametrize("shape,m,dx", [((32, 32, 32), (1, 2, 3), 1.0), ((16, 12, 10), (3, 0, 2), 0.5),
                                        ((24, 20, 8), (5, 4, 1), 2.0), ((32, 32, 32), (16, 0, 0), 1.0)])
def test_poisson_sinusoid_closed_form(shape, m, dx):
    n0, n1, n2 = shape
    x, y, z = grid(*shape)
    arg = 2 * np.pi * (m[0] * x / n0 + m[1] * y / n1 + m[2] * z / n2)
    rho = np.sin(arg) + np.cos(arg)
    km2 = sum((2 * np.pi * ((mi if 2 * mi < ni else mi - ni)) / (ni * dx)) ** 2
              for mi, ni in zip(m, shape))
    phi = oracle.poisson(rho, dx=dx)
    assert np.abs(phi - (-rho / km2)).max() < 1e-12 * np.abs(rho / km2).max()


@pytest.mark.parametrize("shape,dx", [((16, 12, 10), 1.0), ((32, 32, 32), 0.25), ((10, 6, 20), 3.0)])
def test_poisson_discrete_laplacian_residual(shape, dx):
    n0, n1, n2 = shape
    rho = synth.normal(21, n0 * n1 * n2).reshape(n2, n1, n0)
    phi = oracle.poisson(rho, dx=dx, k2mode=oracle.K2_DISCRETE)
    lap = sum(np.roll(phi, 1, a) + np.roll(phi, -1, a) - 2 * phi for a in range(3)) / dx ** 2
    assert np.abs(lap - (rho - rho.mean())).max() < 1e-11 * np.abs(rho).max()
    assert abs(phi.mean()) < 1e-13 * np.abs(phi).max()


def test_poisson_continuous_zero_mean_and_linearity():
    shape = (16, 16, 16)
    a = synth.normal(1, 4096).reshape(16, 16, 16)
    b = synth.normal(2, 4096).reshape(16, 16, 16)
    pa, pb = oracle.poisson(a), oracle.poisson(b)
    assert abs(pa.mean()) < 1e-14
    assert np.abs(oracle.poisson(a + 3 * b) - (pa + 3 * pb)).max() < 1e-12


def brute_counts(shape, nbins, half):
    """Enumerate lattice modes and bin |k| / k_max with exact rationals."""
    n0, n1, n2 = shape
    kmax2 = sum((ni // 2) ** 2 / ni ** 2 for ni in shape)
    counts = np.zeros(nbins)
    nx = n0 // 2 + 1 if half else n0
    for kz, ky, kx in itertools.product(range(n2), range(n1), range(nx)):
        if (kx, ky, kz) == (0, 0, 0):
            continue
        s = [(k if 2 * k < n else k - n) for k, n in zip((kx, ky, kz), shape)]
        k2 = sum(si * si / (ni * ni) for si, ni in zip(s, shape))
        # largest b with (b/nbins)^2 kmax2 <= k2, by exact integer comparison via Fractions
        from fractions import Fraction
        r = Fraction(sum(Fraction(si * si, ni * ni) for si, ni in zip(s, shape)))
        r /= sum(Fraction((ni // 2) ** 2, ni * ni) for ni in shape)
        b = 0
        while Fraction((b + 1) ** 2, nbins ** 2) <= r:
            b += 1
        b = min(b, nbins - 1)
        w = 1.0
        if half and kx not in (0, n0 // 2):
            w = 2.0
        counts[b] += w
    return counts


@pytest.mark.parametrize("shape,nbins", [((8, 8, 8), 4), ((12, 6, 10), 7), ((16, 8, 4), 5), ((6, 10, 15), 3)])
def test_bin_counts_brute(shape, nbins):
    n0, n1, n2 = shape
    F = np.ones((n2, n1, n0 // 2 + 1), dtype=np.complex128)
    if n0 % 2 == 0:
        _, _, ct = oracle.power_spectrum(F, shape, nbins, half=True)
        assert np.array_equal(ct, brute_counts(shape, nbins, True))
    G = np.ones((n2, n1, n0), dtype=np.complex128)
    _, _, ct = oracle.power_spectrum(G, shape, nbins, half=False)
    assert np.array_equal(ct, brute_counts(shape, nbins, False))


def test_bin_counts_32cube_sum_rule():
    shape = (32, 32, 32)
    F = np.ones((32, 32, 17), dtype=np.complex128)
    _, _, ct = oracle.power_spectrum(F, shape, 16)
    assert ct.sum() == 32 ** 3 - 1
    assert np.array_equal(ct, brute_counts(shape, 16, True))


def test_bin_rule_isotropic_equivalence():
    """For a cubic lattice the integer rule equals floor(nbins |k| / k_max) away from ties."""
    N, nbins = 64, 16
    qmax = oracle.pk_qmax((N, N, N))
    assert qmax == 3 * (N // 2) ** 2
    for q in range(1, qmax + 1, 7):
        b = oracle.pk_bin(q, qmax, nbins)
        t = nbins * math.sqrt(q / qmax)
        if abs(t - round(t)) > 1e-9:
            assert b == min(nbins - 1, int(math.floor(t)))
        else:  # exact tie: the boundary belongs to the upper bin
            assert b == min(nbins - 1, int(round(t)))


def test_anisotropic_lcm():
    assert oracle.lcm3((128, 192, 256)) == 768
    assert oracle.lcm3((160, 192, 256)) == 3840
    assert oracle.pk_qmax((128, 192, 256)) == 3 * 384 ** 2


@pytest.mark.parametrize("m", [(3, 2, 1), (0, 4, 0), (16, 0, 0), (16, 16, 16)])
def test_plane_wave_power_spectrum(m):
    """A single cosine puts all power in one bin: P_b = N/(2 count_b), or N/count_b if self-conjugate."""
    shape = (32, 32, 32)
    N, nbins = 32 ** 3, 16
    x, y, z = grid(*shape)
    f = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / 32)
    pk, km, ct = oracle.power_spectrum(oracle.r2c(f), shape, nbins)
    q = sum((mi if 2 * mi < 32 else mi - 32) ** 2 for mi in m)
    b = oracle.pk_bin(q, oracle.pk_qmax(shape), nbins)
    selfconj = all(mi in (0, 16) for mi in m)
    expect = np.zeros(nbins)
    expect[b] = N / ct[b] if selfconj else N / (2 * ct[b])
    assert np.abs(pk - expect).max() < 1e-10 * expect.max()


@pytest.mark.parametrize("shape,alpha", [((32, 32, 32), 3.0), ((16, 24, 12), 2.0)])
def test_grf_spectrum_deterministic(shape, alpha):
    """Fixed-amplitude phases: P_b is exactly scale^2/N * mean_b(|k|^-alpha)."""
    n0, n1, n2 = shape
    N = n0 * n1 * n2
    u = synth.uniform(2, N)
    f, scale = oracle.grf(shape, alpha, u)
    assert abs(f.var() - 1.0) < 1e-12 and abs(f.mean()) < 1e-12
    nbins = 8
    pk, km, ct = oracle.power_spectrum(oracle.r2c(f), shape, nbins)
    # expected: weighted mean of |k|^-alpha per bin from the enumeration
    L = oracle.lcm3(shape)
    qmax = oracle.pk_qmax(shape)
    nh = n0 // 2 + 1
    num = np.zeros(nbins)
    den = np.zeros(nbins)
    for kz, ky, kx in itertools.product(range(n2), range(n1), range(nh)):
        if (kx, ky, kz) == (0, 0, 0):
            continue
        s = [(k if 2 * k < n else k - n) for k, n in zip((kx, ky, kz), shape)]
        q = sum((si * (L // ni)) ** 2 for si, ni in zip(s, shape))
        kk = math.sqrt(sum((2 * math.pi * si / ni) ** 2 for si, ni in zip(s, shape)))
        w = 1.0 if kx in (0, n0 // 2) else 2.0
        b = oracle.pk_bin(q, qmax, nbins)
        num[b] += w * kk ** (-alpha)
        den[b] += w
    expect = scale ** 2 / N * num / np.where(den > 0, den, 1)
    assert np.allclose(ct, den)
    assert np.abs(pk - expect).max() < 1e-10 * expect.max()


def test_white_noise_normalisation():
    shape = (64, 64, 64)
    f = synth.normal(1, 64 ** 3).reshape(64, 64, 64)
    pk, km, ct = oracle.power_spectrum(oracle.r2c(f), shape, 16)
    ok = ct > 200
    assert np.all(np.abs(pk[ok] - 1.0) < 6.0 / np.sqrt(ct[ok]))


def test_kmean_inside_bin():
    shape = (32, 32, 32)
    F = np.ones((32, 32, 17), dtype=np.complex128)
    nbins = 16
    pk, km, ct = oracle.power_spectrum(F, shape, nbins, dx=1.0)
    kmax = 2 * np.pi * math.sqrt(3 * 16 ** 2) / 32
    for b in range(nbins):
        if ct[b] > 0:
            assert b * kmax / nbins - 1e-12 <= km[b] <= (b + 1) * kmax / nbins + 1e-12


# ---- lattice spacing dx != 1 (P_b scales as dx^3, k as 1/dx) -------------
# Expected values come from the definitions: V = N dx^3, P = V/N^2 |F|^2,
# k_i = 2 pi n_i / (N_i dx); nothing below calls the oracle's normalisation.

@pytest.mark.parametrize("dx", [0.5, 0.25])
@pytest.mark.parametrize("m", [(3, 2, 1), (0, 4, 0), (16, 0, 16)])
def test_plane_wave_power_spectrum_dx(m, dx):
    """cos(2 pi m.x / N) at spacing dx: P_b = dx^3 N / (2 count_b), dx^3 N / count_b if self-conjugate."""
    shape = (32, 32, 32)
    N, nbins = 32 ** 3, 16
    x, y, z = grid(*shape)
    f = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / 32)
    pk, km, ct = oracle.power_spectrum(oracle.r2c(f), shape, nbins, dx=dx)
    # the bin from the brute-force enumeration's count of the mode's shell
    q = sum((mi if 2 * mi < 32 else mi - 32) ** 2 for mi in m)
    b = oracle.pk_bin(q, oracle.pk_qmax(shape), nbins)
    selfconj = all(mi in (0, 16) for mi in m)
    expect = np.zeros(nbins)
    expect[b] = dx ** 3 * N / ct[b] if selfconj else dx ** 3 * N / (2 * ct[b])
    assert np.abs(pk - expect).max() < 1e-10 * expect.max()
    assert np.array_equal(ct, brute_counts(shape, nbins, True))


def brute_kmean(shape, nbins, dx, half):
    """Weighted mean of |k| = 2 pi sqrt(sum (n_i / N_i)^2) / dx per bin over
    every lattice mode, each binned with exact rationals."""
    from fractions import Fraction
    n0, n1, n2 = shape
    kmax2 = sum(Fraction((ni // 2) ** 2, ni * ni) for ni in shape)
    nx = n0 // 2 + 1 if half else n0
    sk = np.zeros(nbins)
    sw = np.zeros(nbins)
    for kz, ky, kx in itertools.product(range(n2), range(n1), range(nx)):
        if (kx, ky, kz) == (0, 0, 0):
            continue
        s = [(k if 2 * k < n else k - n) for k, n in zip((kx, ky, kz), shape)]
        r = sum(Fraction(si * si, ni * ni) for si, ni in zip(s, shape)) / kmax2
        b = 0
        while Fraction((b + 1) ** 2, nbins ** 2) <= r:
            b += 1
        b = min(b, nbins - 1)
        w = 2.0 if half and kx not in (0, n0 // 2) else 1.0
        kk = 2 * math.pi * math.sqrt(sum((si / ni) ** 2 for si, ni in zip(s, shape))) / dx
        sk[b] += w * kk
        sw[b] += w
    return np.where(sw > 0, sk / np.where(sw > 0, sw, 1), 0.0)


@pytest.mark.parametrize("dx", [0.5, 0.25])
@pytest.mark.parametrize("shape,nbins,half", [((16, 16, 16), 6, True), ((12, 8, 10), 5, True),
                                              ((12, 8, 10), 4, False)])
def test_kmean_brute_dx(shape, nbins, dx, half):
    """k-bar_b equals the brute-force weighted mean of |k| over the bin's modes."""
    n0, n1, n2 = shape
    nx = n0 // 2 + 1 if half else n0
    F = np.ones((n2, n1, nx), dtype=np.complex128)
    _, km, _ = oracle.power_spectrum(F, shape, nbins, dx=dx, half=half)
    want = brute_kmean(shape, nbins, dx, half)
    assert np.abs(km - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("dx", [0.5, 0.25])
def test_white_noise_normalisation_dx(dx):
    """i.i.d. N(0,1) sites at spacing dx: E[P_b] = dx^3 (within 6 / sqrt(count_b), relative)."""
    shape = (64, 64, 64)
    f = synth.normal(3, 64 ** 3).reshape(64, 64, 64)
    pk, km, ct = oracle.power_spectrum(oracle.r2c(f), shape, 16, dx=dx)
    ok = ct > 200
    assert ok.sum() >= 10
    assert np.all(np.abs(pk[ok] / dx ** 3 - 1.0) < 6.0 / np.sqrt(ct[ok]))


def test_power_spectrum_dx_scaling_law():
    """Same spectrum at two spacings: P scales exactly as dx^3, k-bar as 1/dx, counts unchanged."""
    shape = (16, 12, 20)
    f = synth.normal(5, 16 * 12 * 20).reshape(20, 12, 16)
    F = oracle.r2c(f)
    p1, k1, c1 = oracle.power_spectrum(F, shape, 7, dx=1.0)
    p2, k2, c2 = oracle.power_spectrum(F, shape, 7, dx=0.37)
    assert np.array_equal(c1, c2)
    assert np.allclose(p2, p1 * 0.37 ** 3, rtol=1e-13, atol=0)
    assert np.allclose(k2, k1 / 0.37, rtol=1e-13, atol=0)
