"""GPU parity of the Poisson solve and the power spectrum against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_close, grf_field, real_field, rel_l2, rel_max, tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lf2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_05610_amd as m
    m.load()
    return m


def dev():
    return torch.device("cuda:0")


SHAPES = [(32, 32, 32), (16, 12, 10), (64, 48, 40), (8, 8, 8), (128, 96, 80), (96, 160, 192)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("discrete", [0, 1])
@pytest.mark.parametrize("dx", [1.0, 0.37])
def test_poisson(lf2, shape, discrete, dx):
    print(f"case poisson {shape} discrete={discrete} dx={dx}", flush=True)
    dense, _ = real_field(shape, seed=11)
    f = dense[..., 0]
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    phi = plan.poisson(torch.from_numpy(f).to(dev()), dx=dx,
                       flags=lf2.LF2_POISSON_DISCRETE_K2 if discrete else 0)
    torch.cuda.synchronize()
    ref = oracle.poisson(f.astype(np.float64), dx=dx, k2mode=discrete)
    got = phi.cpu().numpy().astype(np.float64)
    assert_close(got, ref, shape, "phi")


@pytest.mark.parametrize("shape,nbins", [((32, 32, 32), 16), ((64, 48, 40), 24), ((16, 12, 10), 5),
                                         ((128, 96, 80), 64), ((8, 8, 8), 1), ((96, 160, 192), 40)])
def test_power_spectrum_real_space(lf2, shape, nbins):
    print(f"case pk {shape} nbins={nbins}", flush=True)
    dense, _ = real_field(shape, seed=12)
    f = dense[..., 0]
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    xd = torch.from_numpy(f).to(dev())
    pk, km, ct = plan.power_spectrum(xd, nbins, dx=0.5)
    torch.cuda.synchronize()
    opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(f.astype(np.float64)), shape, nbins, dx=0.5)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert_close(pk.cpu().numpy(), opk, shape, "pk")
    print(f"  kmean rel-L2 {rel_l2(km.cpu().numpy(), okm):.3e}", flush=True)
    assert rel_l2(km.cpu().numpy(), okm) <= 1e-12
    # the k-space entry gives the same bins from the spectrum
    F = plan.forward(xd)
    pk2, km2, ct2 = plan.power_spectrum(F, nbins, dx=0.5, field_is_kspace=True)
    torch.cuda.synchronize()
    assert np.array_equal(ct2.cpu().numpy(), oct_)
    assert_close(pk2.cpu().numpy(), opk, shape)


def test_power_spectrum_c2c(lf2):
    shape = (32, 24, 20)
    from gpu_helpers import complex_field
    z = complex_field(shape, seed=13)[..., 0]
    plan = lf2.Plan(shape, lf2.LF2_C2C)
    pk, km, ct = plan.power_spectrum(torch.from_numpy(z).to(dev()), 12)
    torch.cuda.synchronize()
    opk, okm, oct_ = oracle.power_spectrum(oracle.c2c(z.astype(np.complex128), -1), shape, 12,
                                           half=False)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert_close(pk.cpu().numpy(), opk, shape)


@pytest.mark.parametrize("of_phi", [False, True])
def test_poisson_with_pk_and_parseval(lf2, of_phi):
    shape = (64, 48, 40)
    N = int(np.prod(shape))
    dense, _ = real_field(shape, seed=14)
    f = dense[..., 0]
    f64 = f.astype(np.float64)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    flags = lf2.LF2_PK_OF_PHI if of_phi else 0
    res = plan.poisson(torch.from_numpy(f).to(dev()), nbins=20, flags=flags, parseval=not of_phi)
    torch.cuda.synchronize()
    phi, pk, km, ct = res[:4]
    ref_phi = oracle.poisson(f64)
    assert_close(phi.cpu().numpy(), ref_phi, shape)
    src = ref_phi if of_phi else f64
    opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(src), shape, 20)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert_close(pk.cpu().numpy(), opk, shape)
    if not of_phi:
        pv = res[4].cpu().numpy()
        assert abs(pv[0] - np.sum(f64 * f64)) <= 1e-12 * np.sum(f64 * f64)
        assert abs(pv[1] - pv[0]) <= tol(shape) * pv[0]


def test_grf_spectrum_256(lf2):
    """256^3 P(k) ~ k^-3 random field: full-size parity of r2c, c2r, Poisson and 128-bin P(k)."""
    shape = (256, 256, 256)
    print("case grf 256^3", flush=True)
    f32, f64, scale = grf_field(shape, 3.0, seed=2)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(f32).to(dev())
    F = plan.forward(x)
    back = plan.backward(F)
    phi, pk, km, ct = plan.poisson(x, nbins=128)
    torch.cuda.synchronize()
    refF = oracle.r2c(f64)
    opk, okm, oct_ = oracle.power_spectrum(refF, shape, 128)
    assert_close(F.cpu().numpy(), refF, shape, "r2c")
    assert_close(back.cpu().numpy(), float(np.prod(shape)) * f64, shape, "c2r")
    assert_close(phi.cpu().numpy(), oracle.poisson(f64), shape, "poisson")
    assert_close(pk.cpu().numpy(), opk, shape, "pk")
    assert np.array_equal(ct.cpu().numpy(), oct_)


@pytest.mark.parametrize("shape,nbins", [((64, 48, 40), 4096), ((160, 96, 64), 4096),
                                         ((96, 160, 192), 1000), ((8, 6, 1024), 4096)])
def test_many_bins_every_bin(lf2, shape, nbins):
    """Up to the 4096-bin maximum, on lattices whose lcm makes q large: the
    fused pass's bin of every mode must be the exact integer rule's, so each
    bin's power is compared on its own (a mode put into a neighbouring bin
    would move a whole |F|^2 / count there)."""
    print(f"case many bins {shape} nbins={nbins}", flush=True)
    dense, _ = real_field(shape, seed=15)
    f = dense[..., 0]
    f64 = f.astype(np.float64)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(f).to(dev())
    pk, km, ct = plan.power_spectrum(x, nbins)
    phi, pk2, km2, ct2 = plan.poisson(x, nbins=nbins)
    # and from the resident spectrum (k-space kernel, its own histogram)
    pk3, km3, ct3 = plan.power_spectrum(plan.forward(x), nbins, field_is_kspace=True)
    torch.cuda.synchronize()
    opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(f64), shape, nbins)
    assert np.array_equal(ct.cpu().numpy(), oct_) and np.array_equal(ct2.cpu().numpy(), oct_)
    assert np.array_equal(ct3.cpu().numpy(), oct_)
    scale = float(np.mean(opk[oct_ > 0]))
    for got in (pk.cpu().numpy(), pk2.cpu().numpy(), pk3.cpu().numpy()):
        err = np.abs(got - opk)
        worst = float(np.max(err / (scale + np.abs(opk))))
        print(f"  worst per-bin error {worst:.2e}", flush=True)
        assert worst <= 1e-5
    assert_close(phi.cpu().numpy(), oracle.poisson(f64), shape)


@pytest.mark.parametrize("shape", [(8, 4, 1), (4, 6, 2), (6, 10, 3), (10, 5, 12), (12, 20, 5),
                                   (2, 2, 2), (16, 3, 6), (40, 24, 20), (8, 6, 1024), (4, 4, 2048),
                                   (6, 10, 768), (4, 8, 640)])
def test_poisson_pk_short_last_axis(lf2, shape):
    """Last-axis lengths with no or one Stockham stage (1, 2, 3, 5, 6, 12, 20):
    the fused pass's register hand-off between its forward and backward
    transforms degenerates there (no LDS stages, or a single radix-3/5 stage);
    and the longest lines (640..2048), whose fused tiles fit one per CU."""
    print(f"case short last axis {shape}", flush=True)
    dense, _ = real_field(shape, seed=16)
    f = dense[..., 0]
    f64 = f.astype(np.float64)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(f).to(dev())
    phi, pk, km, ct = plan.poisson(x, nbins=4)
    pk2, km2, ct2 = plan.power_spectrum(x, 4)
    torch.cuda.synchronize()
    assert_close(phi.cpu().numpy(), oracle.poisson(f64), shape)
    opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(f64), shape, 4)
    for p_, c_ in ((pk, ct), (pk2, ct2)):
        assert np.array_equal(c_.cpu().numpy(), oct_)
        assert_close(p_.cpu().numpy(), opk, shape)


@pytest.mark.parametrize("shape,nbins", [((128, 96, 80), 48), ((512, 64, 512), 128),
                                         ((64, 48, 1024), 100)])
def test_poisson_repeatable(lf2, shape, nbins):
    """Repeated solves are bitwise equal: phi, the real-space sum of squares,
    and the binned sums (P(k), the k-space Parseval sum), whose LDS
    histograms are one per wave and summed in a fixed order."""
    print(f"case repeatable {shape} nbins={nbins}", flush=True)
    f = real_field(shape, seed=19)[0][..., 0]
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(f).to(dev())
    runs = [plan.poisson(x, nbins=nbins, parseval=True) for _ in range(3)]
    pks = [plan.power_spectrum(x, nbins)[0] for _ in range(2)]
    torch.cuda.synchronize()
    phi0, pk0, km0, ct0, pv0 = [t.cpu().numpy() for t in runs[0]]
    for r in runs[1:]:
        phi, pk, km, ct, pv = [t.cpu().numpy() for t in r]
        assert np.array_equal(phi, phi0)
        assert np.array_equal(ct, ct0) and np.array_equal(km, km0)
        assert pv[0] == pv0[0]
        assert pv[1] == pv0[1]
        assert np.array_equal(pk, pk0)
    assert torch.equal(pks[0], pks[1])


def test_parseval_many_x_blocks(lf2):
    """Parseval partials from 5120 x-pass blocks (512 x 256 x 320, 16 rows a
    block): the fixed-order reduction runs its four-loads-in-flight loop and
    its tail, and must give the FP64 sum of squares and the k-space sum."""
    shape = (512, 256, 320)
    print("case parseval, 5120 x blocks", flush=True)
    f = real_field(shape, seed=20)[0][..., 0]
    f64 = f.astype(np.float64)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    phi, pk, km, ct, pv = plan.poisson(torch.from_numpy(f).to(dev()), nbins=16, parseval=True)
    torch.cuda.synchronize()
    pv = pv.cpu().numpy()
    s2 = float(np.sum(f64 * f64))
    assert abs(pv[0] - s2) <= 1e-12 * s2
    assert abs(pv[1] - pv[0]) <= tol(shape) * pv[0]
    opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(f64), shape, 16)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert_close(pk.cpu().numpy(), opk, shape)
    assert_close(phi.cpu().numpy(), oracle.poisson(f64), shape)


# the fused Poisson pass with its tile in registers (tuning axis 3, z lines of
# 32 to 2048 points, powers of two): phi and P(k) (of rho, of phi, with the Parseval
# sums) against the oracle and against the LDS-staged tile, both k^2 kinds,
# ragged column counts, and a bin count (400 on 1024-point lines) whose
# waves share one histogram per block
@pytest.mark.parametrize("shape,nbins,flags,dx", [
    ((16, 8, 512), 24, 0, 1.0), ((24, 10, 512), 32, 1, 0.5), ((10, 6, 512), 7, 2, 1.0),
    ((64, 32, 512), 128, 0, 0.37), ((48, 20, 512), 0, 1, 1.0),
    ((16, 12, 256), 40, 0, 1.0), ((40, 9, 256), 16, 3, 0.5), ((64, 64, 256), 128, 1, 1.0),
    ((12, 8, 1024), 64, 0, 1.0), ((20, 6, 1024), 400, 1, 0.5), ((32, 16, 1024), 0, 2, 1.0),
    ((8, 4, 2048), 32, 0, 1.0), ((6, 5, 2048), 64, 3, 0.5),
    ((32, 32, 32), 16, 0, 1.0), ((10, 6, 32), 8, 2, 0.5), ((12, 10, 64), 16, 1, 1.0),
    ((20, 6, 128), 24, 2, 1.0), ((64, 48, 128), 64, 0, 0.37)])
def test_fused_register_tile(lf2, shape, nbins, flags, dx):
    print(f"case fused register tile {shape} nbins={nbins} flags={flags} dx={dx}", flush=True)
    if nbins == 0 and flags & 2:
        flags &= ~2  # P(k) of phi needs bins
    f = real_field(shape, seed=23)[0][..., 0]
    f64 = f.astype(np.float64)
    x = torch.from_numpy(f).to(dev())
    fl = (lf2.LF2_POISSON_DISCRETE_K2 if flags & 1 else 0) | (lf2.LF2_PK_OF_PHI if flags & 2 else 0)
    pr = lf2.Plan(shape, lf2.LF2_R2C)
    if shape[2] >= 64:
        assert pr.tuning(3)[0] == 1  # the default on power-of-two z lines of 64 to 2048
    pr.set_tuning(3, 1)
    pl = lf2.Plan(shape, lf2.LF2_R2C)
    pl.set_tuning(3, 0)
    assert pl.tuning(3)[0] == 0
    pv_on = nbins > 0 and not flags & 2  # Parseval sums are those of rho
    res_r = pr.poisson(x, dx=dx, flags=fl, nbins=nbins, parseval=pv_on)
    res_l = pl.poisson(x, dx=dx, flags=fl, nbins=nbins, parseval=pv_on)
    torch.cuda.synchronize()
    phi_r = (res_r[0] if nbins else res_r).cpu().numpy()
    phi_l = (res_l[0] if nbins else res_l).cpu().numpy()
    ref_phi = oracle.poisson(f64, dx=dx, k2mode=flags & 1)
    assert_close(phi_r, ref_phi, shape, "phi")
    assert rel_l2(phi_r, phi_l) <= 1e-6
    if nbins:
        src = ref_phi if flags & 2 else f64
        opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(src), shape, nbins, dx=dx)
        pk, km, ct = (t.cpu().numpy() for t in res_r[1:4])
        assert np.array_equal(ct, oct_)
        assert_close(pk, opk, shape, "pk")
        assert rel_l2(km, okm) <= 1e-12
        if pv_on:
            pv = res_r[4].cpu().numpy()
            s2 = float(np.sum(f64 * f64))
            assert abs(pv[0] - s2) <= 1e-12 * s2
            assert abs(pv[1] - pv[0]) <= tol(shape) * pv[0]


def test_fused_register_tile_settings(lf2):
    """Tuning axis 3 is the fused pass's tile: the register tile only for z
    lines of 32 to 2048 points (powers of two; the default from 64), variants
    0 and 1 only."""
    p = lf2.Plan((16, 8, 96), lf2.LF2_R2C)
    assert p.tuning(3)[0] == 0
    with pytest.raises(lf2.LF2Error) as ei:
        p.set_tuning(3, 1)
    assert ei.value.status == lf2.LF2_ERR_UNSUPPORTED
    for z in (64, 128, 256, 1024, 2048):
        assert lf2.Plan((16, 8, z), lf2.LF2_R2C).tuning(3)[0] == 1
    r = lf2.Plan((16, 8, 32), lf2.LF2_R2C)  # supported, not the default
    assert r.tuning(3)[0] == 0
    r.set_tuning(3, 1)
    assert r.tuning(3)[0] == 1
    q = lf2.Plan((16, 8, 512), lf2.LF2_R2C)
    assert q.tuning(3)[0] == 1
    with pytest.raises(lf2.LF2Error) as ei:
        q.set_tuning(3, 2)
    assert ei.value.status == lf2.LF2_ERR_INVALID_ARG
    q.set_tuning(3, 0)
    assert q.tuning(3)[0] == 0
