"""GPU parity of the paper's k-space orders (section 3.6: r2c (k_x, k_z, k_y),
c2c (k_z, k_x, k_y))
and of in-place transforms (section 3.6), against the oracle and against
the natural out-of-place results."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_close, real_field, complex_field, rel_l2, rel_max, tol

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


SHAPES = [(32, 24, 16), (64, 48, 40), (20, 12, 10), (16, 512, 8)]


@pytest.mark.parametrize("shape", SHAPES)
def test_r2c_paper_layout_forward_backward(lf2, shape):
    print(f"case paper layout r2c {shape}", flush=True)
    f = real_field(shape, seed=31)[0][..., 0]
    p = lf2.Plan(shape, lf2.LF2_R2C, paper_layout=True)
    n0, n1, n2 = shape
    assert p.k_shape == (n1, n2, n0 // 2 + 1)
    F = p.forward(torch.from_numpy(f).to(dev()))
    back = p.backward(F)
    torch.cuda.synchronize()
    ref = oracle.to_paper_layout(oracle.r2c(f.astype(np.float64)), "r2c")
    assert_close(F.cpu().numpy(), ref, shape, "fwd")
    assert_close(back.cpu().numpy() / np.prod(shape), f, shape)


def test_r2c_paper_layout_components(lf2):
    shape = (16, 8, 12)
    dense = real_field(shape, seed=32, ncomp=3)[0]
    p = lf2.Plan(shape, lf2.LF2_R2C, ncomp=3, paper_layout=True)
    F = p.forward(torch.from_numpy(dense).to(dev()))
    torch.cuda.synchronize()
    Fg = F.cpu().numpy()
    for c in range(3):
        ref = oracle.to_paper_layout(oracle.r2c(dense[..., c].astype(np.float64)), "r2c")
        assert_close(Fg[..., c], ref, shape)


@pytest.mark.parametrize("shape", [(32, 24, 16), (64, 64, 64)])
def test_poisson_and_pk_paper_layout(lf2, shape):
    print(f"case poisson paper layout {shape}", flush=True)
    nb = 12
    f = real_field(shape, seed=33)[0][..., 0]
    rho = torch.from_numpy(f).to(dev())
    pp = lf2.Plan(shape, lf2.LF2_R2C, paper_layout=True)
    pn = lf2.Plan(shape, lf2.LF2_R2C)
    phi, pk, km, ct = pp.poisson(rho, nbins=nb)
    phin, pkn, _, ctn = pn.poisson(rho, nbins=nb)
    # P(k) of a spectrum given in the paper's order
    F = pp.forward(rho)
    pk2, _, ct2 = pp.power_spectrum(F, nb, field_is_kspace=True)
    torch.cuda.synchronize()
    f64 = f.astype(np.float64)
    assert_close(phi.cpu().numpy(), oracle.poisson(f64), shape)
    opk, _, oct_ = oracle.power_spectrum(oracle.r2c(f64), shape, nb)
    assert_close(pk.cpu().numpy(), opk, shape)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert_close(pk2.cpu().numpy(), opk, shape)
    assert np.array_equal(ct2.cpu().numpy(), oct_)
    assert rel_l2(phi.cpu().numpy(), phin.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("shape", [(32, 24, 16), (64, 48, 40), (512, 4, 4)])
@pytest.mark.parametrize("paper", [False, True])
def test_r2c_in_place(lf2, shape, paper):
    print(f"case in-place r2c {shape} paper={paper}", flush=True)
    n0, n1, n2 = shape
    f = real_field(shape, seed=34)[0][..., 0]
    p = lf2.Plan(shape, lf2.LF2_R2C, in_place=True, paper_layout=paper)
    x = torch.zeros(p.x_shape, dtype=torch.float32, device=dev())
    assert p.x_shape == (n2, n1, 2 * (n0 // 2 + 1))
    x[..., :n0] = torch.from_numpy(f).to(dev())
    k = p.forward_(x)
    torch.cuda.synchronize()
    ref = oracle.r2c(f.astype(np.float64))
    if paper:
        ref = oracle.to_paper_layout(ref, "r2c")
    assert_close(k.cpu().numpy(), ref, shape)
    back = p.backward_(k)
    torch.cuda.synchronize()
    assert_close(back[..., :n0].cpu().numpy() / np.prod(shape), f, shape)


@pytest.mark.parametrize("shape,ncomp", [((32, 24, 16), 1), ((16, 12, 10), 3), ((4, 4, 512), 1)])
def test_c2c_in_place(lf2, shape, ncomp):
    print(f"case in-place c2c {shape} ncomp={ncomp}", flush=True)
    z = complex_field(shape, seed=35, ncomp=ncomp)
    zz = z if ncomp > 1 else z[..., 0]
    p = lf2.Plan(shape, lf2.LF2_C2C, ncomp=ncomp, in_place=True)
    q = lf2.Plan(shape, lf2.LF2_C2C, ncomp=ncomp)
    x = torch.from_numpy(zz).to(dev())
    ref = q.forward(x)
    y = x.clone()
    k = p.forward_(y)
    torch.cuda.synchronize()
    assert rel_l2(k.cpu().numpy(), ref.cpu().numpy()) <= 1e-6
    got = k.cpu().numpy()
    if ncomp == 1:
        got = got[..., None]
    for c in range(ncomp):
        assert_close(got[..., c], oracle.c2c(z[..., c].astype(np.complex128), -1), shape)
    b = p.backward_(k)
    torch.cuda.synchronize()
    assert_close(b.cpu().numpy() / np.prod(shape), zz, shape)


@pytest.mark.parametrize("shape", [(32, 24, 16), (32, 24, 64)])  # LDS-staged, register fused pass
def test_poisson_in_place(lf2, shape):
    n0, n1, n2 = shape
    f = real_field(shape, seed=36)[0][..., 0]
    p = lf2.Plan(shape, lf2.LF2_R2C, in_place=True)
    x = torch.zeros(p.x_shape, dtype=torch.float32, device=dev())
    x[..., :n0] = torch.from_numpy(f).to(dev())
    p.poisson(x, phi=x)
    torch.cuda.synchronize()
    assert_close(x[..., :n0].cpu().numpy(), oracle.poisson(f.astype(np.float64)), shape)


@pytest.mark.parametrize("shape,ncomp", [((32, 24, 16), 1), ((16, 12, 10), 3), ((8, 6, 512), 1),
                                         ((24, 10, 20), 2), ((12, 8, 6), 6)])
def test_c2c_paper_layout(lf2, shape, ncomp):
    print(f"case paper layout c2c {shape} ncomp={ncomp}", flush=True)
    n0, n1, n2 = shape
    z = complex_field(shape, seed=37, ncomp=ncomp)
    zz = z if ncomp > 1 else z[..., 0]
    p = lf2.Plan(shape, lf2.LF2_C2C, ncomp=ncomp, paper_layout=True)
    assert p.k_shape[:3] == (n1, n0, n2)
    F = p.forward(torch.from_numpy(zz).to(dev()))
    back = p.backward(F)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy()
    if ncomp == 1:
        Fg = Fg[..., None]
    for c in range(ncomp):
        ref = oracle.to_paper_layout(oracle.c2c(z[..., c].astype(np.complex128), -1), "c2c")
        assert_close(Fg[..., c], ref, shape, f"comp {c}")
    assert_close(back.cpu().numpy() / np.prod(shape), zz, shape)
    # in place, and the power spectrum of a spectrum in this order
    if ncomp == 1:
        q = lf2.Plan(shape, lf2.LF2_C2C, in_place=True, paper_layout=True)
        y = torch.from_numpy(zz).to(dev())
        k = q.forward_(y)
        pk, _, ct = q.power_spectrum(k, 8, field_is_kspace=True)
        torch.cuda.synchronize()
        assert rel_l2(k.cpu().numpy(), F.cpu().numpy()) <= 1e-6
        opk, _, oct_ = oracle.power_spectrum(oracle.c2c(z[..., 0].astype(np.complex128), -1), shape,
                                             8, half=False)
        assert_close(pk.cpu().numpy(), opk, shape)
        assert np.array_equal(ct.cpu().numpy(), oct_)
