"""The HIP path against the hand-derived fixtures of tests/golden/ (the same
ones the oracle is pinned to): r2c forward, c2c forward and c2r backward of
two small lattices, and the one-mode Poisson solution with continuous and
discrete k^2 at two lattice spacings."""
import numpy as np
import pytest

from golden_fixtures import line_4x2x2, poisson_cos_8x4x4, ramp_2x2x2
from gpu_helpers import rel_l2, rel_max, tol

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


def check(name, got, ref, shape):
    e, em = rel_l2(got, ref), rel_max(got, ref)
    print(f"[{name} {shape}] rel-L2 {e:.3e} max {em:.3e} tol {tol(shape):.2e}", flush=True)
    assert e <= tol(shape) and em <= tol(shape)


@pytest.mark.parametrize("case", [ramp_2x2x2, line_4x2x2])
def test_dft_fixtures(lf2, case):
    f, F = case()
    n2, n1, n0 = f.shape
    shape = (n0, n1, n2)
    print(f"case golden dft {case.__name__} {shape}", flush=True)
    half = F[..., : n0 // 2 + 1]
    pr = lf2.Plan(shape, lf2.LF2_R2C)
    H = pr.forward(torch.from_numpy(f.astype(np.float32)).to(dev()))
    back = pr.backward(torch.from_numpy(half.astype(np.complex64)).to(dev()))
    pc = lf2.Plan(shape, lf2.LF2_C2C)
    C = pc.forward(torch.from_numpy(f.astype(np.complex64)).to(dev()))
    torch.cuda.synchronize()
    check("r2c", H.cpu().numpy(), half, shape)
    check("c2c", C.cpu().numpy(), F, shape)
    check("c2r", back.cpu().numpy(), f.size * f, shape)  # unnormalised inverse


def test_poisson_fixture(lf2):
    rho, cases = poisson_cos_8x4x4()
    shape = (8, 4, 4)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(rho.astype(np.float32)).to(dev())
    for dx, k2mode, a in cases:
        print(f"case golden poisson dx={dx} k2mode={k2mode}", flush=True)
        flags = lf2.LF2_POISSON_DISCRETE_K2 if k2mode else 0
        phi = plan.poisson(x, dx=dx, flags=flags)
        torch.cuda.synchronize()
        check(f"poisson dx={dx} k2mode={k2mode}", phi.cpu().numpy(), a * rho, shape)
