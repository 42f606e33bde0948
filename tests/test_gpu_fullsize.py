"""Parity at the benchmark's full size, in the launch configuration bench.py
times (512^3, autotuned plans, the same seeded inputs: real N(0,1) seed 3,
complex64 3-component N(0,1) seed 4).  The whole-field oracle is too slow
here, so: spectrum modes sampled one by one from the definition (single-mode
FP64 DFT), and properties that hold at any size (round trips, Parseval, the
discrete Laplacian of the discrete-k^2 Poisson solution, the fused P(k)
against the oracle's binning of the GPU's own spectrum, exact shell counts)."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

S = 512
N = S ** 3
TOL = 1e-5 * math.log2(N)  # 2.7e-4
# sampled modes (k_x, k_y, k_z): zero, low, Nyquist planes and generic ones
MODES = [(0, 0, 0), (1, 2, 3), (S // 2, 0, 0), (0, S // 2, S // 2), (S // 2, S // 2, S // 2),
         (7, S - 1, S // 3), (S // 4, S // 2 + 1, 5), (S // 2 - 1, 17, S - 2), (100, 300, 411)]


@pytest.fixture(scope="module")
def lf2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_05610_amd as m
    m.load()
    return m


def dev():
    return torch.device("cuda:0")


def test_r2c_c2r_poisson_pk_512(lf2):
    print("case full size 512^3 real (seed 3)", flush=True)
    n = (S, S, S)
    f32 = synth.white_field(3, n)[..., 0]
    f64 = f32.astype(np.float64)
    x = torch.from_numpy(f32).to(dev())
    p = lf2.Plan(n, lf2.LF2_R2C, autotune=True)
    F = p.forward(x)
    back = p.backward(F)
    nb = 128
    phi, pk, km, ct, pv = p.poisson(x, nbins=nb, parseval=True)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy()
    # sampled spectrum modes against the definition (FP64, one mode at a time)
    scale = math.sqrt(N)  # |F| of N(0,1) white noise ~ sqrt(N)
    worst = 0.0
    for kx, ky, kz in MODES:
        want = oracle.dft3d_at(f64, (kx, ky, kz))
        worst = max(worst, abs(complex(Fg[kz, ky, kx]) - want) / scale)
    print(f"  sampled r2c modes: worst |err|/sqrt(N) {worst:.2e}", flush=True)
    assert worst <= TOL
    # round trip over the whole field
    e = rel_l2(back.cpu().numpy() / N, f64)
    print(f"  c2r(r2c(f)) / N rel-L2 {e:.2e}", flush=True)
    assert e <= TOL
    # Parseval: the fused pass's FP64 sums
    sumsq = float(np.sum(f64 * f64))
    pvg = pv.cpu().numpy()
    assert abs(pvg[0] - sumsq) <= 1e-12 * sumsq
    assert abs(pvg[1] - sumsq) <= TOL * sumsq
    # the fused P(k) against the oracle's binning of the GPU's spectrum
    opk, okm, oct_ = oracle.power_spectrum(Fg.astype(np.complex128), n, nb)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    e = rel_l2(pk.cpu().numpy(), opk)
    print(f"  fused P(k) vs oracle binning rel-L2 {e:.2e}", flush=True)
    assert e <= TOL
    assert int(oct_.sum()) == N - 1


def test_discrete_poisson_laplacian_512(lf2):
    print("case full size 512^3 discrete Poisson", flush=True)
    n = (S, S, S)
    f32 = synth.white_field(3, n)[..., 0]
    x = torch.from_numpy(f32).to(dev())
    p = lf2.Plan(n, lf2.LF2_R2C, autotune=True)
    phi = p.poisson(x, flags=lf2.LF2_POISSON_DISCRETE_K2).double()
    # the 7-point Laplacian of the discrete-k^2 solution returns rho - <rho>
    lap = -6.0 * phi
    for d in range(3):
        lap += torch.roll(phi, 1, dims=d) + torch.roll(phi, -1, dims=d)
    rho = x.double()
    e = float(torch.linalg.vector_norm(lap - (rho - rho.mean())) / torch.linalg.vector_norm(rho))
    print(f"  Laplacian(phi) vs rho - <rho> rel-L2 {e:.2e}", flush=True)
    assert e <= TOL
    assert abs(float(phi.mean())) <= 1e-6 * float(phi.abs().max())


def test_c2c_3comp_512(lf2):
    print("case full size 512^3 complex 3-comp (seed 4)", flush=True)
    n = (S, S, S)
    z3 = synth.white_field(4, n, ncomp=3, complex_values=True)
    z = torch.from_numpy(z3).to(dev()).view(torch.complex64).reshape(S, S, S, 3)
    p = lf2.Plan(n, lf2.LF2_C2C, ncomp=3, autotune=True)
    Z = p.forward(z)
    back = p.backward(Z)
    torch.cuda.synchronize()
    Zg = Z.cpu().numpy()
    zz = z.cpu().numpy()
    scale = math.sqrt(N)
    worst = 0.0
    for c in range(3):
        zc = zz[..., c].astype(np.complex128)
        for kx, ky, kz in MODES:
            want = oracle.dft3d_at(zc, (kx, ky, kz))
            worst = max(worst, abs(complex(Zg[kz, ky, kx, c]) - want) / scale)
    print(f"  sampled c2c modes: worst |err|/sqrt(N) {worst:.2e}", flush=True)
    assert worst <= TOL
    e = float(torch.linalg.vector_norm(back / N - z) / torch.linalg.vector_norm(z))
    print(f"  c2c round trip rel-L2 {e:.2e}", flush=True)
    assert e <= TOL
