"""Parity at the benchmark's full size, in the launch configuration bench.py
times (512^3, autotuned plans, the same seeded inputs: real N(0,1) seed 3,
complex64 3-component N(0,1) seed 4).  Every result is compared with the FP64
oracle over the whole field, element by element, on rel-L2 and max error
(the oracle does a 512^3 transform in a few seconds on the host's cores);
spectrum modes sampled one by one from the single-mode definition, and
properties that hold at any size (round trips, Parseval, the discrete
Laplacian of the discrete-k^2 Poisson solution, exact shell counts) come on
top."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import assert_close, rel_l2

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
    # whole spectrum against the oracle's r2c
    Fo = oracle.r2c(f64)
    assert_close(Fg, Fo, n, "r2c whole field")
    # c2r of the GPU spectrum against the oracle's c2r of that same spectrum
    bo = oracle.c2r(Fg.astype(np.complex128), S)
    assert_close(back.cpu().numpy(), bo, n, "c2r whole field")
    # round trip over the whole field
    e = rel_l2(back.cpu().numpy() / N, f64)
    print(f"  c2r(r2c(f)) / N rel-L2 {e:.2e}", flush=True)
    assert e <= TOL
    # Poisson potential against the oracle's solve of the same field
    assert_close(phi.cpu().numpy(), oracle.poisson(f64), n, "poisson whole field")
    # Parseval: the fused pass's FP64 sums
    sumsq = float(np.sum(f64 * f64))
    pvg = pv.cpu().numpy()
    assert abs(pvg[0] - sumsq) <= 1e-12 * sumsq
    assert abs(pvg[1] - sumsq) <= TOL * sumsq
    # the fused P(k) against the oracle's P(k) of the field, and against the
    # oracle's binning of the GPU's own spectrum
    opk, okm, oct_ = oracle.power_spectrum(Fo, n, nb)
    assert np.array_equal(ct.cpu().numpy(), oct_)
    assert_close(pk.cpu().numpy(), opk, n, "fused P(k)")
    assert rel_l2(km.cpu().numpy(), okm) <= 1e-12
    gpk, _, _ = oracle.power_spectrum(Fg.astype(np.complex128), n, nb)
    assert_close(pk.cpu().numpy(), gpk, n, "fused P(k) vs binning of the GPU spectrum")
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


_C2C = {}


def _c2c_run(lf2):
    """The 3-component c2c forward and backward at the bench's configuration,
    computed once per module: (input, forward output, backward output)."""
    if not _C2C:
        n = (S, S, S)
        z3 = synth.white_field(4, n, ncomp=3, complex_values=True)
        z = torch.from_numpy(z3).to(dev()).view(torch.complex64).reshape(S, S, S, 3)
        del z3
        p = lf2.Plan(n, lf2.LF2_C2C, ncomp=3, autotune=True)
        Z = p.forward(z)
        back = p.backward(Z)
        torch.cuda.synchronize()
        _C2C["z"] = z.cpu().numpy()
        _C2C["Z"] = Z.cpu().numpy()
        _C2C["back"] = back.cpu().numpy()
        del z, Z, back
        p.close()
        torch.cuda.empty_cache()
    return _C2C["z"], _C2C["Z"], _C2C["back"]


def test_c2c_3comp_512_forward(lf2):
    print("case full size 512^3 complex 3-comp forward (seed 4)", flush=True)
    n = (S, S, S)
    zz, Zg, _ = _c2c_run(lf2)
    scale = math.sqrt(N)
    worst = 0.0
    for c in range(3):
        zc = zz[..., c].astype(np.complex128)
        for kx, ky, kz in MODES:
            want = oracle.dft3d_at(zc, (kx, ky, kz))
            worst = max(worst, abs(complex(Zg[kz, ky, kx, c]) - want) / scale)
        # every mode of the component against the oracle's c2c
        assert_close(Zg[..., c], oracle.c2c(zc, oracle.FORWARD), n, f"c2c fwd comp {c}")
        del zc
    print(f"  sampled c2c modes: worst |err|/sqrt(N) {worst:.2e}", flush=True)
    assert worst <= TOL


def test_c2c_3comp_512_backward(lf2):
    print("case full size 512^3 complex 3-comp backward of the GPU spectrum", flush=True)
    n = (S, S, S)
    zz, Zg, back = _c2c_run(lf2)
    for c in range(3):
        ref = oracle.c2c(Zg[..., c].astype(np.complex128), oracle.BACKWARD)
        assert_close(back[..., c], ref, n, f"c2c bwd comp {c}")
        del ref
    e = rel_l2(back / N, zz)
    print(f"  c2c round trip rel-L2 {e:.2e}", flush=True)
    assert e <= TOL
