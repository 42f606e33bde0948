"""Parity at the paper's benchmark sizes (section 4.1: 1024^3 with one and
three components, 2048^3 with one) through properties that hold at any size,
checked over the whole field on the device:

* a separable input f = a(x) b(y) c(z) has the separable spectrum
  F = A(k_x) B(k_y) C(k_z), the factors being 1-D oracle transforms of a, b
  and c (FP64), and the unnormalised c2r of that spectrum is N f;
* one Fourier mode rho = cos(2 pi m.n / N) has phi = -rho / k^2 and all of
  its power in one bin, P_b = N / (2 count_b) (dx = 1)."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CHUNK = 64  # z planes per comparison chunk


@pytest.fixture(scope="module")
def lf2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1508_05610_amd as m
    m.load()
    return m


def dev():
    return torch.device("cuda:0")


class Err:
    """rel-L2 and max error (relative to the largest reference value),
    accumulated chunk by chunk in FP64."""

    def __init__(self):
        self.d2 = self.r2 = self.dmax = self.rmax = 0.0

    def add(self, got, ref):
        d = (got.to(ref.dtype) - ref).abs()
        r = ref.abs()
        self.d2 += float((d * d).sum())
        self.r2 += float((r * r).sum())
        self.dmax = max(self.dmax, float(d.max()))
        self.rmax = max(self.rmax, float(r.max()))

    def check(self, name, shape):
        e, em = math.sqrt(self.d2 / self.r2), self.dmax / self.rmax
        print(f"[{name} {shape}] rel-L2 {e:.3e} max {em:.3e} tol {tol(shape):.2e}", flush=True)
        assert e <= tol(shape) and em <= tol(shape)


def factors(shape, seed):
    """Seeded 1-D factors (FP64) and their oracle transforms (FP64)."""
    vs = [synth.normal(seed, n, stream=i) for i, n in enumerate(shape)]
    return vs, [oracle.fft1d(v) for v in vs]


def outer(c, b, a, z0, z1):
    return c[z0:z1, None, None] * b[None, :, None] * a[None, None, :]


@pytest.mark.parametrize("shape,kind,ncomp", [((1024, 1024, 1024), "r2c", 1),
                                              ((1024, 1024, 1024), "c2c", 1),
                                              ((1024, 1024, 1024), "c2c", 3),
                                              ((2048, 2048, 2048), "r2c", 1)])
def test_separable_full_size(lf2, shape, kind, ncomp):
    print(f"case separable {kind} {shape} ncomp={ncomp}", flush=True)
    n0, n1, n2 = shape
    (a, b, c), (A, B, C) = factors(shape, seed=31)
    ta, tb, tc = (torch.from_numpy(v).to(dev()) for v in (a, b, c))
    tA, tB, tC = (torch.from_numpy(v).to(dev()) for v in (A, B, C))
    scale = torch.arange(1, ncomp + 1, dtype=torch.float64, device=dev())  # component c: (c + 1) f
    if kind == "r2c":
        plan = lf2.Plan(shape, lf2.LF2_R2C)
        x = torch.empty(plan.x_shape, dtype=torch.float32, device=dev())
        for z0 in range(0, n2, CHUNK):
            x[z0:z0 + CHUNK] = outer(tc, tb, ta, z0, z0 + CHUNK).float()
        F = plan.forward(x)
        torch.cuda.synchronize()
        nh = n0 // 2 + 1
        ef = Err()
        for z0 in range(0, n2, CHUNK):
            ef.add(F[z0:z0 + CHUNK], outer(tC, tB, tA[:nh], z0, z0 + CHUNK))
        ef.check("r2c separable", shape)
        # the c2r of the exact separable spectrum is N f
        for z0 in range(0, n2, CHUNK):
            F[z0:z0 + CHUNK] = outer(tC, tB, tA[:nh], z0, z0 + CHUNK).to(torch.complex64)
        y = plan.backward(F)
        torch.cuda.synchronize()
        eb = Err()
        for z0 in range(0, n2, CHUNK):
            eb.add(y[z0:z0 + CHUNK], float(n0 * n1 * n2) * outer(tc, tb, ta, z0, z0 + CHUNK))
        eb.check("c2r separable", shape)
    else:
        plan = lf2.Plan(shape, lf2.LF2_C2C, ncomp=ncomp)
        x = torch.empty(plan.x_shape, dtype=torch.complex64, device=dev())
        for z0 in range(0, n2, CHUNK):
            f = outer(tc, tb, ta, z0, z0 + CHUNK)
            x[z0:z0 + CHUNK] = (f[..., None] * scale if ncomp > 1 else f).to(torch.complex64)
        F = plan.forward(x)
        torch.cuda.synchronize()
        ef = Err()
        for z0 in range(0, n2, CHUNK):
            r = outer(tC, tB, tA, z0, z0 + CHUNK)
            ef.add(F[z0:z0 + CHUNK], r[..., None] * scale if ncomp > 1 else r)
        ef.check(f"c2c separable ncomp={ncomp}", shape)


@pytest.mark.parametrize("shape", [(1024, 1024, 1024), (2048, 2048, 2048)])
def test_plane_wave_poisson_full_size(lf2, shape):
    print(f"case plane-wave Poisson + P(k) {shape}", flush=True)
    n0, n1, n2 = shape
    m = (3, 5, 7)
    nbins = 128
    k2 = sum((2 * math.pi * mi / ni) ** 2 for mi, ni in zip(m, shape))
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    assert plan.tuning(3)[0] == 1  # the register fused pass at these z lengths

    def wave(z0, z1):
        z = torch.arange(z0, z1, dtype=torch.float64, device=dev())
        y = torch.arange(n1, dtype=torch.float64, device=dev())
        x = torch.arange(n0, dtype=torch.float64, device=dev())
        th = 2 * math.pi * (m[2] * z[:, None, None] / n2 + m[1] * y[None, :, None] / n1 +
                            m[0] * x[None, None, :] / n0)
        return torch.cos(th)

    rho = torch.empty(plan.x_shape, dtype=torch.float32, device=dev())
    for z0 in range(0, n2, CHUNK):
        rho[z0:z0 + CHUNK] = wave(z0, min(z0 + CHUNK, n2)).float()
    phi, pk, km, ct = plan.poisson(rho, nbins=nbins)
    torch.cuda.synchronize()
    e = Err()
    for z0 in range(0, n2, CHUNK):
        e.add(phi[z0:z0 + CHUNK], -wave(z0, min(z0 + CHUNK, n2)) / k2)
    e.check("plane-wave phi", shape)
    # all the power in the bin of |m|^2 (a cubic lattice: q = |m|^2)
    b = oracle.pk_bin(sum(mi * mi for mi in m), oracle.pk_qmax(shape), nbins)
    pk, ct = pk.cpu().numpy(), ct.cpu().numpy()
    want = n0 * n1 * n2 / (2.0 * ct[b])
    print(f"  bin {b}: P {pk[b]:.9e} want {want:.9e} count {ct[b]:.0f}", flush=True)
    assert abs(pk[b] - want) <= tol(shape) * want
    others = np.delete(pk, b)
    assert np.abs(others).max() <= 1e-9 * want  # FP32 rounding noise only
