"""GPU parity of the field operations (paper section 4.2) against the FP64
oracle: periodic halo update (bitwise: it is a copy) and the first-order
derivative of every component."""
import numpy as np
import pytest

import synth
from oracle import fieldops
from gpu_helpers import rel_max

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


def padded_field(shape, h, nc, seed, complex_values=False):
    n0, n1, n2 = shape
    p = (n2 + 2 * h, n1 + 2 * h, n0 + 2 * h)
    words = nc * (2 if complex_values else 1)
    a = synth.normal(seed, int(np.prod(p)) * words, dtype=np.float32).reshape(p + (words,))
    return a


@pytest.mark.parametrize("shape,h,nc,cplx", [((16, 12, 10), 1, 1, False), ((8, 6, 4), 2, 3, False),
                                             ((10, 8, 6), 1, 2, True), ((5, 7, 3), 3, 1, False),
                                             ((64, 2, 1), 1, 6, False), ((96, 80, 64), 1, 3, False),
                                             ((300, 4, 5), 2, 1, True)])
def test_update_halo_bitwise(lf2, shape, h, nc, cplx):
    print(f"case halo {shape} h={h} nc={nc} complex={cplx}", flush=True)
    a = padded_field(shape, h, nc, seed=20, complex_values=cplx)
    ref = fieldops.halo_fill(a, h)
    t = torch.from_numpy(a).to(dev())
    if cplx:
        t = t.view(torch.complex64)
    lf2.update_halo(t, shape, h)
    torch.cuda.synchronize()
    got = t.view(torch.float32).cpu().numpy() if cplx else t.cpu().numpy()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("shape,h,nc,dx", [((16, 12, 10), 1, 1, 1.0), ((32, 24, 16), 1, 3, 0.5),
                                           ((8, 6, 40), 2, 2, 0.25), ((64, 48, 40), 1, 3, 1.0),
                                           ((5, 7, 3), 1, 6, 1.0), ((100, 9, 5), 1, 2, 2.0),
                                           # rows split over several blocks, the last one ragged
                                           ((300, 6, 5), 1, 3, 1.0), ((520, 5, 3), 2, 2, 1.0),
                                           ((20, 3, 3), 1, 64, 1.0)])
def test_gradient_matches_oracle(lf2, shape, h, nc, dx):
    print(f"case gradient {shape} h={h} nc={nc}", flush=True)
    a = padded_field(shape, h, nc, seed=21)
    t = torch.from_numpy(a).to(dev())
    lf2.update_halo(t, shape, h)
    out = torch.full(t.shape[:3] + (3 * nc,), float("nan"), dtype=torch.float32, device=dev())
    lf2.gradient(t, shape, h, dx=dx, out=out)
    torch.cuda.synchronize()
    ref = fieldops.gradient(fieldops.interior(a, h).astype(np.float64), dx=dx)
    o = out.cpu().numpy()
    got = fieldops.interior(o, h)
    e = rel_max(got, ref)
    print(f"  rel max {e:.2e}", flush=True)
    assert e <= 1e-6
    mask = np.ones(o.shape[:3], bool)
    mask[h:-h, h:-h, h:-h] = False
    assert np.all(np.isnan(o[mask])), "the output halo must not be written"
