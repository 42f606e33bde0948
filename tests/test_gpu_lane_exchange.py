"""GPU parity of the x pass whose two radix-8 stages exchange values across
the lanes of a row (ds_bpermute or DPP moves) instead of through LDS: c2c
rows of 64 points, one component, forward and backward, against the FP64
oracle and against the LDS exchange."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_close, complex_field, rel_l2

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


SHAPES = [(64, 48, 40), (64, 64, 64), (64, 1, 3), (64, 128, 16)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("direction", [-1, 1])
def test_lane_exchange_matches_oracle_and_lds(lf2, shape, variant, direction):
    print(f"case lane exchange {shape} variant={variant} dir={direction}", flush=True)
    z = complex_field(shape, seed=8)[..., 0]
    zin = torch.from_numpy(z).to(dev())
    lds = lf2.Plan(shape, lf2.LF2_C2C)
    lane = lf2.Plan(shape, lf2.LF2_C2C)
    lane.set_tuning(0, variant)
    assert lane.tuning(0)[0] == variant and lds.tuning(0)[0] == 0
    a = lds.forward(zin) if direction < 0 else lds.backward(zin)
    b = lane.forward(zin) if direction < 0 else lane.backward(zin)
    torch.cuda.synchronize()
    ref = oracle.c2c(z.astype(np.complex128), direction)
    assert_close(b.cpu().numpy(), ref, shape, "lane exchange")
    # the same twiddles multiply the same values: only the exchange differs
    d = rel_l2(b.cpu().numpy(), a.cpu().numpy())
    print(f"  vs LDS exchange rel-L2 {d:.3e}", flush=True)
    assert d <= 1e-6


def test_lane_exchange_in_place_round_trip(lf2):
    shape = (64, 40, 24)
    print(f"case lane exchange in place {shape}", flush=True)
    z = complex_field(shape, seed=9)[..., 0]
    plan = lf2.Plan(shape, lf2.LF2_C2C, in_place=True)
    plan.set_tuning(0, 2)
    buf = torch.from_numpy(z).to(dev())
    plan.forward_(buf)
    torch.cuda.synchronize()
    assert_close(buf.cpu().numpy(), oracle.c2c(z.astype(np.complex128), -1), shape, "in place")
    plan.backward_(buf)
    torch.cuda.synchronize()
    assert_close(buf.cpu().numpy() / np.prod(shape), z.astype(np.complex128), shape, "round trip")


def test_lane_exchange_refused_elsewhere(lf2):
    for shape, kind in [((128, 8, 8), lf2.LF2_C2C), ((64, 8, 8), lf2.LF2_R2C)]:
        plan = lf2.Plan(shape, kind)
        with pytest.raises(lf2.LF2Error):
            plan.set_tuning(0, 1)
        plan.set_tuning(0, 0)
    plan = lf2.Plan((64, 8, 8), lf2.LF2_C2C, ncomp=3)
    with pytest.raises(lf2.LF2Error):
        plan.set_tuning(0, 2)


def test_autotune_times_the_exchanges(lf2):
    plan = lf2.Plan((64, 256, 256), lf2.LF2_C2C, autotune=True)
    v, chunk, us0, us1 = plan.tuning(0)
    print(f"  x exchange chosen {v}: LDS {us0:.1f} us, chosen {us1:.1f} us", flush=True)
    assert v in (0, 1, 2) and chunk == 0
    assert us0 > 0 and 0 < us1 <= us0
