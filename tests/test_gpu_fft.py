"""GPU parity of the transforms against the FP64 oracle, through the C ABI.

Gate: relative L2 error <= 1e-5 * log2(N) (N = lattice points); the max
error relative to the largest oracle value is reported beside it.  Inputs
are the same seeded float32 values on both sides (the oracle promotes them
to float64).
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_close, complex_field, real_field, rel_l2, rel_max, tol

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


R2C_SHAPES = [(32, 32, 32), (8, 8, 8), (16, 12, 10), (64, 48, 40), (2, 4, 6), (96, 20, 12),
              (160, 6, 10), (128, 96, 80), (6, 256, 5), (256, 3, 64), (384, 16, 8),
              (10, 24, 192), (512, 8, 4), (4, 512, 4), (4, 4, 512), (1024, 2, 2), (2, 1, 1)]


def report(name, shape, err, errmax):
    print(f"[{name} {shape}] rel-L2 {err:.3e} max {errmax:.3e} tol {tol(shape):.2e}", flush=True)


@pytest.mark.parametrize("shape", R2C_SHAPES)
def test_r2c_forward(lf2, shape):
    print(f"case r2c_forward {shape}", flush=True)
    dense, _ = real_field(shape, seed=1)
    f = dense[..., 0]
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    F = plan.forward(torch.from_numpy(f).to(dev()))
    torch.cuda.synchronize()
    ref = oracle.r2c(f.astype(np.float64))
    got = F.cpu().numpy().astype(np.complex128)
    e, em = rel_l2(got, ref), rel_max(got, ref)
    report("r2c", shape, e, em)
    assert e <= tol(shape)
    assert em <= tol(shape)


@pytest.mark.parametrize("shape", R2C_SHAPES)
def test_c2r_backward(lf2, shape):
    print(f"case c2r_backward {shape}", flush=True)
    n0 = shape[0]
    dense, _ = real_field(shape, seed=2)
    H = oracle.r2c(dense[..., 0].astype(np.float64)).astype(np.complex64)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    Hd = torch.from_numpy(H).to(dev())
    Hkeep = Hd.clone()
    out = plan.backward(Hd)
    torch.cuda.synchronize()
    ref = oracle.c2r(H.astype(np.complex128), n0)
    got = out.cpu().numpy().astype(np.float64)
    e, em = rel_l2(got, ref), rel_max(got, ref)
    report("c2r", shape, e, em)
    assert e <= tol(shape)
    assert em <= tol(shape)
    assert torch.equal(Hd, Hkeep), "c2r modified its input"


def test_c2r_non_hermitian_reprojection(lf2):
    """c2r of an arbitrary half spectrum: the Re-projection the oracle defines."""
    shape = (16, 12, 10)
    rng = np.random.default_rng(3)
    G = (rng.standard_normal((10, 12, 9)) + 1j * rng.standard_normal((10, 12, 9))).astype(np.complex64)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    out = plan.backward(torch.from_numpy(G).to(dev()))
    torch.cuda.synchronize()
    ref = oracle.c2r(G.astype(np.complex128), 16)
    assert_close(out.cpu().numpy(), ref, shape)


C2C_SHAPES = [(32, 32, 32), (8, 8, 8), (12, 10, 6), (64, 48, 40), (3, 5, 4), (160, 12, 6),
              (512, 4, 4), (4, 4, 512), (1, 1, 16), (16, 1, 1)]


@pytest.mark.parametrize("shape", C2C_SHAPES)
@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("direction", [-1, 1])
def test_c2c(lf2, shape, ncomp, direction):
    _c2c_case(lf2, shape, ncomp, direction)


# the paper's FFT benchmark component counts (section 4.1): 1, 2, 3 and 6
@pytest.mark.parametrize("shape", [(32, 24, 16), (64, 8, 12), (1024, 4, 2), (6, 10, 512)])
@pytest.mark.parametrize("ncomp", [2, 6])
@pytest.mark.parametrize("direction", [-1, 1])
def test_c2c_paper_components(lf2, shape, ncomp, direction):
    _c2c_case(lf2, shape, ncomp, direction)


def _c2c_case(lf2, shape, ncomp, direction):
    print(f"case c2c {shape} ncomp={ncomp} dir={direction}", flush=True)
    z = complex_field(shape, seed=4, ncomp=ncomp)
    plan = lf2.Plan(shape, lf2.LF2_C2C, ncomp=ncomp)
    zin = torch.from_numpy(z if ncomp > 1 else z[..., 0]).to(dev())
    out = plan.forward(zin) if direction < 0 else plan.backward(zin)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    if ncomp == 1:
        got = got[..., None]
    for c in range(ncomp):
        ref = oracle.c2c(z[..., c].astype(np.complex128), direction)
        e, em = rel_l2(got[..., c], ref), rel_max(got[..., c], ref)
        report(f"c2c comp{c} dir{direction}", shape, e, em)
        assert e <= tol(shape)
        assert em <= tol(shape)


@pytest.mark.parametrize("shape", [(16, 12, 10), (32, 32, 32)])
@pytest.mark.parametrize("halo", [1, 2])
def test_halo_matches_dense(lf2, shape, halo):
    """Halo sites (set to NaN) are never read; the interior result equals the dense one."""
    print(f"case halo {shape} h={halo}", flush=True)
    dense, pad = real_field(shape, seed=5, halo=halo)
    p0 = lf2.Plan(shape, lf2.LF2_R2C)
    ph = lf2.Plan(shape, lf2.LF2_R2C, halo=halo)
    F0 = p0.forward(torch.from_numpy(dense[..., 0]).to(dev()))
    Fh = ph.forward(torch.from_numpy(pad[..., 0]).to(dev()))
    torch.cuda.synchronize()
    # odd halos take the general kernel, even ones the paired fast kernel
    assert rel_l2(Fh.cpu().numpy(), F0.cpu().numpy()) <= 1e-6
    # backward writes the interior only
    out = torch.full(ph.x_shape, 7.0, dtype=torch.float32, device=dev())
    ph.backward(Fh, out=out)
    ref = p0.backward(F0)
    torch.cuda.synchronize()
    h = halo
    o = out.cpu().numpy()
    n0, n1, n2 = shape
    assert rel_l2(o[h:h + n2, h:h + n1, h:h + n0], ref.cpu().numpy()) <= 1e-6
    mask = np.ones(o.shape, bool)
    mask[h:h + n2, h:h + n1, h:h + n0] = False
    assert np.all(o[mask] == 7.0)


def test_aos_three_components_equal_scalar(lf2):
    shape = (32, 24, 20)
    z = complex_field(shape, seed=6, ncomp=3)
    p3 = lf2.Plan(shape, lf2.LF2_C2C, ncomp=3)
    p1 = lf2.Plan(shape, lf2.LF2_C2C, ncomp=1)
    F3 = p3.forward(torch.from_numpy(z).to(dev()))
    for c in range(3):
        F1 = p1.forward(torch.from_numpy(np.ascontiguousarray(z[..., c])).to(dev()))
        torch.cuda.synchronize()
        assert rel_l2(F3[..., c].cpu().numpy(), F1.cpu().numpy()) <= 1e-6


def test_deterministic(lf2):
    shape = (64, 48, 40)
    dense, _ = real_field(shape, seed=7)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(dense[..., 0]).to(dev())
    a = plan.forward(x)
    b = plan.forward(x)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_round_trip(lf2):
    shape = (64, 48, 40)
    dense, _ = real_field(shape, seed=8)
    plan = lf2.Plan(shape, lf2.LF2_R2C)
    x = torch.from_numpy(dense[..., 0]).to(dev())
    back = plan.backward(plan.forward(x)) / float(np.prod(shape))
    torch.cuda.synchronize()
    assert_close(back.cpu().numpy(), dense[..., 0], shape)


# lines of 256..2048 points along y or z take either tile variant
WIDE_CASES = [((16, 256, 384), 0, 1), ((32, 64, 512), 0, 1), ((8, 24, 1024), 0, 1),
              ((40, 320, 96), 0, 1), ((12, 96, 768), 0, 1), ((6, 640, 16), 0, 1),
              ((16, 512, 256), 1, 3), ((10, 16, 512), 1, 1), ((4, 2048, 8), 0, 1),
              ((8, 6, 2048), 1, 2), ((40, 1024, 6), 1, 1), ((10, 6, 1024), 1, 3)]


@pytest.mark.parametrize("shape,kind,ncomp", WIDE_CASES)
def test_wide_tiles_match_oracle_and_narrow(lf2, shape, kind, ncomp):
    print(f"case wide tiles {shape} kind={kind} ncomp={ncomp}", flush=True)
    pn = lf2.Plan(shape, kind, ncomp=ncomp)
    pw = lf2.Plan(shape, kind, ncomp=ncomp)
    for axis in (1, 2):
        if shape[axis] >= 256:  # wide tiles; nontemporal accesses on z
            v = 1 if axis == 1 else 3
            pw.set_tuning(axis, v, chunk=4 if axis == 1 else 64)
            assert pw.tuning(axis)[:2] == (v, 4 if axis == 1 else 64)
        else:
            pw.set_tuning(axis, 2)  # narrow tiles, nontemporal accesses
    if kind == lf2.LF2_R2C:
        f = real_field(shape, seed=11)[0][..., 0]
        x = torch.from_numpy(f).to(dev())
        ref = oracle.r2c(f.astype(np.float64))
    else:
        z = complex_field(shape, seed=12, ncomp=ncomp)
        x = torch.from_numpy(z if ncomp > 1 else z[..., 0]).to(dev())
        ref = oracle.c2c(z[..., 0].astype(np.complex128), -1)
    Fn = pn.forward(x)
    Fw = pw.forward(x)
    bn = pn.backward(Fn)
    bw = pw.backward(Fw)
    torch.cuda.synchronize()
    got = Fw.cpu().numpy()
    if ncomp > 1:
        got = got[..., 0]
    e, em = rel_l2(got, ref), rel_max(got, ref)
    report("wide fwd", shape, e, em)
    assert e <= tol(shape)
    assert em <= tol(shape)
    print(f"  wide == narrow bitwise: fwd {bool(torch.equal(Fn, Fw))} bwd {bool(torch.equal(bn, bw))}",
          flush=True)
    assert rel_l2(Fw.cpu().numpy(), Fn.cpu().numpy()) <= 1e-6
    assert rel_l2(bw.cpu().numpy(), bn.cpu().numpy()) <= 1e-6

# lines of 1024 or 2048 points along y or z in the register tile (32 or 16
# columns held as a 32 x 32 or 32 x 64 decomposition): column counts that
# leave the last tile ragged
REG_CASES = [((8, 1024, 40), 1, 1), ((10, 6, 1024), 1, 3), ((12, 1024, 6), 0, 1),
             ((6, 10, 1024), 0, 2), ((2, 1024, 1024), 1, 1), ((6, 2048, 5), 1, 1),
             ((4, 3, 2048), 1, 3), ((8, 2048, 3), 0, 1), ((10, 4, 2048), 0, 1)]


@pytest.mark.parametrize("shape,kind,ncomp", REG_CASES)
def test_register_tile_matches_oracle_and_narrow(lf2, shape, kind, ncomp):
    print(f"case register tile {shape} kind={kind} ncomp={ncomp}", flush=True)
    pn = lf2.Plan(shape, kind, ncomp=ncomp)
    pr = lf2.Plan(shape, kind, ncomp=ncomp)
    for axis in (1, 2):
        if shape[axis] in (1024, 2048):  # plain and nontemporal accesses
            v = 4 if axis == 1 else 6
            pr.set_tuning(axis, v, chunk=8)
            assert pr.tuning(axis)[:2] == (v, 8)
    if kind == lf2.LF2_R2C:
        fs = real_field(shape, seed=13, ncomp=ncomp)[0]
        f = fs[..., 0]
        x = torch.from_numpy(fs if ncomp > 1 else f).to(dev())
        ref = oracle.r2c(f.astype(np.float64))
    else:
        z = complex_field(shape, seed=14, ncomp=ncomp)
        x = torch.from_numpy(z if ncomp > 1 else z[..., 0]).to(dev())
        ref = oracle.c2c(z[..., 0].astype(np.complex128), -1)
    Fn = pn.forward(x)
    Fr = pr.forward(x)
    bn = pn.backward(Fn)
    br = pr.backward(Fr)
    torch.cuda.synchronize()
    got = Fr.cpu().numpy()
    if ncomp > 1:
        got = got[..., 0]
    e, em = rel_l2(got, ref), rel_max(got, ref)
    report("register fwd", shape, e, em)
    assert e <= tol(shape)
    assert em <= tol(shape)
    assert rel_l2(Fr.cpu().numpy(), Fn.cpu().numpy()) <= 1e-6
    assert rel_l2(br.cpu().numpy(), bn.cpu().numpy()) <= 1e-6
    if kind == lf2.LF2_R2C:
        back = br.cpu().numpy() / float(np.prod(shape))
        assert rel_l2(back, fs if ncomp > 1 else f) <= tol(shape)



def test_autotune_picks_a_setting(lf2):
    shape = (64, 256, 512)
    print(f"case autotune {shape}", flush=True)
    p = lf2.Plan(shape, lf2.LF2_R2C, autotune=True)
    for axis in (1, 2):
        v, c, ud, ut = p.tuning(axis)
        print(f"  axis {axis}: variant {v} chunk {c} default {ud:.1f} us tuned {ut:.1f} us", flush=True)
        assert v in (0, 1, 2, 3) and c in (4, 16, 64) and 0 < ut <= ud
    q = lf2.Plan((64, 48, 40), lf2.LF2_R2C, autotune=True)
    v, c, ud, ut = q.tuning(1)
    assert (v & 1) == 0 and 0 < ut <= ud  # no wide tiles for these lengths
    f = real_field(shape, seed=13)[0][..., 0]
    F = p.forward(torch.from_numpy(f).to(dev()))
    torch.cuda.synchronize()
    assert_close(F.cpu().numpy(), oracle.r2c(f.astype(np.float64)), shape)


@pytest.mark.parametrize("shape", [(32, 24, 16), (48, 10, 6), (512, 4, 4), (2048, 2, 2)])
@pytest.mark.parametrize("ncomp", [2, 3, 6])
def test_r2c_c2r_components(lf2, shape, ncomp):
    """AoS real fields with several components: r2c and c2r per component."""
    print(f"case r2c/c2r {shape} ncomp={ncomp}", flush=True)
    dense, _ = real_field(shape, seed=14, ncomp=ncomp)
    plan = lf2.Plan(shape, lf2.LF2_R2C, ncomp=ncomp)
    F = plan.forward(torch.from_numpy(dense).to(dev()))
    back = plan.backward(F)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy()
    bg = back.cpu().numpy()
    for c in range(ncomp):
        f64 = dense[..., c].astype(np.float64)
        ref = oracle.r2c(f64)
        e, em = rel_l2(Fg[..., c], ref), rel_max(Fg[..., c], ref)
        report(f"r2c comp{c}", shape, e, em)
        assert e <= tol(shape)
        assert em <= tol(shape)
        refb = oracle.c2r(Fg[..., c].astype(np.complex128), shape[0])
        assert_close(bg[..., c], refb, shape)
