"""lf2_poisson_solve_noalloc (static per-device workspace, no allocation)
against lf2_poisson_solve, through the C ABI: two calls in a row, the second
on a smaller lattice, each compared with the allocating entry point on the
same inputs (and with the oracle)."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_close, real_field

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05610_amd import _lib
    _lib.load()
    return _lib


def _plan(lib, shape):
    return lib.lf2_fft_plan(shape, 0, 1, lib.LF2_R2C, 0)


def _solve(lib, fn, plan, rho, nbins, dx, flags, stream):
    dev = rho.device
    phi = torch.full_like(rho, float("nan"))
    pk, km, ct = (torch.full((nbins,), float("nan"), dtype=torch.float64, device=dev)
                  for _ in range(3))
    pv = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
    st = getattr(lib.load(), fn)(plan, rho.data_ptr(), phi.data_ptr(), dx, flags, nbins,
                                 pk.data_ptr(), km.data_ptr(), ct.data_ptr(), pv.data_ptr(), stream)
    return st, phi, pk, km, ct, pv


def test_noalloc_matches_allocating_call_twice(lib):
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    cases = [((128, 128, 128), 64, 1.0, 0, 21), ((64, 48, 40), 16, 0.5, lib.LF2_POISSON_DISCRETE_K2, 22)]
    for shape, nbins, dx, flags, seed in cases:
        print(f"case noalloc poisson {shape} nbins={nbins} dx={dx} flags={flags}", flush=True)
        f = real_field(shape, seed=seed)[0][..., 0]
        rho = torch.from_numpy(f).to(dev)
        plan = _plan(lib, shape)
        try:
            # the allocating call builds the plan's tables for (dx, flags, nbins)
            st, *ref = _solve(lib, "lf2_poisson_solve", plan, rho, nbins, dx, flags, stream)
            assert st == lib.LF2_OK, lib.last_error()
            st, *got = _solve(lib, "lf2_poisson_solve_noalloc", plan, rho, nbins, dx, flags, stream)
            assert st == lib.LF2_OK, lib.last_error()
            torch.cuda.synchronize()
            names = ("phi", "pk", "kmean", "count", "parseval")
            for name, a, b in zip(names, got, ref):
                a, b = a.cpu().numpy(), b.cpu().numpy()
                assert np.all(np.isfinite(a)), name
                assert_close(a, b, shape, f"noalloc vs allocating {name}")
            print(f"  phi bitwise equal: {bool(torch.equal(got[0], ref[0]))}", flush=True)
            assert np.array_equal(got[3].cpu().numpy(), ref[3].cpu().numpy())
            f64 = f.astype(np.float64)
            phio = oracle.poisson(f64, dx=dx, k2mode=1 if flags else 0)
            assert_close(got[0].cpu().numpy(), phio, shape, "noalloc vs oracle phi")
            opk, _, oct_ = oracle.power_spectrum(oracle.r2c(f64), shape, nbins, dx=dx)
            assert_close(got[1].cpu().numpy(), opk, shape, "noalloc vs oracle pk")
            assert np.array_equal(got[3].cpu().numpy(), oct_)
        finally:
            lib.load().lf2_plan_destroy(plan)


def test_noalloc_refusals(lib):
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    # tables not built yet on a fresh plan: nothing is enqueued
    shape = (32, 32, 32)
    plan = _plan(lib, shape)
    try:
        rho = torch.zeros(32, 32, 32, device=dev)
        st, *_ = _solve(lib, "lf2_poisson_solve_noalloc", plan, rho, 8, 1.0, 0, stream)
        assert st == lib.LF2_ERR_NOT_READY, lib.last_error()
        assert "k^2 table" in lib.last_error()
    finally:
        lib.load().lf2_plan_destroy(plan)
    # a lattice whose workspace exceeds the static array
    shape = (384, 384, 384)
    assert 8 * (shape[0] // 2 + 1) * shape[1] * shape[2] > lib.LF2_NOALLOC_SCRATCH_BYTES
    plan = _plan(lib, shape)
    try:
        # small stand-ins, never touched: the size check comes before any enqueue
        rho = torch.zeros(64, device=dev)
        phi = torch.zeros(64, device=dev)
        st = lib.load().lf2_poisson_solve_noalloc(plan, rho.data_ptr(), phi.data_ptr(), 1.0, 0, 0,
                                                  None, None, None, None, stream)
        assert st == lib.LF2_ERR_UNSUPPORTED, (st, lib.last_error())
        assert "workspace" in lib.last_error()
    finally:
        lib.load().lf2_plan_destroy(plan)
    torch.cuda.synchronize()
