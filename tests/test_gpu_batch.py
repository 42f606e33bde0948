"""GPU tests of the batched solves -- one persistent launch by default, and
the grouped launches -- every field against the FP64 oracle, batch against
solo solves, and repeated graph launches with eager work in between."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import assert_close, grf_field, rel_l2, tol

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


SMALL = [(32, 32, 32), (64, 48, 32), (96, 64, 128), (32, 16, 48), (160, 80, 96), (64, 384, 16),
         (384, 32, 64), (128, 192, 256)]


def fields_for(sizes, seed):
    out = []
    for i, (n0, n1, n2) in enumerate(sizes):
        out.append(synth.normal(seed, n0 * n1 * n2, stream=i, dtype=np.float32).reshape(n2, n1, n0))
    return out


@pytest.mark.parametrize("grouped", [False, True])
def test_batch_tiny(lf2, grouped):
    """Two small fields; a dependency wait that gives up shows up as error bit 0."""
    sizes = [(32, 32, 32), (64, 32, 16)]
    fs = fields_for(sizes, seed=30)
    b = lf2.Batch(sizes, nbins=8, grouped=grouped)
    print(f"case batch tiny grouped={grouped}: items {b.nitems} launches {b.launches}", flush=True)
    assert grouped or b.launches == 1
    rhos = [torch.from_numpy(f).to(dev()) for f in fs]
    phis = [torch.zeros_like(r) for r in rhos]
    pks = [torch.zeros(8, dtype=torch.float64, device=dev()) for _ in fs]
    b.run(rhos, phis, pks)
    torch.cuda.synchronize()
    err = b.error()
    print(f"  ran, error bits {err}", flush=True)
    assert err == 0
    for s, f, p, pk in zip(sizes, fs, phis, pks):
        f64 = f.astype(np.float64)
        assert_close(p.cpu().numpy(), oracle.poisson(f64), s)
        opk, _, _ = oracle.power_spectrum(oracle.r2c(f64), s, 8)
        assert_close(pk.cpu().numpy(), opk, s)


@pytest.mark.parametrize("mode", ["xcd", "one_queue", "grouped"])
def test_batch_matches_oracle_and_solo(lf2, mode):
    print(f"case batch small mixed sizes mode={mode}", flush=True)
    nb = 16
    fs = fields_for(SMALL, seed=31)
    b = lf2.Batch(SMALL, nbins=nb, grouped=mode == "grouped", one_queue=mode == "one_queue")
    print(f"  launches {b.launches} queues {b.queues} per-XCD {b.per_xcd}", flush=True)
    assert mode == "grouped" or b.launches == 1
    if mode == "one_queue":
        assert b.queues == 1 and b.per_xcd == 0
    rhos = [torch.from_numpy(f).to(dev()) for f in fs]
    phis = [torch.zeros_like(r) for r in rhos]
    pks = [torch.zeros(nb, dtype=torch.float64, device=dev()) for _ in fs]
    kms = [torch.zeros(nb, dtype=torch.float64, device=dev()) for _ in fs]
    cts = [torch.zeros(nb, dtype=torch.float64, device=dev()) for _ in fs]
    b.run(rhos, phis, pks, kms, cts)
    torch.cuda.synchronize()
    assert b.error() == 0
    for i, (s, f) in enumerate(zip(SMALL, fs)):
        f64 = f.astype(np.float64)
        ref = oracle.poisson(f64)
        opk, okm, oct_ = oracle.power_spectrum(oracle.r2c(f64), s, nb)
        assert_close(phis[i].cpu().numpy(), ref, s, f"field {i} {s} phi")
        assert_close(pks[i].cpu().numpy(), opk, s, f"field {i} {s} pk")
        assert np.array_equal(cts[i].cpu().numpy(), oct_)
        assert rel_l2(kms[i].cpu().numpy(), okm) <= 1e-12
        # the same field solved alone gives the same potential
        plan = lf2.Plan(s, lf2.LF2_R2C)
        solo, spk, _, _ = plan.poisson(rhos[i], nbins=nb)
        torch.cuda.synchronize()
        print(f"  field {i}: batch == solo bitwise: {bool(torch.equal(solo, phis[i]))}", flush=True)
        assert rel_l2(solo.cpu().numpy(), phis[i].cpu().numpy()) <= 1e-6
        assert rel_l2(spk.cpu().numpy(), pks[i].cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("grouped", [False, True])
def test_batch_graph_replays_with_eager_work(lf2, grouped):
    print(f"case batch replays grouped={grouped}", flush=True)
    sizes = [(64, 64, 64), (96, 32, 48), (32, 128, 64)]
    fs = fields_for(sizes, seed=32)
    b = lf2.Batch(sizes, nbins=8, grouped=grouped)
    rhos = [torch.from_numpy(f).to(dev()) for f in fs]
    phis = [torch.zeros_like(r) for r in rhos]
    b.run(rhos, phis)
    torch.cuda.synchronize()
    first = [p.clone() for p in phis]
    plan = lf2.Plan(sizes[0], lf2.LF2_R2C)
    for rep in range(3):
        for p in phis:
            p.zero_()
        eager = plan.poisson(rhos[0])           # eager work between replays
        torch.cuda.synchronize()
        b.run(rhos, phis)
        torch.cuda.synchronize()
        assert b.error() == 0
        for a0, p in zip(first, phis):
            assert torch.equal(a0, p), f"replay {rep} differs"
        assert rel_l2(eager.cpu().numpy(), phis[0].cpu().numpy()) <= 1e-6


def test_batch_new_pointers_reupload(lf2):
    sizes = [(32, 32, 32), (64, 32, 16)]
    b = lf2.Batch(sizes)
    for seed in (41, 42):
        fs = fields_for(sizes, seed=seed)
        rhos = [torch.from_numpy(f).to(dev()) for f in fs]
        phis = [torch.zeros_like(r) for r in rhos]
        b.run(rhos, phis)
        torch.cuda.synchronize()
        for s, f, p in zip(sizes, fs, phis):
            assert_close(p.cpu().numpy(), oracle.poisson(f.astype(np.float64)), s)


def test_batch_config_48_uneven_grf(lf2):
    """48 P(k) ~ k^-2 fields, extents per axis from {64,...,256}, field 0 = 128x192x256."""
    S = [64, 96, 128, 160, 192, 256]
    draws = synth.choice(5, 48 * 3, len(S)).reshape(48, 3)
    sizes = [(128, 192, 256)] + [tuple(S[j] for j in d) for d in draws[1:]]
    print("case batch 48 fields", flush=True)
    fl = []
    for i, s in enumerate(sizes):
        f32, f64, _ = grf_field(s, 2.0, seed=1000 + i)
        fl.append((f32, f64))
    b = lf2.Batch(sizes, nbins=32)
    print(f"  one persistent launch: {b.launches} launch(es), {b.nitems} work items, "
          f"{b.queues} queues, per-XCD {b.per_xcd}", flush=True)
    assert b.launches == 1
    rhos = [torch.from_numpy(f32).to(dev()) for f32, _ in fl]
    phis = [torch.zeros_like(r) for r in rhos]
    pks = [torch.zeros(32, dtype=torch.float64, device=dev()) for _ in fl]
    b.run(rhos, phis, pks)
    torch.cuda.synchronize()
    assert b.error() == 0
    # a second replay gives the same bits (the queue resets itself)
    phis2 = [torch.zeros_like(r) for r in rhos]
    b.run(rhos, phis2, pks)
    torch.cuda.synchronize()
    assert b.error() == 0
    assert all(torch.equal(a, c) for a, c in zip(phis, phis2))
    worst = 0.0
    for i, (s, (f32, f64)) in enumerate(zip(sizes, fl)):
        opk, _, _ = oracle.power_spectrum(oracle.r2c(f64), s, 32)
        e, em = assert_close(phis[i].cpu().numpy(), oracle.poisson(f64), s)
        epk, epm = assert_close(pks[i].cpu().numpy(), opk, s)
        worst = max(worst, e / tol(s), em / tol(s), epk / tol(s), epm / tol(s))
    print(f"  worst error / tolerance {worst:.3e}", flush=True)


@pytest.mark.parametrize("discrete,dx,grouped", [(0, 0.5, False), (1, 1.0, False), (1, 0.25, True)])
def test_batch_without_pk_flags_and_dx(lf2, discrete, dx, grouped):
    """Poisson-only batches (no binning epilogue, no finalize) with the
    discrete-Laplacian k^2 and a lattice spacing: every field against the
    oracle and against its solo solve with the same settings."""
    print(f"case batch no pk discrete={discrete} dx={dx} grouped={grouped}", flush=True)
    flags = lf2.LF2_POISSON_DISCRETE_K2 if discrete else 0
    fs = fields_for(SMALL, seed=33)
    b = lf2.Batch(SMALL, nbins=0, dx=dx, poisson_flags=flags, grouped=grouped)
    bp = lf2.Batch(SMALL, nbins=8, dx=dx, poisson_flags=flags, grouped=grouped)
    if grouped:
        assert b.launches + 1 == bp.launches  # the finalize launch only with binning
    else:
        assert b.launches == bp.launches == 1
        assert b.nitems + len(SMALL) == bp.nitems  # one finalize item per field
    bp.close()
    rhos = [torch.from_numpy(f).to(dev()) for f in fs]
    phis = [torch.zeros_like(r) for r in rhos]
    b.run(rhos, phis)
    torch.cuda.synchronize()
    assert b.error() == 0
    for i, (s, f) in enumerate(zip(SMALL, fs)):
        ref = oracle.poisson(f.astype(np.float64), dx=dx, k2mode=discrete)
        assert_close(phis[i].cpu().numpy(), ref, s)
        plan = lf2.Plan(s, lf2.LF2_R2C)
        solo = plan.poisson(rhos[i], dx=dx, flags=flags)
        torch.cuda.synchronize()
        assert rel_l2(solo.cpu().numpy(), phis[i].cpu().numpy()) <= 1e-6
