"""GPU tests of the request server: requests of mixed lattice sizes served
concurrently on several streams under an HBM budget give the potentials and
power spectra of solo solves and of the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import assert_close, rel_l2, tol

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


SIZES = [(32, 32, 32), (64, 64, 64), (128, 128, 128), (96, 64, 48), (64, 32, 128),
         (256, 256, 256), (160, 96, 80), (48, 48, 48)]


def make_inputs(sizes, seed, nb):
    reqs = []
    for i, (n0, n1, n2) in enumerate(sizes):
        f = synth.normal(seed, n0 * n1 * n2, stream=i, dtype=np.float32).reshape(n2, n1, n0)
        rho = torch.from_numpy(f).to(dev())
        phi = torch.full_like(rho, float("nan"))
        pk = torch.full((nb,), float("nan"), dtype=torch.float64, device=dev())
        cnt = torch.zeros(nb, dtype=torch.float64, device=dev())
        reqs.append((f, rho, phi, pk, cnt))
    torch.cuda.synchronize()
    return reqs


def test_served_equals_solo_and_oracle(lf2):
    nb = 16
    print("case server 8 mixed sizes, 3 streams, 4 slots", flush=True)
    srv = lf2.Server(8 << 30, max_slots=4, nstreams=3)
    reqs = make_inputs(SIZES, seed=61, nb=nb)
    tickets = []
    for (f, rho, phi, pk, cnt) in reqs:
        st, t = srv.submit(rho, phi, nbins=nb, pk=pk, count=cnt)
        assert st == lf2.LF2_OK
        tickets.append(t)
    res = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert all(r[0] == lf2.LF2_OK for r in res), res
    assert stats["completed"] == len(SIZES) and stats["bytes_in_flight"] == 0
    for i, (s, (f, rho, phi, pk, cnt)) in enumerate(zip(SIZES, reqs)):
        plan = lf2.Plan(s, lf2.LF2_R2C)
        solo, spk, _, scnt = plan.poisson(rho, nbins=nb)
        torch.cuda.synchronize()
        e_solo = rel_l2(phi.cpu().numpy(), solo.cpu().numpy())
        e_pk = rel_l2(pk.cpu().numpy(), spk.cpu().numpy())
        print(f"  request {i} {s}: served vs solo phi {e_solo:.2e} pk {e_pk:.2e}", flush=True)
        assert e_solo <= 1e-6 and e_pk <= 1e-6
        assert torch.equal(cnt, scnt)
        if s[0] * s[1] * s[2] <= 128 ** 3:
            f64 = f.astype(np.float64)
            assert_close(phi.cpu().numpy(), oracle.poisson(f64), s)
            opk, _, oct_ = oracle.power_spectrum(oracle.r2c(f64), s, nb)
            assert_close(pk.cpu().numpy(), opk, s)
            assert np.array_equal(cnt.cpu().numpy(), oct_)


def test_budget_queues_and_pool_reuse(lf2):
    nb = 8
    sizes = [(128, 128, 128)] * 3 + [(64, 64, 64)] * 3
    fp = lf2.Server(1, fake=True).footprint((128, 128, 128), nbins=nb)
    budget = 2 * fp + fp // 2
    print(f"case server budget {budget} bytes, two waves", flush=True)
    srv = lf2.Server(budget, max_slots=8, nstreams=4)
    srv.prepare(sorted(set(sizes)), nbins=nb)
    assert srv.stats()["plans_cached"] == 2
    for wave, seed in enumerate((62, 63)):
        reqs = make_inputs(sizes, seed=seed, nb=nb)
        tickets = [srv.submit(rho, phi, nbins=nb, pk=pk)[1] for (_, rho, phi, pk, _) in reqs]
        res = [srv.poll(t) for t in tickets]
        assert all(r[0] == lf2.LF2_OK for r in res)
        for s, (f, rho, phi, pk, _) in zip(sizes, reqs):
            f64 = f.astype(np.float64)
            assert_close(phi.cpu().numpy(), oracle.poisson(f64), s)
        print(f"  wave {wave} ok", flush=True)
    stats = srv.stats()
    srv.close()
    assert stats["peak_bytes_in_flight"] <= budget
    assert stats["completed"] == 2 * len(sizes)


def test_discrete_k2_and_pk_of_phi(lf2):
    s = (64, 48, 32)
    nb = 12
    f = synth.normal(64, s[0] * s[1] * s[2], dtype=np.float32).reshape(s[2], s[1], s[0])
    rho = torch.from_numpy(f).to(dev())
    phi = torch.empty_like(rho)
    pk = torch.zeros(nb, dtype=torch.float64, device=dev())
    torch.cuda.synchronize()
    srv = lf2.Server(1 << 30)
    flags = lf2.LF2_POISSON_DISCRETE_K2 | lf2.LF2_PK_OF_PHI
    st, t = srv.submit(rho, phi, dx=0.5, flags=flags, nbins=nb, pk=pk)
    assert st == lf2.LF2_OK and srv.poll(t)[0] == lf2.LF2_OK
    srv.close()
    plan = lf2.Plan(s, lf2.LF2_R2C)
    solo, spk, _, _ = plan.poisson(rho, dx=0.5, flags=flags, nbins=nb)
    torch.cuda.synchronize()
    assert rel_l2(phi.cpu().numpy(), solo.cpu().numpy()) <= 1e-6
    assert rel_l2(pk.cpu().numpy(), spk.cpu().numpy()) <= 1e-6


def test_serving_config_sizes_against_oracle(lf2):
    """One request of each cubic size of the serving workload (N in {32, 64,
    128, 256, 384}, 64 bins, 8 GiB budget), the largest at full size, each
    served result against the oracle."""
    nb = 64
    sizes = [(n, n, n) for n in (384, 32, 256, 64, 128)]
    print("case serving config sizes 32..384 vs oracle", flush=True)
    srv = lf2.Server(8 << 30, max_slots=16, nstreams=4)
    reqs = make_inputs(sizes, seed=6, nb=nb)
    tickets = []
    for (f, rho, phi, pk, cnt) in reqs:
        st, t = srv.submit(rho, phi, nbins=nb, pk=pk, count=cnt)
        assert st == lf2.LF2_OK
        tickets.append(t)
    res = [srv.poll(t) for t in tickets]
    srv.close()
    assert all(r[0] == lf2.LF2_OK for r in res), res
    for s, (f, rho, phi, pk, cnt) in zip(sizes, reqs):
        f64 = f.astype(np.float64)
        opk, _, oct_ = oracle.power_spectrum(oracle.r2c(f64), s, nb)
        assert_close(phi.cpu().numpy(), oracle.poisson(f64), s, f"{s} phi")
        assert_close(pk.cpu().numpy(), opk, s, f"{s} pk")
        assert np.array_equal(cnt.cpu().numpy(), oct_)
