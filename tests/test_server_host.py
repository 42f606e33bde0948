"""Host-side tests of the request server's admission logic with the fake
executor (no kernels launched): FIFO admission under the slot and HBM-budget
limits, queue-full and over-budget rejection, injected failures releasing
their capacity, non-blocking polls, latency timestamps and drain on destroy."""
import time

import pytest

import paper_1508_05610_amd as lf2
from paper_1508_05610_amd import _lib

LIB_OK = True
try:
    _lib.load()
except ImportError:
    LIB_OK = False

pytestmark = pytest.mark.skipif(not LIB_OK, reason="liblf2.so not built")

# fake device addresses: never dereferenced by the fake executor
RHO, PHI = 1 << 20, 2 << 20


def overlap_max(results):
    """Largest number of requests whose [t_admit, t_done) intervals overlap."""
    ev = []
    for _, _, ta, td in results:
        ev.append((ta, 1))
        ev.append((td, -1))
    ev.sort(key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_fifo_and_slot_limit():
    # distinct bin counts: no two requests can share a grouped solve, so each
    # is a launch unit of its own and takes a slot
    s = lf2.Server(1 << 40, max_slots=2, fake=True, delay_us=15000)
    tickets = [s.submit_raw((64, 64, 64), RHO, PHI, nbins=i + 1)[1] for i in range(6)]
    res = [s.poll(t) for t in tickets]
    s.close()
    assert all(r[0] == lf2.LF2_OK for r in res)
    admits = [r[2] for r in res]
    assert admits == sorted(admits), "admission must follow arrival order"
    assert overlap_max(res) <= 2
    # three waves of two: the last request waits for two earlier completions
    assert res[5][2] >= res[1][3] - 1e-6
    for ta, tb, tc in ((r[1], r[2], r[3]) for r in res):
        assert ta <= tb <= tc


def test_budget_limits_bytes_in_flight():
    fp = lf2.Server(1, fake=True).footprint((64, 64, 64), nbins=16)
    budget = int(2.5 * fp)
    s = lf2.Server(budget, max_slots=16, fake=True, delay_us=10000)
    tickets = [s.submit_raw((64, 64, 64), RHO, PHI, nbins=16)[1] for _ in range(6)]
    res = [s.poll(t) for t in tickets]
    st = s.stats()
    s.close()
    assert overlap_max(res) <= 2
    assert st["peak_bytes_in_flight"] <= budget
    assert st["peak_bytes_in_flight"] >= 2 * fp
    assert st["bytes_in_flight"] == 0 and st["completed"] == 6


def test_over_budget_request_rejected():
    s = lf2.Server(1 << 20, fake=True, delay_us=100)
    st, _ = s.submit_raw((128, 128, 128), RHO, PHI)
    assert st == lf2.LF2_ERR_BUDGET
    st2, t = s.submit_raw((16, 16, 16), RHO, PHI)
    assert st2 == lf2.LF2_OK
    assert s.poll(t)[0] == lf2.LF2_OK
    stats = s.stats()
    s.close()
    assert stats["rejected_budget"] == 1 and stats["submitted"] == 1


def test_queue_full_is_busy():
    s = lf2.Server(1 << 40, max_slots=1, max_queue=3, fake=True, delay_us=200000)
    out = [s.submit_raw((32, 32, 32), RHO, PHI) for _ in range(6)]
    busy = sum(1 for st, _ in out if st == lf2.LF2_ERR_BUSY)
    ok = [t for st, t in out if st == lf2.LF2_OK]
    stats = s.stats()
    assert busy >= 2 and busy + len(ok) == 6
    assert stats["rejected_busy"] == busy and stats["submitted"] == len(ok)
    for t in ok:
        assert s.poll(t)[0] == lf2.LF2_OK
    s.close()


def test_injected_failure_releases_capacity():
    fp = lf2.Server(1, fake=True).footprint((32, 32, 32))
    s = lf2.Server(fp, max_slots=4, fake=True, delay_us=2000, fail_ticket=2)
    tickets = [s.submit_raw((32, 32, 32), RHO, PHI)[1] for _ in range(4)]
    res = {t: s.poll(t) for t in tickets}
    stats = s.stats()
    s.close()
    assert res[2][0] == lf2.LF2_ERR_DEVICE
    assert all(res[t][0] == lf2.LF2_OK for t in tickets if t != 2)
    assert stats["failed"] == 1 and stats["completed"] == 3
    assert stats["bytes_in_flight"] == 0 and stats["in_flight"] == 0


def test_nonblocking_poll_and_forget():
    s = lf2.Server(1 << 40, fake=True, delay_us=100000)
    _, t = s.submit_raw((32, 32, 32), RHO, PHI)
    assert s.poll(t, wait=False) is None
    r = s.poll(t, wait=True)
    assert r[0] == lf2.LF2_OK and r[3] - r[2] >= 0.1 - 1e-3
    with pytest.raises(lf2.LF2Error):
        s.poll(t)
    with pytest.raises(lf2.LF2Error):
        s.poll(12345)
    s.close()


def test_late_arrival_joins_running_work():
    """Continuous batching: a request arriving while another runs starts
    before the first one finishes when a slot is free."""
    s = lf2.Server(1 << 40, max_slots=4, fake=True, delay_us=80000)
    _, t1 = s.submit_raw((64, 64, 64), RHO, PHI)
    time.sleep(0.02)
    _, t2 = s.submit_raw((32, 32, 32), RHO, PHI)
    r1, r2 = s.poll(t1), s.poll(t2)
    s.close()
    assert r2[2] < r1[3]


def test_arrival_time_is_kept():
    s = lf2.Server(1 << 40, fake=True, delay_us=1000)
    t0 = _lib.lf2_server_now() - 0.5
    _, t = s.submit_raw((32, 32, 32), RHO, PHI, t_arrival=t0)
    r = s.poll(t)
    s.close()
    assert r[1] == t0 and r[2] - r[1] >= 0.5


def test_destroy_drains():
    s = lf2.Server(1 << 40, max_slots=2, fake=True, delay_us=30000)
    for _ in range(4):
        assert s.submit_raw((32, 32, 32), RHO, PHI)[0] == lf2.LF2_OK
    t0 = time.monotonic()
    s.close()
    assert time.monotonic() - t0 >= 0.05


@pytest.mark.parametrize("sizes,kw,status", [
    ((33, 32, 32), {}, _lib.LF2_ERR_UNSUPPORTED),          # odd N0
    ((32, 32, 32), {"nbins": 5000}, _lib.LF2_ERR_UNSUPPORTED),
    ((32, 32, 32), {"nbins": -1}, _lib.LF2_ERR_UNSUPPORTED),
    ((32, 32, 32), {"dx": 0.0}, _lib.LF2_ERR_INVALID_ARG),
    ((32, 32, 32), {"flags": 8}, _lib.LF2_ERR_INVALID_ARG),
    ((0, 32, 32), {}, _lib.LF2_ERR_INVALID_ARG),
    ((32, 7 * 11, 32), {}, _lib.LF2_ERR_UNSUPPORTED),       # no kernels for length 77
])
def test_submit_validation(sizes, kw, status):
    s = lf2.Server(1 << 40, fake=True)
    st, _ = s.submit_raw(sizes, RHO, PHI, **kw)
    s.close()
    assert st == status


def test_submit_pointer_validation():
    s = lf2.Server(1 << 40, fake=True)
    assert s.submit_raw((32, 32, 32), 0, PHI)[0] == _lib.LF2_ERR_INVALID_ARG
    assert s.submit_raw((32, 32, 32), RHO, RHO)[0] == _lib.LF2_ERR_INVALID_ARG
    assert s.submit_raw((32, 32, 32), RHO + 2, PHI)[0] == _lib.LF2_ERR_INVALID_ARG
    s.close()


def test_footprint_formula():
    """rho + phi + half spectrum + bin partials, each rounded to 256 bytes."""
    def a256(b):
        return (b + 255) // 256 * 256
    s = lf2.Server(1, fake=True)
    for n0, n1, n2, nb in ((64, 48, 32, 0), (128, 96, 160, 64)):
        n = n0 * n1 * n2
        want = 8 * n + a256((n0 // 2 + 1) * n1 * n2 * 8)
        if nb:
            want += a256(1024 * (nb + 1) * 8) + a256((nb + 1) * 8)
        assert s.footprint((n0, n1, n2), nbins=nb) == want
    s.close()


def test_create_validation():
    with pytest.raises(lf2.LF2Error):
        lf2.Server(0, fake=True)
    with pytest.raises(lf2.LF2Error):
        lf2.Server(1 << 20, max_slots=0, fake=True)


def _lattices(n):
    """n distinct supported lattices."""
    lens = [16, 32, 48, 64, 80, 96, 128]
    out = []
    for a in lens:
        for b in lens:
            out.append((a, b, 32))
            if len(out) == n:
                return out
    raise AssertionError


def test_plan_cache_lru_eviction():
    s = lf2.Server(1 << 40, max_slots=64, fake=True, delay_us=0)

    def run(lat):
        _, t = s.submit_raw(lat, RHO, PHI)
        assert s.poll(t)[0] == lf2.LF2_OK

    lats = _lattices(33)
    for lat in lats[:32]:
        run(lat)
    st = s.stats()
    assert st["plans_cached"] == 32 and st["plan_misses"] == 32 and st["plan_hits"] == 0
    run(lats[0])                      # touch the oldest: now lats[1] is least recent
    run(lats[32])                     # a 33rd lattice evicts lats[1]
    st = s.stats()
    assert st["plans_cached"] == 32 and st["plan_hits"] == 1 and st["plan_misses"] == 33
    run(lats[0])                      # still resident
    assert s.stats()["plan_misses"] == 33
    run(lats[1])                      # was evicted
    assert s.stats()["plan_misses"] == 34
    s.close()


def test_latency_percentiles_nearest_rank():
    v = list(range(100, 0, -1))       # 1..100 shuffled order
    assert lf2.latency_percentiles(v, (50, 99, 100)) == (50.0, 99.0, 100.0)
    assert lf2.latency_percentiles([3.0], (50, 99)) == (3.0, 3.0)
    # n = 10: p50 is the 5th smallest, p99 the 10th
    w = [0.5, 9, 2, 7, 1, 8, 3, 6, 4, 5]
    assert lf2.latency_percentiles(w, (50, 99)) == (4.0, 9.0)
    with pytest.raises(ValueError):
        lf2.latency_percentiles([], (50,))


def test_pooled_workspace_counts_against_budget():
    """A mix of sizes under a small budget: in-flight plus idle pooled
    workspace never exceeds the budget (idle buffers that do not fit are
    freed to make room), and buffers are reused."""
    import random
    sizes = [(32, 32, 32), (64, 64, 64), (64, 32, 48), (96, 64, 64), (128, 64, 32)]
    fp = {sz: lf2.Server(1, fake=True).footprint(sz, nbins=16) for sz in sizes}
    budget = int(2.2 * max(fp.values()))
    s = lf2.Server(budget, max_slots=8, max_queue=64, fake=True, delay_us=3000)
    rng = random.Random(7)
    tickets = []
    for i in range(60):
        sz = rng.choice(sizes)
        st, t = s.submit_raw(sz, RHO, PHI, nbins=16)
        while st == lf2.LF2_ERR_BUSY:
            time.sleep(0.002)
            st, t = s.submit_raw(sz, RHO, PHI, nbins=16)
        assert st == lf2.LF2_OK
        tickets.append(t)
        if i % 7 == 0:
            time.sleep(0.004)
        cur = s.stats()
        assert cur["bytes_in_flight"] + cur["pooled_idle_bytes"] <= budget
    res = [s.poll(t) for t in tickets]
    st = s.stats()
    s.close()
    assert all(r[0] == lf2.LF2_OK for r in res)
    assert st["peak_bytes_in_use"] <= budget
    assert st["bytes_in_flight"] == 0
    assert 0 < st["pooled_idle_bytes"] <= budget


def test_requests_queued_together_are_grouped():
    """Requests that wait for a slot are admitted in launch units: the head
    of the queue with every queued request of the same lattice, dx, k^2 kind
    and bin count, as one grouped solve in one slot; the others wait their
    turn in order."""
    s = lf2.Server(1 << 40, max_slots=1, max_queue=64, fake=True, delay_us=30000)
    first = s.submit_raw((32, 32, 32), RHO, PHI)[1]          # takes the only slot
    a = [s.submit_raw((64, 64, 64), RHO, PHI, nbins=8)[1] for _ in range(2)]
    b = s.submit_raw((64, 64, 64), RHO, PHI, nbins=16)[1]     # another bin count
    a += [s.submit_raw((64, 64, 64), RHO, PHI, nbins=8)[1] for _ in range(2)]
    res = {t: s.poll(t) for t in [first] + a + [b]}
    st = s.stats()
    s.close()
    assert all(r[0] == lf2.LF2_OK for r in res.values())
    assert st["groups"] == 1 and st["grouped_requests"] == 4
    # the four nbins=8 requests ran together, after the first and before b
    ta = {res[t][2] for t in a}
    assert len(ta) == 1
    assert res[first][3] <= min(ta) + 1e-6
    assert res[b][2] >= res[a[0]][3] - 1e-6


def test_group_caps_by_lattice_points():
    """Grouping stops at 2^26 lattice points per grouped solve (four 256^3
    requests), and lattices above 2^24 points (384^3) always run alone."""
    s = lf2.Server(1 << 40, max_slots=1, max_queue=64, fake=True, delay_us=20000)
    first = s.submit_raw((32, 32, 32), RHO, PHI)[1]          # takes the only slot
    big = [s.submit_raw((256, 256, 256), RHO, PHI, nbins=8)[1] for _ in range(6)]
    huge = [s.submit_raw((384, 384, 384), RHO, PHI, nbins=8)[1] for _ in range(3)]
    res = {t: s.poll(t) for t in [first] + big + huge}
    st = s.stats()
    s.close()
    assert all(r[0] == lf2.LF2_OK for r in res.values())
    assert st["groups"] == 2 and st["grouped_requests"] == 6
    admits = sorted({res[t][2] for t in big})
    assert len(admits) == 2
    assert sum(res[t][2] == admits[0] for t in big) == 4
    assert len({res[t][2] for t in huge}) == 3
