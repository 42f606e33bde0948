#!/usr/bin/env python3
"""Throughput of the lf2 hot path on one MI355X.

One step = one pass of the whole transform path over the 512^3 FP32
workload:
  r2c forward + c2r backward of a real N(0,1) field (1 component),
  c2c forward + backward of a complex64 3-component AoS N(0,1) field,
  Poisson solve of the real field with a fused 128-bin power spectrum and
  FP64 Parseval sums.
value = 3-D FFT GFLOP/s with the conventional 5 N log2 N per transform and
component (10 transforms per step).  Inputs are resident in HBM before the
timed region.  Prints one JSON line.

Extra fields: per-op times, algorithmic GB/s, the dominant kernel's HBM
roofline (its average duration measured with HIP events inside the timed
region), the FP64 oracle timed on the host cores (CPU baseline), and the
relative errors of the results against that oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def kernel_source_hash() -> str:
    """Hash of the sources that decide the transform kernels and their launch
    shapes (the batch and server sources do not)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1508_05610_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".hpp")) or fn == "lf2_api.cpp":
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def tuning_spec(tuning: dict) -> str:
    """The --tuning string of a plan_tuning table."""
    return ";".join(
        nm + ":" + ",".join(f"{a}={t[f'axis{i}']['variant']}/{t[f'axis{i}']['chunk']}"
                            for i, a in ((1, "y"), (2, "z")))
        for nm, t in tuning.items())


def measured_traffic(record: str, tuning: str):
    """HBM bytes per launch of the kernel record `record` (kernel, pass and
    shape) from the committed PMC summary, if it was taken on the current
    kernel sources with the same pass tuning; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash() or t.get("tuning") != tuning:
        return None
    k = t.get("records", {}).get(record)
    return None if k is None else k.get("hbm_bytes_per_launch")


def parse_tuning(spec: str) -> dict:
    """'r2c:y=0/16,z=1/4;c2c3:y=1/16,z=1/64' -> {'r2c': {1: (0, 16), 2: (1, 4)}, ...}"""
    out = {}
    for part in spec.split(";"):
        nm, rest = part.split(":")
        d = {}
        for item in rest.split(","):
            ax, vc = item.split("=")
            v, c = vc.split("/")
            d[{"y": 1, "z": 2}[ax]] = (int(v), int(c))
        out[nm] = d
    return out


def bench_batch(args, torch, np, lf2, stream):
    """48 Poisson solves with fused 32-bin P(k) on uneven lattices (extents per
    axis from {64, 96, 128, 160, 192, 256}, field 0 = 128x192x256): one
    persistent launch replayed from a hipGraph, against the grouped launches
    (one per pass and line length) and against 48 plain lf2_poisson_solve
    calls.
    Inputs are seeded N(0,1) fields (run time does not depend on values; the
    random-field parity of the same workload is in the tests)."""
    import synth
    from paper_1508_05610_amd import _lib
    S = [64, 96, 128, 160, 192, 256]
    draws = synth.choice(5, 48 * 3, len(S)).reshape(48, 3)
    sizes = [(128, 192, 256)] + [tuple(S[j] for j in d) for d in draws[1:]]
    nb = 32
    dev = torch.device("cuda:0")
    rhos = [torch.from_numpy(synth.normal(5, a * b * c, stream=i, dtype=np.float32)
                             .reshape(c, b, a)).to(dev) for i, (a, b, c) in enumerate(sizes)]
    phis = [torch.empty_like(r) for r in rhos]
    pks = [torch.empty(nb, dtype=torch.float64, device=dev) for _ in sizes]
    kms = [torch.empty(nb, dtype=torch.float64, device=dev) for _ in sizes]
    cts = [torch.empty(nb, dtype=torch.float64, device=dev) for _ in sizes]
    batch = lf2.Batch(sizes, nbins=nb)
    one_q = lf2.Batch(sizes, nbins=nb, one_queue=True)
    grouped = lf2.Batch(sizes, nbins=nb, grouped=True)
    plans = {}
    for s in sizes:
        if s not in plans:
            plans[s] = lf2.Plan(s, lf2.LF2_R2C)
    sh = int(stream.cuda_stream)

    def run_batch():
        batch.run(rhos, phis, pks, kms, cts, stream=stream)

    def run_grouped():
        grouped.run(rhos, phis, pks, kms, cts, stream=stream)

    def run_one_queue():
        one_q.run(rhos, phis, pks, kms, cts, stream=stream)

    def run_plain():
        for s, r, p, a, b, c in zip(sizes, rhos, phis, pks, kms, cts):
            _lib.lf2_poisson_solve(plans[s].handle, r.data_ptr(), p.data_ptr(), 1.0, 0, nb,
                                   a.data_ptr(), b.data_ptr(), c.data_ptr(), 0, sh)

    def timed(fn, reps):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(3, args.steps)
    t_batch = timed(run_batch, reps)
    err = batch.error()
    t_grouped = timed(run_grouped, reps)
    t_one_q = timed(run_one_queue, reps)
    err |= one_q.error()
    t_plain = timed(run_plain, reps)
    points = sum(a * b * c for a, b, c in sizes)
    alg = sum(8.0 * a * b * c + 64.0 * (a // 2 + 1) * b * c for a, b, c in sizes)
    nitems, launches, wsb = batch.nitems, batch.launches, batch.workspace_bytes
    g_launches = grouped.launches
    queues, per_xcd = batch.queues, batch.per_xcd
    batch.close()
    grouped.close()
    one_q.close()
    return {
        "workload": "48 Poisson + 32-bin P(k) solves, extents per axis from {64..256}, "
                    "field 0 = 128x192x256",
        "points": points, "batch_ms": round(t_batch, 4), "plain_ms": round(t_plain, 4),
        "speedup_vs_plain": round(t_plain / t_batch, 3),
        "batch_gbps_algorithmic": round(alg / (t_batch * 1e-3) / 1e9, 1),
        "plain_gbps_algorithmic": round(alg / (t_plain * 1e-3) / 1e9, 1),
        "work_items": nitems, "launches_per_run": launches, "plain_launches_per_run": 48 * 7,
        "queues": queues, "queue_per_xcd": per_xcd,
        "one_queue_ms": round(t_one_q, 4),
        "grouped_ms": round(t_grouped, 4), "grouped_launches_per_run": g_launches,
        "error_bits": err,
    }


def _timed_median(torch, np, fn, stream, reps):
    """Median, p10 and p90 in ms over `reps` repetitions, each bracketed by
    its own events on `stream` (two warm-ups first)."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return float(np.median(t)), float(np.percentile(t, 10)), float(np.percentile(t, 90))


def bench_copy(torch, np, stream):
    """HBM bandwidth a plain device copy reaches (1 GiB read + 1 GiB written)."""
    dev = torch.device("cuda:0")
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    ms, _, _ = _timed_median(torch, np, lambda: dst.copy_(src), stream, 20)
    del src, dst
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def bench_small_configs(args, torch, np, lf2, stream):
    """The two smaller workloads, each timed and checked against the FP64 oracle:
    32^3 FP64 N(0,1) field (seed 1; the GPU gets its FP32 rounding): r2c, c2r,
    Poisson, 16-bin P(k);
    256^3 FP32 Gaussian random field with P ~ k^-3 (fixed amplitude, seeded
    phases, seed 2): r2c, c2r, Poisson with a fused 128-bin P(k)."""
    import oracle
    import synth
    from paper_1508_05610_amd import _lib
    dev = torch.device("cuda:0")
    sh = int(stream.cuda_stream)
    out = {}

    def rel_l2(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    def rel_max(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    for name, S, nb in (("tiny_32", 32, 16), ("grf_256", 256, 128)):
        n = (S, S, S)
        N = S ** 3
        if S == 32:
            f64 = synth.normal(1, N).reshape(S, S, S)
            f32 = f64.astype(np.float32)
            recipe = "32^3 FP64 N(0,1) field, seed 1 (FP32 copy on the GPU)"
        else:
            u = synth.uniform(2, N)
            g64, _ = oracle.grf(n, 3.0, u)
            f32 = g64.astype(np.float32)
            f64 = f32.astype(np.float64)
            recipe = "256^3 FP32 GRF, P ~ k^-3, fixed amplitude, seeded phases (seed 2)"
        p = lf2.Plan(n, lf2.LF2_R2C, autotune=S >= 256)
        x = torch.from_numpy(f32).to(dev)
        F = torch.empty(p.k_shape, dtype=torch.complex64, device=dev)
        back = torch.empty(p.x_shape, dtype=torch.float32, device=dev)
        phi = torch.empty(p.x_shape, dtype=torch.float32, device=dev)
        pk = torch.empty(nb, dtype=torch.float64, device=dev)
        km = torch.empty(nb, dtype=torch.float64, device=dev)
        ct = torch.empty(nb, dtype=torch.float64, device=dev)
        ops = {
            "r2c_fwd": lambda: _lib.lf2_fft_execute(p.handle, lf2.LF2_FORWARD, x.data_ptr(),
                                                    F.data_ptr(), sh),
            "c2r_bwd": lambda: _lib.lf2_fft_execute(p.handle, lf2.LF2_BACKWARD, F.data_ptr(),
                                                    back.data_ptr(), sh),
            "poisson_pk": lambda: _lib.lf2_poisson_solve(p.handle, x.data_ptr(), phi.data_ptr(),
                                                         1.0, 0, nb, pk.data_ptr(), km.data_ptr(),
                                                         ct.data_ptr(), 0, sh),
        }
        nh = S // 2 + 1
        alg = {"r2c_fwd": 4.0 * N + 5 * 8.0 * nh * S * S, "c2r_bwd": 4.0 * N + 5 * 8.0 * nh * S * S,
               "poisson_pk": 8.0 * N + 8 * 8.0 * nh * S * S}
        res = {"workload": recipe, "nbins": nb, "ops": {}}
        reps = 100 if S <= 32 else 50
        for k, fn in ops.items():
            med, p10, p90 = _timed_median(torch, np, fn, stream, reps)
            res["ops"][k] = {"ms": round(med, 5), "p10": round(p10, 5), "p90": round(p90, 5),
                             "gbps": round(alg[k] / (med * 1e-3) / 1e9, 1),
                             "gflops": round(5.0 * N * math.log2(N) / (med * 1e-3) / 1e9, 1)}
        # errors against the oracle (the results of the last timed calls)
        torch.cuda.synchronize()
        Fo = oracle.r2c(f64)
        Fg = F.cpu().numpy()
        bg = back.cpu().numpy()
        bo = oracle.c2r(Fg.astype(np.complex128), S)
        phio = oracle.poisson(f64)
        opk, okm, oct_ = oracle.power_spectrum(Fo, n, nb)
        res["errors"] = {
            "r2c_fwd": {"rel_l2": rel_l2(Fg, Fo), "max": rel_max(Fg, Fo)},
            "c2r_bwd": {"rel_l2": rel_l2(bg, bo), "max": rel_max(bg, bo)},
            "poisson_phi": {"rel_l2": rel_l2(phi.cpu().numpy(), phio),
                            "max": rel_max(phi.cpu().numpy(), phio)},
            "pk": {"rel_l2": rel_l2(pk.cpu().numpy(), opk), "max": rel_max(pk.cpu().numpy(), opk),
                   "counts_exact": bool(np.array_equal(ct.cpu().numpy(), oct_))},
            "tolerance_rel_l2": 1e-5 * math.log2(N),
        }
        p.close()
        out[name] = res
    return out


def bench_lane_exchange(args, torch, lf2, _lib):
    """The x pass of a 64x1024x1024 c2c transform (one component, 1 GiB of
    traffic per pass) with the exchange between its two radix-8 stages
    through LDS (tuning 0), ds_bpermute (1) or DPP moves (2): average
    microseconds per launch from the library's event records."""
    shape = (64, 1024, 1024)
    g = torch.Generator(device="cuda").manual_seed(11)
    z = torch.randn(shape[2], shape[1], shape[0], dtype=torch.complex64, device="cuda",
                    generator=g)
    out = torch.empty_like(z)
    res = {}
    for v, name in ((0, "lds"), (1, "ds_bpermute"), (2, "dpp")):
        plan = lf2.Plan(shape, lf2.LF2_C2C)
        plan.set_tuning(0, v)
        for _ in range(args.warmup):
            plan.forward(z, out=out)
        torch.cuda.synchronize()
        _lib.lf2_profile_enable(True)
        _lib.lf2_profile_reset()
        for _ in range(args.steps):
            plan.forward(z, out=out)
        torch.cuda.synchronize()
        t = _lib.profile_table()
        _lib.lf2_profile_enable(False)
        for k, (n_, ms_, by_) in t.items():
            if k.startswith("k_x"):
                res[name] = {"kernel": k, "avg_us": round(1e3 * ms_ / n_, 2),
                             "gbps": round(by_ / n_ / (ms_ / n_ * 1e-3) / 1e9, 1)}
    return {"lane_exchange": res, "lattice": list(shape), "steps": args.steps}


def bench_tile_variants(args, torch, lf2, _lib):
    """The strided passes of an N^3 lattice (c2c, and r2c) forward in each
    tile setting of the y and z passes -- narrow (0), wide (1), register
    tile (4, lines of 1024 and 2048 points), each plain or nontemporal (+2)
    -- and the fused Poisson + 128-bin P(k) pass in its LDS-staged (0) and
    register (1) tile (tuning axis 3, 256-, 512- and 1024-point z lines):
    average microseconds and algorithmic GB/s per launch from the library's
    event records.  Inputs: torch N(0,1) on the device, seed 12."""
    n = args.variants
    shape = (n, n, n)
    g = torch.Generator(device="cuda").manual_seed(12)
    out = {"lattice": list(shape), "steps": args.steps, "strided": {}, "fused": {}}

    def records(run, prefix):
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        _lib.lf2_profile_enable(True)
        _lib.lf2_profile_reset()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        t = _lib.profile_table()
        _lib.lf2_profile_enable(False)
        return {k: {"avg_us": round(1e3 * ms_ / n_, 1),
                    "gbps": round(by_ / n_ / (ms_ / n_ * 1e-3) / 1e9, 1)}
                for k, (n_, ms_, by_) in t.items() if prefix(k)}

    kinds = [("r2c", lf2.LF2_R2C)] + ([("c2c", lf2.LF2_C2C)] if n <= 1024 else [])
    for name, kind in kinds:
        if kind == lf2.LF2_C2C:
            x = torch.randn(n, n, n, dtype=torch.complex64, device="cuda", generator=g)
        else:
            x = torch.randn(n, n, n, dtype=torch.float32, device="cuda", generator=g)
        res = {}
        for v in (0, 1, 2, 3, 4, 6):
            plan = lf2.Plan(shape, kind)
            try:
                plan.set_tuning(1, v)
                plan.set_tuning(2, v)
            except lf2.LF2Error:
                continue  # no such tile for this length
            y = plan.forward(x)
            res[str(v)] = records(lambda: plan.forward(x, out=y),
                                  lambda k: k.startswith("k_strided"))
            del plan, y
            torch.cuda.empty_cache()
        out["strided"][name] = res
        del x
        torch.cuda.empty_cache()
    x = torch.randn(n, n, n, dtype=torch.float32, device="cuda", generator=g)
    phi = torch.empty_like(x)
    for v in (0, 1):
        plan = lf2.Plan(shape, lf2.LF2_R2C)
        try:
            plan.set_tuning(3, v)
        except lf2.LF2Error:
            continue
        out["fused"][str(v)] = records(lambda: plan.poisson(x, phi=phi, nbins=128),
                                       lambda k: "+poisson" in k)
        del plan
    return out


def bench_serving(args, torch, np, lf2):
    """Request serving: Poisson + 64-bin P(k) solves on cubic lattices with
    N uniform over {32, 64, 128, 256, 384}, Poisson arrivals at 200 req/s
    (seed 6), 8 GiB HBM admission budget, plans resident.  Latency is
    t_done - t_arrival.  Compared with a plain loop that launches each
    request with lf2_poisson_solve on one stream and waits for it, on the
    same arrival schedule; then both at saturation (every request arriving at
    once)."""
    import collections

    import synth
    from paper_1508_05610_amd import _lib
    NS = [32, 64, 128, 256, 384]
    nb = 64
    rate = 200.0
    nreq = args.serve_requests
    dev = torch.device("cuda:0")
    draws = synth.choice(6, nreq, len(NS))
    req_n = [NS[int(d)] for d in draws]
    u = synth.uniform(6, nreq, stream=1)
    gaps = -np.log1p(-u) / rate
    pool = 20  # buffer sets per lattice size (caller-owned request memory)
    bufs = {}
    for j, n in enumerate(NS):
        f = torch.from_numpy(synth.normal(6, n ** 3, stream=10 + j, dtype=np.float32)
                             .reshape(n, n, n)).to(dev)
        rho = [f.clone() for _ in range(pool)]
        phi = [torch.empty_like(f) for _ in range(pool)]
        pks = [torch.empty((3, nb), dtype=torch.float64, device=dev) for _ in range(pool)]
        bufs[n] = (rho, phi, pks)
    torch.cuda.synchronize()
    plans = {n: lf2.Plan((n, n, n), lf2.LF2_R2C) for n in NS}
    budget = 8 << 30
    srv = lf2.Server(budget, max_slots=16, nstreams=4, max_queue=1 << 16)
    srv.prepare([(n, n, n) for n in NS], nbins=nb)
    now = _lib.lf2_server_now

    def args_of(n, k):
        rho, phi, pks = bufs[n]
        p = pks[k]
        return (rho[k].data_ptr(), phi[k].data_ptr(), p[0].data_ptr(), p[1].data_ptr(),
                p[2].data_ptr())

    def served(arrivals):
        free = {n: list(range(pool)) for n in NS}
        out = collections.OrderedDict()   # ticket -> (n, slot)
        lat, last = [], {}
        t_first = now()

        def reap(block):
            done = []
            for t, (n, k) in out.items():
                r = srv.poll(t, wait=block)
                if r is None:
                    if block:
                        raise RuntimeError("blocking poll returned no result")
                    continue
                if r[0] != lf2.LF2_OK:
                    raise RuntimeError(f"request {t} failed: {_lib.status_string(r[0])}")
                lat.append(r[3] - r[1])
                free[n].append(k)
                done.append(t)
                if block:
                    break
            for t in done:
                del out[t]

        for i, n in enumerate(req_n):
            ta = arrivals[i]
            while now() < ta:
                reap(False)
                if ta - now() > 5e-4:
                    time.sleep(2e-4)
            while not free[n]:
                reap(True)
            k = free[n].pop()
            rp, pp, a, b, c = args_of(n, k)
            while True:
                st, t = srv.submit_raw((n, n, n), rp, pp, 1.0, 0, nb, a, b, c, t_arrival=ta)
                if st == lf2.LF2_OK:
                    break
                if st != lf2.LF2_ERR_BUSY:
                    raise RuntimeError(f"submit: {_lib.status_string(st)}")
                reap(True)
            out[t] = (n, k)
            last[n] = k
        while out:
            reap(True)
        return lat, now() - t_first, last

    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    def plain(arrivals, sync_each=True):
        lat = []
        slot = {n: 0 for n in NS}
        t_first = now()
        for i, n in enumerate(req_n):
            ta = arrivals[i]
            while now() < ta:
                if ta - now() > 5e-4:
                    time.sleep(2e-4)
            k = slot[n]
            slot[n] = (k + 1) % pool
            rp, pp, a, b, c = args_of(n, k)
            _lib.lf2_poisson_solve(plans[n].handle, rp, pp, 1.0, 0, nb, a, b, c, 0, sh)
            if sync_each:
                stream.synchronize()
                lat.append(now() - ta)
        stream.synchronize()
        return lat, now() - t_first

    # warm every path once
    served([0.0] * nreq)
    plain([0.0] * nreq)
    torch.cuda.synchronize()

    t0 = now() + 0.05
    arr = list(t0 + np.cumsum(gaps))
    lat_s, wall_s, _ = served(arr)
    t0 = now() + 0.05
    arr = list(t0 + np.cumsum(gaps))
    lat_p, wall_p = plain(arr)
    sat = [0.0] * nreq
    _, sat_s, last = served(sat)
    stats = srv.stats()
    # served results against solo solves of the same inputs
    worst = 0.0
    for n, k in last.items():
        rho, phi, pks = bufs[n]
        solo, spk, _, _ = plans[n].poisson(rho[k], nbins=nb)
        torch.cuda.synchronize()
        worst = max(worst, float(torch.linalg.vector_norm((phi[k] - solo).double())
                                 / torch.linalg.vector_norm(solo.double())),
                    float(torch.linalg.vector_norm(pks[k][0] - spk) / torch.linalg.vector_norm(spk)))
    _, sat_p = plain(sat)
    _, sat_q = plain(sat, sync_each=False)
    srv.close()
    p50s, p99s = lf2.latency_percentiles(lat_s)
    p50p, p99p = lf2.latency_percentiles(lat_p)
    mean_pts = float(np.mean([n ** 3 for n in req_n]))
    return {
        "workload": f"{nreq} Poisson + {nb}-bin P(k) requests, cubic N uniform over "
                    f"{{32,64,128,256,384}} (seed 6), Poisson arrivals {rate:.0f}/s, "
                    f"budget 8 GiB, 16 slots, 4 streams",
        "p50_ms": round(1e3 * p50s, 4), "p99_ms": round(1e3 * p99s, 4),
        "throughput_req_s": round(nreq / wall_s, 1),
        "saturation_req_s": round(nreq / sat_s, 1),
        "saturation_mpoints_s": round(nreq * mean_pts / sat_s / 1e6, 1),
        "plain_p50_ms": round(1e3 * p50p, 4), "plain_p99_ms": round(1e3 * p99p, 4),
        "plain_throughput_req_s": round(nreq / wall_p, 1),
        "plain_saturation_req_s": round(nreq / sat_p, 1),
        "plain_enqueue_only_saturation_req_s": round(nreq / sat_q, 1),
        "saturation_speedup_vs_plain": round(sat_p / sat_s, 3),
        "saturation_speedup_vs_plain_enqueue_only": round(sat_q / sat_s, 3),
        "served_vs_solo_rel_l2_max": worst,
        "peak_bytes_in_flight": stats["peak_bytes_in_flight"],
        "plan_misses": stats["plan_misses"],
    }


def bench_field_ops(args, torch, lf2):
    """The paper's field-operation benchmark (section 4.2) on one GPU: the
    periodic halo update and the first-order derivative of all components
    of a 512^3 3-component FP32 field with halo 1 into a 9-component field.
    Algorithmic bytes: the halo sites' words read and written once; the
    derivative reads the field once and writes the output once (16 bytes per
    site and component).  Input: torch N(0,1) on the device, seed 8."""
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(8)
    n, h, nc = 512, 1, 3
    p = n + 2 * h
    f = torch.randn((p, p, p, nc), generator=gen, device=dev, dtype=torch.float32)
    out = torch.zeros((p, p, p, 3 * nc), device=dev, dtype=torch.float32)
    sizes = (n, n, n)

    def timed(fn, reps):
        fn()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(5, args.steps)
    th = timed(lambda: lf2.update_halo(f, sizes, h), reps)
    tg = timed(lambda: lf2.gradient(f, sizes, h, out=out), reps)
    halo_sites = p ** 3 - n ** 3
    hb = 2.0 * halo_sites * nc * 4
    gb = 16.0 * nc * n ** 3
    del f, out
    torch.cuda.empty_cache()
    return {"workload": f"{n}^3 FP32 x {nc} components, halo {h}: halo update + forward "
                        "derivative of every component along x, y, z",
            "update_halo_ms": round(th, 4), "update_halo_gbps": round(hb / (th * 1e-3) / 1e9, 1),
            "gradient_ms": round(tg, 4), "gradient_gbps": round(gb / (tg * 1e-3) / 1e9, 1),
            "gradient_frac": round(gb / (tg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_paper_shapes(args, torch, lf2):
    """The paper's FFT benchmark shapes (section 4.1) on one GPU: 512^3 and
    1024^3 with 1, 2, 3 and 6 components, r2c forward / c2r backward and c2c
    forward / backward, plus 2048^3 with one component.  Absolute times and
    algorithmic HBM GB/s (one pass per axis) instead of the paper's parallel
    efficiency; the round trip backward(forward(x)) / N - x is the check (it
    holds at any size).  Inputs: torch N(0,1) on the device, seed 7."""
    import math
    from paper_1508_05610_amd import _lib
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    rows = []
    sizes = [int(v) for v in args.paper_sizes.split(",")]
    cases = [(n, nc) for n in (512, 1024) if n in sizes for nc in (1, 2, 3, 6)]
    cases += [(2048, 1)] if 2048 in sizes else []
    for n, nc in cases:
        for kind in (lf2.LF2_R2C, lf2.LF2_C2C):
            if n == 2048 and kind == lf2.LF2_C2C:
                continue
            N = n ** 3
            p = lf2.Plan((n, n, n), kind, ncomp=nc, autotune=True)
            comp = (nc,) if nc > 1 else ()
            if kind == lf2.LF2_R2C:
                x = torch.randn((n, n, n) + comp, generator=gen, device=dev, dtype=torch.float32)
                bpp = nc * (4.0 + 5 * 8.0 * (n // 2 + 1) / n)   # bytes per point, 3 passes
            else:
                x = torch.randn((n, n, n) + comp + (2,), generator=gen, device=dev,
                                dtype=torch.float32).view(torch.complex64).reshape((n, n, n) + comp)
                bpp = nc * 48.0
            F = p.forward(x)
            back = p.backward(F)
            torch.cuda.synchronize()
            err = float(torch.linalg.vector_norm((back / N - x).flatten()) /
                        torch.linalg.vector_norm(x.flatten()))

            def timed(fn, reps=3):
                fn()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                a.record()
                for _ in range(reps):
                    fn()
                b.record()
                torch.cuda.synchronize()
                return a.elapsed_time(b) / reps

            passes = {}
            for d, fn in (("fwd", lambda: p.forward(x, out=F)), ("bwd", lambda: p.backward(F, out=back))):
                fn()
                torch.cuda.synchronize()
                _lib.lf2_profile_reset()
                _lib.lf2_profile_enable(True)
                fn()
                torch.cuda.synchronize()
                passes[d] = {k: round(1e3 * ms / c, 1) for k, (c, ms, _) in _lib.profile_table().items()}
                _lib.lf2_profile_enable(False)
            tf = timed(lambda: p.forward(x, out=F))
            tb = timed(lambda: p.backward(F, out=back))
            for d, t in (("fwd", tf), ("bwd", tb)):
                gbs = bpp * N / (t * 1e-3) / 1e9
                rows.append({"n": n, "ncomp": nc, "kind": "r2c" if kind == lf2.LF2_R2C else "c2c",
                             "dir": d, "ms": round(t, 3), "gbps": round(gbs, 1),
                             "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "gflops": round(5.0 * N * math.log2(N) * nc / (t * 1e-3) / 1e9, 1),
                             "round_trip_rel_l2": err, "passes_us": passes[d],
                             "tuning": [p.tuning(1)[:2], p.tuning(2)[:2]]})
            print(f"paper shape {n}^3 x{nc} {'r2c' if kind == 0 else 'c2c'}: fwd {tf:.3f} ms "
                  f"bwd {tb:.3f} ms round trip {err:.2e}", file=sys.stderr, flush=True)
            p.close()
            del x, F, back
            torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--nbins", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-small-configs", action="store_true",
                    help="skip the 32^3 and 256^3 GRF workloads")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-field-ops", action="store_true")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="also time the paper's FFT benchmark shapes (512^3 and 1024^3 x 1/2/3/6 "
                         "components, 2048^3 x 1)")
    ap.add_argument("--paper-sizes", default="512,1024,2048",
                    help="lattice sizes of --paper-shapes to run (comma-separated)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--tuning", default=None,
                    help="fixed strided-pass tuning instead of autotuning, e.g. "
                         "'r2c:y=0/16,z=0/16;c2c3:y=1/16,z=1/64' (variant/chunk)")
    ap.add_argument("--only", default=None,
                    help="time one op alone (r2c_fwd, c2r_bwd, c2c_fwd_3comp, c2c_bwd_3comp, "
                         "poisson_pk, copy, field_ops) for profiler runs")
    ap.add_argument("--variants", type=int, default=0,
                    help="only time the tile settings of the strided and fused passes of an "
                         "N^3 lattice (one JSON line)")
    ap.add_argument("--lane-exchange", action="store_true",
                    help="only time the x pass of a 64x1024x1024 c2c lattice with its stage "
                         "exchange through LDS, ds_bpermute and DPP (one JSON line)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a single large lattice would shard as z-slabs with one all-to-all; "
              "not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1508_05610_amd as lf2
    from paper_1508_05610_amd import _lib

    lf2.load()
    dev = torch.device("cuda:0")
    if args.lane_exchange:
        print(json.dumps(bench_lane_exchange(args, torch, lf2, _lib)), flush=True)
        return
    if args.variants:
        print(json.dumps({"tile_variants": bench_tile_variants(args, torch, lf2, _lib)}), flush=True)
        return
    if args.only == "field_ops":
        print(json.dumps({"only": args.only, **bench_field_ops(args, torch, lf2)}), flush=True)
        return
    S = args.size
    n = (S, S, S)
    N = S ** 3
    flops_fft = 5.0 * N * math.log2(N)

    # ---- inputs (seeded, synthetic; resident before timing)
    f32 = synth.white_field(3, n)[..., 0]
    z3 = synth.white_field(4, n, ncomp=3, complex_values=True)
    x = torch.from_numpy(f32).to(dev)
    z = torch.from_numpy(z3).to(dev).view(torch.complex64).reshape(S, S, S, 3)
    del z3

    # plans autotuned at creation (tile variant and XCD chunk per strided
    # axis; untimed), or set from --tuning (profiler runs, where counters
    # distort the tuner's timings)
    fixed = parse_tuning(args.tuning) if args.tuning else None
    pr = lf2.Plan(n, lf2.LF2_R2C, autotune=fixed is None)
    pc = lf2.Plan(n, lf2.LF2_C2C, ncomp=3, autotune=fixed is None)
    if fixed:
        for nm, p_ in (("r2c", pr), ("c2c3", pc)):
            for ax, (v, c) in fixed.get(nm, {}).items():
                p_.set_tuning(ax, v, c)
    tuning = {nm: {f"axis{ax}": dict(zip(("variant", "chunk", "us_default", "us_tuned"),
                                         p_.tuning(ax)))
                   for ax in (1, 2)} for nm, p_ in (("r2c", pr), ("c2c3", pc))}
    F = torch.empty(pr.k_shape, dtype=torch.complex64, device=dev)
    back = torch.empty(pr.x_shape, dtype=torch.float32, device=dev)
    Z = torch.empty(pc.k_shape, dtype=torch.complex64, device=dev)
    zb = torch.empty(pc.x_shape, dtype=torch.complex64, device=dev)
    phi = torch.empty(pr.x_shape, dtype=torch.float32, device=dev)
    nb = args.nbins
    pk = torch.empty(nb, dtype=torch.float64, device=dev)
    km = torch.empty(nb, dtype=torch.float64, device=dev)
    ct = torch.empty(nb, dtype=torch.float64, device=dev)
    pv = torch.empty(2, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    def op_r2c():
        _lib.lf2_fft_execute(pr.handle, lf2.LF2_FORWARD, x.data_ptr(), F.data_ptr(), sh)

    def op_c2r():
        _lib.lf2_fft_execute(pr.handle, lf2.LF2_BACKWARD, F.data_ptr(), back.data_ptr(), sh)

    def op_c2c_f():
        _lib.lf2_fft_execute(pc.handle, lf2.LF2_FORWARD, z.data_ptr(), Z.data_ptr(), sh)

    def op_c2c_b():
        _lib.lf2_fft_execute(pc.handle, lf2.LF2_BACKWARD, Z.data_ptr(), zb.data_ptr(), sh)

    def op_poisson():
        _lib.lf2_poisson_solve(pr.handle, x.data_ptr(), phi.data_ptr(), 1.0, 0, nb, pk.data_ptr(),
                               km.data_ptr(), ct.data_ptr(), pv.data_ptr(), sh)

    ops = [("r2c_fwd", op_r2c, 1), ("c2r_bwd", op_c2r, 1), ("c2c_fwd_3comp", op_c2c_f, 3),
           ("c2c_bwd_3comp", op_c2c_b, 3), ("poisson_pk", op_poisson, 2)]
    n_transforms = sum(w for _, _, w in ops)

    if args.only:
        # one op alone, for profiler runs; "copy" is a plain 1 GiB device copy
        # whose counter readings calibrate the HBM byte counters
        if args.only == "copy":
            src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
            dst = torch.empty_like(src)
            fn = lambda: dst.copy_(src)  # noqa: E731
        else:
            fn = dict((nm, f) for nm, f, _ in ops)[args.only]
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        print(json.dumps({"only": args.only, "ms": a.elapsed_time(b) / args.steps,
                          "steps": args.steps}), flush=True)
        return

    def step():
        for _, fn, _ in ops:
            fn()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K steps, kernel timing on
    _lib.lf2_profile_enable(True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for _ in range(args.steps):
        step()
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = t_start.elapsed_time(t_end) / args.steps
    table = _lib.profile_table()
    _lib.lf2_profile_enable(False)

    # ---- per-op times (separate loop, events around each repetition):
    # median, p10 and p90 over >= 20 repetitions
    per_op, per_op_p10, per_op_p90 = {}, {}, {}
    reps = max(20, args.steps)
    for name, fn, _ in ops:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        t = np.array([a.elapsed_time(b) for a, b in evs])
        per_op[name] = float(np.median(t))
        per_op_p10[name] = float(np.percentile(t, 10))
        per_op_p90[name] = float(np.percentile(t, 90))

    step_bytes = sum(v[2] for v in table.values()) / args.steps
    # the dominant kernel: the record (kernel, pass and shape; one launch
    # configuration) with the most time in the step
    dname, (dn, dms, dbytes) = max(table.items(), key=lambda kv: kv[1][1])
    achieved = (dbytes / dn) / (dms / dn * 1e-3) / 1e9
    traffic = measured_traffic(dname, tuning_spec(tuning))
    kernels = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / v[0],
                   "alg_bytes_per_launch": v[2] / v[0],
                   "gbps": (v[2] / v[0]) / (v[1] / v[0] * 1e-3) / 1e9} for k, v in table.items()}

    value = n_transforms * flops_fft / (ms_step * 1e-3) / 1e9
    res = {
        "metric": "3D FFT GFLOP/s (5N*log2N) + HBM GB/s at 512^3 FP32",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"{S}^3 FP32 lattice: r2c fwd + c2r bwd (real N(0,1), seed 3), "
                        f"c2c fwd + bwd (complex64 3-comp AoS N(0,1), seed 4), "
                        f"Poisson with fused {nb}-bin P(k) + FP64 Parseval",
            "lattice": [S, S, S], "transforms_per_step": n_transforms,
        },
        "plan_tuning": tuning,
        "gbps_algorithmic": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "ops_ms": {k: round(v, 4) for k, v in per_op.items()},
        "ops_ms_p10": {k: round(v, 4) for k, v in per_op_p10.items()},
        "ops_ms_p90": {k: round(v, 4) for k, v in per_op_p90.items()},
        "ops_reps": reps,
        "roofline": {
            "bound": "hbm", "kernel": dname,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "avg_us": round(1e3 * dms / dn, 2),
            "alg_bytes_per_launch": dbytes / dn,
        },
        "kernels": kernels,
        "wall_s_timed": round(wall, 3),
    }
    # r2c forward / c2r backward: 3 passes, 4 + 5 * 8 Nh/N0 bytes per point
    # (x pass reads reals and writes the half spectrum, y and z read and
    # write it).
    r2c_ms = per_op["r2c_fwd"]
    nh = S // 2 + 1
    alg_r2c = 4.0 * N + 8.0 * nh * S * S + 2 * (2 * 8.0 * nh * S * S)
    res["r2c_fwd_gbps"] = round(alg_r2c / (r2c_ms * 1e-3) / 1e9, 1)
    res["r2c_fwd_roofline_frac"] = round(alg_r2c / (r2c_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    res["c2r_bwd_roofline_frac"] = round(alg_r2c / (per_op["c2r_bwd"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    copy_gbps = bench_copy(torch, np, stream)
    res["roofline"]["measured_copy_gbps"] = round(copy_gbps, 1)
    res["roofline"]["frac_of_copy"] = round(achieved / copy_gbps, 4)
    if not args.no_small_configs:
        res["small_configs"] = bench_small_configs(args, torch, np, lf2, stream)
    if not args.no_batch:
        res["batch"] = bench_batch(args, torch, np, lf2, stream)
    if not args.no_serve:
        res["serving"] = bench_serving(args, torch, np, lf2)
    if not args.no_field_ops:
        res["field_ops"] = bench_field_ops(args, torch, lf2)
    if args.paper_shapes:
        res["paper_shapes"] = bench_paper_shapes(args, torch, lf2)

    # ---- CPU baseline: the FP64 oracle on the host cores, bounded sample
    errors = {}
    if not args.no_cpu_baseline or not args.no_errors:
        import oracle
        f64 = f32.astype(np.float64)
        # one warm-up, then the median of three timed r2c + c2r pairs (one
        # pair only when the baseline is not asked for: errors need one)
        runs = []
        for rep in range(4 if not args.no_cpu_baseline else 1):
            t0 = time.perf_counter()
            Fo = oracle.r2c(f64)
            t1 = time.perf_counter()
            bo = oracle.c2r(Fo, S)
            t2 = time.perf_counter()
            if rep > 0 or args.no_cpu_baseline:
                runs.append((t2 - t0, t1 - t0, t2 - t1))
        runs.sort()
        cpu_s, t_r2c, t_c2r = runs[len(runs) // 2]
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = {
                "value": round(2 * flops_fft / cpu_s / 1e9, 3), "unit": "GFLOP/s",
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"one r2c forward + one c2r backward of the {S}^3 field "
                          f"(2 of the {n_transforms} transforms of a step), median of 3 after "
                          f"one warm-up: {t_r2c:.2f} s + {t_c2r:.2f} s",
            }
            # the same oracle on one thread, r2c forward of a quarter-size cube
            s1 = S // 2
            nthreads = oracle.num_threads()
            oracle.set_num_threads(1)
            t3 = time.perf_counter()
            oracle.r2c(f64[:s1, :s1, :s1].copy())
            t4 = time.perf_counter()
            oracle.set_num_threads(nthreads)
            n1_ = s1 ** 3
            res["cpu_baseline"]["single_thread"] = {
                "value": round(5.0 * n1_ * math.log2(n1_) / (t4 - t3) / 1e9, 3), "unit": "GFLOP/s",
                "cores": 1, "sample": f"one r2c forward of a {s1}^3 sub-cube: {t4 - t3:.2f} s",
            }
        if not args.no_errors:
            def rel_l2(a, b):
                return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

            def rel_max(a, b):
                return float(np.abs(a - b).max() / np.abs(b).max())

            op_r2c()
            op_c2r()
            op_poisson()
            op_c2c_f()
            torch.cuda.synchronize()
            Fg = F.cpu().numpy()
            errors["r2c_fwd"] = {"rel_l2": rel_l2(Fg, Fo), "max": rel_max(Fg, Fo)}
            bg = back.cpu().numpy()
            errors["c2r_bwd_chain"] = {"rel_l2": rel_l2(bg, bo), "max": rel_max(bg, bo)}
            opk, okm, oct_ = oracle.power_spectrum(Fo, n, nb)
            pkg = pk.cpu().numpy()
            errors["pk"] = {"rel_l2": rel_l2(pkg, opk), "max": rel_max(pkg, opk),
                            "counts_exact": bool(np.array_equal(ct.cpu().numpy(), oct_))}
            phio = oracle.poisson(f64)
            phig = phi.cpu().numpy()
            errors["poisson_phi"] = {"rel_l2": rel_l2(phig, phio), "max": rel_max(phig, phio)}
            pvg = pv.cpu().numpy()
            sumsq = float(np.sum(f64 * f64))
            errors["parseval"] = {"sum_f2_rel": abs(float(pvg[0]) - sumsq) / sumsq,
                                  "sum_wF2_over_N_rel": abs(float(pvg[1]) - sumsq) / sumsq}
            # c2c 3-comp: every mode of every component against the oracle's
            # c2c, forward of the input and backward of the GPU spectrum
            op_c2c_b()
            torch.cuda.synchronize()
            fw = {"rel_l2": 0.0, "max": 0.0}
            bw = {"rel_l2": 0.0, "max": 0.0}
            for c in range(3):
                zc = z[..., c].cpu().numpy().astype(np.complex128)
                Zc = Z[..., c].cpu().numpy()
                ref = oracle.c2c(zc, oracle.FORWARD)
                fw["rel_l2"] = max(fw["rel_l2"], rel_l2(Zc, ref))
                fw["max"] = max(fw["max"], rel_max(Zc, ref))
                del zc, ref
                ref = oracle.c2c(Zc.astype(np.complex128), oracle.BACKWARD)
                bc = zb[..., c].cpu().numpy()
                bw["rel_l2"] = max(bw["rel_l2"], rel_l2(bc, ref))
                bw["max"] = max(bw["max"], rel_max(bc, ref))
                del Zc, ref, bc
            errors["c2c_fwd_3comp"] = {**fw, "of": "worst component, whole field"}
            errors["c2c_bwd_3comp"] = {**bw, "of": "worst component, whole field (input: the GPU spectrum)"}
            errors["tolerance_rel_l2"] = 1e-5 * math.log2(N)
            res["errors"] = errors
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
