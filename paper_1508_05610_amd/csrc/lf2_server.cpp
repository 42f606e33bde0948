// lf2_server.cpp -- continuous-batching request loop for Poisson solves with
// power spectra on lattices of mixed sizes.
//
// submit() appends to a bounded FIFO.  The scheduler thread admits requests
// from the head while the in-flight footprint stays within the HBM budget
// and a slot is free, and launches each admitted request immediately on the
// next of K streams (its own pooled workspace, a resident plan), recording
// an event after its kernels.  The completion thread polls the in-flight
// events, timestamps finished requests, returns their workspace and budget
// and wakes the scheduler, so new arrivals join while earlier work is still
// running on the device.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "lf2_internal.hpp"
#include "lf2_plan.hpp"

using namespace lf2;
using namespace lf2::host;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

using LatKey = std::tuple<int64_t, int64_t, int64_t>;

struct Req {
    uint64_t ticket = 0;
    lf2_request r{};
    size_t bytes = 0;     // admission footprint
    size_t ws_bytes = 0;  // workspace part of it
    double t_arr = 0, t_adm = 0, t_done = 0, due = 0;
    lf2_status st = LF2_OK;
    bool done = false, has_plan = false;
    hipEvent_t ev = nullptr;
    char *ws = nullptr;
    LatKey key{};
};

// Workspace bytes of a Poisson solve (the same layout the solver uses).
size_t ws_bytes_of(const lf2_lattice &lat, int32_t nbins)
{
    lf2_plan_s tmp;
    tmp.kind = LF2_R2C;
    tmp.nc = 1;
    for (int i = 0; i < 3; ++i) tmp.n[i] = lat.size[i];
    tmp.nh = lat.size[0] / 2 + 1;
    tmp.nxk = tmp.nh;
    tmp.ntot = lat.size[0] * lat.size[1] * lat.size[2];
    tmp.len[0] = (int)(lat.size[0] / 2);
    tmp.len[1] = (int)lat.size[1];
    tmp.len[2] = (int)lat.size[2];
    return poisson_ws_bytes(&tmp, nbins, false);
}

size_t footprint_of(const lf2_request &r)
{
    const size_t n = (size_t)(r.lat.size[0] * r.lat.size[1] * r.lat.size[2]);
    return 8 * n + ws_bytes_of(r.lat, r.nbins);
}

lf2_status validate(const lf2_request *r)
{
    if (!r) return fail(LF2_ERR_INVALID_ARG, "request is NULL");
    const lf2_lattice &L = r->lat;
    if (L.dim != 3) return fail(LF2_ERR_UNSUPPORTED, "request lattice must be 3-d");
    if (L.halo != 0) return fail(LF2_ERR_UNSUPPORTED, "requests take dense lattices (halo 0)");
    for (int i = 0; i < 3; ++i)
        if (L.size[i] < 1) return fail(LF2_ERR_INVALID_ARG, "size[%d] < 1", i);
    if (L.size[0] % 2) return fail(LF2_ERR_UNSUPPORTED, "N0 must be even");
    if (!x_supported((int)(L.size[0] / 2), 1) || !s_supported((int)L.size[1]) ||
        !s_supported((int)L.size[2]))
        return fail(LF2_ERR_UNSUPPORTED, "lattice %lldx%lldx%lld has no kernels",
                    (long long)L.size[0], (long long)L.size[1], (long long)L.size[2]);
    lf2_status st;
    if ((st = check_ptr(r->rho, "rho", 4)) || (st = check_ptr(r->phi, "phi", 4))) return st;
    if ((const void *)r->rho == (const void *)r->phi)
        return fail(LF2_ERR_INVALID_ARG, "rho and phi must not alias");
    if (!(r->dx > 0.0) || !std::isfinite(r->dx)) return fail(LF2_ERR_INVALID_ARG, "dx must be > 0");
    if (r->flags & ~(uint32_t)(LF2_POISSON_DISCRETE_K2 | LF2_PK_OF_PHI))
        return fail(LF2_ERR_INVALID_ARG, "unknown Poisson flags 0x%x", r->flags);
    if (r->nbins < 0 || r->nbins > kMaxBins)
        return fail(LF2_ERR_UNSUPPORTED, "nbins %d outside [0, %d]", r->nbins, kMaxBins);
    return LF2_OK;
}

struct PlanEntry {
    lf2_plan plan = nullptr;
    int refs = 0;
    uint64_t last_use = 0;
};

}  // namespace

struct lf2_server_s {
    bool fake = false;
    uint32_t delay_us = 0;
    uint64_t fail_ticket = 0;
    int device = 0;
    size_t budget = 0;
    int max_slots = 1, nstreams = 1, max_queue = 1;
    std::vector<hipStream_t> streams;
    std::atomic<unsigned> rr{0};

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_compl;
    std::deque<Req *> queue;
    std::vector<Req *> inflight;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next_ticket = 1;
    size_t bytes_inflight = 0, peak = 0;
    int launching = 0;  // admitted, not yet in flight
    int64_t n_sub = 0, n_done = 0, n_fail = 0, n_busy = 0, n_budget = 0;
    bool draining = false, stop = false;

    // scheduler-thread state (plans, workspaces, events)
    std::mutex pmu;
    std::map<LatKey, PlanEntry> plans;
    uint64_t use_clock = 0;
    int64_t plan_hits = 0, plan_misses = 0;
    std::multimap<size_t, char *> ws_free;
    std::vector<char *> ws_all;
    std::vector<hipEvent_t> ev_free, ev_all;

    std::thread sched, compl_;
};

namespace {

constexpr size_t kMaxPlans = 32;  // resident plans; the least recently used idle one goes

lf2_status get_plan(lf2_server s, const LatKey &key, const lf2_lattice &lat, lf2_plan *out)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    auto it = s->plans.find(key);
    if (it == s->plans.end()) {
        if (s->plans.size() >= kMaxPlans) {
            // evict the least recently used idle plan
            auto victim = s->plans.end();
            for (auto j = s->plans.begin(); j != s->plans.end(); ++j)
                if (j->second.refs == 0 &&
                    (victim == s->plans.end() || j->second.last_use < victim->second.last_use))
                    victim = j;
            if (victim != s->plans.end()) {
                if (victim->second.plan) lf2_plan_destroy(victim->second.plan);
                s->plans.erase(victim);
            }
        }
        PlanEntry e;
        if (!s->fake) {  // the fake executor keeps cache entries without plans
            lf2_status st = lf2_fft_plan(&e.plan, &lat, 1, LF2_R2C, 0);
            if (st) return st;
        }
        it = s->plans.emplace(key, e).first;
        s->plan_misses += 1;
    } else {
        s->plan_hits += 1;
    }
    it->second.refs += 1;
    it->second.last_use = ++s->use_clock;
    *out = it->second.plan;
    return LF2_OK;
}

void put_plan(lf2_server s, const LatKey &key)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    auto it = s->plans.find(key);
    if (it != s->plans.end() && it->second.refs > 0) it->second.refs -= 1;
}

char *ws_get(lf2_server s, size_t bytes)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    auto it = s->ws_free.lower_bound(bytes);
    if (it != s->ws_free.end() && it->first <= 2 * bytes) {
        char *p = it->second;
        s->ws_free.erase(it);
        return p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    s->ws_all.push_back((char *)p);
    return (char *)p;
}

void ws_put(lf2_server s, char *p, size_t bytes)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(s->pmu);
    s->ws_free.emplace(bytes, p);
}

hipEvent_t ev_get(lf2_server s)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    if (!s->ev_free.empty()) {
        hipEvent_t e = s->ev_free.back();
        s->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    s->ev_all.push_back(e);
    return e;
}

void ev_put(lf2_server s, hipEvent_t e)
{
    if (!e) return;
    std::lock_guard<std::mutex> lk(s->pmu);
    s->ev_free.push_back(e);
}

// Launch one admitted request (no server lock held; the scheduler thread or
// a submitting thread).  On failure nothing of the request is left running
// on the device.
void launch(lf2_server s, Req *q)
{
    lf2_plan plan = nullptr;
    lf2_status st = get_plan(s, q->key, q->r.lat, &plan);
    if (st) {
        q->st = st;
        return;
    }
    q->has_plan = true;
    if (s->fake) {
        q->st = (q->ticket == s->fail_ticket) ? LF2_ERR_DEVICE : LF2_OK;
        return;
    }
    q->ws = ws_get(s, q->ws_bytes);
    q->ev = ev_get(s);
    if (!q->ws || !q->ev) {
        q->st = LF2_ERR_OUT_OF_MEMORY;
        return;
    }
    hipStream_t strm = s->streams[s->rr.fetch_add(1) % (unsigned)s->nstreams];
    {
        // Tables a plan builds on first use are written on this stream;
        // later requests may run on other streams, so wait for them once.
        std::lock_guard<std::mutex> lk(s->pmu);
        const size_t nk = plan->k2.size(), ns = plan->shells.size();
        const double *k2[3];
        ShellEntry sh{};
        st = get_k2(plan, q->r.dx, (q->r.flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0, strm, k2);
        if (st == LF2_OK && q->r.nbins > 0) st = get_shell(plan, q->r.nbins, strm, &sh);
        if (st == LF2_OK && (plan->k2.size() != nk || plan->shells.size() != ns) &&
            hipStreamSynchronize(strm) != hipSuccess)
            st = LF2_ERR_DEVICE;
        if (st == LF2_OK)
            st = poisson_impl(plan, q->r.rho, q->r.phi, q->r.dx, q->r.flags, q->r.nbins,
                              q->r.d_pk, q->r.d_kmean, q->r.d_count, nullptr, strm, q->ws,
                              q->ws_bytes);
    }
    if (st == LF2_OK && hipEventRecord(q->ev, strm) != hipSuccess) st = LF2_ERR_DEVICE;
    if (st != LF2_OK) (void)hipStreamSynchronize(strm);
    q->st = st;
}

// Return a finished request's resources (completion thread).
void release(lf2_server s, Req *q)
{
    if (!s->fake) {
        ws_put(s, q->ws, q->ws_bytes);
        ev_put(s, q->ev);
    }
    if (q->has_plan) put_plan(s, q->key);
    q->ws = nullptr;
    q->ev = nullptr;
}

// Admit from the head of the queue while a slot and budget are free (FIFO:
// a request that does not fit holds back the ones behind it).  Server lock
// held.
void admit_locked(lf2_server s, std::vector<Req *> &adm)
{
    while (!s->queue.empty()) {
        Req *q = s->queue.front();
        if ((int)s->inflight.size() + s->launching >= s->max_slots) break;
        if (s->bytes_inflight + q->bytes > s->budget) break;
        s->queue.pop_front();
        s->bytes_inflight += q->bytes;
        s->peak = std::max(s->peak, s->bytes_inflight);
        s->launching += 1;
        q->t_adm = now_s();
        adm.push_back(q);
    }
}

// Launch admitted requests and hand them to the completion thread; called
// and returns with the server lock held.
void launch_admitted(lf2_server s, std::unique_lock<std::mutex> &lk, std::vector<Req *> &adm)
{
    if (adm.empty()) return;
    lk.unlock();
    int prev = -1;
    if (!s->fake && hipGetDevice(&prev) == hipSuccess && prev != s->device)
        (void)hipSetDevice(s->device);  // a submitting thread may have another device current
    for (Req *q : adm) {
        launch(s, q);
        if (s->fake) q->due = q->t_adm + 1e-6 * s->delay_us;
    }
    if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
    lk.lock();
    s->launching -= (int)adm.size();
    for (Req *q : adm) s->inflight.push_back(q);
    s->cv_compl.notify_one();
}

void scheduler_main(lf2_server s)
{
    if (!s->fake) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_sched.wait(lk, [&] {
            if (s->stop) return true;
            if (s->queue.empty()) return false;
            return (int)s->inflight.size() + s->launching < s->max_slots &&
                   s->bytes_inflight + s->queue.front()->bytes <= s->budget;
        });
        if (s->stop) break;
        std::vector<Req *> adm;
        admit_locked(s, adm);
        launch_admitted(s, lk, adm);
    }
}

void completion_main(lf2_server s)
{
    if (!s->fake) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_compl.wait_for(lk, std::chrono::milliseconds(2),
                             [&] { return s->stop || !s->inflight.empty(); });
        if (s->stop && s->inflight.empty()) break;
        if (s->inflight.empty()) continue;
        std::vector<Req *> cur = s->inflight;
        lk.unlock();
        std::vector<Req *> fin;
        const double t = now_s();
        for (Req *q : cur) {
            if (q->st != LF2_OK) {  // failed at launch, nothing pending
                fin.push_back(q);
                continue;
            }
            if (s->fake) {
                if (t >= q->due) fin.push_back(q);
                continue;
            }
            hipError_t e = hipEventQuery(q->ev);
            if (e == hipSuccess) {
                fin.push_back(q);
            } else if (e != hipErrorNotReady) {
                q->st = LF2_ERR_DEVICE;
                fin.push_back(q);
            }
        }
        const double tdone = now_s();
        for (Req *q : fin) release(s, q);
        lk.lock();
        if (fin.empty()) {
            // requests in flight: poll again at once (yield the core to
            // other runnable threads); the fake executor's delays are long
            lk.unlock();
            if (s->fake)
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            else
                std::this_thread::yield();
            lk.lock();
            continue;
        }
        for (Req *q : fin) {
            s->inflight.erase(std::find(s->inflight.begin(), s->inflight.end(), q));
            s->bytes_inflight -= q->bytes;
            q->t_done = tdone;
            q->done = true;
            if (q->st == LF2_OK)
                s->n_done += 1;
            else
                s->n_fail += 1;
        }
        s->cv_done.notify_all();
        s->cv_sched.notify_one();
    }
}

lf2_status server_start(lf2_server s)
{
    try {
        s->sched = std::thread(scheduler_main, s);
        s->compl_ = std::thread(completion_main, s);
    } catch (...) {
        return fail(LF2_ERR_OUT_OF_MEMORY, "server threads could not start");
    }
    return LF2_OK;
}

}  // namespace

extern "C" {

double lf2_server_now(void) { return now_s(); }

lf2_status lf2_server_create(lf2_server *out, size_t hbm_budget_bytes, int32_t max_slots,
                             int32_t nstreams, int32_t max_queue)
{
    if (!out) return fail(LF2_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_slots < 1 || nstreams < 1 || max_queue < 1)
        return fail(LF2_ERR_INVALID_ARG, "budget, slots, streams and queue must be positive");
    lf2_server s = new (std::nothrow) lf2_server_s();
    if (!s) return fail(LF2_ERR_OUT_OF_MEMORY, "server allocation");
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->nstreams = nstreams;
    s->max_queue = max_queue;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(LF2_ERR_DEVICE, "hipGetDevice");
    }
    for (int i = 0; i < nstreams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return fail(LF2_ERR_DEVICE, "stream creation");
        }
        s->streams.push_back(st);
    }
    lf2_status st = server_start(s);
    if (st) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        delete s;
        return st;
    }
    *out = s;
    return LF2_OK;
}

lf2_status lf2_server_create_fake(lf2_server *out, size_t hbm_budget_bytes, int32_t max_slots,
                                  int32_t max_queue, uint32_t delay_us, uint64_t fail_ticket)
{
    if (!out) return fail(LF2_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0 || max_slots < 1 || max_queue < 1)
        return fail(LF2_ERR_INVALID_ARG, "budget, slots and queue must be positive");
    lf2_server s = new (std::nothrow) lf2_server_s();
    if (!s) return fail(LF2_ERR_OUT_OF_MEMORY, "server allocation");
    s->fake = true;
    s->delay_us = delay_us;
    s->fail_ticket = fail_ticket;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->max_queue = max_queue;
    lf2_status st = server_start(s);
    if (st) {
        delete s;
        return st;
    }
    *out = s;
    return LF2_OK;
}

lf2_status lf2_server_prepare(lf2_server s, int32_t n, const lf2_lattice *lats, int32_t nbins,
                              double dx, uint32_t flags)
{
    if (!s || (n > 0 && !lats)) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    if (s->fake) return LF2_OK;
    if (!(dx > 0.0)) return fail(LF2_ERR_INVALID_ARG, "dx must be > 0");
    for (int i = 0; i < n; ++i) {
        const lf2_lattice &L = lats[i];
        const LatKey key{L.size[0], L.size[1], L.size[2]};
        lf2_plan p = nullptr;
        lf2_status st = get_plan(s, key, L, &p);
        if (st) return st;
        const double *k2[3];
        {
            std::lock_guard<std::mutex> lk(s->pmu);
            st = get_k2(p, dx, (flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0, nullptr, k2);
            ShellEntry sh{};
            if (st == LF2_OK && nbins > 0) st = get_shell(p, nbins, nullptr, &sh);
        }
        put_plan(s, key);
        if (st) return st;
        // one workspace of this size in the pool
        lf2_request r{};
        r.lat = L;
        r.nbins = nbins;
        const size_t wb = ws_bytes_of(L, nbins);
        char *w = ws_get(s, wb);
        if (!w) return fail(LF2_ERR_OUT_OF_MEMORY, "workspace");
        ws_put(s, w, wb);
    }
    LF2_HIP(hipDeviceSynchronize());
    return LF2_OK;
}

lf2_status lf2_server_footprint(const lf2_request *r, size_t *bytes)
{
    if (!r || !bytes) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    if (r->lat.dim != 3) return fail(LF2_ERR_UNSUPPORTED, "request lattice must be 3-d");
    for (int i = 0; i < 3; ++i)
        if (r->lat.size[i] < 1) return fail(LF2_ERR_INVALID_ARG, "size[%d] < 1", i);
    *bytes = footprint_of(*r);
    return LF2_OK;
}

lf2_status lf2_server_submit(lf2_server s, const lf2_request *r, uint64_t *ticket)
{
    if (!s || !ticket) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    lf2_status st = validate(r);
    if (st) return st;
    Req *q = new (std::nothrow) Req();
    if (!q) return fail(LF2_ERR_OUT_OF_MEMORY, "request allocation");
    q->r = *r;
    q->bytes = footprint_of(*r);
    q->ws_bytes = ws_bytes_of(r->lat, r->nbins);
    q->key = LatKey{r->lat.size[0], r->lat.size[1], r->lat.size[2]};
    q->t_arr = r->t_arrival > 0 ? r->t_arrival : now_s();
    std::unique_lock<std::mutex> lk(s->mu);
    if (q->bytes > s->budget) {
        s->n_budget += 1;
        const size_t b = q->bytes;
        delete q;
        return fail(LF2_ERR_BUDGET, "request footprint %zu bytes exceeds the budget %zu", b,
                    s->budget);
    }
    if (s->draining || (int)s->queue.size() >= s->max_queue) {
        s->n_busy += 1;
        delete q;
        return fail(LF2_ERR_BUSY, "request queue is full");
    }
    q->ticket = s->next_ticket++;
    s->reqs[q->ticket] = q;
    s->queue.push_back(q);
    s->n_sub += 1;
    *ticket = q->ticket;
    if (s->queue.size() == 1) {
        // nothing waits ahead of it: admit and launch on this thread, which
        // saves the hand-off to the scheduler thread
        std::vector<Req *> adm;
        admit_locked(s, adm);
        launch_admitted(s, lk, adm);
    }
    if (!s->queue.empty()) s->cv_sched.notify_one();
    return LF2_OK;
}

lf2_status lf2_server_poll(lf2_server s, uint64_t ticket, lf2_result *res, int32_t wait)
{
    if (!s || !res) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(LF2_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    Req *q = it->second;
    if (!q->done) {
        if (!wait) return LF2_ERR_NOT_READY;
        s->cv_done.wait(lk, [&] { return q->done; });
    }
    res->status = q->st;
    res->t_arrival = q->t_arr;
    res->t_admit = q->t_adm;
    res->t_done = q->t_done;
    s->reqs.erase(q->ticket);
    delete q;
    return LF2_OK;
}

lf2_status lf2_server_get_stats(lf2_server s, lf2_server_stats *st)
{
    if (!s || !st) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->n_sub;
    st->completed = s->n_done;
    st->failed = s->n_fail;
    st->rejected_busy = s->n_busy;
    st->rejected_budget = s->n_budget;
    st->in_flight = (int64_t)s->inflight.size();
    st->queued = (int64_t)s->queue.size();
    st->bytes_in_flight = s->bytes_inflight;
    st->peak_bytes_in_flight = s->peak;
    {
        std::lock_guard<std::mutex> pk(s->pmu);
        st->plans_cached = (int64_t)s->plans.size();
        st->plan_hits = s->plan_hits;
        st->plan_misses = s->plan_misses;
    }
    return LF2_OK;
}

lf2_status lf2_server_destroy(lf2_server s)
{
    if (!s) return fail(LF2_ERR_INVALID_ARG, "server is NULL");
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->draining = true;
        s->cv_done.wait(lk, [&] {
            return s->queue.empty() && s->inflight.empty() && s->launching == 0;
        });
        s->stop = true;
    }
    s->cv_sched.notify_all();
    s->cv_compl.notify_all();
    if (s->sched.joinable()) s->sched.join();
    if (s->compl_.joinable()) s->compl_.join();
    for (auto &kv : s->reqs) delete kv.second;
    if (!s->fake) {
        for (hipStream_t x : s->streams) (void)hipStreamSynchronize(x);
        for (auto &kv : s->plans)
            if (kv.second.plan) lf2_plan_destroy(kv.second.plan);
        for (char *p : s->ws_all) (void)hipFree(p);
        for (hipEvent_t e : s->ev_all) (void)hipEventDestroy(e);
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    }
    delete s;
    return LF2_OK;
}

}  // extern "C"
