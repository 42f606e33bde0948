// lf2_server.cpp -- continuous-batching request loop for Poisson solves with
// power spectra on lattices of mixed sizes.
//
// submit() appends to a bounded FIFO.  The scheduler thread admits requests
// from the head while the in-flight footprint plus the idle pooled
// workspace stays within the HBM budget and a slot is free (idle workspace
// is freed to make room when needed).  Requests admitted together that
// share a lattice, lattice spacing, k^2 kind and bin count run as one
// grouped solve -- one launch per pass over all of them plus one finalize
// -- and the others one by one; each unit goes on the next of K streams
// with its own pooled workspaces and a resident plan, and an event is
// recorded after its kernels.  The completion thread polls the in-flight
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

// Resources of a grouped solve, shared by its requests: the completion
// event and the staging of its descriptors; the last request to finish
// returns them.
struct Group {
    hipEvent_t ev = nullptr;
    char *stage_host = nullptr, *stage_dev = nullptr;
    size_t stage_bytes = 0;
    int refs = 0;
};

constexpr int kMaxGroup = 16;  // requests in one grouped solve
// Grouped solves pay where launches and tails dominate (small lattices); a
// lattice above kGroupFieldPoints runs alone on the tuned per-lattice path,
// which is faster there, and a group holds at most kGroupPoints lattice
// points, so that its requests do not wait long for each other.
constexpr int64_t kGroupFieldPoints = (int64_t)1 << 24;  // 256^3
constexpr int64_t kGroupPoints = (int64_t)1 << 26;

struct Req {
    uint64_t ticket = 0;
    lf2_request r{};
    size_t bytes = 0;     // admission footprint (nominal workspace)
    size_t charge = 0;    // what it holds of the budget once its workspace is taken
    size_t ws_bytes = 0;  // nominal workspace part of the footprint
    size_t ws_real = 0;   // size of the workspace buffer it got
    double t_arr = 0, t_adm = 0, t_done = 0, due = 0;
    lf2_status st = LF2_OK;
    bool done = false, has_plan = false;
    hipEvent_t ev = nullptr;
    Group *grp = nullptr;
    char *ws = nullptr;
    LatKey key{};
};

// Workspace bytes of a request: enough for a solve alone (the layout the
// solver uses) and for a grouped solve (bin rows per z tile).
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
    const size_t solo = poisson_ws_bytes(&tmp, nbins, false);
    const size_t grouped = group_supported(&tmp) ? group_ws_bytes(&tmp, nbins) : 0;
    return solo > grouped ? solo : grouped;
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

// Requests that may run as one grouped solve.
using GroupKey = std::tuple<int64_t, int64_t, int64_t, double, uint32_t, int32_t>;
GroupKey group_key(const Req *q)
{
    return GroupKey{q->r.lat.size[0], q->r.lat.size[1], q->r.lat.size[2], q->r.dx, q->r.flags,
                    q->r.nbins};
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
    int launching = 0;  // requests admitted, not yet in flight
    int units_busy = 0; // launch units (a request, or a group) admitted and not finished
    int64_t n_sub = 0, n_done = 0, n_fail = 0, n_busy = 0, n_budget = 0;
    bool draining = false, stop = false;

    // scheduler-thread state (plans, workspaces, events)
    std::mutex pmu;
    std::map<LatKey, PlanEntry> plans;
    uint64_t use_clock = 0;
    int64_t plan_hits = 0, plan_misses = 0;
    // workspace pool: idle buffers by their real size; the idle bytes count
    // against the budget (pool lock; admission reads ws_idle holding both locks)
    std::multimap<size_t, char *> ws_free;
    std::map<char *, size_t> ws_size;
    size_t ws_idle = 0;
    // workspaces come from a memory pool of the server's own, allocated and
    // freed in stream order, so that freeing an idle buffer does not wait
    // for the whole device (hipFree would); plain hipMalloc where the device
    // has no memory pools
    hipMemPool_t mpool = nullptr;
    int64_t n_ws_alloc = 0, n_ws_free = 0;
    size_t peak_use = 0;  // largest in-flight + idle bytes seen
    std::vector<hipEvent_t> ev_free, ev_all;
    std::multimap<size_t, std::pair<char *, char *>> stage_free;  // pinned host, device
    std::vector<std::pair<char *, char *>> stage_all;
    int64_t n_groups = 0, n_grouped = 0;

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

// A new workspace buffer, allocated in order on the stream that will use it.
char *ws_alloc(lf2_server s, size_t bytes, hipStream_t strm)
{
    s->n_ws_alloc += 1;
    if (s->fake) return (char *)malloc(1);  // a token: the fake executor runs no kernels
    void *p = nullptr;
    const hipError_t e = s->mpool ? hipMallocFromPoolAsync(&p, bytes, s->mpool, strm)
                                  : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return (char *)p;
}

// Free an idle buffer (its last use has completed).
void ws_release(lf2_server s, char *p)
{
    s->n_ws_free += 1;
    if (s->fake)
        free(p);
    else if (s->mpool)
        (void)hipFreeAsync(p, s->streams[0]);
    else
        (void)hipFree(p);
}

// Free idle buffers, those that would not serve a `keep`-byte request
// first, until `need` more bytes fit the budget next to `inflight` (pool
// lock held by the caller; `mu` too).
void ws_trim_locked(lf2_server s, size_t inflight, size_t need, size_t keep)
{
    for (int pass = 0; pass < 2; ++pass) {
        for (auto it = s->ws_free.begin(); it != s->ws_free.end();) {
            if (inflight + s->ws_idle + need <= s->budget) return;
            const bool fits = it->first >= keep && it->first <= 2 * keep;
            if (pass == 0 && fits) {
                ++it;
                continue;
            }
            ws_release(s, it->second);
            s->ws_idle -= it->first;
            s->ws_size.erase(it->second);
            it = s->ws_free.erase(it);
        }
    }
}

// A workspace of at least `bytes`: an idle buffer of at most twice that
// size, else a new one (after freeing idle buffers that do not fit, if the
// allocation fails).  *real: its size.
char *ws_get(lf2_server s, size_t bytes, size_t *real, hipStream_t strm)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    auto it = s->ws_free.lower_bound(bytes);
    if (it != s->ws_free.end() && it->first <= 2 * bytes) {
        char *p = it->second;
        *real = it->first;
        s->ws_idle -= it->first;
        s->ws_free.erase(it);
        return p;
    }
    char *p = ws_alloc(s, bytes, strm);
    if (!p) {
        for (auto &kv : s->ws_free) {
            ws_release(s, kv.second);
            s->ws_size.erase(kv.second);
        }
        s->ws_free.clear();
        s->ws_idle = 0;
        p = ws_alloc(s, bytes, strm);
        if (!p) return nullptr;
    }
    s->ws_size[p] = bytes;
    *real = bytes;
    return p;
}

void ws_put(lf2_server s, char *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(s->pmu);
    auto it = s->ws_size.find(p);
    const size_t real = it == s->ws_size.end() ? 0 : it->second;
    s->ws_free.emplace(real, p);
    s->ws_idle += real;
}

// Staging for a grouped solve's descriptors: pinned host and device memory
// of at least `bytes`, pooled.
bool stage_get(lf2_server s, size_t bytes, Group *g)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    auto it = s->stage_free.lower_bound(bytes);
    if (it != s->stage_free.end()) {
        g->stage_host = it->second.first;
        g->stage_dev = it->second.second;
        g->stage_bytes = it->first;
        s->stage_free.erase(it);
        return true;
    }
    const size_t b = bytes < 4096 ? 4096 : bytes;
    void *h = nullptr, *d = nullptr;
    if (hipHostMalloc(&h, b, 0) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (hipMalloc(&d, b) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return false;
    }
    s->stage_all.emplace_back((char *)h, (char *)d);
    g->stage_host = (char *)h;
    g->stage_dev = (char *)d;
    g->stage_bytes = b;
    return true;
}

void stage_put(lf2_server s, Group *g)
{
    if (!g->stage_host) return;
    std::lock_guard<std::mutex> lk(s->pmu);
    s->stage_free.emplace(g->stage_bytes, std::make_pair(g->stage_host, g->stage_dev));
    g->stage_host = g->stage_dev = nullptr;
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

// The plan's tables for a request, made on first use on stream `strm` (and
// waited for once, since later requests may run on other streams); the plan
// lists are only touched under the pool lock, which is not held while
// kernels are enqueued.
lf2_status request_tables(lf2_server s, lf2_plan plan, const lf2_request &r, hipStream_t strm,
                          PoissonTables *t)
{
    std::lock_guard<std::mutex> lk(s->pmu);
    const size_t nk = plan->k2.size(), ns = plan->shells.size();
    lf2_status st = get_k2(plan, r.dx, (r.flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0, strm, t->k2);
    t->sh = ShellEntry{};
    if (st == LF2_OK && r.nbins > 0) st = get_shell(plan, r.nbins, strm, &t->sh);
    if (st == LF2_OK && (plan->k2.size() != nk || plan->shells.size() != ns) &&
        hipStreamSynchronize(strm) != hipSuccess)
        st = fail(LF2_ERR_DEVICE, "plan tables");
    return st;
}

// Take the request's workspace and settle its budget charge (server lock
// not held).
bool take_ws(lf2_server s, Req *q, hipStream_t strm)
{
    if (q->ws) return true;  // an idle buffer reserved at admission
    size_t real = 0;
    q->ws = ws_get(s, q->ws_bytes, &real, strm);
    if (!q->ws) return false;
    q->ws_real = real;
    std::lock_guard<std::mutex> lk(s->mu);
    // an idle buffer larger than asked moves from the pool to the request:
    // in-flight plus idle bytes do not grow by more than the admission check
    q->charge = q->bytes - q->ws_bytes + real;
    s->bytes_inflight += q->charge - q->bytes;
    return true;
}

// Launch admitted requests that form one unit: a single request, or a
// group sharing lattice, dx, k^2 kind and bin count (no server lock held;
// the scheduler thread or a submitting thread).  On failure nothing of the
// unit is left running on the device and every request of it carries the
// error.
void launch_unit(lf2_server s, std::vector<Req *> &unit)
{
    Req *q0 = unit[0];
    lf2_plan plan = nullptr;
    lf2_status st = get_plan(s, q0->key, q0->r.lat, &plan);
    if (st) {
        for (Req *q : unit) q->st = st;
        return;
    }
    q0->has_plan = true;
    for (size_t i = 1; i < unit.size(); ++i) {
        lf2_plan p2 = nullptr;
        st = get_plan(s, unit[i]->key, unit[i]->r.lat, &p2);  // a reference per request
        if (st) break;
        unit[i]->has_plan = true;
    }
    if (s->fake) {
        for (Req *q : unit) {
            if (st == LF2_OK && !take_ws(s, q, nullptr)) st = LF2_ERR_OUT_OF_MEMORY;
            q->st = st ? st : (q->ticket == s->fail_ticket ? LF2_ERR_DEVICE : LF2_OK);
        }
        if (unit.size() > 1) {
            Group *g = new Group();
            g->refs = (int)unit.size();
            for (Req *q : unit) q->grp = g;
            std::lock_guard<std::mutex> lk(s->mu);
            s->n_groups += 1;
            s->n_grouped += (int64_t)unit.size();
        }
        return;
    }
    hipStream_t strm = s->streams[s->rr.fetch_add(1) % (unsigned)s->nstreams];
    for (Req *q : unit)
        if (st == LF2_OK && !take_ws(s, q, strm)) st = fail(LF2_ERR_OUT_OF_MEMORY, "workspace");
    PoissonTables tabs{};
    if (st == LF2_OK) st = request_tables(s, plan, q0->r, strm, &tabs);
    const int R = (int)unit.size();
    Group *g = nullptr;
    if (st == LF2_OK && R > 1) {
        g = new (std::nothrow) Group();
        if (!g || !stage_get(s, group_stage_bytes(plan, R), g)) {
            st = fail(LF2_ERR_OUT_OF_MEMORY, "group staging");
        } else {
            std::vector<GroupReq> gr(R);
            for (int i = 0; i < R; ++i)
                gr[i] = GroupReq{unit[i]->r.rho, unit[i]->r.phi, unit[i]->r.d_pk,
                                 unit[i]->r.d_kmean, unit[i]->r.d_count, unit[i]->ws};
            st = group_enqueue(plan, R, gr.data(), q0->r.dx, q0->r.flags, q0->r.nbins, tabs,
                               g->stage_host, g->stage_dev, g->stage_bytes, strm);
        }
    } else if (st == LF2_OK) {
        st = poisson_impl(plan, q0->r.rho, q0->r.phi, q0->r.dx, q0->r.flags, q0->r.nbins,
                          q0->r.d_pk, q0->r.d_kmean, q0->r.d_count, nullptr, strm, q0->ws,
                          q0->ws_real, false, &tabs);
    }
    hipEvent_t ev = st == LF2_OK ? ev_get(s) : nullptr;
    if (st == LF2_OK && (!ev || hipEventRecord(ev, strm) != hipSuccess)) st = LF2_ERR_DEVICE;
    if (st != LF2_OK) {
        (void)hipStreamSynchronize(strm);
        if (ev) ev_put(s, ev);
        ev = nullptr;
        if (g) {
            stage_put(s, g);
            delete g;
            g = nullptr;
        }
    }
    if (g) {
        g->ev = ev;
        g->refs = R;
        std::lock_guard<std::mutex> lk(s->mu);
        s->n_groups += 1;
        s->n_grouped += R;
    }
    for (Req *q : unit) {
        q->st = st;
        q->ev = ev;
        q->grp = g;
    }
}

// Return a finished request's resources but its workspace (completion
// thread, server lock not held).  True when this was the last request of
// its launch unit.  The workspace goes back to the pool under the server
// lock, in the same step that takes the request's charge off the in-flight
// bytes, so that no one sees it both idle and in flight.
bool release(lf2_server s, Req *q)
{
    bool unit_done = true;
    if (q->grp) {
        Group *g = q->grp;
        if (--g->refs == 0) {  // the completion thread is the only one touching refs here
            if (g->ev) ev_put(s, g->ev);
            stage_put(s, g);
            delete g;
        } else {
            unit_done = false;
        }
    } else if (!s->fake && q->ev) {
        ev_put(s, q->ev);
    }
    if (q->has_plan) put_plan(s, q->key);
    q->ev = nullptr;
    q->grp = nullptr;
    return unit_done;
}

int64_t points_of(const Req *q)
{
    return q->r.lat.size[0] * q->r.lat.size[1] * q->r.lat.size[2];
}

// Whether requests of this key can run as one grouped solve.
bool groupable(const Req *q)
{
    if (points_of(q) > kGroupFieldPoints) return false;
    lf2_plan_s tmp;
    tmp.kind = LF2_R2C;
    tmp.nc = 1;
    tmp.len[0] = (int)(q->r.lat.size[0] / 2);
    tmp.len[1] = (int)q->r.lat.size[1];
    tmp.len[2] = (int)q->r.lat.size[2];
    return group_supported(&tmp) && q->r.nbins <= kBatchMaxBins;
}

// Budget check of one request; charges it when it fits.  An idle buffer
// that fits its workspace (at most twice the size) is reserved for it at
// once: it moves from the pool to the request, so the bytes in use grow by
// the request's rho and phi only (other idle buffers are freed if that makes
// room).  Otherwise the request needs a new workspace, and idle buffers are
// freed to make room for it.  Whenever the in-flight bytes leave room for
// the request's footprint, one of the two succeeds.  Server lock held.
bool fits_budget_locked(lf2_server s, Req *q)
{
    std::lock_guard<std::mutex> pk(s->pmu);
    const size_t own = q->bytes - q->ws_bytes;  // rho + phi
    auto it = s->ws_free.lower_bound(q->ws_bytes);
    if (it != s->ws_free.end() && it->first <= 2 * q->ws_bytes) {
        const size_t sz = it->first;
        char *buf = it->second;
        s->ws_free.erase(it);
        s->ws_idle -= sz;
        if (s->bytes_inflight + s->ws_idle + own + sz > s->budget)
            ws_trim_locked(s, s->bytes_inflight, own + sz, q->ws_bytes);
        if (s->bytes_inflight + s->ws_idle + own + sz <= s->budget) {
            q->ws = buf;
            q->ws_real = sz;
            q->charge = own + sz;
            s->bytes_inflight += q->charge;
            s->peak_use = std::max(s->peak_use, s->bytes_inflight + s->ws_idle);
            s->peak = std::max(s->peak, s->bytes_inflight);
            return true;
        }
        s->ws_free.emplace(sz, buf);  // not this way: back to the pool
        s->ws_idle += sz;
    }
    if (s->bytes_inflight + q->bytes > s->budget) return false;
    if (s->bytes_inflight + s->ws_idle + q->bytes > s->budget)
        ws_trim_locked(s, s->bytes_inflight, q->bytes, q->ws_bytes);
    if (s->bytes_inflight + s->ws_idle + q->bytes > s->budget) return false;
    s->bytes_inflight += q->bytes;
    q->charge = q->bytes;
    s->peak_use = std::max(s->peak_use, s->bytes_inflight + s->ws_idle);
    s->peak = std::max(s->peak, s->bytes_inflight);
    return true;
}

// Admit launch units from the head of the queue while a slot is free: the
// head request, joined by later queued requests of the same lattice, dx,
// k^2 kind and bin count (at most kMaxGroup in all and kGroupPoints lattice
// points, lattices up to kGroupFieldPoints) while the budget holds
// them -- those run as one grouped solve.  A unit takes one slot.  FIFO for
// the heads: a head that does not fit the budget holds back the ones behind
// it.  Server lock held.
void admit_locked(lf2_server s, std::vector<std::vector<Req *>> &adm)
{
    while (!s->queue.empty()) {
        if (s->units_busy >= s->max_slots) break;
        Req *q = s->queue.front();
        if (!fits_budget_locked(s, q)) break;
        s->queue.pop_front();
        std::vector<Req *> unit{q};
        if (groupable(q)) {
            const GroupKey k = group_key(q);
            const int64_t pts = points_of(q);
            int64_t total = pts;
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)unit.size() < kMaxGroup &&
                                              total + pts <= kGroupPoints;) {
                if (group_key(*it) == k && fits_budget_locked(s, *it)) {
                    unit.push_back(*it);
                    total += pts;
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
        }
        const double t = now_s();
        for (Req *u : unit) u->t_adm = t;
        s->launching += (int)unit.size();
        s->units_busy += 1;
        adm.push_back(std::move(unit));
    }
}

// Launch admitted units and hand them to the completion thread; called and
// returns with the server lock held.
void launch_admitted(lf2_server s, std::unique_lock<std::mutex> &lk,
                     std::vector<std::vector<Req *>> &adm)
{
    if (adm.empty()) return;
    lk.unlock();
    int prev = -1;
    if (!s->fake && hipGetDevice(&prev) == hipSuccess && prev != s->device)
        (void)hipSetDevice(s->device);  // a submitting thread may have another device current
    for (std::vector<Req *> &u : adm) {
        launch_unit(s, u);
        if (s->fake)
            for (Req *q : u) q->due = q->t_adm + 1e-6 * s->delay_us;
    }
    if (prev >= 0 && prev != s->device) (void)hipSetDevice(prev);
    lk.lock();
    for (std::vector<Req *> &u : adm) {
        s->launching -= (int)u.size();
        for (Req *q : u) s->inflight.push_back(q);
    }
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
            return s->units_busy < s->max_slots &&
                   s->bytes_inflight + s->queue.front()->bytes <= s->budget;
        });
        if (s->stop) break;
        std::vector<std::vector<Req *>> adm;
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
        int units_done = 0;
        for (Req *q : fin) units_done += release(s, q) ? 1 : 0;
        lk.lock();
        s->units_busy -= units_done;
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
            s->bytes_inflight -= q->charge;
            ws_put(s, q->ws);  // pool lock inside the server lock, as in admission
            q->ws = nullptr;
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
    int pools = 0;
    if (hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, s->device) ==
            hipSuccess &&
        pools) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = s->device;
        if (hipMemPoolCreate(&s->mpool, &props) != hipSuccess) {
            (void)hipGetLastError();
            s->mpool = nullptr;
        }
    }
    for (int i = 0; i < nstreams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            if (s->mpool) (void)hipMemPoolDestroy(s->mpool);
            delete s;
            return fail(LF2_ERR_DEVICE, "stream creation");
        }
        s->streams.push_back(st);
    }
    lf2_status st = server_start(s);
    if (st) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        if (s->mpool) (void)hipMemPoolDestroy(s->mpool);
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
        {
            // only while the budget holds it next to what is in flight
            std::lock_guard<std::mutex> lk(s->mu);
            std::lock_guard<std::mutex> pk(s->pmu);
            if (s->bytes_inflight + s->ws_idle + wb > s->budget) continue;
        }
        size_t real = 0;
        char *w = ws_get(s, wb, &real, s->fake ? nullptr : s->streams[0]);
        if (!w) return fail(LF2_ERR_OUT_OF_MEMORY, "workspace");
        ws_put(s, w);
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
        std::vector<std::vector<Req *>> adm;
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
    st->groups = s->n_groups;
    st->grouped_requests = s->n_grouped;
    {
        std::lock_guard<std::mutex> pk(s->pmu);
        st->plans_cached = (int64_t)s->plans.size();
        st->plan_hits = s->plan_hits;
        st->plan_misses = s->plan_misses;
        st->pooled_idle_bytes = s->ws_idle;
        st->peak_bytes_in_use = s->peak_use;
        st->workspace_allocs = s->n_ws_alloc;
        st->workspace_frees = s->n_ws_free;
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
    for (auto &kv : s->ws_free) ws_release(s, kv.second);  // every buffer is idle now
    if (!s->fake) {
        for (hipStream_t x : s->streams) (void)hipStreamSynchronize(x);
        for (auto &kv : s->plans)
            if (kv.second.plan) lf2_plan_destroy(kv.second.plan);
        for (hipEvent_t e : s->ev_all) (void)hipEventDestroy(e);
        for (auto &hd : s->stage_all) {
            (void)hipHostFree(hd.first);
            (void)hipFree(hd.second);
        }
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        if (s->mpool) (void)hipMemPoolDestroy(s->mpool);
    }
    delete s;
    return LF2_OK;
}

}  // extern "C"
