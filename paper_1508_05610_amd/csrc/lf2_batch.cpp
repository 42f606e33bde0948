// lf2_batch.cpp -- batched Poisson solves (with optional fused power spectra)
// on many lattices of different sizes.
//
// Persistent mode (the default): every (field, pass, tile) work item of the
// batch, the power-spectrum finalizes included, runs in one launch of a
// persistent kernel whose blocks take items from a work queue
// (lf2_queue.hpp) in an order where every item comes after what it depends
// on; the launch is captured in a hipGraph.
// Grouped mode (LF2_BATCH_GROUPED): items grouped by pass and line length,
// one launch per group plus one finalize launch, captured in one hipGraph in
// which a group waits only for the groups of the previous pass that hold its
// fields.
#include <stddef.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "lf2_internal.hpp"
#include "lf2_plan.hpp"

using namespace lf2;
using namespace lf2::host;

namespace {
struct Group {
    int pass, len, offset, count;
    std::vector<int> fields;
};
}  // namespace

struct lf2_batch_s {
    int device = 0;
    int nfields = 0;
    uint32_t ops = 0;
    int nbins = 0;
    double dx = 1.0;
    uint32_t pflags = 0;
    std::vector<lf2_plan> plans;   // one per distinct lattice
    std::vector<int> pidx;         // plan of each field
    std::vector<BatchField> hf;    // descriptors without the caller's pointers
    BatchField *pinned = nullptr;  // staging for the descriptor upload
    BatchField *d_fields = nullptr;
    BatchItem *d_items = nullptr;
    int nitems = 0;
    std::vector<Group> groups;
    char *ws = nullptr;            // spectra of all fields
    size_t ws_bytes = 0;
    double *d_partial = nullptr;
    double alg_bytes = 0.0;        // algorithmic HBM bytes of one execution
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> last;  // caller pointers of the last upload
    bool persistent = true;
    QItem *d_qitems = nullptr;     // persistent mode: the work lists of the queues
    uint32_t *d_qmeta = nullptr;   // qstart[nq + 1], qcount[nq + 1]
    int32_t *d_xq = nullptr;       // queue of each XCC id (16)
    QCtl *d_ctl = nullptr;         // tickets, exit count, error word (nq + 1)
    uint32_t *d_done = nullptr;    // per-(field, pass) completion counters
    int ndone = 0;
    int nq = 1;                    // queues (one per XCD, or one)
    int local = 0;                 // 1: each block serves its XCD's queue
    int pgrid = 0;                 // blocks of the persistent launch
    int per_item = 1;              // tiles per work item
};

// Polls of a dependency wait before the persistent kernel gives up on it.
// A poll sleeps about 128 clocks and reads memory, so the limit is at least
// a tenth of a second; a run of the whole 48-field batch takes under 3 ms.
constexpr uint32_t kSpinLimit = 1u << 20;

static void batch_free(lf2_batch b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->pinned) (void)hipHostFree(b->pinned);
    (void)hipFree(b->d_fields);
    (void)hipFree(b->d_items);
    (void)hipFree(b->ws);
    (void)hipFree(b->d_partial);
    (void)hipFree(b->d_qitems);
    (void)hipFree(b->d_qmeta);
    (void)hipFree(b->d_xq);
    (void)hipFree(b->d_ctl);
    (void)hipFree(b->d_done);
    for (lf2_plan p : b->plans) lf2_plan_destroy(p);
    delete b;
}

// Capture one execution into b->graph from the origin stream cs: every group
// on a stream of its own (joined into the capture through events) after the
// groups of the previous pass that share a field with it; the finalize after
// all fused z groups; the origin stream finally joins every group.
// The XCC (XCD) ids that blocks of a launch run on, sorted (probed once per
// device: the ids the hardware reports, whatever the partition mode).
static hipError_t xcc_ids(int device, std::vector<int> &ids)
{
    static std::mutex mu;
    static std::map<int, std::vector<int>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(device);
    if (it != cache.end()) {
        ids = it->second;
        return hipSuccess;
    }
    const int n = 4096;
    int32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int32_t) * n);
    std::vector<int32_t> h(n, -1);
    if (e == hipSuccess) e = launch_xcc_probe(d, n, nullptr);
    if (e == hipSuccess) e = hipMemcpy(h.data(), d, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (d) (void)hipFree(d);
    if (e != hipSuccess) return e;
    std::vector<int> out;
    for (int v : h)
        if (v >= 0 && v < 16 && std::find(out.begin(), out.end(), v) == out.end()) out.push_back(v);
    std::sort(out.begin(), out.end());
    cache[device] = out;
    ids = out;
    return hipSuccess;
}

static hipError_t capture_persistent(lf2_batch b, hipStream_t cs)
{
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    e = batch_persistent_launch(b->d_fields, b->d_qitems, b->d_qmeta, b->d_qmeta + b->nq + 1, b->nq,
                                b->d_xq, b->d_ctl, b->d_done, b->ndone, kSpinLimit, b->local,
                                b->pgrid, cs);
    const hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
    return e != hipSuccess ? e : e2;
}

static hipError_t capture(lf2_batch b, hipStream_t cs)
{
    const size_t ng = b->groups.size();
    std::vector<hipStream_t> st(ng, nullptr);
    std::vector<hipEvent_t> done(ng, nullptr);
    hipEvent_t start = nullptr;
    hipError_t e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    for (size_t g = 0; g < ng && e == hipSuccess; ++g) {
        e = hipStreamCreateWithFlags(&st[g], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done[g], hipEventDisableTiming);
    }
    bool capturing = false;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    capturing = e == hipSuccess;
    if (e == hipSuccess) e = hipEventRecord(start, cs);
    // group of (pass, field), filled pass by pass
    std::vector<int> owner((size_t)BP_COUNT * b->nfields, -1);
    for (size_t g = 0; g < ng && e == hipSuccess; ++g) {
        const Group &G = b->groups[g];
        std::vector<int> deps;
        for (int f : G.fields) {
            owner[(size_t)G.pass * b->nfields + f] = (int)g;
            const int h = G.pass > BP_XF ? owner[(size_t)(G.pass - 1) * b->nfields + f] : -1;
            bool seen = false;
            for (int d : deps) seen = seen || d == h;
            if (!seen) deps.push_back(h);
        }
        for (int h : deps)
            if (e == hipSuccess) e = hipStreamWaitEvent(st[g], h < 0 ? start : done[h], 0);
        if (e == hipSuccess)
            e = batch_group_launch(G.pass, G.len, b->d_fields, b->d_items + G.offset, G.count,
                                   b->nbins, (b->pflags & LF2_POISSON_DISCRETE_K2) ? 0 : 1,
                                   st[g]);
        if (e == hipSuccess) e = hipEventRecord(done[g], st[g]);
    }
    if (b->nbins > 0) {
        for (size_t g = 0; g < ng && e == hipSuccess; ++g)
            if (b->groups[g].pass == BP_Z) e = hipStreamWaitEvent(cs, done[g], 0);
        if (e == hipSuccess) e = batch_finalize_launch(b->d_fields, b->nfields, cs);
    }
    for (size_t g = 0; g < ng && e == hipSuccess; ++g) e = hipStreamWaitEvent(cs, done[g], 0);
    if (capturing) {
        const hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
        if (e == hipSuccess) e = e2;
    }
    // streams and events only shape the capture; the graph does not use them
    for (size_t g = 0; g < ng; ++g) {
        if (done[g]) (void)hipEventDestroy(done[g]);
        if (st[g]) (void)hipStreamDestroy(st[g]);
    }
    if (start) (void)hipEventDestroy(start);
    return e;
}

extern "C" {

lf2_status lf2_batch_plan(lf2_batch *out, int32_t nfields, const lf2_lattice *lats, uint32_t ops,
                          int32_t nbins, double dx, uint32_t poisson_flags)
{
    if (!out) return fail(LF2_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nfields < 1 || !lats) return fail(LF2_ERR_INVALID_ARG, "need at least one lattice");
    if (!(ops & LF2_BATCH_POISSON) ||
        (ops & ~(uint32_t)(LF2_BATCH_POISSON | LF2_BATCH_PK | LF2_BATCH_GROUPED |
                           LF2_BATCH_ONE_QUEUE)))
        return fail(LF2_ERR_UNSUPPORTED,
                    "batch ops 0x%x: LF2_BATCH_POISSON [| LF2_BATCH_PK] [| LF2_BATCH_GROUPED | "
                    "LF2_BATCH_ONE_QUEUE]", ops);
    const bool pk = (ops & LF2_BATCH_PK) != 0;
    if (pk && (nbins < 1 || nbins > kBatchMaxBins))
        return fail(LF2_ERR_UNSUPPORTED, "batch binning needs 1 <= nbins <= %d", kBatchMaxBins);
    if (!pk) nbins = 0;
    if (!(dx > 0.0)) return fail(LF2_ERR_INVALID_ARG, "dx must be > 0");
    if (poisson_flags & ~(uint32_t)LF2_POISSON_DISCRETE_K2)
        return fail(LF2_ERR_UNSUPPORTED, "batch Poisson flags 0x%x", poisson_flags);
    for (int f = 0; f < nfields; ++f) {
        const lf2_lattice &L = lats[f];
        if (L.dim != 3 || L.halo != 0)
            return fail(LF2_ERR_UNSUPPORTED, "field %d: batches take dense 3-d lattices (halo 0)", f);
        if (L.size[0] < 2 || L.size[0] % 2)
            return fail(LF2_ERR_UNSUPPORTED, "field %d: N0 must be even", f);
        if (!batch_len_supported((int)(L.size[0] / 2)) || !batch_len_supported((int)L.size[1]) ||
            !batch_len_supported((int)L.size[2]))
            return fail(LF2_ERR_UNSUPPORTED,
                        "field %d: extents %lldx%lldx%lld outside the batch kernels' line lengths", f,
                        (long long)L.size[0], (long long)L.size[1], (long long)L.size[2]);
    }
    lf2_batch b = new (std::nothrow) lf2_batch_s();
    if (!b) return fail(LF2_ERR_OUT_OF_MEMORY, "batch allocation");
    lf2_status st = LF2_OK;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return fail(LF2_ERR_DEVICE, "hipGetDevice");
    }
    b->nfields = nfields;
    b->ops = ops;
    b->nbins = nbins;
    b->dx = dx;
    b->pflags = poisson_flags;
    b->persistent = (ops & LF2_BATCH_GROUPED) == 0;

    // plans, tables and spectra per field
    std::map<std::tuple<int64_t, int64_t, int64_t>, int> cache;
    std::vector<size_t> wofs(nfields), pofs(nfields);
    size_t wtot = 0, ptot = 0;
    std::vector<std::vector<int>> tiles(nfields, std::vector<int>(BP_COUNT, 0));
    for (int f = 0; f < nfields && st == LF2_OK; ++f) {
        auto key = std::make_tuple(lats[f].size[0], lats[f].size[1], lats[f].size[2]);
        auto it = cache.find(key);
        int pi;
        if (it == cache.end()) {
            lf2_plan p = nullptr;
            st = lf2_fft_plan(&p, &lats[f], 1, LF2_R2C, 0);
            if (st) break;
            pi = (int)b->plans.size();
            b->plans.push_back(p);
            cache[key] = pi;
        } else {
            pi = it->second;
        }
        b->pidx.push_back(pi);
        lf2_plan p = b->plans[pi];
        wofs[f] = wtot;
        wtot += align256(spectrum_bytes(p));
        const int64_t nh = p->nh, n1 = p->n[1], n2 = p->n[2];
        const int xr = b->persistent ? batch_px_rows(p->len[0]) : batch_x_rows(p->len[0]);
        const int b1 = s_cols_per_block(p->len[1]), b2 = s_cols_per_block(p->len[2]);
        tiles[f][BP_XF] = (int)((n1 * n2 + xr - 1) / xr);
        tiles[f][BP_XI] = tiles[f][BP_XF];
        tiles[f][BP_YF] = (int)((n2 * nh + b1 - 1) / b1);
        tiles[f][BP_YI] = tiles[f][BP_YF];
        tiles[f][BP_Z] = (int)((n1 * nh + b2 - 1) / b2);
        tiles[f][BP_FIN] = (b->persistent && pk) ? 1 : 0;
        pofs[f] = ptot;
        ptot += pk ? (size_t)tiles[f][BP_Z] * (nbins + 1) : 0;
        // x r2c 4N + 8H, y / z / y-inverse 16H each, x c2r 8H + 4N
        b->alg_bytes += 8.0 * (double)p->ntot + 64.0 * (double)(nh * n1 * n2);
    }
    if (st) {
        batch_free(b);
        return st;
    }
    auto alloc = [&](void **ptr, size_t bytes) -> lf2_status {
        hipError_t e = hipMalloc(ptr, bytes < 256 ? 256 : bytes);
        return e == hipSuccess ? LF2_OK
                               : fail(LF2_ERR_OUT_OF_MEMORY, "batch hipMalloc(%zu): %s", bytes,
                                      hipGetErrorString(e));
    };
    b->ws_bytes = wtot;
    if ((st = alloc((void **)&b->ws, wtot)) || (st = alloc((void **)&b->d_partial, ptot * 8)) ||
        (st = alloc((void **)&b->d_fields, sizeof(BatchField) * nfields))) {
        batch_free(b);
        return st;
    }
    if (hipHostMalloc((void **)&b->pinned, sizeof(BatchField) * nfields, 0) != hipSuccess) {
        batch_free(b);
        return fail(LF2_ERR_OUT_OF_MEMORY, "pinned descriptor staging");
    }

    // descriptors
    b->hf.resize(nfields);
    for (int f = 0; f < nfields && st == LF2_OK; ++f) {
        lf2_plan p = b->plans[b->pidx[f]];
        void *W = b->ws + wofs[f];
        BatchField &F = b->hf[f];
        memset(&F, 0, sizeof F);
        F.xf = x_args(p, nullptr, W, true, false, true);
        F.xi = x_args(p, W, nullptr, false, true, true);
        F.yf = s_args(p, 1, W, W, EPI_STORE);
        F.yi = s_args(p, 1, W, W, EPI_STORE);
        F.z = s_args(p, 2, W, W, EPI_STORE | EPI_POISSON | (pk ? EPI_PK : 0));
        const double *k2[3];
        if ((st = get_k2(p, dx, (poisson_flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0, nullptr, k2)))
            break;
        for (int i = 0; i < 3; ++i) F.z.mt.k2[i] = k2[i];
        set_k2_units(F.z.mt, p, dx, (poisson_flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0);
        // bin histograms per wave where the z tile's LDS leaves room for them
        F.z.hcopies = pk ? epi_hist_copies(p->len[2], nbins,
                                           b->persistent ? batch_persistent_lds() : 80 * 1024)
                         : 1;
        if (F.z.hcopies < 1) F.z.hcopies = 1;
        F.m = p->len[0];
        F.l1 = p->len[1];
        F.l2 = p->len[2];
        for (int i = 0; i < BP_COUNT; ++i) F.ntiles[i] = tiles[f][i];
        F.nbins = nbins;
        if (pk) {
            ShellEntry sh{};
            if ((st = get_shell(p, nbins, nullptr, &sh))) break;
            use_shell(F.z.mt, sh);
            F.partial = b->d_partial + pofs[f];
            F.count = sh.count;
            F.sumk = sh.sumk;
            F.norm = dx * dx * dx / (double)p->ntot;
            F.kscale = 6.283185307179586476925286766559 / ((double)p->lcm * dx);
        }
    }
    if (st) {
        batch_free(b);
        return st;
    }

    if (b->persistent) {
        std::vector<std::array<int, BP_COUNT>> tl(nfields);
        std::vector<double> fwork(nfields);
        for (int f = 0; f < nfields; ++f) {
            for (int p = 0; p < BP_COUNT; ++p) tl[f][p] = tiles[f][p];
            lf2_plan p = b->plans[b->pidx[f]];
            fwork[f] = 8.0 * (double)p->ntot + 64.0 * (double)(p->nh * p->n[1] * p->n[2]);
        }
        // one queue per XCD when the fields spread evenly over them (every
        // field's passes then stay in one L2); one queue otherwise
        std::vector<int> ids;
        hipError_t e = xcc_ids(b->device, ids);
        if (e != hipSuccess) {
            batch_free(b);
            return fail(LF2_ERR_DEVICE, "XCD probe: %s", hipGetErrorString(e));
        }
        std::vector<int> queue_of(nfields, 0);
        b->nq = 1;
        b->local = 0;
        if (!(ops & LF2_BATCH_ONE_QUEUE) && ids.size() >= 2 && nfields >= (int)ids.size()) {
            const int nx = (int)ids.size();
            std::vector<int> qo = balance_queues(fwork, nx);
            std::vector<double> load(nx, 0.0);
            double tot = 0.0;
            for (int f = 0; f < nfields; ++f) {
                load[qo[f]] += fwork[f];
                tot += fwork[f];
            }
            const double mx = *std::max_element(load.begin(), load.end());
            if (mx <= 1.25 * tot / nx) {
                queue_of = qo;
                b->nq = nx;
                b->local = 1;
            }
        }
        // tiles per item: about fifteen items per block, so that each item's
        // wait and publication (and the call into its tile code) are spread
        // over several tiles while the last items of a pass stay short
        int64_t ntiles_all = 0;
        for (int f = 0; f < nfields; ++f)
            for (int p = 0; p < BP_COUNT; ++p) ntiles_all += tiles[f][p];
        int ncu0 = 0;
        if (hipDeviceGetAttribute(&ncu0, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
            ncu0 < 1)
            ncu0 = 256;
        int per_item = (int)(ntiles_all / (2 * ncu0 * 15));
        if (const char *ev = getenv("LF2_BATCH_TILES_PER_ITEM")) per_item = atoi(ev);
        per_item = per_item < 1 ? 1 : per_item > 64 ? 64 : per_item;
        b->per_item = per_item;
        std::vector<uint32_t> qstart, qcount;
        const std::vector<QItem> q = batch_items(tl, per_item, queue_of, b->nq, qstart, qcount);
        qstart.push_back((uint32_t)q.size());  // the empty queue
        qcount.push_back(0);
        std::vector<uint32_t> meta(qstart);
        meta.insert(meta.end(), qcount.begin(), qcount.end());
        std::vector<int32_t> xq(16, b->nq);
        if (b->local)
            for (int i = 0; i < b->nq; ++i) xq[ids[i]] = i;
        b->nitems = (int)q.size();
        b->ndone = nfields * BP_COUNT;
        int ncu = 0;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device);
        // two 512-thread blocks fit one CU (LDS and registers)
        b->pgrid = 2 * (e == hipSuccess && ncu > 0 ? ncu : 256);
        if ((st = alloc((void **)&b->d_qitems, sizeof(QItem) * q.size())) ||
            (st = alloc((void **)&b->d_qmeta, sizeof(uint32_t) * meta.size())) ||
            (st = alloc((void **)&b->d_xq, sizeof(int32_t) * 16)) ||
            (st = alloc((void **)&b->d_ctl, sizeof(QCtl) * (b->nq + 1))) ||
            (st = alloc((void **)&b->d_done, sizeof(uint32_t) * b->ndone))) {
            batch_free(b);
            return st;
        }
        e = hipMemcpy(b->d_qitems, q.data(), sizeof(QItem) * q.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_qmeta, meta.data(), sizeof(uint32_t) * meta.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_xq, xq.data(), sizeof(int32_t) * 16, hipMemcpyHostToDevice);
        // the queues start empty; every run leaves them empty again
        if (e == hipSuccess) e = hipMemset(b->d_ctl, 0, sizeof(QCtl) * (b->nq + 1));
        if (e == hipSuccess) e = hipMemset(b->d_done, 0, sizeof(uint32_t) * b->ndone);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        hipStream_t cs = nullptr;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = capture_persistent(b, cs);
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (cs) (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            batch_free(b);
            return fail(LF2_ERR_DEVICE, "persistent batch setup: %s", hipGetErrorString(e));
        }
        *out = b;
        return LF2_OK;
    }

    // work items grouped by (pass, line length), passes in order
    std::vector<BatchItem> items;
    for (int pass = BP_XF; pass <= BP_XI; ++pass) {
        std::map<int, std::vector<int>> by_len;
        for (int f = 0; f < nfields; ++f) {
            const BatchField &F = b->hf[f];
            const int len = (pass == BP_XF || pass == BP_XI) ? F.m
                            : (pass == BP_Z)                 ? F.l2
                                                             : F.l1;
            by_len[len].push_back(f);
        }
        for (auto &kv : by_len) {
            Group g{pass, kv.first, (int)items.size(), 0, kv.second};
            for (int f : kv.second)
                for (int t = 0; t < tiles[f][pass]; ++t) items.push_back(BatchItem{f, t});
            g.count = (int)items.size() - g.offset;
            b->groups.push_back(g);
        }
    }
    b->nitems = (int)items.size();
    if ((st = alloc((void **)&b->d_items, sizeof(BatchItem) * items.size()))) {
        batch_free(b);
        return st;
    }
    hipError_t e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        batch_free(b);
        return fail(LF2_ERR_DEVICE, "batch setup: %s", hipGetErrorString(e));
    }

    // graph of the grouped launches
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = capture(b, cs);
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(LF2_ERR_DEVICE, "batch graph capture: %s", hipGetErrorString(e));
    }
    *out = b;
    return LF2_OK;
}

lf2_status lf2_batch_execute(lf2_batch b, const float *const *rho, float *const *phi,
                             double *const *d_pk, double *const *d_kmean, double *const *d_count,
                             void *stream)
{
    if (!b) return fail(LF2_ERR_INVALID_ARG, "batch is NULL");
    if (!rho || !phi) return fail(LF2_ERR_INVALID_ARG, "rho and phi pointer arrays are required");
    int dev = -1;
    LF2_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(LF2_ERR_INVALID_ARG, "batch was made on device %d", b->device);
    std::vector<const void *> ptrs;
    ptrs.reserve((size_t)b->nfields * 5);
    for (int f = 0; f < b->nfields; ++f) {
        lf2_status st;
        if ((st = check_ptr(rho[f], "rho[f]", 8)) || (st = check_ptr(phi[f], "phi[f]", 8))) return st;
        if ((const void *)rho[f] == (const void *)phi[f])
            return fail(LF2_ERR_INVALID_ARG, "rho[%d] and phi[%d] alias", f, f);
        ptrs.push_back(rho[f]);
        ptrs.push_back(phi[f]);
        ptrs.push_back(d_pk ? d_pk[f] : nullptr);
        ptrs.push_back(d_kmean ? d_kmean[f] : nullptr);
        ptrs.push_back(d_count ? d_count[f] : nullptr);
    }
    hipStream_t s = (hipStream_t)stream;
    if (ptrs != b->last) {
        // the staging buffer may still feed an earlier upload on this stream
        LF2_HIP(hipStreamSynchronize(s));
        for (int f = 0; f < b->nfields; ++f) {
            BatchField F = b->hf[f];
            F.xf.in = rho[f];
            F.xi.out = phi[f];
            F.pk = d_pk ? d_pk[f] : nullptr;
            F.kmean = d_kmean ? d_kmean[f] : nullptr;
            F.count_out = d_count ? d_count[f] : nullptr;
            b->pinned[f] = F;
        }
        LF2_HIP(hipMemcpyAsync(b->d_fields, b->pinned, sizeof(BatchField) * b->nfields,
                               hipMemcpyHostToDevice, s));
        b->last = ptrs;
    }
    const int t = prof::begin("batch_graph", b->alg_bytes, s);
    hipError_t e = hipGraphLaunch(b->exec, s);
    prof::end(t, s);
    LF2_HIP(e);
    return LF2_OK;
}

lf2_status lf2_batch_error(lf2_batch b, uint32_t *err)
{
    if (!b || !err) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    *err = 0;
    LF2_HIP(hipDeviceSynchronize());
    if (b->d_ctl) {
        QCtl c{};
        LF2_HIP(hipMemcpy(&c, b->d_ctl, sizeof c, hipMemcpyDeviceToHost));
        *err = c.error;
        if (c.error) {
            // results of that run are not valid; the queues themselves were reset
            const uint32_t zero = 0;
            LF2_HIP(hipMemcpy((char *)b->d_ctl + offsetof(QCtl, error), &zero, sizeof zero,
                              hipMemcpyHostToDevice));
        }
    }
    return LF2_OK;
}

lf2_status lf2_batch_queues(lf2_batch b, int32_t *nqueues, int32_t *per_xcd)
{
    if (!b) return fail(LF2_ERR_INVALID_ARG, "batch is NULL");
    if (nqueues) *nqueues = b->persistent ? b->nq : 0;
    if (per_xcd) *per_xcd = b->local;
    return LF2_OK;
}

lf2_status lf2_batch_info(lf2_batch b, int64_t *nitems, int32_t *launches, size_t *workspace_bytes)
{
    if (!b) return fail(LF2_ERR_INVALID_ARG, "batch is NULL");
    if (nitems) *nitems = b->nitems;
    if (launches)
        *launches = b->persistent ? 1 : (int32_t)b->groups.size() + (b->nbins > 0 ? 1 : 0);
    if (workspace_bytes) *workspace_bytes = b->ws_bytes;
    return LF2_OK;
}

lf2_status lf2_batch_destroy(lf2_batch b)
{
    if (!b) return fail(LF2_ERR_INVALID_ARG, "batch is NULL");
    batch_free(b);
    return LF2_OK;
}

}  // extern "C"

// ------------------------------------------------ grouped solves of one lattice
// The serving loop batches requests admitted together: R Poisson solves on
// one lattice (one plan, one dx, k^2 kind and bin count) run as one launch
// per pass over all R fields plus one finalize launch, on one stream.

namespace lf2 {
namespace host {

namespace {
struct GroupShape {
    int64_t tx, ty, tz;   // tiles of the x, y and z passes of one field
    size_t part_rows;     // bin rows of one field (one per z tile)
};

GroupShape group_shape(const lf2_plan_s *p)
{
    GroupShape g{};
    const int xr = batch_x_rows(p->len[0]);
    const int b1 = s_cols_per_block(p->len[1]), b2 = s_cols_per_block(p->len[2]);
    g.tx = (p->n[1] * p->n[2] + xr - 1) / xr;
    g.ty = (p->n[2] * p->nh + b1 - 1) / b1;
    g.tz = (p->n[1] * p->nh + b2 - 1) / b2;
    g.part_rows = (size_t)g.tz;
    return g;
}
}  // namespace

bool group_supported(const lf2_plan_s *p)
{
    return p->kind == LF2_R2C && p->nc == 1 && p->halo == 0 && !p->inplace && p->klay == 0 &&
           batch_len_supported(p->len[0]) && batch_len_supported(p->len[1]) &&
           batch_len_supported(p->len[2]);
}

size_t group_ws_bytes(const lf2_plan_s *p, int32_t nbins)
{
    const GroupShape g = group_shape(p);
    return align256(spectrum_bytes(p)) +
           (nbins > 0 ? align256(g.part_rows * (size_t)(nbins + 1) * 8) : 0);
}

size_t group_stage_bytes(const lf2_plan_s *p, int R)
{
    const GroupShape g = group_shape(p);
    return align256(sizeof(BatchField) * (size_t)R) +
           sizeof(BatchItem) * (size_t)R * (size_t)(g.tx + g.ty + g.tz);
}

lf2_status group_enqueue(lf2_plan p, int R, const GroupReq *req, double dx, uint32_t flags,
                         int32_t nbins, const PoissonTables &tabs, void *stage_host,
                         void *stage_dev, size_t stage_bytes, hipStream_t s)
{
    if (R < 1) return fail(LF2_ERR_INVALID_ARG, "empty group");
    if (!group_supported(p)) return fail(LF2_ERR_UNSUPPORTED, "lattice without grouped kernels");
    if (nbins > kBatchMaxBins) return fail(LF2_ERR_UNSUPPORTED, "grouped binning takes <= %d bins", kBatchMaxBins);
    if (stage_bytes < group_stage_bytes(p, R)) return fail(LF2_ERR_INVALID_ARG, "stage too small");
    const GroupShape g = group_shape(p);
    const bool pk = nbins > 0;
    const bool of_phi = (flags & LF2_PK_OF_PHI) != 0;
    BatchField *hf = (BatchField *)stage_host;
    for (int r = 0; r < R; ++r) {
        BatchField &F = hf[r];
        memset(&F, 0, sizeof F);
        void *W = req[r].ws;
        F.xf = x_args(p, req[r].rho, W, true, false, true);
        F.xi = x_args(p, W, req[r].phi, false, true, true);
        F.yf = s_args(p, 1, W, W, EPI_STORE);
        F.yi = s_args(p, 1, W, W, EPI_STORE);
        F.z = s_args(p, 2, W, W, EPI_STORE | EPI_POISSON | (pk ? (of_phi ? EPI_PK_AFTER : EPI_PK) : 0));
        for (int i = 0; i < 3; ++i) F.z.mt.k2[i] = tabs.k2[i];
        set_k2_units(F.z.mt, p, dx, (flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0);
        F.z.hcopies = pk ? epi_hist_copies(p->len[2], nbins, 80 * 1024) : 1;
        if (F.z.hcopies < 1) F.z.hcopies = 1;
        F.m = p->len[0];
        F.l1 = p->len[1];
        F.l2 = p->len[2];
        F.ntiles[BP_XF] = F.ntiles[BP_XI] = (int)g.tx;
        F.ntiles[BP_YF] = F.ntiles[BP_YI] = (int)g.ty;
        F.ntiles[BP_Z] = (int)g.tz;
        F.nbins = nbins;
        if (pk) {
            use_shell(F.z.mt, tabs.sh);
            F.partial = (double *)((char *)W + align256(spectrum_bytes(p)));
            F.count = tabs.sh.count;
            F.sumk = tabs.sh.sumk;
            // phi's spectrum is the scaled rho spectrum times N
            const double vs = of_phi ? (double)p->ntot * (double)p->ntot : 1.0;
            F.norm = vs * dx * dx * dx / (double)p->ntot;
            F.kscale = 6.283185307179586476925286766559 / ((double)p->lcm * dx);
            F.pk = req[r].pk;
            F.kmean = req[r].kmean;
            F.count_out = req[r].count;
        }
    }
    // items: x passes (forward and backward share a list), y passes, z pass
    BatchItem *it = (BatchItem *)((char *)stage_host + align256(sizeof(BatchField) * (size_t)R));
    BatchItem *ix = it, *iy = ix + (size_t)R * g.tx, *iz = iy + (size_t)R * g.ty;
    for (int r = 0; r < R; ++r) {
        for (int64_t t = 0; t < g.tx; ++t) ix[r * g.tx + t] = BatchItem{r, (int)t};
        for (int64_t t = 0; t < g.ty; ++t) iy[r * g.ty + t] = BatchItem{r, (int)t};
        for (int64_t t = 0; t < g.tz; ++t) iz[r * g.tz + t] = BatchItem{r, (int)t};
    }
    const size_t used = group_stage_bytes(p, R);
    LF2_HIP(hipMemcpyAsync(stage_dev, stage_host, used, hipMemcpyHostToDevice, s));
    const BatchField *df = (const BatchField *)stage_dev;
    const BatchItem *dit = (const BatchItem *)((char *)stage_dev + align256(sizeof(BatchField) * (size_t)R));
    const BatchItem *dx_ = dit, *dy_ = dx_ + (size_t)R * g.tx, *dz_ = dy_ + (size_t)R * g.ty;
    const int k2c = (flags & LF2_POISSON_DISCRETE_K2) ? 0 : 1;
    const double alg = (double)R * (8.0 * (double)p->ntot + 64.0 * (double)(p->nh * p->n[1] * p->n[2]));
    const int t = prof::begin(kname("serve_group %lldx%lldx%lld x%d", (long long)p->n[0],
                                    (long long)p->n[1], (long long)p->n[2], R),
                              alg, s);
    hipError_t e = batch_group_launch(BP_XF, p->len[0], df, dx_, (int)(R * g.tx), nbins, k2c, s);
    if (e == hipSuccess) e = batch_group_launch(BP_YF, p->len[1], df, dy_, (int)(R * g.ty), nbins, k2c, s);
    if (e == hipSuccess) e = batch_group_launch(BP_Z, p->len[2], df, dz_, (int)(R * g.tz), nbins, k2c, s);
    if (e == hipSuccess) e = batch_group_launch(BP_YI, p->len[1], df, dy_, (int)(R * g.ty), nbins, k2c, s);
    if (e == hipSuccess) e = batch_group_launch(BP_XI, p->len[0], df, dx_, (int)(R * g.tx), nbins, k2c, s);
    if (e == hipSuccess && pk) e = batch_finalize_launch(df, R, s);
    prof::end(t, s);
    if (e != hipSuccess) return fail(LF2_ERR_DEVICE, "grouped solve launch: %s", hipGetErrorString(e));
    return LF2_OK;
}

}  // namespace host
}  // namespace lf2
