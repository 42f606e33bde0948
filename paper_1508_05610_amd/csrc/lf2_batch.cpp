// lf2_batch.cpp -- batched Poisson solves (with optional fused power spectra)
// on many lattices of different sizes.  Work items (field, tile) are grouped
// by pass and line length; one launch per group plus one finalize launch for
// the power spectra, all captured in one hipGraph.  A group waits only for
// the groups of the previous pass that hold its fields, so groups of one
// pass (disjoint fields) and groups of consecutive passes on unrelated
// fields run concurrently and fill each other's tails.
#include <stdio.h>
#include <string.h>

#include <map>
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
};

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
    for (lf2_plan p : b->plans) lf2_plan_destroy(p);
    delete b;
}

// Capture one execution into b->graph from the origin stream cs: every group
// on a stream of its own (joined into the capture through events) after the
// groups of the previous pass that share a field with it; the finalize after
// all fused z groups; the origin stream finally joins every group.
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
                                   b->nbins, st[g]);
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
    if (!(ops & LF2_BATCH_POISSON) || (ops & ~(uint32_t)(LF2_BATCH_POISSON | LF2_BATCH_PK)))
        return fail(LF2_ERR_UNSUPPORTED, "batch ops 0x%x: LF2_BATCH_POISSON [| LF2_BATCH_PK]", ops);
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
        const int xr = batch_x_rows(p->len[0]);
        const int b1 = s_cols_per_block(p->len[1]), b2 = s_cols_per_block(p->len[2]);
        tiles[f][BP_XF] = (int)((n1 * n2 + xr - 1) / xr);
        tiles[f][BP_XI] = tiles[f][BP_XF];
        tiles[f][BP_YF] = (int)((n2 * nh + b1 - 1) / b1);
        tiles[f][BP_YI] = tiles[f][BP_YF];
        tiles[f][BP_Z] = (int)((n1 * nh + b2 - 1) / b2);
        tiles[f][BP_FIN] = 0;
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
        F.m = p->len[0];
        F.l1 = p->len[1];
        F.l2 = p->len[2];
        for (int i = 0; i < BP_COUNT; ++i) F.ntiles[i] = tiles[f][i];
        F.nbins = nbins;
        if (pk) {
            ShellEntry sh{};
            if ((st = get_shell(p, nbins, nullptr, &sh))) break;
            F.z.mt.thresh = sh.thresh;
            F.z.mt.nbins = nbins;
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
    return LF2_OK;
}

lf2_status lf2_batch_info(lf2_batch b, int64_t *nitems, int32_t *launches, size_t *workspace_bytes)
{
    if (!b) return fail(LF2_ERR_INVALID_ARG, "batch is NULL");
    if (nitems) *nitems = b->nitems;
    if (launches) *launches = (int32_t)b->groups.size() + (b->nbins > 0 ? 1 : 0);
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
