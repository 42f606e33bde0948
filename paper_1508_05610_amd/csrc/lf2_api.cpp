// lf2_api.cpp -- plans, validation and the C ABI (include/lf2.h).
//
// A plan holds the per-axis twiddle tables (FP64 on the device, rounded once
// to FP32), the integer wavevector tables used by the binning, lazily built
// k^2 tables (per lattice spacing) and shell tables (per bin count).  The
// pass sequence per call:
//   r2c forward : x r2c (in -> out), y (out), z (out)
//   c2r         : z (in -> W), y (W), x c2r (W -> out)       input untouched
//   c2c         : x (in -> out), y (out), z (out) / z, y, x backward
//   Poisson     : x r2c (rho -> W), y (W), z fwd * -1/(N k^2) * z bwd with
//                 optional binning (W), y bwd (W), x c2r (W -> phi)
//   P(k)        : x, y (into W), z forward with a read-only binning epilogue
// followed, when binning, by a fixed-order FP64 reduction and finalize.
#include "../../include/lf2.h"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "lf2_device.hpp"
#include "lf2_internal.hpp"
#include "lf2_plan.hpp"

using namespace lf2;

namespace lf2 {
namespace host {

thread_local std::string g_err;

lf2_status fail(lf2_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

constexpr int kMaxDevices = 64;

// Shared workspace per device (the paper's temporary memory shared by plans).
struct SharedWs {
    std::mutex mu;
    void *ptr = nullptr;
    size_t bytes = 0;
};
SharedWs g_ws[kMaxDevices];

int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Columns of a run-time-schedule strided tile of lines of L points: as many
// as fit the block's LDS (at most 64), 0 if not even one does.
int gs_cols(const lf2_plan_s *p, int L, int nbins)
{
    int b = 64;
    while (b > 0 && gs_lds_bytes(L, b, nbins) > p->lds_max) --b;
    return b;
}

// Rows of a run-time-schedule x tile: about 4096 complex values per tile (as
// the compiled x tiles), fewer if the LDS does not hold them, 0 if not even
// one row fits.
int gx_rows(const lf2_plan_s *p, int M, int nc)
{
    int rb = 4096 / (M * nc);
    rb = rb < 1 ? 1 : rb > 256 ? 256 : rb;
    while (rb > 0 && gx_lds_bytes(M, nc, rb) > p->lds_max) --rb;
    return rb;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// ------------------------------------------------------------- kernel timing
namespace prof {
struct Rec {
    int id;
    hipEvent_t a, b;
    double bytes;
};
struct Agg {
    int64_t n = 0;
    double ms = 0.0, bytes = 0.0;
};
std::mutex mu;
bool on = false;
std::vector<std::string> names;
std::vector<Agg> agg;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;

hipEvent_t take()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Set while a call that must not allocate runs on this thread: its launches
// are not recorded (recording may create events).
thread_local bool t_quiet = false;

// Returns a record index, or -1 when timing is off.
int begin(const std::string &name, double bytes, hipStream_t s)
{
    if (t_quiet) return -1;
    std::lock_guard<std::mutex> lk(mu);
    if (!on) return -1;
    int id = -1;
    for (size_t i = 0; i < names.size(); ++i)
        if (names[i] == name) id = (int)i;
    if (id < 0) {
        names.push_back(name);
        agg.emplace_back();
        id = (int)names.size() - 1;
    }
    Rec r{id, take(), take(), bytes};
    if (!r.a || !r.b) return -1;
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
    return (int)recs.size() - 1;
}

void end(int idx, hipStream_t s)
{
    if (idx < 0) return;
    std::lock_guard<std::mutex> lk(mu);
    if (idx < (int)recs.size()) (void)hipEventRecord(recs[idx].b, s);
}

void drain()
{
    for (Rec &r : recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            agg[r.id].n += 1;
            agg[r.id].ms += ms;
            agg[r.id].bytes += r.bytes;
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
}

void reset()
{
    drain();
    names.clear();
    agg.clear();
}
}  // namespace prof

std::string kname(const char *fmt, ...)
{
    char buf[128];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return buf;
}

lf2_status plan_alloc(lf2_plan p, void **dst, size_t bytes)
{
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess)
        return fail(LF2_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    p->allocs.push_back(ptr);
    *dst = ptr;
    return LF2_OK;
}

// Bytes of spectrum-sized workspace W for a call.
size_t spectrum_bytes(const lf2_plan_s *p)
{
    return (size_t)p->nxk * p->n[1] * p->n[2] * p->nc * 8;
}

int x_grid_blocks(const lf2_plan_s *p)
{
    const int rb = p->gen[0] ? p->gen_rb : x_rows_per_block(p->len[0], p->nc);
    return (int)((p->n[1] * p->n[2] + rb - 1) / rb);
}

// Workspace layout: [W spectrum][pk partials][bin sums][sumsq partials][sumsq]
struct WsLayout {
    size_t w, part, sums, sq, sqt, total;
};

WsLayout ws_layout(const lf2_plan_s *p, bool need_w, int nbins, bool parseval)
{
    WsLayout l{};
    size_t off = 0;
    l.w = off;
    off += need_w ? align256(spectrum_bytes(p)) : 0;
    l.part = off;
    off += nbins > 0 ? align256((size_t)kPkGrid * (nbins + 1) * 8) : 0;
    l.sums = off;
    off += nbins > 0 ? align256((size_t)(nbins + 1) * 8) : 0;
    l.sq = off;
    off += parseval ? align256((size_t)x_grid_blocks(p) * 8) : 0;
    l.sqt = off;
    off += parseval ? 256 : 0;
    l.total = off;
    return l;
}

lf2_status get_workspace(lf2_plan p, size_t need, char **out)
{
    if (need == 0) {
        *out = nullptr;
        return LF2_OK;
    }
    if (p->own_ws) {
        if (p->own_ws_bytes < need)
            return fail(LF2_ERR_INVALID_ARG, "plan workspace of %zu bytes is smaller than the %zu needed",
                        p->own_ws_bytes, need);
        *out = (char *)p->own_ws;
        return LF2_OK;
    }
    SharedWs &ws = g_ws[p->device];
    std::lock_guard<std::mutex> lk(ws.mu);
    if (ws.bytes < need) {
        if (ws.ptr) {
            LF2_HIP(hipDeviceSynchronize());
            LF2_HIP(hipFree(ws.ptr));
            ws.ptr = nullptr;
            ws.bytes = 0;
        }
        void *ptr = nullptr;
        hipError_t e = hipMalloc(&ptr, need);
        if (e != hipSuccess)
            return fail(LF2_ERR_OUT_OF_MEMORY, "workspace hipMalloc(%zu) failed: %s", need,
                        hipGetErrorString(e));
        ws.ptr = ptr;
        ws.bytes = need;
    }
    *out = (char *)ws.ptr;
    return LF2_OK;
}

lf2_status check_device(const lf2_plan_s *p)
{
    int dev = -1;
    LF2_HIP(hipGetDevice(&dev));
    if (dev != p->device)
        return fail(LF2_ERR_INVALID_ARG, "plan was made on device %d but device %d is current",
                    p->device, dev);
    return LF2_OK;
}

ModeTables base_tables(const lf2_plan_s *p)
{
    ModeTables mt{};
    mt.nxk = (int)p->nxk;
    mt.n0 = (int)p->n[0];
    mt.n1 = (int)p->n[1];
    mt.half = p->kind == LF2_R2C ? 1 : 0;
    for (int i = 0; i < 3; ++i) {
        mt.k2[i] = nullptr;
        mt.q[i] = p->q[i];
    }
    mt.thresh = nullptr;
    mt.nbins = 0;
    mt.qmax = (double)p->qmax;
    mt.scale_n = 1.0 / (double)p->ntot;
    // below 2^32 whenever N2 > 1 (it is then at most qmax); unused for N2 = 1
    const int64_t uz = p->lcm / p->n[2];
    mt.qz_unit = (uint32_t)(uz * uz);
    // (lcm / N_i)^2 <= qmax < 2^32 for N_i > 1; m = 0 only along N_i = 1
    const int64_t ux = p->lcm / p->n[0], uy = p->lcm / p->n[1];
    mt.qx_unit = (uint32_t)(ux * ux);
    mt.qy_unit = (uint32_t)(uy * uy);
    mt.k2z_unit = mt.k2x_unit = mt.k2y_unit = 0.0;
    return mt;
}

void set_k2_units(ModeTables &mt, const lf2_plan_s *p, double dx, int discrete)
{
    double u[3] = {0.0, 0.0, 0.0};
    if (!discrete)
        for (int i = 0; i < 3; ++i) {
            const double a = 6.283185307179586476925286766559 / ((double)p->n[i] * dx);
            u[i] = a * a;
        }
    mt.k2x_unit = u[0];
    mt.k2y_unit = u[1];
    mt.k2z_unit = u[2];
}

lf2_status get_k2(lf2_plan p, double dx, int discrete, hipStream_t s, const double *out[3],
                  bool lookup_only)
{
    for (auto &e : p->k2)
        if (e.dx == dx && e.discrete == discrete) {
            for (int i = 0; i < 3; ++i) out[i] = e.tab[i];
            return LF2_OK;
        }
    if (lookup_only)
        return fail(LF2_ERR_NOT_READY,
                    "no k^2 table for dx = %g (%s) on this plan yet: an allocating call with "
                    "these arguments builds it", dx, discrete ? "discrete" : "continuous");
    K2Entry e{dx, discrete, {nullptr, nullptr, nullptr}};
    const int64_t cnt[3] = {p->nxk, p->n[1], p->n[2]};
    for (int i = 0; i < 3; ++i) {
        void *ptr;
        lf2_status st = plan_alloc(p, &ptr, (size_t)cnt[i] * 8);
        if (st) return st;
        e.tab[i] = (double *)ptr;
        LF2_HIP(launch_k2_table(e.tab[i], (int)p->n[i], (int)cnt[i], dx, discrete, s));
    }
    p->k2.push_back(e);
    for (int i = 0; i < 3; ++i) out[i] = e.tab[i];
    return LF2_OK;
}

// Whether one step of m = |n_z| (q_xy + m^2 q_u to q_xy + (m + 1)^2 q_u)
// crosses at most one of the thresholds t_1 .. t_{nbins-1}.  A step from
// q < t_b has m^2 q_u <= q < t_b, so it moves q by (2 m + 1) q_u <
// 2 sqrt(t_b q_u) + q_u; if every gap t_{b+1} - t_b is at least that (plus
// one for the rounding of the square root), no step spans two thresholds.
static bool walk_one_step(const std::vector<int64_t> &t, uint32_t qu)
{
    const int nb = (int)t.size() - 1;
    for (int b = 0; b + 1 <= nb - 1; ++b) {
        const double need = 2.0 * std::sqrt((double)t[b] * (double)qu) + (double)qu + 1.0;
        if ((double)(t[b + 1] - t[b]) < need) return false;
    }
    return true;
}

lf2_status get_shell(lf2_plan p, int nbins, hipStream_t s, ShellEntry *out, bool lookup_only)
{
    for (auto &e : p->shells)
        if (e.nbins == nbins) {
            *out = e;
            return LF2_OK;
        }
    if (lookup_only)
        return fail(LF2_ERR_NOT_READY,
                    "no %d-bin shell table on this plan yet: an allocating call with this bin "
                    "count builds it", nbins);
    ShellEntry e{nbins, nullptr, nullptr, nullptr, 0};
    void *ptr;
    lf2_status st = plan_alloc(p, &ptr, (size_t)(nbins + 1) * 8);
    if (st) return st;
    e.thresh = (int64_t *)ptr;
    if ((st = plan_alloc(p, &ptr, (size_t)nbins * 8))) return st;
    e.count = (double *)ptr;
    if ((st = plan_alloc(p, &ptr, (size_t)nbins * 8))) return st;
    e.sumk = (double *)ptr;
    LF2_HIP(launch_thresholds(e.thresh, nbins, p->qmax, s));
    // shell sums over the lattice (plan-time work, kept with the plan)
    const int grid = 512;
    double *pc = nullptr, *pkk = nullptr;
    LF2_HIP(hipMalloc(&pc, (size_t)grid * nbins * 8));
    hipError_t e2 = hipMalloc(&pkk, (size_t)grid * nbins * 8);
    if (e2 != hipSuccess) {
        (void)hipFree(pc);
        return fail(LF2_ERR_OUT_OF_MEMORY, "hipMalloc failed: %s", hipGetErrorString(e2));
    }
    ModeTables mt = base_tables(p);
    mt.thresh = e.thresh;
    mt.nbins = nbins;
    mt.walk1 = 0;
    hipError_t e3 = launch_shell_partials(mt, (int)p->n[1], (int)p->n[2], 0.0, pc, pkk, grid, s);
    if (e3 == hipSuccess) e3 = launch_reduce_cols(pc, grid, nbins, e.count, s);
    if (e3 == hipSuccess) e3 = launch_reduce_cols(pkk, grid, nbins, e.sumk, s);
    if (e3 == hipSuccess) e3 = hipStreamSynchronize(s);
    (void)hipFree(pc);
    (void)hipFree(pkk);
    if (e3 != hipSuccess) return fail(LF2_ERR_DEVICE, "shell table: %s", hipGetErrorString(e3));
    std::vector<int64_t> th((size_t)nbins + 1);
    LF2_HIP(hipMemcpy(th.data(), e.thresh, th.size() * 8, hipMemcpyDeviceToHost));
    e.walk1 = walk_one_step(th, mt.qz_unit) ? 1 : 0;
    p->shells.push_back(e);
    *out = e;
    return LF2_OK;
}

lf2_status check_ptr(const void *ptr, const char *what, size_t align)
{
    if (!ptr) return fail(LF2_ERR_INVALID_ARG, "%s is NULL", what);
    if (((uintptr_t)ptr) % align)
        return fail(LF2_ERR_INVALID_ARG, "%s is not %zu-byte aligned", what, align);
    return LF2_OK;
}

// ------------------------------------------------------------- pass runners

XArgs x_args(const lf2_plan_s *p, const void *in, void *out, bool in_is_x, bool out_is_x,
             bool real_x)
{
    // x-space arrays carry the halo; k-space arrays do not.  Units are the
    // array's elements: floats for real fields, complex for complex ones.
    XArgs a{};
    a.in = in;
    a.out = out;
    a.nrows = p->n[1] * p->n[2];
    a.n1 = (int)p->n[1];
    const int64_t h = p->halo, nc = p->nc;
    // in-place r2c: real rows padded to the spectrum row's 2 Nh floats
    const int64_t xrow = (p->inplace && p->kind == LF2_R2C) ? 2 * p->nh * nc : (p->n[0] + 2 * h) * nc;
    const int64_t xplane = (p->n[1] + 2 * h) * xrow;
    const int64_t xoff = h * nc + h * xrow + h * xplane;
    // k-space rows: natural [N2][N1][Nk]; the paper's r2c order [N1][N2][Nh]
    const int64_t C1 = p->nxk * nc;
    const int64_t krow = p->klay == 1 ? p->n[2] * C1 : C1, kplane = p->klay == 1 ? C1 : p->n[1] * C1;
    (void)real_x;
    if (in_is_x) {
        a.in_off = xoff;
        a.in_row = xrow;
        a.in_plane = xplane;
    } else {
        a.in_off = 0;
        a.in_row = krow;
        a.in_plane = kplane;
    }
    if (out_is_x) {
        a.out_off = xoff;
        a.out_row = xrow;
        a.out_plane = xplane;
    } else {
        a.out_off = 0;
        a.out_row = krow;
        a.out_plane = kplane;
    }
    a.tw = p->tw[0];
    a.tw_post = p->tw_post;
    a.sumsq = nullptr;
    return a;
}

SArgs s_args(const lf2_plan_s *p, int axis, const void *in, void *out, int epi)
{
    SArgs a{};
    a.in = in;
    a.out = out;
    const int64_t C1 = p->nxk * p->nc;
    if (p->klay == 1) {  // r2c in the paper's order [N1][N2][Nh]
        if (axis == 1) {  // y is the slowest dimension; every (k_x, z) column is contiguous
            a.stride = p->n[2] * C1;
            a.ncols_inner = p->n[2] * C1;
            a.outer = 0;
            a.ncols = p->n[2] * C1;
        } else {  // z jumps a row; columns (k_x, y): column f at (f / C1) N2 C1 + f mod C1
            a.stride = C1;
            a.ncols_inner = C1;
            a.outer = p->n[2] * C1;
            a.ncols = p->n[1] * C1;
        }
    } else if (axis == 1) {
        a.stride = C1;
        a.ncols_inner = C1;
        a.outer = p->n[1] * C1;
        a.ncols = p->n[2] * C1;
    } else {
        a.stride = p->n[1] * C1;
        a.ncols_inner = p->n[1] * C1;
        a.outer = 0;
        a.ncols = p->n[1] * C1;
    }
    a.epi = epi;
    a.tw = p->tw[axis];
    a.mt = base_tables(p);
    a.partial = nullptr;
    return a;
}

// z pass between the natural order and the paper's c2c order
SArgs t_args(const lf2_plan_s *p, const void *in, void *out, int epi)
{
    SArgs a = s_args(p, 2, in, out, epi);
    a.t_n0 = p->n[0];
    a.t_n2 = p->n[2];
    a.t_nc = p->nc;
    return a;
}

lf2_status run_strided(const lf2_plan_s *p, int axis, int sign, const SArgs &a, int grid_cap,
                       hipStream_t s, int *grid_used)
{
    const double sb = (double)spectrum_bytes(p);
    const bool epi = (a.epi & (EPI_PK | EPI_PK_AFTER | EPI_POISSON)) != 0;
    const bool tr = (a.epi & (EPI_TSTORE | EPI_TLOAD)) != 0;
    // run-time schedule: lengths without compiled kernels, and plain passes
    // whose tuned schedule beat the compiled kernels
    if (p->gen_only[axis] || (p->gen[axis] && !epi)) {
        if (tr)
            return fail(LF2_ERR_UNSUPPORTED, "no transposing pass for line length %d", p->len[axis]);
        const bool pk = (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
        const int b = gs_cols(p, p->len[axis], pk ? a.mt.nbins : 0);
        if (b < 1)
            return fail(LF2_ERR_UNSUPPORTED, "line length %d with %d bins does not fit a tile",
                        p->len[axis], pk ? a.mt.nbins : 0);
        const int t = prof::begin(kname("k_gs<%d,%d> %s%s%s %lldx%lldx%lld/%d", sign, epi ? 1 : 0,
                                        axis == 1 ? "y" : "z",
                                        (a.epi & EPI_POISSON) ? "+poisson" : "", pk ? "+pk" : "",
                                        (long long)p->n[0], (long long)p->n[1], (long long)p->n[2],
                                        p->nc),
                                  (a.epi & EPI_STORE) ? 2 * sb : sb, s);
        hipError_t e = launch_gs(sign, a, p->sched[axis], p->len[axis], b, grid_cap, s, grid_used);
        prof::end(t, s);
        if (e != hipSuccess)
            return fail(LF2_ERR_DEVICE, "strided pass (axis %d, L=%d) launch: %s", axis,
                        p->len[axis], hipGetErrorString(e));
        return LF2_OK;
    }
    const bool freg = epi && sign < 0 && (a.epi & EPI_POISSON) && p->fvar == 1 &&
                      fused_reg_supported(p->len[axis]) &&
                      fused_reg_fits(p->len[axis], (a.epi & (EPI_PK | EPI_PK_AFTER)) ? a.mt.nbins : 0);
    const int variant = tr ? 0 : epi ? (freg ? 8 : 0) : p->svar[axis];
    const int ntm = ((variant & 2) || epi) ? 1 : 0;  // the fused pass always streams
    // "<kernel symbol> <pass>": the symbol part matches the profiler's name
    const std::string sym = tr ? kname("k_strided_t<%d,%d>", p->len[axis], sign)
                            : freg ? kname("k_fused_r<%d,%d>", p->len[axis], a.mt.k2z_unit > 0.0 ? 1 : 2)
                            : (variant & 1) ? kname("k_strided_w<%d,%d,%d>", p->len[axis], sign, ntm)
                            : (variant & 4) ? kname("k_strided_r<%d,%d,%d>", p->len[axis], sign, ntm)
                                            : kname("k_strided<%d,%d,%d,%d>", p->len[axis], sign,
                                                    epi ? 1 : 0, ntm);
    const int t = prof::begin(sym + kname(" %s%s%s %lldx%lldx%lld/%d", axis == 1 ? "y" : "z",
                                    (a.epi & EPI_POISSON) ? "+poisson" : "",
                                    (a.epi & (EPI_PK | EPI_PK_AFTER)) ? "+pk" : "",
                                    (long long)p->n[0], (long long)p->n[1], (long long)p->n[2], p->nc),
                              (a.epi & EPI_STORE) ? 2 * sb : sb, s);
    hipError_t e = launch_strided(p->len[axis], sign, a, grid_cap, s, grid_used, variant,
                                  epi ? 16 : p->schunk[axis]);
    prof::end(t, s);
    if (e != hipSuccess)
        return fail(LF2_ERR_DEVICE, "strided pass (axis %d, L=%d) launch: %s", axis, p->len[axis],
                    hipGetErrorString(e));
    return LF2_OK;
}

lf2_status run_x(const lf2_plan_s *p, int which, int sign, const XArgs &a, hipStream_t s)
{
    hipError_t e;
    const double rb = (double)p->ntot * p->nc * 4.0;  // real field
    const double sb = (double)spectrum_bytes(p);
    int t;
    // the same layout test the launchers apply to pick the paired fast kernels
    auto paired = [](const void *q, int64_t off, int64_t row, int64_t plane) {
        return ((uintptr_t)q % 8) == 0 && off % 2 == 0 && row % 2 == 0 && plane % 2 == 0;
    };
    const std::string shape = kname(" %lldx%lldx%lld/%d", (long long)p->n[0], (long long)p->n[1],
                                    (long long)p->n[2], p->nc);
    if (p->gen[0]) {
        static const char *const kModes[] = {"r2c", "c2r", "c2c"};
        const int mode = which == 0 ? 1 : which == 1 ? 2 : 0;
        t = prof::begin(kname("k_gx<%s>", kModes[which]) + shape, which == 2 ? 2 * sb : rb + sb, s);
        e = launch_gx(mode, sign, a, p->sched[0], p->len[0], p->nc, p->gen_rb, s);
        prof::end(t, s);
        if (e != hipSuccess)
            return fail(LF2_ERR_DEVICE, "x pass (L=%d) launch: %s", p->len[0], hipGetErrorString(e));
        return LF2_OK;
    }
    if (which == 0) {
        const bool v = p->nc == 1 && paired(a.in, a.in_off, a.in_row, a.in_plane);
        t = prof::begin((v ? kname("k_x_r2c_v<%d>", p->len[0]) : kname("k_x_r2c<%d,%d>", p->len[0], p->nc)) + shape,
                        rb + sb, s);
        e = launch_x_r2c(p->len[0], p->nc, a, s);
    } else if (which == 1) {
        const bool v = p->nc == 1 && paired(a.out, a.out_off, a.out_row, a.out_plane);
        t = prof::begin((v ? kname("k_x_c2r_v<%d>", p->len[0]) : kname("k_x_c2r<%d,%d>", p->len[0], p->nc)) + shape,
                        rb + sb, s);
        e = launch_x_c2r(p->len[0], p->nc, a, s);
    } else if (p->xx) {
        t = prof::begin(kname("k_x_c2c_s64<%s,%d>", p->xx == 2 ? "dpp" : "bpermute", sign) + shape,
                        2 * sb, s);
        e = launch_x_c2c_shfl(sign, p->xx == 2, a, s);
    } else {
        t = prof::begin(kname("k_x_c2c_v<%d,%d,%d>", p->len[0], p->nc, sign) + shape, 2 * sb, s);
        e = launch_x_c2c(p->len[0], p->nc, sign, a, s);
    }
    prof::end(t, s);
    if (e != hipSuccess)
        return fail(LF2_ERR_DEVICE, "x pass (L=%d) launch: %s", p->len[0], hipGetErrorString(e));
    return LF2_OK;
}

// Binning tail: reduce partials, finalize into the caller's arrays.
// sq_part (nullable): sq_rows per-block sums of squares of the real field,
// reduced into *sq_total in the same launch as the bin partials.
lf2_status pk_tail(lf2_plan p, const ShellEntry &sh, double *part, int grid, double *sums,
                   double dx, double vscale, double *d_pk, double *d_kmean, double *d_count,
                   double *d_parseval, const double *sq_part, int64_t sq_rows, double *sq_total,
                   hipStream_t s)
{
    const int nb = sh.nbins;
    LF2_HIP(launch_reduce_cols2(part, grid, nb + 1, sums, sq_part, sq_rows, sq_part ? 1 : 0,
                                sq_total, s));
    const double *sumsq_total = sq_part ? sq_total : nullptr;
    const double norm = dx * dx * dx / (double)p->ntot;
    const double kscale = 6.283185307179586476925286766559 / ((double)p->lcm * dx);
    LF2_HIP(launch_pk_finalize(sums, nb, sh.count, sh.sumk, norm, vscale, kscale, d_pk, d_kmean,
                               d_count, d_parseval, sumsq_total, 1.0 / (double)p->ntot, s));
    return LF2_OK;
}

lf2_status check_bins(const lf2_plan_s *p, int32_t nbins)
{
    if (nbins < 0) return fail(LF2_ERR_INVALID_ARG, "nbins %d < 0", nbins);
    if (nbins > kMaxBins) return fail(LF2_ERR_UNSUPPORTED, "nbins %d > %d", nbins, kMaxBins);
    if (nbins > 0) {
        // nbins^2 * qmax must fit the exact integer bin rule
        long double lim = (long double)nbins * nbins * (long double)p->qmax;
        if (lim > 4.0e18L) return fail(LF2_ERR_UNSUPPORTED, "nbins^2 * qmax overflows the integer bin rule");
    }
    return LF2_OK;
}

}  // namespace host
}  // namespace lf2

using namespace lf2::host;

// ===================================================================== C ABI

extern "C" {

const char *lf2_status_string(lf2_status s)
{
    switch (s) {
    case LF2_OK: return "LF2_OK";
    case LF2_ERR_INVALID_ARG: return "LF2_ERR_INVALID_ARG";
    case LF2_ERR_UNSUPPORTED: return "LF2_ERR_UNSUPPORTED";
    case LF2_ERR_OUT_OF_MEMORY: return "LF2_ERR_OUT_OF_MEMORY";
    case LF2_ERR_DEVICE: return "LF2_ERR_DEVICE";
    case LF2_ERR_BUDGET: return "LF2_ERR_BUDGET";
    case LF2_ERR_BUSY: return "LF2_ERR_BUSY";
    case LF2_ERR_NOT_READY: return "LF2_ERR_NOT_READY";
    }
    return "LF2_ERR_UNKNOWN";
}

const char *lf2_last_error(void) { return g_err.c_str(); }

lf2_status lf2_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::reset();
    prof::on = on != 0;
    return LF2_OK;
}

lf2_status lf2_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::reset();
    return LF2_OK;
}

int32_t lf2_profile_count(void)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    prof::drain();
    return (int32_t)prof::names.size();
}

lf2_status lf2_profile_get(int32_t i, char *name, size_t name_len, int64_t *launches, double *ms,
                           double *bytes)
{
    std::lock_guard<std::mutex> lk(prof::mu);
    if (i < 0 || i >= (int32_t)prof::names.size())
        return fail(LF2_ERR_INVALID_ARG, "profile index %d out of range", i);
    if (name && name_len > 0) {
        strncpy(name, prof::names[i].c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    if (launches) *launches = prof::agg[i].n;
    if (ms) *ms = prof::agg[i].ms;
    if (bytes) *bytes = prof::agg[i].bytes;
    return LF2_OK;
}

const char *lf2_version(void) { return "lf2 0.1.0 gfx950"; }

}  // extern "C"

namespace {

// Whether the x pass can exchange across lanes: c2c rows of 64 points, one
// component, compiled kernels.
bool x_lane_exchange_ok(const lf2_plan_s *p)
{
    return p->kind == LF2_C2C && p->len[0] == 64 && p->nc == 1 && !p->gen[0] && !p->gen_only[0];
}

// Time the x pass's stage exchange (64-point c2c rows: LDS or across
// lanes), the tile variants and XCD chunk sizes of the y and z passes, and the
// candidate radix schedules of the run-time-schedule kernels (every axis
// without a compiled kernel, and the y and z passes as an alternative to
// the compiled ones), on a scratch spectrum of the plan's shape (one
// warm-up, then the mean of three launches each; the compiled tile settings
// of the y and z passes in two sweeps, each keeping its faster time), and
// keep the fastest, the default (compiled narrow tiles, chunk 16, or the
// first schedule) first.
// Without memory for the scratch spectrum the defaults stay.
lf2_status autotune(lf2_plan p)
{
    const size_t bytes = spectrum_bytes(p);
    void *w = nullptr, *w2 = nullptr;
    if (hipMalloc(&w, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return LF2_OK;
    }
    if ((p->gen_only[0] || x_lane_exchange_ok(p)) && hipMalloc(&w2, bytes) != hipSuccess) {
        (void)hipGetLastError();
        w2 = nullptr;
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lf2_status st = LF2_OK;
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && st == LF2_OK) st = fail(LF2_ERR_DEVICE, "autotune %s: %s", what, hipGetErrorString(e));
        return st == LF2_OK;
    };
    // mean microseconds of three launches after a warm-up (-1 on failure)
    auto time_it = [&](auto &&launch) -> double {
        hip_ok(launch(), "launch");
        hip_ok(hipEventRecord(e0, s), "record");
        for (int r = 0; r < 3; ++r) hip_ok(launch(), "launch");
        hip_ok(hipEventRecord(e1, s), "record");
        float ms = 0.f;
        if (!hip_ok(hipEventSynchronize(e1), "sync") || !hip_ok(hipEventElapsedTime(&ms, e0, e1), "elapsed"))
            return -1.0;
        return 1e3 * ms / 3.0;
    };
    static const int kChunks[] = {16, 4, 64};  // the default first
    if (hip_ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream") &&
        hip_ok(hipEventCreate(&e0), "event") && hip_ok(hipEventCreate(&e1), "event") &&
        hip_ok(hipMemsetAsync(w, 0, bytes, s), "memset") &&
        (!w2 || hip_ok(hipMemsetAsync(w2, 0, bytes, s), "memset"))) {
        // x axis without a compiled kernel: its schedules, on dense rows
        if (p->gen_only[0] && w2) {
            XArgs a{};
            a.nrows = p->n[1] * p->n[2];
            a.n1 = (int)p->n[1];
            a.tw = p->tw[0];
            a.tw_post = p->tw_post;
            const int64_t c1 = p->nxk * p->nc;
            const int64_t xr = p->n[0] * p->nc;  // floats (r2c) or complex (c2c) per row
            a.in = w;
            a.out = w2;
            a.in_row = xr;
            a.in_plane = xr * p->n[1];
            a.out_row = c1;
            a.out_plane = c1 * p->n[1];
            const int mode = p->kind == LF2_R2C ? 1 : 0;
            double best = -1.0;
            for (const GSched &sc : sched_candidates(p->len[0])) {
                if (st != LF2_OK) break;
                const double us = time_it([&] {
                    return launch_gx(mode, -1, a, sc, p->len[0], p->nc, p->gen_rb, s);
                });
                if (p->tune_us[0][0] < 0) p->tune_us[0][0] = us;
                if (us >= 0 && (best < 0 || us < 0.97 * best)) {
                    best = us;
                    p->sched[0] = sc;
                }
            }
            p->tune_us[0][1] = best;
        }
        // 64-point c2c rows: the stage exchange through LDS or across lanes
        if (x_lane_exchange_ok(p) && w2) {
            XArgs a{};
            a.nrows = p->n[1] * p->n[2];
            a.n1 = (int)p->n[1];
            a.tw = p->tw[0];
            a.in = w;
            a.out = w2;
            a.in_row = a.out_row = p->n[0];
            a.in_plane = a.out_plane = p->n[0] * p->n[1];
            double best = -1.0;
            for (int v = 0; v < 3 && st == LF2_OK; ++v) {
                const double us = time_it([&] {
                    return v == 0 ? launch_x_c2c(64, 1, -1, a, s) : launch_x_c2c_shfl(-1, v == 2, a, s);
                });
                if (v == 0) p->tune_us[0][0] = us;
                if (us >= 0 && (best < 0 || us < 0.97 * best)) {
                    best = us;
                    p->xx = v;
                }
            }
            p->tune_us[0][1] = best;
        }
        for (int axis = 1; axis <= 2 && st == LF2_OK; ++axis) {
            const bool wide = !p->gen_only[axis] && s_wide_supported(p->len[axis]);
            const bool reg = !p->gen_only[axis] && s_reg_supported(p->len[axis]);
            const SArgs a = s_args(p, axis, w, w, EPI_STORE);
            double best = -1.0;
            if (!p->gen_only[axis]) {
                // two sweeps over the settings, each setting keeping its
                // faster time: a setting timed while the chip's clocks or
                // memory state drift is timed again in the other sweep
                // Order: the default first, then the nontemporal settings,
                // then the rest; within 3 % the earlier one stays.  Timed in
                // short bursts, the cached-store settings of long-stride passes
                // come out faster than they run inside a transform (the
                // 3-component 512^3 z pass: plain wide tile 1.35-1.37 ms in the
                // tuner, 1.53-1.67 ms in the transforms; nontemporal wide tile
                // 1.33 ms and 1.40-1.42 ms), so ties go to the streaming ones.
                std::vector<std::pair<int, int>> cfg{{0, 16}};
                for (int pass = 0; pass < 2; ++pass)
                    for (int v = 0; v < 8; ++v) {
                        if (((v & 2) != 0) != (pass == 0)) continue;
                        if ((v & 1) && !wide) continue;
                        if ((v & 4) && (!reg || (v & 1))) continue;
                        for (int c : kChunks)
                            if (v != 0 || c != 16) cfg.emplace_back(v, c);
                    }
                std::vector<double> t(cfg.size(), -1.0);
                for (int sweep = 0; sweep < 2 && st == LF2_OK; ++sweep)
                    for (size_t i = 0; i < cfg.size() && st == LF2_OK; ++i) {
                        const double us = time_it([&] {
                            return launch_strided(p->len[axis], -1, a, kStridedGridCap, s, nullptr,
                                                  cfg[i].first, cfg[i].second);
                        });
                        if (us >= 0 && (t[i] < 0 || us < t[i])) t[i] = us;
                    }
                for (size_t i = 0; i < cfg.size(); ++i) {
                    if (t[i] < 0) continue;
                    if (i == 0) p->tune_us[axis][0] = t[i];  // variant 0, chunk 16
                    // another setting must beat the current choice by 3 %, so
                    // that timing noise does not flip the choice from run to run
                    if (best < 0 || t[i] < 0.97 * best) {
                        best = t[i];
                        p->svar[axis] = cfg[i].first;
                        p->schunk[axis] = cfg[i].second;
                    }
                }
            }
            const int b = gs_cols(p, p->len[axis], 0);
            for (const GSched &sc : sched_candidates(p->len[axis])) {
                if (st != LF2_OK || b < 1) break;
                const double us = time_it([&] {
                    return launch_gs(-1, a, sc, p->len[axis], b, kStridedGridCap, s, nullptr);
                });
                if (p->tune_us[axis][0] < 0) p->tune_us[axis][0] = us;
                if (us >= 0 && (best < 0 || us < 0.97 * best)) {
                    best = us;
                    p->gen[axis] = true;
                    p->sched[axis] = sc;
                }
            }
            p->tune_us[axis][1] = best;
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(w);
    if (w2) (void)hipFree(w2);
    return st;
}

}  // namespace

extern "C" {

lf2_status lf2_fft_plan(lf2_plan *out, const lf2_lattice *lat, int32_t ncomp, lf2_fft_kind kind,
                        uint32_t flags)
{
    if (!out) return fail(LF2_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!lat) return fail(LF2_ERR_INVALID_ARG, "lattice is NULL");
    if (lat->dim != 3) return fail(LF2_ERR_UNSUPPORTED, "dim %d: only 3-d lattices have an FFT", lat->dim);
    if (lat->halo < 0) return fail(LF2_ERR_INVALID_ARG, "halo %d < 0", lat->halo);
    if (kind != LF2_R2C && kind != LF2_C2C) return fail(LF2_ERR_INVALID_ARG, "bad kind %d", (int)kind);
    if (ncomp < 1) return fail(LF2_ERR_INVALID_ARG, "ncomp %d < 1", ncomp);
    if (flags & ~(LF2_PLAN_AUTOTUNE | LF2_IN_PLACE | LF2_KLAYOUT_PAPER))
        return fail(LF2_ERR_UNSUPPORTED, "plan flags 0x%x not supported", flags);
    if ((flags & LF2_IN_PLACE) && lat->halo != 0)
        return fail(LF2_ERR_UNSUPPORTED, "in-place transforms need halo 0");
    for (int i = 0; i < 3; ++i) {
        if (lat->size[i] < 1) return fail(LF2_ERR_INVALID_ARG, "size[%d] = %lld < 1", i, (long long)lat->size[i]);
        if (lat->size[i] > (1 << 20)) return fail(LF2_ERR_UNSUPPORTED, "size[%d] too large", i);
        if (!gen_factorable(lat->size[i]))
            return fail(LF2_ERR_UNSUPPORTED, "size[%d] = %lld must be 2^a 3^b 5^c", i,
                        (long long)lat->size[i]);
    }
    if (kind == LF2_R2C && lat->size[0] % 2)
        return fail(LF2_ERR_UNSUPPORTED, "r2c needs an even size[0] (got %lld)", (long long)lat->size[0]);
    int lens[3] = {(int)(kind == LF2_R2C ? lat->size[0] / 2 : lat->size[0]), (int)lat->size[1],
                   (int)lat->size[2]};
    bool gen_only[3];
    for (int i = 0; i < 3; ++i) {
        gen_only[i] = i == 0 ? !x_supported(lens[0], ncomp) : !s_supported(lens[i]);
        if (gen_only[i] && lens[i] > kGenMaxLen)
            return fail(LF2_ERR_UNSUPPORTED, "line length %d along dimension %d is longer than %d",
                        lens[i], i, kGenMaxLen);
    }
    if (gen_only[2] && (flags & LF2_KLAYOUT_PAPER) && kind == LF2_C2C)
        return fail(LF2_ERR_UNSUPPORTED, "the c2c paper k-space order needs a compiled z length");

    lf2_plan p = new (std::nothrow) lf2_plan_s();
    if (!p) return fail(LF2_ERR_OUT_OF_MEMORY, "plan allocation");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess || p->device < 0 || p->device >= kMaxDevices) {
        delete p;
        return fail(LF2_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) ==
            hipSuccess &&
        lds > 0)
        p->lds_max = (size_t)lds;
    // compiled kernels where they exist; run-time radix schedules otherwise
    for (int i = 0; i < 3; ++i) {
        p->gen_only[i] = gen_only[i];
        p->gen[i] = gen_only[i];
        const std::vector<GSched> cand = sched_candidates(lens[i]);
        if (!cand.empty()) p->sched[i] = cand[0];
    }
    // the fused Poisson pass keeps its tile in registers where it can (at 32
    // points the LDS-staged tile is as fast)
    p->fvar = fused_reg_supported(lens[2]) && lens[2] >= 64 ? 1 : 0;
    if (p->gen_only[0] && (p->gen_rb = gx_rows(p, lens[0], ncomp)) < 1) {
        delete p;
        return fail(LF2_ERR_UNSUPPORTED, "x lines of %d points with %d components do not fit a tile",
                    lens[0], ncomp);
    }
    for (int i = 1; i < 3; ++i)
        if (p->gen_only[i] && gs_cols(p, lens[i], 0) < 1) {
            delete p;
            return fail(LF2_ERR_UNSUPPORTED, "strided lines of %d points do not fit a tile", lens[i]);
        }

    p->kind = kind;
    p->nc = ncomp;
    p->halo = lat->halo;
    p->flags = flags;
    p->inplace = (flags & LF2_IN_PLACE) != 0;
    p->klay = (flags & LF2_KLAYOUT_PAPER) ? (kind == LF2_R2C ? 1 : 2) : 0;
    for (int i = 0; i < 3; ++i) {
        p->n[i] = lat->size[i];
        p->len[i] = lens[i];
    }
    p->nh = p->n[0] / 2 + 1;
    p->nxk = kind == LF2_R2C ? p->nh : p->n[0];
    p->ntot = p->n[0] * p->n[1] * p->n[2];
    p->lcm = p->n[0];
    p->lcm = p->lcm / gcd64(p->lcm, p->n[1]) * p->n[1];
    p->lcm = p->lcm / gcd64(p->lcm, p->n[2]) * p->n[2];
    p->qmax = 0;
    for (int i = 0; i < 3; ++i) {
        int64_t a = (p->n[i] / 2) * (p->lcm / p->n[i]);
        p->qmax += a * a;
    }
    hipStream_t s = nullptr;
    lf2_status st = LF2_OK;
    // the fused binning evaluates the bin rule in 32 x 32 -> 64-bit products
    // (qmax < 7.1e8 for every supported line length)
    if (p->qmax >= ((int64_t)1 << 32))
        st = fail(LF2_ERR_UNSUPPORTED, "lattice too large for the exact bin rule");
    for (int i = 0; i < 3 && st == LF2_OK; ++i) {
        st = plan_alloc(p, &p->tw[i], (size_t)p->len[i] * 8);
        if (st == LF2_OK && launch_twiddles(p->tw[i], p->len[i], s) != hipSuccess)
            st = fail(LF2_ERR_DEVICE, "twiddle kernel launch");
    }
    if (st == LF2_OK && kind == LF2_R2C) {
        st = plan_alloc(p, &p->tw_post, (size_t)p->nh * 8);
        if (st == LF2_OK && launch_twiddles(p->tw_post, -(int)p->n[0], s) != hipSuccess)
            st = fail(LF2_ERR_DEVICE, "twiddle kernel launch");
    }
    const int64_t cnt[3] = {p->nxk, p->n[1], p->n[2]};
    for (int i = 0; i < 3 && st == LF2_OK; ++i) {
        void *ptr = nullptr;
        st = plan_alloc(p, &ptr, (size_t)cnt[i] * 8);
        p->q[i] = (int64_t *)ptr;
        if (st == LF2_OK && launch_q_table(p->q[i], (int)p->n[i], (int)cnt[i], p->lcm / p->n[i], s) != hipSuccess)
            st = fail(LF2_ERR_DEVICE, "q table launch");
    }
    if (st == LF2_OK) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) st = fail(LF2_ERR_DEVICE, "plan setup: %s", hipGetErrorString(e));
    }
    if (st == LF2_OK && (flags & LF2_PLAN_AUTOTUNE)) st = autotune(p);
    if (st != LF2_OK) {
        lf2_plan_destroy(p);
        return st;
    }
    *out = p;
    return LF2_OK;
}

lf2_status lf2_plan_get_tuning(lf2_plan p, int32_t axis, int32_t *variant, int32_t *chunk,
                               double *us_default, double *us_tuned)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (axis < 0 || axis > 3) return fail(LF2_ERR_INVALID_ARG, "axis %d is not 0, 1, 2 or 3", axis);
    if (axis == 3) {
        if (variant) *variant = p->fvar;
        if (chunk) *chunk = 16;
        if (us_default) *us_default = -1.0;
        if (us_tuned) *us_tuned = -1.0;
        return LF2_OK;
    }
    if (axis == 0) {
        if (variant) *variant = p->gen[0] ? -1 : p->xx;
        if (chunk) *chunk = 0;
        if (us_default) *us_default = p->tune_us[0][0];
        if (us_tuned) *us_tuned = p->tune_us[0][1];
        return LF2_OK;
    }
    if (variant) *variant = p->gen[axis] ? -1 : p->svar[axis];
    if (chunk) *chunk = p->schunk[axis];
    if (us_default) *us_default = p->tune_us[axis][0];
    if (us_tuned) *us_tuned = p->tune_us[axis][1];
    return LF2_OK;
}

lf2_status lf2_plan_get_schedule(lf2_plan p, int32_t axis, int32_t radices[15], int32_t *nst,
                                 int32_t *runtime)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (axis < 0 || axis > 2) return fail(LF2_ERR_INVALID_ARG, "axis %d is not 0, 1 or 2", axis);
    int n = 0;
    int r[kGenMaxStages] = {};
    if (p->gen[axis]) {
        n = p->sched[axis].n;
        for (int i = 0; i < n; ++i) r[i] = p->sched[axis].r[i];
    } else {
        // the compiled kernels' schedule (lf2_device.hpp)
        n = lf2::nstages(p->len[axis]);
        for (int i = 0; i < n && i < kGenMaxStages; ++i) r[i] = lf2::radix_at(p->len[axis], i);
    }
    if (nst) *nst = n;
    if (runtime) *runtime = p->gen[axis] ? 1 : 0;
    if (radices)
        for (int i = 0; i < kGenMaxStages; ++i) radices[i] = i < n ? r[i] : 0;
    return LF2_OK;
}

lf2_status lf2_plan_set_schedule(lf2_plan p, int32_t axis, const int32_t *radices, int32_t nstages)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (axis < 0 || axis > 2) return fail(LF2_ERR_INVALID_ARG, "axis %d is not 0, 1 or 2", axis);
    if (nstages < 0 || nstages > kGenMaxStages || (nstages > 0 && !radices))
        return fail(LF2_ERR_INVALID_ARG, "bad schedule (%d stages)", nstages);
    GSched sc{};
    sc.n = nstages;
    for (int i = 0; i < nstages; ++i) sc.r[i] = radices[i];
    if (!sched_valid(sc, p->len[axis]))
        return fail(LF2_ERR_INVALID_ARG,
                    "radices must each be 2, 3, 4, 5, 8 or 16 with product %d", p->len[axis]);
    if (axis == 0 && !p->gen_only[0])
        return fail(LF2_ERR_UNSUPPORTED, "the x pass of length %d runs compiled kernels only",
                    p->len[0]);
    if (axis > 0 && gs_cols(p, p->len[axis], 0) < 1)
        return fail(LF2_ERR_UNSUPPORTED, "line length %d does not fit a tile", p->len[axis]);
    p->sched[axis] = sc;
    p->gen[axis] = true;
    return LF2_OK;
}

lf2_status lf2_plan_set_tuning(lf2_plan p, int32_t axis, int32_t variant, int32_t chunk)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (axis == 0) {
        if (variant < 0 || variant > 2) return fail(LF2_ERR_INVALID_ARG, "variant %d outside [0, 2]", variant);
        if (p->gen_only[0])
            return fail(LF2_ERR_UNSUPPORTED, "no compiled kernels for line length %d", p->len[0]);
        const bool was_gen = p->gen[0];
        p->gen[0] = false;  // the compiled kernels again
        if (variant && !x_lane_exchange_ok(p)) {
            p->gen[0] = was_gen;
            return fail(LF2_ERR_UNSUPPORTED,
                        "lane exchange needs c2c rows of 64 points and one component");
        }
        p->xx = variant;
        return LF2_OK;
    }
    if (axis == 3) {
        if (variant < 0 || variant > 1) return fail(LF2_ERR_INVALID_ARG, "variant %d outside [0, 1]", variant);
        if (variant == 1 && !fused_reg_supported(p->len[2]))
            return fail(LF2_ERR_UNSUPPORTED, "no register tile for the fused pass over %d points",
                        p->len[2]);
        p->fvar = variant;
        return LF2_OK;
    }
    if (axis != 1 && axis != 2) return fail(LF2_ERR_INVALID_ARG, "axis %d is not 0, 1, 2 or 3", axis);
    if (variant < 0 || variant > 7) return fail(LF2_ERR_INVALID_ARG, "variant %d outside [0, 7]", variant);
    if (chunk < 1 || chunk > 1024) return fail(LF2_ERR_INVALID_ARG, "chunk %d outside [1, 1024]", chunk);
    if (p->gen_only[axis])
        return fail(LF2_ERR_UNSUPPORTED, "no compiled kernels for line length %d", p->len[axis]);
    if ((variant & 1) && !s_wide_supported(p->len[axis]))
        return fail(LF2_ERR_UNSUPPORTED, "no wide tiles for line length %d", p->len[axis]);
    if ((variant & 4) && ((variant & 1) || !s_reg_supported(p->len[axis])))
        return fail(LF2_ERR_UNSUPPORTED, "no register tile for line length %d (or with wide tiles)",
                    p->len[axis]);
    p->svar[axis] = variant;
    p->schunk[axis] = chunk;
    p->gen[axis] = false;  // the compiled kernels again
    return LF2_OK;
}

lf2_status lf2_plan_destroy(lf2_plan p)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    for (void *ptr : p->allocs) (void)hipFree(ptr);
    delete p;
    return LF2_OK;
}

lf2_status lf2_fft_kspace(lf2_plan p, int64_t ksize[3], int64_t kstride[3])
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (ksize) {
        ksize[0] = p->nxk;
        ksize[1] = p->n[1];
        ksize[2] = p->n[2];
    }
    if (kstride) {
        kstride[0] = p->nc;
        if (p->klay == 2) {  // c2c (k_z, k_x, k_y): [N1][N0][N2]
            kstride[0] = p->nc * p->n[2];
            kstride[1] = p->nc * p->n[2] * p->n[0];
            kstride[2] = p->nc;
        } else {
            kstride[1] = p->klay == 1 ? p->nc * p->nxk * p->n[2] : p->nc * p->nxk;
            kstride[2] = p->klay == 1 ? p->nc * p->nxk : p->nc * p->nxk * p->n[1];
        }
    }
    return LF2_OK;
}

lf2_status lf2_plan_workspace_bytes(lf2_plan p, size_t *bytes)
{
    if (!p || !bytes) return fail(LF2_ERR_INVALID_ARG, "NULL argument");
    *bytes = ws_layout(p, true, kMaxBins, true).total;
    return LF2_OK;
}

lf2_status lf2_plan_set_workspace(lf2_plan p, void *dev_ptr, size_t bytes)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (dev_ptr && ((uintptr_t)dev_ptr % 256))
        return fail(LF2_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    p->own_ws = dev_ptr;
    p->own_ws_bytes = dev_ptr ? bytes : 0;
    return LF2_OK;
}

lf2_status lf2_fft_execute(lf2_plan p, lf2_direction dir, const void *in, void *out, void *stream)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (dir != LF2_FORWARD && dir != LF2_BACKWARD) return fail(LF2_ERR_INVALID_ARG, "bad direction %d", (int)dir);
    lf2_status st;
    if ((st = check_ptr(in, "in", 8)) || (st = check_ptr(out, "out", 8))) return st;
    if (in == out && !p->inplace)
        return fail(LF2_ERR_UNSUPPORTED, "in == out needs a plan made with LF2_IN_PLACE");
    if ((st = check_device(p))) return st;
    hipStream_t s = (hipStream_t)stream;
    if (p->kind == LF2_R2C && dir == LF2_FORWARD) {
        if (p->klay == 1 && in == out) {
            // in place in the paper's order: the x pass moves row (y, z) to
            // another row's place, so it writes the workspace and the y pass
            // brings the spectrum back
            WsLayout L = ws_layout(p, true, 0, false);
            char *ws;
            if ((st = get_workspace(p, L.total, &ws))) return st;
            void *W = ws + L.w;
            if ((st = run_x(p, 0, -1, x_args(p, in, W, true, false, true), s))) return st;
            if ((st = run_strided(p, 1, -1, s_args(p, 1, W, out, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        } else {
            if ((st = run_x(p, 0, -1, x_args(p, in, out, true, false, true), s))) return st;
            if ((st = run_strided(p, 1, -1, s_args(p, 1, out, out, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        }
        return run_strided(p, 2, -1, s_args(p, 2, out, out, EPI_STORE), kStridedGridCap, s, nullptr);
    }
    if (p->kind == LF2_R2C) {
        WsLayout L = ws_layout(p, true, 0, false);
        char *ws;
        if ((st = get_workspace(p, L.total, &ws))) return st;
        void *W = ws + L.w;
        if ((st = run_strided(p, 2, +1, s_args(p, 2, in, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        if ((st = run_strided(p, 1, +1, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        return run_x(p, 1, +1, x_args(p, W, out, false, true, true), s);
    }
    // c2c
    const int sg = (int)dir;
    if (p->klay == 2) {
        // the paper's (k_z, k_x, k_y) order: natural passes in the workspace,
        // the z pass stores (forward) or loads (backward) transposed
        WsLayout L = ws_layout(p, true, 0, false);
        char *ws;
        if ((st = get_workspace(p, L.total, &ws))) return st;
        void *W = ws + L.w;
        if (dir == LF2_FORWARD) {
            if ((st = run_x(p, 2, sg, x_args(p, in, W, true, false, false), s))) return st;
            if ((st = run_strided(p, 1, sg, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
            return run_strided(p, 2, sg, t_args(p, W, out, EPI_STORE | EPI_TSTORE), kStridedGridCap, s, nullptr);
        }
        if ((st = run_strided(p, 2, sg, t_args(p, in, W, EPI_STORE | EPI_TLOAD), kStridedGridCap, s, nullptr))) return st;
        if ((st = run_strided(p, 1, sg, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        return run_x(p, 2, sg, x_args(p, W, out, false, true, false), s);
    }
    if (dir == LF2_FORWARD) {
        if ((st = run_x(p, 2, sg, x_args(p, in, out, true, false, false), s))) return st;
        if ((st = run_strided(p, 1, sg, s_args(p, 1, out, out, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        return run_strided(p, 2, sg, s_args(p, 2, out, out, EPI_STORE), kStridedGridCap, s, nullptr);
    }
    if (p->halo == 0) {
        if ((st = run_strided(p, 2, sg, s_args(p, 2, in, out, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        if ((st = run_strided(p, 1, sg, s_args(p, 1, out, out, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        return run_x(p, 2, sg, x_args(p, out, out, false, true, false), s);
    }
    WsLayout L = ws_layout(p, true, 0, false);
    char *ws;
    if ((st = get_workspace(p, L.total, &ws))) return st;
    void *W = ws + L.w;
    if ((st = run_strided(p, 2, sg, s_args(p, 2, in, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
    if ((st = run_strided(p, 1, sg, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
    return run_x(p, 2, sg, x_args(p, W, out, false, true, false), s);
}

}  // extern "C"

namespace lf2 {
namespace host {

size_t poisson_ws_bytes(const lf2_plan_s *p, int32_t nbins, bool parseval)
{
    const int nb = nbins > 0 ? nbins : (parseval ? 1 : 0);
    return ws_layout(p, true, nb, parseval).total;
}

// Poisson solve on `stream`; ws_given (nullable) is a workspace of at least
// poisson_ws_bytes bytes reserved for this call, else the plan's workspace.
lf2_status poisson_impl(lf2_plan p, const float *rho, float *phi, double dx, uint32_t flags,
                        int32_t nbins, double *d_pk, double *d_kmean, double *d_count,
                        double *d_parseval, hipStream_t stream, char *ws_given,
                        size_t ws_given_bytes, bool noalloc, const PoissonTables *tabs)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (p->kind != LF2_R2C || p->nc != 1)
        return fail(LF2_ERR_UNSUPPORTED, "Poisson needs an r2c plan with ncomp = 1");
    lf2_status st;
    if ((st = check_ptr(rho, "rho", 4)) || (st = check_ptr(phi, "phi", 4))) return st;
    if ((const void *)rho == (const void *)phi && !p->inplace)
        return fail(LF2_ERR_INVALID_ARG, "rho and phi alias: needs a plan made with LF2_IN_PLACE");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LF2_ERR_INVALID_ARG, "dx must be > 0");
    if (flags & ~(uint32_t)(LF2_POISSON_DISCRETE_K2 | LF2_PK_OF_PHI))
        return fail(LF2_ERR_INVALID_ARG, "unknown Poisson flags 0x%x", flags);
    if ((st = check_bins(p, nbins))) return st;
    if (d_parseval && (flags & LF2_PK_OF_PHI))
        return fail(LF2_ERR_INVALID_ARG, "Parseval sums are defined for rho; drop LF2_PK_OF_PHI");
    if ((st = check_device(p))) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool parseval = d_parseval != nullptr;
    const int nb = nbins > 0 ? nbins : (parseval ? 1 : 0);
    WsLayout L = ws_layout(p, true, nb, parseval);
    char *ws;
    if (ws_given) {
        if (ws_given_bytes < L.total)
            return fail(noalloc ? LF2_ERR_UNSUPPORTED : LF2_ERR_INVALID_ARG,
                        "workspace of %zu bytes < %zu needed", ws_given_bytes, L.total);
        ws = ws_given;
    } else if (noalloc) {
        return fail(LF2_ERR_INVALID_ARG, "no workspace for a call that must not allocate");
    } else if ((st = get_workspace(p, L.total, &ws))) {
        return st;
    }
    void *W = ws + L.w;
    const double *k2[3];
    ShellEntry sh{};
    if (tabs) {
        for (int i = 0; i < 3; ++i) k2[i] = tabs->k2[i];
        sh = tabs->sh;
        if (nb > 0 && sh.nbins != nb) return fail(LF2_ERR_INVALID_ARG, "shell table of another bin count");
    } else {
        if ((st = get_k2(p, dx, (flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0, s, k2, noalloc))) return st;
        if (nb > 0 && (st = get_shell(p, nb, s, &sh, noalloc))) return st;
    }

    XArgs xa = x_args(p, rho, W, true, false, true);
    if (parseval) xa.sumsq = (double *)(ws + L.sq);
    if ((st = run_x(p, 0, -1, xa, s))) return st;
    if ((st = run_strided(p, 1, -1, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
    int epi = EPI_STORE | EPI_POISSON;
    if (nb > 0) epi |= (flags & LF2_PK_OF_PHI) ? EPI_PK_AFTER : EPI_PK;
    SArgs za = s_args(p, 2, W, W, epi);
    for (int i = 0; i < 3; ++i) za.mt.k2[i] = k2[i];
    set_k2_units(za.mt, p, dx, (flags & LF2_POISSON_DISCRETE_K2) ? 1 : 0);
    int grid = 0;
    if (nb > 0) {
        use_shell(za.mt, sh);
        za.partial = (double *)(ws + L.part);
    }
    if ((st = run_strided(p, 2, -1, za, nb > 0 ? kPkGrid : kStridedGridCap, s, &grid))) return st;
    if ((st = run_strided(p, 1, +1, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
    if ((st = run_x(p, 1, +1, x_args(p, W, phi, false, true, true), s))) return st;
    if (nb > 0) {
        const double vscale = (flags & LF2_PK_OF_PHI) ? (double)p->ntot * (double)p->ntot : 1.0;
        const bool user_bins = nbins > 0;
        if ((st = pk_tail(p, sh, (double *)(ws + L.part), grid, (double *)(ws + L.sums), dx, vscale,
                          user_bins ? d_pk : nullptr, user_bins ? d_kmean : nullptr,
                          user_bins ? d_count : nullptr, d_parseval,
                          parseval ? (const double *)(ws + L.sq) : nullptr,
                          parseval ? x_grid_blocks(p) : 0,
                          parseval ? (double *)(ws + L.sqt) : nullptr, s)))
            return st;
    }
    return LF2_OK;
}

}  // namespace host
}  // namespace lf2

extern "C" {

lf2_status lf2_poisson_solve(lf2_plan p, const float *rho, float *phi, double dx, uint32_t flags,
                             int32_t nbins, double *d_pk, double *d_kmean, double *d_count,
                             double *d_parseval, void *stream)
{
    return poisson_impl(p, rho, phi, dx, flags, nbins, d_pk, d_kmean, d_count, d_parseval,
                        (hipStream_t)stream, nullptr, 0);
}

}  // extern "C"

// ------------------------------------------------ static scratch (no allocation)
// Workspace of lf2_poisson_solve_noalloc: one array per device, held by the
// code object for the life of the process.  In host code `scratch` names a
// host-side stand-in, not device memory: only the address that
// hipGetSymbolAddress returns on a device is used (kernel arguments), and it
// is looked up once per device with that device current.
static __device__ __align__(256) char scratch[LF2_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

lf2_status scratch_on(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LF2_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return LF2_OK;
}
}  // namespace

extern "C" {

lf2_status lf2_poisson_solve_noalloc(lf2_plan p, const float *rho, float *phi, double dx,
                                     uint32_t flags, int32_t nbins, double *d_pk,
                                     double *d_kmean, double *d_count, double *d_parseval,
                                     void *stream)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    lf2_status st;
    if ((st = check_device(p))) return st;
    char *ws = nullptr;
    if ((st = scratch_on(p->device, &ws))) return st;
    prof::t_quiet = true;
    st = poisson_impl(p, rho, phi, dx, flags, nbins, d_pk, d_kmean, d_count, d_parseval,
                      (hipStream_t)stream, ws, LF2_NOALLOC_SCRATCH_BYTES, true);
    prof::t_quiet = false;
    return st;
}

lf2_status lf2_power_spectrum(lf2_plan p, const void *field, int32_t field_is_kspace, int32_t nbins,
                              double dx, double *d_pk, double *d_kmean, double *d_count,
                              void *stream)
{
    if (!p) return fail(LF2_ERR_INVALID_ARG, "plan is NULL");
    if (p->nc != 1) return fail(LF2_ERR_UNSUPPORTED, "power spectrum needs ncomp = 1");
    lf2_status st;
    if ((st = check_ptr(field, "field", field_is_kspace || p->kind == LF2_C2C ? 8 : 4))) return st;
    if (nbins < 1) return fail(LF2_ERR_INVALID_ARG, "nbins %d < 1", nbins);
    if ((st = check_bins(p, nbins))) return st;
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(LF2_ERR_INVALID_ARG, "dx must be > 0");
    if ((st = check_device(p))) return st;
    hipStream_t s = (hipStream_t)stream;
    WsLayout L = ws_layout(p, !field_is_kspace, nbins, false);
    char *ws;
    if ((st = get_workspace(p, L.total, &ws))) return st;
    ShellEntry sh{};
    if ((st = get_shell(p, nbins, s, &sh))) return st;
    double *part = (double *)(ws + L.part);
    int grid = 0;
    if (field_is_kspace) {
        ModeTables mt = base_tables(p);
        use_shell(mt, sh);
        grid = kPkGrid;
        const int t = prof::begin("k_pk_kspace", (double)spectrum_bytes(p), s);
        int64_t kst[3];
        (void)lf2_fft_kspace(p, nullptr, kst);
        hipError_t e = launch_pk_kspace(field, (int)p->n[1], (int)p->n[2], kst[0], kst[1], kst[2], mt,
                                        part, grid, s);
        prof::end(t, s);
        LF2_HIP(e);
    } else {
        void *W = ws + L.w;
        if (p->kind == LF2_R2C) {
            if ((st = run_x(p, 0, -1, x_args(p, field, W, true, false, true), s))) return st;
        } else {
            if ((st = run_x(p, 2, -1, x_args(p, field, W, true, false, false), s))) return st;
        }
        if ((st = run_strided(p, 1, -1, s_args(p, 1, W, W, EPI_STORE), kStridedGridCap, s, nullptr))) return st;
        SArgs za = s_args(p, 2, W, W, EPI_PK);
        use_shell(za.mt, sh);
        za.partial = part;
        if ((st = run_strided(p, 2, -1, za, kPkGrid, s, &grid))) return st;
    }
    return pk_tail(p, sh, part, grid, (double *)(ws + L.sums), dx, 1.0, d_pk, d_kmean, d_count,
                   nullptr, nullptr, 0, nullptr, s);
}

}  // extern "C"
