// lf2_plan.hpp -- host-side plan object and helpers shared by the C ABI
// sources (lf2_api.cpp: transforms; lf2_batch.cpp: batched launches).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lf2.h"
#include "lf2_internal.hpp"

struct K2Entry {
    double dx;
    int discrete;
    double *tab[3];
};

struct ShellEntry {
    int nbins;
    int64_t *thresh;  // nbins + 1
    double *count;    // nbins
    double *sumk;     // nbins (sum w sqrt(q))
    int walk1;        // ModeTables::walk1 for these thresholds
};

// The binning fields of the mode tables from a shell table.
inline void use_shell(lf2::ModeTables &mt, const ShellEntry &sh)
{
    mt.thresh = sh.thresh;
    mt.nbins = sh.nbins;
    mt.walk1 = sh.walk1;
}

struct lf2_plan_s {
    int device = 0;
    lf2_fft_kind kind = LF2_R2C;
    int nc = 1;
    int halo = 0;
    uint32_t flags = 0;
    bool inplace = false;   // LF2_IN_PLACE
    int klay = 0;           // 0 natural k-space order, 1 the paper's (LF2_KLAYOUT_PAPER)
    int64_t n[3] = {0, 0, 0};
    int64_t nh = 0;    // N0/2 + 1
    int64_t nxk = 0;   // k-space extent of dimension 0
    int64_t ntot = 0;  // N0 N1 N2
    int len[3] = {0, 0, 0};
    int svar[3] = {0, 0, 0};              // strided tile variant per axis (1, 2)
    int fvar = 0;                         // fused last-axis pass: 0 LDS stages, 1 register tile
    int xx = 0;                           // x pass exchange (c2c, N0 = 64, one component):
                                          // 0 LDS, 1 ds_bpermute, 2 DPP
    int schunk[3] = {16, 16, 16};         // tiles per XCD chunk per axis
    double tune_us[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};  // [axis][default, tuned]
    // run-time-schedule kernels: gen_only = no compiled kernel for the axis'
    // length; gen = the plain passes of the axis use them (gen_only, or the
    // tuner found a schedule faster than the compiled kernels)
    bool gen_only[3] = {false, false, false};
    bool gen[3] = {false, false, false};
    lf2::GSched sched[3] = {};
    int gen_rb = 1;          // x tile rows of the run-time x kernels
    size_t lds_max = 65536;  // LDS bytes a block may use on the plan's device
    void *tw[3] = {nullptr, nullptr, nullptr};
    void *tw_post = nullptr;
    int64_t *q[3] = {nullptr, nullptr, nullptr};
    int64_t lcm = 1, qmax = 0;
    std::vector<K2Entry> k2;
    std::vector<ShellEntry> shells;
    void *own_ws = nullptr;
    size_t own_ws_bytes = 0;
    std::vector<void *> allocs;
};

namespace lf2 {
namespace host {

constexpr int kPkGrid = 1024;  // blocks of a binning pass (partials rows)
constexpr int kStridedGridCap = 1 << 30;

lf2_status fail(lf2_status st, const char *fmt, ...);

#define LF2_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            return ::lf2::host::fail(                                                       \
                e_ == hipErrorOutOfMemory ? LF2_ERR_OUT_OF_MEMORY : LF2_ERR_DEVICE,         \
                "%s failed: %s", #call, hipGetErrorString(e_));                             \
        }                                                                                   \
    } while (0)

size_t align256(size_t b);
std::string kname(const char *fmt, ...);
namespace prof {
int begin(const std::string &name, double bytes, hipStream_t s);
void end(int idx, hipStream_t s);
}  // namespace prof

lf2_status plan_alloc(lf2_plan p, void **dst, size_t bytes);
size_t spectrum_bytes(const lf2_plan_s *p);
ModeTables base_tables(const lf2_plan_s *p);
// (2 pi / (N2 dx))^2 for the continuous k^2 (the fused pass then computes
// the last axis' k^2 from |n_z|), 0 for the discrete one.
// Continuous k^2 units (2 pi / (N_i dx))^2 of the three dimensions (zero for
// the discrete k^2, which the kernels read from the tables).
void set_k2_units(ModeTables &mt, const lf2_plan_s *p, double dx, int discrete);
// Tables of a plan, built on first use (lookup_only: never build; a
// missing table is LF2_ERR_NOT_READY).
lf2_status get_k2(lf2_plan p, double dx, int discrete, hipStream_t s, const double *out[3],
                  bool lookup_only = false);
lf2_status get_shell(lf2_plan p, int nbins, hipStream_t s, ShellEntry *out,
                     bool lookup_only = false);
lf2_status check_device(const lf2_plan_s *p);
lf2_status check_ptr(const void *ptr, const char *what, size_t align);
XArgs x_args(const lf2_plan_s *p, const void *in, void *out, bool in_is_x, bool out_is_x,
             bool real_x);
SArgs s_args(const lf2_plan_s *p, int axis, const void *in, void *out, int epi);
lf2_status check_bins(const lf2_plan_s *p, int32_t nbins);

size_t poisson_ws_bytes(const lf2_plan_s *p, int32_t nbins, bool parseval);
// The plan tables a Poisson solve reads (k^2 of its dx and kind, shell
// table of its bin count).
struct PoissonTables {
    const double *k2[3];
    ShellEntry sh;
};
// noalloc: use only tables that already exist (LF2_ERR_NOT_READY otherwise)
// and make no allocation; ws_given must then be given.  tabs (nullable):
// tables the caller already looked up, so the plan's table lists are not
// read (callers that share plans across threads look them up under a lock).
lf2_status poisson_impl(lf2_plan p, const float *rho, float *phi, double dx, uint32_t flags,
                        int32_t nbins, double *d_pk, double *d_kmean, double *d_count,
                        double *d_parseval, hipStream_t stream, char *ws_given,
                        size_t ws_given_bytes, bool noalloc = false,
                        const PoissonTables *tabs = nullptr);

// Grouped Poisson solves of one lattice (lf2_batch.cpp): R requests with
// the same plan, dx, k^2 kind and bin count as one launch per pass.
struct GroupReq {
    const float *rho;
    float *phi;
    double *pk, *kmean, *count;  // nullable
    void *ws;                    // group_ws_bytes of workspace
};
bool group_supported(const lf2_plan_s *p);
size_t group_ws_bytes(const lf2_plan_s *p, int32_t nbins);
size_t group_stage_bytes(const lf2_plan_s *p, int R);
// stage_host (pinned) and stage_dev: group_stage_bytes each; both must stay
// untouched until the stream has passed the group's launches.
lf2_status group_enqueue(lf2_plan p, int R, const GroupReq *req, double dx, uint32_t flags,
                         int32_t nbins, const PoissonTables &tabs, void *stage_host,
                         void *stage_dev, size_t stage_bytes, hipStream_t s);

}  // namespace host
}  // namespace lf2
