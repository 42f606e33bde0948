// lf2_kbatch.hip -- batched Poisson solves on lattices of different sizes.
//
// A batch runs pass by pass.  For each pass and each line length present in
// the batch there is one grouped launch whose blocks each take one
// (field, tile) work item; a field's arguments come from a descriptor table
// in device memory.  The tiles are the same device functions, with the same
// thread counts, as the standalone passes, so every field gives the same
// result alone and in a batch.  The host captures the whole sequence (about
// five launches per distinct line length, plus one finalize launch for the
// power spectra) in a hipGraph; kernel boundaries order the passes.
#include "lf2_kernels.hpp"
#include "lf2_queue.hpp"

namespace lf2 {

#define LF2_BATCH_LENGTHS(X) X(16) X(32) X(48) X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(384)

bool batch_len_supported(int len)
{
    switch (len) {
#define LF2_CASE(L) case L:
        LF2_BATCH_LENGTHS(LF2_CASE)
#undef LF2_CASE
        return true;
    default:
        return false;
    }
}

int batch_x_rows(int m) { return x_rb(m, 1, kXThreads); }

// ------------------------------------------------------------ grouped kernels

template <int L>
__global__ __launch_bounds__(kXThreads) void k_bx_fwd(const BatchField *fields,
                                                      const BatchItem *items)
{
    using T = XR2CV<L, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    const BatchItem it = items[blockIdx.x];
    const BatchField &F = fields[it.field];
    T::tables(F.xf, sm, threadIdx.x);
    __syncthreads();
    [[clang::always_inline]] T::tile(F.xf, it.tile, sm, threadIdx.x, nullptr);
}

template <int L>
__global__ __launch_bounds__(kXThreads) void k_bx_inv(const BatchField *fields,
                                                      const BatchItem *items)
{
    using T = XC2RV<L, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    const BatchItem it = items[blockIdx.x];
    const BatchField &F = fields[it.field];
    T::tables(F.xi, sm, threadIdx.x);
    __syncthreads();
    [[clang::always_inline]] T::tile(F.xi, it.tile, sm, threadIdx.x);
}

// S = -1: forward y pass; S = +1: backward y pass.
template <int L, int S>
__global__ __launch_bounds__(kSThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_by(
    const BatchField *fields, const BatchItem *items)
{
    using T = STile<L, S, false, kSThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    const BatchItem it = items[blockIdx.x];
    const BatchField &F = fields[it.field];
    const SArgs &a = S < 0 ? F.yf : F.yi;
    T::tables(a, sm, threadIdx.x);
    __syncthreads();
    [[clang::always_inline]] T::tile(a, it.tile, sm, threadIdx.x, nullptr, nullptr);
}

// z pass: forward * -1/(N k^2) * backward, with the tile's w|F|^2 bin sums
// written to its own row of the field's partials.
template <int L, int K2>
__global__ __launch_bounds__(kSThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_bz(
    const BatchField *fields, const BatchItem *items)
{
    using T = STile<L, -1, true, kSThreads, true, K2>;
    __shared__ __align__(16) char sm[T::BYTES];
    extern __shared__ double dyn[];  // hist[hcopies][nbins + 1], edges[nbins + 1]
    const int tid = threadIdx.x;
    const BatchItem it = items[blockIdx.x];
    const BatchField &F = fields[it.field];
    const int nb = F.nbins;
    double *hist = dyn;
    BinEdge *edges = (BinEdge *)(dyn + F.z.hcopies * (nb + 1));
    T::tables(F.z, sm, tid);
    if (nb > 0) hist_init(F.z.mt, F.z.hcopies, hist, edges, tid, kSThreads);
    __syncthreads();
    [[clang::always_inline]] T::tile(F.z, it.tile, sm, tid, hist, edges);
    if (nb > 0)
        hist_flush(nb, F.z.hcopies, hist, F.partial + (int64_t)it.tile * (nb + 1), tid, kSThreads);
}

// One block per field: fixed-order reduction of the z tiles' bin rows, then
// pk = norm * S_b / count_b and kmean = kscale * sumk_b / count_b.
constexpr int kBFinThreads = 1024;
__global__ __launch_bounds__(kBFinThreads) void k_bfin(const BatchField *fields)
{
    constexpr int NT = kBFinThreads;
    __shared__ double red[NT];
    const int tid = threadIdx.x;
    const BatchField &F = fields[blockIdx.x];
    if (F.nbins <= 0) return;  // uniform over the block
    const int nbr = F.nbins + 1;
    const int G = NT / nbr;  // >= 2 because nbins <= kBatchMaxBins
    const int nt = F.ntiles[BP_Z];
    if (tid < G * nbr) {
        // group g sums tiles g, g + G, ... of bin b with four running sums
        // (four loads in flight), combined in a fixed order
        const int b = tid % nbr, g = tid / nbr;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int t = g;
        for (; t + 3 * G < nt; t += 4 * G) {
            s0 += F.partial[(int64_t)t * nbr + b];
            s1 += F.partial[(int64_t)(t + G) * nbr + b];
            s2 += F.partial[(int64_t)(t + 2 * G) * nbr + b];
            s3 += F.partial[(int64_t)(t + 3 * G) * nbr + b];
        }
        for (; t < nt; t += G) s0 += F.partial[(int64_t)t * nbr + b];
        red[tid] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    if (tid < F.nbins) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += red[g * nbr + tid];
        const double c = F.count[tid];
        if (F.pk) F.pk[tid] = c > 0 ? F.norm * s / c : 0.0;
        if (F.kmean) F.kmean[tid] = c > 0 ? F.kscale * F.sumk[tid] / c : 0.0;
        if (F.count_out) F.count_out[tid] = c;
    }
}

// ------------------------------------------------------- persistent kernel
// One launch runs every (field, pass, tile) item of the batch: blocks take
// items from the work queue of lf2_queue.hpp (a ticket counter in item
// order, per-(field, pass) completion counters) and run the same tile
// functions as the grouped kernels, here with 512 threads for every pass.

constexpr int kPThreads = 512;

int batch_px_rows(int m) { return x_rb(m, 1, kPThreads); }

// The queue's leader is the block's first wave as a whole, so that every
// branch of the claim loop is uniform over each wave.  With one leader lane
// the compiler may join the leader's publication at the end of an item and
// its claim of the next one into a path of their own around the loop's back
// edge; the first wave's other lanes (and the other waves) then reach the
// claim barrier before the new ticket is written, read the old one again
// and repeat the same item without end.  The leader's atomics act once per
// wave: lane 0 adds its operand, the other lanes add zero, and every lane
// takes lane 0's result.
__device__ __forceinline__ bool lane0()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)) == 0u;
}
__device__ __forceinline__ uint32_t uni(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

struct DevAtomics {
    static __device__ uint32_t fetch_add_relaxed(uint32_t *p, uint32_t v)
    {
        return uni(__hip_atomic_fetch_add(p, lane0() ? v : 0u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT));
    }
    static __device__ uint32_t fetch_add_acq_rel(uint32_t *p, uint32_t v)
    {
        return uni(__hip_atomic_fetch_add(p, lane0() ? v : 0u, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT));
    }
    static __device__ uint32_t fetch_or_relaxed(uint32_t *p, uint32_t v)
    {
        return uni(__hip_atomic_fetch_or(p, lane0() ? v : 0u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT));
    }
    static __device__ uint32_t load_relaxed(const uint32_t *p)
    {
        return uni(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    // every lane stores the same value
    static __device__ void store_relaxed(uint32_t *p, uint32_t v)
    {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // Completion counts are relaxed atomics (performed in the L2); the
    // ordering of the tile data around them is the policy's wave and leader
    // operations.  (Release / acquire at agent scope here would write back
    // and invalidate the whole L2 at every publication and every poll.)
    static __device__ uint32_t publish_add(uint32_t *p, uint32_t v) { return fetch_add_relaxed(p, v); }
    static __device__ uint32_t poll_load(const uint32_t *p) { return load_relaxed(p); }
    static __device__ void pause() { __builtin_amdgcn_s_sleep(2); }
    // every wave: its stores have reached the L2 (the L1 writes through)
    static __device__ void wave_release() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
    // every wave: drop the CU's L1 lines, so loads read the L2
    static __device__ void wave_acquire() { asm volatile("buffer_inv sc0" ::: "memory"); }
};

// Producer and consumer of every tile on one XCD (one queue per XCD): the
// L2 they share is the point of coherence, so only the L1 needs care (the
// wave operations).
struct DevLocal : DevAtomics {
    static __device__ void leader_release() {}
    static __device__ void leader_acquire() {}
};

// One queue for the whole chip: a tile written through one XCD's L2 is read
// through another's, so the leader writes the L2 back before publishing and
// invalidates it after its wait (once per item, not once per wave or poll).
struct DevAgent : DevAtomics {
    static __device__ void leader_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
    static __device__ void leader_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
};

struct DevBlock {
    uint32_t *word;  // LDS
    // the first wave, a condition the compiler sees as uniform over each wave
    __device__ bool leader() const { return uni(threadIdx.x) < 64u; }
    __device__ void share(uint32_t v) { *word = v; }  // the leader's lanes: the same v
    __device__ uint32_t shared() const { return uni(*word); }
    __device__ void barrier() { __syncthreads(); }
};

// The XCD (XCC) this wave runs on: hardware register HW_REG_XCC_ID, bits 0..3.
__device__ __forceinline__ int xcc_id()
{
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u);
}

__global__ void k_xcc_probe(int32_t *out, int n)
{
    if (threadIdx.x == 0 && (int)blockIdx.x < n) out[blockIdx.x] = xcc_id();
}

hipError_t launch_xcc_probe(int32_t *out, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_xcc_probe, dim3(n), dim3(64), 0, s, out, n);
    return hipGetLastError();
}

// LDS of the largest tile of a length (the z tile with its bin histogram
// and edge table behind it).
template <int L>
constexpr size_t p_bytes()
{
    constexpr size_t a = XR2CV<L, kPThreads>::BYTES, b = XC2RV<L, kPThreads>::BYTES;
    constexpr size_t c = STile<L, -1, false, kPThreads>::BYTES;
    constexpr size_t d = STile<L, -1, true, kPThreads, true>::BYTES + 16 * (kBatchMaxBins + 1);
    constexpr size_t ab = a > b ? a : b, cd = c > d ? c : d;
    return ab > cd ? ab : cd;
}
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
#define LF2_PB(L) p_bytes<L>(),
constexpr size_t kPBytesList[] = {LF2_BATCH_LENGTHS(LF2_PB) 8 * kPThreads};
#undef LF2_PB
constexpr size_t p_max(int i = 0)
{
    return i == (int)(sizeof(kPBytesList) / sizeof(kPBytesList[0]))
               ? 0
               : cmax(kPBytesList[i], p_max(i + 1));
}
constexpr size_t kPBytes = p_max();
static_assert(2 * kPBytes <= 160 * 1024, "two persistent blocks must fit one CU's LDS");

size_t batch_persistent_lds() { return kPBytes; }

// Fixed-order finalize of one field's power spectrum (the k_bfin body with
// the persistent block's threads).
__device__ void p_finalize(const BatchField &F, double *red)
{
    constexpr int NT = kPThreads;
    const int tid = threadIdx.x;
    const int nbr = F.nbins + 1;
    const int G = NT / nbr;  // >= 1 because nbins <= kBatchMaxBins
    const int nt = F.ntiles[BP_Z];
    if (tid < G * nbr) {
        const int b = tid % nbr, g = tid / nbr;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int t = g;
        for (; t + 3 * G < nt; t += 4 * G) {
            s0 += F.partial[(int64_t)t * nbr + b];
            s1 += F.partial[(int64_t)(t + G) * nbr + b];
            s2 += F.partial[(int64_t)(t + 2 * G) * nbr + b];
            s3 += F.partial[(int64_t)(t + 3 * G) * nbr + b];
        }
        for (; t < nt; t += G) s0 += F.partial[(int64_t)t * nbr + b];
        red[tid] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    if (tid < F.nbins) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += red[g * nbr + tid];
        const double c = F.count[tid];
        if (F.pk) F.pk[tid] = c > 0 ? F.norm * s / c : 0.0;
        if (F.kmean) F.kmean[tid] = c > 0 ? F.kscale * F.sumk[tid] / c : 0.0;
        if (F.count_out) F.count_out[tid] = c;
    }
    __syncthreads();
}

// Not inlined: each (length) body is register-allocated on its own, as in
// its grouped kernel, instead of all of them inside one function.
// The tiles t0 .. t1 - 1 of one item of pass P (line length L), after one
// load of the pass tables; z tiles (fused Poisson scale and binning, K2 as
// for STile) each write their own row of bin sums.  One function per
// (L, P, K2), not inlined into the kernel: each is register-allocated on
// its own, as a standalone pass kernel would be, and the tile code is
// inlined into it, so the only call is the one per item.
template <int L, int P, int K2 = 0>
__device__ __attribute__((noinline)) void p_pass(const BatchField &F, const QItem &it, char *sm)
{
    const int tid = threadIdx.x;
    const int t0 = it.tile, t1 = it.tile + it.ntile;
    if constexpr (P == BP_XF) {
        using T = XR2CV<L, kPThreads>;
        T::tables(F.xf, sm, tid);
        __syncthreads();
        for (int t = t0; t < t1; ++t)
            [[clang::always_inline]] T::tile(F.xf, t, sm, opaque_tid<true>(tid), nullptr);
    } else if constexpr (P == BP_XI) {
        using T = XC2RV<L, kPThreads>;
        T::tables(F.xi, sm, tid);
        __syncthreads();
        for (int t = t0; t < t1; ++t)
            [[clang::always_inline]] T::tile(F.xi, t, sm, opaque_tid<true>(tid));
    } else if constexpr (P == BP_YF || P == BP_YI) {
        using T = STile<L, P == BP_YF ? -1 : 1, false, kPThreads>;
        const SArgs &a = P == BP_YF ? F.yf : F.yi;
        T::tables(a, sm, tid);
        __syncthreads();
        for (int t = t0; t < t1; ++t)
            [[clang::always_inline]] T::tile(a, t, sm, opaque_tid<true>(tid), nullptr, nullptr);
    } else {
        using T = STile<L, -1, true, kPThreads, true, K2>;
        const int nb = F.nbins;
        double *hist = (double *)(sm + T::BYTES);
        BinEdge *edges = (BinEdge *)(hist + F.z.hcopies * (nb + 1));
        T::tables(F.z, sm, tid);
        if (nb > 0) hist_init(F.z.mt, F.z.hcopies, hist, edges, tid, kPThreads);
        __syncthreads();
        for (int t = t0; t < t1; ++t) {
            [[clang::always_inline]] T::tile(F.z, t, sm, opaque_tid<true>(tid), hist, edges);
            if (nb > 0) {
                hist_flush(nb, F.z.hcopies, hist, F.partial + (int64_t)t * (nb + 1), tid,
                           kPThreads);
                __syncthreads();
            }
        }
    }
}

template <int L>
__device__ __forceinline__ void p_item(const BatchField &F, const QItem &it, char *sm)
{
    switch (it.pass) {
    case BP_XF: p_pass<L, BP_XF>(F, it, sm); break;
    case BP_YF: p_pass<L, BP_YF>(F, it, sm); break;
    case BP_Z:
        if (F.z.mt.k2z_unit > 0.0)
            p_pass<L, BP_Z, 1>(F, it, sm);
        else
            p_pass<L, BP_Z, 2>(F, it, sm);
        break;
    case BP_YI: p_pass<L, BP_YI>(F, it, sm); break;
    case BP_XI: p_pass<L, BP_XI>(F, it, sm); break;
    default: break;
    }
}

// The line length of an item's pass, then the tile function of that length.
__device__ void p_run(const BatchField *fields, const QItem &it, char *sm)
{
    const BatchField &F = fields[it.field];
    if (it.pass == BP_FIN) {
        if (F.nbins > 0) p_finalize(F, (double *)sm);
        return;
    }
    const int len = (it.pass == BP_XF || it.pass == BP_XI) ? F.m : it.pass == BP_Z ? F.l2 : F.l1;
    switch (len) {
#define LF2_CASE(L)                \
    case L:                        \
        p_item<L>(F, it, sm);      \
        break;
        LF2_BATCH_LENGTHS(LF2_CASE)
#undef LF2_CASE
    default:
        break;
    }
}

// local = 1: block serves the queue of its XCD (xq[XCC id]; xq = nq, an
// empty queue, for an XCD the host did not see); 0: every block serves
// queue 0.  qstart / qcount have nq + 1 entries (the last one empty).
__global__ __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_bpersist(
    const BatchField *fields, const QItem *items, const uint32_t *qstart, const uint32_t *qcount,
    int nq, const int32_t *xq, QCtl *ctl, uint32_t *done, int ndone, uint32_t spin_limit,
    int local)
{
    __shared__ __align__(16) char sm[kPBytes];
    __shared__ uint32_t word;
    DevBlock blk{&word};
    auto work = [&](const QItem &it) { p_run(fields, it, sm); };
    if (local)
        run_queue<DevLocal>(blk, ctl, xq[xcc_id()], nq, done, ndone, items, qstart, qcount,
                            gridDim.x, spin_limit, work);
    else
        run_queue<DevAgent>(blk, ctl, 0, nq, done, ndone, items, qstart, qcount, gridDim.x,
                            spin_limit, work);
}

hipError_t batch_persistent_launch(const BatchField *fields, const QItem *items,
                                   const uint32_t *qstart, const uint32_t *qcount, int nq,
                                   const int32_t *xq, QCtl *ctl, uint32_t *done, int ndone,
                                   uint32_t spin_limit, int local, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_bpersist, dim3(grid), dim3(kPThreads), 0, s, fields, items, qstart, qcount,
                       nq, xq, ctl, done, ndone, spin_limit, local);
    return hipGetLastError();
}

hipError_t batch_group_launch(int pass, int len, const BatchField *fields,
                              const BatchItem *items, int nitems, int nbins, int k2cont,
                              hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const int zc = nbins > 0 ? epi_hist_copies(len, nbins, 80 * 1024) : 1;
    const size_t zdyn = nbins > 0 ? (size_t)(nbins + 1) * 8 * (zc + 1) : 16;
#define LF2_CASE(L)                                                                          \
    case L:                                                                                  \
        switch (pass) {                                                                      \
        case BP_XF:                                                                          \
            hipLaunchKernelGGL((k_bx_fwd<L>), dim3(nitems), dim3(kXThreads), 0, s, fields,   \
                               items);                                                       \
            break;                                                                           \
        case BP_YF:                                                                          \
            hipLaunchKernelGGL((k_by<L, -1>), dim3(nitems), dim3(kSThreads), 0, s, fields,   \
                               items);                                                       \
            break;                                                                           \
        case BP_Z:                                                                           \
            if (k2cont)                                                                      \
                hipLaunchKernelGGL((k_bz<L, 1>), dim3(nitems), dim3(kSThreads), zdyn, s,     \
                                   fields, items);                                           \
            else                                                                             \
                hipLaunchKernelGGL((k_bz<L, 2>), dim3(nitems), dim3(kSThreads), zdyn, s,     \
                                   fields, items);                                           \
            break;                                                                           \
        case BP_YI:                                                                          \
            hipLaunchKernelGGL((k_by<L, 1>), dim3(nitems), dim3(kSThreads), 0, s, fields,    \
                               items);                                                       \
            break;                                                                           \
        case BP_XI:                                                                          \
            hipLaunchKernelGGL((k_bx_inv<L>), dim3(nitems), dim3(kXThreads), 0, s, fields,   \
                               items);                                                       \
            break;                                                                           \
        default:                                                                             \
            return hipErrorInvalidValue;                                                     \
        }                                                                                    \
        return hipGetLastError();
    switch (len) {
        LF2_BATCH_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}

hipError_t batch_finalize_launch(const BatchField *fields, int nfields, hipStream_t s)
{
    hipLaunchKernelGGL(k_bfin, dim3(nfields), dim3(kBFinThreads), 0, s, fields);
    return hipGetLastError();
}

}  // namespace lf2
