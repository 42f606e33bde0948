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
    T::tile(F.xf, it.tile, sm, threadIdx.x, nullptr);
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
    T::tile(F.xi, it.tile, sm, threadIdx.x);
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
    T::tile(a, it.tile, sm, threadIdx.x, nullptr, nullptr);
}

// z pass: forward * -1/(N k^2) * backward, with the tile's w|F|^2 bin sums
// written to its own row of the field's partials.
template <int L>
__global__ __launch_bounds__(kSThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_bz(
    const BatchField *fields, const BatchItem *items)
{
    using T = STile<L, -1, true, kSThreads, true>;
    __shared__ __align__(16) char sm[T::BYTES];
    extern __shared__ double dyn[];  // hist[nbins + 1], edges[nbins + 1]
    const int tid = threadIdx.x;
    const BatchItem it = items[blockIdx.x];
    const BatchField &F = fields[it.field];
    const int nb = F.nbins;
    double *hist = dyn;
    BinEdge *edges = (BinEdge *)(dyn + (nb + 1));
    T::tables(F.z, sm, tid);
    if (nb > 0) load_edges(F.z.mt, hist, edges, tid, kSThreads);
    __syncthreads();
    T::tile(F.z, it.tile, sm, tid, hist, edges);
    if (nb > 0) {
        for (int i = tid; i <= nb; i += kSThreads)
            F.partial[(int64_t)it.tile * (nb + 1) + i] = hist[i];
    }
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

hipError_t batch_group_launch(int pass, int len, const BatchField *fields,
                              const BatchItem *items, int nitems, int nbins, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const size_t zdyn = nbins > 0 ? (size_t)(nbins + 1) * 16 : 16;
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
            hipLaunchKernelGGL((k_bz<L>), dim3(nitems), dim3(kSThreads), zdyn, s, fields,    \
                               items);                                                       \
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
