// lf2_kreg.hip -- strided (y / z) pass over 1024-point lines with the tile
// held in registers: a 32 x 32 decomposition with one exchange.
//
// A line of L = 1024 points splits as n = j + 32 r (j, r in [0, 32)) and
// k = k1 + 32 k2; then
//   X[k1 + 32 k2] = sum_j W_32^{S j k2} W_1024^{S j k1} sum_r x[j + 32 r] W_32^{S r k1}.
// Thread (column c, j) loads the 32 points j + 32 r of its column straight
// into registers, takes the inner 32-point DFT over r, multiplies by
// W_1024^{S j k1}, and hands value k1 to thread (c, k1) through LDS; that
// thread takes the outer 32-point DFT over j and stores point k1 + 32 k2.
// A tile is 32 adjacent columns x 1024 points (256 KB) with 1024 threads:
// every load and store instruction of a wave covers two 256-byte row
// segments, twice the segment of the LDS-staged wide tile at this length,
// which the tile's 256 KB could not fit in LDS.  The register tile needs
// only one exchange, done in two halves (real parts, then imaginary parts)
// through 132 KB of LDS.  No epilogue: plain passes only.
#include "lf2_kernels.hpp"

namespace lf2 {

namespace {

constexpr int kRL = 1024;        // line length
constexpr int kRP = 32;          // points per thread (r and j range)
constexpr int kRB = 32;          // columns per tile
constexpr int kRThreads = 1024;  // kRB x kRP
// exchange rows: value (k1, j, c) at k1 * kRRow + j * kRB + c; the 32-word
// pad puts the two k1 rows a wave reads in different banks
constexpr int kRRow = kRP * kRB + 32;

template <int S, bool NTM>
__global__ __launch_bounds__(kRThreads) void k_strided_r(SArgs a)
{
    __shared__ float ex[kRP * kRRow];
    __shared__ c32 tw[kRL];
    const int tid = threadIdx.x;
    load_table(tw, a.tw, kRL, tid, kRThreads);
    __syncthreads();
    const int64_t ntiles = (a.ncols + kRB - 1) / kRB;
    const int64_t K = a.xcd_chunk;  // the XCD-aware walk of k_strided
    const int64_t span = (ntiles + 8 * K - 1) / (8 * K) * (8 * K);
    const bool store = (a.epi & EPI_STORE) != 0;
    for (int64_t vb = blockIdx.x; vb < span; vb += gridDim.x) {
        const int64_t lb = vb / 8;
        const int64_t t = ((lb / K) * 8 + (vb % 8)) * K + lb % K;
        if (t >= ntiles) continue;  // uniform over the block
        // per-thread offsets are derived from the thread index afresh in
        // every tile (opaque to the optimiser), not hoisted out of the loop
        // where the 31 twiddle and exchange addresses would stay live
        const int ot = opaque_tid<true>(tid);
        const int c = ot % kRB;  // column of the tile
        const int j = ot / kRB;  // j in the first half, k1 in the second
        const int64_t f = t * kRB + c;
        const bool valid = f < a.ncols;
        const int64_t base = valid ? col_base(a, f) : 0;
        // a column past the end reads column 0 (in bounds) and is not stored
        c32 v[kRP];
        gload_pts<kRP, NTM>(v, (const c32 *)a.in + base + (int64_t)j * a.stride,
                            (int64_t)kRP * a.stride, true);
        Dft<kRP, S>::run(v);  // v[k1] = inner DFT of x[j + 32 r] over r
#pragma unroll
        for (int k1 = 1; k1 < kRP; ++k1) {
            c32 w = tw[j * k1];  // W_1024^{j k1}, j k1 < 1024
            if (S > 0) w = conjg(w);
            v[k1] = mul(v[k1], w);
        }
        // hand value k1 to thread (c, k1): real parts, then imaginary parts
        float re[kRP];
#pragma unroll
        for (int k1 = 0; k1 < kRP; ++k1) ex[k1 * kRRow + j * kRB + c] = v[k1].x;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < kRP; ++jj) re[jj] = ex[j * kRRow + jj * kRB + c];
        __syncthreads();
#pragma unroll
        for (int k1 = 0; k1 < kRP; ++k1) ex[k1 * kRRow + j * kRB + c] = v[k1].y;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < kRP; ++jj) v[jj] = c32{re[jj], ex[j * kRRow + jj * kRB + c]};
        __syncthreads();  // the next tile rewrites ex
        Dft<kRP, S>::run(v);  // v[k2] = point j + 32 k2 of the line (j = k1)
        if (valid && store)
            gstore_pts<kRP, NTM>(v, (c32 *)a.out + base + (int64_t)j * a.stride,
                                 (int64_t)kRP * a.stride);
    }
}

template <bool NTM>
void launch_r(int sign, int g, const SArgs &a, hipStream_t s)
{
    if (sign < 0)
        hipLaunchKernelGGL((k_strided_r<-1, NTM>), dim3(g), dim3(kRThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_strided_r<1, NTM>), dim3(g), dim3(kRThreads), 0, s, a);
}

}  // namespace

bool s_reg_supported(int len) { return len == kRL; }

hipError_t launch_strided_reg(int len, int sign, const SArgs &a, int grid_cap, hipStream_t s,
                              int *grid_used, int chunk, bool ntm)
{
    if (len != kRL) return hipErrorInvalidValue;
    const int64_t ntiles = (a.ncols + kRB - 1) / kRB;
    const int64_t span = (ntiles + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
    const int g = (int)(span < grid_cap ? span : grid_cap);
    if (grid_used) *grid_used = g;
    if (ntm)
        launch_r<true>(sign, g, a, s);
    else
        launch_r<false>(sign, g, a, s);
    return hipGetLastError();
}

}  // namespace lf2
