// lf2_kreg.hip -- strided (y / z) pass over long lines (1024 and 2048
// points) with the tile held in registers: a 32 x Q decomposition with one
// exchange.
//
// A line of L = 32 Q points splits as n = j + Q r (r in [0, 32), j in
// [0, Q)) and k = k1 + 32 k2 (k1 in [0, 32), k2 in [0, Q)); then
//   X[k1 + 32 k2] = sum_j W_Q^{S j k2} W_L^{S j k1} sum_r x[j + Q r] W_32^{S r k1}.
// Thread (column c, j) loads the 32 points j + Q r of its column straight
// into registers, takes the inner 32-point DFT over r, multiplies by
// W_L^{S j k1}, and hands value k1 to the threads of (c, k1) through LDS,
// which take the outer Q-point DFT over j and store point k1 + 32 k2.  At
// L = 1024 (Q = 32) one thread does the outer DFT; at L = 2048 (Q = 64) two
// adjacent lanes h = 0, 1 take the 32-point DFTs over the even and the odd
// j, and finish with one radix-2 step across the lane pair (a DPP swap):
// the lane h keeps outputs k2 = k2' + 32 h.
// A tile is B = 1024 / Q adjacent columns x L points (256 KB) with 1024
// threads: 32 columns (256-byte row segments) at L = 1024 and 16 (128-byte
// segments) at L = 2048, twice what an LDS tile of whole lines holds.  The
// one exchange goes through 132 KB of LDS in two halves (real parts, then
// imaginary parts).  No epilogue: plain passes only.
#include "lf2_kernels.hpp"

namespace lf2 {

namespace {

constexpr int kRThreads = 1024;

template <int L>
struct RegTile {
    static constexpr int P = 32;                  // points per thread; inner DFT length
    static constexpr int Q = L / P;               // outer DFT length (range of j)
    static constexpr int B = kRThreads / Q;       // columns per tile
    static constexpr int H = Q / P;               // threads per (column, k1)
    // exchange rows: value (k1, j, c) at k1 * ROW + j * B + c; the 32-word
    // pad puts the two k1 rows a wave reads in different banks
    static constexpr int ROW = Q * B + 32;
    static_assert(Q * P == L && (H == 1 || H == 2), "1024 or 2048 points");
};

// The value of the adjacent lane (lane ^ 1), by a DPP quad permutation.
__device__ __forceinline__ float lane_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

template <int L, int S, bool NTM>
__global__ __launch_bounds__(kRThreads) void k_strided_r(SArgs a)
{
    using T = RegTile<L>;
    constexpr int P = T::P, B = T::B, H = T::H, ROW = T::ROW;
    __shared__ float ex[P * ROW];
    __shared__ c32 tw[L];
    const int tid = threadIdx.x;
    load_table(tw, a.tw, L, tid, kRThreads);
    __syncthreads();
    const int64_t ntiles = (a.ncols + B - 1) / B;
    const int64_t K = a.xcd_chunk;  // the XCD-aware walk of k_strided
    const int64_t span = (ntiles + 8 * K - 1) / (8 * K) * (8 * K);
    const bool store = (a.epi & EPI_STORE) != 0;
    for (int64_t vb = blockIdx.x; vb < span; vb += gridDim.x) {
        const int64_t lb = vb / 8;
        const int64_t t = ((lb / K) * 8 + (vb % 8)) * K + lb % K;
        if (t >= ntiles) continue;  // uniform over the block
        // per-thread offsets are derived from the thread index afresh in
        // every tile (opaque to the optimiser), not hoisted out of the loop
        // where the twiddle and exchange addresses would stay live
        const int ot = opaque_tid<true>(tid);
        // first half: thread (c, j)
        const int c = ot % B, j = ot / B;
        const int64_t f = t * B + c;
        // a column past the end reads column 0 (in bounds) and is not stored
        const int64_t base = f < a.ncols ? col_base(a, f) : 0;
        c32 v[P];
        gload_pts<P, NTM>(v, (const c32 *)a.in + base + (int64_t)j * a.stride,
                            (int64_t)T::Q * a.stride, true);
        Dft<P, S>::run(v);  // v[k1] = inner DFT of x[j + Q r] over r
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) {
            c32 w = tw[j * k1];  // W_L^{j k1}, j k1 < L
            if (S > 0) w = conjg(w);
            v[k1] = mul(v[k1], w);
        }
        // second half: thread (c2, k1, h) takes j = H j' + h, j' in [0, 32)
        const int h = ot % H, c2 = (ot / H) % B, k1 = ot / (H * B);
        float re[P];
#pragma unroll
        for (int q = 0; q < P; ++q) ex[q * ROW + j * B + c] = v[q].x;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < P; ++jj) re[jj] = ex[k1 * ROW + (H * jj + h) * B + c2];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) ex[q * ROW + j * B + c] = v[q].y;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < P; ++jj) v[jj] = c32{re[jj], ex[k1 * ROW + (H * jj + h) * B + c2]};
        __syncthreads();  // the next tile rewrites ex
        Dft<P, S>::run(v);  // v[k2'] = DFT over j' of the values of this h
        if constexpr (H == 2) {
            // outputs k2' + 32 k3: Y0 + (-1)^k3 W_Q^{k2'} Y1; lane h gives
            // its own term (Y0, or W Y1: the twiddle is W_L^0 = 1 for h = 0)
            // and keeps k3 = h, so it adds (h = 0) or subtracts (h = 1) it
            const float sg = h ? -1.f : 1.f;
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                c32 w = tw[P * k2 * h];  // W_L^{P k2' h} = W_Q^{k2' h}
                if (S > 0) w = conjg(w);
                const c32 own = mul(v[k2], w);
                const c32 p = c32{lane_swap(own.x), lane_swap(own.y)};
                v[k2] = c32{fmaf(sg, own.x, p.x), fmaf(sg, own.y, p.y)};
            }
        }
        const int64_t f2 = t * B + c2;
        if (f2 < a.ncols && store) {
            const int64_t base2 = col_base(a, f2);
            gstore_pts<P, NTM>(v, (c32 *)a.out + base2 + (int64_t)(k1 + P * P * h) * a.stride,
                                 (int64_t)P * a.stride);
        }
    }
}

template <int L, bool NTM>
void launch_r(int sign, int g, const SArgs &a, hipStream_t s)
{
    if (sign < 0)
        hipLaunchKernelGGL((k_strided_r<L, -1, NTM>), dim3(g), dim3(kRThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_strided_r<L, 1, NTM>), dim3(g), dim3(kRThreads), 0, s, a);
}

template <int L>
hipError_t launch_len(int sign, const SArgs &a, int grid_cap, hipStream_t s, int *grid_used,
                      int chunk, bool ntm)
{
    constexpr int B = RegTile<L>::B;
    const int64_t ntiles = (a.ncols + B - 1) / B;
    const int64_t span = (ntiles + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
    const int g = (int)(span < grid_cap ? span : grid_cap);
    if (grid_used) *grid_used = g;
    if (ntm)
        launch_r<L, true>(sign, g, a, s);
    else
        launch_r<L, false>(sign, g, a, s);
    return hipGetLastError();
}

}  // namespace

bool s_reg_supported(int len) { return len == 1024 || len == 2048; }

hipError_t launch_strided_reg(int len, int sign, const SArgs &a, int grid_cap, hipStream_t s,
                              int *grid_used, int chunk, bool ntm)
{
    if (len == 1024) return launch_len<1024>(sign, a, grid_cap, s, grid_used, chunk, ntm);
    if (len == 2048) return launch_len<2048>(sign, a, grid_cap, s, grid_used, chunk, ntm);
    return hipErrorInvalidValue;
}

}  // namespace lf2
