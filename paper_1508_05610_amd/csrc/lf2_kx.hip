// lf2_kx.hip -- instantiations and launchers of the x-pass kernels.
// LF2_KX_PART selects the family compiled by this translation unit
// (0: r2c, 1: c2r, 2: c2c) so that the families build in parallel.
// One-component rows with 8-byte aligned element offsets take the fast
// kernels (complex loads/stores straight into/out of the Stockham stages);
// everything else (components interleaved, odd halo offsets) takes the
// general kernels, which load or store each component's packed pairs as
// floats.
#include <stdint.h>

#include "lf2_kernels.hpp"
#include "lf2_lengths.hpp"

namespace lf2 {

#ifndef LF2_KX_PART
#define LF2_KX_PART 0
#endif

static inline unsigned x_grid(int64_t nrows, int rb) { return (unsigned)((nrows + rb - 1) / rb); }

// Real-array side of an r2c/c2r pass viewed as complex pairs: pointer and
// every row/plane offset must be even (in floats).
static inline bool pairs_aligned(const void *p, int64_t off, int64_t row, int64_t plane)
{
    return ((uintptr_t)p % 8) == 0 && off % 2 == 0 && row % 2 == 0 && plane % 2 == 0;
}

#if LF2_KX_PART == 0
bool x_supported(int len, int nc)
{
    if (nc != 1 && nc != 2 && nc != 3 && nc != 6) return false;
    switch (len) {
#define LF2_CASE(L) case L:
        LF2_LENGTHS(LF2_CASE)
#undef LF2_CASE
        return true;
    default:
        return false;
    }
}

int x_rows_per_block(int len, int nc) { return x_rb(len, nc); }

template <int L, int NC>
static void r2c_nc(const XArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_x_r2c<L, NC>), dim3(x_grid(a.nrows, x_rb(L, NC))), dim3(kXThreads), 0, s,
                       a);
}

hipError_t launch_x_r2c(int m, int nc, const XArgs &a, hipStream_t s)
{
    const bool vec = nc == 1 && pairs_aligned(a.in, a.in_off, a.in_row, a.in_plane);
#define LF2_CASE(L)                                                                          \
    case L:                                                                                  \
        if (vec)                                                                             \
            hipLaunchKernelGGL((k_x_r2c_v<L>), dim3(x_grid(a.nrows, x_rb(L, 1))),            \
                               dim3(kXThreads), 0, s, a);                                    \
        else if (nc == 1)                                                                    \
            r2c_nc<L, 1>(a, s);                                                              \
        else if (nc == 2)                                                                    \
            r2c_nc<L, 2>(a, s);                                                              \
        else if (nc == 3)                                                                    \
            r2c_nc<L, 3>(a, s);                                                              \
        else if (nc == 6)                                                                    \
            r2c_nc<L, 6>(a, s);                                                              \
        else                                                                                 \
            return hipErrorInvalidValue;                                                     \
        return hipGetLastError();
    switch (m) {
        LF2_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}
#endif

#if LF2_KX_PART == 1
template <int L, int NC>
static void c2r_nc(const XArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_x_c2r<L, NC>), dim3(x_grid(a.nrows, x_rb(L, NC))), dim3(kXThreads), 0, s,
                       a);
}

hipError_t launch_x_c2r(int m, int nc, const XArgs &a, hipStream_t s)
{
    const bool vec = nc == 1 && pairs_aligned(a.out, a.out_off, a.out_row, a.out_plane);
#define LF2_CASE(L)                                                                          \
    case L:                                                                                  \
        if (vec)                                                                             \
            hipLaunchKernelGGL((k_x_c2r_v<L>), dim3(x_grid(a.nrows, x_rb(L, 1))),            \
                               dim3(kXThreads), 0, s, a);                                    \
        else if (nc == 1)                                                                    \
            c2r_nc<L, 1>(a, s);                                                              \
        else if (nc == 2)                                                                    \
            c2r_nc<L, 2>(a, s);                                                              \
        else if (nc == 3)                                                                    \
            c2r_nc<L, 3>(a, s);                                                              \
        else if (nc == 6)                                                                    \
            c2r_nc<L, 6>(a, s);                                                              \
        else                                                                                 \
            return hipErrorInvalidValue;                                                     \
        return hipGetLastError();
    switch (m) {
        LF2_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}
#endif

#if LF2_KX_PART == 2
template <int L, int NC>
static void c2c_nc(int sign, const XArgs &a, hipStream_t s)
{
    if (sign < 0)
        hipLaunchKernelGGL((k_x_c2c_v<L, NC, -1>), dim3(x_grid(a.nrows, x_rb(L, NC))),
                           dim3(kXThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_x_c2c_v<L, NC, 1>), dim3(x_grid(a.nrows, x_rb(L, NC))),
                           dim3(kXThreads), 0, s, a);
}

// Lane j ^ M's value of v, for lanes in groups of eight (M = 1, 2, 4).
// DPP: data-parallel moves of the VALU (quad permutes for M = 1 and 2; for
// M = 4 a shift by four lanes either way within each row of sixteen lanes,
// the right one selected per lane); otherwise ds_bpermute (the LDS
// crossbar, no LDS memory).
template <int M, bool DPP>
__device__ __forceinline__ float lane_xor(float v, int j)
{
    if constexpr (!DPP) {
        return __shfl_xor(v, M);
    } else {
        const int x = __float_as_int(v);
        if constexpr (M == 1) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));
        if constexpr (M == 2) return __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));
        const int up = __builtin_amdgcn_update_dpp(0, x, 0x104, 0xF, 0xF, false);    // lane + 4
        const int down = __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // lane - 4
        return __int_as_float((j & 4) ? down : up);
    }
}

// One pair of one round of the 8 x 8 exchange (registers r0 and r1 = r0 | M
// of lanes j and j ^ M): the lane with bit M clear keeps r0 and receives its
// partner's r0 into r1; the other keeps r1 and receives r0.
template <int M, bool DPP>
__device__ __forceinline__ void xpair(c32 &a0, c32 &a1, int j)
{
    const bool hi = (j & M) != 0;
    const c32 b0 = a0, b1 = a1;  // values, so that the selects are of values
    const c32 send = c32{hi ? b0.x : b1.x, hi ? b0.y : b1.y};
    const c32 got = c32{lane_xor<M, DPP>(send.x, j), lane_xor<M, DPP>(send.y, j)};
    a0 = c32{hi ? got.x : b0.x, hi ? got.y : b0.y};
    a1 = c32{hi ? b1.x : got.x, hi ? b1.y : got.y};
}

// The three rounds (lane bits 4, 2, 1), each swapping a register bit with
// the same lane bit: element (lane j, register k) ends in lane k, register j.
template <bool DPP>
__device__ __forceinline__ void xchg8(c32 (&v)[8], int j)
{
    xpair<4, DPP>(v[0], v[4], j);
    xpair<4, DPP>(v[1], v[5], j);
    xpair<4, DPP>(v[2], v[6], j);
    xpair<4, DPP>(v[3], v[7], j);
    xpair<2, DPP>(v[0], v[2], j);
    xpair<2, DPP>(v[1], v[3], j);
    xpair<2, DPP>(v[4], v[6], j);
    xpair<2, DPP>(v[5], v[7], j);
    xpair<1, DPP>(v[0], v[1], j);
    xpair<1, DPP>(v[2], v[3], j);
    xpair<1, DPP>(v[4], v[5], j);
    xpair<1, DPP>(v[6], v[7], j);
}

// c2c rows of 64 points (one component) with the exchange between the two
// radix-8 stages done across lanes instead of through LDS: eight lanes per
// row, lane j holding points j + 8 r.  Stage one is an 8-point DFT per
// lane; after the twiddles W_64^(j k), lane j holds element (j, k) of an
// 8 x 8 block spread over the row's lanes, and three rounds of lane
// exchanges (lane bits 4, 2, 1) leave element (j, k) in lane k, register
// j, where stage two runs; lane k then holds the outputs k + 8 k2.  No LDS
// exchange and no block barrier.  DPP: the exchanges as VALU moves, else
// as ds_bpermute.
template <int S, bool DPP>
__global__ __launch_bounds__(256) void k_x_c2c_s64(XArgs a)
{
    constexpr int L = 64, R = 8, ROWS = 256 / R;
    __shared__ c32 tw[L];
    load_table(tw, a.tw, L, threadIdx.x, 256);
    __syncthreads();
    const int j = threadIdx.x & (R - 1);
    const int64_t row = (int64_t)blockIdx.x * ROWS + (threadIdx.x >> 3);
    if (row >= a.nrows) return;  // whole 8-lane groups leave together
    const int64_t z = row / a.n1, y = row - z * a.n1;
    const c32 *src = (const c32 *)a.in + a.in_off + z * a.in_plane + y * a.in_row + j;
    c32 *dst = (c32 *)a.out + a.out_off + z * a.out_plane + y * a.out_row + j;
    c32 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = gload<true>(src + R * r);
    Dft<R, S>::run(v);
#pragma unroll
    for (int k = 1; k < R; ++k) {
        c32 w = tw[(j * k) & (L - 1)];
        if (S > 0) w = conjg(w);
        v[k] = mul(v[k], w);
    }
    xchg8<DPP>(v, j);
    Dft<R, S>::run(v);
#pragma unroll
    for (int k2 = 0; k2 < R; ++k2) gstore<true>(dst + R * k2, v[k2]);
}

hipError_t launch_x_c2c_shfl(int sign, bool dpp, const XArgs &a, hipStream_t s)
{
    const unsigned g = x_grid(a.nrows, 256 / 8);
    if (sign < 0 && dpp)
        hipLaunchKernelGGL((k_x_c2c_s64<-1, true>), dim3(g), dim3(256), 0, s, a);
    else if (sign < 0)
        hipLaunchKernelGGL((k_x_c2c_s64<-1, false>), dim3(g), dim3(256), 0, s, a);
    else if (dpp)
        hipLaunchKernelGGL((k_x_c2c_s64<1, true>), dim3(g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_x_c2c_s64<1, false>), dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_x_c2c(int len, int nc, int sign, const XArgs &a, hipStream_t s)
{
#define LF2_CASE(L)                                                                          \
    case L:                                                                                  \
        if (nc == 1)                                                                         \
            c2c_nc<L, 1>(sign, a, s);                                                        \
        else if (nc == 2)                                                                    \
            c2c_nc<L, 2>(sign, a, s);                                                        \
        else if (nc == 3)                                                                    \
            c2c_nc<L, 3>(sign, a, s);                                                        \
        else if (nc == 6)                                                                    \
            c2c_nc<L, 6>(sign, a, s);                                                        \
        else                                                                                 \
            return hipErrorInvalidValue;                                                     \
        return hipGetLastError();
    switch (len) {
        LF2_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}
#endif

}  // namespace lf2
