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
