// lf2_ks.hip -- instantiations and launcher of the strided (y / z) pass.
#include "lf2_kernels.hpp"
#include "lf2_lengths.hpp"

namespace lf2 {

bool s_supported(int len)
{
    switch (len) {
#define LF2_CASE(L) case L:
        LF2_S_LENGTHS(LF2_CASE)
#undef LF2_CASE
        return true;
    default:
        return false;
    }
}

int s_cols_per_block(int len) { return s_b(len); }

int epi_hist_copies(int len, int nbins, size_t budget)
{
    constexpr int kWaves = kSThreads / 64;
    switch (len) {
#define LF2_CASE(L)                                                                          \
    case L: {                                                                                \
        const size_t tile = STile<L, -1, true, kSThreads, true>::BYTES;                      \
        return tile + (size_t)(nbins + 1) * 8 * (kWaves + 1) <= budget ? kWaves : 1;         \
    }
        LF2_S_LENGTHS(LF2_CASE)
#undef LF2_CASE
    default:
        return 0;
    }
}

// Lengths with a wide (split-exchange) tile: the long lines, whose narrow
// tiles read the shortest row segments.
#define LF2_WIDE_LENGTHS(X) X(256) X(320) X(384) X(512) X(640) X(768) X(1024) X(2048)

bool s_wide_supported(int len)
{
    switch (len) {
#define LF2_CASE(L) case L:
        LF2_WIDE_LENGTHS(LF2_CASE)
#undef LF2_CASE
        return true;
    default:
        return false;
    }
}

template <int L, bool NTM>
static void wide_k(int sign, int g, const SArgs &a, hipStream_t s)
{
    if (sign < 0)
        hipLaunchKernelGGL((k_strided_w<L, -1, NTM>), dim3(g), dim3(kSWThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_strided_w<L, 1, NTM>), dim3(g), dim3(kSWThreads), 0, s, a);
}

template <int L, bool NTM>
static void narrow_k(int sign, int g, const SArgs &a, hipStream_t s)
{
    if (sign < 0)
        hipLaunchKernelGGL((k_strided<L, -1, false, NTM>), dim3(g), dim3(kSThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_strided<L, 1, false, NTM>), dim3(g), dim3(kSThreads), 0, s, a);
}

static hipError_t launch_wide(int len, int sign, const SArgs &a, int grid_cap, hipStream_t s,
                              int *grid_used, int chunk, bool ntm)
{
#define LF2_CASE(L)                                                                          \
    case L: {                                                                                \
        constexpr int B = STileW<L, 1, kSWThreads>::B;                                        \
        int64_t ntiles = (a.ncols + B - 1) / B;                                              \
        int64_t span = (ntiles + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);                 \
        int g = (int)(span < grid_cap ? span : grid_cap);                                    \
        if (grid_used) *grid_used = g;                                                       \
        if (ntm)                                                                             \
            wide_k<L, true>(sign, g, a, s);                                                  \
        else                                                                                 \
            wide_k<L, false>(sign, g, a, s);                                                 \
        return hipGetLastError();                                                            \
    }
    switch (len) {
        LF2_WIDE_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}

static hipError_t launch_transposed(int len, int sign, const SArgs &a, int grid_cap,
                                    hipStream_t s, int *grid_used)
{
#define LF2_CASE(L)                                                                          \
    case L: {                                                                                \
        int64_t ntiles = (a.ncols + s_b(L) - 1) / s_b(L);                                    \
        int g = (int)(ntiles < grid_cap ? ntiles : grid_cap);                                \
        if (grid_used) *grid_used = g;                                                       \
        if (sign < 0)                                                                        \
            hipLaunchKernelGGL((k_strided_t<L, -1>), dim3(g), dim3(kSThreads), 0, s, a);     \
        else                                                                                 \
            hipLaunchKernelGGL((k_strided_t<L, 1>), dim3(g), dim3(kSThreads), 0, s, a);      \
        return hipGetLastError();                                                            \
    }
    switch (len) {
        LF2_S_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}

hipError_t launch_strided(int len, int sign, const SArgs &a_in, int grid_cap, hipStream_t s,
                          int *grid_used, int variant, int chunk)
{
    // `chunk` tiles per XCD chunk; the grid is a multiple of 8 (grid_cap is).
    const int kChunk = chunk > 0 ? chunk : 16;
    SArgs a = a_in;
    a.xcd_chunk = kChunk;
    grid_cap = grid_cap / 8 * 8;
    if (grid_cap < 8) grid_cap = 8;
    const bool pk = (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
    const bool epi = (a.epi & (EPI_PK | EPI_PK_AFTER | EPI_POISSON)) != 0;
    // one histogram per wave where the LDS allows (two blocks per CU, one
    // for lines of 1024 points and more)
    a.hcopies = pk ? epi_hist_copies(len, a.mt.nbins, len >= 1024 ? 160 * 1024 : 80 * 1024) : 1;
    if (a.hcopies < 1) a.hcopies = 1;
    const size_t shm = pk ? (size_t)(a.mt.nbins + 1) * 8 * (a.hcopies + 1) : 0;
    if (a.epi & (EPI_TSTORE | EPI_TLOAD)) {
        if (epi) return hipErrorInvalidValue;
        return launch_transposed(len, sign, a, grid_cap, s, grid_used);
    }
    if (variant & 8) {
        if (!epi || sign > 0 || !(a.epi & EPI_POISSON) || !fused_reg_supported(len))
            return hipErrorInvalidValue;
        return launch_fused_reg(len, a, shm, grid_cap, s, grid_used);
    }
    const bool ntm = (variant & 2) != 0;
    if (variant & 4) {
        if (epi || (variant & 1) || !s_reg_supported(len)) return hipErrorInvalidValue;
        return launch_strided_reg(len, sign, a, grid_cap, s, grid_used, kChunk, ntm);
    }
    if (variant & 1) {
        if (epi || !s_wide_supported(len)) return hipErrorInvalidValue;
        return launch_wide(len, sign, a, grid_cap, s, grid_used, kChunk, ntm);
    }
    if (epi && ntm) return hipErrorInvalidValue;
#define LF2_CASE(L)                                                                          \
    case L: {                                                                                \
        int64_t ntiles = (a.ncols + s_b(L) - 1) / s_b(L);                                    \
        int64_t span = (ntiles + 8 * kChunk - 1) / (8 * kChunk) * (8 * kChunk);              \
        int g = (int)(span < grid_cap ? span : grid_cap);                                    \
        if (grid_used) *grid_used = g;                                                       \
        if (epi && sign < 0 && a.mt.k2z_unit > 0.0)                                          \
            hipLaunchKernelGGL((k_strided<L, -1, true, true, 1>), dim3(g), dim3(kSThreads), shm, \
                               s, a);                                                        \
        else if (epi && sign < 0)                                                            \
            hipLaunchKernelGGL((k_strided<L, -1, true, true, 2>), dim3(g), dim3(kSThreads), shm, \
                               s, a);                                                        \
        else if (epi)                                                                        \
            return hipErrorInvalidValue;                                                     \
        else if (ntm)                                                                        \
            narrow_k<L, true>(sign, g, a, s);                                                \
        else                                                                                 \
            narrow_k<L, false>(sign, g, a, s);                                               \
        return hipGetLastError();                                                            \
    }
    switch (len) {
        LF2_S_LENGTHS(LF2_CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef LF2_CASE
}

}  // namespace lf2
