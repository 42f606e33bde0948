// lf2_kfield.hip -- field operations of the paper's second benchmark
// (section 4.2): the periodic halo update of a halo-padded field and the
// first-order forward derivative of every component into another field.
// Both are HBM-bound copies/stencils with one pass over the data.
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "lf2_internal.hpp"

namespace lf2 {

// Periodic halo update.  The halo sites of the padded box are enumerated so
// that no thread visits an interior site: whole padded rows for the 2h
// z-planes (all y) and for the 2h y-rows of the interior planes, one block
// per row with the row's source computed once and 4-byte words walked
// contiguously; then the 2h x-sites at both ends of every interior row,
// one thread per (row, site, word).  Every source is the interior site at
// the coordinates taken modulo the extents (any h, also h > n).
struct HaloArgs {
    uint32_t *f;
    int64_t n0, n1, n2, h;
    int64_t p0, p1;    // padded extents of x and y
    int64_t words;     // 4-byte words per site
    int64_t rows_z;    // 2h p1 rows of the z slabs
    int64_t rows;      // rows_z + n2 2h rows of the y slabs (one block each)
    int64_t xwork;     // n2 n1 2h words threads of the x slabs
};

__device__ __forceinline__ int64_t halo_wrap(int64_t c, int64_t h, int64_t n)
{
    return h + ((c - h) % n + n) % n;
}

__global__ __launch_bounds__(256) void k_update_halo(HaloArgs a)
{
    const int words = (int)a.words, p0 = (int)a.p0, h = (int)a.h, n0 = (int)a.n0;
    const int64_t rowwords = a.p0 * a.words;
    if ((int64_t)blockIdx.x < a.rows) {
        const int64_t r = blockIdx.x;
        int64_t z, y;
        if (r < a.rows_z) {  // z slabs: planes [0, h) and [n2 + h, n2 + 2h), all rows
            const int64_t pl = r / a.p1;
            y = r - pl * a.p1;
            z = pl < a.h ? pl : a.n2 + pl;
        } else {  // y slabs of the interior planes
            const int64_t u = r - a.rows_z, pl = u / (2 * a.h), row = u - pl * (2 * a.h);
            z = a.h + pl;
            y = row < a.h ? row : a.n1 + row;
        }
        const uint32_t *src =
            a.f + (halo_wrap(z, a.h, a.n2) * a.p1 + halo_wrap(y, a.h, a.n1)) * rowwords;
        uint32_t *dst = a.f + (z * a.p1 + y) * rowwords;
        for (int i = threadIdx.x; i < p0 * words; i += 256) {
            const int x = i / words, w = i - x * words;
            const int sx = (x >= h && x < h + n0) ? x : h + ((x - h) % n0 + n0) % n0;
            dst[i] = src[sx * words + w];
        }
        return;
    }
    const int64_t e = ((int64_t)blockIdx.x - a.rows) * 256 + threadIdx.x;
    if (e >= a.xwork) return;
    const int per = 2 * h * words;  // words of the x halo of one row
    const int64_t row = e / per;
    const int c = (int)(e - row * per), k = c / words, w = c - k * words;
    const int64_t zi = row / a.n1, yi = row - zi * a.n1;
    const int x = k < h ? k : n0 + k;
    const int sx = h + ((x - h) % n0 + n0) % n0;
    uint32_t *base = a.f + ((a.h + zi) * a.p1 + a.h + yi) * rowwords;
    base[x * words + w] = base[sx * words + w];
}

hipError_t launch_update_halo(void *field, const int64_t n[3], int64_t h, int64_t site_words,
                              hipStream_t s)
{
    if (h == 0) return hipSuccess;
    HaloArgs a;
    a.f = (uint32_t *)field;
    a.n0 = n[0];
    a.n1 = n[1];
    a.n2 = n[2];
    a.h = h;
    a.p0 = n[0] + 2 * h;
    a.p1 = n[1] + 2 * h;
    a.words = site_words;
    a.rows_z = 2 * h * a.p1;
    a.rows = a.rows_z + n[2] * 2 * h;
    a.xwork = n[2] * n[1] * 2 * h * site_words;
    const int64_t blocks = a.rows + (a.xwork + 255) / 256;
    if (blocks > 0x7fffffff || a.p0 * site_words > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_update_halo, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// First-order forward derivative of every component along x, y and z:
// out(x)[3 c + i] = (f(x + e_i) - f(x))[c] / dx.  The input's halo (width
// h >= 1) supplies the neighbours across the upper faces; the output has
// the same halo layout and only its interior is written.  A row of the
// field is a run of N0 ncomp words (site-major, components inner).  A row
// is split evenly over the fewest blocks of at most 768 threads (one word a
// thread): long contiguous runs per block matter more here than deep row
// groups.  A block covers its words in GY consecutive rows and marches
// through ZC planes: per plane it reads GY + 1 rows of the following plane
// (the extra row is the y neighbour of the group's last row), which later
// serve as the current plane.  Those reads run one plane ahead of the
// arithmetic.  The x neighbour is the word ncomp further on: the current
// plane's rows go through LDS (plus the ncomp words past the block's end,
// read from memory), so it is not read again.  The three results of a word
// are adjacent in the output and leave as one 12-byte store, so every store
// of a wave is one contiguous run.  Tiles that overlap (the boundary rows,
// planes and cache lines they share) are walked by one XCD at a time, so
// the shared lines mostly come from L2.
struct GradArgs {
    const float *in;
    float *out;
    int64_t n0, n1, n2, h, p0, p1;
    int nc;
    float inv_dx;
    int zc;
    int width;       // words per tile along x (the block size)
    int gx, gy, gz;  // tiles along x (width words), y (GY rows), z (zc planes)
};

constexpr int kGradMaxThreads = 768;  // widest block (words of a row)
constexpr int kGradRows = 4;          // GY
constexpr int kGradPlanes = 32;       // ZC
constexpr int kGradMaxComp = 64;  // largest ncomp

// Three adjacent floats at a 4-byte aligned address.
struct __attribute__((packed, aligned(4))) Float3 {
    float x, y, z;
};

__global__ __launch_bounds__(kGradMaxThreads) void k_gradient(GradArgs a)
{
    constexpr int GY = kGradRows;
    __shared__ float cur[GY][kGradMaxThreads + kGradMaxComp];
    const int tid = threadIdx.x;
    const int nt = a.width;  // threads (words) of a block
    const int64_t rowwords = a.n0 * a.nc;
    // The chip hands block ids to its 8 XCDs in turn.  Block i serves tile
    // number start(i mod 8) + i / 8, so each XCD walks a contiguous range of
    // tiles (x fastest, then y, then z): neighbouring tiles, which share the
    // cache lines at their x ends (rows are not 128-byte aligned) and their
    // boundary rows, run at the same time behind one L2.
    const int nb = a.gx * a.gy * a.gz;
    const int q = nb >> 3, r = nb & 7, j = blockIdx.x & 7;
    const int tile = j * q + (j < r ? j : r) + (int)(blockIdx.x >> 3);
    const int bx = tile % a.gx, byz = tile / a.gx;
    const int by = byz % a.gy, bz = byz / a.gy;
    const int64_t w0 = (int64_t)bx * nt;
    const int64_t w = w0 + tid;
    // words up to rowwords + ncomp - 1 (the upper halo site) are read: the
    // last interior words take their x neighbours from them
    const bool ld = w < rowwords + a.nc;
    const bool st = w < rowwords;
    const int64_t y0 = (int64_t)by * GY;
    const int ny = (int)(a.n1 - y0 < GY ? a.n1 - y0 : GY);  // rows of this group
    const int64_t z0 = (int64_t)bz * a.zc;
    const int64_t z1 = z0 + a.zc < a.n2 ? z0 + a.zc : a.n2;
    const int64_t sy = a.p0 * a.nc, sz = a.p1 * a.p0 * a.nc;  // input strides (words)
    // input word w of interior row y0 + i of plane z0; rows past the group
    // are read from row min(y0 + i, n1), which exists (upper halo row n1)
    const float *f = a.in + ((a.h + z0) * a.p1 + a.h + y0) * sy + a.h * a.nc + (ld ? w : 0);
    // row offsets (words; below 2^31: GY rows of at most 2^31 / GY words)
    int roff[GY + 1];
#pragma unroll
    for (int i = 0; i <= GY; ++i) roff[i] = (i <= ny ? i : ny) * (int)sy;
    // c: plane z, nx: plane z + 1 (both rows y0 .. y0 + GY)
    float c[GY + 1], nx[GY + 1];
#pragma unroll
    for (int i = 0; i <= GY; ++i) {
        c[i] = ld ? f[roff[i]] : 0.f;
        nx[i] = ld ? f[sz + roff[i]] : 0.f;
    }
    // words w0 + nt + t (t < ncomp) hold the last threads' x neighbours;
    // they exist while w0 + nt + t < rowwords + ncomp (upper halo site)
    const bool extra = tid < a.nc && w0 + nt + tid < rowwords + a.nc;
    const float *fe = a.in + ((a.h + z0) * a.p1 + a.h + y0) * sy + a.h * a.nc +
                      (extra ? w0 + nt + tid : 0);
    float *o = a.out + ((a.h + z0) * a.p1 + a.h + y0) * (sy * 3) + a.h * a.nc * 3 + 3 * w;
    const int64_t oy = sy * 3;
    for (int64_t z = z0; z < z1; ++z) {
        // the next step's planes, read only while z + 2 <= z1 <= n2 (the
        // upper halo plane n2 exists)
        float nn[GY + 1];
        const bool more = z + 1 < z1;
#pragma unroll
        for (int i = 0; i <= GY; ++i) nn[i] = (ld && more) ? f[2 * sz + roff[i]] : 0.f;
#pragma unroll
        for (int i = 0; i < GY; ++i) {
            cur[i][tid] = c[i];
            if (extra) cur[i][nt + tid] = fe[roff[i]];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < GY; ++i) {
            if (st && i < ny) {
                const float xn = cur[i][tid + a.nc];
                *(Float3 *)(o + i * oy) = Float3{(xn - c[i]) * a.inv_dx, (c[i + 1] - c[i]) * a.inv_dx,
                                                 (nx[i] - c[i]) * a.inv_dx};
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i <= GY; ++i) {
            c[i] = nx[i];
            nx[i] = nn[i];
        }
        f += sz;
        fe += sz;
        o += sz * 3;
    }
}

hipError_t launch_gradient(const float *in, float *out, const int64_t n[3], int64_t h, int nc,
                           double dx, hipStream_t s)
{
    GradArgs a;
    a.in = in;
    a.out = out;
    a.n0 = n[0];
    a.n1 = n[1];
    a.n2 = n[2];
    a.h = h;
    a.p0 = n[0] + 2 * h;
    a.p1 = n[1] + 2 * h;
    a.nc = nc;
    a.inv_dx = (float)(1.0 / dx);
    a.zc = kGradPlanes;
    const int64_t rowwords = n[0] * nc;
    if ((int64_t)(kGradRows + 1) * a.p0 * nc > 0x7fffffff) return hipErrorInvalidValue;
    // the fewest blocks of at most kGradMaxThreads words per row, as even
    // as whole wavefronts allow
    const int64_t gx = (rowwords + kGradMaxThreads - 1) / kGradMaxThreads;
    a.width = (int)(((rowwords + gx - 1) / gx + 63) / 64 * 64);
    const int64_t gy = (n[1] + kGradRows - 1) / kGradRows, gz = (n[2] + a.zc - 1) / a.zc;
    if (gx * gy * gz > 0x7fffffff) return hipErrorInvalidValue;
    a.gx = (int)gx;
    a.gy = (int)gy;
    a.gz = (int)gz;
    hipLaunchKernelGGL(k_gradient, dim3((unsigned)(gx * gy * gz)), dim3(a.width), 0, s, a);
    return hipGetLastError();
}

}  // namespace lf2
