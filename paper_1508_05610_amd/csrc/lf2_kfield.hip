// lf2_kfield.hip -- field operations of the paper's second benchmark
// (section 4.2): the periodic halo update of a halo-padded field and the
// first-order forward derivative of every component into another field.
// Both are HBM-bound copies/stencils with one pass over the data.
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "lf2_internal.hpp"

namespace lf2 {

// Periodic halo update.  The halo sites of the padded box are enumerated in
// three slabs so that no thread visits an interior site: the 2h z-planes
// (all y, x), the 2h y-rows of the interior planes (all x), and the 2h
// x-sites of the interior rows.  Thread = (halo site, 4-byte word of the
// site), words fastest, so rows copy contiguously.
struct HaloArgs {
    uint32_t *f;
    int64_t n0, n1, n2, h;
    int64_t p0, p1;  // padded extents of x and y
    int64_t words;   // 4-byte words per site
    int64_t nz, ny, nx, total;  // sites in the three slabs and their sum
};

__global__ __launch_bounds__(256) void k_update_halo(HaloArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < a.total * a.words;
         t += stride) {
        const int64_t s = t / a.words, w = t - s * a.words;
        int64_t x, y, z;
        if (s < a.nz) {  // z slabs: 2h planes of p1 x p0 sites
            const int64_t pl = s / (a.p1 * a.p0), r = s - pl * (a.p1 * a.p0);
            z = pl < a.h ? pl : a.n2 + pl;  // [0, h) then [n2 + h, n2 + 2h)
            y = r / a.p0;
            x = r - y * a.p0;
        } else if (s < a.nz + a.ny) {  // y slabs: n2 planes x 2h rows x p0
            const int64_t u = s - a.nz;
            const int64_t pl = u / (2 * a.h * a.p0), r = u - pl * (2 * a.h * a.p0);
            const int64_t row = r / a.p0;
            z = a.h + pl;
            y = row < a.h ? row : a.n1 + row;
            x = r - row * a.p0;
        } else {  // x slabs: n2 x n1 interior rows x 2h sites
            const int64_t u = s - a.nz - a.ny;
            const int64_t rowi = u / (2 * a.h), c = u - rowi * (2 * a.h);
            z = a.h + rowi / a.n1;
            y = a.h + rowi % a.n1;
            x = c < a.h ? c : a.n0 + c;
        }
        // source: the interior site at the coordinates modulo the extents
        const int64_t sz = a.h + ((z - a.h) % a.n2 + a.n2) % a.n2;
        const int64_t sy = a.h + ((y - a.h) % a.n1 + a.n1) % a.n1;
        const int64_t sx = a.h + ((x - a.h) % a.n0 + a.n0) % a.n0;
        const int64_t dst = ((z * a.p1 + y) * a.p0 + x) * a.words + w;
        const int64_t src = ((sz * a.p1 + sy) * a.p0 + sx) * a.words + w;
        a.f[dst] = a.f[src];
    }
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
    a.nz = 2 * h * a.p1 * a.p0;
    a.ny = n[2] * 2 * h * a.p0;
    a.nx = n[2] * n[1] * 2 * h;
    a.total = a.nz + a.ny + a.nx;
    const int64_t work = a.total * a.words;
    const int64_t blocks = (work + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_update_halo, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

// First-order forward derivative of every component along x, y and z:
// out(x)[3 c + i] = (f(x + e_i) - f(x))[c] / dx.  The input's halo (width
// h >= 1) supplies the neighbours across the upper faces; the output has
// the same halo layout and only its interior is written.  A row of the
// field is a run of N0 ncomp words (site-major, components inner); a block
// covers 256 consecutive words of one row and marches through ZC planes,
// carrying f(z + 1) over as the next plane's f(z).  Its x neighbour is the
// word ncomp further on and its y neighbour the same word of the next row,
// both loaded by this or a neighbouring block at the same time (cache
// hits).  The three results of a word are staged through LDS so that every
// store of a wave is contiguous.
struct GradArgs {
    const float *in;
    float *out;
    int64_t n0, n1, n2, h, p0, p1;
    int nc;
    float inv_dx;
    int zc;
};

constexpr int kGradThreads = 256;

__global__ __launch_bounds__(kGradThreads) void k_gradient(GradArgs a)
{
    __shared__ float stage[3 * kGradThreads];
    const int tid = threadIdx.x;
    const int64_t rowwords = a.n0 * a.nc;
    const int64_t w0 = (int64_t)blockIdx.x * kGradThreads;
    const int64_t w = w0 + tid;
    const bool ok = w < rowwords;
    const int64_t y = blockIdx.y;
    const int64_t z0 = (int64_t)blockIdx.z * a.zc;
    const int64_t z1 = z0 + a.zc < a.n2 ? z0 + a.zc : a.n2;
    const int64_t sy = a.p0 * a.nc, sz = a.p1 * a.p0 * a.nc;  // input strides (words)
    const int64_t osz = sz * 3;                                 // output plane stride
    const int64_t ib = ((a.h + z0) * a.p1 + a.h + y) * sy + a.h * a.nc;
    const int64_t ob = ((a.h + z0) * a.p1 + a.h + y) * (sy * 3) + a.h * a.nc * 3;
    const float *f = a.in + ib + (ok ? w : 0);
    float *o = a.out + ob + 3 * w0;
    const int nst = (int)(3 * (rowwords - w0 < kGradThreads ? rowwords - w0 : kGradThreads));
    float cur = ok ? f[0] : 0.f;
    // the next plane's x and y neighbours are loaded one step ahead
    float fx = ok ? f[a.nc] : 0.f, fy = ok ? f[sy] : 0.f;
    for (int64_t z = z0; z < z1; ++z) {
        float nxt = 0.f, fx2 = 0.f, fy2 = 0.f;
        if (ok) {
            nxt = f[sz];
            if (z + 1 < z1) {
                fx2 = f[sz + a.nc];
                fy2 = f[sz + sy];
            }
        }
        stage[3 * tid + 0] = (fx - cur) * a.inv_dx;
        stage[3 * tid + 1] = (fy - cur) * a.inv_dx;
        stage[3 * tid + 2] = (nxt - cur) * a.inv_dx;
        __syncthreads();
        for (int j = tid; j < nst; j += kGradThreads) o[j] = stage[j];
        __syncthreads();
        cur = nxt;
        fx = fx2;
        fy = fy2;
        f += sz;
        o += osz;
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
    a.zc = 16;
    const int64_t rowwords = n[0] * nc;
    dim3 grid((unsigned)((rowwords + kGradThreads - 1) / kGradThreads), (unsigned)n[1],
              (unsigned)((n[2] + a.zc - 1) / a.zc));
    hipLaunchKernelGGL(k_gradient, grid, dim3(kGradThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace lf2
