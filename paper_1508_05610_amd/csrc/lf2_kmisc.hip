// lf2_kmisc.hip -- plan-time tables (FP64 on the device) and the FP64
// reductions of the power spectrum.
#include "lf2_kernels.hpp"

namespace lf2 {

// exp(-2 pi i m / period) for m in [0, count), evaluated in FP64 with the
// exact integer m (< period) and rounded once to FP32.
__global__ void k_twiddles(c32 *tw, int count, int period)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < count) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)period, &sn, &cs);
        tw[m] = c32{(float)cs, (float)(-sn)};
    }
}

hipError_t launch_twiddles(void *tw, int len, hipStream_t s)
{
    // len > 0: table of `len` entries with period len; len < 0: r2c post
    // table of N0/2 + 1 entries with period N0 = -len.
    const int period = len > 0 ? len : -len;
    const int count = len > 0 ? len : period / 2 + 1;
    hipLaunchKernelGGL(k_twiddles, dim3((count + 255) / 256), dim3(256), 0, s, (c32 *)tw, count,
                       period);
    return hipGetLastError();
}

// Per-axis k^2 contribution for index i of an axis of extent n:
//   continuous: (2 pi nt / (n dx))^2, nt the signed wavenumber;
//   discrete:   (2/dx)^2 sin^2(pi i / n).
__global__ void k_k2_table(double *dst, int n, int count, double dx, int discrete)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        double v;
        if (discrete) {
            const double sn = sinpi((double)i / (double)n);
            v = (4.0 / (dx * dx)) * sn * sn;
        } else {
            const int nt = (2 * i < n) ? i : i - n;
            const double a = 6.283185307179586476925286766559 * (double)nt / ((double)n * dx);
            v = a * a;
        }
        dst[i] = v;
    }
}

hipError_t launch_k2_table(double *dst, int n, int count, double dx, int discrete, hipStream_t s)
{
    hipLaunchKernelGGL(k_k2_table, dim3((count + 255) / 256), dim3(256), 0, s, dst, n, count, dx,
                       discrete);
    return hipGetLastError();
}

// (nt * lfac)^2 for the signed wavenumber nt of index i.
__global__ void k_q_table(int64_t *dst, int n, int count, int64_t lfac)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const int64_t nt = (2 * i < n) ? i : i - n;
        dst[i] = (nt * lfac) * (nt * lfac);
    }
}

hipError_t launch_q_table(int64_t *dst, int n, int count, int64_t lfac, hipStream_t s)
{
    hipLaunchKernelGGL(k_q_table, dim3((count + 255) / 256), dim3(256), 0, s, dst, n, count, lfac);
    return hipGetLastError();
}

// thresh[b] = ceil(b^2 qmax / nbins^2), b = 0..nbins: the smallest integer q
// with b^2 qmax <= nbins^2 q.
__global__ void k_thresholds(int64_t *dst, int nbins, int64_t qmax)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= nbins) {
        const int64_t d = (int64_t)nbins * nbins;
        const int64_t num = (int64_t)b * b * qmax;
        dst[b] = (num + d - 1) / d;
    }
}

hipError_t launch_thresholds(int64_t *dst, int nbins, int64_t qmax, hipStream_t s)
{
    hipLaunchKernelGGL(k_thresholds, dim3((nbins + 1 + 255) / 256), dim3(256), 0, s, dst, nbins,
                       qmax);
    return hipGetLastError();
}

// Shell table of the lattice: per bin, the weighted mode count sum w and
// sum w sqrt(q) over the half (r2c) or full spectrum, zero mode excluded.
// Thread (col, rg) walks a run of kz of one (kx, ky) column (64 adjacent
// columns per tile), keeps the run's sums while the bin stays the same and
// adds them to the block's LDS histograms when it changes (the bin rule and
// edge table of the fused pass).  Partials [grid][nbins] of each.
__global__ __launch_bounds__(256) void k_shell_partials(ModeTables mt, int n1, int n2, double *pc,
                                                        double *pkk)
{
    constexpr int B = 64, NT = 256, RG = NT / B;
    extern __shared__ double sh[];
    const int nb = mt.nbins;
    double *hc = sh;
    double *hk = sh + nb;
    BinEdge *edges = (BinEdge *)(sh + 2 * nb);
    for (int i = threadIdx.x; i < nb; i += NT) {
        hc[i] = 0.0;
        hk[i] = 0.0;
    }
    for (int i = threadIdx.x; i <= nb; i += NT)
        edges[i] = BinEdge{(uint32_t)mt.thresh[i], i < nb - 1 ? (uint32_t)mt.thresh[i + 1] : 0xffffffffu};
    __syncthreads();
    const float cq = (float)((double)nb * nb / mt.qmax);
    const uint32_t qu = mt.qz_unit;
    const int64_t ncols = (int64_t)mt.nxk * n1;
    const int64_t ntiles = (ncols + B - 1) / B;
    const int col = threadIdx.x % B, rg = threadIdx.x / B;
    const int ep = (n2 + RG - 1) / RG;
    const int k0 = rg * ep;
    const int k1 = k0 + ep < n2 ? k0 + ep : n2;  // this thread's run [k0, k1)
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t f = t * B + col;
        if (f >= ncols) continue;
        const int kx = (int)(f % mt.nxk), ky = (int)(f / mt.nxk);
        // the half-spectrum weight (1 or 2, exact) is applied at each flush
        const double w = (mt.half && !(kx == 0 || 2 * kx == mt.n0)) ? 2.0 : 1.0;
        const uint32_t qxy = (uint32_t)(mt.q[0][kx] + mt.q[1][ky]);  // q < 2^32 (plan check)
        int cur = -1;
        double cnt = 0.0, sk = 0.0;
        for (int kz = k0; kz < k1; ++kz) {
            if (kx == 0 && ky == 0 && kz == 0) continue;  // the zero mode is in no bin
            const uint32_t m = (uint32_t)(2 * kz < n2 ? kz : n2 - kz);
            const uint32_t q = qxy + m * m * qu;
            const int b = bin_edge(q, nb, cq, edges);
            if (b != cur) {
                if (cur >= 0) {
                    atomicAdd(&hc[cur], w * cnt);
                    atomicAdd(&hk[cur], w * sk);
                }
                cur = b;
                cnt = 0.0;
                sk = 0.0;
            }
            cnt += 1.0;
            sk += sqrt((double)q);
        }
        if (cur >= 0) {
            atomicAdd(&hc[cur], w * cnt);
            atomicAdd(&hk[cur], w * sk);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += NT) {
        pc[(int64_t)blockIdx.x * nb + i] = hc[i];
        pkk[(int64_t)blockIdx.x * nb + i] = hk[i];
    }
}

hipError_t launch_shell_partials(const ModeTables &mt, int n1, int n2, double /*lscale*/,
                                 double *partial_cnt, double *partial_k, int grid, hipStream_t s)
{
    const size_t shm = (size_t)mt.nbins * 16 + (size_t)(mt.nbins + 1) * 8;
    hipLaunchKernelGGL(k_shell_partials, dim3(grid), dim3(256), shm, s, mt, n1, n2, partial_cnt,
                       partial_k);
    return hipGetLastError();
}

// Fixed-order column sums: out[b] = sum over g of partial[g * width + b].
// One block per column (blocks width1.. serve an optional second array, so
// that two reductions share a launch); thread t keeps four running sums
// over the rows g = t + kRedThreads (4 i + j), j = 0..3 (four loads in
// flight instead of a chain of dependent ones), adds them in a fixed order,
// then a fixed tree combines the thread sums, so the result is reproducible.
constexpr int kRedThreads = 1024;
__global__ __launch_bounds__(kRedThreads) void k_reduce_cols(
    const double *partial1, int64_t grid1, int width1, double *out1, const double *partial2,
    int64_t grid2, int width2, double *out2)
{
    __shared__ double red[kRedThreads];
    const bool first = (int)blockIdx.x < width1;
    const double *partial = first ? partial1 : partial2;
    const int64_t grid = first ? grid1 : grid2;
    const int width = first ? width1 : width2;
    const int b = first ? (int)blockIdx.x : (int)blockIdx.x - width1;
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t g = t;
    for (; g + 3 * kRedThreads < grid; g += 4 * kRedThreads) {
        s0 += partial[g * width + b];
        s1 += partial[(g + kRedThreads) * width + b];
        s2 += partial[(g + 2 * kRedThreads) * width + b];
        s3 += partial[(g + 3 * kRedThreads) * width + b];
    }
    for (; g < grid; g += kRedThreads) s0 += partial[g * width + b];
    red[t] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) (first ? out1 : out2)[b] = red[0];
}

hipError_t launch_reduce_cols2(const double *partial1, int64_t grid1, int width1, double *out1,
                               const double *partial2, int64_t grid2, int width2, double *out2,
                               hipStream_t s)
{
    if (width1 + width2 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_cols, dim3(width1 + width2), dim3(kRedThreads), 0, s, partial1,
                       grid1, width1, out1, partial2, grid2, width2, out2);
    return hipGetLastError();
}

hipError_t launch_reduce_cols(const double *partial, int64_t grid, int width, double *out,
                              hipStream_t s)
{
    return launch_reduce_cols2(partial, grid, width, out, nullptr, 0, 0, nullptr, s);
}

// Power spectrum of a spectrum already in k space ([n2][n1][nxk], ncomp 1).
// Tile of 64 adjacent (kx, ky) columns; thread (col, rg) walks a contiguous
// run of kz, U modes at a time, the next U loads issued before the current
// U modes are binned (one wave reads 64 adjacent modes per load), flushing
// its running bin sum to the LDS histogram when the bin changes.  The bin is the exact integer rule's,
// from the square-root estimate and the LDS edge table as in the fused
// pass.  Partials [grid][nbins + 1] (slot nbins = zero mode).
constexpr int kPkThreads = 512;
__global__ __launch_bounds__(kPkThreads) void k_pk_kspace(const c32 *F, int n1, int n2, int64_t sx,
                                                          int64_t sy, int64_t sz, ModeTables mt,
                                                          double *partial)
{
    constexpr int B = 64, NT = kPkThreads, RG = NT / B, U = 8;
    extern __shared__ double sh[];
    const int nb = mt.nbins;
    double *hist = sh;
    BinEdge *edges = (BinEdge *)(sh + nb + 1);
    load_edges(mt, hist, edges, threadIdx.x, NT);
    __syncthreads();
    const float cq = (float)((double)nb * nb / mt.qmax);
    const uint32_t qu = mt.qz_unit;
    const int64_t ncols = (int64_t)mt.nxk * n1;
    const int64_t ntiles = (ncols + B - 1) / B;
    const int col = threadIdx.x % B, rg = threadIdx.x / B;
    const int ep = (n2 + RG - 1) / RG;
    const int k0 = rg * ep;
    const int k1 = k0 + ep < n2 ? k0 + ep : n2;  // this thread's run [k0, k1)
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t f = t * B + col;
        if (f >= ncols) continue;
        const int kx = (int)(f % mt.nxk), ky = (int)(f / mt.nxk);
        // the half-spectrum weight (1 or 2, exact) is applied at each flush
        const double w = (mt.half && !(kx == 0 || 2 * kx == mt.n0)) ? 2.0 : 1.0;
        const uint32_t qxy = (uint32_t)(mt.q[0][kx] + mt.q[1][ky]);  // q < 2^32 (plan check)
        const c32 *src = F + (int64_t)ky * sy + (int64_t)kx * sx;
        int cur = -1;
        double acc = 0.0;
        c32 vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            vv[u] = k0 + u < k1 ? src[(int64_t)(k0 + u) * sz] : c32{0.f, 0.f};
        for (int kb = k0; kb < k1; kb += U) {
            c32 vn[U];  // the next batch (no loads past the run)
#pragma unroll
            for (int u = 0; u < U; ++u)
                vn[u] = kb + U + u < k1 ? src[(int64_t)(kb + U + u) * sz] : c32{0.f, 0.f};
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kz = kb + u;
                if (kz < k1) {
                    const uint32_t m = (uint32_t)(2 * kz < n2 ? kz : n2 - kz);
                    const uint32_t q = qxy + m * m * qu;
                    const bool zero = kx == 0 && ky == 0 && kz == 0;
                    const int b = zero ? nb : bin_edge(q, nb, cq, edges);
                    const double p = (double)vv[u].x * vv[u].x + (double)vv[u].y * vv[u].y;
                    if (b != cur) {
                        if (cur >= 0) atomicAdd(&hist[cur], w * acc);
                        cur = b;
                        acc = 0.0;
                    }
                    acc += p;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) vv[u] = vn[u];
        }
        if (cur >= 0) atomicAdd(&hist[cur], w * acc);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= nb; i += NT) partial[(int64_t)blockIdx.x * (nb + 1) + i] = hist[i];
}

hipError_t launch_pk_kspace(const void *F, int n1, int n2, int64_t sx, int64_t sy, int64_t sz,
                            const ModeTables &mt, double *partial, int grid, hipStream_t s)
{
    const size_t shm = (size_t)(mt.nbins + 1) * 16;
    hipLaunchKernelGGL(k_pk_kspace, dim3(grid), dim3(kPkThreads), shm, s, (const c32 *)F, n1, n2,
                       sx, sy, sz, mt, partial);
    return hipGetLastError();
}

// From the bin sums S[0..nbins] (S[nbins] = zero mode) and the lattice
// shell table: pk = norm * vscale * S_b / count_b, kmean = kscale * sumk_b /
// count_b (0 for empty bins); parseval = { *sumsq, inv_n * vscale *
// sum_b S_b including the zero mode }.
constexpr int kFinThreads = 256;
__global__ __launch_bounds__(kFinThreads) void k_pk_finalize(
    const double *S, int nbins, const double *count, const double *sumk, double norm,
    double vscale, double kscale, double *pk, double *kmean, double *count_out, double *parseval,
    const double *sumsq, double inv_n)
{
    const int t = threadIdx.x;
    for (int b = t; b < nbins; b += kFinThreads) {
        const double c = count[b];
        if (pk) pk[b] = c > 0 ? norm * vscale * S[b] / c : 0.0;
        if (kmean) kmean[b] = c > 0 ? kscale * sumk[b] / c : 0.0;
        if (count_out) count_out[b] = c;
    }
    if (parseval) {  // uniform over the block
        // sum of all nbins + 1 slots (the zero mode included): per-thread
        // strided sums, then a fixed tree
        __shared__ double red[kFinThreads];
        double a = 0.0;
        for (int b = t; b <= nbins; b += kFinThreads) a += S[b];
        red[t] = a;
        __syncthreads();
        for (int h = kFinThreads / 2; h > 0; h >>= 1) {
            if (t < h) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) {
            parseval[0] = sumsq ? *sumsq : 0.0;
            parseval[1] = inv_n * vscale * red[0];
        }
    }
}

hipError_t launch_pk_finalize(const double *S, int nbins, const double *count, const double *sumk,
                              double norm, double vscale, double kscale, double *pk,
                              double *kmean, double *count_out, double *parseval,
                              const double *sumsq, double inv_n, hipStream_t s)
{
    hipLaunchKernelGGL(k_pk_finalize, dim3(1), dim3(kFinThreads), 0, s, S, nbins, count, sumk, norm,
                       vscale, kscale, pk, kmean, count_out, parseval, sumsq, inv_n);
    return hipGetLastError();
}

}  // namespace lf2
