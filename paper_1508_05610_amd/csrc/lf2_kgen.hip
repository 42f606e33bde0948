// lf2_kgen.hip -- pass kernels whose radix schedule is chosen at run time:
// any line length 2^a 3^b 5^c that has no compiled kernel, and the
// alternative schedules the plan-time tuner times against the compiled ones.
//
// A tile's lines sit in LDS twice (ping-pong): each Stockham stage reads one
// buffer and writes the other, so a stage needs no registers beyond one
// butterfly per thread whatever its radix and the line length.  Tiles:
//   x pass   : RB rows (all components), lines contiguous (row-major);
//   strided  : B adjacent columns x L points, loaded row by row (B * 8
//              contiguous bytes per row), lanes walking adjacent columns.
// The fused last-axis pass (Poisson scale and power-spectrum binning) works
// on the tile in LDS between the forward and the backward transform.
#include "lf2_gen.hpp"
#include "lf2_kernels.hpp"

namespace lf2 {

constexpr int kGThreads = 512;

// One Stockham stage (see lf2_device.hpp) of radix R on NL lines of length
// L, src -> dst.  COLS: element (line l, point p) at l + p NL; otherwise at
// l L + p.  Consecutive threads take consecutive lines (COLS) or points.
template <int R, int S, bool COLS>
__device__ void gstage(const c32 *src, c32 *dst, int NL, int L, int NS, const c32 *tw, int tid)
{
    const int Q = L / R;
    const int tstep = L / (NS * R);
    const int total = NL * Q;
    for (int b = tid; b < total; b += kGThreads) {
        const int l = COLS ? b % NL : b / Q;
        const int j = COLS ? b / NL : b % Q;
        const int k = j % NS;
        c32 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int p = j + r * Q;
            v[r] = COLS ? src[l + p * NL] : src[l * L + p];
        }
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c32 w = tw[r * k * tstep];
                if (S > 0) w = conjg(w);
                v[r] = mul(v[r], w);
            }
        }
        Dft<R, S>::run(v);
        const int p0 = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int p = p0 + r * NS;
            if (COLS)
                dst[l + p * NL] = v[r];
            else
                dst[l * L + p] = v[r];
        }
    }
}

// Every stage of sc over the lines in b0 (b1: the other buffer); returns
// the buffer that holds the transform.  Ends at a barrier.
template <int S, bool COLS>
__device__ c32 *glines(c32 *b0, c32 *b1, int NL, int L, const GSched &sc, const c32 *tw, int tid)
{
    c32 *src = b0, *dst = b1;
    int NS = 1;
    for (int s = 0; s < sc.n; ++s) {
        const int R = sc.r[s];
        switch (R) {
        case 2: gstage<2, S, COLS>(src, dst, NL, L, NS, tw, tid); break;
        case 3: gstage<3, S, COLS>(src, dst, NL, L, NS, tw, tid); break;
        case 4: gstage<4, S, COLS>(src, dst, NL, L, NS, tw, tid); break;
        case 5: gstage<5, S, COLS>(src, dst, NL, L, NS, tw, tid); break;
        case 8: gstage<8, S, COLS>(src, dst, NL, L, NS, tw, tid); break;
        default: gstage<16, S, COLS>(src, dst, NL, L, NS, tw, tid); break;
        }
        __syncthreads();
        NS *= R;
        c32 *t = src;
        src = dst;
        dst = t;
    }
    return src;
}

// ------------------------------------------------------------------ x pass
// LDS of an x tile (bytes, in this order): b0 [RB NC M], b1 [RB NC (M+1)],
// tw [M], twp [M+1], row offsets ib, ob [RB] each, FP64 block sum [NT/64].
size_t gx_lds_bytes(int M, int NC, int RB)
{
    const size_t nl = (size_t)RB * NC;
    return 8 * (nl * M + nl * (M + 1) + M + (M + 1)) + 16 * (size_t)RB + 8 * (kGThreads / 64);
}

// MODE 0: c2c with sign S (complex rows in and out); 1: r2c forward (real
// rows in, Nh = M + 1 bins out); 2: c2r backward (bins in, real rows out).
// XArgs offsets are in floats on real sides and in complex elements on
// complex sides, as for the compiled x kernels.
template <int MODE, int S>
__global__ __launch_bounds__(kGThreads) void k_gx(XArgs a, GSched sc, int M, int NC, int RB)
{
    extern __shared__ __align__(16) char gsm[];
    const int tid = threadIdx.x;
    const int NL = RB * NC;
    c32 *b0 = (c32 *)gsm;
    c32 *b1 = b0 + (size_t)NL * M;
    c32 *tw = b1 + (size_t)NL * (M + 1);
    c32 *twp = tw + M;
    int64_t *ib = (int64_t *)(twp + M + 1);
    int64_t *ob = ib + RB;
    double *red = (double *)(ob + RB);
    for (int i = tid; i < M; i += kGThreads) tw[i] = ((const c32 *)a.tw)[i];
    if (MODE != 0)
        for (int i = tid; i <= M; i += kGThreads) twp[i] = ((const c32 *)a.tw_post)[i];
    const int64_t r0 = (int64_t)blockIdx.x * RB;
    for (int i = tid; i < RB; i += kGThreads) {
        int64_t r = r0 + i;
        if (r >= a.nrows) r = a.nrows - 1;
        const int64_t z = r / a.n1, y = r - z * a.n1;
        ib[i] = a.in_off + z * a.in_plane + y * a.in_row;
        ob[i] = a.out_off + z * a.out_plane + y * a.out_row;
    }
    __syncthreads();
    const int nv = (int)(a.nrows - r0 < RB ? a.nrows - r0 : RB);
    double ss = 0.0;
    if (MODE == 0) {
        const c32 *in = (const c32 *)a.in;
        for (int e = tid; e < NL * M; e += kGThreads) {
            const int q = e / (M * NC), rem = e - q * (M * NC);
            const int p = rem / NC, c = rem - p * NC;
            b0[(q * NC + c) * M + p] = q < nv ? in[ib[q] + rem] : c32{0.f, 0.f};
        }
    } else if (MODE == 1) {
        // point p of component c is the pair (f[2p][c], f[2p + 1][c])
        const float *in = (const float *)a.in;
        for (int e = tid; e < NL * M; e += kGThreads) {
            const int q = e / (M * NC), rem = e - q * (M * NC);
            const int p = rem / NC, c = rem - p * NC;
            c32 v{0.f, 0.f};
            if (q < nv) {
                const float *fp = in + ib[q] + 2 * (int64_t)p * NC + c;
                v = c32{fp[0], fp[NC]};
                ss += (double)v.x * v.x + (double)v.y * v.y;
            }
            b0[(q * NC + c) * M + p] = v;
        }
    } else {
        // bins X[0..M] into b1, then Z[k] = (X[k] + conj X[M-k]) + i conj(W^k) (X[k] - conj X[M-k])
        // with the imaginary parts of X[0] and X[M] dropped
        const c32 *in = (const c32 *)a.in;
        const int H = M + 1;
        for (int e = tid; e < NL * H; e += kGThreads) {
            const int q = e / (H * NC), rem = e - q * (H * NC);
            const int k = rem / NC, c = rem - k * NC;
            b1[(q * NC + c) * H + k] = q < nv ? in[ib[q] + rem] : c32{0.f, 0.f};
        }
        __syncthreads();
        for (int e = tid; e < NL * M; e += kGThreads) {
            const int l = e / M, k = e - l * M;
            const c32 *line = b1 + (size_t)l * H;
            c32 xk = line[k], xm = line[M - k];
            if (k == 0) {
                xk.y = 0.f;
                xm.y = 0.f;
            }
            const c32 xmc = conjg(xm);
            const c32 s1 = add(xk, xmc);
            const c32 d = mul(conjg(twp[k]), sub(xk, xmc));
            b0[(size_t)l * M + k] = c32{s1.x - d.y, s1.y + d.x};
        }
    }
    if (MODE == 1 && a.sumsq) block_sum_f64<kGThreads>(ss, a.sumsq + blockIdx.x, red);
    __syncthreads();
    c32 *res = glines<MODE == 2 ? 1 : (MODE == 1 ? -1 : S), false>(b0, b1, NL, M, sc, tw, tid);
    if (MODE == 0) {
        c32 *out = (c32 *)a.out;
        for (int e = tid; e < NL * M; e += kGThreads) {
            const int q = e / (M * NC), rem = e - q * (M * NC);
            const int p = rem / NC, c = rem - p * NC;
            if (q < nv) out[ob[q] + rem] = res[(q * NC + c) * M + p];
        }
    } else if (MODE == 1) {
        // X[k] = fe + W^k fo, fe = (Z[k] + conj Z[M-k]) / 2, fo = (Z[k] - conj Z[M-k]) / (2i),
        // k = 0..M (Z indices mod M)
        c32 *out = (c32 *)a.out;
        const int H = M + 1;
        for (int e = tid; e < NL * H; e += kGThreads) {
            const int q = e / (H * NC), rem = e - q * (H * NC);
            const int k = rem / NC, c = rem - k * NC;
            if (q < nv) {
                const c32 *line = res + (size_t)(q * NC + c) * M;
                const c32 z = line[k == M ? 0 : k];
                const c32 zc = conjg(line[k == 0 || k == M ? 0 : M - k]);
                const c32 fe = scl(add(z, zc), 0.5f);
                const c32 dd = sub(z, zc);
                const c32 fo = c32{0.5f * dd.y, -0.5f * dd.x};
                out[ob[q] + rem] = add(fe, mul(twp[k], fo));
            }
        }
    } else {
        float *out = (float *)a.out;
        for (int e = tid; e < NL * M; e += kGThreads) {
            const int q = e / (M * NC), rem = e - q * (M * NC);
            const int p = rem / NC, c = rem - p * NC;
            if (q < nv) {
                const c32 v = res[(q * NC + c) * M + p];
                float *fp = out + ob[q] + 2 * (int64_t)p * NC + c;
                fp[0] = v.x;
                fp[NC] = v.y;
            }
        }
    }
}

hipError_t launch_gx(int mode, int sign, const XArgs &a, const GSched &sc, int m, int nc, int rb,
                     hipStream_t s)
{
    const unsigned grid = (unsigned)((a.nrows + rb - 1) / rb);
    const size_t shm = gx_lds_bytes(m, nc, rb);
    if (mode == 1)
        hipLaunchKernelGGL((k_gx<1, -1>), dim3(grid), dim3(kGThreads), shm, s, a, sc, m, nc, rb);
    else if (mode == 2)
        hipLaunchKernelGGL((k_gx<2, 1>), dim3(grid), dim3(kGThreads), shm, s, a, sc, m, nc, rb);
    else if (sign < 0)
        hipLaunchKernelGGL((k_gx<0, -1>), dim3(grid), dim3(kGThreads), shm, s, a, sc, m, nc, rb);
    else
        hipLaunchKernelGGL((k_gx<0, 1>), dim3(grid), dim3(kGThreads), shm, s, a, sc, m, nc, rb);
    return hipGetLastError();
}

// ------------------------------------------------------------ strided pass
// LDS of a strided tile: b0, b1 [B L], tw [L], then (binning) hist [nbins +
// 1] doubles and edges [nbins + 1].
size_t gs_lds_bytes(int L, int B, int nbins)
{
    return 16 * (size_t)B * L + 8 * (size_t)L + (nbins > 0 ? 16 * (size_t)(nbins + 1) : 0);
}

// Plain pass (EPI = false) or the fused last-axis pass (EPI = true, S = -1):
// forward transform, power-spectrum sums and / or the Poisson scale per mode
// in LDS, backward transform.  Tiles are taken grid-stride.
template <int S, bool EPI>
__global__ __launch_bounds__(kGThreads) void k_gs(SArgs a, GSched sc, int L, int B)
{
    extern __shared__ __align__(16) char gsm[];
    const int tid = threadIdx.x;
    c32 *b0 = (c32 *)gsm;
    c32 *b1 = b0 + (size_t)B * L;
    c32 *tw = b1 + (size_t)B * L;
    const int nb = a.mt.nbins;
    const bool pk = EPI && (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
    double *hist = (double *)(tw + L);
    BinEdge *edges = (BinEdge *)(hist + (nb + 1));
    for (int i = tid; i < L; i += kGThreads) tw[i] = ((const c32 *)a.tw)[i];
    if (pk) load_edges(a.mt, hist, edges, tid, kGThreads);
    __syncthreads();
    const bool store = (a.epi & EPI_STORE) != 0;
    const int64_t ntiles = (a.ncols + B - 1) / B;
    const c32 *in = (const c32 *)a.in;
    c32 *out = (c32 *)a.out;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        for (int e = tid; e < B * L; e += kGThreads) {
            const int col = e % B, p = e / B;
            const int64_t f = t * B + col;
            c32 v{0.f, 0.f};
            if (f < a.ncols) {
                const int64_t o = f / a.ncols_inner;
                v = in[o * a.outer + (f - o * a.ncols_inner) + (int64_t)p * a.stride];
            }
            b0[e] = v;
        }
        __syncthreads();
        c32 *res = glines<S, true>(b0, b1, B, L, sc, tw, tid);
        if constexpr (EPI) {
            const float cq = nb > 0 ? (float)((double)nb * nb / a.mt.qmax) : 0.f;
            for (int pass = 0; pass < 2; ++pass) {
                // pass 0: bins of the forward spectrum (EPI_PK) and the
                // Poisson scale; pass 1: bins after the scale (EPI_PK_AFTER)
                const bool bin_now = pass == 0 ? (a.epi & EPI_PK) != 0 : (a.epi & EPI_PK_AFTER) != 0;
                const bool scale_now = pass == 0 && (a.epi & EPI_POISSON) != 0;
                if (!bin_now && !scale_now) continue;
                for (int e = tid; e < B * L; e += kGThreads) {
                    const int col = e % B, kz = e / B;
                    const int64_t f = t * B + col;
                    if (f >= a.ncols) continue;
                    const int kx = (int)(f % a.mt.nxk), ky = (int)(f / a.mt.nxk);
                    const bool zero = kx == 0 && ky == 0 && kz == 0;
                    c32 v = res[e];
                    if (bin_now) {
                        const uint32_t m = (uint32_t)(2 * kz < L ? kz : L - kz);
                        const uint32_t q =
                            (uint32_t)(a.mt.q[0][kx] + a.mt.q[1][ky]) + m * m * a.mt.qz_unit;
                        const int b = zero ? nb : bin_edge(q, nb, cq, edges);
                        const double w =
                            (a.mt.half && !(kx == 0 || 2 * kx == a.mt.n0)) ? 2.0 : 1.0;
                        atomicAdd(&hist[b], w * ((double)v.x * v.x + (double)v.y * v.y));
                    }
                    if (scale_now) {
                        const double k2 = a.mt.k2[0][kx] + a.mt.k2[1][ky] + a.mt.k2[2][kz];
                        const double sc2 = zero ? 0.0 : -a.mt.scale_n / k2;
                        v = c32{(float)((double)v.x * sc2), (float)((double)v.y * sc2)};
                        res[e] = v;
                    }
                }
                __syncthreads();
            }
            if (a.epi & EPI_POISSON) res = glines<1, true>(res, res == b0 ? b1 : b0, B, L, sc, tw, tid);
        }
        if (store) {
            for (int e = tid; e < B * L; e += kGThreads) {
                const int col = e % B, p = e / B;
                const int64_t f = t * B + col;
                if (f < a.ncols) {
                    const int64_t o = f / a.ncols_inner;
                    out[o * a.outer + (f - o * a.ncols_inner) + (int64_t)p * a.stride] = res[e];
                }
            }
        }
        __syncthreads();
    }
    if (pk)
        for (int i = tid; i <= nb; i += kGThreads) a.partial[(int64_t)blockIdx.x * (nb + 1) + i] = hist[i];
}

hipError_t launch_gs(int sign, const SArgs &a, const GSched &sc, int len, int b, int grid_cap,
                     hipStream_t s, int *grid_used)
{
    const bool pk = (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
    const bool epi = pk || (a.epi & EPI_POISSON) != 0;
    const int64_t ntiles = (a.ncols + b - 1) / b;
    const int grid = (int)(ntiles < grid_cap ? ntiles : grid_cap);
    if (grid_used) *grid_used = grid;
    const size_t shm = gs_lds_bytes(len, b, pk ? a.mt.nbins : 0);
    if (epi) {
        if (sign > 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_gs<-1, true>), dim3(grid), dim3(kGThreads), shm, s, a, sc, len, b);
    } else if (sign < 0) {
        hipLaunchKernelGGL((k_gs<-1, false>), dim3(grid), dim3(kGThreads), shm, s, a, sc, len, b);
    } else {
        hipLaunchKernelGGL((k_gs<1, false>), dim3(grid), dim3(kGThreads), shm, s, a, sc, len, b);
    }
    return hipGetLastError();
}

}  // namespace lf2
