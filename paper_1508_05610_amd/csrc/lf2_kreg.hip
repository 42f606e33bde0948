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
static void launch_r(int sign, int g, const SArgs &a, hipStream_t s)
{
    if (sign < 0)
        hipLaunchKernelGGL((k_strided_r<L, -1, NTM>), dim3(g), dim3(kRThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_strided_r<L, 1, NTM>), dim3(g), dim3(kRThreads), 0, s, a);
}

template <int L>
static hipError_t launch_len(int sign, const SArgs &a, int grid_cap, hipStream_t s, int *grid_used,
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

// ---------------------------------------------------------------- fused pass
// The fused last-axis Poisson pass (forward z transform, optional P(k) of
// the modes, the FP64 Poisson scale, optional P(k) after it, backward z
// transform) with the tile in registers: B columns, 512 threads, P points a
// thread, over lines of L = P Q points (32 = 4 x 8 over 64 columns,
// 64 = 8 x 8 over 64, 128 = 8 x 16 over 32, 256 = 16 x 16 over 32,
// 512 = 16 x 32 over 16, 1024 = 32 x 32 over 16, 2048 = 32 x 64 over 8).
// The line splits as n = j + Q r (r in [0, P), j in [0, Q)),
// k = k1 + P k2 (k1 in [0, P), k2 in [0, Q)).  Thread (c, j) loads points
// j + Q r, takes the P-point DFT over r and multiplies by W_L^{j k1};
// through LDS, thread (c, k1) receives the Q values of j and takes the
// Q-point DFT over them -- where Q = 2P (32, 128, 512, 2048) as a lane pair
// (c, k1, h = 0, 1) taking the P-point DFTs over the even (h = 0) and odd
// (h = 1) j and one radix-2 step across the pair (DPP swap), so that lane h
// holds the modes kz = k1 + P (k2' + P h) (k2' in [0, P)).  The scale is
// applied there; the backward transform is the conjugate transpose of these
// steps in reverse order (radix-2 step, DFTs over k2', the exchange back,
// conjugate twiddles, DFTs over k1), which is the unnormalised inverse DFT.
// P(k): each mode's power |F|^2 (FP32) goes to an LDS table in natural
// order, and the binning walk over it (the walk of the LDS-staged fused
// tile: thread (c, j) takes |n_z| in [j EH, j EH + EH) and both modes of
// each, q growing by integer steps, FP64 sums into the wave's histogram)
// runs at the start of the next tile, while that tile's loads are in
// flight; the last tile's walk follows the loop.  The exchanges go through
// LDS in halves (real parts, then imaginary parts): below 1024 points the
// exchange and the power table (at most 32 KB each) leave room for two
// blocks per CU.  (Adding the two powers of each |n_z| into one slot with
// LDS float atomics, to halve the walk's reads, took the 512-point pass
// from 274 to 545 us.)
constexpr int kFThreads = 512;

template <int L>
struct FusedTile {
    static constexpr int P = L >= 1024 ? 32 : L >= 256 ? 16 : L >= 64 ? 8 : 4;  // points a thread
    static constexpr int Q = L / P;                // the outer DFT's length
    static constexpr int H = Q / P;                // lanes per (column, k1)
    static constexpr int B = kFThreads / Q;        // columns
    static constexpr int MH = L / 2;               // largest |n_z|
    static constexpr int RPT = kFThreads / B;      // walk rows (= Q)
    static constexpr int EH = (MH + 1 + RPT - 1) / RPT;  // |n_z| a thread walks
    static constexpr int LDS = (2 * L * B) * 4 + L * 8;  // exchange + powers + twiddles
    static_assert(P * Q == L && (H == 1 || H == 2) && B * P * H == kFThreads, "tile shape");
};

// The binning walk of column col over |n_z| in [rg EH, rg EH + EH), from
// the power table pw[kz * B + col] (both modes kz and L - kz of each |n_z|).
template <int L>
__device__ __forceinline__ void fused_walk(const SArgs &a, const float *pw, int col, int rg, int kx,
                                           bool corner, uint32_t qxy, bool valid, double *hist,
                                           const BinEdge *edges)
{
    using T = FusedTile<L>;
    const int nb = a.mt.nbins;
    const float cq = (float)((double)nb * nb / a.mt.qmax);
    const double wgt = (a.mt.half && !(kx == 0 || 2 * kx == a.mt.n0)) ? 2.0 : 1.0;
    const uint32_t qu = a.mt.qz_unit;
    const bool walk1 = a.mt.walk1 != 0;
    const int m0 = rg * T::EH;
    const int n = T::MH + 1 - m0 < T::EH ? T::MH + 1 - m0 : T::EH;  // may be <= 0
    if (!valid || n <= 0) return;
    uint32_t q = qxy + sq24(m0) * qu;
    uint32_t dq = (uint32_t)(2 * m0 + 1) * qu;
    const uint32_t ddq = 2u * qu;
    // slot nbins: the zero mode (kept for the Parseval sum)
    int b;
    uint32_t hi;
    if (corner && m0 == 0) {
        b = nb;
        hi = 1u;
    } else {
        b = bin_edge(q, nb, cq, edges);
        hi = edges[b].hi;
    }
    double acc = 0.0;
#pragma unroll 3
    for (int e = 0; e < T::EH; ++e) {
        if (e >= n) break;
        const int m = m0 + e;
        const bool two = m != 0 && 2 * m != L;  // the partner mode L - m
        const float pu = pw[m * T::B + col];
        const float pv = two ? pw[(L - m) * T::B + col] : 0.f;
        if (q >= hi) {
            atomicAdd(&hist[b], wgt * acc);
            acc = 0.0;
            if (walk1 && b < nb)
                ++b;
            else
                b = bin_edge(q, nb, cq, edges);
            hi = edges[b].hi;
        }
        acc += (double)pu + (double)pv;
        q += dq;
        dq += ddq;
    }
    atomicAdd(&hist[b], wgt * acc);
}

// The powers |F|^2 (FP32) of the modes kz = k1 + P (k2' + P h) a lane
// holds, into the table in natural order.
template <int L>
__device__ __forceinline__ void put_powers(float *pw, const c32 (&v)[FusedTile<L>::P], int k1, int h,
                                           int c2)
{
    using T = FusedTile<L>;
#pragma unroll
    for (int k2 = 0; k2 < T::P; ++k2)
        pw[(k1 + T::P * (k2 + T::P * h)) * T::B + c2] = fmaf(v[k2].x, v[k2].x, v[k2].y * v[k2].y);
}

// The walk's column data for column f of the (kx, ky) plane.
__device__ __forceinline__ void fused_col(const SArgs &a, int64_t f, bool valid, int &kx, bool &corner,
                                          uint32_t &qxy)
{
    kx = valid ? (int)f % a.mt.nxk : 0;
    const int ky = valid ? (int)f / a.mt.nxk : 0;
    corner = kx == 0 && ky == 0;
    const int mx = 2 * kx <= a.mt.n0 ? kx : a.mt.n0 - kx;
    const int my = 2 * ky <= a.mt.n1 ? ky : a.mt.n1 - ky;
    qxy = a.mt.qx_unit * sq24(mx) + a.mt.qy_unit * sq24(my);
}

template <int L, int K2>
__global__ __launch_bounds__(kFThreads) __attribute__((amdgpu_waves_per_eu(L >= 1024 ? 2 : 4)))
void k_fused_r(SArgs a)
{
    using T = FusedTile<L>;
    constexpr int P = T::P, Q = T::Q, H = T::H, B = T::B;
    constexpr bool CONT = K2 == 1;
    constexpr int ROWX = Q * B;               // exchange words per k1
    __shared__ float ex[P * ROWX];            // one half of the exchange
    __shared__ float pw[L * B];               // the powers, natural order
    __shared__ c32 tw[L];
    extern __shared__ double dyn[];           // hist[hcopies][nbins + 1], edges[nbins + 1]
    const int tid = threadIdx.x;
    load_table(tw, a.tw, L, tid, kFThreads);
    const bool pk = (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
    const bool pk_after = (a.epi & EPI_PK_AFTER) != 0;
    const int nb = a.mt.nbins;
    double *hist = dyn;
    BinEdge *edges = (BinEdge *)(dyn + a.hcopies * (nb + 1));
    if (pk) hist_init(a.mt, a.hcopies, hist, edges, tid, kFThreads);
    __syncthreads();
    double *wh = hist + (a.hcopies > 1 ? (tid >> 6) * (nb + 1) : 0);  // this wave's histogram
    const bool store = (a.epi & EPI_STORE) != 0;
    const int64_t ntiles = (a.ncols + B - 1) / B;
    const int64_t K = a.xcd_chunk;  // the XCD-aware walk of k_strided
    const int64_t span = (ntiles + 8 * K - 1) / (8 * K) * (8 * K);
    int64_t tprev = -1;  // the tile whose powers wait in pw
    for (int64_t vb = blockIdx.x; vb < span; vb += gridDim.x) {
        const int64_t lb = vb / 8;
        const int64_t t = ((lb / K) * 8 + (vb % 8)) * K + lb % K;
        if (t >= ntiles) continue;  // uniform over the block
        const int ot = opaque_tid<true>(tid);
        // thread (c, j): loads, stores and the binning walk (as thread (col, rg))
        const int c = ot % B, j = ot / B;
        const int64_t f = t * B + c;
        const bool valid = f < a.ncols;
        // a column past the end reads column 0 (in bounds) and is not stored
        const int64_t base = valid ? col_base(a, f) : 0;
        c32 v[P];
        gload_pts<P, true>(v, (const c32 *)a.in + base + (int64_t)j * a.stride, (int64_t)Q * a.stride,
                           true);
        asm volatile("" ::: "memory");  // the loads go out before the walk
        if (pk && tprev >= 0) {
            const int64_t fp = tprev * B + c;
            int kx;
            bool corner;
            uint32_t qxy;
            fused_col(a, fp, fp < a.ncols, kx, corner, qxy);
            fused_walk<L>(a, pw, c, j, kx, corner, qxy, fp < a.ncols, wh, edges);
        }
        Dft<P, -1>::run(v);  // v[k1]
#pragma unroll
        for (int k1 = 1; k1 < P; ++k1) v[k1] = mul(v[k1], tw[j * k1]);  // W_L^{j k1}
        // thread (c2, k1, h): j = H j' + h
        const int h = ot % H, c2 = (ot / H) % B, k1 = ot / (H * B);
        float re[P];
#pragma unroll
        for (int q = 0; q < P; ++q) ex[q * ROWX + j * B + c] = v[q].x;
        __syncthreads();  // also: the walk above is done with pw
#pragma unroll
        for (int jj = 0; jj < P; ++jj) re[jj] = ex[k1 * ROWX + (H * jj + h) * B + c2];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) ex[q * ROWX + j * B + c] = v[q].y;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < P; ++jj) v[jj] = c32{re[jj], ex[k1 * ROWX + (H * jj + h) * B + c2]};
        Dft<P, -1>::run(v);  // v[k2'] over the j of this h
        const float sg = h ? -1.f : 1.f;
        if constexpr (H == 2) {
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                const c32 own = mul(v[k2], tw[P * k2 * h]);  // W_Q^{k2' h}
                const c32 p = c32{lane_swap(own.x), lane_swap(own.y)};
                v[k2] = c32{fmaf(sg, own.x, p.x), fmaf(sg, own.y, p.y)};  // mode k1 + P (k2' + P h)
            }
        }
        if (pk && !pk_after) put_powers<L>(pw, v, k1, h, c2);
        {
            // the Poisson scale -1/(N k^2), FP64, rounded once with the product
            const int64_t f2 = t * B + c2;
            const bool valid2 = f2 < a.ncols;
            const int kx2 = valid2 ? (int)f2 % a.mt.nxk : 0, ky2 = valid2 ? (int)f2 / a.mt.nxk : 0;
            const int mx2 = 2 * kx2 <= a.mt.n0 ? kx2 : a.mt.n0 - kx2;
            const int my2 = 2 * ky2 <= a.mt.n1 ? ky2 : a.mt.n1 - ky2;
            const bool corner2 = kx2 == 0 && ky2 == 0;
            double k2xy = 1.0;
            if (valid2)
                k2xy = CONT ? fma(a.mt.k2x_unit, (double)sq24(mx2), a.mt.k2y_unit * (double)sq24(my2))
                            : a.mt.k2[0][kx2] + a.mt.k2[1][ky2];
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                const int kz = k1 + P * (k2 + P * h);
                const int m = 2 * kz < L ? kz : L - kz;
                const double k2z = CONT ? a.mt.k2z_unit * (double)sq24(m) : a.mt.k2[2][kz];
                const double sc = (corner2 && kz == 0) ? 0.0 : -a.mt.scale_n * rcp_f64(k2xy + k2z);
                v[k2] = c32{(float)((double)v[k2].x * sc), (float)((double)v[k2].y * sc)};
            }
        }
        if (pk_after) put_powers<L>(pw, v, k1, h, c2);
        if constexpr (H == 2) {
            // backward: the radix-2 step across the pair (lane 0 keeps Z0 + Z1,
            // lane 1 gets conj(W_Q^{k2'}) (Z0 - Z1))
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                const c32 p = c32{lane_swap(v[k2].x), lane_swap(v[k2].y)};
                const c32 d = c32{fmaf(sg, v[k2].x, p.x), fmaf(sg, v[k2].y, p.y)};
                v[k2] = mul(d, conjg(tw[P * k2 * h]));
            }
        }
        Dft<P, +1>::run(v);  // v[j'] for j = H j' + h
        __syncthreads();  // the forward exchange's reads are done
#pragma unroll
        for (int jj = 0; jj < P; ++jj) ex[k1 * ROWX + (H * jj + h) * B + c2] = v[jj].x;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) re[q] = ex[q * ROWX + j * B + c];
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < P; ++jj) ex[k1 * ROWX + (H * jj + h) * B + c2] = v[jj].y;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) v[q] = c32{re[q], ex[q * ROWX + j * B + c]};
        __syncthreads();  // the next tile rewrites ex; pw is complete for its walk
#pragma unroll
        for (int q = 1; q < P; ++q) v[q] = mul(v[q], conjg(tw[j * q]));
        Dft<P, +1>::run(v);  // v[r]: point j + Q r
        if (valid && store)
            gstore_pts<P, true>(v, (c32 *)a.out + base + (int64_t)j * a.stride, (int64_t)Q * a.stride);
        tprev = t;
    }
    if (pk) {
        if (tprev >= 0) {
            const int c = tid % B, j = tid / B;
            const int64_t fp = tprev * B + c;
            int kx;
            bool corner;
            uint32_t qxy;
            fused_col(a, fp, fp < a.ncols, kx, corner, qxy);
            fused_walk<L>(a, pw, c, j, kx, corner, qxy, fp < a.ncols, wh, edges);
        }
        __syncthreads();
        hist_flush(nb, a.hcopies, hist, a.partial + (int64_t)blockIdx.x * (nb + 1), tid, kFThreads);
    }
}

template <int L>
static hipError_t launch_fused_len(SArgs a, int grid_cap, hipStream_t s, int *grid_used)
{
    using T = FusedTile<L>;
    // one histogram per wave where they fit beside the tile within the
    // block's share of LDS (two blocks per CU below 1024 points, one from
    // there on), else one for the block (which may then take a CU alone)
    const size_t budget = L >= 1024 ? 160 * 1024 : 80 * 1024;
    const bool pk = (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
    const size_t row = (size_t)(a.mt.nbins + 1) * 8;
    constexpr int kWaves = kFThreads / 64;
    a.hcopies = pk && T::LDS + row * (kWaves + 1) <= budget ? kWaves : 1;
    const size_t shm = pk ? row * (a.hcopies + 1) : 0;
    if (T::LDS + shm > 160 * 1024) return hipErrorInvalidValue;
    const int64_t ntiles = (a.ncols + T::B - 1) / T::B;
    const int chunk = a.xcd_chunk;
    const int64_t span = (ntiles + 8 * chunk - 1) / (8 * chunk) * (8 * chunk);
    const int g = (int)(span < grid_cap ? span : grid_cap);
    if (grid_used) *grid_used = g;
    if (a.mt.k2z_unit > 0.0)
        hipLaunchKernelGGL((k_fused_r<L, 1>), dim3(g), dim3(kFThreads), shm, s, a);
    else
        hipLaunchKernelGGL((k_fused_r<L, 2>), dim3(g), dim3(kFThreads), shm, s, a);
    return hipGetLastError();
}

bool s_reg_supported(int len) { return len == 1024 || len == 2048; }

bool fused_reg_supported(int len)
{
    return len == 32 || len == 64 || len == 128 || len == 256 || len == 512 || len == 1024 || len == 2048;
}

template <int L>
static bool fused_fits(int nbins)
{
    const size_t shm = nbins > 0 ? (size_t)(nbins + 1) * 8 * 2 : 0;  // one histogram and the edges
    return FusedTile<L>::LDS + shm <= 160 * 1024;
}

bool fused_reg_fits(int len, int nbins)
{
    switch (len) {
    case 32: return fused_fits<32>(nbins);
    case 64: return fused_fits<64>(nbins);
    case 128: return fused_fits<128>(nbins);
    case 256: return fused_fits<256>(nbins);
    case 512: return fused_fits<512>(nbins);
    case 1024: return fused_fits<1024>(nbins);
    case 2048: return fused_fits<2048>(nbins);
    default: return false;
    }
}

hipError_t launch_fused_reg(int len, const SArgs &a, size_t, int grid_cap, hipStream_t s,
                            int *grid_used)
{
    if ((a.epi & EPI_POISSON) == 0) return hipErrorInvalidValue;
    if (len == 32) return launch_fused_len<32>(a, grid_cap, s, grid_used);
    if (len == 64) return launch_fused_len<64>(a, grid_cap, s, grid_used);
    if (len == 128) return launch_fused_len<128>(a, grid_cap, s, grid_used);
    if (len == 256) return launch_fused_len<256>(a, grid_cap, s, grid_used);
    if (len == 512) return launch_fused_len<512>(a, grid_cap, s, grid_used);
    if (len == 1024) return launch_fused_len<1024>(a, grid_cap, s, grid_used);
    if (len == 2048) return launch_fused_len<2048>(a, grid_cap, s, grid_used);
    return hipErrorInvalidValue;
}

hipError_t launch_strided_reg(int len, int sign, const SArgs &a, int grid_cap, hipStream_t s,
                              int *grid_used, int chunk, bool ntm)
{
    if (len == 1024) return launch_len<1024>(sign, a, grid_cap, s, grid_used, chunk, ntm);
    if (len == 2048) return launch_len<2048>(sign, a, grid_cap, s, grid_used, chunk, ntm);
    return hipErrorInvalidValue;
}

}  // namespace lf2
