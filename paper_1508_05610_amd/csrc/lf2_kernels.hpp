// lf2_kernels.hpp -- pass kernels of the 3-D FFT (gfx950).
//
// Every pass is written as a per-tile device function that works in an LDS
// area handed to it by the caller.  The standalone kernels below run one
// pass over one field; the batch kernels (lf2_kbatch.hip) run the same tile
// functions over the tiles of many fields, one launch per (pass, length).
//
// x pass  : lines along dimension 0 are contiguous in memory.  A tile is RB
//           rows (all components of each row).  r2c packs N0 reals as N0/2
//           complex values, transforms and splits the result into Nh bins;
//           c2r does the reverse.  Dense tiles are read as one run of
//           16-byte loads into LDS; other one-component rows with even
//           element offsets go as complex values straight into the first
//           Stockham stage, and interleaved components of real fields (or
//           odd halo offsets) as float pairs.
// strided : lines along dimension 1 or 2 have a large stride; consecutive
//           columns are adjacent in memory.  A tile is B adjacent columns x
//           L points: loaded row by row (B * 8 bytes contiguous per row)
//           straight into the first stage, transformed in LDS with lanes
//           walking adjacent columns, stored from the last stage.  This
//           replaces the paper's rod transposes (the data never leaves its
//           place; the tile is the transpose).  Epilogues on the last axis:
//           power-spectrum binning and the Poisson scale followed by the
//           backward transform.
#pragma once
#include "lf2_device.hpp"
#include "lf2_internal.hpp"

namespace lf2 {

constexpr int kXThreads = 256;
constexpr int kSThreads = 512;

// Rows per x-pass tile: about 4096 * (NT / 256) complex values of LDS, at
// most 256 rows.
__host__ __device__ constexpr int x_rb(int L, int NC, int NT = kXThreads)
{
    return ((4096 / L) / NC * (NT / 256)) < 1
               ? 1
               : (((4096 / L) / NC * (NT / 256)) > 256 ? 256 : ((4096 / L) / NC * (NT / 256)));
}
// Columns per strided tile: 64 KiB of LDS at most, >= 128-byte row segments
// up to L = 512.
__host__ __device__ constexpr int s_b(int L)
{
    return L <= 128 ? 64 : L <= 256 ? 32 : L <= 512 ? 16 : L <= 1024 ? 8 : 4;
}

__host__ __device__ constexpr size_t al16(size_t b) { return (b + 15) & ~(size_t)15; }

// Row base offsets of the RB rows of tile `blk`, in LDS.
template <int RB, int NT>
__device__ __forceinline__ void row_bases(int64_t *ib, int64_t *ob, const XArgs &a, int64_t r0,
                                          int tid)
{
    for (int i = tid; i < RB; i += NT) {
        int64_t r = r0 + i;
        if (r >= a.nrows) r = a.nrows - 1;
        int64_t z = r / a.n1, y = r - z * a.n1;
        ib[i] = a.in_off + z * a.in_plane + y * a.in_row;
        ob[i] = a.out_off + z * a.out_plane + y * a.out_row;
    }
}

template <int RB>
__device__ __forceinline__ int rows_valid(const XArgs &a, int64_t r0)
{
    const int64_t left = a.nrows - r0;
    return left < RB ? (int)left : RB;
}

// FP64 block sum of v into *dst (thread 0 writes).
template <int NT>
__device__ __forceinline__ void block_sum_f64(double v, double *dst, double *scratch)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < NT / 64; ++w) t += scratch[w];
        *dst = t;
    }
}

// Twiddle tables into LDS (callers wait at a barrier before use).
__device__ __forceinline__ void load_table(c32 *dst, const void *src, int n, int tid, int nt)
{
    const c32 *g = (const c32 *)src;
    for (int i = tid; i < n; i += nt) dst[i] = g[i];
}

// =================================================================== x tiles

// ---- general r2c (interleaved components, any float offsets): the first
// stage loads component c's packed point n = (f[2n][c], f[2n + 1][c]) as two
// floats straight from the row; one padded LDS line per (row, component)
template <int M, int NC, int NT>
struct XR2CGen {
    static constexpr int RB = x_rb(M, NC, NT), NL = RB * NC, LP = row_pitch(M),
                         NH = M + 1;
    static constexpr size_t O_BUF = 0, O_TW = al16(O_BUF + sizeof(c32) * NL * LP),
                            O_TWP = al16(O_TW + sizeof(c32) * M),
                            O_IB = al16(O_TWP + sizeof(c32) * NH), O_OB = O_IB + 8 * RB,
                            O_RED = O_OB + 8 * RB, BYTES = al16(O_RED + 8 * (NT / 64));
    static __device__ void tables(const XArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, M, tid, NT);
        load_table((c32 *)(sm + O_TWP), a.tw_post, NH, tid, NT);
    }
    // sumsq: where to put this tile's FP64 sum of squares (nullptr: skip)
    static __device__ void tile(const XArgs &a, int64_t blk, char *sm, int tid, double *sumsq)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW), *twp = (const c32 *)(sm + O_TWP);
        int64_t *ib = (int64_t *)(sm + O_IB), *ob = (int64_t *)(sm + O_OB);
        const int64_t r0 = blk * RB;
        row_bases<RB, NT>(ib, ob, a, r0, tid);
        __syncthreads();
        const int nv = rows_valid<RB>(a, r0);
        // the first stage reads each component's packed pairs straight from
        // the real rows (two float loads per point; no alignment needed)
        double ss = 0.0;
        row_fft<M, -1, RB, NC, LP, NT, true, false, 0, 1, true, true>(
            buf, (const c32 *)a.in, nullptr, ib, nullptr, nv, tw, tid, sumsq ? &ss : nullptr);
        if (sumsq) block_sum_f64<NT>(ss, sumsq, (double *)(sm + O_RED));
        // X[k] = fe + W^k fo and X[M-k] = conj(fe - W^k fo) per component;
        // work item (row, k, component), component fastest
        c32 *out = (c32 *)a.out;
        constexpr int HALF = M / 2 + 1;
        constexpr int NI = RB * HALF * NC;
#pragma unroll
        for (int i = 0; i < (NI + NT - 1) / NT; ++i) {
            const int idx = tid + i * NT;
            if (idx < NI) {
                const int c = idx % NC, t = idx / NC;
                const int k = t % HALF, l = t / HALF;
                if (l < nv) {
                    const c32 *line = buf + (l * NC + c) * LP;
                    const c32 z = line[lpad(k)];
                    const c32 zc = conjg(line[lpad(k == 0 ? 0 : M - k)]);
                    const c32 fe = scl(add(z, zc), 0.5f);
                    const c32 d = sub(z, zc);
                    const c32 fo = c32{0.5f * d.y, -0.5f * d.x};  // (z - zc) / (2i)
                    const c32 wf = mul(twp[k], fo);
                    c32 *orow = out + ob[l] + c;
                    gstore<true>(orow + k * NC, add(fe, wf));
                    if (2 * k != M) gstore<true>(orow + (M - k) * NC, conjg(sub(fe, wf)));
                }
            }
        }
        __syncthreads();
    }
};

// ---- general c2r (interleaved components, any float offsets): bins through
// LDS, and the last stage stores each packed point as two floats
template <int M, int NC, int NT>
struct XC2RGen {
    static constexpr int RB = x_rb(M, NC, NT), NL = RB * NC, LP = row_pitch(M + 1), NH = M + 1;
    static constexpr size_t O_BUF = 0, O_TW = al16(O_BUF + sizeof(c32) * NL * LP),
                            O_TWP = al16(O_TW + sizeof(c32) * M),
                            O_IB = al16(O_TWP + sizeof(c32) * NH), O_OB = O_IB + 8 * RB,
                            BYTES = al16(O_OB + 8 * RB);
    static __device__ void tables(const XArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, M, tid, NT);
        load_table((c32 *)(sm + O_TWP), a.tw_post, NH, tid, NT);
    }
    // Whole output rows leave as 16-byte nontemporal stores when every row
    // starts 16-byte aligned and holds a multiple of 4 floats.
    static __device__ bool vec_out(const XArgs &a)
    {
        return (2 * M * NC) % 4 == 0 && ((uintptr_t)a.out & 15) == 0 && a.out_off % 4 == 0 &&
               a.out_row % 4 == 0 && a.out_plane % 4 == 0;
    }
    // Real rows from the LDS lines: float x NC + c of row l is part x & 1 of
    // point x >> 1 of line l NC + c.
    static __device__ void store_rows(const XArgs &a, const c32 *buf, const int64_t *ob, int nv,
                                      int tid)
    {
        typedef float nf4 __attribute__((ext_vector_type(4)));
        constexpr int W4 = 2 * M * NC / 4;  // 16-byte words per row
        const float *fb = (const float *)buf;
        float *out = (float *)a.out;
        for (int e = tid; e < nv * W4; e += NT) {
            const int l = e / W4, f0 = 4 * (e - l * W4);
            float w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int f = f0 + u, x = f / NC, c = f - x * NC;
                w[u] = fb[2 * ((l * NC + c) * LP + lpad(x >> 1)) + (x & 1)];
            }
            nf4 v;
            v.x = w[0];
            v.y = w[1];
            v.z = w[2];
            v.w = w[3];
            __builtin_nontemporal_store(v, (nf4 *)(out + ob[l]) + (e - l * W4));
        }
    }
    static __device__ void tile(const XArgs &a, int64_t blk, char *sm, int tid)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW), *twp = (const c32 *)(sm + O_TWP);
        int64_t *ib = (int64_t *)(sm + O_IB), *ob = (int64_t *)(sm + O_OB);
        const int64_t r0 = blk * RB;
        row_bases<RB, NT>(ib, ob, a, r0, tid);
        __syncthreads();
        const c32 *in = (const c32 *)a.in;
        constexpr int NI = RB * NH * NC;
        const int nv = rows_valid<RB>(a, r0);
        // value e of the tile's rows (row-major, component fastest) -> LDS
        auto put = [&](int e, c32 v) {
            const int row = e / (NH * NC), rem = e - row * (NH * NC);
            const int k = rem / NC, c = rem - k * NC;
            buf[(row * NC + c) * LP + lpad(k)] = v;
        };
        const c32 *src = in + ib[0];
        if (a.in_row == NH * NC && a.in_plane == (int64_t)a.n1 * NH * NC &&
            ((uintptr_t)src & 7) == 0) {
            // dense half spectrum: the tile's rows are one contiguous run,
            // read with 16-byte loads from the first 16-byte boundary on
            // (all of a thread's loads are issued before the first LDS write)
            typedef float nf4 __attribute__((ext_vector_type(4)));
            constexpr int NW = (NI / 2 + NT - 1) / NT;
            const int e0 = ((uintptr_t)src & 15) ? 1 : 0;
            const nf4 *s4 = (const nf4 *)(src + e0);
            const int cnt = nv * NH * NC;
            const int np = (cnt - e0) / 2;
            nf4 w[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int e = tid + i * NT;
                if (e < np) w[i] = __builtin_nontemporal_load(s4 + e);
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int e = tid + i * NT;
                if (e < np) {
                    put(e0 + 2 * e, c32{w[i].x, w[i].y});
                    put(e0 + 2 * e + 1, c32{w[i].z, w[i].w});
                }
            }
            if (tid == 0 && e0 && cnt > 0) put(0, src[0]);
            if (tid == 0 && e0 + 2 * np < cnt) put(cnt - 1, src[cnt - 1]);
            for (int e = cnt + tid; e < NI; e += NT) put(e, c32{0.f, 0.f});
        } else {
#pragma unroll
            for (int i = 0; i < (NI + NT - 1) / NT; ++i) {
                const int idx = tid + i * NT;
                if (idx < NI) {
                    const int row = idx / (NH * NC);
                    put(idx, row < nv ? gload<true>(in + ib[row] + (idx - row * (NH * NC)))
                                      : c32{0.f, 0.f});
                }
            }
        }
        __syncthreads();
        // Z[k] = (X[k] + conj X[M-k]) + i W^{-k} (X[k] - conj X[M-k]), k < M,
        // with the imaginary parts of X[0] and X[M] dropped.
        auto zval = [&](const c32 *line, int k) {
            c32 xk = line[lpad(k)], xm = line[lpad(M - k)];
            if (k == 0) {
                xk.y = 0.f;
                xm.y = 0.f;
            }
            const c32 xmc = conjg(xm);
            const c32 sm_ = add(xk, xmc);
            const c32 d = mul(conjg(twp[k]), sub(xk, xmc));
            return c32{sm_.x - d.y, sm_.y + d.x};  // s + i d
        };
        if constexpr (nstages(M) >= 2) {
            // the first inverse stage forms its inputs Z[k] from the bins in
            // LDS as it reads them (butterfly b: component b % NC, then j,
            // then row, as in the row engine), then the remaining stages
            constexpr int R = radix_at(M, 0), Q = M / R;
            constexpr int NBF = NL * Q, NB = (NBF + NT - 1) / NT;
            c32 v[NB][R];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = tid + i * NT;
                if (NBF % NT == 0 || b < NBF) {
                    const int c = b % NC, t = b / NC;
                    const int j = t % Q, q = t / Q;
                    const c32 *line = buf + (q * NC + c) * LP;
#pragma unroll
                    for (int r = 0; r < R; ++r) v[i][r] = zval(line, j + r * Q);
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = tid + i * NT;
                if (NBF % NT == 0 || b < NBF) {
                    const int c = b % NC, t = b / NC;
                    const int j = t % Q, q = t / Q;
                    Dft<R, +1>::run(v[i]);
                    c32 *dst = buf + (q * NC + c) * LP;
#pragma unroll
                    for (int r = 0; r < R; ++r) dst[lpad(j * R + r)] = v[i][r];
                }
            }
            __syncthreads();
            if (vec_out(a)) {
                // remaining stages in LDS, then whole rows out as 16-byte stores
                row_fft<M, +1, RB, NC, LP, NT, false, false, 1, R>(buf, nullptr, nullptr, nullptr,
                                                                   nullptr, nv, tw, tid);
                store_rows(a, buf, ob, nv, tid);
            } else {
                // the last stage stores each component's pairs straight to the rows
                row_fft<M, +1, RB, NC, LP, NT, false, true, 1, R, true, true>(
                    buf, nullptr, (c32 *)a.out, nullptr, ob, nv, tw, tid);
            }
        } else {
            constexpr int NZ = NL * M;
            constexpr int NZT = (NZ + NT - 1) / NT;
            c32 zv[NZT];
#pragma unroll
            for (int i = 0; i < NZT; ++i) {
                const int idx = tid + i * NT;
                if (idx < NZ) zv[i] = zval(buf + (idx / M) * LP, idx % M);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NZT; ++i) {
                const int idx = tid + i * NT;
                if (idx < NZ) buf[(idx / M) * LP + lpad(idx % M)] = zv[i];
            }
            __syncthreads();
            row_fft<M, +1, RB, NC, LP, NT, false, true, 0, 1, true, true>(
                buf, nullptr, (c32 *)a.out, nullptr, ob, nv, tw, tid);
        }
        __syncthreads();
    }
};

// ---- one-component fast r2c.
// X[k] = fe + W^k fo and X[M-k] = conj(fe - W^k fo), with
// fe = (Z[k] + conj Z[M-k]) / 2, fo = (Z[k] - conj Z[M-k]) / (2i).
template <int M, int NT>
struct XR2CV {
    // LDS lines hold the M packed points, then the NH = M + 1 output bins
    static constexpr int RB = x_rb(M, 1, NT), LP = row_pitch(M + 1), NH = M + 1, HALF = M / 2 + 1;
    static constexpr size_t O_BUF = 0, O_TW = al16(O_BUF + sizeof(c32) * RB * LP),
                            O_TWP = al16(O_TW + sizeof(c32) * M),
                            O_IB = al16(O_TWP + sizeof(c32) * NH), O_OB = O_IB + 8 * RB,
                            O_RED = O_OB + 8 * RB, BYTES = al16(O_RED + 8 * (NT / 64));
    static __device__ void tables(const XArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, M, tid, NT);
        load_table((c32 *)(sm + O_TWP), a.tw_post, NH, tid, NT);
    }
    static __device__ void tile(const XArgs &a, int64_t blk, char *sm, int tid, double *sumsq)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW), *twp = (const c32 *)(sm + O_TWP);
        int64_t *ib = (int64_t *)(sm + O_IB), *ob = (int64_t *)(sm + O_OB);
        const int64_t r0 = blk * RB;
        row_bases<RB, NT>(ib, ob, a, r0, tid);
        __syncthreads();
        const int nv = rows_valid<RB>(a, r0);
        double ss = 0.0;
        const float *src = (const float *)a.in + ib[0];
        if (M % 2 == 0 && a.in_row == 2 * M && a.in_plane == (int64_t)a.n1 * 2 * M &&
            ((uintptr_t)src & 15) == 0) {
            // Dense rows: the tile is one contiguous run of nv N0 reals, read
            // with 16-byte loads (all of a thread's loads issued first) into
            // the padded LDS lines, then transformed there.
            typedef float nf4 __attribute__((ext_vector_type(4)));
            constexpr int NW = (RB * M / 2 + NT - 1) / NT;
            const nf4 *s4 = (const nf4 *)src;
            const int np = nv * M / 2;
            auto put = [&](int e, c32 v) {
                const int l = e / M, k = e - l * M;
                buf[l * LP + lpad(k)] = v;
            };
            nf4 w[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int e = tid + i * NT;
                if (e < np) w[i] = __builtin_nontemporal_load(s4 + e);
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const int e = tid + i * NT;
                if (e < np) {
                    put(2 * e, c32{w[i].x, w[i].y});
                    put(2 * e + 1, c32{w[i].z, w[i].w});
                    if (sumsq)
                        ss += ((double)w[i].x * w[i].x + (double)w[i].y * w[i].y) +
                              ((double)w[i].z * w[i].z + (double)w[i].w * w[i].w);
                }
            }
            for (int e = nv * M + tid; e < RB * M; e += NT) put(e, c32{0.f, 0.f});
            __syncthreads();
            row_fft<M, -1, RB, 1, LP, NT, false, false>(buf, nullptr, nullptr, nullptr, nullptr, nv,
                                                        tw, tid);
        } else {
            for (int i = tid; i < RB; i += NT) ib[i] >>= 1;  // float offset -> complex offset
            __syncthreads();
            row_fft<M, -1, RB, 1, LP, NT, true, false, 0, 1, true>(
                buf, (const c32 *)a.in, nullptr, ib, nullptr, nv, tw, tid, sumsq ? &ss : nullptr);
        }
        if (sumsq) block_sum_f64<NT>(ss, sumsq, (double *)(sm + O_RED));
        // bins of every line in place: the thread of pair (k, M - k) reads
        // and writes only those two slots (k = 0 writes X[M] to slot M)
        constexpr int NI = RB * HALF;
#pragma unroll
        for (int i = 0; i < (NI + NT - 1) / NT; ++i) {
            const int idx = tid + i * NT;
            if (idx < NI) {
                const int l = idx / HALF;
                const int k = idx - l * HALF;
                if (l < nv) {
                    c32 *line = buf + l * LP;
                    const c32 z = line[lpad(k)];
                    const c32 zc = conjg(line[lpad(k == 0 ? 0 : M - k)]);
                    const c32 fe = scl(add(z, zc), 0.5f);
                    const c32 d = sub(z, zc);
                    const c32 fo = c32{0.5f * d.y, -0.5f * d.x};
                    const c32 wf = mul(twp[k], fo);
                    line[lpad(k)] = add(fe, wf);
                    if (2 * k != M) line[lpad(M - k)] = conjg(sub(fe, wf));
                }
            }
        }
        __syncthreads();
        c32 *out = (c32 *)a.out;
        auto bin = [&](int e) {  // value e of the tile's output rows, row-major
            const int l = e / NH;
            return buf[l * LP + lpad(e - l * NH)];
        };
        if (a.out_row == NH && a.out_plane == (int64_t)a.n1 * NH) {
            // dense half spectrum: the tile's rows are one contiguous run,
            // written with 16-byte nontemporal stores from the first 16-byte
            // boundary on
            typedef float nf4 __attribute__((ext_vector_type(4)));
            c32 *dst = out + ob[0];
            const int cnt = nv * NH;
            const int e0 = ((uintptr_t)dst & 15) ? 1 : 0;
            const int np = (cnt - e0) / 2;
            nf4 *d4 = (nf4 *)(dst + e0);
            for (int e = tid; e < np; e += NT) {
                const c32 u = bin(e0 + 2 * e), w = bin(e0 + 2 * e + 1);
                nf4 v;
                v.x = u.x;
                v.y = u.y;
                v.z = w.x;
                v.w = w.y;
                __builtin_nontemporal_store(v, d4 + e);
            }
            if (tid == 0 && e0 && cnt > 0) gstore<true>(dst, bin(0));
            if (tid == 0 && e0 + 2 * np < cnt) gstore<true>(dst + (cnt - 1), bin(cnt - 1));
        } else {
            for (int e = tid; e < nv * NH; e += NT) {
                const int l = e / NH;
                gstore<true>(out + ob[l] + (e - l * NH), bin(e));
            }
        }
        __syncthreads();
    }
};

// ---- one-component fast c2r.
// Z[k] = (X[k] + conj X[M-k]) + i W^{-k} (X[k] - conj X[M-k]); every thread
// owns the pair (k, M-k), so the update is in place without a barrier.
template <int M, int NT>
struct XC2RV {
    static constexpr int RB = x_rb(M, 1, NT), LP = row_pitch(M + 1), NH = M + 1, HALF = M / 2 + 1;
    static constexpr size_t O_BUF = 0, O_TW = al16(O_BUF + sizeof(c32) * RB * LP),
                            O_TWP = al16(O_TW + sizeof(c32) * M),
                            O_IB = al16(O_TWP + sizeof(c32) * NH), O_OB = O_IB + 8 * RB,
                            BYTES = al16(O_OB + 8 * RB);
    static __device__ void tables(const XArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, M, tid, NT);
        load_table((c32 *)(sm + O_TWP), a.tw_post, NH, tid, NT);
    }
    static __device__ void tile(const XArgs &a, int64_t blk, char *sm, int tid)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW), *twp = (const c32 *)(sm + O_TWP);
        int64_t *ib = (int64_t *)(sm + O_IB), *ob = (int64_t *)(sm + O_OB);
        const int64_t r0 = blk * RB;
        row_bases<RB, NT>(ib, ob, a, r0, tid);
        __syncthreads();
        for (int i = tid; i < RB; i += NT) ob[i] >>= 1;
        const int nv = rows_valid<RB>(a, r0);
        const c32 *in = (const c32 *)a.in;
        if (a.in_row == NH && a.in_plane == (int64_t)a.n1 * NH) {
            // Dense half spectrum: the tile's rows are one contiguous run of
            // nv * NH values, read with 16-byte loads when the run is 16-byte
            // aligned and placed into the padded LDS rows.
            const c32 *src = in + ib[0];
            const int cnt = nv * NH;
            auto put = [&](int e, c32 v) {
                const int l = e / NH, k = e - l * NH;
                buf[l * LP + lpad(k)] = v;
            };
            if (((uintptr_t)src & 15) == 0) {
                // all of a thread's loads are issued before the first LDS write
                typedef float nf4 __attribute__((ext_vector_type(4)));
                constexpr int NW = (RB * NH / 2 + NT - 1) / NT;
                const nf4 *s4 = (const nf4 *)src;
                nf4 w[NW];
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    const int e = tid + i * NT;
                    if (e < cnt / 2) w[i] = __builtin_nontemporal_load(s4 + e);
                }
#pragma unroll
                for (int i = 0; i < NW; ++i) {
                    const int e = tid + i * NT;
                    if (e < cnt / 2) {
                        put(2 * e, c32{w[i].x, w[i].y});
                        put(2 * e + 1, c32{w[i].z, w[i].w});
                    }
                }
                if ((cnt & 1) && tid == 0) put(cnt - 1, src[cnt - 1]);
            } else {
                for (int e = tid; e < cnt; e += NT) put(e, src[e]);
            }
            for (int e = cnt + tid; e < RB * NH; e += NT) put(e, c32{0.f, 0.f});
        } else {
            // TPR threads per row, each walking one row: a single row offset
            // per thread, loads of a wave contiguous within each row.
            constexpr int TPR = NT / RB >= 1 ? NT / RB : 1;
            constexpr int NK = (NH + TPR - 1) / TPR;
            for (int l = tid / TPR; l < RB; l += NT / TPR) {
                const int64_t base = ib[l];
                const bool ok = l < nv;
                const int k0 = tid % TPR;
#pragma unroll
                for (int i = 0; i < NK; ++i) {
                    const int k = k0 + i * TPR;
                    if (k < NH) buf[l * LP + lpad(k)] = ok ? in[base + k] : c32{0.f, 0.f};
                }
            }
        }
        __syncthreads();
        if constexpr (nstages(M) >= 2) {
            // The first inverse stage forms its inputs Z[k] from the bins
            // X[k], X[M-k] in LDS as it reads them (every read before the
            // barrier, every write after it), then the remaining stages.
            constexpr int R = radix_at(M, 0), Q = M / R;
            constexpr int NBF = RB * Q, NB = (NBF + NT - 1) / NT;
            c32 v[NB][R];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = tid + i * NT;
                if (NBF % NT == 0 || b < NBF) {
                    const int j = b % Q, q = b / Q;
                    const c32 *line = buf + q * LP;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int k = j + r * Q;
                        c32 xk = line[lpad(k)], xm = line[lpad(M - k)];
                        if (k == 0) {
                            xk.y = 0.f;
                            xm.y = 0.f;
                        }
                        const c32 s1 = add(xk, conjg(xm));
                        const c32 d1 = mul(conjg(twp[k]), sub(xk, conjg(xm)));
                        v[i][r] = c32{s1.x - d1.y, s1.y + d1.x};
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const int b = tid + i * NT;
                if (NBF % NT == 0 || b < NBF) {
                    const int j = b % Q, q = b / Q;
                    Dft<R, +1>::run(v[i]);
                    c32 *dst = buf + q * LP;
#pragma unroll
                    for (int r = 0; r < R; ++r) dst[lpad(j * R + r)] = v[i][r];
                }
            }
            __syncthreads();
            row_fft<M, +1, RB, 1, LP, NT, false, true, 1, R, true>(buf, nullptr, (c32 *)a.out, nullptr,
                                                             ob, nv, tw, tid);
        } else {
            constexpr int NP = RB * HALF;
#pragma unroll
            for (int i = 0; i < (NP + NT - 1) / NT; ++i) {
                const int idx = tid + i * NT;
                if (idx < NP) {
                    const int l = idx / HALF;
                    const int k = idx - l * HALF;
                    c32 *line = buf + l * LP;
                    c32 xk = line[lpad(k)], xm = line[lpad(M - k)];
                    if (k == 0) {
                        xk.y = 0.f;
                        xm.y = 0.f;
                    }
                    const c32 s1 = add(xk, conjg(xm));
                    const c32 d1 = mul(conjg(twp[k]), sub(xk, conjg(xm)));
                    const c32 zk = c32{s1.x - d1.y, s1.y + d1.x};
                    if (k != 0 && 2 * k != M) {
                        const c32 s2 = add(xm, conjg(xk));
                        const c32 d2 = mul(conjg(twp[M - k]), sub(xm, conjg(xk)));
                        line[lpad(M - k)] = c32{s2.x - d2.y, s2.y + d2.x};
                    }
                    line[lpad(k)] = zk;
                }
            }
            __syncthreads();
            row_fft<M, +1, RB, 1, LP, NT, false, true>(buf, nullptr, (c32 *)a.out, nullptr, ob, nv,
                                                       tw, tid);
        }
        __syncthreads();
    }
};

// ---- c2c with NC interleaved components, register-direct both ends
template <int L, int NC, int S, int NT>
struct XC2CV {
    static constexpr int RB = x_rb(L, NC, NT), LP = row_pitch(L);
    static constexpr size_t O_BUF = 0, O_TW = al16(O_BUF + sizeof(c32) * RB * NC * LP),
                            O_IB = al16(O_TW + sizeof(c32) * L), O_OB = O_IB + 8 * RB,
                            BYTES = al16(O_OB + 8 * RB);
    static __device__ void tables(const XArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, L, tid, NT);
    }
    static __device__ void tile(const XArgs &a, int64_t blk, char *sm, int tid)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW);
        int64_t *ib = (int64_t *)(sm + O_IB), *ob = (int64_t *)(sm + O_OB);
        const int64_t r0 = blk * RB;
        row_bases<RB, NT>(ib, ob, a, r0, tid);
        __syncthreads();
        const int nv = rows_valid<RB>(a, r0);
        row_fft<L, S, RB, NC, LP, NT, true, true, 0, 1, true>(buf, (const c32 *)a.in, (c32 *)a.out, ib, ob,
                                                  nv, tw, tid);
        __syncthreads();
    }
};

// ================================================================ binning
// Exact bin of integer squared radius q: max{b <= nbins-1 : thresh[b] <= q},
// thresh[b] = ceil(b^2 qmax / nbins^2), from an estimate corrected by
// integer comparisons against the bin's edges, so the result never depends
// on rounding.

// Bin edges (thresh[b], thresh[b + 1]) of bin b = 0..nbins as one 8-byte
// LDS entry; thresholds are < 2^32.  hi = 2^32 - 1 for the last bin (which
// also holds q = qmax) and past it.
struct BinEdge {
    uint32_t lo, hi;
};

// That bin for q < 2^32 and nbins <= 4096 from the edge table: the FP32
// estimate nbins sqrt(q / qmax) (cq = nbins^2 / qmax) is within 1e-3 of the
// exact value, so one comparison each way against the estimated bin's
// edges makes it exact.
__device__ __forceinline__ int bin_est(uint32_t q, float cq)
{
    // hardware square root (about 1 ulp; the correction absorbs it)
    return (int)__builtin_amdgcn_sqrtf((float)q * cq);  // 0..nbins
}
__device__ __forceinline__ int bin_fix(uint32_t q, int b, BinEdge e, int nbins)
{
    b += (q >= e.hi ? 1 : 0) - (q < e.lo ? 1 : 0);
    return b < nbins - 1 ? b : nbins - 1;
}
__device__ __forceinline__ int bin_edge(uint32_t q, int nbins, float cq, const BinEdge *edges)
{
    const int b = bin_est(q, cq);
    return bin_fix(q, b, edges[b], nbins);
}

// Zero the block's LDS histogram and fill its edge table.
__device__ __forceinline__ void load_edges(const ModeTables &mt, double *hist, BinEdge *edges,
                                           int tid, int nt)
{
    for (int i = tid; i <= mt.nbins; i += nt) {
        hist[i] = 0.0;
        edges[i] = BinEdge{(uint32_t)mt.thresh[i],
                           i < mt.nbins - 1 ? (uint32_t)mt.thresh[i + 1] : 0xffffffffu};
    }
}

// The same for `copies` histograms of nbins + 1 entries, one after another
// (one per wave of the block, or one for all).
__device__ __forceinline__ void hist_init(const ModeTables &mt, int copies, double *hist,
                                          BinEdge *edges, int tid, int nt)
{
    load_edges(mt, hist, edges, tid, nt);
    for (int i = mt.nbins + 1 + tid; i < copies * (mt.nbins + 1); i += nt) hist[i] = 0.0;
}

// out[i] = sum of the copies' entry i, copy 0 first (a fixed order: the
// block's binned sums do not depend on how its waves were scheduled); the
// copies are zeroed for the next tile.  Callers wait at a barrier before
// the histograms are used again.
__device__ __forceinline__ void hist_flush(int nbins, int copies, double *hist, double *out,
                                           int tid, int nt)
{
    const int w = nbins + 1;
    for (int i = tid; i < w; i += nt) {
        double s = hist[i];
        hist[i] = 0.0;
        for (int c = 1; c < copies; ++c) {
            s += hist[c * w + i];
            hist[c * w + i] = 0.0;
        }
        out[i] = s;
    }
}

// 1/d for d > 0 in FP64: the hardware reciprocal refined by one Newton step,
// which squares the estimate's relative error; the scale it feeds multiplies
// FP32 modes in FP64 and is rounded to FP32 with the product.
__device__ __forceinline__ double rcp_f64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    return fma(fma(-d, r, 1.0), r, r);
}

// The thread index, hidden from the optimiser once per tile when OPAQUE: the
// per-thread LDS and global offsets derived from it are then recomputed in
// every tile instead of being hoisted out of the tile loop, where dozens of
// them would stay live (and spill) across the fused pass.  The empty asm
// statement emits no instruction.
template <bool OPAQUE>
__device__ __forceinline__ int opaque_tid(int tid)
{
    if constexpr (OPAQUE) asm volatile("" : "+v"(tid));
    return tid;
}

// ============================================================ strided tiles
// EPI = false: plain pass (no epilogue code, fewest registers);
// EPI = true : last-axis pass with the binning / Poisson epilogue.
// hist / edges: LDS arrays (EPI with binning only): a.hcopies histograms of
// nbins + 1 entries (wave w adds into copy w, or all into copy 0) and the
// edge table; the tile adds its w|F|^2 sums into them.
// K2 (EPI): 1 the continuous k^2 of the last axis from |n_z|, 2 its table,
// 0 either, chosen per call (fewer kernels, more registers).
// m^2 for 0 <= m < 2^12 (mode indices) with a full-rate 24-bit multiply.
__device__ __forceinline__ uint32_t sq24(int m) { return __umul24((unsigned)m, (unsigned)m); }

// Element offset of column f of a strided pass: outer group o = f / C,
// then f - o C within it.  Passes have fewer than 2^31 columns (at most
// (N0 / 2 + 1) N1 nc of a 2048^3 lattice), so 32-bit division suffices.
__device__ __forceinline__ int64_t col_base(const SArgs &a, int64_t f)
{
    const int fi = (int)f, c = (int)a.ncols_inner;
    const int o = fi / c;
    return (int64_t)o * a.outer + (fi - o * c);
}

template <int L, int S, bool EPI, int NT, bool NTM = false, int K2 = 0>
struct STile {
    static constexpr int B = s_b(L);
    static constexpr int RPT = NT / B;  // row groups in the epilogue
    static constexpr size_t O_BUF = 0, O_TW = al16(sizeof(c32) * L * B),
                            BYTES = al16(O_TW + sizeof(c32) * L);
    static __device__ void tables(const SArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, L, tid, NT);
    }
    // The fused tile's inputs: the first forward stage's inputs, rows
    // j + r L/R0 of the thread's column (radix R0), all loads issued before
    // any of them is used (a column past the end loads column 0 and is
    // zeroed).
    static constexpr int R0 = nstages(L) == 0 ? 1 : radix_sel(L, 0, false);
    static constexpr int NB0 = col_nb(L, R0, B, NT);
    struct In {
        c32 v[NB0][R0];
    };
    static __device__ __forceinline__ void load_in(const SArgs &a, int64_t t, int tid, In &in)
    {
        constexpr int Q0 = L / R0;
        constexpr int JS = NT / B;
        const int col = tid % B;
        const int64_t f = t * B + col;
        const bool valid = f < a.ncols;
        // a column past the end reads column 0 (in bounds) and keeps zeros
        const int64_t base = valid ? col_base(a, f) : 0;
        const c32 *gin = (const c32 *)a.in + base;
        const int j0 = tid / B;
#pragma unroll
        for (int i = 0; i < NB0; ++i) {
            const int j = j0 + i * JS;
            if (Q0 % JS == 0 || j < Q0) {
                gload_pts<R0, NTM>(in.v[i], gin + (int64_t)j * a.stride, (int64_t)Q0 * a.stride,
                                   true);
#pragma unroll
                for (int r = 0; r < R0; ++r)
                    if (!valid) in.v[i][r] = c32{0.f, 0.f};
            } else {
#pragma unroll
                for (int r = 0; r < R0; ++r) in.v[i][r] = c32{0.f, 0.f};
            }
        }
    }

    static __device__ void tile(const SArgs &a, int64_t t, char *sm, int tid, double *hist,
                                const BinEdge *edges)
    {
        if constexpr (EPI) {
            In in;
            load_in(a, t, tid, in);
            tile_in(a, t, sm, tid, hist, edges, in);
            return;
        }
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW);
        const int col = tid % B;
        const bool store = (a.epi & EPI_STORE) != 0;
        const int64_t f = t * B + col;
        const bool valid = f < a.ncols;
        const int64_t base = valid ? col_base(a, f) : 0;
        const c32 *gin = (const c32 *)a.in + base;
        c32 *gout = (c32 *)a.out + base;
        // global -> registers -> stages -> registers -> global
        col_fft<L, S, B, NT, true, true, 0, 1, NTM>(buf, gin, gout, a.stride, valid && store, tw,
                                                     tid);
        __syncthreads();
    }

    // The fused tile from its loaded inputs (load_in of the same t).
    static __device__ __forceinline__ void tile_in(const SArgs &a, int64_t t, char *sm, int tid,
                                                   double *hist, const BinEdge *edges, In &in)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW);
        const int col = tid % B;
        const int rg = tid / B;
        const bool store = (a.epi & EPI_STORE) != 0;
        const int64_t f = t * B + col;
        const bool valid = f < a.ncols;
        const int64_t base = valid ? col_base(a, f) : 0;
        c32 *gout = (c32 *)a.out + base;
        epilogue(a, buf, tw, tid, col, rg, f, valid, store, gout, hist, edges, in);
        __syncthreads();
    }

    // Last-axis epilogue.  The forward transform stops with its last stage in
    // registers: thread (col, j0) holds the modes kz = j + r QL of column col
    // for its butterflies j.  The Poisson scale is applied there, and the
    // backward transform runs its radices in reverse order, so that its first
    // stage (radix RL, inputs at points j + r QL) starts from those same
    // registers.  The P(k) sums need runs of consecutive kz (so that
    // neighbouring modes share a bin): for them the modes are also written
    // to LDS in natural order and thread (col, rg) walks kz in
    // [rg EP, rg EP + EP).
    static __device__ __forceinline__ void epilogue(const SArgs &a, c32 *buf, const c32 *tw,
                                                    int tid, int col, int rg, int64_t f,
                                                    bool valid, bool store, c32 *gout,
                                                    double *hist, const BinEdge *edges, In &in)
    {
        constexpr int NST = nstages(L);
        constexpr int RL = NST == 0 ? 1 : radix_at(L, NST - 1);
        constexpr int QL = L / RL;
        constexpr int NB = col_nb(L, RL, B, NT);
        const int j0 = tid / B;
        // first forward stage (no twiddles) on the loaded inputs
#pragma unroll
        for (int i = 0; i < NB0; ++i) Dft<R0, S>::run(in.v[i]);
        c32 v[NB][RL];
        if constexpr (NST <= 1) {
            static_assert(NB0 == NB && R0 == RL, "one stage: its inputs are its butterflies");
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int r = 0; r < RL; ++r) v[i][r] = in.v[i][r];
        } else {
            col_stage_out<L, R0, 1, B, NT, false>(buf, nullptr, 0, false, tid, in.v);
            col_fft<L, S, B, NT, false, false, 1, R0, NTM, false, true>(buf, nullptr, nullptr, 0,
                                                                      false, tw, tid);
            col_stage_in<L, RL, QL, S, B, NT, false>(buf, nullptr, 0, false, tw, tid, v);
        }
        // column f = ky nxk + kx of the (kx, ky) plane (fewer than 2^31 columns)
        const int kx = valid ? (int)f % a.mt.nxk : 0;
        const int ky = valid ? (int)f / a.mt.nxk : 0;
        const bool corner = kx == 0 && ky == 0;
        // the column's |n_x|, |n_y| (the r2c half spectrum holds kx <= N0 / 2)
        const int mx = 2 * kx <= a.mt.n0 ? kx : a.mt.n0 - kx;
        const int my = 2 * ky <= a.mt.n1 ? ky : a.mt.n1 - ky;
        // this wave's histogram
        double *wh = hist + (a.hcopies > 1 ? (tid >> 6) * (a.mt.nbins + 1) : 0);
        // q_x + q_y of the column (exact integers below 2^32)
        const uint32_t qxy = a.mt.qx_unit * sq24(mx) + a.mt.qy_unit * sq24(my);
        if (a.epi & EPI_PK) {
            col_stage_out<L, RL, QL, B, NT, false>(buf, nullptr, 0, false, tid, v);
            bin_walk(a, buf, col, rg, kx, corner, qxy, valid, wh, edges);
        }
        if (a.epi & EPI_POISSON) {
            if (K2 == 1 || (K2 == 0 && a.mt.k2z_unit > 0.0)) {
                // continuous k^2 from |n_x|, |n_y|, |n_z|
                const double k2xy = valid ? fma(a.mt.k2x_unit, (double)sq24(mx),
                                                a.mt.k2y_unit * (double)sq24(my))
                                          : 1.0;
                scale_modes<true>(a, v, j0, k2xy, corner);
            } else {
                // the tables
                const double k2xy = valid ? a.mt.k2[0][kx] + a.mt.k2[1][ky] : 1.0;
                scale_modes<false>(a, v, j0, k2xy, corner);
            }
        }
        if (a.epi & EPI_PK_AFTER) {
            col_stage_out<L, RL, QL, B, NT, false>(buf, nullptr, 0, false, tid, v);
            bin_walk(a, buf, col, rg, kx, corner, qxy, valid, wh, edges);
        }
        if constexpr (S < 0) {
            if (a.epi & EPI_POISSON) {
                // backward transform: first stage (radix RL, no twiddles) from
                // the registers, the rest through LDS in reverse radix order
#pragma unroll
                for (int i = 0; i < NB; ++i) Dft<RL, +1>::run(v[i]);
                if constexpr (NST <= 1) {
                    col_stage_out<L, RL, 1, B, NT, true, NTM>(buf, gout, a.stride, valid && store,
                                                              tid, v);
                } else {
                    col_stage_out<L, RL, 1, B, NT, false>(buf, nullptr, 0, false, tid, v);
                    col_fft<L, +1, B, NT, false, true, 1, RL, NTM, true>(
                        buf, nullptr, gout, a.stride, valid && store, tw, tid);
                }
                return;
            }
        }
        if (store)  // spectrum out: the modes are still in registers
            col_stage_out<L, RL, QL, B, NT, true, NTM>(buf, gout, a.stride, valid, tid, v);
    }

    // The Poisson scale -1/(N k^2) (FP64, rounded once with the product) of
    // the modes kz = j + r QL a thread holds after the forward transform.
    template <bool CONT, int RL, int NB>
    static __device__ __forceinline__ void scale_modes(const SArgs &a, c32 (&v)[NB][RL], int j0,
                                                       double k2xy, bool corner)
    {
        constexpr int QL = L / RL;
        constexpr int JS = NT / B;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = j0 + i * JS;
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int kz = j + r * QL;
                if (QL % JS == 0 || j < QL) {
                    const int m = 2 * kz < L ? kz : L - kz;
                    const double k2z = CONT ? a.mt.k2z_unit * (double)sq24(m) : a.mt.k2[2][kz];
                    const double sc =
                        (corner && kz == 0) ? 0.0 : -a.mt.scale_n * rcp_f64(k2xy + k2z);
                    v[i][r] = c32{(float)((double)v[i][r].x * sc), (float)((double)v[i][r].y * sc)};
                }
            }
        }
    }

    // P(k) partial sums of the modes in LDS (natural order).  The modes kz
    // and L - kz have the same m = |n_z|, hence the same q and bin, so
    // thread (col, rg) walks m upward over its run [rg EH, rg EH + EH) of
    // 0 .. L/2 and takes both modes of each m (one at m = 0, and at m = L/2
    // for even L).  Along the run q = q_xy + m^2 q_u grows by integer
    // differences, and the bin changes where q reaches the current bin's
    // upper edge: to the next bin when one step of m never crosses two
    // thresholds (mt.walk1, checked when the thresholds are made), else to
    // the exact bin of q.  w |F|^2 sums go to `hist` -- the wave's own LDS
    // histogram, or the block's one -- at each change, in program order, so
    // with one histogram per wave the sums do not depend on scheduling.
    // Ends at a barrier, so LDS may be rewritten afterwards.
    static constexpr int MH = L / 2;                       // largest m
    static constexpr int EH = (MH + 1 + RPT - 1) / RPT;    // m values per row group
    static __device__ void bin_walk(const SArgs &a, const c32 *buf, int col, int rg, int kx,
                                    bool corner, uint32_t qxy, bool valid, double *hist,
                                    const BinEdge *edges)
    {
        const int nb = a.mt.nbins;
        const float cq = (float)((double)nb * nb / a.mt.qmax);
        // the half-spectrum weight is the same for the whole column
        const double wgt = (a.mt.half && !(kx == 0 || 2 * kx == a.mt.n0)) ? 2.0 : 1.0;
        const uint32_t qu = a.mt.qz_unit;
        const bool walk1 = a.mt.walk1 != 0;
        const int m0 = rg * EH;
        const int n = MH + 1 - m0 < EH ? MH + 1 - m0 : EH;  // may be <= 0
        if (valid && n > 0) {
            // q at m0 and its first difference (m0 + 1)^2 - m0^2 = 2 m0 + 1
            uint32_t q = qxy + sq24(m0) * qu;
            uint32_t dq = (uint32_t)(2 * m0 + 1) * qu;
            const uint32_t ddq = 2u * qu;
            // slot nbins: the zero mode (kept for the Parseval sum); q = 0
            // there, and the next mode's bin is then found from scratch
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
#pragma unroll 4
            for (int e = 0; e < EH; ++e) {
                if (EH * RPT != MH + 1 && e >= n) break;
                const int m = m0 + e;
                const c32 u = buf[m * B + col];
                // the partner mode L - m (none for m = 0, the same mode for 2 m = L)
                const bool two = m != 0 && 2 * m != L;
                const c32 w = buf[(two ? L - m : m) * B + col];
                if (q >= hi) {
                    atomicAdd(&hist[b], wgt * acc);
                    acc = 0.0;
                    if (walk1 && b < nb)
                        ++b;
                    else
                        b = bin_edge(q, nb, cq, edges);
                    hi = edges[b].hi;
                }
                double pw = (double)u.x * u.x + (double)u.y * u.y;
                if (two) pw += (double)w.x * w.x + (double)w.y * w.y;
                acc += pw;
                q += dq;
                dq += ddq;
            }
            atomicAdd(&hist[b], wgt * acc);
        }
        __syncthreads();
    }
};

// Wide strided tile: twice the columns of STile (256-byte row segments at
// L = 512) with twice the threads, one block per CU: for long strides (the
// last axis of large or multi-component fields), where longer contiguous
// segments per row pay for the lower block count.  No epilogue.
constexpr int kSWThreads = 1024;

template <int L, int S, int NT, bool NTM = false>
struct STileW {
    static constexpr int B = 2 * s_b(L);
    static constexpr size_t O_BUF = 0, O_TW = al16(sizeof(c32) * L * B),
                            BYTES = al16(O_TW + sizeof(c32) * L);
    static __device__ void tables(const SArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, L, tid, NT);
    }
    static __device__ void tile(const SArgs &a, int64_t t, char *sm, int tid)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW);
        const int col = tid % B;
        const int64_t f = t * B + col;
        const bool valid = f < a.ncols;
        const int64_t base = valid ? col_base(a, f) : 0;
        col_fft<L, S, B, NT, true, true, 0, 1, NTM>(buf, (const c32 *)a.in + base, (c32 *)a.out + base,
                                         a.stride, valid && (a.epi & EPI_STORE) != 0, tw, tid);
        __syncthreads();
    }
};

// Transposing strided tile for the z pass of a c2c plan in the paper's
// k-space order (k_z, k_x, k_y): every column's points are contiguous there
// (stride ncomp).  Forward (EPI_TSTORE): natural columns in, the last stage
// writes LDS and the tile is stored point-fastest; backward (EPI_TLOAD): the
// tile is loaded point-fastest into LDS and the last stage writes the
// natural columns.  Threads walk the tile's (column, point) pairs with the
// point fastest, so each column's run is read or written contiguously.
template <int L, int S, int NT>
struct STileT {
    static constexpr int B = s_b(L);
    static constexpr size_t O_BUF = 0, O_TW = al16(sizeof(c32) * L * B),
                            BYTES = al16(O_TW + sizeof(c32) * L);
    static __device__ void tables(const SArgs &a, char *sm, int tid)
    {
        load_table((c32 *)(sm + O_TW), a.tw, L, tid, NT);
    }
    static __device__ __forceinline__ int64_t tpos(const SArgs &a, int64_t f, int kz)
    {
        const int64_t c1 = a.t_n0 * a.t_nc;
        const int64_t y = f / c1, r = f - y * c1;
        const int64_t x = r / a.t_nc, c = r - x * a.t_nc;
        return ((y * a.t_n0 + x) * a.t_n2 + kz) * a.t_nc + c;
    }
    static __device__ void tile(const SArgs &a, int64_t t, char *sm, int tid)
    {
        c32 *buf = (c32 *)(sm + O_BUF);
        const c32 *tw = (const c32 *)(sm + O_TW);
        const int col = tid % B;
        const int64_t f0 = t * B;
        const int64_t f = f0 + col;
        const bool valid = f < a.ncols;
        const int64_t base = valid ? f : 0;  // natural z pass: column f at f
        if (a.epi & EPI_TLOAD) {
            const c32 *in = (const c32 *)a.in;
            for (int e = tid; e < B * L; e += NT) {
                const int kz = e % L, cl = e / L;
                const int64_t ff = f0 + cl;
                buf[kz * B + cl] = ff < a.ncols ? in[tpos(a, ff, kz)] : c32{0.f, 0.f};
            }
            __syncthreads();
            col_fft<L, S, B, NT, false, true>(buf, nullptr, (c32 *)a.out + base, a.stride, valid,
                                              tw, tid);
        } else {
            col_fft<L, S, B, NT, true, false>(buf, (const c32 *)a.in + base, nullptr, a.stride,
                                              valid, tw, tid);
            c32 *out = (c32 *)a.out;
            for (int e = tid; e < B * L; e += NT) {
                const int kz = e % L, cl = e / L;
                const int64_t ff = f0 + cl;
                if (ff < a.ncols) out[tpos(a, ff, kz)] = buf[kz * B + cl];
            }
        }
        __syncthreads();
    }
};

// ======================================================= standalone kernels
// One x tile per block (tile index = blockIdx.x).

template <int M, int NC>
__global__ __launch_bounds__(kXThreads) void k_x_r2c(XArgs a)
{
    using T = XR2CGen<M, NC, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    T::tables(a, sm, threadIdx.x);
    T::tile(a, blockIdx.x, sm, threadIdx.x, a.sumsq ? a.sumsq + blockIdx.x : nullptr);
}

template <int M, int NC>
__global__ __launch_bounds__(kXThreads) void k_x_c2r(XArgs a)
{
    using T = XC2RGen<M, NC, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    T::tables(a, sm, threadIdx.x);
    T::tile(a, blockIdx.x, sm, threadIdx.x);
}

template <int M>
__global__ __launch_bounds__(kXThreads) void k_x_r2c_v(XArgs a)
{
    using T = XR2CV<M, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    T::tables(a, sm, threadIdx.x);
    T::tile(a, blockIdx.x, sm, threadIdx.x, a.sumsq ? a.sumsq + blockIdx.x : nullptr);
}

template <int M>
__global__ __launch_bounds__(kXThreads) void k_x_c2r_v(XArgs a)
{
    using T = XC2RV<M, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    T::tables(a, sm, threadIdx.x);
    T::tile(a, blockIdx.x, sm, threadIdx.x);
}

template <int L, int NC, int S>
__global__ __launch_bounds__(kXThreads) void k_x_c2c_v(XArgs a)
{
    using T = XC2CV<L, NC, S, kXThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    T::tables(a, sm, threadIdx.x);
    T::tile(a, blockIdx.x, sm, threadIdx.x);
}

// Strided pass: persistent-style walk over tiles.
// Occupancy target: four waves per SIMD (two blocks per CU) except where the
// fused pass's LDS tables leave room for one block (lines of 1024 points and
// more), where two waves per SIMD are all it can reach.
template <int L, int S, bool EPI, bool NTM = false, int K2 = 0>
__global__ __launch_bounds__(kSThreads)
    __attribute__((amdgpu_waves_per_eu(EPI && L >= 1024 ? 2 : 4))) void k_strided(SArgs a)
{
    using T = STile<L, S, EPI, kSThreads, NTM, K2>;
    constexpr int NT = kSThreads;
    constexpr int B = T::B;
    __shared__ __align__(16) char sm[T::BYTES];
    extern __shared__ double dyn[];  // hist[hcopies][nbins + 1], edges[nbins + 1]
    const int tid = threadIdx.x;
    T::tables(a, sm, tid);
    const bool pk = EPI && (a.epi & (EPI_PK | EPI_PK_AFTER)) != 0;
    const int nb = a.mt.nbins;
    double *hist = dyn;
    BinEdge *edges = (BinEdge *)(dyn + a.hcopies * (nb + 1));
    if (pk) hist_init(a.mt, a.hcopies, hist, edges, tid, NT);
    __syncthreads();
    const int64_t ntiles = (a.ncols + B - 1) / B;
    // XCD-aware walk over virtual block ids vb = blockIdx.x + i * G (G is a
    // multiple of 8).  The chip hands block ids to its 8 XCDs in turn, so
    // vb mod 8 is this block's XCD.  Chunks of K consecutive tiles go to one
    // XCD and the chunks rotate over the XCDs: neighbouring tiles, which
    // share cache lines when rows are not 128-byte aligned, meet in one L2,
    // while all XCDs stream from nearby addresses.
    const int64_t K = a.xcd_chunk;
    const int64_t span = (ntiles + 8 * K - 1) / (8 * K) * (8 * K);
    auto tile_of = [&](int64_t vb) {
        const int64_t lb = vb / 8;
        return ((lb / K) * 8 + (vb % 8)) * K + lb % K;
    };
    for (int64_t vb = blockIdx.x; vb < span; vb += gridDim.x) {
        const int64_t t = tile_of(vb);
        if (t >= ntiles) continue;  // uniform over the block
        T::tile(a, t, sm, opaque_tid<EPI>(tid), hist, edges);
    }
    if (pk) {
        __syncthreads();
        hist_flush(nb, a.hcopies, hist, a.partial + (int64_t)blockIdx.x * (nb + 1), tid, NT);
    }
}

template <int L, int S, bool NTM = false>
__global__ __launch_bounds__(kSWThreads) void k_strided_w(SArgs a)
{
    using T = STileW<L, S, kSWThreads, NTM>;
    constexpr int B = T::B;
    __shared__ __align__(16) char sm[T::BYTES];
    const int tid = threadIdx.x;
    T::tables(a, sm, tid);
    __syncthreads();
    const int64_t ntiles = (a.ncols + B - 1) / B;
    const int64_t K = a.xcd_chunk;  // the XCD-aware walk of k_strided
    const int64_t span = (ntiles + 8 * K - 1) / (8 * K) * (8 * K);
    for (int64_t vb = blockIdx.x; vb < span; vb += gridDim.x) {
        const int64_t lb = vb / 8;
        const int64_t t = ((lb / K) * 8 + (vb % 8)) * K + lb % K;
        if (t >= ntiles) continue;  // uniform over the block
        T::tile(a, t, sm, tid);
    }
}

template <int L, int S>
__global__ __launch_bounds__(kSThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_strided_t(SArgs a)
{
    using T = STileT<L, S, kSThreads>;
    __shared__ __align__(16) char sm[T::BYTES];
    const int tid = threadIdx.x;
    T::tables(a, sm, tid);
    __syncthreads();
    const int64_t ntiles = (a.ncols + T::B - 1) / T::B;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) T::tile(a, t, sm, tid);
}

}  // namespace lf2
