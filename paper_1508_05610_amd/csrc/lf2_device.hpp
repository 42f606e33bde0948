// lf2_device.hpp -- device-side FFT engine for gfx950.
//
// Radix butterflies and an LDS-resident Stockham (autosort, decimation in
// time) driver.  One stage of radix R on a line of length L, after the
// stages already done have combined sub-transforms of length Ns, computes
// for every butterfly j in [0, L/R):
//   v_r = a[j + r L/R] * W_{Ns R}^{S r (j mod Ns)}        (r = 0..R-1)
//   v   = DFT_R(v)
//   b[(j div Ns) Ns R + (j mod Ns) + r Ns] = v_r
// and after the last stage the line holds its DFT in natural order.  Any
// order of radices whose product is L works; W_n = exp(2 pi i / n), S = -1
// forward and +1 backward.
//
// Lines live in LDS at address  line * LS + point * PS  (LS/PS chosen by the
// caller: contiguous lines for the x pass, interleaved columns for the
// strided passes so that lanes touch consecutive words).  A stage first
// reads every butterfly input of the thread into registers, waits at a
// barrier, then writes its outputs in place, and waits again.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf2 {

struct c32 {
    float x, y;
};

__device__ __forceinline__ c32 mk(float a, float b) { return c32{a, b}; }
__device__ __forceinline__ c32 add(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 sub(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c32 mul(c32 a, c32 b)
{
    return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ c32 conjg(c32 a) { return c32{a.x, -a.y}; }
__device__ __forceinline__ c32 scl(c32 a, float s) { return c32{a.x * s, a.y * s}; }
// s * i * a  (s = +-1)
template <int S>
__device__ __forceinline__ c32 muli(c32 a)
{
    return S > 0 ? c32{-a.y, a.x} : c32{a.y, -a.x};
}

// ---------------------------------------------------------------- butterflies
// In-place DFT of R values: v_k <- sum_r v_r exp(S 2 pi i r k / R).

template <int R, int S>
struct Dft;

template <int S>
struct Dft<1, S> {
    static __device__ __forceinline__ void run(c32 *) {}
};

template <int S>
struct Dft<2, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        c32 a = v[0], b = v[1];
        v[0] = add(a, b);
        v[1] = sub(a, b);
    }
};

template <int S>
struct Dft<3, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
        c32 t = add(v[1], v[2]);
        c32 u = sub(v[1], v[2]);
        c32 m = c32{v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y};
        c32 r = muli<S>(scl(u, h));
        v[0] = add(v[0], t);
        v[1] = add(m, r);
        v[2] = sub(m, r);
    }
};

template <int S>
struct Dft<4, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        c32 a = add(v[0], v[2]), b = sub(v[0], v[2]);
        c32 c = add(v[1], v[3]), d = muli<S>(sub(v[1], v[3]));
        v[0] = add(a, c);
        v[2] = sub(a, c);
        v[1] = add(b, d);
        v[3] = sub(b, d);
    }
};

template <int S>
struct Dft<5, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
        const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
        const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
        const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
        c32 t1 = add(v[1], v[4]), t2 = add(v[2], v[3]);
        c32 t3 = sub(v[1], v[4]), t4 = sub(v[2], v[3]);
        c32 a0 = v[0];
        c32 m1 = c32{a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y};
        c32 m2 = c32{a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y};
        c32 n1 = muli<S>(c32{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
        c32 n2 = muli<S>(c32{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
        v[0] = add(a0, add(t1, t2));
        v[1] = add(m1, n1);
        v[4] = sub(m1, n1);
        v[2] = add(m2, n2);
        v[3] = sub(m2, n2);
    }
};

template <int S>
struct Dft<8, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        const float r2 = 0.70710678118654752440f;
        c32 e[4] = {v[0], v[2], v[4], v[6]};
        c32 o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, S>::run(e);
        Dft<4, S>::run(o);
        // o[k] *= W8^{S k}
        o[1] = c32{r2 * (o[1].x - S * o[1].y), r2 * (o[1].y + S * o[1].x)};
        o[2] = muli<S>(o[2]);
        o[3] = c32{r2 * (-o[3].x - S * o[3].y), r2 * (-o[3].y + S * o[3].x)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = add(e[k], o[k]);
            v[k + 4] = sub(e[k], o[k]);
        }
    }
};

template <int S>
struct Dft<16, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        // 4 x 4: inner DFT4 over n1 (stride 4), twiddle W16^{n2 k1}, outer DFT4 over n2.
        const float c1 = 0.92387953251128675613f;  // cos(pi/8)
        const float s1 = 0.38268343236508977173f;  // sin(pi/8)
        const float r2 = 0.70710678118654752440f;
        c32 t[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) t[n2][n1] = v[4 * n1 + n2];
            Dft<4, S>::run(t[n2]);
        }
        // twiddles W16^{S n2 k1}: angle = S 2 pi n2 k1 / 16
        // n2 = 1: k1 = 1,2,3 -> (c1, S s1), (r2, S r2), (s1, S c1)
        // n2 = 2: k1 = 1,2,3 -> (r2, S r2), (0, S), (-r2, S r2)
        // n2 = 3: k1 = 1,2,3 -> (s1, S c1), (-r2, S r2), (-c1, -S s1)
        const c32 w11 = c32{c1, S * s1}, w12 = c32{r2, S * r2}, w13 = c32{s1, S * c1};
        const c32 w22 = c32{0.f, (float)S}, w23 = c32{-r2, S * r2};
        const c32 w33 = c32{-c1, -S * s1};
        t[1][1] = mul(t[1][1], w11);
        t[1][2] = mul(t[1][2], w12);
        t[1][3] = mul(t[1][3], w13);
        t[2][1] = mul(t[2][1], w12);
        t[2][2] = mul(t[2][2], w22);
        t[2][3] = mul(t[2][3], w23);
        t[3][1] = mul(t[3][1], w13);
        t[3][2] = mul(t[3][2], w23);
        t[3][3] = mul(t[3][3], w33);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            c32 u[4] = {t[0][k1], t[1][k1], t[2][k1], t[3][k1]};
            Dft<4, S>::run(u);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = u[k2];
        }
    }
};

template <int S>
struct Dft<32, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        // 2 x 16: radix 2 over n1 (n = 16 n1 + n2), twiddle W32^{n2 k1},
        // DFT16 over n2 for each k1; output k = k1 + 2 k2.
        const float c1 = 0.98078528040323044913f;  // cos(pi/16)
        const float s1 = 0.19509032201612826785f;  // sin(pi/16)
        const float c2 = 0.92387953251128675613f;  // cos(pi/8)
        const float s2 = 0.38268343236508977173f;  // sin(pi/8)
        const float c3 = 0.83146961230254523708f;  // cos(3 pi/16)
        const float s3 = 0.55557023301960222474f;  // sin(3 pi/16)
        const float r2 = 0.70710678118654752440f;
        // cos and sin of 2 pi m / 32, m = 0 .. 15
        const float cs[16] = {1.f, c1, c2, c3, r2, s3, s2, s1, 0.f, -s1, -s2, -s3, -r2, -c3, -c2, -c1};
        const float sn[16] = {0.f, s1, s2, s3, r2, c3, c2, c1, 1.f, c1, c2, c3, r2, s3, s2, s1};
        c32 e[16], o[16];
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
            const c32 a = v[n2], b = v[16 + n2];
            e[n2] = add(a, b);
            const c32 d = sub(a, b);
            if (n2 == 0)
                o[n2] = d;
            else if (n2 == 8)
                o[n2] = muli<S>(d);
            else
                o[n2] = mul(d, c32{cs[n2], S * sn[n2]});
        }
        Dft<16, S>::run(e);
        Dft<16, S>::run(o);
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            v[2 * k2] = e[k2];
            v[2 * k2 + 1] = o[k2];
        }
    }
};

// ---------------------------------------------------------------- radix plan
// Radices for a line of length L = 2^a * 3^b * 5^c: the power-of-two part in
// ceil(a/4) stages of 2..16 with the bits spread evenly (512 -> 8,8,8;
// 256 -> 16,16; 128 -> 16,8), then the factors 3 and 5.

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }
__host__ __device__ constexpr int pow2part(int n) { return (n % 2 == 0) ? 2 * pow2part(n / 2) : 1; }
__host__ __device__ constexpr int nstages_pow2(int L) { return (ilog2c(pow2part(L)) + 3) / 4; }
__host__ __device__ constexpr int count_factor(int n, int p) { return (n % p == 0 && n > 1) ? 1 + count_factor(n / p, p) : 0; }
__host__ __device__ constexpr int nstages(int L)
{
    return nstages_pow2(L) + count_factor(L, 3) + count_factor(L, 5);
}
__host__ __device__ constexpr int radix_at(int L, int st)
{
    // power-of-two stages first
    return st < nstages_pow2(L)
               ? (1 << (ilog2c(pow2part(L)) / nstages_pow2(L) +
                        (st < ilog2c(pow2part(L)) % nstages_pow2(L) ? 1 : 0)))
               : (st < nstages_pow2(L) + count_factor(L, 3) ? 3 : 5);
}
__host__ __device__ constexpr int max_radix(int L, int st = 0)
{
    return st >= nstages(L) ? 1
                            : (radix_at(L, st) > max_radix(L, st + 1) ? radix_at(L, st)
                                                                      : max_radix(L, st + 1));
}

// ------------------------------------------------------------ column engine
// NL interleaved lines (columns of a strided pass), element (line l, point p)
// at buf[l + p * NL].  NT is a multiple of NL, so thread tid always works on
// line tid % NL and on butterflies j = tid / NL + i * (NT / NL).  The first
// stage may take its inputs straight from global memory (rows j + r L/R of
// the thread's column, which for consecutive lanes are adjacent addresses)
// and the last stage may store its outputs straight to global memory (the
// last stage of a Stockham DIT writes point j + r L/R).  Stages that read
// and write LDS wait at a barrier between their reads and their writes.

// Global loads and stores of one complex value; NTM = true marks them
// nontemporal (streamed past the caches' normal allocation), which pays for
// the long-stride passes whose lines are touched once.
typedef float lf2_f2 __attribute__((ext_vector_type(2)));

template <bool NTM>
__device__ __forceinline__ c32 gload(const c32 *p)
{
    if constexpr (NTM) {
        const lf2_f2 t = __builtin_nontemporal_load((const lf2_f2 *)p);
        return c32{t.x, t.y};
    } else {
        return *p;
    }
}

template <bool NTM>
__device__ __forceinline__ void gstore(c32 *p, c32 v)
{
    if constexpr (NTM) {
        lf2_f2 t;
        t.x = v.x;
        t.y = v.y;
        __builtin_nontemporal_store(t, (lf2_f2 *)p);
    } else {
        *p = v;
    }
}

// Twiddle index r k C (C = L / (NS R), r < R, k < NS, all below 2^24) with
// a 24-bit multiply (full rate) rather than a 32-bit one.
template <int C>
__device__ __forceinline__ int tw_index(int r, int k)
{
    return (int)__umul24((unsigned)k, (unsigned)(r * C));
}

// Points p, p + qs, ..., p + (R - 1) qs of a column (zeros when !gv), and
// the stores back: one 64-bit pointer add per access, no multiplies.
template <int R, bool NTM>
__device__ __forceinline__ void gload_pts(c32 (&v)[R], const c32 *p, int64_t qs, bool gv)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        v[r] = gv ? gload<NTM>(p) : c32{0.f, 0.f};
        p += qs;
    }
}
template <int R, bool NTM>
__device__ __forceinline__ void gstore_pts(const c32 (&v)[R], c32 *p, int64_t qs)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        gstore<NTM>(p, v[r]);
        p += qs;
    }
}

template <int L, int R, int NS, int S, int NL, int NT, bool SRC_G, bool DST_G, bool NTM = false>
__device__ __forceinline__ void col_stage(c32 *buf, const c32 *gin, c32 *gout, int64_t gs,
                                          bool gv, const c32 *tw, int tid)
{
    constexpr int Q = L / R;
    constexpr int JS = NT / NL;
    constexpr int NB = (Q + JS - 1) / JS;
    static_assert(NT % NL == 0, "threads must tile the lines");
    static_assert(!DST_G || NS * R == L, "only the last stage stores to global memory");
    const int l = tid % NL;
    const int j0 = tid / NL;
    c32 v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = j0 + i * JS;
        if (Q % JS == 0 || j < Q) {
            if (SRC_G) {
                gload_pts<R, NTM>(v[i], gin + (int64_t)j * gs, (int64_t)Q * gs, gv);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = buf[l + (j + r * Q) * NL];
            }
        }
    }
    if (!SRC_G && !DST_G) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = j0 + i * JS;
        if (Q % JS == 0 || j < Q) {
            const int k = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    c32 w = tw[tw_index<L / (NS * R)>(r, k)];
                    if (S > 0) w = conjg(w);
                    v[i][r] = mul(v[i][r], w);
                }
            }
            Dft<R, S>::run(v[i]);
            if (DST_G) {
                if (gv) gstore_pts<R, NTM>(v[i], gout + (int64_t)j * gs, (int64_t)Q * gs);
            } else {
                c32 *dst = buf + l + ((j / NS) * NS * R + k) * NL;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * NS * NL] = v[i][r];
            }
        }
    }
    if (!DST_G) __syncthreads();
}

// ------------------------------------------------------------ row engine
// RB rows of NC interleaved components (the x pass): component c of point p
// of row q sits at global offset rowoff[q] + p * NC + c and at
// buf[(q * NC + c) * LP + lpad(p)] in LDS (one LDS line per row and
// component).  lpad inserts one empty slot after every 16 points, so the
// stride-R writes of the early Stockham stages (points j R + r over
// consecutive j) fall in different banks; LP must be at least
// lpad(points per line - 1) + 1 (row_pitch).
// Butterfly b = tid + i NT of a stage maps to component b % NC, then
// j = (b / NC) % Q, then row b / (NC Q): consecutive lanes walk consecutive
// memory, so the first stage's global loads (point j + r Q) and the last
// stage's global stores are contiguous across a wave.  Only rows < nvalid
// exist in memory.
// PACK (real rows of the r2c / c2r x pass): the global side is a float
// array with row offsets in floats, and point p of component c is the pair
// (f[2p][c], f[2p + 1][c]) = floats (2p) NC + c and (2p + 1) NC + c, loaded
// (first stage) or stored (last stage) as two floats.

__host__ __device__ constexpr int lpad(int p) { return p + (p >> 4); }
__host__ __device__ constexpr int row_pitch(int npoints) { return lpad(npoints - 1) + 1; }

template <bool NTM>
__device__ __forceinline__ float gloadf(const float *p)
{
    if constexpr (NTM)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NTM>
__device__ __forceinline__ void gstoref(float *p, float v)
{
    if constexpr (NTM)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int L, int R, int NS, int S, int RB, int NC, int LP, int NT, bool SRC_G, bool DST_G,
          bool NTM = false, bool PACK = false>
__device__ __forceinline__ void row_stage(c32 *buf, const c32 *gin, c32 *gout,
                                          const int64_t *rowoff_in, const int64_t *rowoff_out,
                                          int nvalid, const c32 *tw, int tid, double *ssq)
{
    constexpr int Q = L / R;
    constexpr int NBF = RB * NC * Q;
    constexpr int NB = (NBF + NT - 1) / NT;
    static_assert(!DST_G || NS * R == L, "only the last stage stores to global memory");
    c32 v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid + i * NT;
        if (NBF % NT == 0 || b < NBF) {
            const int c = b % NC, t = b / NC;
            const int j = t % Q, q = t / Q;
            const int l = q * NC + c;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (SRC_G && PACK) {
                    const float *fp = (const float *)gin + rowoff_in[q] + 2 * (j + r * Q) * NC + c;
                    v[i][r] = q < nvalid ? c32{gloadf<NTM>(fp), gloadf<NTM>(fp + NC)}
                                         : c32{0.f, 0.f};
                } else if (SRC_G) {
                    v[i][r] = q < nvalid ? gload<NTM>(gin + rowoff_in[q] + (j + r * Q) * NC + c)
                                         : c32{0.f, 0.f};
                } else {
                    v[i][r] = buf[l * LP + lpad(j + r * Q)];
                }
            }
            if (SRC_G && ssq) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    *ssq += (double)v[i][r].x * v[i][r].x + (double)v[i][r].y * v[i][r].y;
            }
        }
    }
    if (!SRC_G && !DST_G) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid + i * NT;
        if (NBF % NT == 0 || b < NBF) {
            const int c = b % NC, t = b / NC;
            const int j = t % Q, q = t / Q;
            const int l = q * NC + c;
            const int k = j % NS;
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    c32 w = tw[tw_index<L / (NS * R)>(r, k)];
                    if (S > 0) w = conjg(w);
                    v[i][r] = mul(v[i][r], w);
                }
            }
            Dft<R, S>::run(v[i]);
            if (DST_G && PACK) {
                if (q < nvalid) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        float *fp = (float *)gout + rowoff_out[q] + 2 * (j + r * Q) * NC + c;
                        gstoref<NTM>(fp, v[i][r].x);
                        gstoref<NTM>(fp + NC, v[i][r].y);
                    }
                }
            } else if (DST_G) {
                if (q < nvalid) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        gstore<NTM>(gout + rowoff_out[q] + (j + r * Q) * NC + c, v[i][r]);
                }
            } else {
                c32 *dst = buf + l * LP;
                const int p0 = (j / NS) * NS * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[lpad(p0 + r * NS)] = v[i][r];
            }
        }
    }
    if (!DST_G) __syncthreads();
}

template <int L, int S, int RB, int NC, int LP, int NT, bool SRC_G, bool DST_G, int ST = 0,
          int NS = 1, bool NTM = false, bool PACK = false>
__device__ __forceinline__ void row_fft(c32 *buf, const c32 *gin, c32 *gout,
                                        const int64_t *rowoff_in, const int64_t *rowoff_out,
                                        int nvalid, const c32 *tw, int tid, double *ssq = nullptr)
{
    if constexpr (L == 1) {
        for (int b = tid; b < RB * NC; b += NT) {
            const int c = b % NC, q = b / NC;
            c32 v = buf[b * LP];
            if (SRC_G && PACK) {
                const float *fp = (const float *)gin + rowoff_in[q] + c;
                v = q < nvalid ? c32{fp[0], fp[NC]} : c32{0.f, 0.f};
            } else if (SRC_G) {
                v = q < nvalid ? gin[rowoff_in[q] + c] : c32{0.f, 0.f};
            }
            if (SRC_G && ssq) *ssq += (double)v.x * v.x + (double)v.y * v.y;
            if (DST_G && PACK) {
                if (q < nvalid) {
                    float *fp = (float *)gout + rowoff_out[q] + c;
                    fp[0] = v.x;
                    fp[NC] = v.y;
                }
            } else if (DST_G) {
                if (q < nvalid) gout[rowoff_out[q] + c] = v;
            } else {
                buf[b * LP] = v;
            }
        }
        __syncthreads();
    } else if constexpr (NS < L) {
        constexpr int R = radix_at(L, ST);
        constexpr bool first = ST == 0, last = NS * R == L;
        row_stage<L, R, NS, S, RB, NC, LP, NT, first && SRC_G, last && DST_G, NTM, PACK>(
            buf, gin, gout, rowoff_in, rowoff_out, nvalid, tw, tid, ssq);
        row_fft<L, S, RB, NC, LP, NT, SRC_G, DST_G, ST + 1, NS * R, NTM, PACK>(
            buf, gin, gout, rowoff_in, rowoff_out, nvalid, tw, tid, ssq);
    }
}

// Radix of stage st, in the plan's order or (REV) in reverse order.  Any
// order of the factors gives the same DFT; the reverse order lets a
// transform start with the radix another one ended with (register hand-off
// in the fused Poisson pass).
__host__ __device__ constexpr int radix_sel(int L, int st, bool rev)
{
    return rev ? radix_at(L, nstages(L) - 1 - st) : radix_at(L, st);
}

// Butterflies per thread of a column stage with Q = L / R butterflies per
// line and NT / NL threads per line.
__host__ __device__ constexpr int col_nb(int L, int R, int NL, int NT)
{
    return (L / R + NT / NL - 1) / (NT / NL);
}

// First half of a column stage: load the butterfly inputs (global memory or
// LDS), apply the stage twiddles and the radix-R DFT, and leave the R outputs
// of each butterfly j in v (they belong at points j + r Q when this is the
// last stage).  After LDS reads the block waits at a barrier, so LDS may be
// rewritten afterwards.
template <int L, int R, int NS, int S, int NL, int NT, bool SRC_G, bool NTM = false>
__device__ __forceinline__ void col_stage_in(const c32 *buf, const c32 *gin, int64_t gs, bool gv,
                                             const c32 *tw, int tid,
                                             c32 (&v)[col_nb(L, R, NL, NT)][R])
{
    constexpr int Q = L / R;
    constexpr int JS = NT / NL;
    constexpr int NB = col_nb(L, R, NL, NT);
    const int l = tid % NL;
    const int j0 = tid / NL;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = j0 + i * JS;
        if (Q % JS == 0 || j < Q) {
            if (SRC_G) {
                gload_pts<R, NTM>(v[i], gin + (int64_t)j * gs, (int64_t)Q * gs, gv);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = buf[l + (j + r * Q) * NL];
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = c32{0.f, 0.f};
        }
    }
    if (!SRC_G) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = j0 + i * JS;
        const int k = j % NS;
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                c32 w = tw[tw_index<L / (NS * R)>(r, k)];
                if (S > 0) w = conjg(w);
                v[i][r] = mul(v[i][r], w);
            }
        }
        Dft<R, S>::run(v[i]);
    }
}

// Second half of a column stage: store v (as produced by col_stage_in with
// the same L, R, NS) to global memory (last stage only) or to the LDS slots
// the next stage reads; LDS writes end at a barrier.
template <int L, int R, int NS, int NL, int NT, bool DST_G, bool NTM = false>
__device__ __forceinline__ void col_stage_out(c32 *buf, c32 *gout, int64_t gs, bool gv, int tid,
                                              const c32 (&v)[col_nb(L, R, NL, NT)][R])
{
    constexpr int Q = L / R;
    constexpr int JS = NT / NL;
    constexpr int NB = col_nb(L, R, NL, NT);
    static_assert(!DST_G || NS * R == L, "only the last stage stores to global memory");
    const int l = tid % NL;
    const int j0 = tid / NL;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = j0 + i * JS;
        if (Q % JS == 0 || j < Q) {
            const int k = j % NS;
            if (DST_G) {
                if (gv) gstore_pts<R, NTM>(v[i], gout + (int64_t)j * gs, (int64_t)Q * gs);
            } else {
                c32 *dst = buf + l + ((j / NS) * NS * R + k) * NL;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * NS * NL] = v[i][r];
            }
        }
    }
    if (!DST_G) __syncthreads();
}

// Whole transform of the NL columns; SRC_G / DST_G select global input for
// the first stage and global output for the last stage.  L = 1 is a copy.
// REV runs the radices in reverse order; SKIP_LAST stops before the last
// stage (whose inputs are then in LDS).
template <int L, int S, int NL, int NT, bool SRC_G, bool DST_G, int ST = 0, int NS = 1,
          bool NTM = false, bool REV = false, bool SKIP_LAST = false>
__device__ __forceinline__ void col_fft(c32 *buf, const c32 *gin, c32 *gout, int64_t gs, bool gv,
                                        const c32 *tw, int tid)
{
    if constexpr (L == 1) {
        if (tid < NL) {
            const int l = tid;
            c32 v = SRC_G ? (gv ? gin[0] : c32{0.f, 0.f}) : buf[l];
            if (DST_G) {
                if (gv) gout[0] = v;
            } else {
                buf[l] = v;
            }
        }
        __syncthreads();
    } else if constexpr (NS < L) {
        constexpr int R = radix_sel(L, ST, REV);
        constexpr bool first = ST == 0, last = NS * R == L;
        if constexpr (!(last && SKIP_LAST)) {
            col_stage<L, R, NS, S, NL, NT, first && SRC_G, last && DST_G, NTM>(buf, gin, gout, gs,
                                                                               gv, tw, tid);
            col_fft<L, S, NL, NT, SRC_G, DST_G, ST + 1, NS * R, NTM, REV, SKIP_LAST>(buf, gin, gout,
                                                                                    gs, gv, tw, tid);
        }
    }
}

}  // namespace lf2
