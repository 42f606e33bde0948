/*
 * lf2 oracle: plain FP64 CPU reference for the 3-D FFT, spectral Poisson
 * solve and power-spectrum binning of LATfield2 (Daverio, Hindmarsh & Bevis,
 * arXiv:1508.05610).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library calls, links or
 * includes this file; only the tests, the smoke check and the bench's CPU
 * baseline leg use it.  It shares no code with the HIP path.
 *
 * Conventions (the paper fixes none of them; the readings are listed in the
 * design notes of the repository):
 *   - Lattice N0 x N1 x N2, row-major with dimension 0 fastest (paper,
 *     section 3.4: Site indexing runs from dimension 0 to the last one).
 *     A real field is double[N2][N1][N0]; a complex field stores
 *     (re, im) pairs, double[N2][N1][N0][2].
 *   - Forward transform uses exp(-2 pi i k.x / N), backward exp(+...);
 *     neither direction is normalised (the FFT is built on FFTW's 1-d
 *     transforms, section 3.6, whose convention this is).
 *   - r2c keeps the first Nh = N0/2 + 1 entries along dimension 0 (the
 *     halved axis is listed first in the r2c k-space layout, section 3.6).
 *   - Periodic boundaries (section 3, Lattice: periodic conditions only).
 *
 * Every twiddle is cos/sin of 2 pi m / n with the integer m reduced modulo
 * n first.  The file is compiled with -ffp-contract=off.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double ORC_TWO_PI = 6.283185307179586476925286766559;

/* exp(sign * 2 pi i * j / n) with j reduced modulo n in integers first. */
static cplx unit_root(int64_t j, int64_t n, int sign)
{
    int64_t m = j % n;
    if (m < 0) m += n;
    double a = ORC_TWO_PI * (double)m / (double)n;
    return CMPLX(cos(a), (double)sign * sin(a));
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* 1-D transforms                                                      */
/* ------------------------------------------------------------------ */

/* Direct definition: out[k] = sum_j in[j] exp(sign 2 pi i j k / n). */
void orc_dft1d(int64_t n, const double *in, double *out, int sign)
{
    const cplx *x = (const cplx *)in;
    cplx *y = (cplx *)out;
    for (int64_t k = 0; k < n; ++k) {
        cplx acc = 0;
        for (int64_t j = 0; j < n; ++j) acc += x[j] * unit_root(j * k, n, sign);
        y[k] = acc;
    }
}

/* Per-length table of exp(sign 2 pi i m / n), m in [0, n). */
typedef struct {
    int64_t n;
    int sign;
    cplx *w;
} root_table;

static root_table table_make(int64_t n, int sign)
{
    root_table t;
    t.n = n;
    t.sign = sign;
    t.w = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 0 ? n : 1));
    for (int64_t m = 0; m < n; ++m) t.w[m] = unit_root(m, n, sign);
    return t;
}

static void table_free(root_table *t) { free(t->w); t->w = NULL; }

/* exp(sign 2 pi i j / len) for a divisor len of t->n. */
static inline cplx table_root(const root_table *t, int64_t j, int64_t len)
{
    int64_t m = j % len;
    return t->w[m * (t->n / len)];
}

static int smallest_factor(int64_t n)
{
    if (n % 2 == 0) return 2;
    if (n % 3 == 0) return 3;
    if (n % 5 == 0) return 5;
    for (int64_t p = 7; p * p <= n; p += 2)
        if (n % p == 0) return (int)p;
    return (int)n;
}

/*
 * Decimation in time, one prime factor p of n per level:
 *   X[k + q m] = sum_{r<p} exp(sign 2 pi i r (k + q m) / n) Y_r[k],
 * where m = n / p and Y_r is the length-m DFT of x[r], x[r+p], x[r+2p], ...
 * Input x with element stride s; output y contiguous.  scratch holds n.
 */
static void fft_rec(int64_t n, const cplx *x, int64_t s, cplx *y, const root_table *t,
                    cplx *scratch)
{
    if (n == 1) {
        y[0] = x[0];
        return;
    }
    int p = smallest_factor(n);
    int64_t m = n / p;
    for (int r = 0; r < p; ++r) fft_rec(m, x + r * s, s * p, y + r * m, t, scratch);
    for (int64_t q = 0; q < p; ++q)
        for (int64_t k = 0; k < m; ++k) {
            cplx acc = 0;
            for (int r = 0; r < p; ++r) acc += table_root(t, r * (k + q * m), n) * y[r * m + k];
            scratch[k + q * m] = acc;
        }
    memcpy(y, scratch, sizeof(cplx) * (size_t)n);
}

/* In-place 1-D FFT of a contiguous complex array. */
void orc_fft1d(int64_t n, double *data, int sign)
{
    root_table t = table_make(n, sign);
    cplx *in = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *scr = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    memcpy(in, data, sizeof(cplx) * (size_t)n);
    fft_rec(n, in, 1, (cplx *)data, &t, scr);
    free(in);
    free(scr);
    table_free(&t);
}

/*
 * Transform every line of a complex array along one axis.
 * The array has n_line points along the axis at stride `stride` (in complex
 * elements); lines are enumerated by (outer, inner) with
 *   base = outer * outer_stride + inner, inner < n_inner.
 */
static void fft_axis(cplx *a, int64_t n_line, int64_t stride, int64_t n_inner, int64_t n_outer,
                     int64_t outer_stride, int sign)
{
    if (n_line <= 1) return;
    root_table t = table_make(n_line, sign);
    int64_t nlines = n_inner * n_outer;
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n_line);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)n_line);
        cplx *scr = (cplx *)malloc(sizeof(cplx) * (size_t)n_line);
#pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; ++l) {
            int64_t outer = l / n_inner, inner = l % n_inner;
            cplx *base = a + outer * outer_stride + inner;
            for (int64_t j = 0; j < n_line; ++j) buf[j] = base[j * stride];
            fft_rec(n_line, buf, 1, res, &t, scr);
            for (int64_t j = 0; j < n_line; ++j) base[j * stride] = res[j];
        }
        free(buf);
        free(res);
        free(scr);
    }
    table_free(&t);
}

/* Separable 3-D c2c on a dense complex array [n2][n1][n0] (in place):
 * along dimension 0, then 1, then 2. */
static void c2c3d_inplace(cplx *a, const int64_t n[3], int sign)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2];
    fft_axis(a, n0, 1, 1, n1 * n2, n0, sign);          /* x lines */
    fft_axis(a, n1, n0, n0, n2, n0 * n1, sign);        /* y lines */
    fft_axis(a, n2, n0 * n1, n0 * n1, 1, 0, sign);     /* z lines */
}

/* 3-D DFT of a complex field, c2c, unnormalised.  in and out may alias. */
void orc_c2c3d(const int64_t n[3], const double *in, double *out, int sign)
{
    int64_t tot = n[0] * n[1] * n[2];
    if (out != in) memcpy(out, in, sizeof(cplx) * (size_t)tot);
    c2c3d_inplace((cplx *)out, n, sign);
}

/* r2c: first Nh = n0/2+1 entries along dimension 0 of the forward c2c
 * transform of the real field.  in: double[n2][n1][n0]; out: complex
 * [n2][n1][nh]. */
void orc_r2c3d(const int64_t n[3], const double *in, double *out)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2], nh = n0 / 2 + 1;
    int64_t rows = n1 * n2;
    root_table t = table_make(n0, -1);
    cplx *o = (cplx *)out;
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
        cplx *scr = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            for (int64_t x = 0; x < n0; ++x) buf[x] = in[r * n0 + x];
            fft_rec(n0, buf, 1, res, &t, scr);
            for (int64_t k = 0; k < nh; ++k) o[r * nh + k] = res[k];
        }
        free(buf);
        free(res);
        free(scr);
    }
    table_free(&t);
    fft_axis(o, n1, nh, nh, n2, nh * n1, -1);
    fft_axis(o, n2, nh * n1, nh * n1, 1, 0, -1);
}

/*
 * c2r of a half spectrum G[n2][n1][nh] (input untouched):
 *   out(x) = sum over half-spectrum modes k of c(k_x) Re(G_k exp(+2 pi i k.x/N)),
 * with c = 1 for k_x in {0, n0/2} and c = 2 otherwise.  For a Hermitian
 * half spectrum this is the unnormalised inverse DFT; for any other input it
 * is the real part of the inverse DFT of the weighted half spectrum.
 * Steps: backward c2c along dimensions 2 and 1 on a copy, then per row the
 * full-length backward transform of Y[k] = c(k) H[k] (k <= n0/2), Y[k] = 0
 * above, keeping the real part.
 */
void orc_c2r3d(const int64_t n[3], const double *in, double *out)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2], nh = n0 / 2 + 1;
    int64_t rows = n1 * n2;
    cplx *h = (cplx *)malloc(sizeof(cplx) * (size_t)(nh * rows));
    memcpy(h, in, sizeof(cplx) * (size_t)(nh * rows));
    fft_axis(h, n2, nh * n1, nh * n1, 1, 0, +1);
    fft_axis(h, n1, nh, nh, n2, nh * n1, +1);
    root_table t = table_make(n0, +1);
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
        cplx *scr = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            for (int64_t k = 0; k < n0; ++k) {
                if (k < nh) {
                    double c = (k == 0 || 2 * k == n0) ? 1.0 : 2.0;
                    buf[k] = c * h[r * nh + k];
                } else {
                    buf[k] = 0;
                }
            }
            fft_rec(n0, buf, 1, res, &t, scr);
            for (int64_t x = 0; x < n0; ++x) out[r * n0 + x] = creal(res[x]);
        }
        free(buf);
        free(res);
        free(scr);
    }
    table_free(&t);
    free(h);
}

/*
 * One mode of the 3-D DFT straight from the definition,
 *   F(k) = sum_{x,y,z} f(x,y,z) exp(sign 2 pi i (kx x/n0 + ky y/n1 + kz z/n2)),
 * summed over x, then y, then z.  f is real (is_complex = 0) or complex.
 * Cost O(N) per mode; used to sample large transforms one output at a time.
 */
void orc_dft3d_at(const int64_t n[3], const double *f, int is_complex, const int64_t k[3],
                  int sign, double *res)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2];
    cplx *wx = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
    cplx *wy = (cplx *)malloc(sizeof(cplx) * (size_t)n1);
    cplx *wz = (cplx *)malloc(sizeof(cplx) * (size_t)n2);
    for (int64_t x = 0; x < n0; ++x) wx[x] = unit_root(k[0] * x, n0, sign);
    for (int64_t y = 0; y < n1; ++y) wy[y] = unit_root(k[1] * y, n1, sign);
    for (int64_t z = 0; z < n2; ++z) wz[z] = unit_root(k[2] * z, n2, sign);
    cplx *bz = (cplx *)malloc(sizeof(cplx) * (size_t)n2);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < n2; ++z) {
        cplx sy = 0;
        for (int64_t y = 0; y < n1; ++y) {
            cplx sx = 0;
            int64_t row = (z * n1 + y) * n0;
            if (is_complex) {
                const cplx *fc = (const cplx *)f;
                for (int64_t x = 0; x < n0; ++x) sx += fc[row + x] * wx[x];
            } else {
                for (int64_t x = 0; x < n0; ++x) sx += f[row + x] * wx[x];
            }
            sy += sx * wy[y];
        }
        bz[z] = sy * wz[z];
    }
    cplx acc = 0;
    for (int64_t z = 0; z < n2; ++z) acc += bz[z];
    res[0] = creal(acc);
    res[1] = cimag(acc);
    free(wx);
    free(wy);
    free(wz);
    free(bz);
}

/* ------------------------------------------------------------------ */
/* Wavevectors                                                         */
/* ------------------------------------------------------------------ */

/* Signed integer wavenumber: n if n < N/2, else n - N (Nyquist -> -N/2). */
static inline int64_t signed_mode(int64_t n, int64_t N) { return (2 * n < N) ? n : n - N; }

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int64_t orc_lcm3(const int64_t n[3])
{
    int64_t l = n[0];
    l = l / gcd64(l, n[1]) * n[1];
    l = l / gcd64(l, n[2]) * n[2];
    return l;
}

/*
 * Poisson:  laplacian(phi) = rho on the periodic lattice with spacing dx.
 *   phi_hat(n) = -rho_hat(n) / k^2(n) for n != 0, phi_hat(0) = 0,
 *   phi = c2r(phi_hat) / N.
 * k2mode 0 (continuous spectral): k^2 = sum_i (2 pi nt_i / (N_i dx))^2
 * k2mode 1 (discrete 7-point):    k^2 = sum_i (2/dx)^2 sin^2(pi n_i / N_i)
 * where nt_i is the signed wavenumber.  rho: double[n2][n1][n0].
 */
void orc_poisson(const int64_t n[3], double dx, int k2mode, const double *rho, double *phi)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2], nh = n0 / 2 + 1;
    int64_t tot = n0 * n1 * n2;
    cplx *F = (cplx *)malloc(sizeof(cplx) * (size_t)(nh * n1 * n2));
    orc_r2c3d(n, rho, (double *)F);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < n2; ++z)
        for (int64_t y = 0; y < n1; ++y)
            for (int64_t kx = 0; kx < nh; ++kx) {
                int64_t idx = (z * n1 + y) * nh + kx;
                if (kx == 0 && y == 0 && z == 0) {
                    F[idx] = 0;
                    continue;
                }
                double k2;
                if (k2mode == 0) {
                    double ax = ORC_TWO_PI * (double)signed_mode(kx, n0) / ((double)n0 * dx);
                    double ay = ORC_TWO_PI * (double)signed_mode(y, n1) / ((double)n1 * dx);
                    double az = ORC_TWO_PI * (double)signed_mode(z, n2) / ((double)n2 * dx);
                    k2 = ax * ax + ay * ay + az * az;
                } else {
                    double sx = sin(M_PI * (double)kx / (double)n0);
                    double sy = sin(M_PI * (double)y / (double)n1);
                    double sz = sin(M_PI * (double)z / (double)n2);
                    k2 = (4.0 / (dx * dx)) * (sx * sx + sy * sy + sz * sz);
                }
                F[idx] = -F[idx] / k2;
            }
    orc_c2r3d(n, (const double *)F, phi);
    for (int64_t i = 0; i < tot; ++i) phi[i] /= (double)tot;
    free(F);
}

/*
 * Power-spectrum bin of a mode with integer squared radius
 *   q = sum_i (nt_i L / N_i)^2,  L = lcm(N0, N1, N2),
 * relative to the corner q_max = sum_i (floor(N_i/2) L / N_i)^2:
 *   b = min(nbins - 1, max{ b : b^2 q_max <= nbins^2 q }).
 */
int64_t orc_pk_bin(int64_t q, int64_t qmax, int64_t nbins)
{
    int64_t rhs = nbins * nbins * q;
    int64_t b = (int64_t)floor((double)nbins * sqrt((double)q / (double)qmax));
    if (b < 0) b = 0;
    while (b > 0 && b * b * qmax > rhs) --b;
    while ((b + 1) * (b + 1) * qmax <= rhs) ++b;
    return b < nbins - 1 ? b : nbins - 1;
}

int64_t orc_pk_qmax(const int64_t n[3])
{
    int64_t L = orc_lcm3(n), q = 0;
    for (int i = 0; i < 3; ++i) {
        int64_t a = (n[i] / 2) * (L / n[i]);
        q += a * a;
    }
    return q;
}

/*
 * Shell-averaged power spectrum of a transformed field F.
 *   half = 1: F is the r2c half spectrum complex[n2][n1][nh], modes carry
 *             weight w = 1 at k_x in {0, n0/2} and w = 2 otherwise;
 *   half = 0: F is a full spectrum complex[n2][n1][n0], w = 1.
 * The zero mode is excluded.  For each bin b:
 *   count_b = sum w,
 *   pk_b    = (dx^3 / N) sum w |F|^2 / count_b,
 *   kmean_b = sum w |k| / count_b,  |k| = 2 pi sqrt(q) / (L dx),
 * and 0 for empty bins.  Sums are accumulated per bin in FP64 in lattice
 * order (z outermost, x innermost).
 */
void orc_power_spectrum(const int64_t n[3], int half, const double *Fin, int64_t nbins, double dx,
                        double *pk, double *kmean, double *count)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2];
    int64_t nx = half ? n0 / 2 + 1 : n0;
    int64_t L = orc_lcm3(n), qmax = orc_pk_qmax(n);
    const cplx *F = (const cplx *)Fin;
    double *sp = (double *)calloc((size_t)nbins, sizeof(double));
    double *sk = (double *)calloc((size_t)nbins, sizeof(double));
    double *sw = (double *)calloc((size_t)nbins, sizeof(double));
    for (int64_t z = 0; z < n2; ++z)
        for (int64_t y = 0; y < n1; ++y)
            for (int64_t kx = 0; kx < nx; ++kx) {
                if (kx == 0 && y == 0 && z == 0) continue;
                int64_t a = signed_mode(kx, n0) * (L / n0);
                int64_t b = signed_mode(y, n1) * (L / n1);
                int64_t c = signed_mode(z, n2) * (L / n2);
                int64_t q = a * a + b * b + c * c;
                int64_t bin = orc_pk_bin(q, qmax, nbins);
                double w = 1.0;
                if (half && !(kx == 0 || 2 * kx == n0)) w = 2.0;
                cplx v = F[(z * n1 + y) * nx + kx];
                double p2 = creal(v) * creal(v) + cimag(v) * cimag(v);
                sp[bin] += w * p2;
                sk[bin] += w * (ORC_TWO_PI * sqrt((double)q) / ((double)L * dx));
                sw[bin] += w;
            }
    double norm = dx * dx * dx / (double)(n0 * n1 * n2);
    for (int64_t b = 0; b < nbins; ++b) {
        count[b] = sw[b];
        pk[b] = sw[b] > 0 ? norm * sp[b] / sw[b] : 0.0;
        kmean[b] = sw[b] > 0 ? sk[b] / sw[b] : 0.0;
    }
    free(sp);
    free(sk);
    free(sw);
}

/*
 * Gaussian random field with a fixed-amplitude spectrum |F| = |k|^(-alpha/2)
 * (so P(k) is proportional to k^-alpha) and seeded phases:
 *   F(n) = |k|^(-alpha/2) exp(i theta(n)),  F(0) = 0,
 * theta = 2 pi u[m] with m the larger of the flat full-lattice indices of n
 * and its partner -n (mod N); the member with the smaller index gets -theta,
 * so the spectrum is Hermitian.  A self-conjugate mode (n = -n mod N) takes
 * the real value |k|^(-alpha/2) sign(cos theta).
 * u: uniform draws on [0,1), one per full-lattice flat index.
 * The field is c2r(F)/N scaled to unit variance; the scale is returned.
 * |k| uses the continuous wavevector with dx = 1.
 */
double orc_grf(const int64_t n[3], double alpha, const double *u, double *out)
{
    int64_t n0 = n[0], n1 = n[1], n2 = n[2], nh = n0 / 2 + 1;
    int64_t tot = n0 * n1 * n2;
    cplx *F = (cplx *)malloc(sizeof(cplx) * (size_t)(nh * n1 * n2));
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < n2; ++z)
        for (int64_t y = 0; y < n1; ++y)
            for (int64_t kx = 0; kx < nh; ++kx) {
                int64_t idx = (z * n1 + y) * nh + kx;
                if (kx == 0 && y == 0 && z == 0) {
                    F[idx] = 0;
                    continue;
                }
                int64_t px = (n0 - kx) % n0, py = (n1 - y) % n1, pz = (n2 - z) % n2;
                int64_t me = (z * n1 + y) * n0 + kx;
                int64_t partner = (pz * n1 + py) * n0 + px;
                int64_t canon = me > partner ? me : partner;
                double theta = ORC_TWO_PI * u[canon];
                double ax = ORC_TWO_PI * (double)signed_mode(kx, n0) / (double)n0;
                double ay = ORC_TWO_PI * (double)signed_mode(y, n1) / (double)n1;
                double az = ORC_TWO_PI * (double)signed_mode(z, n2) / (double)n2;
                double kk = sqrt(ax * ax + ay * ay + az * az);
                double amp = pow(kk, -0.5 * alpha);
                if (me == partner)
                    F[idx] = cos(theta) >= 0 ? amp : -amp;
                else if (me == canon)
                    F[idx] = amp * CMPLX(cos(theta), sin(theta));
                else
                    F[idx] = amp * CMPLX(cos(theta), -sin(theta));
            }
    orc_c2r3d(n, (const double *)F, out);
    double ss = 0;
    for (int64_t i = 0; i < tot; ++i) {
        out[i] /= (double)tot;
        ss += out[i] * out[i];
    }
    double scale = 1.0 / sqrt(ss / (double)tot);
    for (int64_t i = 0; i < tot; ++i) out[i] *= scale;
    free(F);
    return scale;
}
