/* Exercise of the FP64 oracle (oracle/lf2_oracle.c) on small lattices of
 * every kind it handles -- powers of two, radix 3 and 5, odd primes, extents
 * of 1 -- for a build under AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py).  Each step checks a property that holds
 * exactly up to rounding: the 1-D FFT against the O(N^2) DFT, r2c against
 * c2c, round trips, the Poisson residual of one Fourier mode, the sum of
 * the power-spectrum counts.  Exit status 0 when every check passes. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_dft1d(int64_t n, const double *in, double *out, int sign);
void orc_fft1d(int64_t n, double *data, int sign);
void orc_c2c3d(const int64_t n[3], const double *in, double *out, int sign);
void orc_r2c3d(const int64_t n[3], const double *in, double *out);
void orc_c2r3d(const int64_t n[3], const double *in, double *out);
void orc_dft3d_at(const int64_t n[3], const double *f, int is_complex, const int64_t k[3],
                  int sign, double out[2]);
void orc_poisson(const int64_t n[3], double dx, int k2mode, const double *rho, double *phi);
int64_t orc_pk_qmax(const int64_t n[3]);
void orc_power_spectrum(const int64_t n[3], int half, const double *Fin, int64_t nbins, double dx,
                        double *pk, double *kmean, double *count);

static int failures = 0;

static void expect(int ok, const char *what, double v)
{
    if (!ok) {
        printf("FAIL %s: %.3e\n", what, v);
        ++failures;
    }
}

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static void lines(void)
{
    static const int64_t lens[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 12, 13, 15, 16, 25, 30, 45, 64, 97};
    uint64_t s = 1;
    for (size_t i = 0; i < sizeof(lens) / sizeof(lens[0]); ++i) {
        int64_t n = lens[i];
        double *x = malloc(sizeof(double) * 2 * n), *y = malloc(sizeof(double) * 2 * n);
        for (int64_t j = 0; j < 2 * n; ++j) x[j] = urand(&s);
        orc_dft1d(n, x, y, -1);
        double *f = malloc(sizeof(double) * 2 * n);
        memcpy(f, x, sizeof(double) * 2 * n);
        orc_fft1d(n, f, -1);
        double e = 0.0;
        for (int64_t j = 0; j < 2 * n; ++j) e = fmax(e, fabs(f[j] - y[j]));
        expect(e <= 1e-12 * n, "fft1d against dft1d", e);
        orc_fft1d(n, f, +1);
        e = 0.0;
        for (int64_t j = 0; j < 2 * n; ++j) e = fmax(e, fabs(f[j] / (double)n - x[j]));
        expect(e <= 1e-13 * n, "fft1d round trip", e);
        free(x);
        free(y);
        free(f);
    }
}

static void lattice(int64_t n0, int64_t n1, int64_t n2)
{
    const int64_t n[3] = {n0, n1, n2};
    const int64_t tot = n0 * n1 * n2, nh = n0 / 2 + 1;
    uint64_t s = (uint64_t)(n0 * 131 + n1 * 17 + n2);
    double *f = malloc(sizeof(double) * tot), *fc = calloc(2 * tot, sizeof(double));
    double *F = malloc(sizeof(double) * 2 * tot), *H = malloc(sizeof(double) * 2 * nh * n1 * n2);
    double *b = malloc(sizeof(double) * tot);
    for (int64_t i = 0; i < tot; ++i) fc[2 * i] = f[i] = urand(&s);
    orc_c2c3d(n, fc, F, -1);
    orc_r2c3d(n, f, H);
    double e = 0.0, m = 0.0;
    for (int64_t z = 0; z < n2; ++z)
        for (int64_t y = 0; y < n1; ++y)
            for (int64_t k = 0; k < nh; ++k)
                for (int c = 0; c < 2; ++c) {
                    double a = H[2 * ((z * n1 + y) * nh + k) + c], r = F[2 * ((z * n1 + y) * n0 + k) + c];
                    e = fmax(e, fabs(a - r));
                    m = fmax(m, fabs(r));
                }
    expect(e <= 1e-12 * (m + 1.0), "r2c against c2c", e);
    const int64_t kk[3] = {n0 / 3, n1 - 1, n2 / 2};
    double at[2];
    orc_dft3d_at(n, f, 0, kk, -1, at);
    const double *r = F + 2 * ((kk[2] * n1 + kk[1]) * n0 + kk[0]);
    expect(fabs(at[0] - r[0]) + fabs(at[1] - r[1]) <= 1e-11 * (m + 1.0), "dft3d_at against c2c",
           fabs(at[0] - r[0]));
    orc_c2r3d(n, H, b);
    e = 0.0;
    for (int64_t i = 0; i < tot; ++i) e = fmax(e, fabs(b[i] / (double)tot - f[i]));
    expect(e <= 1e-12, "r2c / c2r round trip", e);
    /* one Fourier mode along dimension 0 (when it has one): phi = -rho / k^2 */
    if (n0 > 2) {
        for (int k2mode = 0; k2mode < 2; ++k2mode) {
            for (int64_t i = 0; i < tot; ++i) f[i] = cos(2.0 * M_PI * (double)(i % n0) / (double)n0);
            orc_poisson(n, 0.5, k2mode, f, b);
            double k2 = k2mode ? 16.0 * pow(sin(M_PI / (double)n0), 2.0)
                               : pow(2.0 * M_PI / ((double)n0 * 0.5), 2.0);
            e = 0.0;
            for (int64_t i = 0; i < tot; ++i) e = fmax(e, fabs(b[i] + f[i] / k2));
            expect(e <= 1e-12 / k2, "one-mode Poisson", e);
        }
    }
    /* power spectrum: the counts add up to every mode but k = 0 */
    const int64_t nb = 7;
    double pk[7], km[7], ct[7];
    for (int half = 0; half < 2; ++half) {
        orc_power_spectrum(n, half, half ? H : F, nb, 1.0, pk, km, ct);
        double sum = 0.0;
        for (int64_t i = 0; i < nb; ++i) sum += ct[i];
        expect(fabs(sum - (double)(tot - 1)) < 0.5 || orc_pk_qmax(n) == 0, "bin counts", sum);
    }
    free(f);
    free(fc);
    free(F);
    free(H);
    free(b);
}

int main(void)
{
    lines();
    static const int64_t shapes[][3] = {{8, 6, 5}, {9, 4, 3}, {7, 1, 1}, {1, 1, 1}, {16, 16, 16},
                                        {15, 10, 6}, {2, 2, 2}, {11, 13, 2}};
    for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i)
        lattice(shapes[i][0], shapes[i][1], shapes[i][2]);
    printf("oracle checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
