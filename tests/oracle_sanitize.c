/* oracle_sanitize.c -- runs every entry point of oracle/oracle.c on small
 * shapes under AddressSanitizer + UndefinedBehaviorSanitizer (test
 * infrastructure; built with gcc by tests/test_sanitizers.py).  Besides the
 * sanitizers' own checks it asserts two facts of the oracle's arithmetic so
 * that the calls are not optimised away: the line FFT equals the naive DFT,
 * and c2r(r2c(x)) = N x.  Prints "ok oracle" and exits 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dft1d(int64_t n, int sign, const double* in, double* out);
int oracle_fft1d(int64_t n, int sign, const double* in, double* out);
int oracle_r2c(int64_t n0, int64_t n1, int64_t n2, const double* x, double* X, int threads);
int oracle_c2r(int64_t n0, int64_t n1, int64_t n2, const double* X, double* y, int threads);
int oracle_c2r_ex(int64_t n0, int64_t n1, int64_t n2, const double* X, double* y, int threads, double* max_imag);
int oracle_r2c_direct(int64_t n0, int64_t n1, int64_t n2, const double* x, double* X);
int oracle_c2r_direct(int64_t n0, int64_t n1, int64_t n2, const double* X, double* y);
int oracle_r2c_point(int64_t n0, int64_t n1, int64_t n2, const double* x, int64_t k0, int64_t k1, int64_t k2,
                     double* out);
int oracle_c2r_point(int64_t n0, int64_t n1, int64_t n2, const double* X, int64_t j0, int64_t j1, int64_t j2,
                     double* out);
int oracle_max_threads(void);

static uint64_t g_s = 7;
static double uni(void)
{
    g_s = g_s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int fail(const char* what)
{
    fprintf(stderr, "FAIL: %s\n", what);
    return 1;
}

int main(void)
{
    /* 1D: every length up to 130 and a few larger mixed and prime ones */
    int64_t lens[160];
    int nl = 0;
    for (int64_t n = 1; n <= 130; ++n) lens[nl++] = n;
    const int64_t more[] = {243, 256, 343, 625, 1024, 1031, 1536, 2401};
    for (int i = 0; i < 8; ++i) lens[nl++] = more[i];
    for (int i = 0; i < nl; ++i) {
        const int64_t n = lens[i];
        double* a = malloc(sizeof(double) * 2 * n);
        double* b = malloc(sizeof(double) * 2 * n);
        double* c = malloc(sizeof(double) * 2 * n);
        for (int64_t k = 0; k < 2 * n; ++k) a[k] = uni();
        for (int sign = -1; sign <= 1; sign += 2) {
            if (oracle_fft1d(n, sign, a, b) || oracle_dft1d(n, sign, a, c)) return fail("1D call");
            double e = 0, r = 0;
            for (int64_t k = 0; k < 2 * n; ++k) {
                e += (b[k] - c[k]) * (b[k] - c[k]);
                r += c[k] * c[k];
            }
            if (sqrt(e / r) > 1e-13) return fail("line FFT against the naive DFT");
        }
        free(a);
        free(b);
        free(c);
    }
    /* 3D on small odd and even shapes, one thread and all threads */
    const int64_t shapes[][3] = {{1, 1, 1}, {1, 1, 2}, {2, 3, 4}, {3, 5, 7}, {4, 6, 8}, {5, 1, 9}, {8, 8, 8}, {6, 10, 15}};
    for (int s = 0; s < 8; ++s) {
        const int64_t n0 = shapes[s][0], n1 = shapes[s][1], n2 = shapes[s][2], h = n2 / 2 + 1;
        const int64_t N = n0 * n1 * n2, M = n0 * n1 * h;
        double* x = malloc(sizeof(double) * N);
        double* y = malloc(sizeof(double) * N);
        double* yd = malloc(sizeof(double) * N);
        double* X = malloc(sizeof(double) * 2 * M);
        double* Xd = malloc(sizeof(double) * 2 * M);
        for (int64_t k = 0; k < N; ++k) x[k] = uni();
        for (int th = 1; th >= 0; --th) {
            if (oracle_r2c(n0, n1, n2, x, X, th) || oracle_c2r(n0, n1, n2, X, y, th)) return fail("3D call");
            double mi = 0;
            if (oracle_c2r_ex(n0, n1, n2, X, y, th, &mi)) return fail("c2r_ex");
            double e = 0, r = 0;
            for (int64_t k = 0; k < N; ++k) {
                e += (y[k] - N * x[k]) * (y[k] - N * x[k]);
                r += (N * x[k]) * (N * x[k]);
            }
            if (sqrt(e / r) > 1e-13) return fail("round trip");
        }
        if (oracle_r2c_direct(n0, n1, n2, x, Xd) || oracle_c2r_direct(n0, n1, n2, X, yd)) return fail("direct");
        double pt[2];
        for (int64_t k0 = 0; k0 < n0; ++k0)
            for (int64_t k2 = 0; k2 < h; ++k2) {
                if (oracle_r2c_point(n0, n1, n2, x, k0, n1 - 1, k2, pt)) return fail("r2c point");
                if (oracle_c2r_point(n0, n1, n2, X, k0, n1 / 2, k2, pt)) return fail("c2r point");
            }
        free(x);
        free(y);
        free(yd);
        free(X);
        free(Xd);
    }
    if (oracle_max_threads() < 1) return fail("threads");
    puts("ok oracle");
    return 0;
}
