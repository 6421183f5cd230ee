/*
 * oracle.c -- plain, slow FP64 CPU reference for the 3D real DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may use it.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * What is computed (paper, Sec. 2 "FFT implementation", problem statement):
 * the forward real-to-complex (r2c) transform of an n0 x n1 x n2 real array
 * to n0 x n1 x (n2/2+1) complex, and the complex-to-real (c2r) inverse.
 *
 * Readings where the paper is silent (it builds on FFTW, Sec. 2.2 and Sec. 3):
 *   - sign: minus in the forward transform, plus in the inverse;
 *   - no normalisation either way, so c2r(r2c(x)) = n0*n1*n2 * x;
 *   - C order, n2 fastest; complex values interleaved (re, im);
 *   - the spectrum stays in natural order n0 x n1 x H, H = n2/2+1 (integer
 *     division), offset (k0*n1 + k1)*H + k2 -- never transposed (Sec. 2.2,
 *     Fig. 4: after the transpose-free exchange the n0 data is strided);
 *   - c2r of an arbitrary half spectrum X is y = Re(IDFT3(E(X))), where E
 *     extends along k2 with E[k0,k1,n2-k2] = conj(X[-k0,-k1,k2]) for
 *     0 < k2 < n2-k2 and keeps the k2 = 0 (and, n2 even, k2 = n2/2) planes
 *     as given.  Equivalently: after the inverse n0 and n1 passes, the
 *     imaginary parts of the k2 = 0 and k2 = n2/2 bins of every row are
 *     dropped before the n2 c2r.
 *
 * Three ways to the same numbers, each written plainly:
 *   oracle_*_direct : the definition, one exponent per term (tiny sizes);
 *   oracle_*_point  : one output value from the definition, sums taken axis
 *                     by axis (O(N) per value; used to sample large outputs);
 *   oracle_r2c/c2r  : the paper's step order (Sec. 2.1 items 1 and 3, reverse
 *                     order for the inverse) with a plain recursive mixed-radix
 *                     1D FFT on each line.  Prime lengths use the naive DFT.
 *
 * Twiddles: e^{+-2 pi i e/n} with the integer e reduced mod n first, evaluated
 * with long double cosl/sinl and rounded to double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cplx;

static const long double TWO_PI_L = 6.283185307179586476925286766559005768L;

/* e^{sign * 2 pi i * e / n} */
static cplx root_of_unity(int64_t e, int64_t n, int sign)
{
    e %= n;
    if (e < 0) e += n;
    long double a = TWO_PI_L * (long double)e / (long double)n;
    cplx w;
    w.re = (double)cosl(a);
    w.im = (double)(sign * sinl(a));
    return w;
}

static cplx cmul(cplx a, cplx b)
{
    cplx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}

static int64_t smallest_prime_factor(int64_t n)
{
    for (int64_t p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

int oracle_abi_version(void) { return 1; }

/* ---------------------------------------------------------------- 1D ---- */

/* Naive DFT, the definition: out[k] = sum_j in[j] e^{sign 2 pi i jk/n}.
 * Accumulates in long double.  in/out: n interleaved complex values. */
int oracle_dft1d(int64_t n, int sign, const double* in, double* out)
{
    if (n < 1 || (sign != 1 && sign != -1) || !in || !out) return -1;
    for (int64_t k = 0; k < n; ++k) {
        long double sr = 0.0L, si = 0.0L;
        for (int64_t j = 0; j < n; ++j) {
            long double a = TWO_PI_L * (long double)((j * k) % n) / (long double)n;
            long double c = cosl(a), s = sign * sinl(a);
            long double xr = in[2 * j], xi = in[2 * j + 1];
            sr += xr * c - xi * s;
            si += xr * s + xi * c;
        }
        out[2 * k] = (double)sr;
        out[2 * k + 1] = (double)si;
    }
    return 0;
}

/* A plan for one 1D length: the table w[e] = e^{sign 2 pi i e/n}, e < n,
 * and a scratch line. */
typedef struct {
    int64_t n;
    int sign;
    cplx* w;
    cplx* tmp;
    cplx* a;
    cplx* b;
} line_fft;

static int line_fft_init(line_fft* f, int64_t n, int sign)
{
    f->n = n;
    f->sign = sign;
    f->w = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    f->tmp = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    f->a = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    f->b = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    if (!f->w || !f->tmp || !f->a || !f->b) return -1;
    for (int64_t e = 0; e < n; ++e) f->w[e] = root_of_unity(e, n, sign);
    return 0;
}

static void line_fft_free(line_fft* f)
{
    free(f->w);
    free(f->tmp);
    free(f->a);
    free(f->b);
}

/* out[k] = sum_{j<m} in[j*s] e^{sign 2 pi i jk/m} for k < m, where m divides
 * the table length N and e^{sign 2 pi i e/m} = w[e * (N/m)].
 * Decimation in time on the smallest prime factor p of m: with m = p*q,
 *   X[k] = sum_{r<p} e^{sign 2 pi i rk/m} Y_r[k mod q],
 *   Y_r  = the length-q DFT of in[r + p t], t < q.                        */
static void fft_rec(const line_fft* f, int64_t m, const cplx* in, int64_t s, cplx* out)
{
    const int64_t N = f->n;
    const int64_t step = N / m; /* index step into the table for length m */
    if (m == 1) {
        out[0] = in[0];
        return;
    }
    int64_t p = smallest_prime_factor(m);
    if (p == m) { /* prime length: naive DFT */
        for (int64_t k = 0; k < m; ++k) {
            cplx acc = {0.0, 0.0};
            for (int64_t j = 0; j < m; ++j) {
                cplx t = cmul(in[j * s], f->w[((j * k) % m) * step]);
                acc.re += t.re;
                acc.im += t.im;
            }
            out[k] = acc;
        }
        return;
    }
    int64_t q = m / p;
    for (int64_t r = 0; r < p; ++r) fft_rec(f, q, in + r * s, s * p, out + r * q);
    for (int64_t k = 0; k < m; ++k) {
        cplx acc = {0.0, 0.0};
        for (int64_t r = 0; r < p; ++r) {
            cplx t = cmul(out[r * q + (k % q)], f->w[((r * k) % m) * step]);
            acc.re += t.re;
            acc.im += t.im;
        }
        f->tmp[k] = acc;
    }
    memcpy(out, f->tmp, sizeof(cplx) * (size_t)m);
}

/* Transform the line held in f->a into f->b. */
static void line_fft_run(const line_fft* f) { fft_rec(f, f->n, f->a, 1, f->b); }

/* Recursive mixed-radix FFT of one line.  Same result as oracle_dft1d up to
 * rounding. */
int oracle_fft1d(int64_t n, int sign, const double* in, double* out)
{
    if (n < 1 || (sign != 1 && sign != -1) || !in || !out) return -1;
    line_fft f;
    if (line_fft_init(&f, n, sign)) {
        line_fft_free(&f);
        return -3;
    }
    memcpy(f.a, in, sizeof(cplx) * (size_t)n);
    line_fft_run(&f);
    memcpy(out, f.b, sizeof(cplx) * (size_t)n);
    line_fft_free(&f);
    return 0;
}

/* ------------------------------------------------- axis passes (3D) ---- */

static int set_threads(int threads)
{
#ifdef _OPENMP
    if (threads <= 0) threads = omp_get_max_threads();
    return threads;
#else
    (void)threads;
    return 1;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* In-place complex DFT of length n along the lines
 *   A[base(l) + i*stride], i < n, l < nlines,
 * with base(l) = (l / inner) * outer_stride + (l % inner). */
static int axis_pass(cplx* A, int64_t n, int sign, int64_t stride, int64_t nlines, int64_t inner,
                     int64_t outer_stride, int threads)
{
    if (n == 1) return 0;
    int err = 0;
    int nt = set_threads(threads);
#pragma omp parallel num_threads(nt) reduction(| : err)
    {
        line_fft f;
        int ok = line_fft_init(&f, n, sign) == 0;
        if (!ok) err |= 1;
        /* every thread reaches the worksharing loop, allocated or not */
#pragma omp for schedule(static)
        for (int64_t l = 0; l < nlines; ++l) {
            if (!ok) continue;
            int64_t base = (l / inner) * outer_stride + (l % inner);
            for (int64_t i = 0; i < n; ++i) f.a[i] = A[base + i * stride];
            line_fft_run(&f);
            for (int64_t i = 0; i < n; ++i) A[base + i * stride] = f.b[i];
        }
        line_fft_free(&f);
    }
    return err ? -3 : 0;
}

/* ------------------------------------------------------------- r2c ---- */

/* Forward transform, paper's step order (Sec. 2.1):
 *   step 1: 2D r2c of every n1 x n2 plane -- each n2 row (real input, bins
 *           0..n2/2 kept), then each n1 column of the plane (stride H);
 *   step 3: length-n0 c2c of every column c = k1*H + k2 of the natural-order
 *           spectrum, stride n1*H (the strided step of Sec. 2.2).
 * x: n0*n1*n2 doubles.  X: n0*n1*H interleaved complex.  threads <= 0: all. */
int oracle_r2c(int64_t n0, int64_t n1, int64_t n2, const double* x, double* Xd, int threads)
{
    if (n0 < 1 || n1 < 1 || n2 < 1 || !x || !Xd) return -1;
    const int64_t H = n2 / 2 + 1;
    const int64_t C = n1 * H;
    cplx* X = (cplx*)Xd;
    int err = 0;
    int nt = set_threads(threads);

    /* step 1a: rows along n2 */
#pragma omp parallel num_threads(nt) reduction(| : err)
    {
        line_fft f;
        int ok = line_fft_init(&f, n2, -1) == 0;
        if (!ok) err |= 1;
#pragma omp for schedule(static)
        for (int64_t row = 0; row < n0 * n1; ++row) {
            if (!ok) continue;
            for (int64_t j = 0; j < n2; ++j) {
                f.a[j].re = x[row * n2 + j];
                f.a[j].im = 0.0;
            }
            line_fft_run(&f);
            for (int64_t k = 0; k < H; ++k) X[row * H + k] = f.b[k];
        }
        line_fft_free(&f);
    }
    if (err) return -3;
    /* step 1b: n1 columns of each plane: lines (j0, k2), stride H */
    if (axis_pass(X, n1, -1, H, n0 * H, H, C, threads)) return -3;
    /* step 3: n0 columns over the flattened c = k1*H + k2, stride C */
    if (axis_pass(X, n0, -1, C, C, C, 0, threads)) return -3;
    return 0;
}

/* ------------------------------------------------------------- c2r ---- */

/* Inverse transform, the steps of oracle_r2c in reverse order (Sec. 2.1):
 * n0 columns (sign +), n1 columns (sign +), then per row the n2 c2r: the full
 * row spectrum is built with Z[0] and (n2 even) Z[n2/2] taken real and
 * Z[n2-k] = conj(Z[k]), transformed with sign +, real part kept.
 * X is not modified.  y: n0*n1*n2 doubles.
 * If max_imag is non-null it receives the largest |Im| seen in the n2 rows
 * (a consistency check: it is rounding noise). */
int oracle_c2r_ex(int64_t n0, int64_t n1, int64_t n2, const double* Xd, double* y, int threads,
                  double* max_imag)
{
    if (n0 < 1 || n1 < 1 || n2 < 1 || !Xd || !y) return -1;
    const int64_t H = n2 / 2 + 1;
    const int64_t C = n1 * H;
    const int64_t M = n0 * C;
    cplx* B = (cplx*)malloc(sizeof(cplx) * (size_t)M);
    if (!B) return -3;
    memcpy(B, Xd, sizeof(cplx) * (size_t)M);
    int err = 0;
    if (axis_pass(B, n0, +1, C, C, C, 0, threads)) err = 1;
    if (!err && axis_pass(B, n1, +1, H, n0 * H, H, C, threads)) err = 1;
    double worst = 0.0;
    if (!err) {
        int nt = set_threads(threads);
#pragma omp parallel num_threads(nt) reduction(| : err) reduction(max : worst)
        {
            line_fft f;
            int ok = line_fft_init(&f, n2, +1) == 0;
            if (!ok) err |= 1;
#pragma omp for schedule(static)
            for (int64_t row = 0; row < n0 * n1; ++row) {
                if (!ok) continue;
                const cplx* Z = B + row * H;
                for (int64_t k = 0; k < H; ++k) f.a[k] = Z[k];
                f.a[0].im = 0.0;
                if (n2 % 2 == 0) f.a[n2 / 2].im = 0.0;
                for (int64_t k = 1; k < H; ++k) {
                    if (n2 - k == k) continue;
                    f.a[n2 - k].re = Z[k].re;
                    f.a[n2 - k].im = -Z[k].im;
                }
                line_fft_run(&f);
                for (int64_t j = 0; j < n2; ++j) {
                    y[row * n2 + j] = f.b[j].re;
                    double im = fabs(f.b[j].im);
                    if (im > worst) worst = im;
                }
            }
            line_fft_free(&f);
        }
    }
    free(B);
    if (max_imag) *max_imag = worst;
    return err ? -3 : 0;
}

int oracle_c2r(int64_t n0, int64_t n1, int64_t n2, const double* Xd, double* y, int threads)
{
    return oracle_c2r_ex(n0, n1, n2, Xd, y, threads, NULL);
}

/* -------------------------------------------------- direct definitions ---- */

/* One exponent for the whole 3D phase: k.j/n as a fraction over N. */
static cplx phase3(int64_t n0, int64_t n1, int64_t n2, int64_t k0, int64_t k1, int64_t k2,
                   int64_t j0, int64_t j1, int64_t j2, int sign)
{
    const int64_t N = n0 * n1 * n2;
    int64_t e = ((k0 * j0) % n0) * (n1 * n2) + ((k1 * j1) % n1) * (n0 * n2) +
                ((k2 * j2) % n2) * (n0 * n1);
    return root_of_unity(e % N, N, sign);
}

/* r2c by the triple sum of the definition.  Tiny sizes only (O(N^2)). */
int oracle_r2c_direct(int64_t n0, int64_t n1, int64_t n2, const double* x, double* X)
{
    if (n0 < 1 || n1 < 1 || n2 < 1 || !x || !X) return -1;
    const int64_t H = n2 / 2 + 1;
    for (int64_t k0 = 0; k0 < n0; ++k0)
        for (int64_t k1 = 0; k1 < n1; ++k1)
            for (int64_t k2 = 0; k2 < H; ++k2) {
                long double sr = 0.0L, si = 0.0L;
                for (int64_t j0 = 0; j0 < n0; ++j0)
                    for (int64_t j1 = 0; j1 < n1; ++j1)
                        for (int64_t j2 = 0; j2 < n2; ++j2) {
                            cplx w = phase3(n0, n1, n2, k0, k1, k2, j0, j1, j2, -1);
                            double v = x[(j0 * n1 + j1) * n2 + j2];
                            sr += (long double)v * w.re;
                            si += (long double)v * w.im;
                        }
                int64_t o = (k0 * n1 + k1) * H + k2;
                X[2 * o] = (double)sr;
                X[2 * o + 1] = (double)si;
            }
    return 0;
}

/* c2r by the definition: build E(X) on the full n0 x n1 x n2 grid, then
 * y[j] = Re sum_k E[k] e^{+2 pi i k.j/n}.  Tiny sizes only (O(N^2)). */
int oracle_c2r_direct(int64_t n0, int64_t n1, int64_t n2, const double* X, double* y)
{
    if (n0 < 1 || n1 < 1 || n2 < 1 || !X || !y) return -1;
    const int64_t H = n2 / 2 + 1;
    const int64_t N = n0 * n1 * n2;
    cplx* E = (cplx*)malloc(sizeof(cplx) * (size_t)N);
    if (!E) return -3;
    for (int64_t k0 = 0; k0 < n0; ++k0)
        for (int64_t k1 = 0; k1 < n1; ++k1)
            for (int64_t k2 = 0; k2 < n2; ++k2) {
                cplx v;
                if (k2 < H) {
                    int64_t o = (k0 * n1 + k1) * H + k2;
                    v.re = X[2 * o];
                    v.im = X[2 * o + 1];
                } else { /* mirrored bin: conj(X[-k0, -k1, n2-k2]) */
                    int64_t m0 = (n0 - k0) % n0, m1 = (n1 - k1) % n1, m2 = n2 - k2;
                    int64_t o = (m0 * n1 + m1) * H + m2;
                    v.re = X[2 * o];
                    v.im = -X[2 * o + 1];
                }
                E[(k0 * n1 + k1) * n2 + k2] = v;
            }
    for (int64_t j0 = 0; j0 < n0; ++j0)
        for (int64_t j1 = 0; j1 < n1; ++j1)
            for (int64_t j2 = 0; j2 < n2; ++j2) {
                long double s = 0.0L;
                for (int64_t k0 = 0; k0 < n0; ++k0)
                    for (int64_t k1 = 0; k1 < n1; ++k1)
                        for (int64_t k2 = 0; k2 < n2; ++k2) {
                            cplx w = phase3(n0, n1, n2, k0, k1, k2, j0, j1, j2, +1);
                            cplx e = E[(k0 * n1 + k1) * n2 + k2];
                            s += (long double)e.re * w.re - (long double)e.im * w.im;
                        }
                y[(j0 * n1 + j1) * n2 + j2] = (double)s;
            }
    free(E);
    return 0;
}

/* -------------------------------------------------------- point values ---- */

/* One r2c output X[k0,k1,k2] from the definition, summed axis by axis:
 *   sum_j0 w0^{k0 j0} sum_j1 w1^{k1 j1} sum_j2 x[j] w2^{k2 j2},  w_a = e^{-2 pi i/n_a}.
 * O(N) work.  out: 2 doubles. */
int oracle_r2c_point(int64_t n0, int64_t n1, int64_t n2, const double* x, int64_t k0, int64_t k1,
                     int64_t k2, double* out)
{
    if (n0 < 1 || n1 < 1 || n2 < 1 || !x || !out) return -1;
    if (k0 < 0 || k0 >= n0 || k1 < 0 || k1 >= n1 || k2 < 0 || k2 > n2 / 2) return -1;
    cplx* w0 = (cplx*)malloc(sizeof(cplx) * (size_t)n0);
    cplx* w1 = (cplx*)malloc(sizeof(cplx) * (size_t)n1);
    cplx* w2 = (cplx*)malloc(sizeof(cplx) * (size_t)n2);
    if (!w0 || !w1 || !w2) {
        free(w0);
        free(w1);
        free(w2);
        return -3;
    }
    for (int64_t j = 0; j < n0; ++j) w0[j] = root_of_unity(k0 * j, n0, -1);
    for (int64_t j = 0; j < n1; ++j) w1[j] = root_of_unity(k1 * j, n1, -1);
    for (int64_t j = 0; j < n2; ++j) w2[j] = root_of_unity(k2 * j, n2, -1);
    long double tr = 0.0L, ti = 0.0L;
    for (int64_t j0 = 0; j0 < n0; ++j0) {
        long double pr = 0.0L, pi = 0.0L;
        for (int64_t j1 = 0; j1 < n1; ++j1) {
            long double rr = 0.0L, ri = 0.0L;
            const double* row = x + (j0 * n1 + j1) * n2;
            for (int64_t j2 = 0; j2 < n2; ++j2) {
                rr += (long double)row[j2] * w2[j2].re;
                ri += (long double)row[j2] * w2[j2].im;
            }
            pr += rr * w1[j1].re - ri * w1[j1].im;
            pi += rr * w1[j1].im + ri * w1[j1].re;
        }
        tr += pr * w0[j0].re - pi * w0[j0].im;
        ti += pr * w0[j0].im + pi * w0[j0].re;
    }
    free(w0);
    free(w1);
    free(w2);
    out[0] = (double)tr;
    out[1] = (double)ti;
    return 0;
}

/* One c2r output y[j0,j1,j2] from the definition written over the half
 * spectrum: y = sum_{k0,k1,k2<H} c(k2) Re(X[k] e^{+2 pi i k.j/n}), with
 * c(k2) = 1 for k2 = 0 and for k2 = n2/2 (n2 even), else 2 (the mirrored
 * bins of E contribute the complex conjugate of their partner's term).
 * O(M) work. */
int oracle_c2r_point(int64_t n0, int64_t n1, int64_t n2, const double* X, int64_t j0, int64_t j1,
                     int64_t j2, double* out)
{
    if (n0 < 1 || n1 < 1 || n2 < 1 || !X || !out) return -1;
    if (j0 < 0 || j0 >= n0 || j1 < 0 || j1 >= n1 || j2 < 0 || j2 >= n2) return -1;
    const int64_t H = n2 / 2 + 1;
    cplx* w0 = (cplx*)malloc(sizeof(cplx) * (size_t)n0);
    cplx* w1 = (cplx*)malloc(sizeof(cplx) * (size_t)n1);
    cplx* w2 = (cplx*)malloc(sizeof(cplx) * (size_t)H);
    if (!w0 || !w1 || !w2) {
        free(w0);
        free(w1);
        free(w2);
        return -3;
    }
    for (int64_t k = 0; k < n0; ++k) w0[k] = root_of_unity(k * j0, n0, +1);
    for (int64_t k = 0; k < n1; ++k) w1[k] = root_of_unity(k * j1, n1, +1);
    for (int64_t k = 0; k < H; ++k) w2[k] = root_of_unity(k * j2, n2, +1);
    long double total = 0.0L;
    for (int64_t k0 = 0; k0 < n0; ++k0) {
        for (int64_t k1 = 0; k1 < n1; ++k1) {
            cplx w01 = cmul(w0[k0], w1[k1]);
            for (int64_t k2 = 0; k2 < H; ++k2) {
                cplx w = cmul(w01, w2[k2]);
                int64_t o = (k0 * n1 + k1) * H + k2;
                long double re = (long double)X[2 * o] * w.re - (long double)X[2 * o + 1] * w.im;
                int edge = (k2 == 0) || (n2 % 2 == 0 && k2 == n2 / 2);
                total += edge ? re : 2.0L * re;
            }
        }
    }
    free(w0);
    free(w1);
    free(w2);
    out[0] = (double)total;
    return 0;
}
