/*
 * FP64 CPU oracle for the free-space FFT-convolution potential solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load.  It shares no source, header, table or helper with the HIP library;
 * the two agree only because both compute the same mathematics.
 *
 * What is computed
 * ----------------
 * The paper's benchmark (section 3, the convolution method for potential
 * fields on nested grids, with the FFT named in section 1 as the
 * performance-critical GPU operation) solves for the gravitational potential
 * of a density sampled on an N^3 mesh of spacing dx.  Its free-space
 * solution is the discrete convolution
 *
 *     phi[i] = G * dx^3 * sum_{j in [0,N)^3} K(i - j) * rho[j]
 *     K(d)   = -1 / (dx * |d|)        for d != 0   (point value of -1/r)
 *     K(0)   = -self_coeff / dx                     (the self cell; 2.38 is
 *              the cube average of 1/|r| over one cell, 3 ln(2+sqrt 3) - pi/2
 *              = 2.38008, rounded)
 *
 * with d the integer cell displacement.  Two routines compute it:
 *
 *   or_direct_sum       the definition above, term by term, O(N^6);
 *   or_fft_conv         the same sum via the convolution theorem: both
 *                       operands zero-padded to P = 2N per axis (so the
 *                       cyclic convolution of length P equals the linear one
 *                       on the cropped [0,N)^3 output), the kernel laid out
 *                       with displacement min(i, P - i) per axis, full
 *                       complex 3D DFTs (no real-to-complex, no pruning, no
 *                       symmetry tricks), pointwise product, inverse DFT
 *                       divided by P^3, real part, crop.
 *
 * The DFT is a plain recursive decimation-in-time FFT over the smallest prime
 * factor of the length (radix 2 or 3 at each level; a direct O(n^2) sum if
 * the smallest factor exceeds 3), applied axis by axis on gathered pencils.
 * Sign convention: forward uses exp(-2 pi i jk / n), inverse exp(+2 pi i jk / n),
 * neither normalised.
 *
 * All arithmetic is IEEE double.  OpenMP parallelises over output cells and
 * over pencils only; each result is computed by one thread in a fixed order,
 * so results do not depend on the thread count.
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

/* Planted-mistake builds for the tests that check the pins catch mistakes:
 * compiled with -DORACLE_MUTATION=k, one deliberate error is switched on.
 * The default build (0) has none. */
#ifndef ORACLE_MUTATION
#define ORACLE_MUTATION 0
#endif
#define MUT(k) (ORACLE_MUTATION == (k))

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_NOMEM (-2)

static const double OR_TWO_PI = 6.283185307179586476925286766559;

int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* K(d) for an integer displacement (di, dj, dk). */
double or_kernel_value(long di, long dj, long dk, double dx, double self_coeff)
{
    if (di == 0 && dj == 0 && dk == 0) return MUT(1) ? self_coeff / dx : -self_coeff / dx;
    double r2 = (double)(di * di) + (double)(dj * dj) + (double)(dk * dk);
    if (MUT(10)) return -1.0 / (dx * r2);
    return -1.0 / (dx * sqrt(r2));
}

/* ---------------------------------------------------------------------------
 * Direct summation (the definition).
 * ------------------------------------------------------------------------- */

/* Table of K over non-negative displacements [0,N)^3, index [a][b][c] =
 * K(c, b, a) in (x, y, z) order; K depends only on |d| per axis. */
static double *kernel_table(int n, double dx, double self_coeff)
{
    size_t m = (size_t)n * n * n;
    double *k = (double *)malloc(m * sizeof(double));
    if (!k) return NULL;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            for (int c = 0; c < n; ++c)
                k[((size_t)a * n + b) * n + c] = or_kernel_value(c, b, a, dx, self_coeff);
    return k;
}

/* One output cell.  Each x-row of terms is summed directly; the N^2 row sums
 * are combined with Neumaier's compensated summation so the rounding error
 * of the O(N^3)-term sum stays near that of one row. */
static double direct_one(int n, const double *ktab, const double *rho, int iz, int iy, int ix)
{
    double sum = 0.0, comp = 0.0;
    for (int jz = 0; jz < n; ++jz) {
        const int az = abs(iz - jz);
        for (int jy = 0; jy < n; ++jy) {
            const int ay = abs(iy - jy);
            const double *kr = ktab + ((size_t)az * n + ay) * n;
            const double *rr = rho + ((size_t)jz * n + jy) * n;
            double row = 0.0;
            for (int jx = 0; jx < n; ++jx) {
                if (MUT(6) && az == 0 && ay == 0 && jx == ix) continue;
                row += kr[abs(ix - jx)] * rr[jx];
            }
            const double t = sum + row;
            if (fabs(sum) >= fabs(row)) comp += (sum - t) + row;
            else comp += (row - t) + sum;
            sum = t;
        }
    }
    return sum + comp;
}

/* phi = G dx^3 sum_j K(i-j) rho[j] on all N^3 cells.  rho, phi: [z][y][x]. */
int or_direct_sum(int n, double dx, double g, double self_coeff, const double *rho, double *phi)
{
    if (n <= 0 || dx <= 0.0 || !rho || !phi) return OR_ERR_ARG;
    double *ktab = kernel_table(n, dx, self_coeff);
    if (!ktab) return OR_ERR_NOMEM;
    const double scale = g * dx * dx * dx;
    const long m = (long)n * n * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (long c = 0; c < m; ++c) {
        int iz = (int)(c / ((long)n * n)), iy = (int)((c / n) % n), ix = (int)(c % n);
        phi[c] = scale * direct_one(n, ktab, rho, iz, iy, ix);
    }
    free(ktab);
    return OR_OK;
}

/* The definition at a list of cells.  cells: ncells triples (z, y, x). */
int or_direct_sum_cells(int n, double dx, double g, double self_coeff, const double *rho,
                        int ncells, const int *cells, double *out)
{
    if (n <= 0 || dx <= 0.0 || !rho || !out || ncells < 0 || (ncells > 0 && !cells)) return OR_ERR_ARG;
    for (int c = 0; c < ncells; ++c)
        for (int a = 0; a < 3; ++a)
            if (cells[3 * c + a] < 0 || cells[3 * c + a] >= n) return OR_ERR_ARG;
    double *ktab = kernel_table(n, dx, self_coeff);
    if (!ktab) return OR_ERR_NOMEM;
    const double scale = g * dx * dx * dx;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncells; ++c)
        out[c] = scale * direct_one(n, ktab, rho, cells[3 * c], cells[3 * c + 1], cells[3 * c + 2]);
    free(ktab);
    return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Recursive FFT.
 * ------------------------------------------------------------------------- */

static int smallest_factor(int n)
{
    if (n % 2 == 0) return 2;
    for (int p = 3; (long)p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* exp(sign * 2 pi i * e / len) for e in [0, len). */
static cplx *twiddle_table(int len, int sign)
{
    cplx *t = (cplx *)malloc((size_t)len * sizeof(cplx));
    if (!t) return NULL;
    for (int e = 0; e < len; ++e) {
        double a = OR_TWO_PI * (double)e / (double)len;
        t[e] = cos(a) + (double)sign * sin(a) * I;
    }
    return t;
}

/* out[k] = sum_{j<n} in[j*stride] * w_n^(j k), w_n = exp(sign 2 pi i / n).
 * tw holds exp(sign 2 pi i e / len) for the top-level length len, which n
 * divides, so w_n^e = tw[(e mod n) * (len / n)].  scratch holds >= n values
 * and is only used after the sub-transforms have returned. */
static void fft_rec(int n, const cplx *in, long stride, cplx *out, cplx *scratch,
                    const cplx *tw, int len)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const long step = len / n;
    const int p = smallest_factor(n);
    if (p > 3) {
        for (int k = 0; k < n; ++k) {
            cplx acc = 0.0;
            for (int j = 0; j < n; ++j) acc += in[j * stride] * tw[(((long)j * k) % n) * step];
            scratch[k] = acc;
        }
        memcpy(out, scratch, (size_t)n * sizeof(cplx));
        return;
    }
    const int m = n / p;
    /* sub-sequence q holds in[(p j + q) * stride], j < m; its DFT goes to out[q m ...] */
    for (int q = 0; q < p; ++q) fft_rec(m, in + q * stride, stride * p, out + (long)q * m, scratch, tw, len);
    /* X[k + s m] = sum_q w_n^(q (k + s m)) Y_q[k] */
    for (int k = 0; k < m; ++k)
        for (int s = 0; s < p; ++s) {
            const long kk = k + (long)s * m;
            cplx acc = 0.0;
            for (int q = 0; q < p; ++q) {
                long e = ((long)q * (MUT(9) ? k : kk)) % n;
                if (MUT(3) && p == 2) e = (n - e) % n;
                acc += out[(long)q * m + k] * tw[e * step];
            }
            scratch[kk] = acc;
        }
    memcpy(out, scratch, (size_t)n * sizeof(cplx));
}

/* One-dimensional DFT of n complex values (interleaved re, im). */
int or_fft(int n, const double *in, double *out, int sign)
{
    if (n <= 0 || !in || !out || (sign != 1 && sign != -1)) return OR_ERR_ARG;
    cplx *tw = twiddle_table(n, sign);
    cplx *buf = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *res = (cplx *)malloc((size_t)n * sizeof(cplx));
    cplx *scr = (cplx *)malloc((size_t)n * sizeof(cplx));
    if (!tw || !buf || !res || !scr) {
        free(tw); free(buf); free(res); free(scr);
        return OR_ERR_NOMEM;
    }
    memcpy(buf, in, (size_t)n * sizeof(cplx));
    fft_rec(n, buf, 1, res, scr, tw, n);
    memcpy(out, res, (size_t)n * sizeof(cplx));
    free(tw); free(buf); free(res); free(scr);
    return OR_OK;
}

/* Cubic DFT of side p on a[z][y][x] (complex, in place), one axis at a time:
 * every pencil is gathered into a contiguous buffer, transformed, scattered. */
static int fft3_inplace(int p, cplx *a, int sign)
{
    cplx *tw = twiddle_table(p, sign);
    if (!tw) return OR_ERR_NOMEM;
    const long pp = (long)p * p;
    int err = 0;
    for (int axis = 0; axis < (MUT(7) ? 2 : 3); ++axis) {
        const long stride = axis == 0 ? 1 : (axis == 1 ? p : pp);
#pragma omp parallel
        {
            cplx *g = (cplx *)malloc((size_t)p * sizeof(cplx));
            cplx *r = (cplx *)malloc((size_t)p * sizeof(cplx));
            cplx *s = (cplx *)malloc((size_t)p * sizeof(cplx));
            if (!g || !r || !s) {
#pragma omp atomic write
                err = 1;
            } else {
#pragma omp for schedule(static)
                for (long q = 0; q < pp; ++q) {
                    /* pencil q: the two other coordinates */
                    const long hi = q / p, lo = q % p;
                    long base;
                    if (axis == 0) base = hi * pp + lo * p;       /* (z, y) */
                    else if (axis == 1) base = hi * pp + lo;      /* (z, x) */
                    else base = hi * p + lo;                      /* (y, x) */
                    for (int t = 0; t < p; ++t) g[t] = a[base + t * stride];
                    fft_rec(p, g, 1, r, s, tw, p);
                    for (int t = 0; t < p; ++t) a[base + t * stride] = r[t];
                }
            }
            free(g); free(r); free(s);
        }
        if (err) break;
    }
    free(tw);
    return err ? OR_ERR_NOMEM : OR_OK;
}

/* Cubic DFT of side p, interleaved complex in place. */
int or_fft3(int p, double *data, int sign)
{
    if (p <= 0 || !data || (sign != 1 && sign != -1)) return OR_ERR_ARG;
    return fft3_inplace(p, (cplx *)data, sign);
}

/* The padded kernel: kpad[z][y][x] = K(min(x,P-x), min(y,P-y), min(z,P-z)),
 * P = 2N.  Index N (displacement +-N) never reaches the cropped output. */
int or_kernel_pad(int n, double dx, double self_coeff, double *kpad)
{
    if (n <= 0 || dx <= 0.0 || !kpad) return OR_ERR_ARG;
    const int p = 2 * n;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < p; ++z)
        for (long y = 0; y < p; ++y)
            for (long x = 0; x < p; ++x) {
                const long w = MUT(2) ? p - 1 : p;
                const long dz = z < p - z ? z : w - z, dy = y < p - y ? y : w - y, dxx = x < p - x ? x : w - x;
                kpad[(z * p + y) * p + x] = or_kernel_value(dxx, dy, dz, dx, self_coeff);
            }
    return OR_OK;
}

/* Transformed kernel: ghat = forward DFT of kpad, full P^3 complex. */
int or_green_hat(int n, double dx, double self_coeff, double *ghat)
{
    if (n <= 0 || dx <= 0.0 || !ghat) return OR_ERR_ARG;
    const int p = 2 * n;
    const long m = (long)p * p * p;
    double *k = (double *)malloc((size_t)m * sizeof(double));
    if (!k) return OR_ERR_NOMEM;
    int rc = or_kernel_pad(n, dx, self_coeff, k);
    cplx *g = (cplx *)ghat;
    for (long i = 0; i < m; ++i) g[i] = k[i];
    free(k);
    if (rc) return rc;
    return fft3_inplace(p, g, -1);
}

/* Convolution theorem with a caller-supplied padded kernel kpad (P^3 real,
 * P = 2N): phi = G dx^3 Re(IDFT(DFT(rho_pad) * DFT(kpad)) / P^3)[0,N)^3. */
int or_fft_conv_kernel(int n, double dx, double g, const double *kpad, const double *rho, double *phi)
{
    if (n <= 0 || dx <= 0.0 || !kpad || !rho || !phi) return OR_ERR_ARG;
    const int p = 2 * n;
    const long m = (long)p * p * p;
    cplx *a = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *k = (cplx *)malloc((size_t)m * sizeof(cplx));
    if (!a || !k) {
        free(a); free(k);
        return OR_ERR_NOMEM;
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < m; ++i) k[i] = kpad[i];
#pragma omp parallel for schedule(static)
    for (long z = 0; z < n; ++z)
        for (long y = 0; y < n; ++y)
            for (long x = 0; x < n; ++x) a[(z * p + y) * p + x] = rho[(z * n + y) * n + x];
    int rc = fft3_inplace(p, k, -1);
    if (!rc) rc = fft3_inplace(p, a, -1);
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) a[i] *= k[i];
        rc = fft3_inplace(p, a, +1);
    }
    if (!rc) {
        double scale = g * dx * dx * dx / (double)m;
        if (MUT(4)) scale = g * dx * dx * dx;
        if (MUT(5)) scale = g * dx * dx / (double)m;
#pragma omp parallel for schedule(static)
        for (long z = 0; z < n; ++z)
            for (long y = 0; y < n; ++y)
                for (long x = 0; x < n; ++x)
                    phi[(z * n + y) * n + x] = scale * creal(a[(z * p + y) * p + x + (MUT(8) ? 1 : 0)]);
    }
    free(a);
    free(k);
    return rc;
}

/* The FFT-convolution solve with the standard padded kernel. */
int or_fft_conv(int n, double dx, double g, double self_coeff, const double *rho, double *phi)
{
    if (n <= 0 || dx <= 0.0 || !rho || !phi) return OR_ERR_ARG;
    const int p = 2 * n;
    const long m = (long)p * p * p;
    double *k = (double *)malloc((size_t)m * sizeof(double));
    if (!k) return OR_ERR_NOMEM;
    int rc = or_kernel_pad(n, dx, self_coeff, k);
    if (!rc) rc = or_fft_conv_kernel(n, dx, g, k, rho, phi);
    free(k);
    return rc;
}
