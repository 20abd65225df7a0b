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
 * Boxes of nx x ny x nz cells (the "_box" routines: or_direct_sum_box,
 * or_direct_sum_cells_box, or_kernel_pad_box, or_fft3_box, or_fft_conv_box)
 * take the same definition with one length per axis; the convolution pads
 * each axis to twice its own length.
 *
 * Cells with spacings dx, dy, dz along x, y, z (the "3" routines): the
 * displacement length is |(di dx, dj dy, dk dz)|, the volume factor dx dy dz,
 * and the self cell takes the cell average of 1/|r| over the dx x dy x dz
 * box (closed form below) scaled by self_coeff / (3 ln(2 + sqrt 3) - pi/2),
 * the factor that turns the exact unit-cube average into self_coeff; a cube
 * gets exactly -self_coeff/dx.  (The paper's cells are cubes; this reading
 * extends its self-cell value to boxes.)
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

/* phi = gv Re(IDFT(DFT(rho_pad) * DFT(kpad)) / P^3)[0,N)^3, gv = G times the
 * cell volume (each caller forms it). */
static int conv_core(int n, double gv, const double *kpad, const double *rho, double *phi);

/* Convolution theorem with a caller-supplied padded kernel kpad (P^3 real,
 * P = 2N): phi = G dx^3 Re(IDFT(DFT(rho_pad) * DFT(kpad)) / P^3)[0,N)^3. */
int or_fft_conv_kernel(int n, double dx, double g, const double *kpad, const double *rho, double *phi)
{
    if (n <= 0 || dx <= 0.0 || !kpad || !rho || !phi) return OR_ERR_ARG;
    double gv = g * dx * dx * dx;
    if (MUT(5)) gv = g * dx * dx;
    return conv_core(n, gv, kpad, rho, phi);
}

static int conv_core(int n, double gv, const double *kpad, const double *rho, double *phi)
{
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
        double scale = gv / (double)m;
        if (MUT(4)) scale = gv;
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

/* ---------------------------------------------------------------------------
 * Cells with spacings dx, dy, dz.
 * ------------------------------------------------------------------------- */

/* Integral of 1/|r| over the box [0,a] x [0,b] x [0,c], a, b, c > 0:
 *   bc asinh(a / sqrt(b^2+c^2)) + ca asinh(b / sqrt(c^2+a^2)) + ab asinh(c / sqrt(a^2+b^2))
 *   - a^2/2 atan(bc / (a r)) - b^2/2 atan(ca / (b r)) - c^2/2 atan(ab / (c r)),
 * r = sqrt(a^2 + b^2 + c^2) (integrate 1/r along one axis, then the other two). */
static double inv_r_box(double a, double b, double c)
{
    const double r = sqrt(a * a + b * b + c * c);
    return b * c * asinh(a / hypot(b, c)) + c * a * asinh(b / hypot(c, a)) + a * b * asinh(c / hypot(a, b)) -
           0.5 * a * a * atan(b * c / (a * r)) - 0.5 * b * b * atan(c * a / (b * r)) -
           0.5 * c * c * atan(a * b / (c * r));
}

/* Average of 1/|r| over a dx x dy x dz cell centred on the origin (eight octants). */
double or_cell_average_inv_r(double dx, double dy, double dz)
{
    if (!(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0)) return NAN;
    return 8.0 * inv_r_box(0.5 * dx, 0.5 * dy, 0.5 * dz) / (dx * dy * dz);
}

/* K(d) for an integer displacement (di, dj, dk) on cells dx x dy x dz. */
double or_kernel_value3(long di, long dj, long dk, double dx, double dy, double dz, double self_coeff)
{
    if (di == 0 && dj == 0 && dk == 0) {
        if ((dx == dy && dy == dz) || MUT(11)) return -self_coeff / dx;
        const double unit_cube = 3.0 * log(2.0 + sqrt(3.0)) - 2.0 * atan(1.0);  /* 3 ln(2 + sqrt 3) - pi/2 */
        return -(self_coeff / unit_cube) * or_cell_average_inv_r(dx, dy, dz);
    }
    const double x = (double)di * dx, y = (double)dj * (MUT(12) ? dz : dy), z = (double)dk * (MUT(12) ? dy : dz);
    return -1.0 / sqrt(x * x + y * y + z * z);
}

static double *kernel_table3(int n, double dx, double dy, double dz, double self_coeff)
{
    size_t m = (size_t)n * n * n;
    double *k = (double *)malloc(m * sizeof(double));
    if (!k) return NULL;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            for (int c = 0; c < n; ++c)
                k[((size_t)a * n + b) * n + c] = or_kernel_value3(c, b, a, dx, dy, dz, self_coeff);
    return k;
}

static int bad_spacing(double dx, double dy, double dz) { return !(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0); }

/* phi = G dx dy dz sum_j K(i-j) rho[j] on all N^3 cells. */
int or_direct_sum3(int n, double dx, double dy, double dz, double g, double self_coeff, const double *rho,
                   double *phi)
{
    if (n <= 0 || bad_spacing(dx, dy, dz) || !rho || !phi) return OR_ERR_ARG;
    double *ktab = kernel_table3(n, dx, dy, dz, self_coeff);
    if (!ktab) return OR_ERR_NOMEM;
    const double scale = g * dx * dy * dz;
    const long m = (long)n * n * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (long c = 0; c < m; ++c) {
        int iz = (int)(c / ((long)n * n)), iy = (int)((c / n) % n), ix = (int)(c % n);
        phi[c] = scale * direct_one(n, ktab, rho, iz, iy, ix);
    }
    free(ktab);
    return OR_OK;
}

int or_direct_sum_cells3(int n, double dx, double dy, double dz, double g, double self_coeff, const double *rho,
                         int ncells, const int *cells, double *out)
{
    if (n <= 0 || bad_spacing(dx, dy, dz) || !rho || !out || ncells < 0 || (ncells > 0 && !cells)) return OR_ERR_ARG;
    for (int c = 0; c < ncells; ++c)
        for (int a = 0; a < 3; ++a)
            if (cells[3 * c + a] < 0 || cells[3 * c + a] >= n) return OR_ERR_ARG;
    double *ktab = kernel_table3(n, dx, dy, dz, self_coeff);
    if (!ktab) return OR_ERR_NOMEM;
    const double scale = g * dx * dy * dz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncells; ++c)
        out[c] = scale * direct_one(n, ktab, rho, cells[3 * c], cells[3 * c + 1], cells[3 * c + 2]);
    free(ktab);
    return OR_OK;
}

/* kpad[z][y][x] = K(min(x,P-x), min(y,P-y), min(z,P-z)) on dx x dy x dz cells. */
int or_kernel_pad3(int n, double dx, double dy, double dz, double self_coeff, double *kpad)
{
    if (n <= 0 || bad_spacing(dx, dy, dz) || !kpad) return OR_ERR_ARG;
    const int p = 2 * n;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < p; ++z)
        for (long y = 0; y < p; ++y)
            for (long x = 0; x < p; ++x) {
                const long az = z < p - z ? z : p - z, ay = y < p - y ? y : p - y, ax = x < p - x ? x : p - x;
                kpad[(z * p + y) * p + x] = or_kernel_value3(ax, ay, az, dx, dy, dz, self_coeff);
            }
    return OR_OK;
}

/* The FFT-convolution solve on dx x dy x dz cells. */
int or_fft_conv3(int n, double dx, double dy, double dz, double g, double self_coeff, const double *rho,
                 double *phi)
{
    if (n <= 0 || bad_spacing(dx, dy, dz) || !rho || !phi) return OR_ERR_ARG;
    const int p = 2 * n;
    const long m = (long)p * p * p;
    double *k = (double *)malloc((size_t)m * sizeof(double));
    if (!k) return OR_ERR_NOMEM;
    int rc = or_kernel_pad3(n, dx, dy, dz, self_coeff, k);
    if (!rc) rc = conv_core(n, MUT(13) ? g * dx * dx * dx : g * dx * dy * dz, k, rho, phi);
    free(k);
    return rc;
}

/* ---------------------------------------------------------------------------
 * Boxes of nx x ny x nz cells (x, y, z) with spacings dx, dy, dz: the same
 * definition with a separate length per axis, and the convolution theorem
 * with each axis padded to twice its own length.
 * ------------------------------------------------------------------------- */

static int bad_box(int nx, int ny, int nz) { return nx <= 0 || ny <= 0 || nz <= 0; }

/* Table of K over non-negative displacements, index [az][ay][ax]. */
static double *kernel_table_box(int nx, int ny, int nz, double dx, double dy, double dz, double self_coeff)
{
    double *k = (double *)malloc((size_t)nx * ny * nz * sizeof(double));
    if (!k) return NULL;
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < ny; ++b)
            for (int c = 0; c < nx; ++c)
                k[((size_t)a * ny + b) * nx + c] = or_kernel_value3(c, b, a, dx, dy, dz, self_coeff);
    return k;
}

/* One output cell of the box sum: x-rows summed directly, row sums combined
 * with Neumaier's compensated summation (as direct_one). */
static double direct_one_box(int nx, int ny, int nz, const double *ktab, const double *rho, int iz, int iy, int ix)
{
    double sum = 0.0, comp = 0.0;
    for (int jz = 0; jz < nz; ++jz) {
        const int az = abs(iz - jz);
        for (int jy = 0; jy < ny; ++jy) {
            const int ay = abs(iy - jy);
            const double *kr = ktab + ((size_t)az * ny + ay) * nx;
            const double *rr = rho + ((size_t)jz * ny + jy) * nx;
            double row = 0.0;
            for (int jx = 0; jx < nx; ++jx) row += kr[abs(ix - jx)] * rr[jx];
            const double t = sum + row;
            if (fabs(sum) >= fabs(row)) comp += (sum - t) + row;
            else comp += (row - t) + sum;
            sum = t;
        }
    }
    return sum + comp;
}

/* phi = G dx dy dz sum_j K(i-j) rho[j] on all cells of the box; rho, phi: [z][y][x]. */
int or_direct_sum_box(int nx, int ny, int nz, double dx, double dy, double dz, double g, double self_coeff,
                      const double *rho, double *phi)
{
    if (bad_box(nx, ny, nz) || bad_spacing(dx, dy, dz) || !rho || !phi) return OR_ERR_ARG;
    double *ktab = kernel_table_box(nx, ny, nz, dx, dy, dz, self_coeff);
    if (!ktab) return OR_ERR_NOMEM;
    const double scale = g * dx * dy * dz;
    const long m = (long)nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 16)
    for (long c = 0; c < m; ++c) {
        const int iz = (int)(c / ((long)nx * ny)), iy = (int)((c / nx) % ny), ix = (int)(c % nx);
        phi[c] = scale * direct_one_box(nx, ny, nz, ktab, rho, iz, iy, ix);
    }
    free(ktab);
    return OR_OK;
}

/* The box sum at a list of cells (z, y, x). */
int or_direct_sum_cells_box(int nx, int ny, int nz, double dx, double dy, double dz, double g, double self_coeff,
                            const double *rho, int ncells, const int *cells, double *out)
{
    if (bad_box(nx, ny, nz) || bad_spacing(dx, dy, dz) || !rho || !out || ncells < 0 || (ncells > 0 && !cells))
        return OR_ERR_ARG;
    for (int c = 0; c < ncells; ++c)
        if (cells[3 * c] < 0 || cells[3 * c] >= nz || cells[3 * c + 1] < 0 || cells[3 * c + 1] >= ny ||
            cells[3 * c + 2] < 0 || cells[3 * c + 2] >= nx)
            return OR_ERR_ARG;
    double *ktab = kernel_table_box(nx, ny, nz, dx, dy, dz, self_coeff);
    if (!ktab) return OR_ERR_NOMEM;
    const double scale = g * dx * dy * dz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncells; ++c)
        out[c] = scale * direct_one_box(nx, ny, nz, ktab, rho, cells[3 * c], cells[3 * c + 1], cells[3 * c + 2]);
    free(ktab);
    return OR_OK;
}

/* DFT of a px x py x pz box a[z][y][x] (complex, in place), one axis at a
 * time on gathered pencils, each axis with its own length. */
static int fft3_box_inplace(int px, int py, int pz, cplx *a, int sign)
{
    const int len[3] = {px, py, pz};
    const long stride[3] = {1, px, (long)px * py};
    int err = 0;
    for (int axis = 0; axis < 3 && !err; ++axis) {
        const int L = len[axis];
        cplx *tw = twiddle_table(L, sign);
        if (!tw) return OR_ERR_NOMEM;
        /* the two other axes, o1 the faster one */
        const int o1 = axis == 0 ? 1 : 0, o2 = axis == 2 ? 1 : 2;
        const long npen = (long)len[o1] * len[o2];
#pragma omp parallel
        {
            cplx *g = (cplx *)malloc((size_t)L * sizeof(cplx));
            cplx *r = (cplx *)malloc((size_t)L * sizeof(cplx));
            cplx *s = (cplx *)malloc((size_t)L * sizeof(cplx));
            if (!g || !r || !s) {
#pragma omp atomic write
                err = 1;
            } else {
#pragma omp for schedule(static)
                for (long q = 0; q < npen; ++q) {
                    const long base = (q % len[o1]) * stride[o1] + (q / len[o1]) * stride[o2];
                    for (int t = 0; t < L; ++t) g[t] = a[base + t * stride[axis]];
                    fft_rec(L, g, 1, r, s, tw, L);
                    for (int t = 0; t < L; ++t) a[base + t * stride[axis]] = r[t];
                }
            }
            free(g); free(r); free(s);
        }
        free(tw);
    }
    return err ? OR_ERR_NOMEM : OR_OK;
}

/* Box DFT, interleaved complex in place, a[z][y][x] of pz x py x px. */
int or_fft3_box(int px, int py, int pz, double *data, int sign)
{
    if (bad_box(px, py, pz) || !data || (sign != 1 && sign != -1)) return OR_ERR_ARG;
    return fft3_box_inplace(px, py, pz, (cplx *)data, sign);
}

/* kpad[z][y][x] = K(min(x,Px-x), min(y,Py-y), min(z,Pz-z)), Pa = 2 Na per axis. */
int or_kernel_pad_box(int nx, int ny, int nz, double dx, double dy, double dz, double self_coeff, double *kpad)
{
    if (bad_box(nx, ny, nz) || bad_spacing(dx, dy, dz) || !kpad) return OR_ERR_ARG;
    const long px = 2L * nx, py = 2L * ny, pz = 2L * nz;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < pz; ++z)
        for (long y = 0; y < py; ++y)
            for (long x = 0; x < px; ++x) {
                const long az = z < pz - z ? z : pz - z, ay = y < py - y ? y : py - y, ax = x < px - x ? x : px - x;
                kpad[(z * py + y) * px + x] = MUT(15) ? or_kernel_value3(ax, az, ay, dx, dy, dz, self_coeff)
                                                      : or_kernel_value3(ax, ay, az, dx, dy, dz, self_coeff);
            }
    return OR_OK;
}

/* The FFT-convolution solve on a box: both operands zero-padded to
 * 2nx x 2ny x 2nz, full complex DFTs, product, inverse divided by the padded
 * size, real part, crop, times G dx dy dz. */
int or_fft_conv_box(int nx, int ny, int nz, double dx, double dy, double dz, double g, double self_coeff,
                    const double *rho, double *phi)
{
    if (bad_box(nx, ny, nz) || bad_spacing(dx, dy, dz) || !rho || !phi) return OR_ERR_ARG;
    const long px = 2L * nx, py = 2L * ny, pz = 2L * nz, m = px * py * pz;
    double *kp = (double *)malloc((size_t)m * sizeof(double));
    cplx *a = (cplx *)calloc((size_t)m, sizeof(cplx));
    cplx *k = (cplx *)malloc((size_t)m * sizeof(cplx));
    if (!kp || !a || !k) {
        free(kp); free(a); free(k);
        return OR_ERR_NOMEM;
    }
    int rc = or_kernel_pad_box(nx, ny, nz, dx, dy, dz, self_coeff, kp);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < m; ++i) k[i] = kp[i];
    free(kp);
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) a[(z * py + y) * px + x] = rho[(z * ny + y) * nx + x];
    if (!rc) rc = fft3_box_inplace((int)px, (int)py, (int)pz, k, -1);
    if (!rc) rc = fft3_box_inplace((int)px, (int)py, (int)pz, a, -1);
    if (!rc) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) a[i] *= k[i];
        rc = fft3_box_inplace((int)px, (int)py, (int)pz, a, +1);
    }
    if (!rc) {
        const double scale = g * dx * dy * dz / (double)(MUT(14) ? px * px * pz : m);
#pragma omp parallel for schedule(static)
        for (long z = 0; z < nz; ++z)
            for (long y = 0; y < ny; ++y)
                for (long x = 0; x < nx; ++x)
                    phi[(z * ny + y) * nx + x] = scale * creal(a[(z * py + y) * px + x]);
    }
    free(a);
    free(k);
    return rc;
}
