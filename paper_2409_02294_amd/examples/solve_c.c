/* The solver's C ABI from plain C: no torch, device memory from the HIP
 * runtime.  For each precision, one plan, its workspace, the transformed
 * kernel, then the potential of a point mass: a density of 1/dx^3 in cell c
 * has the potential G K(i - c) exactly (K(d) = -1/(dx |d|), K(0) =
 * -self_coeff/dx), which the program checks at every cell.  It also runs a
 * two-member batched solve and one rejected call.  Exit status 0 on success.
 *
 * Build (see build.py): gcc -std=c11 solve_c.c -I<include> -I/opt/rocm/include
 *   -D__HIP_PLATFORM_AMD__ -L<pkg> -lps -L/opt/rocm/lib -lamdhip64 -lm
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ps.h"

static int check(ps_status s, const char *what)
{
    if (s != PS_OK) {
        fprintf(stderr, "%s: %s (%s)\n", what, ps_status_str(s), ps_last_error());
        return 1;
    }
    return 0;
}

/* impulse response of an n^3 solve in the given precision; returns max relative error or -1 */
static double impulse(int n, ps_precision prec, int real_bytes)
{
    const double dx = 1.0 / n, G = 1.0, self = 2.38;
    const size_t cells = (size_t)n * n * n, bytes = cells * (size_t)real_bytes;
    const int cz = n / 3, cy = n / 2, cx = n - 2;
    ps_plan p = NULL;
    size_t ws_bytes = 0;
    void *ws = NULL, *d_rho = NULL, *d_phi = NULL;
    double *h64 = calloc(cells, sizeof(double));
    float *h32 = calloc(cells, sizeof(float));
    double err = -1.0;
    if (!h64 || !h32) goto done;
    if (check(ps_plan_create(&p, n, dx, prec, NULL), "ps_plan_create")) goto done;
    if (check(ps_plan_workspace_bytes(p, &ws_bytes), "ps_plan_workspace_bytes")) goto done;
    if (hipMalloc(&ws, ws_bytes) != hipSuccess || hipMalloc(&d_rho, bytes) != hipSuccess ||
        hipMalloc(&d_phi, bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        goto done;
    }
    if (check(ps_green_build(p, ws, G, self, NULL), "ps_green_build")) goto done;
    const size_t c = ((size_t)cz * n + cy) * n + cx;
    if (real_bytes == 8) h64[c] = 1.0 / (dx * dx * dx);
    else h32[c] = (float)(1.0 / (dx * dx * dx));
    if (hipMemcpy(d_rho, real_bytes == 8 ? (void *)h64 : (void *)h32, bytes, hipMemcpyHostToDevice) != hipSuccess)
        goto done;
    if (check(ps_solve(p, d_rho, d_phi, NULL), "ps_solve")) goto done;
    if (hipMemcpy(real_bytes == 8 ? (void *)h64 : (void *)h32, d_phi, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        goto done;
    double emax = 0.0, vmax = 0.0;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const double d = sqrt((double)(z - cz) * (z - cz) + (double)(y - cy) * (y - cy) +
                                      (double)(x - cx) * (x - cx));
                const double want = G * (d == 0.0 ? -self / dx : -1.0 / (dx * d));
                const size_t i = ((size_t)z * n + y) * n + x;
                const double got = real_bytes == 8 ? h64[i] : (double)h32[i];
                if (fabs(got - want) > emax) emax = fabs(got - want);
                if (fabs(want) > vmax) vmax = fabs(want);
            }
    err = emax / vmax;
done:
    if (d_phi) hipFree(d_phi);
    if (d_rho) hipFree(d_rho);
    if (ws) hipFree(ws);
    ps_plan_destroy(p);
    free(h64);
    free(h32);
    return err;
}

/* two-member batch (n = 32 and 48, FP64) against single solves of the same densities */
static int batch(void)
{
    const int ns[2] = {32, 48};
    ps_plan plans[2] = {NULL, NULL};
    void *ws[2] = {NULL, NULL}, *rho[2] = {NULL, NULL}, *phi[2] = {NULL, NULL}, *ref[2] = {NULL, NULL};
    double *h = NULL, *g = NULL;
    int rc = 1;
    for (int k = 0; k < 2; ++k) {
        const int n = ns[k];
        const size_t bytes = (size_t)n * n * n * sizeof(double);
        size_t wb = 0;
        if (check(ps_plan_create(&plans[k], n, 1.0 / n, PS_F64, NULL), "ps_plan_create")) goto done;
        if (check(ps_plan_workspace_bytes(plans[k], &wb), "ps_plan_workspace_bytes")) goto done;
        if (hipMalloc(&ws[k], wb) || hipMalloc(&rho[k], bytes) || hipMalloc(&phi[k], bytes) ||
            hipMalloc(&ref[k], bytes))
            goto done;
        if (check(ps_green_build(plans[k], ws[k], 1.0, 2.38, NULL), "ps_green_build")) goto done;
        free(h);
        h = malloc(bytes);
        if (!h) goto done;
        for (size_t i = 0; i < (size_t)n * n * n; ++i) h[i] = (double)((i * 2654435761u) % 1000) / 1000.0;
        if (hipMemcpy(rho[k], h, bytes, hipMemcpyHostToDevice)) goto done;
        if (check(ps_solve(plans[k], rho[k], ref[k], NULL), "ps_solve")) goto done;
    }
    if (check(ps_solve_batched(plans, 2, (const void *const *)rho, phi, NULL), "ps_solve_batched")) goto done;
    if (hipDeviceSynchronize()) goto done;
    for (int k = 0; k < 2; ++k) {
        const size_t cells = (size_t)ns[k] * ns[k] * ns[k];
        free(h);
        free(g);
        h = malloc(cells * sizeof(double));
        g = malloc(cells * sizeof(double));
        if (!h || !g) goto done;
        if (hipMemcpy(h, phi[k], cells * sizeof(double), hipMemcpyDeviceToHost) ||
            hipMemcpy(g, ref[k], cells * sizeof(double), hipMemcpyDeviceToHost))
            goto done;
        for (size_t i = 0; i < cells; ++i)
            if (h[i] != g[i]) {
                fprintf(stderr, "batch member %d differs from ps_solve at %zu\n", k, i);
                goto done;
            }
    }
    rc = 0;
done:
    for (int k = 0; k < 2; ++k) {
        if (ref[k]) hipFree(ref[k]);
        if (phi[k]) hipFree(phi[k]);
        if (rho[k]) hipFree(rho[k]);
        if (ws[k]) hipFree(ws[k]);
        ps_plan_destroy(plans[k]);
    }
    free(h);
    free(g);
    return rc;
}

int main(void)
{
    const double e64 = impulse(32, PS_F64, 8);
    const double e32 = impulse(48, PS_F32, 4);
    printf("impulse response f64 n=32: max rel err %.3e\n", e64);
    printf("impulse response f32 n=48: max rel err %.3e\n", e32);
    if (e64 < 0.0 || e64 > 1e-13 || e32 < 0.0 || e32 > 1e-6) return 1;
    if (batch()) return 1;
    printf("batched f64 (n = 32, 48): members equal to ps_solve\n");
    /* an unsupported size is rejected with a status, not an abort */
    ps_plan q = NULL;
    const ps_status s = ps_plan_create(&q, 7, 1.0 / 7, PS_F64, NULL);
    printf("n = 7: %s (%s)\n", ps_status_str(s), ps_last_error());
    if (s != PS_ERR_UNSUPPORTED || q != NULL) return 1;
    printf("ok\n");
    return 0;
}
