/*
 * Driver for the host-sanitizer run of the CPU oracle: builds the oracle's
 * own source with AddressSanitizer and UndefinedBehaviorSanitizer and
 * exercises every entry point (hierarchy build, single operators on every
 * level and order, V-cycles, solves in all boundary-order modes and
 * schedules, initial guesses, Dirichlet data) on ragged, odd, tiny and
 * island-rich masks.  Any out-of-bounds access, use of freed memory, leak,
 * signed overflow or other undefined behaviour aborts with a report.
 */
#include "../oracle/mg_oracle.c"

#include <stdio.h>

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double urand(void) {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

static void run_case(int nx, int ny, int nz, double frac, int with_b) {
    const size_t n = (size_t)nx * ny * nz;
    int8_t *mask = malloc(n);
    double *rho = malloc(n * sizeof(double)), *phi = malloc(n * sizeof(double));
    double *B = malloc(n * sizeof(double)), *x = malloc(n * sizeof(double)), *r = malloc(n * sizeof(double));
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                const size_t p = ((size_t)k * ny + j) * nx + i;
                const int frame = i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1;
                mask[p] = (!frame && urand() < frac) ? 1 : -1;
                rho[p] = urand() - 0.5;
                B[p] = urand() - 0.5;
            }
    orc_h *H = orc_create(mask, nx, ny, nz, 1.0 / nx, 4);
    if (!H) {  /* no active cell is a valid rejection */
        free(mask); free(rho); free(phi); free(B); free(x); free(r);
        return;
    }
    const double *Bp = with_b ? B : NULL;
    for (int order = 1; order <= 2; order++)
        for (int l = 0; l < orc_nlevels(H, order); l++) {
            int d[3];
            orc_level_dims(H, l, d);
            const size_t m = (size_t)d[0] * d[1] * d[2];
            double *xl = calloc(m, sizeof(double)), *fl = calloc(m, sizeof(double)), *rl = calloc(m, sizeof(double));
            double *dg = calloc(m, sizeof(double));
            int64_t *cn = calloc(m, sizeof(int64_t));
            uint8_t *ac = calloc(m, 1);
            orc_level_counts(H, l, cn);
            orc_level_active(H, l, order, ac);
            orc_level_diag(H, l, order, dg);
            for (size_t p = 0; p < m; p++) {
                xl[p] = ac[p] ? urand() : 0.0;
                fl[p] = ac[p] ? urand() : 0.0;
            }
            orc_smooth(H, l, order, xl, l ? fl : rho, l ? NULL : Bp, 2);
            orc_residual(H, l, order, xl, l ? fl : rho, l ? NULL : Bp, rl);
            if (l + 1 < orc_nlevels(H, order)) {
                int dc[3];
                orc_level_dims(H, l + 1, dc);
                const size_t mc = (size_t)dc[0] * dc[1] * dc[2];
                double *fc = calloc(mc, sizeof(double));
                orc_restrict(H, l, order, rl, fc);
                orc_prolong(H, l, order, fc, xl);
                free(fc);
            }
            free(xl); free(fl); free(rl); free(dg); free(cn); free(ac);
        }
    orc_opts o;
    orc_info info;
    for (int mode = 0; mode < 6; mode++) {
        orc_default_opts(&o);
        if (mode == 1) o.bc_order = 1;
        if (mode == 2) o.bc_order = 2;
        if (mode == 3) o.n_cycles = 2;
        if (mode == 4) { o.n_pre = 1; o.n_post = 0; o.max_cycles = 3; }
        if (mode == 5) { o.n_pre = 3; o.n_post = 1; o.n_coarse = 5; }
        for (size_t p = 0; p < n; p++) phi[p] = mode == 3 ? urand() : 0.0;
        orc_solve(H, rho, phi, Bp, 1e-10, &o, &info);
        memcpy(x, phi, n * sizeof(double));
        orc_vcycle(H, 2, x, rho, Bp, &o);
        (void)orc_residual_norm(H, rho, x, Bp);
    }
    orc_destroy(H);
    free(mask); free(rho); free(phi); free(B); free(x); free(r);
}

int main(void) {
    run_case(16, 16, 16, 0.8, 0);
    run_case(24, 40, 56, 0.7, 1);   /* ragged, three levels */
    run_case(5, 7, 9, 0.9, 1);      /* odd dims: one level */
    run_case(32, 32, 32, 0.55, 1);  /* islands below the coarse cell size */
    run_case(8, 8, 8, 0.0, 0);      /* no active cell: rejected */
    run_case(6, 10, 10, 0.8, 1);
    run_case(48, 16, 16, 0.95, 0);  /* deep in x only */
    printf("oracle sanitizer run: ok\n");
    return 0;
}
