/*
 * Drives the CPU reference through every curvature model, both collision
 * operators, walls with wetting, the bubble model and the frozen mode on
 * small lattices, reads every output and checks mass conservation. Built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitizers.py; any invalid access, leak or undefined
 * behaviour ends the run with an error. Exit status 0 when every case ran
 * and conserved mass.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fslbm_oracle.h"

static const double PI = 3.14159265358979323846;

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* A sphere (or, with inverse, a bubble) as a linear ramp of the fill level
 * across its surface; walls at k = 0 and k = nz - 1 when walls is set. */
static void shape(int nx, int ny, int nz, double cx, double cy, double cz, double r, int inverse, int walls,
                  double *fill, unsigned char *obst)
{
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long i = x + (long)nx * (y + (long)ny * z);
                const double d = sqrt((x + 0.5 - cx) * (x + 0.5 - cx) + (y + 0.5 - cy) * (y + 0.5 - cy) +
                                      (z + 0.5 - cz) * (z + 0.5 - cz));
                const double v = clamp01(r + 0.5 - d);
                fill[i] = inverse ? 1.0 - v : v;
                obst[i] = 0;
                if (walls && (z == 0 || z == nz - 1)) {
                    obst[i] = 1;
                    fill[i] = 0.0;
                }
            }
}

static int run_case(const char *name, int n, int nz, int walls, int inverse, double cz, double r, orc_params p,
                    long steps, double u0)
{
    const long N = (long)n * n * nz;
    double *fill = malloc(sizeof(double) * N), *out = malloc(sizeof(double) * 3 * N);
    double *pdf = malloc(sizeof(double) * 19 * N), *rho = malloc(sizeof(double) * N), *u = calloc(3 * N, sizeof(double));
    unsigned char *obst = malloc(N), *flags = malloc(N);
    int *list = malloc(sizeof(int) * N);
    int ok = 1;
    shape(n, n, nz, n / 2.0, n / 2.0, cz, r, inverse, walls, fill, obst);
    orc_lattice *L = orc_create(n, n, nz, fill, obst, &p);
    if (!L) {
        printf("%s: create failed\n", name);
        ok = 0;
        goto done;
    }
    if (u0 != 0.0) {
        for (long i = 0; i < N; ++i) {
            rho[i] = 1.0;
            u[i] = u0;
        }
        orc_set_equilibrium(L, rho, u);
    }
    const double m0 = orc_get_mass(L);
    orc_step(L, steps);
    orc_get_fill(L, out);
    for (long i = 0; i < N; ++i)
        if (!isfinite(out[i])) ok = 0;
    orc_get_flags(L, flags);
    orc_get_density(L, out);
    orc_get_velocity(L, out);
    orc_get_curvature(L, out);
    orc_get_normal(L, out);
    orc_get_plic(L, out);
    orc_get_mass_field(L, out);
    (void)orc_get_reservoir(L);
    (void)orc_get_gas_density(L);
    (void)orc_interface_list(L, list);
    orc_get_pdf(L, pdf);
    orc_set_pdf(L, pdf);
    orc_step(L, 1);
    const double m1 = orc_get_mass(L);
    if (!(fabs(m1 - m0) <= 1e-10 * fabs(m0))) {
        printf("%s: mass %.17g -> %.17g\n", name, m0, m1);
        ok = 0;
    }
    orc_destroy(L);
done:
    printf("%s: %s\n", name, ok ? "ok" : "FAILED");
    free(fill);
    free(out);
    free(pdf);
    free(rho);
    free(u);
    free(obst);
    free(flags);
    free(list);
    return ok;
}

static int building_blocks(void)
{
    const double nh[3] = {0.48, 0.6, 0.64};
    const double a = orc_plic_offset(nh, 0.3);
    int ok = fabs(orc_cut_volume(nh, a) - 0.3) < 1e-9;
    const double M[12] = {1, 0, 0, 1, 1, 1, 2, 1, 3, 1, 0, 2};
    const double b[4] = {1, 2, 3, 4};
    double x[3];
    ok &= orc_lsq_solve(4, 3, M, b, x) == 1 && isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
    ok &= isfinite(orc_quadric_curvature(0.1, 0.2, 0.05, 0.01, -0.02));
    double pts[27 * 3], d[26 * 3], coef[5];
    int np = 0;
    for (int k = -1; k <= 1; ++k)
        for (int j = -1; j <= 1; ++j)
            for (int i = -1; i <= 1; ++i) {
                pts[3 * np] = i;
                pts[3 * np + 1] = j;
                pts[3 * np + 2] = 0.05 * (i * i + j * j) + 0.01 * k;
                ++np;
            }
    (void)orc_lsqr_fit_points(np, pts, (const double[3]){0, 0, 1}, coef);
    int nd = 0;
    for (int j = -1; j <= 1; ++j)
        for (int i = -1; i <= 1; ++i) {
            if (!i && !j) continue;
            d[3 * nd] = i;
            d[3 * nd + 1] = j;
            d[3 * nd + 2] = -0.05 * (i * i + j * j);
            ++nd;
        }
    ok &= isfinite(orc_tr_curvature_points(nd, d, (const double[3]){0, 0, 1}));
    printf("building blocks: %s\n", ok ? "ok" : "FAILED");
    return ok;
}

int main(void)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.sigma = 5e-3;
    p.tau = 0.8;
    p.theta = PI / 2;
    p.rho_gas = 1.0;
    p.eps_c = 1e-3;
    p.trt_magic = 3.0 / 16.0;
    int ok = 1;

    p.curv_model = ORC_CURV_FD;
    ok &= run_case("FD droplet, moving (conversions)", 14, 14, 0, 0, 7.0, 4.0, p, 12, 0.03);
    p.curv_model = ORC_CURV_LSQR;
    p.collision = ORC_TRT;
    ok &= run_case("LSQR droplet, TRT", 14, 14, 0, 0, 7.0, 4.0, p, 8, 0.0);
    p.collision = ORC_SRT;
    p.curv_model = ORC_CURV_TR;
    ok &= run_case("TR droplet, moving", 14, 14, 0, 0, 7.0, 4.0, p, 8, 0.02);
    p.curv_model = ORC_CURV_LSQR;
    p.theta = PI / 3;
    ok &= run_case("LSQR sessile drop, 60 deg", 14, 10, 1, 0, 1.0, 4.5, p, 10, 0.0);
    p.curv_model = ORC_CURV_FD;
    p.theta = 2 * PI / 3;
    ok &= run_case("FD sessile drop, 120 deg", 14, 10, 1, 0, 1.0, 4.5, p, 10, 0.0);
    p.curv_model = ORC_CURV_TR;
    ok &= run_case("TR sessile drop", 14, 10, 1, 0, 1.0, 4.5, p, 6, 0.0);
    p.curv_model = ORC_CURV_LSQR;
    p.theta = PI / 2;
    p.bubble = 1;
    ok &= run_case("LSQR bubble with the bubble model, walls", 14, 14, 1, 1, 7.0, 3.5, p, 10, 0.0);
    p.bubble = 0;
    p.frozen = 1;
    ok &= run_case("LSQR droplet, frozen types", 14, 14, 0, 0, 7.0, 4.0, p, 10, 0.02);
    p.frozen = 0;
    ok &= building_blocks();
    return ok ? 0 : 1;
}
