/*
 * fslbm_oracle_tl.cpp -- tangent-linear (forward-mode) build of the CPU
 * reference: the source of fslbm_oracle.c compiled with every
 * double carried as a dual number (fslbm_dual.hpp), so that one directional
 * derivative of the whole step -- with respect to sigma, theta and the
 * initial fill level, in any combination -- is propagated through the same
 * operations in the same order as the values.
 *
 * TEST INFRASTRUCTURE ONLY: the reference gradient of the frozen-topology
 * window, for every curvature model. The one replaced step is the PLIC
 * offset's derivative (below): the bisection that finds the offset carries
 * none, so it is taken from the implicit function of the cut volume.
 *
 * Entry points take and return plain doubles:
 *   orc_tl_create   fill and its seed direction (or NULL), obstacle mask,
 *                   parameters with the seeds dsigma and dtheta; the
 *                   lattice runs with frozen cell types;
 *   orc_tl_set_equilibrium, orc_tl_step, orc_tl_get_fill (value and
 *                   derivative of phi), orc_tl_destroy.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fslbm_dual.hpp"

// The PLIC offset found by bisection carries no derivative. Inside (0, 1)
// it gets the one of the implicit function V(n, a) = phi:
// da = (dphi - dV/dn . dn) / (dV/da), both partials from dual evaluations
// of the cut volume. At phi = 0 or 1 (clamped) the plane sits on a corner of
// the cell, a = +-Ls/2, and the bracket's own derivative is that of +-Ls/2.
static Dual plic_result_tl(const Dual nhat[3], Dual phi, Dual a);
#define ORC_PLIC_RESULT(nhat, phi, a) plic_result_tl(nhat, phi, a)

#define double Dual
#include "fslbm_oracle.c"
#undef double

static Dual plic_result_tl(const Dual nhat[3], Dual phi, Dual a)
{
    if (!(phi.v > 0.0 && phi.v < 1.0)) return a;
    const Dual nv[3] = {Dual(nhat[0].v, 0.0), Dual(nhat[1].v, 0.0), Dual(nhat[2].v, 0.0)};
    const Dual vn = orc_cut_volume(nhat, Dual(a.v, 0.0));  // dV/dn . dn
    const Dual va = orc_cut_volume(nv, Dual(a.v, 1.0));    // dV/da
    if (va.d == 0.0) return a;
    return Dual(a.v, (phi.d - vn.d) / va.d);
}

extern "C" {

orc_lattice *orc_tl_create(int nx, int ny, int nz, const double *fill, const double *fill_dot,
                           const unsigned char *obstacle, double sigma, double dsigma, double tau, double theta,
                           double dtheta, double rho_gas, double eps_c, int curv_model, int collision,
                           double trt_magic)
{
    const long n = (long)nx * ny * nz;
    Dual *f = (Dual *)malloc(sizeof(Dual) * n);
    for (long i = 0; i < n; ++i) f[i] = Dual(fill[i], fill_dot ? fill_dot[i] : 0.0);
    orc_params p;
    memset(&p, 0, sizeof p);
    p.sigma = Dual(sigma, dsigma);
    p.tau = tau;
    p.theta = Dual(theta, dtheta);
    p.rho_gas = rho_gas;
    p.eps_c = eps_c;
    p.trt_magic = trt_magic;
    p.curv_model = curv_model;
    p.collision = collision;
    p.frozen = 1;
    p.bubble = 0;
    orc_lattice *L = orc_create(nx, ny, nz, f, obstacle, &p);
    free(f);
    return L;
}

void orc_tl_set_equilibrium(orc_lattice *L, const double *rho, const double *u3)
{
    const long n = L->n;
    Dual *r = (Dual *)malloc(sizeof(Dual) * n), *u = (Dual *)malloc(sizeof(Dual) * 3 * n);
    for (long i = 0; i < n; ++i) r[i] = rho[i];
    for (long i = 0; i < 3 * n; ++i) u[i] = u3[i];
    orc_set_equilibrium(L, r, u);
    free(r);
    free(u);
}

void orc_tl_step(orc_lattice *L, long nsteps) { orc_step(L, nsteps); }

void orc_tl_get_fill(const orc_lattice *L, double *val, double *dot)
{
    for (long i = 0; i < L->n; ++i) {
        val[i] = L->phi[i].v;
        dot[i] = L->phi[i].d;
    }
}

void orc_tl_destroy(orc_lattice *L) { orc_destroy(L); }

}  // extern "C"
