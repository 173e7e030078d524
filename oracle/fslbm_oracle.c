/*
 * fslbm_oracle.c -- plain FP64 CPU reference of one FSLBM time step.
 *
 * TEST INFRASTRUCTURE ONLY (see fslbm_oracle.h): the checker of the GPU
 * library, never part of the product path.
 *
 * Everything is written as plain loops over cells in ascending linear index,
 * one phase after the other, with a separate output array per phase so that
 * no phase reads what it writes. Each function names the passage of the
 * paper (Bogner, Ruede, Harting, Sec. II) it follows. Where the paper defers
 * to other work or is silent, the reading used here is stated in the comment.
 *
 * Time step, in order:
 *   1  stream (eq. lbe1) with bounce-back at walls, gas-link reconstruction
 *      (eq. reconstruct) with rho_b = (p_g + p_s)/c_s^2, p_s = sigma*K, and
 *      the corner-node rule of Fig. inhomo; mass exchange (eq. advection1/2)
 *      in mass form; moments; collision (eq. lbe2, SRT or TRT)
 *   2  fill / empty classification of interface cells
 *   3  cell-type conversion, closure of the interface layer (every
 *      interface cell keeps a gas and a liquid D3Q19 neighbour, Sec. II.D)
 *      and excess-mass redistribution
 *   4  fill levels phi = m / rho, obstacle fill reflection (Sec. II.A)
 *   5  interface normals (eq. normal) and PLIC points (Sec. II.B), curvature
 *      by FD (eq. curvature, K8 mollifier), LSQR (Sec. II.C, eqs.
 *      LSQR-model, LSQR-error, anacurv, contactNormal, contactConstraint) or
 *      TR (Sec. II.B: triangle fan of the PLIC points, Taubin's estimate)
 *
 * Pins: the test suite checks this file against closed forms (PLIC volumes,
 * the graph curvature, planes, spheres, cylinders, lattice viscosity),
 * physical laws (Laplace law, flat surface at rest, exact mass conservation,
 * contact-angle response) and library routines (least squares). Parity
 * unpinned: the conversion rules of step 3 (thresholds, priority, new-cell
 * initialisation, excess split), which the paper defers to Koerner et al.;
 * they are checked only through mass conservation and the cell-type
 * invariants of Sec. II (no liquid cell next to a gas cell; every interface
 * cell with a gas and a liquid neighbour).
 */
#include "fslbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- D3Q19 velocity set (Sec. II; Qian et al. 1992 weights) ------------ */
#define NQ 19
static const int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static int OPP(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
static double WQ(int q)
{
    int nz = (CX[q] != 0) + (CY[q] != 0) + (CZ[q] != 0);
    return nz == 0 ? 1.0 / 3.0 : (nz == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

struct orc_lattice {
    int nx, ny, nz;
    long n;
    orc_params p;
    unsigned char *type;
    double *f;      /* post-collision PDFs f'(t), [q*n + i] */
    double *fnew;   /* scratch for f'(t+1) */
    double *m;      /* interface mass */
    double *rho;    /* density of interface cells */
    double *phi;    /* fill level, all cells (obstacles: reflected value) */
    double *K;      /* K = -div(nhat) = 2*mean curvature, interface cells */
    double *nrm;    /* unit Parker-Youngs normal of raw phi, interface, 3n */
    double *plic;   /* PLIC plane offset a, interface cells */
    double reservoir;
    double gas_v0;   /* bubble model: gas volume at creation */
    double rho_g;    /* gas density used by the step: rho_gas, or with the
                      * bubble model rho_gas * V0 / V(t) */
    int *nb;        /* 27 neighbour indices per cell, offset (dx,dy,dz) at
                     * slot (dz+1)*9 + (dy+1)*3 + (dx+1), periodic wrap */
};

/* ---- small helpers ------------------------------------------------------ */
static long wrap(long v, long n) { v %= n; return v < 0 ? v + n : v; }
static long idx_of(const orc_lattice *L, long x, long y, long z)
{
    return wrap(x, L->nx) + L->nx * (wrap(y, L->ny) + L->ny * wrap(z, L->nz));
}
static void coords(const orc_lattice *L, long i, long *x, long *y, long *z)
{
    *x = i % L->nx;
    *y = (i / L->nx) % L->ny;
    *z = i / ((long)L->nx * L->ny);
}
static long nbr(const orc_lattice *L, long i, int dx, int dy, int dz)
{
    return L->nb[27 * i + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
}
static int is_fluid(unsigned char t) { return t == ORC_LIQUID || t == ORC_INTERFACE; }

/* Second-order equilibrium w_q rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2]; the
 * paper uses it without printing it (cites Koerner et al.). */
static double feq(int q, double rho, const double u[3])
{
    double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return WQ(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* Moments rho = sum f_q, rho u = sum c_q f_q (Sec. II). */
static void moments(const double fq[NQ], double *rho, double u[3])
{
    double r = 0, jx = 0, jy = 0, jz = 0;
    for (int q = 0; q < NQ; ++q) {
        r += fq[q];
        jx += CX[q] * fq[q];
        jy += CY[q] * fq[q];
        jz += CZ[q] * fq[q];
    }
    *rho = r;
    u[0] = jx / r;
    u[1] = jy / r;
    u[2] = jz / r;
}

/* ---- collision (eq. lbe2) ----------------------------------------------- */
/* SRT: f' = f - (f - feq)/tau. TRT (Ginzburg 2007): even and odd parts relax
 * with 1/tau and 1/tau_o, tau_o from Lambda = (tau - 1/2)(tau_o - 1/2). */
static void collide(const orc_params *p, const double fin[NQ], double fout[NQ])
{
    double rho, u[3];
    moments(fin, &rho, u);
    double we = 1.0 / p->tau;
    if (p->collision == ORC_SRT) {
        for (int q = 0; q < NQ; ++q) fout[q] = fin[q] - we * (fin[q] - feq(q, rho, u));
    } else {
        double wo = 1.0 / (0.5 + p->trt_magic / (p->tau - 0.5));
        for (int q = 0; q < NQ; ++q) {
            int o = OPP(q);
            double fp = 0.5 * (fin[q] + fin[o]), fm = 0.5 * (fin[q] - fin[o]);
            double ep = 0.5 * (feq(q, rho, u) + feq(o, rho, u));
            double em = 0.5 * (feq(q, rho, u) - feq(o, rho, u));
            fout[q] = fin[q] - we * (fp - ep) - wo * (fm - em);
        }
    }
}

/* ---- PLIC: cut volume and plane offset (Sec. II.B) --------------------- */
/* Volume of {y in [0,1]^3 : m.y <= alpha} for sorted m1 <= m2 <= m3, m_i >= 0,
 * m1 + m2 + m3 = 1. Inclusion-exclusion over the cube's corners gives
 * [alpha^3 - sum (alpha - m_i)_+^3 + sum (alpha - m_i - m_j)_+^3 - ...]
 * / (6 m1 m2 m3); for alpha <= 1/2 at most the terms below survive, and each
 * branch is rearranged so that no small m_i appears alone in a denominator.
 * For alpha > 1/2 the point reflection y -> 1 - y gives V(alpha) = 1 - V(1-alpha). */
static double vol_below(double m1, double m2, double m3, double alpha)
{
    if (alpha <= 0.0) return 0.0;
    if (alpha >= 1.0) return 1.0;
    if (alpha > 0.5) return 1.0 - vol_below(m1, m2, m3, 1.0 - alpha);
    if (alpha <= m1) /* corner tetrahedron */
        return alpha * alpha * (alpha / m1) / (6.0 * m2 * m3);
    if (alpha <= m2) /* [alpha^3 - (alpha-m1)^3] / (6 m1 m2 m3) */
        return (3.0 * alpha * alpha - 3.0 * alpha * m1 + m1 * m1) / (6.0 * m2 * m3);
    if (alpha <= m1 + m2) {
        double d2 = alpha - m2; /* 0 < d2 <= m1 */
        double num = 3.0 * alpha * alpha - 3.0 * alpha * m1 + m1 * m1 - d2 * d2 * (d2 / m1);
        if (alpha > m3) {
            double d3 = alpha - m3; /* 0 < d3 <= d2 */
            num -= d3 * d3 * (d3 / m1);
        }
        return num / (6.0 * m2 * m3);
    }
    /* m1 + m2 < alpha (< m3): the plane cuts all four edges along y3 */
    return (2.0 * alpha - m1 - m2) / (2.0 * m3);
}

/* Liquid volume of the unit cell centred at the origin on the side
 * (x).nhat >= a of the plane x.nhat = a, for a unit normal nhat. */
double orc_cut_volume(const double nhat[3], double a)
{
    double ax = fabs(nhat[0]), ay = fabs(nhat[1]), az = fabs(nhat[2]);
    double Ls = ax + ay + az;
    if (Ls <= 0.0) return 0.0;
    double m[3] = {ax / Ls, ay / Ls, az / Ls};
    /* sort ascending */
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (m[j] > m[j + 1]) { double t = m[j]; m[j] = m[j + 1]; m[j + 1] = t; }
    /* flipping axes with negative components maps the cell onto [0,1]^3
     * with (x).nhat = sum |n_k| y_k - Ls/2; the liquid side is m.y >= a/Ls + 1/2,
     * whose volume equals V(1/2 - a/Ls) by the point reflection. */
    return vol_below(m[0], m[1], m[2], 0.5 - a / Ls);
}

/* Plane offset a with cut volume phi (clamped to [0,1]), by bisection on
 * [-Ls/2, Ls/2]; 42 halvings bring the bracket below 4e-13, the error bound
 * the paper quotes for its bisection (Sec. II.B). The result passes through
 * ORC_PLIC_RESULT, the identity here; the tangent-linear build replaces it
 * to give the offset the derivative of V(n, a) = phi, which a bisection
 * bracket does not carry. */
#ifndef ORC_PLIC_RESULT
#define ORC_PLIC_RESULT(nhat, phi, a) (a)
#endif
double orc_plic_offset(const double nhat[3], double phi)
{
    double Ls = fabs(nhat[0]) + fabs(nhat[1]) + fabs(nhat[2]);
    if (Ls <= 0.0) return 0.0;
    if (phi < 0.0) phi = 0.0;
    if (phi > 1.0) phi = 1.0;
    double lo = -0.5 * Ls, hi = 0.5 * Ls;
    for (int it = 0; it < 42; ++it) {
        double mid = 0.5 * (lo + hi);
        if (orc_cut_volume(nhat, mid) > phi) lo = mid;
        else hi = mid;
    }
    return ORC_PLIC_RESULT(nhat, phi, 0.5 * (lo + hi));
}

/* ---- least squares by Householder QR (LSQR solve, Sec. II.C) ----------- */
/* Solve min |M x - b| for an rows x cols row-major M (rows >= cols).
 * Returns 1 on success, 0 if a column is rank deficient: the squared norm of
 * the column below the diagonal (= R_kk^2) is below 1e-12 times the sum of
 * squares of all entries of M (= trace of M^T M). */
int orc_lsq_solve(int rows, int cols, const double *M, const double *b, double *x)
{
    if (rows < cols || cols <= 0) return 0;
    double *A = (double *)malloc(sizeof(double) * rows * cols);
    double *y = (double *)malloc(sizeof(double) * rows);
    double *v = (double *)malloc(sizeof(double) * rows);
    memcpy(A, M, sizeof(double) * rows * cols);
    memcpy(y, b, sizeof(double) * rows);
    double tr = 0.0;
    for (int i = 0; i < rows * cols; ++i) tr += A[i] * A[i];
    int ok = tr > 0.0;
    for (int k = 0; k < cols && ok; ++k) {
        double s = 0.0;
        for (int i = k; i < rows; ++i) s += A[i * cols + k] * A[i * cols + k];
        if (s < 1e-12 * tr) { ok = 0; break; }
        double nrm = sqrt(s);
        double alpha = A[k * cols + k] >= 0.0 ? -nrm : nrm;
        double vv = 0.0;
        for (int i = k; i < rows; ++i) {
            v[i] = A[i * cols + k] - (i == k ? alpha : 0.0);
            vv += v[i] * v[i];
        }
        if (vv > 0.0) {
            for (int j = k; j < cols; ++j) {
                double d = 0.0;
                for (int i = k; i < rows; ++i) d += v[i] * A[i * cols + j];
                d = 2.0 * d / vv;
                for (int i = k; i < rows; ++i) A[i * cols + j] -= d * v[i];
            }
            double d = 0.0;
            for (int i = k; i < rows; ++i) d += v[i] * y[i];
            d = 2.0 * d / vv;
            for (int i = k; i < rows; ++i) y[i] -= d * v[i];
        }
    }
    if (ok) {
        for (int k = cols - 1; k >= 0; --k) {
            double s = y[k];
            for (int j = k + 1; j < cols; ++j) s -= A[k * cols + j] * x[j];
            x[k] = s / A[k * cols + k];
        }
    }
    free(A);
    free(y);
    free(v);
    return ok;
}

/* K = 2 * mean curvature of w = A u^2 + B v^2 + C u v + H u + I v at u=v=0:
 * the mean curvature of a graph is
 * [(1+f_v^2) f_uu - 2 f_u f_v f_uv + (1+f_u^2) f_vv] / (2 (1+f_u^2+f_v^2)^{3/2})
 * with f_uu = 2A, f_vv = 2B, f_uv = C, f_u = H, f_v = I. This is eq. anacurv
 * with the cross term C*H*I (the printed factor 2 belongs to a 2Cuv model). */
double orc_quadric_curvature(double A, double B, double C, double H, double I)
{
    double g = 1.0 + H * H + I * I;
    return 2.0 * (A * (1.0 + I * I) + B * (1.0 + H * H) - C * H * I) / (g * sqrt(g));
}

/* Local orthonormal frame (t_u, t_v, n) at an interface point (Sec. II.C):
 * t_u is the axis e_k with the smallest |n_k| made orthogonal to n. */
static void local_frame(const double n[3], double tu[3], double tv[3])
{
    int k = 0;
    if (fabs(n[1]) < fabs(n[k])) k = 1;
    if (fabs(n[2]) < fabs(n[k])) k = 2;
    double e[3] = {0, 0, 0};
    e[k] = 1.0;
    double en = n[k];
    double t[3] = {e[0] - en * n[0], e[1] - en * n[1], e[2] - en * n[2]};
    double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    tu[0] = t[0] / tn; tu[1] = t[1] / tn; tu[2] = t[2] / tn;
    tv[0] = n[1] * tu[2] - n[2] * tu[1];
    tv[1] = n[2] * tu[0] - n[0] * tu[2];
    tv[2] = n[0] * tu[1] - n[1] * tu[0];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Rows of the LSQR system (eq. LSQR-model with J = 0, eq. LSQR-error) and of
 * the contact constraints (eq. contactConstraint). */
typedef struct {
    int nrow;
    double M[80][5];
    double b[80];
    int hard;            /* centre cell carries the contact constraint */
    double hu[5], hv[5]; /* its two rows */
    double hbu, hbv;
} lsq_rows;

static void add_row(lsq_rows *S, double a0, double a1, double a2, double a3, double a4, double rhs)
{
    if (S->nrow >= 80) return;
    double *r = S->M[S->nrow];
    r[0] = a0; r[1] = a1; r[2] = a2; r[3] = a3; r[4] = a4;
    S->b[S->nrow] = rhs;
    S->nrow++;
}

/* Solve the LSQR rows for (A,B,C,H,I). Without a hard constraint: the full
 * 5-parameter model if at least 5 rows and full rank, else the isotropic
 * model A = B, C = 0 (3 parameters), else no fit. With the centre's contact
 * constraint, H and I are eliminated through it and the same cascade runs
 * on (A,B,C) then on A alone (B = A, C = 0). Returns 1 if fitted. */
static int lsq_fit(const lsq_rows *S, double coef[5])
{
    int n = S->nrow;
    double (*Mr)[5] = (double (*)[5])malloc(sizeof(double) * 5 * (n > 0 ? n : 1));
    double *br = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double x[5] = {0, 0, 0, 0, 0};
    int ok = 0;
    if (!S->hard) {
        if (n >= 5) {
            for (int r = 0; r < n; ++r) { for (int c = 0; c < 5; ++c) Mr[r][c] = S->M[r][c]; br[r] = S->b[r]; }
            if (orc_lsq_solve(n, 5, &Mr[0][0], br, x)) {
                for (int c = 0; c < 5; ++c) coef[c] = x[c];
                ok = 1;
            }
        }
        if (!ok && n >= 3) {
            double *Mi = (double *)malloc(sizeof(double) * 3 * n);
            for (int r = 0; r < n; ++r) {
                Mi[r * 3 + 0] = S->M[r][0] + S->M[r][1];
                Mi[r * 3 + 1] = S->M[r][3];
                Mi[r * 3 + 2] = S->M[r][4];
                br[r] = S->b[r];
            }
            if (orc_lsq_solve(n, 3, Mi, br, x)) {
                coef[0] = x[0]; coef[1] = x[0]; coef[2] = 0.0; coef[3] = x[1]; coef[4] = x[2];
                ok = 1;
            }
            free(Mi);
        }
    } else {
        /* Hard rows: hu.(A,B,C,H,I) = hbu with hu = (2uc, 0, vc, 1, 0) and
         * hv = (0, 2vc, uc, 0, 1), so H = hbu - hu0 A - hu2 C and
         * I = hbv - hv1 B - hv2 C. Substituting into a row a.x = b gives
         * (a0 - a3 hu0) A + (a1 - a4 hv1) B + (a2 - a3 hu2 - a4 hv2) C
         *   = b - a3 hbu - a4 hbv. */
        const double *hu = S->hu, *hv = S->hv;
        double (*Me)[3] = (double (*)[3])malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
        for (int r = 0; r < n; ++r) {
            const double *a = S->M[r];
            Me[r][0] = a[0] - a[3] * hu[0];
            Me[r][1] = a[1] - a[4] * hv[1];
            Me[r][2] = a[2] - a[3] * hu[2] - a[4] * hv[2];
            br[r] = S->b[r] - a[3] * S->hbu - a[4] * S->hbv;
        }
        double A = 0, B = 0, C = 0;
        if (n >= 3 && orc_lsq_solve(n, 3, &Me[0][0], br, x)) {
            A = x[0]; B = x[1]; C = x[2];
            ok = 1;
        }
        if (!ok && n >= 1) {
            double *Mi = (double *)malloc(sizeof(double) * n);
            for (int r = 0; r < n; ++r) Mi[r] = Me[r][0] + Me[r][1];
            if (orc_lsq_solve(n, 1, Mi, br, x)) {
                A = x[0]; B = x[0]; C = 0.0;
                ok = 1;
            }
            free(Mi);
        }
        if (ok) {
            coef[0] = A; coef[1] = B; coef[2] = C;
            coef[3] = S->hbu - hu[0] * A - hu[2] * C;
            coef[4] = S->hbv - hv[1] * B - hv[2] * C;
        }
        free(Me);
    }
    free(Mr);
    free(br);
    return ok;
}

int orc_lsqr_fit_points(int npts, const double *pts, const double nhat[3], double *coef5)
{
    double tu[3], tv[3];
    local_frame(nhat, tu, tv);
    lsq_rows S;
    memset(&S, 0, sizeof S);
    for (int k = 0; k < npts; ++k) {
        const double *r = pts + 3 * k;
        double u = dot3(r, tu), v = dot3(r, tv), w = dot3(r, nhat);
        add_row(&S, u * u, v * v, u * v, u, v, w);
    }
    return lsq_fit(&S, coef5);
}

/* ---- fill-level gradients (eq. normal) ---------------------------------- */
/* Parker-Youngs gradient: central differences across the 3x3x3 block with
 * tensor-product weights (1,2,1) in the two transverse directions. The sum
 * is left unscaled (its direction is what the normal needs). */
static double pyw(int d) { return d == 0 ? 2.0 : 1.0; }
static void py_gradient(const orc_lattice *L, const double *g, long i, double out[3])
{
    double gx = 0, gy = 0, gz = 0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b) {
            double w = pyw(a) * pyw(b);
            gx += w * (g[nbr(L, i, 1, a, b)] - g[nbr(L, i, -1, a, b)]);
            gy += w * (g[nbr(L, i, a, 1, b)] - g[nbr(L, i, a, -1, b)]);
            gz += w * (g[nbr(L, i, a, b, 1)] - g[nbr(L, i, a, b, -1)]);
        }
    out[0] = gx; out[1] = gy; out[2] = gz;
}

/* ---- obstacle fill reflection (Sec. II.A) ------------------------------- */
/* phi(x_o) = sum |nw.c^_q| phi(x_o + c_q) / sum |nw.c^_q| over fluid
 * neighbours x_o + c_q whose aperture |nw.c^_q| exceeds alpha = sqrt(2)/2
 * (strictly: the 45-degree links are excluded). nw is the normalised sum of
 * the lattice directions from x_o to its non-obstacle neighbours. */
static void obstacle_fill(orc_lattice *L)
{
    const double alpha = sqrt(2.0) / 2.0 + 1e-12;
    for (long i = 0; i < L->n; ++i) {
        if (L->type[i] != ORC_OBSTACLE) continue;
        double nw[3] = {0, 0, 0};
        for (int q = 1; q < NQ; ++q)
            if (L->type[nbr(L, i, CX[q], CY[q], CZ[q])] != ORC_OBSTACLE) {
                nw[0] += CX[q]; nw[1] += CY[q]; nw[2] += CZ[q];
            }
        double len = sqrt(dot3(nw, nw));
        double num = 0.0, den = 0.0;
        if (len > 0.0) {
            for (int k = 0; k < 3; ++k) nw[k] /= len;
            for (int q = 1; q < NQ; ++q) {
                long j = nbr(L, i, CX[q], CY[q], CZ[q]);
                if (!is_fluid(L->type[j])) continue;
                double cl = sqrt((double)(CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q]));
                double w = fabs((nw[0] * CX[q] + nw[1] * CY[q] + nw[2] * CZ[q]) / cl);
                if (w > alpha) {
                    num += w * L->phi[j];
                    den += w;
                }
            }
        }
        L->phi[i] = den > 0.0 ? num / den : 0.0;
    }
}

/* ---- bubble model (Sec. III.A.1) ------------------------------------------ */
/* Gas volume V = sum over non-obstacle cells of (1 - phi): 1 per gas cell,
 * 1 - phi per interface cell. With the bubble model the whole gas of the
 * lattice is one bubble whose pressure follows its volume isothermally,
 * p_g(t) V(t) = p_g(0) V(0), i.e. rho_gas(t) = rho_gas V0 / V(t). */
static double gas_volume(const orc_lattice *L)
{
    double v = 0.0;
    for (long i = 0; i < L->n; ++i)
        if (L->type[i] != ORC_OBSTACLE) v += 1.0 - L->phi[i];
    return v;
}

static void update_gas_density(orc_lattice *L)
{
    if (!L->p.bubble) {
        L->rho_g = L->p.rho_gas;
        return;
    }
    const double v = gas_volume(L);
    L->rho_g = v > 0.0 ? L->p.rho_gas * L->gas_v0 / v : L->p.rho_gas;
}

/* ---- curvature ---------------------------------------------------------- */
/* Normals from raw phi at interface cells (the corner rule uses them with
 * both models) and, for the LSQR model, PLIC offsets (Sec. II.B: the PLIC
 * normal uses no convolution). An interface cell whose gradient vanishes
 * gets a zero normal and no PLIC point. */
static void normals_and_plic(orc_lattice *L)
{
    for (long i = 0; i < L->n; ++i) {
        L->nrm[3 * i] = L->nrm[3 * i + 1] = L->nrm[3 * i + 2] = 0.0;
        L->plic[i] = 0.0;
        if (L->type[i] != ORC_INTERFACE) continue;
        double g[3];
        py_gradient(L, L->phi, i, g);
        double len = sqrt(dot3(g, g));
        if (len <= 1e-12) continue;
        double nh[3] = {g[0] / len, g[1] / len, g[2] / len};
        L->nrm[3 * i] = nh[0];
        L->nrm[3 * i + 1] = nh[1];
        L->nrm[3 * i + 2] = nh[2];
        if (L->p.curv_model != ORC_CURV_FD) L->plic[i] = orc_plic_offset(nh, L->phi[i]);
    }
}

/* FD wetting (Sec. II.A, eq. contactNormal). At an obstacle cell x_o next
 * to the fluid, w is the normalised sum of the directions to its
 * non-obstacle neighbours (out of the wall) and x_b = x_o + c_b the neighbour
 * along the lattice direction closest to w (the first one on ties). When x_b
 * (a cell of any type but obstacle: the interface normal that the paper
 * projects is the mollified gradient, which exists wherever phi varies)
 * has a mollified unit normal n_b, the wall value
 * m = n_w cos(theta) + n_t sin(theta), with n_w = -w (into the wall) and n_t
 * the normalised projection of n_b onto the wall, is extrapolated linearly
 * to the obstacle node, which lies half a cell beyond the wall on the line
 * from x_b: n(x_o) = normalise(2 m - n_b). The normals of the other cells,
 * and those of x_b themselves, are left as computed. nm holds three planes. */
static void fd_contact_normals(const orc_lattice *L, double *nm)
{
    const long n = L->n;
    const double ct = cos(L->p.theta), st = sin(L->p.theta);
    for (long i = 0; i < n; ++i) {
        if (L->type[i] != ORC_OBSTACLE) continue;
        double w[3] = {0, 0, 0};
        for (int q = 1; q < NQ; ++q)
            if (L->type[nbr(L, i, CX[q], CY[q], CZ[q])] != ORC_OBSTACLE) {
                w[0] += CX[q]; w[1] += CY[q]; w[2] += CZ[q];
            }
        const double lw = sqrt(dot3(w, w));
        if (lw <= 0.0) continue;
        for (int k = 0; k < 3; ++k) w[k] /= lw;
        int qb = 0;
        double best = -2.0;
        for (int q = 1; q < NQ; ++q) {
            const double cl = sqrt((double)(CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q]));
            const double a = (CX[q] * w[0] + CY[q] * w[1] + CZ[q] * w[2]) / cl;
            if (a > best) { best = a; qb = q; }
        }
        const long j = nbr(L, i, CX[qb], CY[qb], CZ[qb]);
        if (L->type[j] == ORC_OBSTACLE) continue;
        const double nb[3] = {nm[j], nm[n + j], nm[2 * n + j]};
        if (dot3(nb, nb) == 0.0) continue;
        const double nw[3] = {-w[0], -w[1], -w[2]};
        const double nn = dot3(nb, nw);
        double nt[3] = {nb[0] - nn * nw[0], nb[1] - nn * nw[1], nb[2] - nn * nw[2]};
        const double lt = sqrt(dot3(nt, nt));
        if (lt < 1e-12) continue;
        for (int k = 0; k < 3; ++k) nt[k] /= lt;
        double e[3];
        for (int k = 0; k < 3; ++k) e[k] = 2.0 * (nw[k] * ct + nt[k] * st) - nb[k];
        const double le = sqrt(dot3(e, e));
        if (le < 1e-12) continue;
        for (int k = 0; k < 3; ++k) nm[k * n + i] = e[k] / le;
    }
}

/* FD curvature (Sec. II.A): mollify phi with the K8 kernel of support
 * eps = 2 (Williams 1998), K8(r) ~ (1 - r^2/eps^2)^4, on the 27 points of the
 * 3x3x3 block: weights 256, 81, 16, 1 for distance 0, 1, sqrt2, sqrt3,
 * normalised by their sum 942. Then nhat = PY gradient of the mollified field,
 * normalised, and K = -div nhat with the same PY-weighted central difference
 * scaled to a derivative (1/16 for the transverse weights, 1/2 for the
 * central difference). */
static void curvature_fd(orc_lattice *L)
{
    long n = L->n;
    double *ms = (double *)malloc(sizeof(double) * n);
    double *nm = (double *)malloc(sizeof(double) * 3 * n);
    static const double k8[4] = {256.0, 81.0, 16.0, 1.0};
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (int c = -1; c <= 1; ++c)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a)
                    s += k8[abs(a) + abs(b) + abs(c)] * L->phi[nbr(L, i, a, b, c)];
        ms[i] = s / 942.0;
    }
    for (long i = 0; i < n; ++i) {
        double g[3];
        py_gradient(L, ms, i, g);
        double len = sqrt(dot3(g, g));
        for (int k = 0; k < 3; ++k) nm[k * n + i] = len > 1e-12 ? g[k] / len : 0.0;
    }
    fd_contact_normals(L, nm);
    for (long i = 0; i < n; ++i) {
        L->K[i] = 0.0;
        if (L->type[i] != ORC_INTERFACE) continue;
        double gx[3], gy[3], gz[3];
        py_gradient(L, nm, i, gx);          /* gradient of nhat_x */
        py_gradient(L, nm + n, i, gy);      /* gradient of nhat_y */
        py_gradient(L, nm + 2 * n, i, gz);  /* gradient of nhat_z */
        double div = (gx[0] + gy[1] + gz[2]) / 32.0;
        L->K[i] = -div;
    }
    free(ms);
    free(nm);
}

static int is_contact_cell(const orc_lattice *L, long j)
{
    if (L->type[j] != ORC_INTERFACE) return 0;
    for (int q = 1; q < NQ; ++q)
        if (L->type[nbr(L, j, CX[q], CY[q], CZ[q])] == ORC_OBSTACLE) return 1;
    return 0;
}

/* LSQR curvature (Sec. II.C). In the frame (t_u, t_v, nhat) of the centre's
 * PLIC point p, each other interface cell i of the 3x3x3 block with a PLIC
 * point p_i adds the row (u^2, v^2, uv, u, v) = w with (u, v, w) the frame
 * coordinates of p_i - p (eq. LSQR-model with J = 0, eq. LSQR-error).
 * Wetting: if the block contains an obstacle cell, every contact-line cell j
 * of the block (an interface cell with an obstacle among its D3Q19
 * neighbours) adds the gradient condition of eq. contactConstraint at its
 * contact point: grad f(u_c, v_c) = -(m_u, m_v)/m_n with
 * m = nw cos(theta) + nt sin(theta) (eq. contactNormal), nw the normalised sum
 * of the directions to j's obstacle neighbours (into the wall), nt the
 * normalised projection of j's normal onto the wall and m_n = m.nhat of the
 * centre. The contact point is the point of the line (j's PLIC plane) ∩
 * (wall plane) nearest to p_j, reached from p_j along the projection of nw
 * onto the PLIC plane (Fig. contactPoint); the wall plane lies half a cell
 * from j's centre along nw (bounce-back wall half-way between nodes). The
 * condition is a hard constraint when j is the centre, else two more rows. */
static double lsqr_cell(const orc_lattice *L, long i)
{
    const double *nh = L->nrm + 3 * i;
    if (dot3(nh, nh) == 0.0) return 0.0;
    double tu[3], tv[3];
    local_frame(nh, tu, tv);
    double pc[3] = {L->plic[i] * nh[0], L->plic[i] * nh[1], L->plic[i] * nh[2]};
    lsq_rows S;
    memset(&S, 0, sizeof S);
    int has_obst = 0;
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
                long j = nbr(L, i, a, b, c);
                if (L->type[j] == ORC_OBSTACLE) has_obst = 1;
                if (a == 0 && b == 0 && c == 0) continue;
                if (L->type[j] != ORC_INTERFACE) continue;
                const double *nj = L->nrm + 3 * j;
                if (dot3(nj, nj) == 0.0) continue;
                double r[3] = {a + L->plic[j] * nj[0] - pc[0], b + L->plic[j] * nj[1] - pc[1],
                               c + L->plic[j] * nj[2] - pc[2]};
                double u = dot3(r, tu), v = dot3(r, tv), w = dot3(r, nh);
                add_row(&S, u * u, v * v, u * v, u, v, w);
            }
    if (has_obst) {
        double ct = cos(L->p.theta), st = sin(L->p.theta);
        for (int c = -1; c <= 1; ++c)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    long j = nbr(L, i, a, b, c);
                    if (!is_contact_cell(L, j)) continue;
                    const double *nj = L->nrm + 3 * j;
                    if (dot3(nj, nj) == 0.0) continue;
                    double nw[3] = {0, 0, 0};
                    for (int q = 1; q < NQ; ++q)
                        if (L->type[nbr(L, j, CX[q], CY[q], CZ[q])] == ORC_OBSTACLE) {
                            nw[0] += CX[q]; nw[1] += CY[q]; nw[2] += CZ[q];
                        }
                    double lw = sqrt(dot3(nw, nw));
                    if (lw <= 0.0) continue;
                    for (int k = 0; k < 3; ++k) nw[k] /= lw;
                    double nn = dot3(nj, nw);
                    double nt[3] = {nj[0] - nn * nw[0], nj[1] - nn * nw[1], nj[2] - nn * nw[2]};
                    double lt = sqrt(dot3(nt, nt));
                    if (lt < 1e-12) continue;
                    for (int k = 0; k < 3; ++k) nt[k] /= lt;
                    double mh[3] = {nw[0] * ct + nt[0] * st, nw[1] * ct + nt[1] * st, nw[2] * ct + nt[2] * st};
                    double g[3] = {nw[0] - nn * nj[0], nw[1] - nn * nj[1], nw[2] - nn * nj[2]};
                    double gn = dot3(g, nw);
                    if (gn < 1e-12) continue;
                    double pj[3] = {L->plic[j] * nj[0], L->plic[j] * nj[1], L->plic[j] * nj[2]};
                    double t = (0.5 - dot3(pj, nw)) / gn;
                    double r[3] = {a + pj[0] + t * g[0] - pc[0], b + pj[1] + t * g[1] - pc[1],
                                   c + pj[2] + t * g[2] - pc[2]};
                    double uc = dot3(r, tu), vc = dot3(r, tv);
                    double mu = dot3(mh, tu), mv = dot3(mh, tv), mn = dot3(mh, nh);
                    if (fabs(mn) < 1e-6) continue;
                    if (a == 0 && b == 0 && c == 0) {
                        S.hard = 1;
                        S.hu[0] = 2 * uc; S.hu[1] = 0; S.hu[2] = vc; S.hu[3] = 1; S.hu[4] = 0;
                        S.hv[0] = 0; S.hv[1] = 2 * vc; S.hv[2] = uc; S.hv[3] = 0; S.hv[4] = 1;
                        S.hbu = -mu / mn;
                        S.hbv = -mv / mn;
                    } else {
                        add_row(&S, 2 * uc, 0, vc, 1, 0, -mu / mn);
                        add_row(&S, 0, 2 * vc, uc, 0, 1, -mv / mn);
                    }
                }
    }
    double coef[5];
    if (!lsq_fit(&S, coef)) return 0.0;
    return orc_quadric_curvature(coef[0], coef[1], coef[2], coef[3], coef[4]);
}

/* TR curvature (Sec. II.B). The paper cites the construction (a triangle
 * fan of the PLIC points of a 3x3x3 block, Pohl 2007; the curvature of the
 * polygonal surface by a variant of Taubin 1995) without its details; this
 * is the reading used here, written from those two methods.
 *   fan:  the neighbours' points, seen from the centre point p in its
 *         tangent plane (frame of local_frame), are ordered by their polar
 *         angle, measured from the direction at 1 rad from t_u (so that
 *         the lattice's symmetric directions never sit on the branch cut);
 *         angles within 1e-12 count as equal and keep block order. Points
 *         on the normal line (u^2 + v^2 < 1e-12) are left out. Consecutive
 *         points k, k+1 (cyclic) span the triangle (p, p_k, p_k+1) unless
 *         the angular gap between them is at least pi - 1e-12 (the fan is
 *         open there, e.g. at a wall).
 *   Taubin: along each edge p -> p_k the normal curvature is
 *         kappa_k = 2 (d_k . n) / |d_k|^2 with d_k = p_k - p; each vertex
 *         is weighted by the area of the fan triangles it belongs to. The
 *         trace of Taubin's matrix M = sum w_k kappa_k T_k T_k^T (unit
 *         tangents T_k, weights summing to 1) is sum w_k kappa_k, and his
 *         principal curvatures 3m1 - m2, 3m2 - m1 add up to 2 tr M, so
 *         K = kappa_1 + kappa_2 = 2 sum w_k kappa_k.
 * Fewer than three points, or no triangle, give K = 0. */
static double edge_curvature(const double d[3], const double n[3]) { return 2.0 * dot3(d, n) / dot3(d, d); }

double orc_tr_curvature_points(int npts, const double *d, const double nhat[3])
{
    const double PI = 3.14159265358979323846;
    double tu[3], tv[3];
    local_frame(nhat, tu, tv);
    const double c1 = cos(1.0), s1 = sin(1.0);
    int idx[32];
    double ang[32];
    int m = 0;
    for (int j = 0; j < npts && m < 32; ++j) {
        double u = dot3(d + 3 * j, tu), v = dot3(d + 3 * j, tv);
        if (u * u + v * v < 1e-12) continue;
        idx[m] = j;
        ang[m] = atan2(-u * s1 + v * c1, u * c1 + v * s1);
        m++;
    }
    if (m < 3) return 0.0;
    /* insertion sort by (angle, block order) */
    for (int a = 1; a < m; ++a) {
        int ki = idx[a];
        double ka = ang[a];
        int b = a - 1;
        while (b >= 0) {
            int before = fabs(ang[b] - ka) > 1e-12 ? ka < ang[b] : ki < idx[b];
            if (!before) break;
            idx[b + 1] = idx[b];
            ang[b + 1] = ang[b];
            --b;
        }
        idx[b + 1] = ki;
        ang[b + 1] = ka;
    }
    double num = 0.0, den = 0.0;
    for (int k = 0; k < m; ++k) {
        int k1 = (k + 1) % m;
        double gap = ang[k1] - ang[k] + (k1 == 0 ? 2.0 * PI : 0.0);
        if (gap >= PI - 1e-12) continue;
        const double *da = d + 3 * idx[k], *db = d + 3 * idx[k1];
        double cr[3] = {da[1] * db[2] - da[2] * db[1], da[2] * db[0] - da[0] * db[2], da[0] * db[1] - da[1] * db[0]};
        double area = 0.5 * sqrt(dot3(cr, cr));
        num += area * (edge_curvature(da, nhat) + edge_curvature(db, nhat));
        den += 2.0 * area;
    }
    return den > 0.0 ? 2.0 * num / den : 0.0;
}

static double tr_cell(const orc_lattice *L, long i)
{
    const double *nh = L->nrm + 3 * i;
    if (dot3(nh, nh) == 0.0) return 0.0;
    double pc[3] = {L->plic[i] * nh[0], L->plic[i] * nh[1], L->plic[i] * nh[2]};
    double d[26 * 3];
    int np = 0;
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
                long j = nbr(L, i, a, b, c);
                if (a == 0 && b == 0 && c == 0) continue;
                if (L->type[j] != ORC_INTERFACE) continue;
                const double *nj = L->nrm + 3 * j;
                if (dot3(nj, nj) == 0.0) continue;
                d[3 * np] = a + L->plic[j] * nj[0] - pc[0];
                d[3 * np + 1] = b + L->plic[j] * nj[1] - pc[1];
                d[3 * np + 2] = c + L->plic[j] * nj[2] - pc[2];
                np++;
            }
    return orc_tr_curvature_points(np, d, nh);
}

static void curvature(orc_lattice *L)
{
    normals_and_plic(L);
    if (L->p.curv_model == ORC_CURV_FD) {
        curvature_fd(L);
    } else if (L->p.curv_model == ORC_CURV_LSQR) {
        for (long i = 0; i < L->n; ++i) L->K[i] = L->type[i] == ORC_INTERFACE ? lsqr_cell(L, i) : 0.0;
    } else {
        for (long i = 0; i < L->n; ++i) L->K[i] = L->type[i] == ORC_INTERFACE ? tr_cell(L, i) : 0.0;
    }
}

/* ---- closure of the interface layer (Sec. II.D) --------------------------
 * The interface tracking defines an interface cell as a cell whose D3Q19
 * neighbourhood holds both gas and liquid cells. Given cell types t (no
 * liquid cell next to a gas cell), the interface cells that break this are
 * reclassified in two passes: first those without a gas neighbour become
 * liquid, then, on the updated types, those without a liquid neighbour
 * become gas. Neither pass can put a liquid cell next to a gas cell, and
 * neither undoes what the other established, so one pass of each suffices.
 * out[i] = 1 (to liquid), 2 (to gas) or 0. */
static int any_nbr_of(const orc_lattice *L, const unsigned char *t, long i, unsigned char want)
{
    for (int q = 1; q < NQ; ++q)
        if (t[nbr(L, i, CX[q], CY[q], CZ[q])] == want) return 1;
    return 0;
}

static void close_layer(const orc_lattice *L, const unsigned char *t, unsigned char *out)
{
    const long n = L->n;
    unsigned char *tb = (unsigned char *)malloc(n);
    for (long i = 0; i < n; ++i) {
        out[i] = 0;
        tb[i] = t[i];
        if (t[i] == ORC_INTERFACE && !any_nbr_of(L, t, i, ORC_GAS)) {
            out[i] = 1;
            tb[i] = ORC_LIQUID;
        }
    }
    for (long i = 0; i < n; ++i)
        if (tb[i] == ORC_INTERFACE && !any_nbr_of(L, tb, i, ORC_LIQUID)) out[i] = 2;
    free(tb);
}

/* ---- lattice construction ----------------------------------------------- */
/* Cell types from the fill level (Sec. II: gas cells have phi = 0, only
 * interface cells lie strictly between 0 and 1). A liquid cell with a gas
 * D3Q19 neighbour becomes an interface cell with phi = 1, so that every
 * gas-liquid contact runs through an interface cell; then the layer is closed
 * (close_layer). f starts at
 * feq(rho = 1, u = 0) and the interface mass at m = phi. */
orc_lattice *orc_create(int nx, int ny, int nz, const double *fill, const unsigned char *obstacle,
                        const orc_params *p)
{
    if (nx < 1 || ny < 1 || nz < 1 || !fill || !p) return NULL;
    if (!(p->tau > 0.5) || p->sigma < 0.0) return NULL;
    orc_lattice *L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->n = (long)nx * ny * nz;
    L->p = *p;
    long n = L->n;
    L->type = (unsigned char *)calloc(n, 1);
    L->f = (double *)calloc(NQ * n, sizeof(double));
    L->fnew = (double *)calloc(NQ * n, sizeof(double));
    L->m = (double *)calloc(n, sizeof(double));
    L->rho = (double *)calloc(n, sizeof(double));
    L->phi = (double *)calloc(n, sizeof(double));
    L->K = (double *)calloc(n, sizeof(double));
    L->nrm = (double *)calloc(3 * n, sizeof(double));
    L->plic = (double *)calloc(n, sizeof(double));
    L->nb = (int *)malloc(sizeof(int) * 27 * n);
    for (long i = 0; i < n; ++i) {
        long x, y, z;
        coords(L, i, &x, &y, &z);
        for (int c = -1; c <= 1; ++c)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a)
                    L->nb[27 * i + (c + 1) * 9 + (b + 1) * 3 + (a + 1)] = (int)idx_of(L, x + a, y + b, z + c);
    }
    for (long i = 0; i < n; ++i) {
        if (obstacle && obstacle[i]) L->type[i] = ORC_OBSTACLE;
        else if (fill[i] >= 1.0) L->type[i] = ORC_LIQUID;
        else if (fill[i] <= 0.0) L->type[i] = ORC_GAS;
        else L->type[i] = ORC_INTERFACE;
    }
    unsigned char *t0 = (unsigned char *)malloc(n);
    memcpy(t0, L->type, n);
    for (long i = 0; i < n; ++i) {
        if (t0[i] != ORC_LIQUID) continue;
        for (int q = 1; q < NQ; ++q)
            if (t0[nbr(L, i, CX[q], CY[q], CZ[q])] == ORC_GAS) { L->type[i] = ORC_INTERFACE; break; }
    }
    /* interface cells lacking a gas or a liquid neighbour: liquid (phi = 1)
     * or gas (phi = 0) */
    close_layer(L, L->type, t0);
    for (long i = 0; i < n; ++i) {
        if (t0[i] == 1) L->type[i] = ORC_LIQUID;
        else if (t0[i] == 2) L->type[i] = ORC_GAS;
    }
    free(t0);
    for (long i = 0; i < n; ++i) {
        for (int q = 0; q < NQ; ++q) L->f[q * n + i] = L->type[i] == ORC_OBSTACLE ? 0.0 : WQ(q);
        switch (L->type[i]) {
        case ORC_LIQUID: L->phi[i] = 1.0; break;
        case ORC_INTERFACE:
            L->phi[i] = fill[i] < 1.0 ? fill[i] : 1.0;
            L->rho[i] = 1.0;
            L->m[i] = L->phi[i];
            break;
        default: L->phi[i] = 0.0;
        }
    }
    obstacle_fill(L);
    L->gas_v0 = gas_volume(L);
    L->rho_g = L->p.rho_gas;
    curvature(L);
    return L;
}

void orc_destroy(orc_lattice *L)
{
    if (!L) return;
    free(L->type); free(L->f); free(L->fnew); free(L->m); free(L->rho);
    free(L->phi); free(L->K); free(L->nrm); free(L->plic); free(L->nb);
    free(L);
}

/* ---- one time step ------------------------------------------------------- */
enum { ST_NONE = 0, ST_FILL = 1, ST_EMPTY = 2 };

static void one_step(orc_lattice *L)
{
    const long n = L->n;
    const orc_params *p = &L->p;
    double *mnew = (double *)calloc(n, sizeof(double));
    double *rnew = (double *)calloc(n, sizeof(double));

    /* Phase 1: pull-stream with boundary rules, mass exchange, collision. */
    for (long i = 0; i < n; ++i) {
        unsigned char t = L->type[i];
        if (!is_fluid(t)) continue;
        double fo[NQ], fin[NQ], fout[NQ];
        for (int q = 0; q < NQ; ++q) fo[q] = L->f[q * n + i];
        /* boundary values (eq. reconstruct): u_b from the cell's own
         * post-collision moments (momentum is a collision invariant),
         * rho_b = (p_g + p_s)/c_s^2 = 3 p_g + 3 sigma K, p_g = rho_gas/3 */
        double rb0, ub[3];
        moments(fo, &rb0, ub);
        double Kc = t == ORC_INTERFACE ? L->K[i] : 0.0;
        double rhob = 3.0 * (L->rho_g / 3.0 + p->sigma * Kc);
        int has_gas = 0;
        double nw[3] = {0, 0, 0};
        for (int q = 1; q < NQ; ++q) {
            unsigned char tn = L->type[nbr(L, i, CX[q], CY[q], CZ[q])];
            if (tn == ORC_GAS) has_gas = 1;
            if (tn == ORC_OBSTACLE) { nw[0] += CX[q]; nw[1] += CY[q]; nw[2] += CZ[q]; }
        }
        /* corner-node rule (Fig. inhomo): at an interface cell with gas and
         * wall links, a wall link whose outgoing direction c_o points against
         * the liquid-pointing normal n projected into the wall takes the free
         * surface rule: c_o . P n < 0 with P the projection onto the wall
         * plane. Since P is symmetric this is (P c_o) . n < 0, and
         * P c_o |nw|^2 = c_o |nw|^2 - (c_o.nw) nw is an exact integer vector:
         * the link normal to the wall projects to exactly zero and stays
         * bounce-back, as in the figure. */
        int corner = (t == ORC_INTERFACE) && has_gas && dot3(nw, nw) > 0.0;
        const double *nn = L->nrm + 3 * i;
        int iw[3] = {(int)nw[0], (int)nw[1], (int)nw[2]};
        int ww = iw[0] * iw[0] + iw[1] * iw[1] + iw[2] * iw[2];
        fin[0] = fo[0];
        for (int q = 1; q < NQ; ++q) {
            long j = nbr(L, i, -CX[q], -CY[q], -CZ[q]); /* upstream node x - c_q */
            unsigned char tj = L->type[j];
            int o = OPP(q);
            int reconstruct = 0;
            if (is_fluid(tj)) {
                fin[q] = L->f[q * n + j];
            } else if (tj == ORC_GAS) {
                reconstruct = 1;
            } else { /* obstacle: half-way bounce-back unless the corner rule applies;
                      * outgoing direction towards the wall is c_o = -c_q */
                int co[3] = {-CX[q], -CY[q], -CZ[q]};
                int cw = co[0] * iw[0] + co[1] * iw[1] + co[2] * iw[2];
                double s = 0.0;
                for (int k = 0; k < 3; ++k) s += (double)(co[k] * ww - cw * iw[k]) * nn[k];
                if (corner && s < 0.0) reconstruct = 1;
                else fin[q] = fo[o];
            }
            if (reconstruct) /* eq. reconstruct with q and qbar renamed */
                fin[q] = feq(q, rhob, ub) + feq(o, rhob, ub) - fo[o];
        }
        /* mass exchange (eq. advection1/2) in mass form:
         * m(t+1) = m(t) + sum_q k(x,q) (f'_qbar(x+c_q) - f'_q(x)) */
        if (t == ORC_INTERFACE) {
            double dm = 0.0;
            for (int q = 1; q < NQ; ++q) {
                long z = nbr(L, i, CX[q], CY[q], CZ[q]);
                unsigned char tz = L->type[z];
                double k;
                if (tz == ORC_LIQUID) k = 1.0;
                else if (tz == ORC_INTERFACE) k = 0.5 * (L->phi[z] + L->phi[i]);
                else k = 0.0;
                dm += k * (L->f[OPP(q) * n + z] - fo[q]);
            }
            mnew[i] = L->m[i] + dm;
        }
        collide(p, fin, fout);
        for (int q = 0; q < NQ; ++q) L->fnew[q * n + i] = fout[q];
        if (t == ORC_INTERFACE) {
            double r = 0.0;
            for (int q = 0; q < NQ; ++q) r += fin[q];
            rnew[i] = r;
        }
    }

    /* Phase 2: classification of interface cells (none with frozen types,
     * the setting of the differentiated window). */
    unsigned char *st = (unsigned char *)calloc(n, 1);
    for (long i = 0; i < n && !p->frozen; ++i) {
        if (L->type[i] != ORC_INTERFACE) continue;
        if (mnew[i] > (1.0 + p->eps_c) * rnew[i]) st[i] = ST_FILL;
        else if (mnew[i] < -p->eps_c * rnew[i]) st[i] = ST_EMPTY;
    }
    /* Phase 3: conversions. Filling has priority: an emptying cell next to a
     * filling cell stays interface. Gas neighbours of filled cells and liquid
     * neighbours of emptied cells become interface. */
    unsigned char *st2 = (unsigned char *)malloc(n);
    memcpy(st2, st, n);
    for (long i = 0; i < n; ++i) {
        if (st[i] != ST_EMPTY) continue;
        for (int q = 1; q < NQ; ++q)
            if (st[nbr(L, i, CX[q], CY[q], CZ[q])] == ST_FILL) { st2[i] = ST_NONE; break; }
    }
    unsigned char *newi = (unsigned char *)calloc(n, 1); /* 1: gas->interface, 2: liquid->interface */
    for (long i = 0; i < n; ++i) {
        if (L->type[i] == ORC_GAS) {
            for (int q = 1; q < NQ; ++q)
                if (st2[nbr(L, i, CX[q], CY[q], CZ[q])] == ST_FILL) { newi[i] = 1; break; }
        } else if (L->type[i] == ORC_LIQUID) {
            for (int q = 1; q < NQ; ++q)
                if (st2[nbr(L, i, CX[q], CY[q], CZ[q])] == ST_EMPTY) { newi[i] = 2; break; }
        }
    }
    /* New interface cells from gas: f' = feq(mean rho, mean u) over their
     * liquid and interface neighbours (old types), m = 0. From liquid: keep f',
     * m = rho. */
    for (long i = 0; i < n; ++i) {
        if (newi[i] == 1) {
            double rs = 0, us[3] = {0, 0, 0};
            int cnt = 0;
            for (int q = 1; q < NQ; ++q) {
                long j = nbr(L, i, CX[q], CY[q], CZ[q]);
                if (!is_fluid(L->type[j])) continue;
                double fq[NQ], r, u[3];
                for (int s = 0; s < NQ; ++s) fq[s] = L->fnew[s * n + j];
                moments(fq, &r, u);
                rs += r; us[0] += u[0]; us[1] += u[1]; us[2] += u[2];
                cnt++;
            }
            double rm = rs / cnt, um[3] = {us[0] / cnt, us[1] / cnt, us[2] / cnt};
            for (int q = 0; q < NQ; ++q) L->fnew[q * n + i] = feq(q, rm, um);
            rnew[i] = rm;
            mnew[i] = 0.0;
        } else if (newi[i] == 2) {
            double r = 0.0;
            for (int q = 0; q < NQ; ++q) r += L->fnew[q * n + i];
            rnew[i] = r;
            mnew[i] = r;
        }
    }
    /* Types after the conversions, then the closure of the interface layer
     * on them: a cell of the layer without a gas neighbour leaves it as
     * liquid, one without a liquid neighbour as gas (none with frozen types). */
    unsigned char *t1 = (unsigned char *)calloc(n, 1);
    unsigned char *cl = (unsigned char *)calloc(n, 1);
    for (long i = 0; i < n; ++i) {
        t1[i] = L->type[i];
        if (L->type[i] == ORC_INTERFACE && st2[i] == ST_FILL) t1[i] = ORC_LIQUID;
        else if (L->type[i] == ORC_INTERFACE && st2[i] == ST_EMPTY) t1[i] = ORC_GAS;
        else if (newi[i]) t1[i] = ORC_INTERFACE;
    }
    if (!p->frozen) close_layer(L, t1, cl);
    /* Excess mass: every cell that leaves the interface layer in this step
     * (filled, emptied, or closed) hands on its excess, m - rho when it
     * becomes liquid and m when it becomes gas, with m and rho as they
     * stand before the redistribution (new cells from gas: m = 0, from
     * liquid: m = rho). It is split equally over the cell's D3Q19
     * neighbours that are interface cells after the step. With no such
     * neighbour the excess goes to a global reservoir. */
    double *share = (double *)calloc(n, sizeof(double));
    for (long i = 0; i < n; ++i) {
        int to_liq = (L->type[i] == ORC_INTERFACE && st2[i] == ST_FILL) || cl[i] == 1;
        int to_gas = (L->type[i] == ORC_INTERFACE && st2[i] == ST_EMPTY) || cl[i] == 2;
        if (!to_liq && !to_gas) continue;
        double mex = to_liq ? mnew[i] - rnew[i] : mnew[i];
        int cnt = 0;
        for (int q = 1; q < NQ; ++q) {
            long j = nbr(L, i, CX[q], CY[q], CZ[q]);
            cnt += t1[j] == ORC_INTERFACE && cl[j] == 0;
        }
        if (cnt > 0) share[i] = mex / cnt;
        else L->reservoir += mex;
    }
    for (long i = 0; i < n; ++i) {
        if (!(t1[i] == ORC_INTERFACE && cl[i] == 0)) continue;
        double acc = 0.0;
        for (int q = 1; q < NQ; ++q) {
            long j = nbr(L, i, CX[q], CY[q], CZ[q]);
            int leaves = (L->type[j] == ORC_INTERFACE && st2[j] != ST_NONE) || cl[j] != 0;
            if (leaves) acc += share[j];
        }
        mnew[i] = mnew[i] + acc;
    }
    for (long i = 0; i < n; ++i) {
        L->type[i] = t1[i];
        if (cl[i] == 1) L->type[i] = ORC_LIQUID;
        else if (cl[i] == 2) L->type[i] = ORC_GAS;
    }
    free(t1); free(cl);
    /* Phase 4: new state and fill levels. */
    double *tmp = L->f; L->f = L->fnew; L->fnew = tmp;
    for (long i = 0; i < n; ++i) {
        switch (L->type[i]) {
        case ORC_INTERFACE:
            L->m[i] = mnew[i];
            L->rho[i] = rnew[i];
            L->phi[i] = mnew[i] / rnew[i];
            break;
        case ORC_LIQUID: L->phi[i] = 1.0; L->m[i] = 0.0; L->rho[i] = 0.0; break;
        case ORC_GAS: L->phi[i] = 0.0; L->m[i] = 0.0; L->rho[i] = 0.0; break;
        default: break;
        }
    }
    obstacle_fill(L);
    update_gas_density(L);
    /* Phase 5: curvature for the next step's pressure jump. */
    curvature(L);
    free(mnew); free(rnew); free(st); free(st2); free(newi); free(share);
}

void orc_step(orc_lattice *L, long nsteps)
{
    for (long s = 0; s < nsteps; ++s) one_step(L);
}

/* ---- read-outs ---------------------------------------------------------- */
void orc_get_fill(const orc_lattice *L, double *out) { memcpy(out, L->phi, sizeof(double) * L->n); }
void orc_get_flags(const orc_lattice *L, unsigned char *out) { memcpy(out, L->type, L->n); }
void orc_get_curvature(const orc_lattice *L, double *out) { memcpy(out, L->K, sizeof(double) * L->n); }
void orc_get_plic(const orc_lattice *L, double *out) { memcpy(out, L->plic, sizeof(double) * L->n); }
void orc_get_mass_field(const orc_lattice *L, double *out) { memcpy(out, L->m, sizeof(double) * L->n); }
double orc_get_reservoir(const orc_lattice *L) { return L->reservoir; }
double orc_get_gas_density(const orc_lattice *L) { return L->rho_g; }

void orc_get_normal(const orc_lattice *L, double *out3)
{
    for (long i = 0; i < L->n; ++i)
        for (int k = 0; k < 3; ++k) out3[k * L->n + i] = L->nrm[3 * i + k];
}

void orc_get_density(const orc_lattice *L, double *out)
{
    for (long i = 0; i < L->n; ++i) {
        if (is_fluid(L->type[i])) {
            double r = 0.0;
            for (int q = 0; q < NQ; ++q) r += L->f[q * L->n + i];
            out[i] = r;
        } else {
            out[i] = L->type[i] == ORC_GAS ? L->rho_g : 0.0;
        }
    }
}

void orc_get_velocity(const orc_lattice *L, double *out3)
{
    long n = L->n;
    for (long i = 0; i < n; ++i) {
        double u[3] = {0, 0, 0};
        if (is_fluid(L->type[i])) {
            double fq[NQ], r;
            for (int q = 0; q < NQ; ++q) fq[q] = L->f[q * n + i];
            moments(fq, &r, u);
        }
        for (int k = 0; k < 3; ++k) out3[k * n + i] = u[k];
    }
}

/* Total mass: liquid cells carry rho, interface cells m, plus the reservoir. */
double orc_get_mass(const orc_lattice *L)
{
    double M = 0.0;
    for (long i = 0; i < L->n; ++i) {
        if (L->type[i] == ORC_LIQUID) {
            double r = 0.0;
            for (int q = 0; q < NQ; ++q) r += L->f[q * L->n + i];
            M += r;
        } else if (L->type[i] == ORC_INTERFACE) {
            M += L->m[i];
        }
    }
    return M + L->reservoir;
}

long orc_interface_list(const orc_lattice *L, int *out)
{
    long c = 0;
    for (long i = 0; i < L->n; ++i)
        if (L->type[i] == ORC_INTERFACE) {
            if (out) out[c] = (int)i;
            c++;
        }
    return c;
}

void orc_get_pdf(const orc_lattice *L, double *out19n) { memcpy(out19n, L->f, sizeof(double) * NQ * L->n); }
void orc_set_pdf(orc_lattice *L, const double *in19n) { memcpy(L->f, in19n, sizeof(double) * NQ * L->n); }

/* Set f' = feq(rho, u) at every fluid cell (rho: n values, u: 3n
 * component-major); interface masses become m = phi * rho. Used to start
 * flows with a prescribed velocity field. */
void orc_set_equilibrium(orc_lattice *L, const double *rho, const double *u3)
{
    long n = L->n;
    for (long i = 0; i < n; ++i) {
        if (!is_fluid(L->type[i])) continue;
        double u[3] = {u3[i], u3[n + i], u3[2 * n + i]};
        for (int q = 0; q < NQ; ++q) L->f[q * n + i] = feq(q, rho[i], u);
        if (L->type[i] == ORC_INTERFACE) {
            L->rho[i] = rho[i];
            L->m[i] = L->phi[i] * rho[i];
        }
    }
}
