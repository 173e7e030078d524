// Interface geometry of the FSLBM step, all in FP64 whatever the storage
// precision:
//   - normals n = grad(phi) by Parker-Youngs central differences over the
//     3x3x3 block (eq. normal) and PLIC plane offsets a, with the cut volume
//     of the cell equal to phi, by bisection (Sec. II.B);
//   - FD curvature K = -div(n^) of the K8-mollified fill level (Sec. II.A,
//     eq. curvature);
//   - LSQR curvature: least-squares quadric through the PLIC points of the
//     3x3x3 block with J = 0, plus the wetting gradient condition at contact
//     points (Sec. II.C, eqs. LSQR-model, LSQR-error, anacurv, contactNormal,
//     contactConstraint), solved through FP64 normal equations by Cholesky.
#pragma once

#include "fslbm_convert.hpp"
#include "fslbm_device.hpp"

namespace fslbm {

// Parker-Youngs weights (1, 2, 1) across the two transverse directions.
__device__ inline double pyw(int d) { return d == 0 ? 2.0 : 1.0; }

// Unscaled PY gradient of a scalar field g (type R) at cell i.
template <class R>
__device__ inline void py_grad(const R *__restrict__ g, const Nbr &nb, double &gx, double &gy, double &gz)
{
    gx = gy = gz = 0.0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            const double w = pyw(a) * pyw(b);
            gx += w * (double(g[nb.at(1, a, b)]) - double(g[nb.at(-1, a, b)]));
            gy += w * (double(g[nb.at(a, 1, b)]) - double(g[nb.at(a, -1, b)]));
            gz += w * (double(g[nb.at(a, b, 1)]) - double(g[nb.at(a, b, -1)]));
        }
}

// --------------------------------------------------------------- PLIC
// Volume of {y in [0,1]^3 : s.y <= t} for 0 <= s1 <= s2 <= s3, s1+s2+s3 = 1
// (from the corner expansion [t^3 - sum (t-s_i)_+^3 + ...] / (6 s1 s2 s3),
// with each case rearranged so that only s2*s3 >= 0 divides, and the
// complement for t > 1/2).
__device__ inline double cube_cut_below(double s1, double s2, double s3, double t)
{
    bool flip = false;
    if (t > 0.5) { t = 1.0 - t; flip = true; }
    double v;
    if (t <= 0.0) {
        v = 0.0;
    } else if (t <= s1) {
        v = t * t * (t / s1) / (6.0 * s2 * s3);
    } else if (t <= s2) {
        v = (3.0 * t * t - 3.0 * t * s1 + s1 * s1) / (6.0 * s2 * s3);
    } else if (t <= s1 + s2) {
        const double e2 = t - s2;
        double num = 3.0 * t * t - 3.0 * t * s1 + s1 * s1 - e2 * e2 * (e2 / s1);
        if (t > s3) {
            const double e3 = t - s3;
            num -= e3 * e3 * (e3 / s1);
        }
        v = num / (6.0 * s2 * s3);
    } else {
        v = (2.0 * t - s1 - s2) / (2.0 * s3);
    }
    return flip ? 1.0 - v : v;
}

// Plane offset a (point p = centre + a n) whose liquid side n.(x - centre) >= a
// cuts volume phi out of the unit cell: 42 bisection halvings of
// [-|n|_1/2, |n|_1/2] (bracket below 4e-13, Sec. II.B).
__device__ inline double plic_offset(double nx, double ny, double nz, double phi)
{
    double m0 = fabs(nx), m1 = fabs(ny), m2 = fabs(nz);
    const double l1 = m0 + m1 + m2;
    if (!(l1 > 0.0)) return 0.0;
    phi = fmin(fmax(phi, 0.0), 1.0);
    m0 /= l1; m1 /= l1; m2 /= l1;
    // sort ascending
    if (m0 > m1) { const double t = m0; m0 = m1; m1 = t; }
    if (m1 > m2) { const double t = m1; m1 = m2; m2 = t; }
    if (m0 > m1) { const double t = m0; m0 = m1; m1 = t; }
    double lo = -0.5 * l1, hi = 0.5 * l1;
    for (int it = 0; it < 42; ++it) {
        const double mid = 0.5 * (lo + hi);
        // liquid volume at offset mid equals V(1/2 - mid/l1)
        if (cube_cut_below(m0, m1, m2, 0.5 - mid / l1) > phi) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

template <class P>
__global__ __launch_bounds__(256) void k_normals_plic(Fields<P> F)
{
    using R = typename P::R;
    const int n = list_count(F.sc);
    const size_t N = F.N;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        const Nbr nb(i, F.nx, F.ny, F.nz);
        double gx, gy, gz;
        py_grad(F.phi, nb, gx, gy, gz);
        const double len = sqrt(gx * gx + gy * gy + gz * gz);
        double nx = 0, ny = 0, nz = 0, a = 0;
        if (len > 1e-12) {
            nx = gx / len; ny = gy / len; nz = gz / len;
            a = plic_offset(nx, ny, nz, double(F.phi[i]));
        }
        F.nrm[i] = R(nx);
        F.nrm[N + i] = R(ny);
        F.nrm[2 * N + i] = R(nz);
        F.plic[i] = R(a);
    }
}

// ----------------------------------------------------------- FD model
// K8 kernel of support 2 on the 27-point block: (1 - r^2/4)^4 gives
// 256, 81, 16, 1 (times 1/256) for r^2 = 0, 1, 2, 3; normalised by 942.
__device__ inline double k8w(int r2) { return r2 == 0 ? 256.0 : (r2 == 1 ? 81.0 : (r2 == 2 ? 16.0 : 1.0)); }

template <class P>
__global__ __launch_bounds__(256) void k_fd_mollify(Fields<P> F)
{
    using R = typename P::R;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    const Nbr nb(i, F.nx, F.ny, F.nz);
    double s = 0.0;
#pragma unroll
    for (int c = -1; c <= 1; ++c)
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int a = -1; a <= 1; ++a) s += k8w(a * a + b * b + c * c) * double(F.phi[nb.at(a, b, c)]);
    F.phis[i] = R(s / 942.0);
}

template <class P>
__global__ __launch_bounds__(256) void k_fd_normals(Fields<P> F)
{
    using R = typename P::R;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    const Nbr nb(i, F.nx, F.ny, F.nz);
    double gx, gy, gz;
    py_grad(F.phis, nb, gx, gy, gz);
    const double len = sqrt(gx * gx + gy * gy + gz * gz);
    const size_t N = F.N;
    const bool ok = len > 1e-12;
    F.nmol[i] = R(ok ? gx / len : 0.0);
    F.nmol[N + i] = R(ok ? gy / len : 0.0);
    F.nmol[2 * N + i] = R(ok ? gz / len : 0.0);
}

// K = -div(n^) with the PY-weighted central difference scaled to a
// derivative: 1/16 for the transverse weights, 1/2 for the difference.
template <class P>
__global__ __launch_bounds__(256) void k_fd_curvature(Fields<P> F)
{
    using R = typename P::R;
    const int n = list_count(F.sc);
    const size_t N = F.N;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        const Nbr nb(i, F.nx, F.ny, F.nz);
        const R *nxf = F.nmol, *nyf = F.nmol + N, *nzf = F.nmol + 2 * N;
        double dxx = 0, dyy = 0, dzz = 0;
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int b = -1; b <= 1; ++b) {
                const double w = pyw(a) * pyw(b);
                dxx += w * (double(nxf[nb.at(1, a, b)]) - double(nxf[nb.at(-1, a, b)]));
                dyy += w * (double(nyf[nb.at(a, 1, b)]) - double(nyf[nb.at(a, -1, b)]));
                dzz += w * (double(nzf[nb.at(a, b, 1)]) - double(nzf[nb.at(a, b, -1)]));
            }
        F.K[i] = R(-((dxx + dyy + dzz) / 32.0));
    }
}

// --------------------------------------------------------- LSQR model
// Normal equations of the least-squares fit, accumulated row by row.
template <int C> struct Gram {
    double G[C][C];
    double g[C];
    __device__ inline Gram()
    {
#pragma unroll
        for (int r = 0; r < C; ++r) {
            g[r] = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) G[r][c] = 0.0;
        }
    }
    __device__ inline void add(const double (&a)[C], double b)
    {
#pragma unroll
        for (int r = 0; r < C; ++r) {
            g[r] += a[r] * b;
#pragma unroll
            for (int c = 0; c <= r; ++c) G[r][c] += a[r] * a[c];
        }
    }
    // Cholesky solve; fails when a pivot falls below 1e-12 * trace(G)
    // (rank deficiency of the row matrix).
    __device__ inline bool solve(double (&x)[C]) const
    {
        double tr = 0.0;
#pragma unroll
        for (int r = 0; r < C; ++r) tr += G[r][r];
        if (!(tr > 0.0)) return false;
        double L[C][C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            double d = G[c][c];
#pragma unroll
            for (int j = 0; j < c; ++j) d -= L[c][j] * L[c][j];
            if (!(d >= 1e-12 * tr)) return false;
            L[c][c] = sqrt(d);
#pragma unroll
            for (int r = c + 1; r < C; ++r) {
                double s = G[r][c];
#pragma unroll
                for (int j = 0; j < c; ++j) s -= L[r][j] * L[c][j];
                L[r][c] = s / L[c][c];
            }
        }
        double y[C];
#pragma unroll
        for (int r = 0; r < C; ++r) {
            double s = g[r];
#pragma unroll
            for (int j = 0; j < r; ++j) s -= L[r][j] * y[j];
            y[r] = s / L[r][r];
        }
#pragma unroll
        for (int r = C - 1; r >= 0; --r) {
            double s = y[r];
#pragma unroll
            for (int j = r + 1; j < C; ++j) s -= L[j][r] * x[j];
            x[r] = s / L[r][r];
        }
        return true;
    }
};

__device__ inline double dot(const double (&a)[3], const double (&b)[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

template <class P>
__device__ inline void load_normal(const Fields<P> &F, int j, double (&n)[3])
{
    const size_t N = F.N;
    n[0] = double(F.nrm[j]);
    n[1] = double(F.nrm[N + j]);
    n[2] = double(F.nrm[2 * N + j]);
}

// Contact point and contact normal of contact-line cell j at offset d from
// the centre (eqs. contactNormal, contactConstraint; Fig. contactPoint).
// Returns false when the condition is skipped.
template <class P>
__device__ inline bool contact_condition(const Fields<P> &F, int j, int dx, int dy, int dz, const double (&pc)[3],
                                         const double (&nc)[3], const double (&tu)[3], const double (&tv)[3],
                                         const Params &prm, double &uc, double &vc, double &ru, double &rv)
{
    double nj[3];
    load_normal(F, j, nj);
    if (nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0) return false;
    const Nbr nb(j, F.nx, F.ny, F.nz);
    int sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q)
        if (F.flags[nb.at(dir_x(q), dir_y(q), dir_z(q))] & FL_OBST) {
            sx += dir_x(q); sy += dir_y(q); sz += dir_z(q);
        }
    const double lw = sqrt(double(sx * sx + sy * sy + sz * sz));
    if (!(lw > 0.0)) return false;
    const double nw[3] = {sx / lw, sy / lw, sz / lw};
    const double nn = dot(nj, nw);
    double nt[3] = {nj[0] - nn * nw[0], nj[1] - nn * nw[1], nj[2] - nn * nw[2]};
    const double lt = sqrt(dot(nt, nt));
    if (lt < 1e-12) return false;
    nt[0] /= lt; nt[1] /= lt; nt[2] /= lt;
    const double mh[3] = {nw[0] * prm.cos_theta + nt[0] * prm.sin_theta, nw[1] * prm.cos_theta + nt[1] * prm.sin_theta,
                          nw[2] * prm.cos_theta + nt[2] * prm.sin_theta};
    const double g[3] = {nw[0] - nn * nj[0], nw[1] - nn * nj[1], nw[2] - nn * nj[2]};
    const double gn = dot(g, nw);
    if (gn < 1e-12) return false;
    const double aj = double(F.plic[j]);
    const double pj[3] = {aj * nj[0], aj * nj[1], aj * nj[2]};
    const double t = (0.5 - dot(pj, nw)) / gn;
    const double r[3] = {dx + pj[0] + t * g[0] - pc[0], dy + pj[1] + t * g[1] - pc[1], dz + pj[2] + t * g[2] - pc[2]};
    uc = dot(r, tu);
    vc = dot(r, tv);
    const double mu = dot(mh, tu), mv = dot(mh, tv), mn = dot(mh, nc);
    if (fabs(mn) < 1e-6) return false;
    ru = -mu / mn;
    rv = -mv / mn;
    return true;
}

template <class P>
__global__ __launch_bounds__(256) void k_curv_lsqr(Fields<P> F, Params prm)
{
    using R = typename P::R;
    const int n = list_count(F.sc);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        double nc[3];
        load_normal(F, i, nc);
        if (nc[0] == 0.0 && nc[1] == 0.0 && nc[2] == 0.0) {
            F.K[i] = R(0);
            continue;
        }
        // frame: t_u from the axis with the smallest |n_k| (first on ties)
        int ax = 0;
        if (fabs(nc[1]) < fabs(nc[ax])) ax = 1;
        if (fabs(nc[2]) < fabs(nc[ax])) ax = 2;
        double tu[3] = {-nc[ax] * nc[0], -nc[ax] * nc[1], -nc[ax] * nc[2]};
        tu[ax] += 1.0;
        const double ltu = sqrt(dot(tu, tu));
        tu[0] /= ltu; tu[1] /= ltu; tu[2] /= ltu;
        const double tv[3] = {nc[1] * tu[2] - nc[2] * tu[1], nc[2] * tu[0] - nc[0] * tu[2], nc[0] * tu[1] - nc[1] * tu[0]};
        const double ac = double(F.plic[i]);
        const double pc[3] = {ac * nc[0], ac * nc[1], ac * nc[2]};
        const Nbr nb(i, F.nx, F.ny, F.nz);
        bool has_obst = false;
#pragma unroll
        for (int c = -1; c <= 1; ++c)
#pragma unroll
            for (int b = -1; b <= 1; ++b)
#pragma unroll
                for (int a = -1; a <= 1; ++a) has_obst |= (F.flags[nb.at(a, b, c)] & FL_OBST) != 0;

        // hard constraint of the centre: H = hu - 2 uc A - vc C, I = hv - 2 vc B - uc C
        bool hard = false;
        double huc = 0, hvc = 0, hu = 0, hv = 0;
        if (has_obst && (F.flags[i] & FL_NEAR_OBST))
            hard = contact_condition(F, i, 0, 0, 0, pc, nc, tu, tv, prm, huc, hvc, hu, hv);

        Gram<5> g5;  // free model (A, B, C, H, I)
        Gram<3> g3;  // free: isotropic (A, H, I); hard: (A, B, C)
        Gram<1> g1;  // hard isotropic (A)
        int rows = 0;
        auto add_row = [&](double r0, double r1, double r2, double r3, double r4, double b) {
            ++rows;
            if (!hard) {
                const double a5[5] = {r0, r1, r2, r3, r4};
                g5.add(a5, b);
                const double a3[3] = {r0 + r1, r3, r4};
                g3.add(a3, b);
            } else {
                const double e0 = r0 - r3 * (2.0 * huc), e1 = r1 - r4 * (2.0 * hvc);
                const double e2 = r2 - r3 * hvc - r4 * huc;
                const double be = b - r3 * hu - r4 * hv;
                const double a3[3] = {e0, e1, e2};
                g3.add(a3, be);
                const double a1[1] = {e0 + e1};
                g1.add(a1, be);
            }
        };
        // data rows: PLIC points of the other interface cells of the block
        for (int c = -1; c <= 1; ++c)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    if (a == 0 && b == 0 && c == 0) continue;
                    const int j = nb.at(a, b, c);
                    if (!(F.flags[j] & FL_IF)) continue;
                    double nj[3];
                    load_normal(F, j, nj);
                    if (nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0) continue;
                    const double aj = double(F.plic[j]);
                    const double r[3] = {a + aj * nj[0] - pc[0], b + aj * nj[1] - pc[1], c + aj * nj[2] - pc[2]};
                    const double u = dot(r, tu), v = dot(r, tv), w = dot(r, nc);
                    add_row(u * u, v * v, u * v, u, v, w);
                }
        // wetting rows of the other contact-line cells
        if (has_obst) {
            for (int c = -1; c <= 1; ++c)
                for (int b = -1; b <= 1; ++b)
                    for (int a = -1; a <= 1; ++a) {
                        if (a == 0 && b == 0 && c == 0) continue;
                        const int j = nb.at(a, b, c);
                        const uint8_t fj = F.flags[j];
                        if (!((fj & FL_IF) && (fj & FL_NEAR_OBST))) continue;
                        double uc, vc, ru, rv;
                        if (!contact_condition(F, j, a, b, c, pc, nc, tu, tv, prm, uc, vc, ru, rv)) continue;
                        add_row(2.0 * uc, 0.0, vc, 1.0, 0.0, ru);
                        add_row(0.0, 2.0 * vc, uc, 0.0, 1.0, rv);
                    }
        }
        double A = 0, B = 0, C = 0, H = 0, I = 0;
        bool ok = false;
        if (!hard) {
            double x5[5];
            if (rows >= 5 && g5.solve(x5)) {
                A = x5[0]; B = x5[1]; C = x5[2]; H = x5[3]; I = x5[4];
                ok = true;
            } else {
                double x3[3];
                if (rows >= 3 && g3.solve(x3)) {
                    A = x3[0]; B = x3[0]; C = 0.0; H = x3[1]; I = x3[2];
                    ok = true;
                }
            }
        } else {
            double x3[3];
            if (rows >= 3 && g3.solve(x3)) {
                A = x3[0]; B = x3[1]; C = x3[2];
                ok = true;
            } else {
                double x1[1];
                if (rows >= 1 && g1.solve(x1)) {
                    A = x1[0]; B = x1[0]; C = 0.0;
                    ok = true;
                }
            }
            H = hu - 2.0 * huc * A - hvc * C;
            I = hv - 2.0 * hvc * B - huc * C;
        }
        double K = 0.0;
        if (ok) {
            const double gg = 1.0 + H * H + I * I;
            K = 2.0 * (A * (1.0 + I * I) + B * (1.0 + H * H) - C * H * I) / (gg * sqrt(gg));
        }
        F.K[i] = R(K);
    }
}

}  // namespace fslbm
