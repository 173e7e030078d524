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
// Both models run tile by tile: one workgroup takes an 8^3 tile of the
// interface bounding box, stages the fill level (and cell flags) of the tile
// and its halo in LDS with coalesced loads, and computes every stencil of
// the tile from LDS.
#pragma once

#include "fslbm_convert.hpp"
#include "fslbm_device.hpp"

namespace fslbm {

// Parker-Youngs weights (1, 2, 1) across the two transverse directions.
__host__ __device__ inline double pyw(int d) { return d == 0 ? 2.0 : 1.0; }

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
// Volume V(t) of {y in [0,1]^3 : s.y <= t} for 0 <= s1 <= s2 <= s3,
// s1+s2+s3 = 1, and its slope, from the corner expansion
// [t^3 - sum (t-s_i)_+^3 + ...] / (6 s1 s2 s3) with each case rearranged so
// that no small s_i divides alone; t > 1/2 by the point reflection
// V(t) = 1 - V(1-t), V'(t) = V'(1-t). Reciprocals are taken once per cell.
template <class G> struct CubeCut {
    G s1, s2, s3, r1, r23, r3;  // r1 = 1/s1, r23 = 1/(6 s2 s3), r3 = 1/(2 s3)
    __host__ __device__ inline CubeCut(G a, G b, G c) : s1(a), s2(b), s3(c)
    {
        r1 = s1 > G(0) ? G(1) / s1 : G(0);
        r23 = s2 > G(0) ? G(1) / (G(6) * s2 * s3) : G(0);
        r3 = G(1) / (G(2) * s3);
    }
    __host__ __device__ inline void eval(G t, G &v, G &dv) const
    {
        const bool flip = t > G(0.5);
        if (flip) t = G(1) - t;
        if (t <= G(0)) {
            v = G(0);
            dv = G(0);
        } else if (t <= s1) {  // corner tetrahedron
            v = t * t * (t * r1) * r23;
            dv = G(3) * t * t * r1 * r23;
        } else if (t <= s2) {
            v = (G(3) * t * t - G(3) * t * s1 + s1 * s1) * r23;
            dv = (G(6) * t - G(3) * s1) * r23;
        } else if (t <= s1 + s2) {
            const G e2 = t - s2;
            G num = G(3) * t * t - G(3) * t * s1 + s1 * s1 - e2 * e2 * (e2 * r1);
            G den = G(6) * t - G(3) * s1 - G(3) * e2 * e2 * r1;
            if (t > s3) {
                const G e3 = t - s3;
                num -= e3 * e3 * (e3 * r1);
                den -= G(3) * e3 * e3 * r1;
            }
            v = num * r23;
            dv = den * r23;
        } else {  // the plane cuts all four edges along y3
            v = (G(2) * t - s1 - s2) * r3;
            dv = G(2) * r3;
        }
        if (flip) v = G(1) - v;
    }
};

// Plane offset a (point p = centre + a n) whose liquid side n.(x - centre) >= a
// cuts volume phi out of the unit cell (Sec. II.B). The liquid volume at
// offset a is V(1/2 - a/|n|_1). For phi <= 1/2 (else by the point
// reflection) the root t <= 1/2 of V(t) = phi is found piece by piece: the
// corner tetrahedron (t <= s1: a cube root), the wedge (s1 <= t <= s2: a
// quadratic) and the prism (t >= s1 + s2: linear) in closed form; the cubic
// piece in between by Newton steps kept inside its bracket, started from the
// wedge's root and stopped when a step falls below the type's resolution
// (at most 5 steps; 3 on most cells). This reaches the root to rounding
// (3.5e-16 in FP64 against an extended-precision solve over 200,000 random
// normals and fills), within the 4e-13 bound of the paper's 40-step
// bisection.
template <class G>
__host__ __device__ inline G plic_offset(G nx, G ny, G nz, G phi)
{
    G m0 = fabs(nx), m1 = fabs(ny), m2 = fabs(nz);
    const G l1 = m0 + m1 + m2;
    if (!(l1 > G(0))) return G(0);
    phi = fmin(fmax(phi, G(0)), G(1));
    const G il1 = G(1) / l1;
    m0 *= il1; m1 *= il1; m2 *= il1;
    if (m0 > m1) { const G t = m0; m0 = m1; m1 = t; }
    if (m1 > m2) { const G t = m1; m1 = m2; m2 = t; }
    if (m0 > m1) { const G t = m0; m0 = m1; m1 = t; }
    const G s1 = m0, s2 = m1, s3 = m2;
    const bool flip = phi > G(0.5);
    const G p = flip ? G(1) - phi : phi;
    G t;
    if (!(s2 > G(0))) {
        t = p;  // normal along an axis: V(t) = t
    } else {
        const G d = G(6) * s2 * s3;
        const G v1 = s1 * s1 / d;                                   // V(s1)
        const G v2 = (G(3) * s2 * s2 - G(3) * s2 * s1 + s1 * s1) / d;  // V(s2)
        const G wedge = (G(3) * s1 + sqrt(fmax(G(12) * d * p - G(3) * s1 * s1, G(0)))) / G(6);
        const G s12 = s1 + s2;
        if (p <= v1) {
            t = cbrt(d * s1 * p);
        } else if (p <= v2) {
            t = wedge;
        } else if (s12 <= G(0.5) && p >= s12 / (G(2) * s3)) {
            t = s3 * p + G(0.5) * s12;
        } else {
            const CubeCut<G> cut(s1, s2, s3);
            const G tol = sizeof(G) == 8 ? G(1e-15) : G(2e-7);
            G lo = s2, hi = fmin(s12, G(0.5));
            t = fmin(fmax(wedge, lo), hi);
            for (int it = 0; it < 40; ++it) {
                G v, dv;
                cut.eval(t, v, dv);
                v -= p;
                if (v <= G(0)) lo = t;  // V(lo) <= p
                else hi = t;            // V(hi) > p
                if (v == G(0) || hi - lo <= tol) break;
                G tn = dv > G(0) ? t - v / dv : G(-1);
                // converged: the Newton step is below the resolution (it
                // may land on a bracket end, which the fallback below would
                // reject and then bisect towards for many steps)
                if (dv > G(0) && fabs(tn - t) <= tol) {
                    t = fmin(fmax(tn, lo), hi);
                    break;
                }
                if (!(tn > lo && tn < hi)) tn = G(0.5) * (lo + hi);
                const G step = fabs(tn - t);
                t = tn;
                if (step <= tol) break;
            }
        }
    }
    if (flip) t = G(1) - t;
    return l1 * (G(0.5) - t);
}

// --------------------------------------------------------- LSQR model
// Normal equations of the least-squares fit, accumulated row by row.
template <int C> struct Gram {
    double G[C][C];
    double g[C];
    __host__ __device__ inline Gram()
    {
#pragma unroll
        for (int r = 0; r < C; ++r) {
            g[r] = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) G[r][c] = 0.0;
        }
    }
    __host__ __device__ inline void add(const double (&a)[C], double b)
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
    __host__ __device__ inline bool solve(double (&x)[C]) const
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


__host__ __device__ inline double dot(const double (&a)[3], const double (&b)[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

constexpr int TILE = 8;

// Tiles covering the interface bounding box; a tile cell is processed when
// its unwrapped coordinates lie inside the box (a box spanning a whole
// periodic axis would otherwise see wrapped cells twice).
struct Tiles {
    CellRange box;
    int tx, ty, tz;
    __device__ inline Tiles(const DevScalars *sc)
    {
        box = CellRange::from(sc->bbox);
        tx = (box.ex + TILE - 1) / TILE;
        ty = (box.ey + TILE - 1) / TILE;
        tz = (box.ez + TILE - 1) / TILE;
    }
    __device__ inline int count() const { return tx * ty * tz; }
    __device__ inline void origin(int t, int &ox, int &oy, int &oz) const
    {
        ox = box.x0 + TILE * (t % tx);
        oy = box.y0 + TILE * ((t / tx) % ty);
        oz = box.z0 + TILE * (t / (tx * ty));
    }
    __device__ inline bool inside(int ux, int uy, int uz) const
    {
        return ux < box.x0 + box.ex && uy < box.y0 + box.ey && uz < box.z0 + box.ez;
    }
};

__device__ inline int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ inline int gidx(int x, int y, int z, int nx, int ny, int nz)
{
    return wrapi(x, nx) + nx * (wrapi(y, ny) + ny * wrapi(z, nz));
}

// Does the tile hold an interface cell? (uniform across the workgroup)
template <class P>
__device__ inline bool tile_has_interface(const Fields<P> &F, const Tiles &T, int ox, int oy, int oz)
{
    int has = 0;
    for (int c = threadIdx.x; c < TILE * TILE * TILE; c += 256) {
        const int lx = c % TILE, ly = (c / TILE) % TILE, lz = c / (TILE * TILE);
        if (!T.inside(ox + lx, oy + ly, oz + lz)) continue;
        has |= F.flags[gidx(ox + lx, oy + ly, oz + lz, F.nx, F.ny, F.nz)] & FL_IF;
    }
    return __syncthreads_or(has) != 0;
}

// Unscaled Parker-Youngs gradient of an LDS cube of edge E at (x, y, z).
template <int E, class G, class A>
__device__ inline void py_grad_lds(const A &g, int x, int y, int z, G &gx, G &gy, G &gz)
{
    auto at = [&](int dx, int dy, int dz) { return g[((z + dz) * E + (y + dy)) * E + (x + dx)]; };
    gx = gy = gz = G(0);
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            const G w = G(pyw(a) * pyw(b));
            gx += w * (at(1, a, b) - at(-1, a, b));
            gy += w * (at(a, 1, b) - at(a, -1, b));
            gz += w * (at(a, b, 1) - at(a, b, -1));
        }
}

// Unit normal (zero when the gradient vanishes) from a PY gradient.
template <class G>
__host__ __device__ inline void unit_normal(G gx, G gy, G gz, G (&n)[3])
{
    const G len = sqrt(gx * gx + gy * gy + gz * gz);
    const bool ok = len > G(1e-12);
    const G il = ok ? G(1) / len : G(0);  // one division for the three components
    n[0] = gx * il;
    n[1] = gy * il;
    n[2] = gz * il;
}

template <class P, class G>
__device__ inline void store_normal(const Fields<P> &F, int i, const G (&n)[3], G a)
{
    using R = typename P::R;
    const size_t N = F.N;
    F.nrm[i] = R(n[0]);
    F.nrm[N + i] = R(n[1]);
    F.nrm[2 * N + i] = R(n[2]);
    F.plic[i] = R(a);
}

// K8 kernel of support 2 on the 27-point block: (1 - r^2/4)^4 gives
// 256, 81, 16, 1 (times 1/256) for r^2 = 0, 1, 2, 3; normalised by 942.
__device__ inline double k8w(int r2) { return r2 == 0 ? 256.0 : (r2 == 1 ? 81.0 : (r2 == 2 ? 16.0 : 1.0)); }
// 1 / (the sum of the K8 weights, 256 + 6 81 + 12 16 + 8 = 942): the
// mollified value is the weighted sum times this factor
constexpr double K8_INV = 1.0 / 942.0;


// FD model, one 8^3 tile per iteration. LDS: the fill level on the tile
// grown by 3 (14^3), the mollified fill level grown by 2 (12^3) and the
// mollified unit normals grown by 1 (10^3, reusing the fill-level space).
// The raw-fill normals of the tile's interface cells (for the corner rule)
// come from the same LDS copy.
template <class G> struct FdLds {
    G buf[3000];  // phi 14^3 (origin -3), later normals 3 x 10^3 (origin -1)
    G mol[1728];  // mollified phi 12^3 (origin -2)
};

// Unit normal of the K8-mollified fill level at cell j, from global memory,
// with the same operations in the same order as the tiled FD kernel.
template <class P>
__device__ inline void fd_mollified_normal(const Fields<P> &F, int j, typename P::G (&n)[3])
{
    using G = typename P::G;
    const Nbr nj(j, F.nx, F.ny, F.nz);
    G m[27];
#pragma unroll
    for (int c = -1; c <= 1; ++c)
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int a = -1; a <= 1; ++a) {
                const Nbr nk(nj.at(a, b, c), F.nx, F.ny, F.nz);
                G s = G(0);
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx)
                            s += G(k8w(dx * dx + dy * dy + dz * dz)) * G(F.phi[nk.at(dx, dy, dz)]);
                m[(c + 1) * 9 + (b + 1) * 3 + (a + 1)] = s * G(K8_INV);
            }
    auto at = [&](int dx, int dy, int dz) { return m[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)]; };
    G gx = G(0), gy = G(0), gz = G(0);
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            const G w = G(pyw(a) * pyw(b));
            gx += w * (at(1, a, b) - at(-1, a, b));
            gy += w * (at(a, 1, b) - at(a, -1, b));
            gz += w * (at(a, b, 1) - at(a, b, -1));
        }
    unit_normal(gx, gy, gz, n);
}

// FD wetting (Sec. II.A, eq. contactNormal) at obstacle cell o: w is the
// normalised sum of the directions to its non-obstacle neighbours (out of
// the wall) and x_b = o + c_qb the neighbour along the lattice direction
// closest to w (the first on ties). Returns qb, or 0 when x_b is an
// obstacle cell (a base cell of any other type carries the wall value when
// its mollified normal is nonzero).
template <class P>
__device__ inline int fd_contact_base(const Fields<P> &F, const Nbr &no, typename P::G (&w)[3])
{
    using G = typename P::G;
    int sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q)
        if (!(F.flags[no.at(dir_x(q), dir_y(q), dir_z(q))] & FL_OBST)) {
            sx += dir_x(q); sy += dir_y(q); sz += dir_z(q);
        }
    const G lw = sqrt(G(sx * sx + sy * sy + sz * sz));
    if (!(lw > G(0))) return 0;
    w[0] = G(sx) / lw; w[1] = G(sy) / lw; w[2] = G(sz) / lw;
    int qb = 0;
    G best = G(-2);
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const G cl = sqrt(G(dir_len2(q)));
        const G a = (G(dir_x(q)) * w[0] + G(dir_y(q)) * w[1] + G(dir_z(q)) * w[2]) / cl;
        if (a > best) { best = a; qb = q; }
    }
    return (F.flags[no.at(dir_x(qb), dir_y(qb), dir_z(qb))] & FL_OBST) ? 0 : qb;
}

// The wall value m = n_w cos(theta) + n_t sin(theta) (n_w = -w into the wall,
// n_t the normalised projection of the base cell's mollified normal n_b onto
// the wall), extrapolated to the obstacle node half a cell beyond the wall:
// n = normalise(2 m - n_b). False when n_b has no component along the wall.
template <class G>
__device__ inline bool fd_contact_normal(const G (&w)[3], const G (&nb)[3], G ct, G st, G (&out)[3])
{
    const G nw[3] = {-w[0], -w[1], -w[2]};
    const G nn = nb[0] * nw[0] + nb[1] * nw[1] + nb[2] * nw[2];
    G nt[3] = {nb[0] - nn * nw[0], nb[1] - nn * nw[1], nb[2] - nn * nw[2]};
    const G lt = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
    if (lt < G(1e-12)) return false;
    nt[0] /= lt; nt[1] /= lt; nt[2] /= lt;
    G e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) e[k] = G(2) * (nw[k] * ct + nt[k] * st) - nb[k];
    const G le = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (le < G(1e-12)) return false;
    out[0] = e[0] / le; out[1] = e[1] / le; out[2] = e[2] / le;
    return true;
}

// Contact normals of the obstacle-list cells of FD lattices (0 where none).
template <class P>
__global__ __launch_bounds__(256) void k_fd_contact_normals(const Batch<P> B, int eos)
{
    const Params &prm = B.p[blockIdx.y];
    end_of_step(B.f[blockIdx.y].sc, eos);
    if (prm.curv != 0) return;
    const Fields<P> &F = B.f[blockIdx.y];
    using G = typename P::G;
    using R = typename P::R;
    const int n = F.sc->ocount;
    const size_t N = F.N;
    const G ct = G(prm.cos_theta), st = G(prm.sin_theta);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int o = F.olist[k];
        const Nbr no(o, F.nx, F.ny, F.nz);
        G w[3], out[3] = {G(0), G(0), G(0)};
        const int qb = fd_contact_base(F, no, w);
        if (qb) {
            G nb[3];
            fd_mollified_normal(F, no.at(dir_x(qb), dir_y(qb), dir_z(qb)), nb);
            if (nb[0] != G(0) || nb[1] != G(0) || nb[2] != G(0)) {
                G c[3];
                if (fd_contact_normal(w, nb, ct, st, c)) { out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; }
            }
        }
        F.cnrm[o] = R(out[0]);
        F.cnrm[N + o] = R(out[1]);
        F.cnrm[2 * N + o] = R(out[2]);
    }
}

template <class P>
__device__ inline void geometry_fd_tiles(const Fields<P> &F)
{
    using R = typename P::R;
    using G = typename P::G;
    __shared__ FdLds<G> L;
    const Tiles T(F.sc);
    const int nt = T.count();
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        int ox, oy, oz;
        T.origin(t, ox, oy, oz);
        __syncthreads();
        if (!tile_has_interface(F, T, ox, oy, oz)) continue;
        // the fill level on the 14^3 block: thread c < 196 takes column
        // (x, y) = (c % 14, c / 14) and walks it in z with a running plane
        // offset (no index division or product per element)
        if (threadIdx.x < 196) {
            const int c = threadIdx.x, x = c % 14, y = c / 14;
            const int col = wrapi(ox - 3 + x, F.nx) + F.nx * wrapi(oy - 3 + y, F.ny);
            const int nxy = F.nx * F.ny;
            int zoff = wrapi(oz - 3, F.nz) * nxy;
#pragma unroll
            for (int z = 0; z < 14; ++z) {
                L.buf[z * 196 + c] = G(F.phi[col + zoff]);
                zoff += nxy;
                if (zoff >= F.N) zoff -= F.N;
            }
        }
        __syncthreads();
        // raw-fill normals of the tile's interface cells
        for (int c = threadIdx.x; c < 512; c += 256) {
            const int lx = c % 8, ly = (c / 8) % 8, lz = c / 64;
            if (!T.inside(ox + lx, oy + ly, oz + lz)) continue;
            const int i = gidx(ox + lx, oy + ly, oz + lz, F.nx, F.ny, F.nz);
            if (!(F.flags[i] & FL_IF)) continue;
            G gx, gy, gz, n[3];
            py_grad_lds<14>(L.buf, lx + 3, ly + 3, lz + 3, gx, gy, gz);
            unit_normal(gx, gy, gz, n);
            store_normal(F, i, n, G(0));
        }
        // K8 mollification on 12^3
        for (int c = threadIdx.x; c < 1728; c += 256) {
            const int x = c % 12, y = (c / 12) % 12, z = c / 144;
            G s = G(0);
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx)
                        s += G(k8w(dx * dx + dy * dy + dz * dz)) * L.buf[((z + 1 + dz) * 14 + y + 1 + dy) * 14 + x + 1 + dx];
            L.mol[c] = s * G(K8_INV);
        }
        __syncthreads();
        // unit normals of the mollified field on 10^3; obstacle cells with a
        // contact normal (FD wetting) take it instead
        const bool walls = F.sc->ocount > 0;
        for (int c = threadIdx.x; c < 1000; c += 256) {
            const int x = c % 10, y = (c / 10) % 10, z = c / 100;
            G gx, gy, gz, n[3];
            py_grad_lds<12>(L.mol, x + 1, y + 1, z + 1, gx, gy, gz);
            unit_normal(gx, gy, gz, n);
            if (walls) {
                const int gi = gidx(ox - 1 + x, oy - 1 + y, oz - 1 + z, F.nx, F.ny, F.nz);
                if (F.flags[gi] & FL_OBST) {
                    const size_t N = F.N;
                    const G c0 = G(F.cnrm[gi]), c1 = G(F.cnrm[N + gi]), c2 = G(F.cnrm[2 * N + gi]);
                    if (c0 != G(0) || c1 != G(0) || c2 != G(0)) { n[0] = c0; n[1] = c1; n[2] = c2; }
                }
            }
            L.buf[c] = n[0];
            L.buf[1000 + c] = n[1];
            L.buf[2000 + c] = n[2];
        }
        __syncthreads();
        // K = -div(n^), PY-weighted central differences scaled by 1/32
        for (int c = threadIdx.x; c < 512; c += 256) {
            const int lx = c % 8, ly = (c / 8) % 8, lz = c / 64;
            if (!T.inside(ox + lx, oy + ly, oz + lz)) continue;
            const int i = gidx(ox + lx, oy + ly, oz + lz, F.nx, F.ny, F.nz);
            if (!(F.flags[i] & FL_IF)) continue;
            G dxx = 0, dyy = 0, dzz = 0;
            auto at = [&](int comp, int dx, int dy, int dz) {
                return L.buf[comp * 1000 + ((lz + 1 + dz) * 10 + ly + 1 + dy) * 10 + lx + 1 + dx];
            };
#pragma unroll
            for (int a = -1; a <= 1; ++a)
#pragma unroll
                for (int b = -1; b <= 1; ++b) {
                    const G w = G(pyw(a) * pyw(b));
                    dxx += w * (at(0, 1, a, b) - at(0, -1, a, b));
                    dyy += w * (at(1, a, 1, b) - at(1, a, -1, b));
                    dzz += w * (at(2, a, b, 1) - at(2, a, b, -1));
                }
            F.K[i] = R(-((dxx + dyy + dzz) / G(32)));
        }
    }
}

template <class P>
__global__ __launch_bounds__(256) void k_geometry_fd(const Batch<P> B, int eos)
{
    end_of_step(B.f[blockIdx.y].sc, eos);
    if (B.p[blockIdx.y].curv != 0) return;
    geometry_fd_tiles(B.f[blockIdx.y]);
}

// LSQR model: one thread per interface cell over the interface list (the
// fit is FP64 arithmetic with long dependency chains, so full wavefronts
// matter more than load coalescing). Neighbour data are read through a view
// centred on the cell; offsets reach 2 cells (a contact cell next to the
// centre needs its own wall neighbours).
template <class P> struct LsqrView {
    const Fields<P> &F;
    int x, y, z;  // centre
    __device__ inline int at(int dx, int dy, int dz) const { return gidx(x + dx, y + dy, z + dz, F.nx, F.ny, F.nz); }
    __device__ inline uint8_t flag(int dx, int dy, int dz) const { return F.flags[at(dx, dy, dz)]; }
    __device__ inline void normal(int dx, int dy, int dz, double (&n)[3]) const
    {
        const int j = at(dx, dy, dz);
        const size_t N = F.N;
        n[0] = double(F.nrm[j]);
        n[1] = double(F.nrm[N + j]);
        n[2] = double(F.nrm[2 * N + j]);
    }
    __device__ inline double plic(int dx, int dy, int dz) const { return double(F.plic[at(dx, dy, dz)]); }
};

// The same view served from LDS: the lanes that share a centre first copy
// the flags of its 5 x 5 x 5 block and the normals and PLIC offsets of its
// 3 x 3 x 3 block (all that the fit and the contact conditions read), as
// independent loads, so the fit's scattered reads wait for memory once
// instead of once per dependent access.
template <class R> struct LsqrStage {
    uint8_t fl[128];  // 125 used: (dz + 2) 25 + (dy + 2) 5 + dx + 2
    R nrm[81];        // 3 per block cell (dz + 1) 9 + (dy + 1) 3 + dx + 1
    R pl[27];
};
template <class R> struct LsqrLdsView {
    const LsqrStage<R> &s;
    __device__ inline uint8_t flag(int dx, int dy, int dz) const { return s.fl[(dz + 2) * 25 + (dy + 2) * 5 + dx + 2]; }
    __device__ inline void normal(int dx, int dy, int dz, double (&n)[3]) const
    {
        const int j = 3 * ((dz + 1) * 9 + (dy + 1) * 3 + dx + 1);
        n[0] = double(s.nrm[j]);
        n[1] = double(s.nrm[j + 1]);
        n[2] = double(s.nrm[j + 2]);
    }
    __device__ inline double plic(int dx, int dy, int dz) const { return double(s.pl[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1]); }
};
// Lane `lane` of the L lanes of centre (x, y, z) copies its share.
template <class P>
__device__ inline void lsqr_stage(const Fields<P> &F, int x, int y, int z, int lane, int L,
                                  LsqrStage<typename P::R> &s)
{
    for (int t = lane; t < 125; t += L)
        s.fl[t] = F.flags[gidx(x + t % 5 - 2, y + (t / 5) % 5 - 2, z + t / 25 - 2, F.nx, F.ny, F.nz)];
    const size_t N = F.N;
    for (int t = lane; t < 27; t += L) {
        const int j = gidx(x + t % 3 - 1, y + (t / 3) % 3 - 1, z + t / 9 - 1, F.nx, F.ny, F.nz);
        s.nrm[3 * t] = F.nrm[j];
        s.nrm[3 * t + 1] = F.nrm[N + j];
        s.nrm[3 * t + 2] = F.nrm[2 * N + j];
        s.pl[t] = F.plic[j];
    }
}

// Contact point and contact normal of the contact-line cell at offset d from
// the centre (eqs. contactNormal, contactConstraint; Fig. contactPoint): the
// point of (PLIC plane) ∩ (wall plane) nearest to the PLIC point, reached
// along the wall normal projected onto the PLIC plane; the wall plane lies
// half a cell from the cell centre along the wall normal (the bounce-back
// wall is half-way between nodes). Returns false when the condition is
// skipped.
template <class View>
__host__ __device__ __forceinline__ bool contact_condition(const View &V, int dx, int dy, int dz, const double (&pc)[3],
                                         const double (&nc)[3], const double (&tu)[3], const double (&tv)[3],
                                         const Params &prm, double &uc, double &vc, double &ru, double &rv)
{
    double nj[3];
    V.normal(dx, dy, dz, nj);
    if (nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0) return false;
    int sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q)
        if (V.flag(dx + dir_x(q), dy + dir_y(q), dz + dir_z(q)) & FL_OBST) {
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
    const double aj = V.plic(dx, dy, dz);
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

// Frame, PLIC point and wetting state of the centre of view V (Sec. II.C):
// t_u from the axis with the smallest |n_k| (first on ties), t_v = n x t_u,
// and, when the centre is a contact-line cell, its hard constraint
// H = hu - 2 huc A - hvc C, I = hv - 2 hvc B - huc C.
struct LsqrFrame {
    double nc[3], tu[3], tv[3], pc[3];
    bool ok, has_obst, hard;
    double huc, hvc, hu, hv;
};

// Completes a frame whose centre normal f.nc and validity f.ok are set,
// given whether the block holds an obstacle cell.
template <class View>
__host__ __device__ __forceinline__ void lsqr_frame_finish(const View &V, const Params &prm, LsqrFrame &f,
                                                           bool has_obst)
{
    f.has_obst = has_obst;
    f.hard = false;
    f.huc = f.hvc = f.hu = f.hv = 0.0;
    if (!f.ok) return;
    const double(&nc)[3] = f.nc;
    int ax = 0;
    if (fabs(nc[1]) < fabs(nc[ax])) ax = 1;
    if (fabs(nc[2]) < fabs(nc[ax])) ax = 2;
    // selects rather than a run-time index keep the frame in registers
    const double nax = ax == 0 ? nc[0] : (ax == 1 ? nc[1] : nc[2]);
    double tu[3] = {-nax * nc[0] + (ax == 0 ? 1.0 : 0.0), -nax * nc[1] + (ax == 1 ? 1.0 : 0.0),
                    -nax * nc[2] + (ax == 2 ? 1.0 : 0.0)};
    const double ltu = sqrt(dot(tu, tu));
    f.tu[0] = tu[0] / ltu; f.tu[1] = tu[1] / ltu; f.tu[2] = tu[2] / ltu;
    f.tv[0] = nc[1] * f.tu[2] - nc[2] * f.tu[1];
    f.tv[1] = nc[2] * f.tu[0] - nc[0] * f.tu[2];
    f.tv[2] = nc[0] * f.tu[1] - nc[1] * f.tu[0];
    const double ac = V.plic(0, 0, 0);
    f.pc[0] = ac * nc[0]; f.pc[1] = ac * nc[1]; f.pc[2] = ac * nc[2];
    if (f.has_obst && (V.flag(0, 0, 0) & FL_NEAR_OBST))
        f.hard = contact_condition(V, 0, 0, 0, f.pc, f.nc, f.tu, f.tv, prm, f.huc, f.hvc, f.hu, f.hv);
}

template <class View>
__host__ __device__ __forceinline__ LsqrFrame lsqr_frame(const View &V, const Params &prm)
{
    LsqrFrame f;
    V.normal(0, 0, 0, f.nc);
    f.ok = !(f.nc[0] == 0.0 && f.nc[1] == 0.0 && f.nc[2] == 0.0);
    bool has_obst = false;
#pragma unroll
    for (int c = -1; c <= 1; ++c)
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int a = -1; a <= 1; ++a) has_obst |= (V.flag(a, b, c) & FL_OBST) != 0;
    lsqr_frame_finish(V, prm, f, has_obst);
    return f;
}

// Cholesky solve of a C x C system held as a packed lower triangle
// (entry (r, c), c <= r, at r (r + 1) / 2 + c); fails when a pivot falls
// below 1e-12 * trace (rank deficiency of the row matrix).
template <int C>
__host__ __device__ __forceinline__ bool packed_solve(const double *G, const double *g, double (&x)[C])
{
    double tr = 0.0;
#pragma unroll
    for (int r = 0; r < C; ++r) tr += G[r * (r + 1) / 2 + r];
    if (!(tr > 0.0)) return false;
    double L[C * (C + 1) / 2];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double d = G[c * (c + 1) / 2 + c];
#pragma unroll
        for (int j = 0; j < c; ++j) d -= L[c * (c + 1) / 2 + j] * L[c * (c + 1) / 2 + j];
        if (!(d >= 1e-12 * tr)) return false;
        L[c * (c + 1) / 2 + c] = sqrt(d);
#pragma unroll
        for (int r = c + 1; r < C; ++r) {
            double s = G[r * (r + 1) / 2 + c];
#pragma unroll
            for (int j = 0; j < c; ++j) s -= L[r * (r + 1) / 2 + j] * L[c * (c + 1) / 2 + j];
            L[r * (r + 1) / 2 + c] = s / L[c * (c + 1) / 2 + c];
        }
    }
    double y[C];
#pragma unroll
    for (int r = 0; r < C; ++r) {
        double s = g[r];
#pragma unroll
        for (int j = 0; j < r; ++j) s -= L[r * (r + 1) / 2 + j] * y[j];
        y[r] = s / L[r * (r + 1) / 2 + r];
    }
#pragma unroll
    for (int r = C - 1; r >= 0; --r) {
        double s = y[r];
#pragma unroll
        for (int j = r + 1; j < C; ++j) s -= L[j * (j + 1) / 2 + r] * x[j];
        x[r] = s / L[r * (r + 1) / 2 + r];
    }
    return true;
}

// Normal equations of the fit in one packed accumulator: the free model
// (A, B, C, H, I), or under the hard constraint the model (A, B, C) in the
// leading 3 x 3 part. The isotropic fallbacks (A = B, C = 0) are contracted
// from these sums when needed.
struct LsqrSums {
    double G[15], g[5];
    int rows = 0;
    __host__ __device__ inline LsqrSums()
    {
#pragma unroll
        for (int k = 0; k < 15; ++k) G[k] = 0.0;
#pragma unroll
        for (int k = 0; k < 5; ++k) g[k] = 0.0;
    }
    template <int C>
    __host__ __device__ __forceinline__ void acc(const double (&a)[C], double b)
    {
#pragma unroll
        for (int r = 0; r < C; ++r) {
            g[r] += a[r] * b;
#pragma unroll
            for (int c = 0; c <= r; ++c) G[r * (r + 1) / 2 + c] += a[r] * a[c];
        }
    }
    __host__ __device__ __forceinline__ void add(const LsqrFrame &f, double r0, double r1, double r2, double r3, double r4,
                                        double b)
    {
        ++rows;
        // a hard-constraint row (e0, e1, e2 | be) goes in as (e0, e1, e2, 0, 0):
        // one code path with fixed indices, the 3 x 3 system is the leading block
        const bool h = f.hard;
        const double e0 = r0 - r3 * (2.0 * f.huc), e1 = r1 - r4 * (2.0 * f.hvc);
        const double e2 = r2 - r3 * f.hvc - r4 * f.huc;
        const double be = b - r3 * f.hu - r4 * f.hv;
        const double a5[5] = {h ? e0 : r0, h ? e1 : r1, h ? e2 : r2, h ? 0.0 : r3, h ? 0.0 : r4};
        acc(a5, h ? be : b);
    }
};

// Rows contributed by the block cell at offset (a, b, c): its PLIC point
// (interface cells other than the centre) and, for contact-line cells other
// than the centre, the two rows of the gradient condition.
template <class View>
__host__ __device__ __forceinline__ void lsqr_cell_rows(const View &V, const Params &prm, const LsqrFrame &f, int a, int b,
                                               int c, LsqrSums &S)
{
    if (a == 0 && b == 0 && c == 0) return;
    const uint8_t fj = V.flag(a, b, c);
    if (!(fj & FL_IF)) return;
    double nj[3];
    V.normal(a, b, c, nj);
    if (nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0) return;
    const double aj = V.plic(a, b, c);
    const double r[3] = {a + aj * nj[0] - f.pc[0], b + aj * nj[1] - f.pc[1], c + aj * nj[2] - f.pc[2]};
    const double u = dot(r, f.tu), v = dot(r, f.tv), w = dot(r, f.nc);
    S.add(f, u * u, v * v, u * v, u, v, w);
}

template <class View>
__host__ __device__ __forceinline__ void lsqr_contact_rows(const View &V, const Params &prm, const LsqrFrame &f, int a, int b,
                                                  int c, LsqrSums &S)
{
    if (a == 0 && b == 0 && c == 0) return;
    const uint8_t fj = V.flag(a, b, c);
    if (!((fj & FL_IF) && (fj & FL_NEAR_OBST))) return;
    double uc, vc, ru, rv;
    if (!contact_condition(V, a, b, c, f.pc, f.nc, f.tu, f.tv, prm, uc, vc, ru, rv)) return;
    S.add(f, 2.0 * uc, 0.0, vc, 1.0, 0.0, ru);
    S.add(f, 0.0, 2.0 * vc, uc, 0.0, 1.0, rv);
}

// Solve the normal equations (model choice as described above) and return
// K = 2 kappa (eq. anacurv, cross term C H I), 0 when no model is solvable.
__host__ __device__ __forceinline__ double lsqr_solve_curvature(const LsqrFrame &f, const LsqrSums &S)
{
    const double *G = S.G, *g = S.g;
    double A = 0, Bq = 0, C = 0, H = 0, I = 0;
    bool ok = false;
    if (!f.hard) {
        double x5[5];
        if (S.rows >= 5 && packed_solve<5>(G, g, x5)) {
            A = x5[0]; Bq = x5[1]; C = x5[2]; H = x5[3]; I = x5[4];
            ok = true;
        } else if (S.rows >= 3) {
            // rows (u^2 + v^2, u, v): contract columns 0 and 1
            const double G3[6] = {G[0] + 2.0 * G[1] + G[2], G[6] + G[7], G[9], G[10] + G[11], G[13], G[14]};
            const double g3[3] = {g[0] + g[1], g[3], g[4]};
            double x3[3];
            if (packed_solve<3>(G3, g3, x3)) {
                A = x3[0]; Bq = x3[0]; C = 0.0; H = x3[1]; I = x3[2];
                ok = true;
            }
        }
    } else {
        double x3[3];
        if (S.rows >= 3 && packed_solve<3>(G, g, x3)) {
            A = x3[0]; Bq = x3[1]; C = x3[2];
            ok = true;
        } else if (S.rows >= 1) {
            const double G1[1] = {G[0] + 2.0 * G[1] + G[2]};
            const double g1[1] = {g[0] + g[1]};
            double x1[1];
            if (packed_solve<1>(G1, g1, x1)) {
                A = x1[0]; Bq = x1[0]; C = 0.0;
                ok = true;
            }
        }
        H = f.hu - 2.0 * f.huc * A - f.hvc * C;
        I = f.hv - 2.0 * f.hvc * Bq - f.huc * C;
    }
    if (!ok) return 0.0;
    const double gg = 1.0 + H * H + I * I;
    return 2.0 * (A * (1.0 + I * I) + Bq * (1.0 + H * H) - C * H * I) / (gg * sqrt(gg));
}

// K = 2 kappa of the least-squares quadric at the centre of view V, rows
// accumulated in block order (data rows, then contact rows).
template <class View>
__host__ __device__ inline double lsqr_curvature(const View &V, const Params &prm)
{
    const LsqrFrame f = lsqr_frame(V, prm);
    if (!f.ok) return 0.0;
    LsqrSums S;
    for (int c = -1; c <= 1; ++c)
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) lsqr_cell_rows(V, prm, f, a, b, c, S);
    if (f.has_obst)
        for (int c = -1; c <= 1; ++c)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) lsqr_contact_rows(V, prm, f, a, b, c, S);
    return lsqr_solve_curvature(f, S);
}

// Normals and PLIC points of the interface cells (LSQR model).
template <class P>
__device__ inline void normals_plic_list(const Fields<P> &F)
{
    using G = typename P::G;
    const int n = list_count(F.sc);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        const Nbr nb(i, F.nx, F.ny, F.nz);
        G gx = 0, gy = 0, gz = 0;
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int b = -1; b <= 1; ++b) {
                const G w = G(pyw(a) * pyw(b));
                gx += w * (G(F.phi[nb.at(1, a, b)]) - G(F.phi[nb.at(-1, a, b)]));
                gy += w * (G(F.phi[nb.at(a, 1, b)]) - G(F.phi[nb.at(a, -1, b)]));
                gz += w * (G(F.phi[nb.at(a, b, 1)]) - G(F.phi[nb.at(a, b, -1)]));
            }
        G nrm[3];
        unit_normal(gx, gy, gz, nrm);
        const bool ok = nrm[0] != G(0) || nrm[1] != G(0) || nrm[2] != G(0);
        const G a = ok ? plic_offset<G>(nrm[0], nrm[1], nrm[2], G(F.phi[i])) : G(0);
        store_normal(F, i, nrm, a);
    }
}

template <class P>
__global__ __launch_bounds__(256) void k_normals_plic(const Batch<P> B, int eos)
{
    end_of_step(B.f[blockIdx.y].sc, eos);
    if (B.p[blockIdx.y].curv == 0) return;  // LSQR and TR
    normals_plic_list(B.f[blockIdx.y]);
}

// First geometry launch of a batch that mixes the models: FD lattices run
// their whole tiled curvature, LSQR lattices their normals and PLIC points
// (the LSQR fit follows in k_curv_lsqr4), so the two overlap on the device.
template <class P>
__global__ __launch_bounds__(256) void k_geometry_mixed(const Batch<P> B, int eos)
{
    end_of_step(B.f[blockIdx.y].sc, eos);
    if (B.p[blockIdx.y].curv == 0) geometry_fd_tiles(B.f[blockIdx.y]);
    else normals_plic_list(B.f[blockIdx.y]);
}

template <class P>
__global__ __launch_bounds__(256) void k_curv_lsqr(const Batch<P> B)
{
    const Params &prm = B.p[blockIdx.y];
    if (prm.curv != 1) return;
    const Fields<P> &F = B.f[blockIdx.y];
    using R = typename P::R;
    const int n = list_count(F.sc);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
        const LsqrView<P> V{F, x, y, z};
        F.K[i] = R(lsqr_curvature(V, prm));
    }
}

// LSQR curvature with 4 lanes per interface cell (64 cells per workgroup):
// lane l of a group scans the block cells s = l, l + 4, ... (s = 0..26,
// x fastest) for obstacles and adds their data and contact rows; the sums
// are reduced over the 4 lanes by an xor butterfly (a fixed order, the same
// result on every lane) and every lane solves the same system. Limited to
// 168 VGPRs for 3 waves per SIMD (a 20-byte spill): this latency-bound
// gather runs faster than at 2 waves with no spill.
template <class P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_curv_lsqr4(const Batch<P> B)
{
    const Params &prm = B.p[blockIdx.y];
    if (prm.curv != 1) return;
    const Fields<P> &F = B.f[blockIdx.y];
    using R = typename P::R;
    const int n = list_count(F.sc);
    const int l = threadIdx.x & 3;
    for (int k = blockIdx.x * 64 + (threadIdx.x >> 2); k < n; k += gridDim.x * 64) {
        const int i = F.ilist[k];
        const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
        const LsqrView<P> V{F, x, y, z};
        LsqrFrame f;
        V.normal(0, 0, 0, f.nc);
        f.ok = !(f.nc[0] == 0.0 && f.nc[1] == 0.0 && f.nc[2] == 0.0);
        // obstacles in the block: each lane scans its share
        bool ob = false;
#pragma unroll
        for (int t = 0; t < 7; ++t) {
            const int s = l + 4 * t;
            if (s < 27) ob |= (V.flag(s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1) & FL_OBST) != 0;
        }
        ob |= __shfl_xor(ob ? 1 : 0, 1, 4) != 0;
        ob |= __shfl_xor(ob ? 1 : 0, 2, 4) != 0;
        lsqr_frame_finish(V, prm, f, ob);
        LsqrSums S;
        if (f.ok) {
#pragma unroll
            for (int t = 0; t < 7; ++t) {
                const int s = l + 4 * t;
                if (s < 27) lsqr_cell_rows(V, prm, f, s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1, S);
            }
            if (f.has_obst)
                for (int t = 0; t < 7; ++t) {
                    const int s = l + 4 * t;
                    if (s < 27) lsqr_contact_rows(V, prm, f, s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1, S);
                }
        }
#pragma unroll
        for (int m = 1; m < 4; m <<= 1) {
#pragma unroll
            for (int e = 0; e < 15; ++e) S.G[e] += __shfl_xor(S.G[e], m, 4);
#pragma unroll
            for (int e = 0; e < 5; ++e) S.g[e] += __shfl_xor(S.g[e], m, 4);
            S.rows += __shfl_xor(S.rows, m, 4);
        }
        const double K = f.ok ? lsqr_solve_curvature(f, S) : 0.0;
        if (l == 0) F.K[i] = R(K);
        if (l == 1 && F.snap && k < F.sc->icount) {
            R *sn = F.snap + (size_t)SNAP * k;
            const size_t N = F.N;
            sn[0] = F.m[i]; sn[1] = F.rho[i]; sn[2] = F.phi[i]; sn[3] = R(K);
            sn[4] = F.nrm[i]; sn[5] = F.nrm[N + i]; sn[6] = F.nrm[2 * N + i]; sn[7] = F.plic[i];
        }
    }
}

// TR curvature (Sec. II.B): a triangle fan of the PLIC points of the 3x3x3
// block around the centre point p, curvature by Taubin's estimate. With
// d_k = p_k - p, the points are ordered by their polar angle in the tangent
// plane (measured from the direction 1 rad from t_u; angles within 1e-12
// keep block order; points with u^2 + v^2 < 1e-12 are left out);
// consecutive points span the triangle (p, p_k, p_k+1) unless their angular
// gap is at least pi - 1e-12. Each vertex is weighted by the area of its
// triangles, and K = 2 sum w_k kappa_k / sum w_k with the edge curvature
// kappa_k = 2 (d_k . n) / |d_k|^2 (twice the trace of Taubin's matrix).
// Fewer than three points or no triangle give K = 0.
//
// 32 lanes per interface cell: lane s < 27 holds block cell s (x fastest).
// Each lane finds the successor of its point in the cyclic order by
// scanning the group with shuffles, adds its triangle (area times the two
// edge curvatures, and twice the area), and the sums are reduced over the
// group by an xor butterfly (fixed order).
constexpr int TR_LANES = 32;

__device__ inline bool tr_before(double aj, int sj, double ak, int sk)
{
    return fabs(aj - ak) > 1e-12 ? aj < ak : sj < sk;
}

template <class P>
__global__ __launch_bounds__(256) void k_curv_tr(const Batch<P> B)
{
    const Params &prm = B.p[blockIdx.y];
    if (prm.curv != 2) return;
    const Fields<P> &F = B.f[blockIdx.y];
    using R = typename P::R;
    const double PI = 3.14159265358979323846;
    const double c1 = 0.54030230586813971740, s1 = 0.84147098480789650665;  // cos 1, sin 1
    const int n = list_count(F.sc);
    const int s = threadIdx.x & (TR_LANES - 1);
    const int groups = 256 / TR_LANES;
    const int n_round = (n + groups - 1) / groups * groups;  // whole groups iterate together
    for (int k = blockIdx.x * groups + (int)(threadIdx.x / TR_LANES); k < n_round; k += gridDim.x * groups) {
        const bool live = k < n;
        const int i = live ? F.ilist[k] : 0;
        const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
        const LsqrView<P> V{F, x, y, z};
        LsqrFrame f;
        V.normal(0, 0, 0, f.nc);
        f.ok = live && !(f.nc[0] == 0.0 && f.nc[1] == 0.0 && f.nc[2] == 0.0);
        lsqr_frame_finish(V, prm, f, false);
        // this lane's point
        const int a = s % 3 - 1, b = (s / 3) % 3 - 1, c = s / 9 - 1;
        bool valid = f.ok && s < 27 && s != 13;
        double d[3] = {0.0, 0.0, 0.0}, ang = 0.0, kap = 0.0;
        if (valid && (V.flag(a, b, c) & FL_IF)) {
            double nj[3];
            V.normal(a, b, c, nj);
            valid = !(nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0);
            if (valid) {
                const double aj = V.plic(a, b, c);
                d[0] = a + aj * nj[0] - f.pc[0];
                d[1] = b + aj * nj[1] - f.pc[1];
                d[2] = c + aj * nj[2] - f.pc[2];
                const double u = dot(d, f.tu), v = dot(d, f.tv);
                valid = u * u + v * v >= 1e-12;
                ang = atan2(-u * s1 + v * c1, u * c1 + v * s1);
                kap = 2.0 * dot(d, f.nc) / dot(d, d);
            }
        } else {
            valid = false;
        }
        int m = valid ? 1 : 0;
#pragma unroll
        for (int w = 1; w < TR_LANES; w <<= 1) m += __shfl_xor(m, w, TR_LANES);
        // successor in the cyclic order: the first point after this one,
        // else (this is the last) the first point of all
        int nxt = -1, first = -1;
        double a_nxt = 0.0, a_first = 0.0;
        for (int j = 0; j < TR_LANES; ++j) {
            const int vj = __shfl(valid ? 1 : 0, j, TR_LANES);
            const double aj = __shfl(ang, j, TR_LANES);
            if (!vj) continue;
            if (first < 0 || tr_before(aj, j, a_first, first)) {
                first = j;
                a_first = aj;
            }
            if (j != s && tr_before(ang, s, aj, j) && (nxt < 0 || tr_before(aj, j, a_nxt, nxt))) {
                nxt = j;
                a_nxt = aj;
            }
        }
        const bool wrap = nxt < 0;
        const int sj = wrap ? first : nxt;
        const double dj0 = __shfl(d[0], sj < 0 ? 0 : sj, TR_LANES);
        const double dj1 = __shfl(d[1], sj < 0 ? 0 : sj, TR_LANES);
        const double dj2 = __shfl(d[2], sj < 0 ? 0 : sj, TR_LANES);
        const double kj = __shfl(kap, sj < 0 ? 0 : sj, TR_LANES);
        double num = 0.0, den = 0.0;
        if (valid && m >= 3) {
            const double gap = (wrap ? a_first : a_nxt) - ang + (wrap ? 2.0 * PI : 0.0);
            if (gap < PI - 1e-12) {
                const double cr[3] = {d[1] * dj2 - d[2] * dj1, d[2] * dj0 - d[0] * dj2, d[0] * dj1 - d[1] * dj0};
                const double area = 0.5 * sqrt(dot(cr, cr));
                num = area * (kap + kj);
                den = 2.0 * area;
            }
        }
#pragma unroll
        for (int w = 1; w < TR_LANES; w <<= 1) {
            num += __shfl_xor(num, w, TR_LANES);
            den += __shfl_xor(den, w, TR_LANES);
        }
        if (live && s == 0) F.K[i] = R(den > 0.0 ? 2.0 * num / den : 0.0);
    }
}

}  // namespace fslbm
