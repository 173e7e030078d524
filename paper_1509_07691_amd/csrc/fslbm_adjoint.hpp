// Discrete adjoint of the FSLBM time step with frozen cell types.
//
// Over a window of T steps the flags, the interface list and the obstacle
// list stay fixed (no fill / empty conversion), so one step is a smooth map
// of the state s_t = (f'_t, m_t, phi_t) given the parameters sigma (through
// rho_b = rho_gas + 3 sigma K, Sec. II) and theta (through the contact
// condition of the LSQR model, eqs. contactNormal, contactConstraint):
//   K_t      = curvature(phi_t)                      (Sec. II.A or II.C)
//   f_in     = pull(f'_t; rho_b(K_t), u_b(f'_t))     (eqs. lbe1, reconstruct)
//   m_{t+1}  = m_t + sum_q k_q(phi_t) (f_in,qbar - f'_q)   (eqs. advection1/2)
//   phi_{t+1}= m_{t+1} / sum_q f_in,q
//   f'_{t+1} = collide(f_in)                          (eq. lbe2)
// The reverse step maps the adjoints (lam = dL/df', mbar, phib) at t+1 to
// those at t. Every kernel is written as a gather (one writer per value) so
// the results do not depend on scheduling:
//   k_adj_prepass      phi_{t+1} = m_{t+1}/rho_{t+1} -> mbar, rhob (phib
//                      with the transposed obstacle fill reflection of
//                      Sec. II.A left by the previous reverse step); the
//                      restore of state t from its snapshot
//   k_adj_stream       per fluid cell: gathers lam_q(x) = own_q(x) +
//                      gin_q(x + c_q) of the previous reverse step, then the
//                      transposed collision, mass exchange and boundary
//                      rules; the adjoint of each pulled value is left at
//                      the receiving cell (gin), the adjoint of the cell's
//                      own outgoing values in own (both double-buffered),
//                      dL/dK in kbar
//   FD:   k_adj_fd_*   transposed stencils of K = -div(n^), n^ from the
//                      K8-mollified fill level
//   LSQR: k_adj_lsqr_* reverse of the least-squares fit per interface cell
//                      (normal equations: y = G^-1 xbar, bbar = M y,
//                      Mbar = r y^T - M y x^T), the PLIC offsets by the
//                      implicit function theorem (da/dphi = -1/A, da/dn =
//                      centroid of the plane section, A its area) and the
//                      Parker-Youngs normals
// All adjoint arithmetic is FP64 whatever the storage precision.
#pragma once

#include "fslbm_geometry.hpp"
#include "fslbm_stream.hpp"

namespace fslbm {

struct Adj {
    const double *gin_in, *own_in;  // the previous reverse step's gin and own
    double *gin;    // 19 planes: dL/df_in,q(x), kept at the receiving cell x
    double *own;    // 19 planes: the cell's own share of dL/df'_q(x)
    double *refl;   // 18 per interface-list entry: transposed reflection weights
    double *mbar;   // dL/dm
    double *phib;   // dL/dphi (at obstacle cells: scratch of the reflection)
    double *rhob;   // dL/drho(t+1) at interface cells
    double *kbar;   // dL/dK at interface cells
    double *sacc;   // per-cell accumulation of dL/dsigma
    double *tacc;   // per-cell accumulation of dL/dtheta
    double *ms;     // FD: mollified fill level
    double *msb;    // FD: its adjoint
    double *gb;     // 3 planes: adjoint of the Parker-Youngs gradient
    double *contrib;  // LSQR: 27 x 4 partials (dK/dn_j, dK/da_j) per list entry
    int *pos;       // list position of each interface cell
};

constexpr int CONTRIB = 27 * 4;

__host__ __device__ constexpr int slot27(int a, int b, int c) { return (c + 1) * 9 + (b + 1) * 3 + (a + 1); }

// ------------------------------------------------------- state snapshots
// The state of a step in the frozen window: f' (19 planes, stored apart)
// and, per interface-list entry, m, rho, phi, K, n (3) and the PLIC offset,
// followed by phi of the obstacle-list cells. Everything else is constant
// while the cell types are frozen.

template <class P>
__global__ __launch_bounds__(256) void k_snap(Fields<P> F, typename P::R *snap, int save)
{
    using R = typename P::R;
    const int n = F.sc->icount, no = F.sc->ocount;
    const size_t N = F.N;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n + no; k += gridDim.x * 256) {
        if (k < n) {
            const int i = F.ilist[k];
            R *s = snap + (size_t)SNAP * k;
            if (save) {
                s[0] = F.m[i]; s[1] = F.rho[i]; s[2] = F.phi[i]; s[3] = F.K[i];
                s[4] = F.nrm[i]; s[5] = F.nrm[N + i]; s[6] = F.nrm[2 * N + i]; s[7] = F.plic[i];
            } else {
                F.m[i] = s[0]; F.rho[i] = s[1]; F.phi[i] = s[2]; F.K[i] = s[3];
                F.nrm[i] = s[4]; F.nrm[N + i] = s[5]; F.nrm[2 * N + i] = s[6]; F.plic[i] = s[7];
            }
        } else {
            const int o = F.olist[k - n];
            R *s = snap + (size_t)SNAP * n + (k - n);
            if (save) *s = F.phi[o];
            else F.phi[o] = *s;
        }
    }
}

// ------------------------------------------------------- set-up kernels
__global__ void k_adj_zero(double *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = 0.0;
}

// pos[] of the interface cells and phib = dL/dphi_T there.
template <class P>
__global__ void k_adj_begin(Fields<P> F, Adj A, const double *dphi)
{
    const int n = F.sc->icount;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        A.pos[i] = k;
        A.phib[i] = dphi[i];
    }
}

// Transposed obstacle fill reflection, deferred to the next reader of
// phib: each reverse step leaves the adjoint of the obstacle fill levels in
// phib at the obstacle cells (k_adj_fd_phib, k_adj_lsqr_phib), and the
// interface cell i (list entry k) adds phib(o) w_oi / den_o over its
// obstacle neighbours o (weights from k_adj_reflect_setup) where it reads
// its own phib: in k_adj_prepass of the next step and in k_adj_finish.
template <class P>
__device__ inline double reflected_phib(const Fields<P> &F, const Adj &A, int k, int i)
{
    if (!(F.flags[i] & FL_NEAR_OBST)) return 0.0;
    const Nbr ni(i, F.nx, F.ny, F.nz);
    const double *c = A.refl + (size_t)(NQ - 1) * k;
    double acc = 0.0;
#pragma unroll
    for (int q = 1; q < NQ; ++q)
        if (c[q - 1] != 0.0) acc += A.phib[ni.at(dir_x(q), dir_y(q), dir_z(q))] * c[q - 1];
    return acc;
}

// dL/dphi_0 = phib + mbar rho_0 at interface cells (m_0 = phi_0 rho_0 with
// the distributions of the window start held fixed).
template <class P>
__global__ void k_adj_finish(Fields<P> F, Adj A, const typename P::R *snap0, double *out)
{
    const int n = F.sc->icount;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        out[i] = (A.phib[i] + reflected_phib(F, A, k, i)) + A.mbar[i] * double(snap0[(size_t)SNAP * k + 1]);
    }
}

// ------------------------------------------------ phi = m / rho (reverse)
// phi = m / rho of step t+1 reversed (m and rho from its snapshot, phib
// with the deferred reflection added), and the state of step t restored
// from its snapshot (as k_snap with save = 0): both go entry by entry over
// the same lists, so they share one launch.
template <class P>
__global__ __launch_bounds__(256) void k_adj_prepass(Fields<P> F, Adj A, const typename P::R *snap_next,
                                                     const typename P::R *snap_cur)
{
    const int n = F.sc->icount, no = F.sc->ocount;
    const size_t N = F.N;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n + no; k += gridDim.x * 256) {
        if (k < n) {
            const int i = F.ilist[k];
            const double m = double(snap_next[(size_t)SNAP * k]), r = double(snap_next[(size_t)SNAP * k + 1]);
            const double pb = A.phib[i] + reflected_phib(F, A, k, i);
            A.mbar[i] += pb / r;
            A.rhob[i] = -pb * m / (r * r);
            A.phib[i] = 0.0;
            const typename P::R *s = snap_cur + (size_t)SNAP * k;
            F.m[i] = s[0]; F.rho[i] = s[1]; F.phi[i] = s[2]; F.K[i] = s[3];
            F.nrm[i] = s[4]; F.nrm[N + i] = s[5]; F.nrm[2 * N + i] = s[6]; F.plic[i] = s[7];
        } else {
            F.phi[F.olist[k - n]] = snap_cur[(size_t)SNAP * n + (k - n)];
        }
    }
}

// ------------------------------------------- transposed collision (eq. lbe2)
// fb = (d collide / d f)^T yb at the pre-collision values f.
template <int COLL>
__device__ inline void collide_adj(const double (&f)[NQ], const double (&yb)[NQ], const Params &p, double (&fb)[NQ])
{
    double rho, ux, uy, uz;
    moments(f, rho, ux, uy, uz);
    const double usq = ux * ux + uy * uy + uz * uz;
    const double we = p.omega;
    double eb[NQ];  // adjoint of feq_q
    if constexpr (COLL == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            fb[q] = (1.0 - we) * yb[q];
            eb[q] = we * yb[q];
        }
    } else {
        const double wo = p.omega_odd;
#pragma unroll
        for (int q = 0; q < NQ; ++q) fb[q] = eb[q] = 0.0;
        // g_q = f_q - we (f+_q - e+_q) - wo (f-_q - e-_q), f+- = (f_q +- f_qbar)/2
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int o = opp(q);
            const double y = yb[q];
            fb[q] += y * (1.0 - 0.5 * we - 0.5 * wo);
            fb[o] += y * (0.5 * wo - 0.5 * we);
            eb[q] += y * (0.5 * we + 0.5 * wo);
            eb[o] += y * (0.5 * we - 0.5 * wo);
        }
    }
    // feq_q = w_q rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
    double rb = 0.0, uxb = 0.0, uyb = 0.0, uzb = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double cx = dir_x(q), cy = dir_y(q), cz = dir_z(q);
        const double cu = cx * ux + cy * uy + cz * uz;
        const double w = weight<double>(q) * eb[q];
        rb += w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        const double s = w * rho * (3.0 + 9.0 * cu), t = w * rho * 3.0;
        uxb += s * cx - t * ux;
        uyb += s * cy - t * uy;
        uzb += s * cz - t * uz;
    }
    // u = j / rho
    const double jxb = uxb / rho, jyb = uyb / rho, jzb = uzb / rho;
    rb -= (uxb * ux + uyb * uy + uzb * uz) / rho;
#pragma unroll
    for (int q = 0; q < NQ; ++q) fb[q] += rb + dir_x(q) * jxb + dir_y(q) * jyb + dir_z(q) * jzb;
}

template <class P>
__device__ inline void load_dirs_d(const Fields<P> &F, const int (&j)[NQ], double (&f)[NQ])
{
    typename P::T t[NQ];
    load_dirs<P>(F, j, t);
#pragma unroll
    for (int q = 0; q < NQ; ++q) f[q] = double(t[q]);
}

// ------------------------------------ reverse stream-collide, one fluid cell
// Recomputes the forward pull of boundary_cell (same rules, in FP64) and
// applies the transposed step. Writes gin and own of the cell; at interface
// cells also kbar, phib (the part from the mass-exchange weights) and the
// sigma accumulator. A liquid cell away from walls has the plain pull and
// writes gin only (its own outgoing values are never read: the cell is
// liquid at every step of the window).
template <class P, int COLL>
__device__ inline void cell_adj(const Fields<P> &F, const Adj &A, const Params &prm, int i, const Nbr &nb, uint8_t fl)
{
    const size_t N = F.N;
    int up[NQ], own[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        up[q] = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
        own[q] = i;
    }
    double pl[NQ];
    load_dirs_d<P>(F, up, pl);
    double yb[NQ];  // dL/df'_q(x) = own_q(x) + gin_q(x + c_q) (x + c_q = up[opp(q)])
    if (fl == FL_LIQ) {  // every neighbour is fluid: plain pull
#pragma unroll
        for (int q = 0; q < NQ; ++q) yb[q] = A.gin_in[q * N + up[opp(q)]];
        double fb[NQ];
        collide_adj<COLL>(pl, yb, prm, fb);
#pragma unroll
        for (int q = 0; q < NQ; ++q) A.gin[q * N + i] = fb[q];
        return;
    }
    const bool is_if = (fl & FL_IF) != 0;
    double fo[NQ];
    load_dirs_d<P>(F, own, fo);
    uint8_t nt[NQ];
    nt[0] = FL_LIQ;
#pragma unroll
    for (int q = 1; q < NQ; ++q) nt[q] = F.flags[up[q]] & FL_TYPE;
    // the neighbour's value is loaded whatever its type (every up[] index is
    // a cell of the lattice), so the loads do not wait for the flags
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double g = A.gin_in[q * N + up[opp(q)]];
        yb[q] = A.own_in[q * N + i] + ((nt[opp(q)] & FL_FLUID) ? g : 0.0);
    }
    double Kc = 0, phx = 0, cnx = 0, cny = 0, cnz = 0;
    if (is_if) {
        Kc = double(F.K[i]);
        phx = double(F.phi[i]);
        cnx = double(F.nrm[i]);
        cny = double(F.nrm[N + i]);
        cnz = double(F.nrm[2 * N + i]);
    }
    bool has_gas = false;
    int nwx = 0, nwy = 0, nwz = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        has_gas |= nt[q] == FL_GAS;
        if (nt[q] == FL_OBST) { nwx -= dir_x(q); nwy -= dir_y(q); nwz -= dir_z(q); }
    }
    double rb0, ubx, uby, ubz;
    moments(fo, rb0, ubx, uby, ubz);
    const double ubsq = ubx * ubx + uby * uby + ubz * ubz;
    const double rhob = prm.rho_gas + 3.0 * prm.sigma * Kc;
    const bool corner = is_if && has_gas && (nwx | nwy | nwz) != 0;
    const int ww = nwx * nwx + nwy * nwy + nwz * nwz;
    double fin[NQ];
    bool rec[NQ];
    fin[0] = fo[0];
    rec[0] = false;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const int o = opp(q);
        const uint8_t t = nt[q];
        const int cox = -dir_x(q), coy = -dir_y(q), coz = -dir_z(q);
        const int cw = cox * nwx + coy * nwy + coz * nwz;
        const double s = double(cox * ww - cw * nwx) * cnx + double(coy * ww - cw * nwy) * cny +
                         double(coz * ww - cw * nwz) * cnz;
        rec[q] = (t == FL_GAS) || (t == FL_OBST && corner && s < 0.0);
        const double vrec = feq_pair<double>(q, rhob, ubx, uby, ubz, ubsq) - fo[o];
        fin[q] = (t & FL_FLUID) ? pl[q] : (rec[q] ? vrec : fo[o]);
    }
    double fb[NQ], fob[NQ];
    collide_adj<COLL>(fin, yb, prm, fb);
#pragma unroll
    for (int q = 0; q < NQ; ++q) fob[q] = 0.0;
    if (is_if) {
        // the neighbours' phi and mbar, loaded whatever their type (used at
        // interface neighbours), so that the loads do not wait for the flags
        double phz[NQ], mbz[NQ];
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int z = up[opp(q)];
            phz[q] = double(F.phi[z]);
            mbz[q] = A.mbar[z];
        }
        // rho(t+1) = sum_q f_in,q
        const double rb = A.rhob[i];
#pragma unroll
        for (int q = 0; q < NQ; ++q) fb[q] += rb;
        // m(t+1) = m(t) + sum_q k_q (f_in,qbar - f'_q)
        const double Mb = A.mbar[i];
        double phb = 0.0;
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int o = opp(q);
            const uint8_t tz = nt[o];  // type of x + c_q
            if (tz == FL_LIQ) {
                fb[o] += Mb;
                fob[q] -= Mb;
            } else if (tz == FL_IF) {
                const double k = 0.5 * (phz[q] + phx);
                fb[o] += k * Mb;
                fob[q] -= k * Mb;
                // both ends of the link carry the weight (phi_x + phi_z)/2
                phb += 0.5 * (fin[o] - fo[q]) * (Mb - mbz[q]);
            }
        }
        A.phib[i] = phb;
    }
    // transposed pull and boundary rules
    double rbb = 0.0, uxb = 0.0, uyb = 0.0, uzb = 0.0;
    A.gin[i] = fb[0];
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const int o = opp(q);
        if (nt[q] & FL_FLUID) {
            A.gin[q * N + i] = fb[q];
            continue;
        }
        A.gin[q * N + i] = 0.0;
        if (rec[q]) {
            // feq_q + feq_qbar = 2 w rho_b (1 + 4.5 (c.u_b)^2 - 1.5 u_b.u_b)
            fob[o] -= fb[q];
            const double cx = dir_x(q), cy = dir_y(q), cz = dir_z(q);
            const double cu = cx * ubx + cy * uby + cz * ubz;
            const double w2 = 2.0 * weight<double>(q) * fb[q];
            rbb += w2 * (1.0 + 4.5 * cu * cu - 1.5 * ubsq);
            const double s = w2 * rhob * 9.0 * cu, t = w2 * rhob * 3.0;
            uxb += s * cx - t * ubx;
            uyb += s * cy - t * uby;
            uzb += s * cz - t * ubz;
        } else {
            fob[o] += fb[q];
        }
    }
    if (uxb != 0.0 || uyb != 0.0 || uzb != 0.0) {
        // u_b = j(f'_t(x)) / rho(f'_t(x))
        const double jxb = uxb / rb0, jyb = uyb / rb0, jzb = uzb / rb0;
        const double r0b = -(uxb * ubx + uyb * uby + uzb * ubz) / rb0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) fob[q] += r0b + dir_x(q) * jxb + dir_y(q) * jyb + dir_z(q) * jzb;
    }
    if (is_if) {
        // rho_b = rho_gas + 3 sigma K
        A.kbar[i] = 3.0 * prm.sigma * rbb;
        A.sacc[i] += 3.0 * Kc * rbb;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) A.own[q * N + i] = fob[q];
}

// Reverse stream-collide over the fluid bounding box (same traversal as the
// forward kernel). Measured on the 128^3 sessile drop: one launch in which
// liquid and boundary wavefronts overlap is faster than a lean liquid pass
// followed by a list pass over the interface and wall cells (0.147 against
// 0.169 ms per reverse step), and capping it at 2 waves per SIMD (spills)
// is slower too.
template <class P, int COLL>
__global__ __launch_bounds__(256) void k_adj_stream(const Fields<P> F, const Adj A, const Params prm)
{
    const CellRange box = CellRange::from(F.sc->fbox);
    const int n = box.size();
    const int nxy = F.nx * F.ny;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int bx = k % box.ex, r = k / box.ex, by = r % box.ey, bz = r / box.ey;
        const int x = box.x0 + bx, y = box.y0 + by, z = box.z0 + bz;
        const int i = x + F.nx * y + nxy * z;
        const uint8_t fl = F.flags[i];
        if (!(fl & FL_FLUID)) continue;
        const Nbr nb(x, y, z, F.nx, F.ny, F.nz);
        cell_adj<P, COLL>(F, A, prm, i, nb, fl);
    }
}

// ------------------------------------------------ FD curvature (reverse)
// Forward (Sec. II.A): ms = K8 * phi / 942, g = PY(ms), n = g/|g|,
// K = -(PY_x n_x + PY_y n_y + PY_z n_z)/32 at interface cells. Each PY
// difference is antisymmetric and its transverse weights symmetric, so the
// transpose of PY_k is -PY_k.
template <class P>
__global__ __launch_bounds__(256) void k_adj_fd_mol(const Fields<P> F, const Adj A)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < F.N; i += gridDim.x * 256) {
        const Nbr nb(i, F.nx, F.ny, F.nz);
        double s = 0.0;
#pragma unroll
        for (int c = -1; c <= 1; ++c)
#pragma unroll
            for (int b = -1; b <= 1; ++b)
#pragma unroll
                for (int a = -1; a <= 1; ++a) s += k8w(a * a + b * b + c * c) * double(F.phi[nb.at(a, b, c)]);
        A.ms[i] = s * K8_INV;
    }
}

// Reverse of the FD contact normal n = normalise(2 m - n_b), m = n_w
// cos(theta) + n_t sin(theta), n_t = normalise(n_b - (n_b.n_w) n_w): given
// nbar = dL/dn, adds dL/dn_b to nbb and dL/dtheta to thb. Returns false
// (nothing added) where the forward kept the mollified normal.
__device__ inline bool fd_contact_normal_adj(const double (&w)[3], const double (&nb)[3], double ct, double st,
                                             const double (&ob)[3], double (&nbb)[3], double &thb)
{
    const double nw[3] = {-w[0], -w[1], -w[2]};
    const double nn = nb[0] * nw[0] + nb[1] * nw[1] + nb[2] * nw[2];
    const double ntr[3] = {nb[0] - nn * nw[0], nb[1] - nn * nw[1], nb[2] - nn * nw[2]};
    const double lt = sqrt(dot(ntr, ntr));
    if (lt < 1e-12) return false;
    const double nt[3] = {ntr[0] / lt, ntr[1] / lt, ntr[2] / lt};
    double e[3];
    for (int k = 0; k < 3; ++k) e[k] = 2.0 * (nw[k] * ct + nt[k] * st) - nb[k];
    const double le = sqrt(dot(e, e));
    if (le < 1e-12) return false;
    const double no[3] = {e[0] / le, e[1] / le, e[2] / le};
    const double on = dot(ob, no);
    double eb[3], mb[3];
    for (int k = 0; k < 3; ++k) {
        eb[k] = (ob[k] - on * no[k]) / le;
        mb[k] = 2.0 * eb[k];
        nbb[k] -= eb[k];
    }
    thb += -st * dot(mb, nw) + ct * dot(mb, nt);
    const double ntb[3] = {st * mb[0], st * mb[1], st * mb[2]};
    const double tt = dot(ntb, nt);
    double trb[3];
    for (int k = 0; k < 3; ++k) trb[k] = (ntb[k] - tt * nt[k]) / lt;
    const double tw = dot(trb, nw);
    for (int k = 0; k < 3; ++k) nbb[k] += trb[k] - tw * nw[k];
    return true;
}

// Base direction qb of obstacle cell o for FD wetting (0: no contact
// normal): the lattice direction closest to the normalised sum w of the
// directions to o's non-obstacle neighbours, when o + c_qb is not an
// obstacle cell (the forward rule, in FP64).
template <class P>
__device__ inline int fd_contact_base_d(const Fields<P> &F, const Nbr &no, double (&w)[3])
{
    int sx = 0, sy = 0, sz = 0;
    for (int q = 1; q < NQ; ++q)
        if (!(F.flags[no.at(dir_x(q), dir_y(q), dir_z(q))] & FL_OBST)) {
            sx += dir_x(q); sy += dir_y(q); sz += dir_z(q);
        }
    const double lw = sqrt(double(sx * sx + sy * sy + sz * sz));
    if (!(lw > 0.0)) return 0;
    w[0] = sx / lw; w[1] = sy / lw; w[2] = sz / lw;
    int qb = 0;
    double best = -2.0;
    for (int q = 1; q < NQ; ++q) {
        const double cl = sqrt(double(dir_len2(q)));
        const double a = (dir_x(q) * w[0] + dir_y(q) * w[1] + dir_z(q) * w[2]) / cl;
        if (a > best) { best = a; qb = q; }
    }
    return (F.flags[no.at(dir_x(qb), dir_y(qb), dir_z(qb))] & FL_OBST) ? 0 : qb;
}

__device__ inline bool unit_of(const double g[3], double (&n)[3], double &len)
{
    len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (!(len > 1e-12)) return false;
    n[0] = g[0] / len; n[1] = g[1] / len; n[2] = g[2] / len;
    return true;
}

// gb = (I - n n^T) nbar / |g| with nbar = PY(kbar)/32. With FD wetting an
// obstacle cell whose normal is the contact normal gets gb = 0, and its nbar
// goes through the contact normal to its base cell (gathered
// there) and to theta (tacc of the base cell).
template <class P>
__global__ __launch_bounds__(256) void k_adj_fd_nbar(const Fields<P> F, const Adj A, const Params prm)
{
    const size_t N = F.N;
    const bool walls = F.sc->ocount > 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < F.N; i += gridDim.x * 256) {
        const Nbr nb(i, F.nx, F.ny, F.nz);
        const uint8_t fl = F.flags[i];
        double b[3];
        py_grad(A.kbar, nb, b[0], b[1], b[2]);
        for (int k = 0; k < 3; ++k) b[k] /= 32.0;
        double o[3] = {0.0, 0.0, 0.0};
        bool overridden = false;
        if (walls && (fl & FL_OBST)) {
            double w[3];
            const int qb = fd_contact_base_d(F, nb, w);
            if (qb) {
                const Nbr nj(nb.at(dir_x(qb), dir_y(qb), dir_z(qb)), F.nx, F.ny, F.nz);
                double g[3], n[3], len, nbb[3] = {0, 0, 0}, thb = 0.0;
                py_grad(A.ms, nj, g[0], g[1], g[2]);
                const double ob[3] = {0, 0, 0};
                overridden = unit_of(g, n, len) && fd_contact_normal_adj(w, n, prm.cos_theta, prm.sin_theta, ob, nbb, thb);
            }
        }
        if (!overridden && walls && !(fl & FL_OBST) && (fl & FL_NEAR_OBST)) {
            // obstacle neighbours o = i - c_q whose base cell is i
            double g[3], n[3], len;
            py_grad(A.ms, nb, g[0], g[1], g[2]);
            if (unit_of(g, n, len)) {
                double thb = 0.0;
                for (int q = 1; q < NQ; ++q) {
                    const int oc = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
                    if (!(F.flags[oc] & FL_OBST)) continue;
                    const Nbr no(oc, F.nx, F.ny, F.nz);
                    double w[3];
                    if (fd_contact_base_d(F, no, w) != q) continue;
                    double ob[3];
                    py_grad(A.kbar, no, ob[0], ob[1], ob[2]);
                    for (int k = 0; k < 3; ++k) ob[k] /= 32.0;
                    fd_contact_normal_adj(w, n, prm.cos_theta, prm.sin_theta, ob, b, thb);
                }
                A.tacc[i] += thb;
            }
        }
        if (!overridden && (b[0] != 0.0 || b[1] != 0.0 || b[2] != 0.0)) {
            double g[3], n[3], len;
            py_grad(A.ms, nb, g[0], g[1], g[2]);
            if (unit_of(g, n, len)) {
                const double d = b[0] * n[0] + b[1] * n[1] + b[2] * n[2];
                for (int k = 0; k < 3; ++k) o[k] = (b[k] - d * n[k]) / len;
            }
        }
        A.gb[i] = o[0];
        A.gb[N + i] = o[1];
        A.gb[2 * N + i] = o[2];
    }
}

// Transposed PY gradient of the three planes of gb: -(PY_x gb_x + PY_y gb_y + PY_z gb_z).
__device__ inline double py_div_t(const double *gb, size_t N, const Nbr &nb)
{
    double s = 0.0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            const double w = pyw(a) * pyw(b);
            s += w * (gb[nb.at(1, a, b)] - gb[nb.at(-1, a, b)]);
            s += w * (gb[N + nb.at(a, 1, b)] - gb[N + nb.at(a, -1, b)]);
            s += w * (gb[2 * N + nb.at(a, b, 1)] - gb[2 * N + nb.at(a, b, -1)]);
        }
    return -s;
}

template <class P>
__global__ __launch_bounds__(256) void k_adj_fd_msb(const Fields<P> F, const Adj A)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < F.N; i += gridDim.x * 256) {
        const Nbr nb(i, F.nx, F.ny, F.nz);
        A.msb[i] = py_div_t(A.gb, F.N, nb);
    }
}

// phib += K8 * msb / 942 at interface cells; at obstacle cells the value is
// kept in phib for the transposed reflection.
template <class P>
__global__ __launch_bounds__(256) void k_adj_fd_phib(const Fields<P> F, const Adj A)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < F.N; i += gridDim.x * 256) {
        const uint8_t fl = F.flags[i];
        if (!(fl & (FL_IF | FL_OBST))) continue;
        const Nbr nb(i, F.nx, F.ny, F.nz);
        double s = 0.0;
#pragma unroll
        for (int c = -1; c <= 1; ++c)
#pragma unroll
            for (int b = -1; b <= 1; ++b)
#pragma unroll
                for (int a = -1; a <= 1; ++a) s += k8w(a * a + b * b + c * c) * A.msb[nb.at(a, b, c)];
        s *= K8_INV;
        if (fl & FL_IF) A.phib[i] += s;
        else A.phib[i] = s;
    }
}

// --------------------------------------- obstacle fill reflection (reverse)
// phi(o) = sum_j w_oj phi(j) / sum_j w_oj over fluid neighbours j with
// aperture w_oj > sqrt(2)/2; interface cell i gathers phib(o) w_oi / den_o
// from each obstacle neighbour o. The weights depend on the cell types only,
// so they are computed once per reverse sweep (k_adj_reflect_setup).
template <class P>
__global__ __launch_bounds__(256) void k_adj_reflect_setup(const Fields<P> F, const Adj A)
{
    const int n = F.sc->icount;
    const double alpha = 0.70710678118654752440 + 1e-12;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        double *c = A.refl + (size_t)(NQ - 1) * k;
        const bool near = (F.flags[i] & FL_NEAR_OBST) != 0;
        const Nbr ni(i, F.nx, F.ny, F.nz);
        for (int q = 1; q < NQ; ++q) {
            c[q - 1] = 0.0;
            if (!near) continue;
            const int o = ni.at(dir_x(q), dir_y(q), dir_z(q));
            if (!(F.flags[o] & FL_OBST)) continue;
            const Nbr no(o, F.nx, F.ny, F.nz);
            int sx = 0, sy = 0, sz = 0;
            for (int p = 1; p < NQ; ++p)
                if (!(F.flags[no.at(dir_x(p), dir_y(p), dir_z(p))] & FL_OBST)) {
                    sx += dir_x(p); sy += dir_y(p); sz += dir_z(p);
                }
            const double len = sqrt(double(sx * sx + sy * sy + sz * sz));
            if (!(len > 0)) continue;
            const double wx = sx / len, wy = sy / len, wz = sz / len;
            double den = 0.0, wi = 0.0;
            for (int p = 1; p < NQ; ++p) {
                const int j = no.at(dir_x(p), dir_y(p), dir_z(p));
                if (!(F.flags[j] & FL_FLUID)) continue;
                const double cl = sqrt(double(dir_len2(p)));
                const double w = fabs((wx * dir_x(p) + wy * dir_y(p) + wz * dir_z(p)) / cl);
                if (w > alpha) {
                    den += w;
                    if (p == opp(q)) wi = w;  // o + c_p = i
                }
            }
            if (den > 0.0 && wi > 0.0) c[q - 1] = wi / den;
        }
    }
}

// ------------------------------------------------ PLIC offset derivatives
// For the plane n.y = a (|n| = 1) through the cell [-1/2, 1/2]^3, the cut
// volume V(a, n) = |{y : n.y >= a}| has dV/da = -A and dV/dn = A c, A the
// area of the plane section and c its centroid. With V(a, n) = phi the
// implicit function theorem gives da/dphi = -1/A and da/dn = c.
__host__ __device__ inline bool plic_section(const double (&n)[3], double a, double &area, double (&cen)[3])
{
    double pts[12][3];
    int np = 0;
    for (int e = 0; e < 3; ++e) {
        if (n[e] == 0.0) continue;
        const int e1 = (e + 1) % 3, e2 = (e + 2) % 3;
        for (int s = 0; s < 4; ++s) {
            const double y1 = (s & 1) ? 0.5 : -0.5, y2 = (s & 2) ? 0.5 : -0.5;
            const double t = (a - n[e1] * y1 - n[e2] * y2) / n[e];
            if (!(t >= -0.5 && t <= 0.5)) continue;
            pts[np][e] = t;
            pts[np][e1] = y1;
            pts[np][e2] = y2;
            ++np;
        }
    }
    if (np < 3) return false;
    double m[3] = {0, 0, 0};
    for (int k = 0; k < np; ++k)
        for (int d = 0; d < 3; ++d) m[d] += pts[k][d] / np;
    // orthonormal basis (b1, b2) of the plane
    int ax = 0;
    if (fabs(n[1]) < fabs(n[ax])) ax = 1;
    if (fabs(n[2]) < fabs(n[ax])) ax = 2;
    double b1[3] = {-n[ax] * n[0], -n[ax] * n[1], -n[ax] * n[2]};
    b1[ax] += 1.0;
    const double l1 = sqrt(dot(b1, b1));
    for (int d = 0; d < 3; ++d) b1[d] /= l1;
    const double b2[3] = {n[1] * b1[2] - n[2] * b1[1], n[2] * b1[0] - n[0] * b1[2], n[0] * b1[1] - n[1] * b1[0]};
    double u[12], v[12], ang[12];
    int idx[12];
    for (int k = 0; k < np; ++k) {
        const double r[3] = {pts[k][0] - m[0], pts[k][1] - m[1], pts[k][2] - m[2]};
        u[k] = dot(r, b1);
        v[k] = dot(r, b2);
        ang[k] = atan2(v[k], u[k]);
        idx[k] = k;
    }
    for (int k = 1; k < np; ++k) {  // insertion sort by angle
        const int c = idx[k];
        int j = k - 1;
        while (j >= 0 && ang[idx[j]] > ang[c]) {
            idx[j + 1] = idx[j];
            --j;
        }
        idx[j + 1] = c;
    }
    double A = 0.0, cu = 0.0, cv = 0.0;
    for (int k = 0; k < np; ++k) {
        const int p = idx[k], q = idx[(k + 1) % np];
        const double t = 0.5 * (u[p] * v[q] - u[q] * v[p]);
        A += t;
        cu += t * (u[p] + u[q]) / 3.0;
        cv += t * (v[p] + v[q]) / 3.0;
    }
    if (!(A > 1e-14)) return false;
    cu /= A;
    cv /= A;
    for (int d = 0; d < 3; ++d) cen[d] = m[d] + cu * b1[d] + cv * b2[d];
    area = A;
    return true;
}

// da/dphi and da/dn of the PLIC offset a(n, phi) of a unit normal; phi is
// clamped to [0, 1] by the offset solver, where a = -+|n|_1/2 and
// da/dn = -+sign(n)/2.
__host__ __device__ inline void plic_derivs(const double (&n)[3], double phi, double a, double &dphi, double (&dn)[3])
{
    dphi = 0.0;
    dn[0] = dn[1] = dn[2] = 0.0;
    if (phi <= 0.0 || phi >= 1.0) {
        const double s = phi <= 0.0 ? 0.5 : -0.5;
        for (int d = 0; d < 3; ++d) dn[d] = n[d] > 0.0 ? s : (n[d] < 0.0 ? -s : 0.0);
        return;
    }
    double A, c[3];
    if (!plic_section(n, a, A, c)) return;
    dphi = -1.0 / A;
    for (int d = 0; d < 3; ++d) dn[d] = c[d];
}

// ------------------------------------------------ LSQR curvature (reverse)
// contact_condition and its reverse in one pass: the forward values
// (u_c, v_c, -m_u/m_n, -m_v/m_n) go to seeds(uc, vc, ru, rv, ucb, vcb, rub,
// rvb), which returns their adjoints; from those the adjoints of p_c, n_c,
// t_u, t_v, of the contact cell's normal and PLIC offset (into its slot of
// cb) and of theta are accumulated. Nothing happens (seeds is not called)
// where contact_condition skips the condition.
template <class View, class Seeds>
__host__ __device__ inline void contact_condition_adj(const View &V, int dx, int dy, int dz, const double (&pc)[3],
                                                      const double (&nc)[3], const double (&tu)[3],
                                                      const double (&tv)[3], const Params &prm, Seeds &&seeds,
                                                      double (&pcb)[3], double (&ncb)[3], double (&tub)[3],
                                                      double (&tvb)[3], double *cb, double &thb)
{
    double nj[3];
    V.normal(dx, dy, dz, nj);
    if (nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0) return;
    int sx = 0, sy = 0, sz = 0;
    for (int q = 1; q < NQ; ++q)
        if (V.flag(dx + dir_x(q), dy + dir_y(q), dz + dir_z(q)) & FL_OBST) {
            sx += dir_x(q); sy += dir_y(q); sz += dir_z(q);
        }
    const double lw = sqrt(double(sx * sx + sy * sy + sz * sz));
    if (!(lw > 0.0)) return;
    const double nw[3] = {sx / lw, sy / lw, sz / lw};
    const double nn = dot(nj, nw);
    const double ntr[3] = {nj[0] - nn * nw[0], nj[1] - nn * nw[1], nj[2] - nn * nw[2]};
    const double lt = sqrt(dot(ntr, ntr));
    if (lt < 1e-12) return;
    const double nt[3] = {ntr[0] / lt, ntr[1] / lt, ntr[2] / lt};
    const double ct = prm.cos_theta, st = prm.sin_theta;
    const double mh[3] = {nw[0] * ct + nt[0] * st, nw[1] * ct + nt[1] * st, nw[2] * ct + nt[2] * st};
    const double g[3] = {nw[0] - nn * nj[0], nw[1] - nn * nj[1], nw[2] - nn * nj[2]};
    const double gn = dot(g, nw);
    if (gn < 1e-12) return;
    const double aj = V.plic(dx, dy, dz);
    const double pj[3] = {aj * nj[0], aj * nj[1], aj * nj[2]};
    const double t = (0.5 - dot(pj, nw)) / gn;
    const double r[3] = {dx + pj[0] + t * g[0] - pc[0], dy + pj[1] + t * g[1] - pc[1], dz + pj[2] + t * g[2] - pc[2]};
    const double mu = dot(mh, tu), mv = dot(mh, tv), mn = dot(mh, nc);
    if (fabs(mn) < 1e-6) return;
    double ucb, vcb, rub, rvb;
    seeds(dot(r, tu), dot(r, tv), -mu / mn, -mv / mn, ucb, vcb, rub, rvb);
    // reverse
    const double mub = -rub / mn, mvb = -rvb / mn, mnb = (rub * mu + rvb * mv) / (mn * mn);
    double mhb[3], rb[3], pjb[3], gb[3], njb[3];
    for (int k = 0; k < 3; ++k) {
        mhb[k] = mub * tu[k] + mvb * tv[k] + mnb * nc[k];
        tub[k] += mub * mh[k] + ucb * r[k];
        tvb[k] += mvb * mh[k] + vcb * r[k];
        ncb[k] += mnb * mh[k];
        rb[k] = ucb * tu[k] + vcb * tv[k];
        pcb[k] -= rb[k];
        pjb[k] = rb[k];
    }
    const double tb = dot(rb, g);
    for (int k = 0; k < 3; ++k) gb[k] = t * rb[k];
    // t = (1/2 - pj.nw) / gn
    const double gnb = -tb * t / gn;
    for (int k = 0; k < 3; ++k) {
        pjb[k] -= (tb / gn) * nw[k];
        gb[k] += gnb * nw[k];
    }
    // g = nw - nn nj
    double nnb = -dot(gb, nj);
    for (int k = 0; k < 3; ++k) njb[k] = -nn * gb[k] + aj * pjb[k];
    const double ajb = dot(pjb, nj);
    // m = nw cos(theta) + nt sin(theta)
    thb += -st * dot(mhb, nw) + ct * dot(mhb, nt);
    double ntb[3] = {st * mhb[0], st * mhb[1], st * mhb[2]};
    const double dn = dot(ntb, nt);
    for (int k = 0; k < 3; ++k) {
        const double ntrb = (ntb[k] - dn * nt[k]) / lt;
        njb[k] += ntrb;
        nnb -= ntrb * nw[k];
    }
    for (int k = 0; k < 3; ++k) njb[k] += nnb * nw[k];
    double *c = cb + 4 * slot27(dx, dy, dz);
    c[0] += njb[0];
    c[1] += njb[1];
    c[2] += njb[2];
    c[3] += ajb;
}

// Sum of v over the L lanes of a group (xor butterfly; L = 1: nothing).
template <int L>
__host__ __device__ inline double group_sum(double v)
{
    if constexpr (L > 1) {
#pragma unroll
        for (int m = 1; m < L; m <<= 1) v += __shfl_xor(v, m, L);
    }
    return v;
}
template <int L>
__host__ __device__ inline int group_sum_int(int v)
{
    if constexpr (L > 1) {
#pragma unroll
        for (int m = 1; m < L; m <<= 1) v += __shfl_xor(v, m, L);
    }
    return v;
}

// Reverse of the LSQR curvature for dL/dK = Kb, by the L lanes of a group
// (lane = 0..L-1; L = 1 is the plain serial form). The forward fit is
// recomputed (same rows and model choice as lsqr_curvature, sums reduced
// over the lanes): the frame, the centre's hard constraint, the normal
// equations, their solution x and y = G^-1 xbar are the same on every lane.
// Lane l owns the block cells s = l, l + L, ... (s = slot27): it forms
// their rows' adjoints (bbar = m.y, mbar = r y - (m.y) x per row) and
// writes dL/dn_s, dL/da_s into cb[4 s + 0..3]. The adjoints of the shared
// quantities (centre point, frame, hard-constraint values, theta) are
// reduced over the lanes; lane 0 then reverses the centre's hard
// constraint and the frame into slot 13 and returns dL/dtheta in thb (the
// other lanes return 0).
template <int L, class View>
__host__ __device__ inline void lsqr_curvature_adj(const View &V, const Params &prm, double Kb, int lane, double *cb,
                                                   double &thb)
{
    thb = 0.0;
    double nc[3];
    V.normal(0, 0, 0, nc);
    if (nc[0] == 0.0 && nc[1] == 0.0 && nc[2] == 0.0) return;
    int ax = 0;
    if (fabs(nc[1]) < fabs(nc[ax])) ax = 1;
    if (fabs(nc[2]) < fabs(nc[ax])) ax = 2;
    const double nax = ax == 0 ? nc[0] : (ax == 1 ? nc[1] : nc[2]);
    double tu[3] = {-nax * nc[0] + (ax == 0 ? 1.0 : 0.0), -nax * nc[1] + (ax == 1 ? 1.0 : 0.0),
                    -nax * nc[2] + (ax == 2 ? 1.0 : 0.0)};
    const double ltu = sqrt(dot(tu, tu));
    tu[0] /= ltu; tu[1] /= ltu; tu[2] /= ltu;
    const double tv[3] = {nc[1] * tu[2] - nc[2] * tu[1], nc[2] * tu[0] - nc[0] * tu[2], nc[0] * tu[1] - nc[1] * tu[0]};
    const double ac = V.plic(0, 0, 0);
    const double pc[3] = {ac * nc[0], ac * nc[1], ac * nc[2]};
    int ob = 0;
    for (int s = lane; s < 27; s += L) ob |= (V.flag(s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1) & FL_OBST) != 0;
    const bool has_obst = group_sum_int<L>(ob) != 0;
    LsqrFrame fr;
    for (int k = 0; k < 3; ++k) {
        fr.nc[k] = nc[k];
        fr.tu[k] = tu[k];
        fr.tv[k] = tv[k];
        fr.pc[k] = pc[k];
    }
    fr.ok = true;
    fr.has_obst = has_obst;
    fr.hard = false;
    fr.huc = fr.hvc = fr.hu = fr.hv = 0.0;
    if (has_obst && (V.flag(0, 0, 0) & FL_NEAR_OBST))
        fr.hard = contact_condition(V, 0, 0, 0, pc, nc, tu, tv, prm, fr.huc, fr.hvc, fr.hu, fr.hv);
    const bool hard = fr.hard;
    const double huc = fr.huc, hvc = fr.hvc, hu = fr.hu, hv = fr.hv;

    // ---- forward fit, rows split over the lanes
    LsqrSums S;
    for (int s = lane; s < 27; s += L) lsqr_cell_rows(V, prm, fr, s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1, S);
    if (has_obst)
        for (int s = lane; s < 27; s += L) lsqr_contact_rows(V, prm, fr, s % 3 - 1, (s / 3) % 3 - 1, s / 9 - 1, S);
    for (int e = 0; e < 15; ++e) S.G[e] = group_sum<L>(S.G[e]);
    for (int e = 0; e < 5; ++e) S.g[e] = group_sum<L>(S.g[e]);
    S.rows = group_sum_int<L>(S.rows);
    // model: 0 none, 1 free 5, 2 free isotropic 3, 3 hard 3, 4 hard isotropic 1
    // (the same choice as lsqr_solve_curvature)
    int model = 0;
    double x[5] = {0, 0, 0, 0, 0};
    double Gm[15];
    double A = 0, Bq = 0, C = 0, H = 0, I = 0;
    const double *G = S.G, *g = S.g;
    const double G3i[6] = {G[0] + 2.0 * G[1] + G[2], G[6] + G[7], G[9], G[10] + G[11], G[13], G[14]};
    const double G1[1] = {G[0] + 2.0 * G[1] + G[2]};
    if (!hard) {
        double x5[5];
        if (S.rows >= 5 && packed_solve<5>(G, g, x5)) {
            model = 1;
            for (int k = 0; k < 5; ++k) x[k] = x5[k];
            A = x5[0]; Bq = x5[1]; C = x5[2]; H = x5[3]; I = x5[4];
        } else if (S.rows >= 3) {
            const double g3[3] = {g[0] + g[1], g[3], g[4]};
            double x3[3];
            if (packed_solve<3>(G3i, g3, x3)) {
                model = 2;
                x[0] = x3[0]; x[1] = x3[1]; x[2] = x3[2];
                A = x3[0]; Bq = x3[0]; C = 0.0; H = x3[1]; I = x3[2];
            }
        }
    } else {
        double x3[3];
        if (S.rows >= 3 && packed_solve<3>(G, g, x3)) {
            model = 3;
            x[0] = x3[0]; x[1] = x3[1]; x[2] = x3[2];
            A = x3[0]; Bq = x3[1]; C = x3[2];
        } else if (S.rows >= 1) {
            const double g1[1] = {g[0] + g[1]};
            double x1[1];
            if (packed_solve<1>(G1, g1, x1)) {
                model = 4;
                x[0] = x1[0];
                A = x1[0]; Bq = x1[0]; C = 0.0;
            }
        }
        H = hu - 2.0 * huc * A - hvc * C;
        I = hv - 2.0 * hvc * Bq - huc * C;
    }
    if (model == 0) return;

    // ---- K = 2 (A (1 + I^2) + B (1 + H^2) - C H I) / (1 + H^2 + I^2)^(3/2)
    const double gg = 1.0 + H * H + I * I;
    const double Nn = A * (1.0 + I * I) + Bq * (1.0 + H * H) - C * H * I;
    const double Nb = 2.0 * Kb / (gg * sqrt(gg));
    const double ggb = -3.0 * Nn * Kb / (gg * gg * sqrt(gg));
    double Ab = Nb * (1.0 + I * I), Bb = Nb * (1.0 + H * H), Cb = -Nb * H * I;
    const double Hb = Nb * (2.0 * Bq * H - C * I) + 2.0 * H * ggb;
    const double Ib = Nb * (2.0 * A * I - C * H) + 2.0 * I * ggb;
    // direct (not per row) adjoints of the centre's hard-constraint values
    double hucb0 = 0, hvcb0 = 0, hub0 = 0, hvb0 = 0;
    if (hard) {
        // H = hu - 2 huc A - hvc C, I = hv - 2 hvc B - huc C
        hub0 = Hb;
        hvb0 = Ib;
        hucb0 = -2.0 * A * Hb - C * Ib;
        hvcb0 = -C * Hb - 2.0 * Bq * Ib;
        Ab += -2.0 * huc * Hb;
        Bb += -2.0 * hvc * Ib;
        Cb += -hvc * Hb - huc * Ib;
    }
    // y = G^-1 xbar for the chosen model
    double y[5] = {0, 0, 0, 0, 0};
    if (model == 1) {
        const double xb[5] = {Ab, Bb, Cb, Hb, Ib};
        double yy[5];
        packed_solve<5>(G, xb, yy);
        for (int k = 0; k < 5; ++k) y[k] = yy[k];
    } else if (model == 2 || model == 3) {
        const double xb[3] = {model == 2 ? Ab + Bb : Ab, model == 2 ? Hb : Bb, model == 2 ? Ib : Cb};
        double yy[3];
        packed_solve<3>(model == 2 ? G3i : G, xb, yy);
        for (int k = 0; k < 3; ++k) y[k] = yy[k];
    } else {
        const double xb[1] = {Ab + Bb};
        double yy[1];
        packed_solve<1>(G1, xb, yy);
        y[0] = yy[0];
    }
    // per-row adjoints; the hard-constraint adjoints they produce are summed
    // in hucb .. hvb (this lane's rows only)
    double hucb = 0, hvcb = 0, hub = 0, hvb = 0;
    auto row_adj = [&](const double (&r)[5], double b, double (&rb)[5], double &bb) {
        for (int k = 0; k < 5; ++k) rb[k] = 0.0;
        bb = 0.0;
        if (model == 1) {
            double ax5 = 0, ay = 0;
            for (int k = 0; k < 5; ++k) { ax5 += r[k] * x[k]; ay += r[k] * y[k]; }
            const double res = b - ax5;
            bb = ay;
            for (int k = 0; k < 5; ++k) rb[k] = res * y[k] - ay * x[k];
        } else if (model == 2) {
            const double a3[3] = {r[0] + r[1], r[3], r[4]};
            double ax3 = 0, ay = 0;
            for (int k = 0; k < 3; ++k) { ax3 += a3[k] * x[k]; ay += a3[k] * y[k]; }
            const double res = b - ax3;
            bb = ay;
            const double a0b = res * y[0] - ay * x[0];
            rb[0] = a0b;
            rb[1] = a0b;
            rb[3] = res * y[1] - ay * x[1];
            rb[4] = res * y[2] - ay * x[2];
        } else {
            const double e0 = r[0] - r[3] * (2.0 * huc), e1 = r[1] - r[4] * (2.0 * hvc);
            const double e2 = r[2] - r[3] * hvc - r[4] * huc;
            const double be = b - r[3] * hu - r[4] * hv;
            double eb0, eb1, eb2, beb;
            if (model == 3) {
                const double e[3] = {e0, e1, e2};
                double ex = 0, ey = 0;
                for (int k = 0; k < 3; ++k) { ex += e[k] * x[k]; ey += e[k] * y[k]; }
                const double res = be - ex;
                beb = ey;
                eb0 = res * y[0] - ey * x[0];
                eb1 = res * y[1] - ey * x[1];
                eb2 = res * y[2] - ey * x[2];
            } else {
                const double e = e0 + e1;
                const double res = be - e * x[0];
                beb = e * y[0];
                eb0 = eb1 = res * y[0] - e * y[0] * x[0];
                eb2 = 0.0;
            }
            rb[0] = eb0;
            rb[1] = eb1;
            rb[2] = eb2;
            rb[3] = -2.0 * huc * eb0 - hvc * eb2 - hu * beb;
            rb[4] = -2.0 * hvc * eb1 - huc * eb2 - hv * beb;
            bb = beb;
            hucb += -2.0 * r[3] * eb0 - r[4] * eb2;
            hvcb += -2.0 * r[4] * eb1 - r[3] * eb2;
            hub += -r[3] * beb;
            hvb += -r[4] * beb;
        }
    };
    double pcb[3] = {0, 0, 0}, ncb[3] = {0, 0, 0}, tub[3] = {0, 0, 0}, tvb[3] = {0, 0, 0};
    double thl = 0.0;
    // ---- data rows of this lane's block cells
    for (int s = lane; s < 27; s += L) {
        const int a = s % 3 - 1, b = (s / 3) % 3 - 1, c = s / 9 - 1;
        if (a == 0 && b == 0 && c == 0) continue;
        if (!(V.flag(a, b, c) & FL_IF)) continue;
        double nj[3];
        V.normal(a, b, c, nj);
        if (nj[0] == 0.0 && nj[1] == 0.0 && nj[2] == 0.0) continue;
        const double aj = V.plic(a, b, c);
        const double r[3] = {a + aj * nj[0] - pc[0], b + aj * nj[1] - pc[1], c + aj * nj[2] - pc[2]};
        const double u = dot(r, tu), v = dot(r, tv), w = dot(r, nc);
        const double row[5] = {u * u, v * v, u * v, u, v};
        double rb5[5], bb;
        row_adj(row, w, rb5, bb);
        const double ub = 2.0 * u * rb5[0] + v * rb5[2] + rb5[3];
        const double vb = 2.0 * v * rb5[1] + u * rb5[2] + rb5[4];
        double rr[3];
        for (int k = 0; k < 3; ++k) {
            rr[k] = ub * tu[k] + vb * tv[k] + bb * nc[k];
            tub[k] += ub * r[k];
            tvb[k] += vb * r[k];
            ncb[k] += bb * r[k];
            pcb[k] -= rr[k];
        }
        double *cs = cb + 4 * s;
        cs[0] += aj * rr[0];
        cs[1] += aj * rr[1];
        cs[2] += aj * rr[2];
        cs[3] += dot(nj, rr);
    }
    // ---- contact rows of this lane's contact-line cells
    if (has_obst) {
        for (int s = lane; s < 27; s += L) {
            const int a = s % 3 - 1, b = (s / 3) % 3 - 1, c = s / 9 - 1;
            if (a == 0 && b == 0 && c == 0) continue;
            const uint8_t fj = V.flag(a, b, c);
            if (!((fj & FL_IF) && (fj & FL_NEAR_OBST))) continue;
            // the two gradient rows of the cell and their adjoints
            auto seeds = [&](double uc, double vc, double ru, double rv, double &ucb, double &vcb, double &rub,
                             double &rvb) {
                const double row1[5] = {2.0 * uc, 0.0, vc, 1.0, 0.0};
                const double row2[5] = {0.0, 2.0 * vc, uc, 0.0, 1.0};
                double p5[5], q5[5];
                row_adj(row1, ru, p5, rub);
                row_adj(row2, rv, q5, rvb);
                ucb = 2.0 * p5[0] + q5[2];
                vcb = p5[2] + 2.0 * q5[1];
            };
            contact_condition_adj(V, a, b, c, pc, nc, tu, tv, prm, seeds, pcb, ncb, tub, tvb, cb, thl);
        }
    }
    // ---- shared adjoints summed over the lanes
    for (int k = 0; k < 3; ++k) {
        pcb[k] = group_sum<L>(pcb[k]);
        ncb[k] = group_sum<L>(ncb[k]);
        tub[k] = group_sum<L>(tub[k]);
        tvb[k] = group_sum<L>(tvb[k]);
    }
    hucb = group_sum<L>(hucb) + hucb0;
    hvcb = group_sum<L>(hvcb) + hvcb0;
    hub = group_sum<L>(hub) + hub0;
    hvb = group_sum<L>(hvb) + hvb0;
    thl = group_sum<L>(thl);
    if (lane != 0) return;
    thb = thl;
    // ---- hard constraint of the centre
    if (hard) {
        auto seeds = [&](double, double, double, double, double &ucb, double &vcb, double &rub, double &rvb) {
            ucb = hucb;
            vcb = hvcb;
            rub = hub;
            rvb = hvb;
        };
        contact_condition_adj(V, 0, 0, 0, pc, nc, tu, tv, prm, seeds, pcb, ncb, tub, tvb, cb, thb);
    }
    // ---- frame: t_v = n x t_u, t_u = w/|w|, w = e_ax - n_ax n; p_c = a_c n
    ncb[0] += tu[1] * tvb[2] - tu[2] * tvb[1];
    ncb[1] += tu[2] * tvb[0] - tu[0] * tvb[2];
    ncb[2] += tu[0] * tvb[1] - tu[1] * tvb[0];
    tub[0] += tvb[1] * nc[2] - tvb[2] * nc[1];
    tub[1] += tvb[2] * nc[0] - tvb[0] * nc[2];
    tub[2] += tvb[0] * nc[1] - tvb[1] * nc[0];
    const double tt = dot(tub, tu);
    double wb[3];
    for (int k = 0; k < 3; ++k) wb[k] = (tub[k] - tt * tu[k]) / ltu;
    const double wn = dot(wb, nc);
    for (int k = 0; k < 3; ++k) ncb[k] += -nax * wb[k];
    ncb[0] += ax == 0 ? -wn : 0.0;
    ncb[1] += ax == 1 ? -wn : 0.0;
    ncb[2] += ax == 2 ? -wn : 0.0;
    const double acb = dot(pcb, nc);
    for (int k = 0; k < 3; ++k) ncb[k] += ac * pcb[k];
    double *c0 = cb + 4 * slot27(0, 0, 0);
    c0[0] += ncb[0];
    c0[1] += ncb[1];
    c0[2] += ncb[2];
    c0[3] += acb;
}

// Per interface cell, 16 lanes (measured faster than 8: the block cells'
// rows and contact conditions spread over more lanes shorten the chain of
// the wall cells, which sets the kernel's time): partials of K w.r.t. the
// normals and PLIC offsets of its block, scaled by dL/dK, into contrib;
// dL/dtheta into tacc.
constexpr int ADJ_LANES = 16;

template <class P>
__device__ inline void plic_derivs_blocks(const Fields<P> &F, const Adj &A, int b, int nb);

// The launch also computes the PLIC derivatives (plic_derivs_blocks): blocks
// from cell_blocks on take that independent work, which then runs in the
// slots the long per-cell blocks leave free instead of after them.
template <class P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_lsqr_cell(const Fields<P> F, const Adj A, const Params prm,
                                                       int cell_blocks)
{
    if ((int)blockIdx.x >= cell_blocks) {
        plic_derivs_blocks<P>(F, A, blockIdx.x - cell_blocks, gridDim.x - cell_blocks);
        return;
    }
    constexpr int per_block = 256 / ADJ_LANES;
    __shared__ LsqrStage<typename P::R> stage[per_block];
    const int n = F.sc->icount;
    const int lane = threadIdx.x % ADJ_LANES, cl = threadIdx.x / ADJ_LANES;
    // every thread of the block runs the same iterations (the stage is
    // shared between its two barriers)
    for (int k0 = blockIdx.x * per_block; k0 < n; k0 += cell_blocks * per_block) {
        const int k = k0 + cl;
        const bool on = k < n;
        const int i = on ? F.ilist[k] : 0;
        const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
        double kb = 0.0;
        if (on) {
            double *cb = A.contrib + (size_t)CONTRIB * k;
            // each slot is written only by the lane that owns it (slot 13,
            // the centre, by lane 0), and cleared by that lane
            for (int s = lane; s < 27; s += ADJ_LANES)
                if (s != 13) cb[4 * s] = cb[4 * s + 1] = cb[4 * s + 2] = cb[4 * s + 3] = 0.0;
            if (lane == 0) cb[52] = cb[53] = cb[54] = cb[55] = 0.0;
            kb = A.kbar[i];  // the same for the whole group
            if (kb != 0.0) lsqr_stage(F, x, y, z, lane, ADJ_LANES, stage[cl]);
        }
        __syncthreads();
        if (on && kb != 0.0) {
            const LsqrLdsView<typename P::R> V{stage[cl]};
            double thb = 0.0;
            lsqr_curvature_adj<ADJ_LANES>(V, prm, kb, lane, A.contrib + (size_t)CONTRIB * k, thb);
            if (lane == 0) A.tacc[i] += thb;
        }
        __syncthreads();
    }
}

// PLIC implicit derivatives of every interface cell, one thread per cell
// (the polygon of the plane section is the heavy part of the PLIC reverse),
// run by blocks b of nb in k_adj_lsqr_cell: dphi goes to ms (unused by the
// LSQR model), dn to the cell's own gb entries, which k_adj_lsqr_plic reads
// back before it overwrites them.
template <class P>
__device__ inline void plic_derivs_blocks(const Fields<P> &F, const Adj &A, int b, int nb)
{
    const int n = F.sc->icount;
    const size_t N = F.N;
    for (int k = b * 256 + threadIdx.x; k < n; k += nb * 256) {
        const int j = F.ilist[k];
        const double nj[3] = {double(F.nrm[j]), double(F.nrm[N + j]), double(F.nrm[2 * N + j])};
        double dphi = 0.0, dn[3] = {0.0, 0.0, 0.0};
        if (nj[0] != 0.0 || nj[1] != 0.0 || nj[2] != 0.0) plic_derivs(nj, double(F.phi[j]), double(F.plic[j]), dphi, dn);
        A.ms[j] = dphi;
        A.gb[j] = dn[0];
        A.gb[N + j] = dn[1];
        A.gb[2 * N + j] = dn[2];
    }
}

// Per interface cell j, ADJ_LANES lanes: gather dL/dn_j, dL/da_j over the
// blocks containing j (lane l takes the block offsets s = l, l + ADJ_LANES,
// ...) and the Parker-Youngs gradient g of phi at j (the same split); lane
// 0 then passes dL/da_j through the PLIC offset (into phib and dL/dn_j) and
// dL/dn_j through n = g/|g| into gb (the PLIC derivatives come from
// plic_derivs_blocks).
template <class P>
__global__ __launch_bounds__(256) void k_adj_lsqr_plic(const Fields<P> F, const Adj A)
{
    const int n = F.sc->icount;
    const size_t N = F.N;
    const int lane = threadIdx.x % ADJ_LANES;
    constexpr int per_block = 256 / ADJ_LANES;
    for (int k = blockIdx.x * per_block + threadIdx.x / ADJ_LANES; k < n; k += gridDim.x * per_block) {
        const int j = F.ilist[k];
        const Nbr nb(j, F.nx, F.ny, F.nz);
        double nbar[3] = {0, 0, 0}, abar = 0, g[3] = {0, 0, 0};
        for (int s = lane; s < 27; s += ADJ_LANES) {
            const int a = s % 3 - 1, b = (s / 3) % 3 - 1, c = s / 9 - 1;
            const int i = nb.at(-a, -b, -c);  // j = i + (a, b, c)
            if (F.flags[i] & FL_IF) {
                const double *cs = A.contrib + (size_t)CONTRIB * A.pos[i] + 4 * s;
                nbar[0] += cs[0];
                nbar[1] += cs[1];
                nbar[2] += cs[2];
                abar += cs[3];
            }
            // PY weights: central difference along one axis, (1, 2, 1) across
            const double ph = double(F.phi[nb.at(a, b, c)]);
            g[0] += a * pyw(b) * pyw(c) * ph;
            g[1] += b * pyw(a) * pyw(c) * ph;
            g[2] += c * pyw(a) * pyw(b) * ph;
        }
        for (int d = 0; d < 3; ++d) {
            nbar[d] = group_sum<ADJ_LANES>(nbar[d]);
            g[d] = group_sum<ADJ_LANES>(g[d]);
        }
        abar = group_sum<ADJ_LANES>(abar);
        if (lane != 0) continue;
        const double nj[3] = {double(F.nrm[j]), double(F.nrm[N + j]), double(F.nrm[2 * N + j])};
        double o[3] = {0, 0, 0};
        if (nj[0] != 0.0 || nj[1] != 0.0 || nj[2] != 0.0) {
            const double dphi = A.ms[j], dn[3] = {A.gb[j], A.gb[N + j], A.gb[2 * N + j]};  // plic_derivs_blocks
            A.phib[j] += abar * dphi;
            for (int d = 0; d < 3; ++d) nbar[d] += abar * dn[d];
            const double len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (len > 1e-12) {
                const double u[3] = {g[0] / len, g[1] / len, g[2] / len};
                const double d = dot(nbar, u);
                for (int e = 0; e < 3; ++e) o[e] = (nbar[e] - d * u[e]) / len;
            }
        }
        A.gb[j] = o[0];
        A.gb[N + j] = o[1];
        A.gb[2 * N + j] = o[2];
    }
}

// phib += -div_PY(gb) at interface cells; the value at obstacle-list cells
// goes to their phib scratch for the reflection.
template <class P>
__global__ __launch_bounds__(256) void k_adj_lsqr_phib(const Fields<P> F, const Adj A)
{
    const int n = F.sc->icount, no = F.sc->ocount;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n + no; k += gridDim.x * 256) {
        const int i = k < n ? F.ilist[k] : F.olist[k - n];
        const Nbr nb(i, F.nx, F.ny, F.nz);
        const double v = py_div_t(A.gb, F.N, nb);
        if (k < n) A.phib[i] += v;
        else A.phib[i] = v;
    }
}

// ------------------------------------------------------ reductions
// Fixed-order sum of n values: per-block partial sums over a fixed
// partition, then one block adds the partials (same scheme as the mass).
__global__ __launch_bounds__(256) void k_adj_sum_partial(const double *v, int n, double *part, int nblocks)
{
    __shared__ double s[256];
    const int chunk = (n + nblocks - 1) / nblocks;
    const int b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    double acc = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += 256) acc += v[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void k_adj_sum_final(const double *part, int nblocks, double *out)
{
    __shared__ double s[1024];
    s[threadIdx.x] = (int)threadIdx.x < nblocks ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

}  // namespace fslbm
