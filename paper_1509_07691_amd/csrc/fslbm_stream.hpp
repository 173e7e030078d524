// Stream-collide kernel of the FSLBM time step (Sec. II), one thread per
// lattice cell, pull scheme over structure-of-arrays distributions:
//   - eq. lbe1 (streaming) with half-way bounce-back at obstacle links,
//   - eq. reconstruct at links from gas cells, with
//     rho_b = (p_g + p_s) / c_s^2 = 3 (rho_gas/3 + sigma K) and u_b the
//     cell's own velocity (momentum is a collision invariant),
//   - the corner-node rule of Fig. inhomo: an obstacle link of an interface
//     cell that also has gas links takes the free-surface rule when the
//     outgoing direction points against the normal projected into the wall,
//   - eq. advection1/2 in mass form at interface cells (the incoming
//     distribution f'_qbar(x + c_q) is exactly the pulled value),
//   - moments and the SRT or TRT collision (eq. lbe2),
//   - fill / empty classification of interface cells (counted only when
//     cell types are not frozen, so that no conversion follows; a frozen
//     window records the first step in which a cell would have converted).
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// c_q . u over the non-zero components of c_q only (a product with a zero
// component cannot be dropped by the compiler, and adding it would not
// change the sum: the two forms agree bit for bit).
template <class T>
__device__ inline T cdot(int q, T ux, T uy, T uz)
{
    const int cx = dir_x(q), cy = dir_y(q), cz = dir_z(q);
    T r = cx ? (cx > 0 ? ux : -ux) : T(0);
    if (cy) r = cx ? (cy > 0 ? r + uy : r - uy) : (cy > 0 ? uy : -uy);
    if (cz) r = (cx || cy) ? (cz > 0 ? r + uz : r - uz) : (cz > 0 ? uz : -uz);
    return r;
}

template <class T>
__device__ inline T feq(int q, T rho, T ux, T uy, T uz, T usq)
{
    const T cu = cdot<T>(q, ux, uy, uz);
    return weight<T>(q) * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
}

// f^eq_q + f^eq_qbar, the sum eq. reconstruct needs: the terms odd in c_q
// cancel.
template <class T>
__device__ inline T feq_pair(int q, T rho, T ux, T uy, T uz, T usq)
{
    const T cu = cdot<T>(q, ux, uy, uz);
    return T(2) * weight<T>(q) * rho * (T(1) + T(4.5) * cu * cu - T(1.5) * usq);
}

// Moments of 19 values: rho in fixed q order, momentum over the directions
// with a non-zero component, u = j (1 / rho).
template <class T>
__device__ inline void moments(const T (&f)[NQ], T &rho, T &ux, T &uy, T &uz)
{
    T r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        r += f[q];
        if (dir_x(q)) jx += T(dir_x(q)) * f[q];
        if (dir_y(q)) jy += T(dir_y(q)) * f[q];
        if (dir_z(q)) jz += T(dir_z(q)) * f[q];
    }
    rho = r;
    const T ir = T(1) / r;
    ux = jx * ir;
    uy = jy * ir;
    uz = jz * ir;
}

template <class T, int COLL>
__device__ inline void collide(T (&f)[NQ], const Params &p)
{
    T rho, ux, uy, uz;
    moments(f, rho, ux, uy, uz);
    const T usq = ux * ux + uy * uy + uz * uz;
    const T we = T(p.omega);
    if constexpr (COLL == 0) {
        f[0] = f[0] - we * (f[0] - feq<T>(0, rho, ux, uy, uz, usq));
        // each pair (q, qbar) shares the even part of f^eq: f^eq = a +- b
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int o = opp(q);
            if (o < q) continue;
            const T cu = cdot<T>(q, ux, uy, uz);
            const T wr = weight<T>(q) * rho;
            const T a = wr * (T(1) + T(4.5) * cu * cu - T(1.5) * usq), b = wr * (T(3) * cu);
            f[q] = f[q] - we * (f[q] - (a + b));
            f[o] = f[o] - we * (f[o] - (a - b));
        }
    } else {
        const T wo = T(p.omega_odd);
        T g[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int o = opp(q);
            const T eq = feq<T>(q, rho, ux, uy, uz, usq), eo = feq<T>(o, rho, ux, uy, uz, usq);
            const T fp = T(0.5) * (f[q] + f[o]), fm = T(0.5) * (f[q] - f[o]);
            const T ep = T(0.5) * (eq + eo), em = T(0.5) * (eq - eo);
            g[q] = f[q] - we * (fp - ep) - wo * (fm - em);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) f[q] = g[q];
    }
}

// a * b + c. The FP32 arithmetic of the shifted forms rounds once (fused);
// FP64, compared value by value with the CPU reference, rounds twice.
template <class T> __device__ inline T mla(T a, T b, T c);
template <> __device__ inline float mla<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ inline double mla<double>(double a, double b, double c) { return a * b + c; }

// Deviation form, used with the shifted storage forms (fslbm_device.hpp):
// the values are d_q = f_q - w_q. The weights sum to 1 and carry no
// momentum, so rho = 1 + sum d and rho u = sum c d, and the equilibrium
// deviation is w_q (rho - 1) + w_q rho [3 c.u + 9/2 (c.u)^2 - 3/2 u^2]. Each
// formula below is its f-form counterpart above rewritten exactly.
//
// LS: the values may be held as D_q = 2^LS d_q, the units of the F16 store
// (its scale 2^12), so that loads and stores need no scaling. Every step is
// then exactly 2^LS times its LS = 0 counterpart (sums, and products with
// one scaled factor; scaling by a power of two does not change a rounding),
// so both give the same stored bits.
template <class T, int LS = 0>
__device__ inline void moments_dev(const T (&d)[NQ], T &drho, T &ux, T &uy, T &uz)
{
    T r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        r += d[q];
        if (dir_x(q)) jx += T(dir_x(q)) * d[q];
        if (dir_y(q)) jy += T(dir_y(q)) * d[q];
        if (dir_z(q)) jz += T(dir_z(q)) * d[q];
    }
    drho = LS ? r * T(1.0 / (1 << LS)) : r;
    T ir = T(1) / (T(1) + drho);
    if (LS) ir = ir * T(1.0 / (1 << LS));
    ux = jx * ir;
    uy = jy * ir;
    uz = jz * ir;
}

// f^eq_q + f^eq_qbar - 2 w_q at rho = 1 + drho: the deviation of the pair
// sum eq. reconstruct needs.
template <class T>
__device__ inline T feq_pair_dev(int q, T drho, T ux, T uy, T uz, T usq)
{
    const T cu = cdot<T>(q, ux, uy, uz);
    return T(2) * weight<T>(q) * (drho + (T(1) + drho) * (T(4.5) * cu * cu - T(1.5) * usq));
}

template <class T, int COLL, int LS = 0>
__device__ inline void collide_dev(T (&d)[NQ], const Params &p)
{
    T drho, ux, uy, uz;
    moments_dev<T, LS>(d, drho, ux, uy, uz);
    const T rho = T(1) + drho;
    const T usq = mla(ux, ux, mla(uy, uy, uz * uz));
    const T u15 = T(1.5) * usq;
    const T we = T(p.omega);
    constexpr double SC = double(1 << LS);
    if constexpr (COLL == 0) {
        d[0] = mla(-we, d[0] - (weight<T>(0) * T(SC)) * mla(-rho, u15, drho), d[0]);
        // each pair (q, qbar): equilibrium deviations a +- b
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int o = opp(q);
            if (o < q) continue;
            const T cu = cdot<T>(q, ux, uy, uz);
            const T w = weight<T>(q) * T(SC), wr = w * rho;
            const T a = mla(wr, mla(T(4.5) * cu, cu, -u15), w * drho), b = wr * (T(3) * cu);
            d[q] = mla(-we, d[q] - (a + b), d[q]);
            d[o] = mla(-we, d[o] - (a - b), d[o]);
        }
    } else {
        const T wo = T(p.omega_odd);
        T g[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int o = opp(q);
            const T cu = cdot<T>(q, ux, uy, uz);
            const T w = weight<T>(q) * T(SC), wr = w * rho;
            // even and odd parts of the equilibrium deviation of q
            const T ev = mla(wr, mla(T(4.5) * cu, cu, -u15), w * drho), od = wr * (T(3) * cu);
            const T dp = T(0.5) * (d[q] + d[o]), dm = T(0.5) * (d[q] - d[o]);
            g[q] = mla(-wo, dm - od, mla(-we, dp - ev, d[q]));
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) d[q] = g[q];
    }
}

// Plane Q of a distribution buffer whose planes are NS elements apart.
template <class P, int Q>
__device__ inline const typename P::S *plane(const typename P::S *base, int NS)
{
    return base + (size_t)Q * (size_t)NS;
}
template <class P, int Q>
__device__ inline typename P::S *plane(typename P::S *base, int NS)
{
    return base + (size_t)Q * (size_t)NS;
}

template <class P>
__device__ inline void store_all(const Fields<P> &F, int i, const typename P::T (&f)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        switch (q) {
#define FSLBM_STORE(QQ) case QQ: store_f<P, QQ>(plane<P, QQ>(F.fdst, F.NS), i, f[q]); break;
            FSLBM_STORE(0) FSLBM_STORE(1) FSLBM_STORE(2) FSLBM_STORE(3) FSLBM_STORE(4)
            FSLBM_STORE(5) FSLBM_STORE(6) FSLBM_STORE(7) FSLBM_STORE(8) FSLBM_STORE(9)
            FSLBM_STORE(10) FSLBM_STORE(11) FSLBM_STORE(12) FSLBM_STORE(13) FSLBM_STORE(14)
            FSLBM_STORE(15) FSLBM_STORE(16) FSLBM_STORE(17) FSLBM_STORE(18)
#undef FSLBM_STORE
        }
    }
}

// Load the 19 distributions f'_q(j_q) with j_q given per direction.
template <class P>
__device__ inline void load_dirs(const Fields<P> &F, const int (&j)[NQ], typename P::T (&f)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        switch (q) {
#define FSLBM_LD(QQ) case QQ: f[q] = load_f<P, QQ>(plane<P, QQ>(F.fsrc, F.NS), j[q]); break;
            FSLBM_LD(0) FSLBM_LD(1) FSLBM_LD(2) FSLBM_LD(3) FSLBM_LD(4)
            FSLBM_LD(5) FSLBM_LD(6) FSLBM_LD(7) FSLBM_LD(8) FSLBM_LD(9)
            FSLBM_LD(10) FSLBM_LD(11) FSLBM_LD(12) FSLBM_LD(13) FSLBM_LD(14)
            FSLBM_LD(15) FSLBM_LD(16) FSLBM_LD(17) FSLBM_LD(18)
#undef FSLBM_LD
        }
    }
}

// The 19 deviations d_q(j_q) (shifted forms).
template <class P>
__device__ inline void load_dirs_dev(const Fields<P> &F, const int (&j)[NQ], typename P::T (&d)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        switch (q) {
#define FSLBM_LD(QQ) case QQ: d[q] = load_d<P, QQ>(plane<P, QQ>(F.fsrc, F.NS), j[q]); break;
            FSLBM_LD(0) FSLBM_LD(1) FSLBM_LD(2) FSLBM_LD(3) FSLBM_LD(4)
            FSLBM_LD(5) FSLBM_LD(6) FSLBM_LD(7) FSLBM_LD(8) FSLBM_LD(9)
            FSLBM_LD(10) FSLBM_LD(11) FSLBM_LD(12) FSLBM_LD(13) FSLBM_LD(14)
            FSLBM_LD(15) FSLBM_LD(16) FSLBM_LD(17) FSLBM_LD(18)
#undef FSLBM_LD
        }
    }
}

// Stores the 19 deviations of cell i (shifted forms; the 16-bit forms round
// stochastically with bits drawn from the cell and the step number).
template <class P>
__device__ inline void store_all_dev(const Fields<P> &F, int i, const typename P::T (&d)[NQ])
{
    if constexpr (sizeof(typename P::S) == 2) {
        // buffer stores, as in the lean pass (no 64-bit address per store)
        const SrBits rb(cell_seed(i, F.sc->step));
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            store_raw<P>(F.fdst + (size_t)q * (size_t)F.NS, i, d[q] * typename P::T(P::SCALE), rb.at(q), F.NS);
        return;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const uint32_t bits = 0u;
        switch (q) {
#define FSLBM_STORE(QQ) case QQ: store_d<P, QQ>(plane<P, QQ>(F.fdst, F.NS), i, d[q], bits); break;
            FSLBM_STORE(0) FSLBM_STORE(1) FSLBM_STORE(2) FSLBM_STORE(3) FSLBM_STORE(4)
            FSLBM_STORE(5) FSLBM_STORE(6) FSLBM_STORE(7) FSLBM_STORE(8) FSLBM_STORE(9)
            FSLBM_STORE(10) FSLBM_STORE(11) FSLBM_STORE(12) FSLBM_STORE(13) FSLBM_STORE(14)
            FSLBM_STORE(15) FSLBM_STORE(16) FSLBM_STORE(17) FSLBM_STORE(18)
#undef FSLBM_STORE
        }
    }
}

// The stream-collide works on f (FP64) or on d = f - w (shifted forms):
// pull, relax and push in the form of the precision.
template <class P>
__device__ inline void pull(const Fields<P> &F, const int (&j)[NQ], typename P::T (&v)[NQ])
{
    if constexpr (P::SHIFT) load_dirs_dev<P>(F, j, v);
    else load_dirs<P>(F, j, v);
}
template <class P, int COLL>
__device__ inline void relax(typename P::T (&v)[NQ], const Params &p)
{
    if constexpr (P::SHIFT) collide_dev<typename P::T, COLL>(v, p);
    else collide<typename P::T, COLL>(v, p);
}
template <class P>
__device__ inline void push(const Fields<P> &F, int i, const typename P::T (&v)[NQ])
{
    if constexpr (P::SHIFT) store_all_dev<P>(F, i, v);
    else store_all<P>(F, i, v);
}
// Moments of the pulled or own values in either form: rho - 1 (dev) or rho.
template <class P>
__device__ inline void moments_any(const typename P::T (&v)[NQ], typename P::T &r, typename P::T &ux,
                                   typename P::T &uy, typename P::T &uz)
{
    if constexpr (P::SHIFT) moments_dev(v, r, ux, uy, uz);
    else moments(v, r, ux, uy, uz);
}
// The pair term of eq. reconstruct in the form of the values (rb: rho_b - 1
// in the deviation form, rho_b otherwise).
template <class P>
__device__ inline typename P::T reconstruct_pair(int q, typename P::T rb, typename P::T ux, typename P::T uy,
                                                 typename P::T uz, typename P::T usq)
{
    if constexpr (P::SHIFT) return feq_pair_dev(q, rb, ux, uy, uz, usq);
    else return feq_pair(q, rb, ux, uy, uz, usq);
}

// Liquid cell away from walls: every D3Q19 neighbour is fluid (a liquid cell
// never touches gas), so the pull needs no neighbour types.
// The shifted forms work here in the units of the store (LS above).
template <class P, int COLL>
__device__ inline void liquid_cell(const Fields<P> &F, const Params &prm, int i, const Nbr &nb)
{
    using T = typename P::T;
    int up[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) up[q] = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
    T fin[NQ];
    if constexpr (P::SHIFT) {
        constexpr int LS = scale_log2<P>();
#pragma unroll
        for (int q = 0; q < NQ; ++q) fin[q] = load_raw<P>(F.fsrc + (size_t)q * (size_t)F.NS, up[q]);
        collide_dev<T, COLL, LS>(fin, prm);
        SrBits rb(sizeof(typename P::S) == 2 ? cell_seed(i, F.sc->step) : 0u);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            store_raw<P>(F.fdst + (size_t)q * (size_t)F.NS, i, fin[q], sizeof(typename P::S) == 2 ? rb.at(q) : 0u, F.NS);
    } else {
        pull<P>(F, up, fin);
        relax<P, COLL>(fin, prm);
        push<P>(F, i, fin);
    }
}

// Cell with wall links (IS_IF = false) or interface cell (IS_IF = true).
// All loads are issued before any of them is used: the cell's own
// distributions, the upstream neighbours' types and distributions (loaded
// whatever the neighbour type; only fluid ones are used) and, at interface
// cells, the neighbours' fill levels.
template <class P, int COLL, bool IS_IF>
__device__ inline void boundary_cell(const Fields<P> &F, const Params &prm, int i, const Nbr &nb)
{
    using T = typename P::T;
    using R = typename P::R;
    const int N = F.N;
    int up[NQ], own[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        up[q] = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
        own[q] = i;
    }
    T fo[NQ], pl[NQ];
    pull<P>(F, own, fo);
    pull<P>(F, up, pl);
    uint8_t nt[NQ];
#pragma unroll
    for (int q = 1; q < NQ; ++q) nt[q] = F.flags[up[q]] & FL_TYPE;
    T phn[NQ];
    T Kc = 0, mc = 0, phx = 0, cnx = 0, cny = 0, cnz = 0;
    if constexpr (IS_IF) {
        // phi of x + c_q, the upstream node of direction opp(q)
#pragma unroll
        for (int q = 1; q < NQ; ++q) phn[q] = T(F.phi[up[opp(q)]]);
        Kc = T(F.K[i]);
        mc = T(F.m[i]);
        phx = T(F.phi[i]);
        cnx = T(F.nrm[i]);
        cny = T(F.nrm[(size_t)N + i]);
        cnz = T(F.nrm[2 * (size_t)N + i]);
    }
    bool has_gas = false;
    int nwx = 0, nwy = 0, nwz = 0;  // sum of the directions towards obstacle neighbours
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        has_gas |= nt[q] == FL_GAS;
        if (nt[q] == FL_OBST) { nwx -= dir_x(q); nwy -= dir_y(q); nwz -= dir_z(q); }
    }
    // boundary values of eq. reconstruct
    T rb0, ubx, uby, ubz;
    moments_any<P>(fo, rb0, ubx, uby, ubz);
    const T ubsq = ubx * ubx + uby * uby + ubz * ubz;
    // rho_b (rho_b - 1 in the deviation form)
    const T rhob = T(gas_density(prm, F.sc) - (P::SHIFT ? 1.0 : 0.0)) + T(3) * T(prm.sigma) * Kc;
    // corner rule: the outgoing link c_o = -c_q takes the free-surface rule
    // when c_o . (P n) < 0, P the projection onto the wall plane; evaluated
    // as (P c_o) . n with P c_o |nw|^2 = c_o |nw|^2 - (c_o . nw) nw in exact
    // integers, so the link normal to the wall tests exactly zero.
    const bool corner = IS_IF && has_gas && (nwx | nwy | nwz) != 0;
    const int ww = nwx * nwx + nwy * nwy + nwz * nwz;
    T fin[NQ];
    fin[0] = fo[0];
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const int o = opp(q);
        const uint8_t t = nt[q];
        bool rec = t == FL_GAS;
        if (corner && t == FL_OBST) {
            const int cox = -dir_x(q), coy = -dir_y(q), coz = -dir_z(q);
            const int cw = cox * nwx + coy * nwy + coz * nwz;
            const T s = T(cox * ww - cw * nwx) * cnx + T(coy * ww - cw * nwy) * cny + T(coz * ww - cw * nwz) * cnz;
            rec = s < T(0);
        }
        const T vrec = reconstruct_pair<P>(q, rhob, ubx, uby, ubz, ubsq) - fo[o];
        fin[q] = (t & FL_FLUID) ? pl[q] : (rec ? vrec : fo[o]);
    }
    if constexpr (IS_IF) {
        // mass exchange: the neighbour x + c_q is the upstream node of o = qbar
        T dm = 0;
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int o = opp(q);
            const uint8_t tz = nt[o];
            const T k = tz == FL_LIQ ? T(1) : (tz == FL_IF ? T(0.5) * (phn[q] + phx) : T(0));
            dm += k * (fin[o] - fo[q]);
        }
        T r = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) r += fin[q];
        if constexpr (P::SHIFT) r = T(1) + r;
        const T mn = mc + dm;
        uint8_t st = CV_NONE;
        if (mn > (T(1) + T(prm.eps_c)) * r) st = CV_FILL;
        else if (mn < -T(prm.eps_c) * r) st = CV_EMPTY;
        F.m[i] = R(mn);
        F.rho[i] = R(r);
        F.conv[i] = st;
        if (st != CV_NONE) {
            if (!prm.frozen) atomicAdd(&F.sc->nconv, 1);
            else atomicMin(&F.sc->conv_out_step, F.sc->step);  // the free method would convert here
        }
    }
    relax<P, COLL>(fin, prm);
    push<P>(F, i, fin);
}

// Any fluid cell, written so that the lanes of a wavefront share the pull,
// the collision and the stores: only the boundary rules (own distributions,
// neighbour types, reconstruction, corner rule, mass exchange) diverge.
// Same arithmetic as liquid_cell / boundary_cell.
template <class P, int COLL>
__device__ inline void fluid_cell(const Fields<P> &F, const Params &prm, int i, const Nbr &nb, uint8_t fl)
{
    using T = typename P::T;
    using R = typename P::R;
    const int N = F.N;
    int up[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) up[q] = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
    T fin[NQ];
    pull<P>(F, up, fin);  // the pull; final wherever the upstream node is fluid
    if (fl != FL_LIQ) {
        const bool is_if = (fl & FL_IF) != 0;
        int own[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) own[q] = i;
        T fo[NQ];
        pull<P>(F, own, fo);
        uint8_t nt[NQ];
#pragma unroll
        for (int q = 1; q < NQ; ++q) nt[q] = F.flags[up[q]] & FL_TYPE;
        T phn[NQ];
        T Kc = 0, mc = 0, phx = 0, cnx = 0, cny = 0, cnz = 0;
        if (is_if) {
#pragma unroll
            for (int q = 1; q < NQ; ++q) phn[q] = T(F.phi[up[opp(q)]]);
            Kc = T(F.K[i]);
            mc = T(F.m[i]);
            phx = T(F.phi[i]);
            cnx = T(F.nrm[i]);
            cny = T(F.nrm[(size_t)N + i]);
            cnz = T(F.nrm[2 * (size_t)N + i]);
        }
        bool has_gas = false;
        int nwx = 0, nwy = 0, nwz = 0;
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            has_gas |= nt[q] == FL_GAS;
            if (nt[q] == FL_OBST) { nwx -= dir_x(q); nwy -= dir_y(q); nwz -= dir_z(q); }
        }
        T rb0, ubx, uby, ubz;
        moments_any<P>(fo, rb0, ubx, uby, ubz);
        const T ubsq = ubx * ubx + uby * uby + ubz * ubz;
        // rho_b (rho_b - 1 in the deviation form)
        const T rhob = T(gas_density(prm, F.sc) - (P::SHIFT ? 1.0 : 0.0)) + T(3) * T(prm.sigma) * Kc;
        const bool corner = is_if && has_gas && (nwx | nwy | nwz) != 0;
        const int ww = nwx * nwx + nwy * nwy + nwz * nwz;
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int o = opp(q);
            const uint8_t t = nt[q];
            bool rec = t == FL_GAS;
            if (corner && t == FL_OBST) {
                const int cox = -dir_x(q), coy = -dir_y(q), coz = -dir_z(q);
                const int cw = cox * nwx + coy * nwy + coz * nwz;
                const T s = T(cox * ww - cw * nwx) * cnx + T(coy * ww - cw * nwy) * cny + T(coz * ww - cw * nwz) * cnz;
                rec = s < T(0);
            }
            const T vrec = reconstruct_pair<P>(q, rhob, ubx, uby, ubz, ubsq) - fo[o];
            fin[q] = (t & FL_FLUID) ? fin[q] : (rec ? vrec : fo[o]);
        }
        if (is_if) {
            T dm = 0;
#pragma unroll
            for (int q = 1; q < NQ; ++q) {
                const int o = opp(q);
                const uint8_t tz = nt[o];
                const T k = tz == FL_LIQ ? T(1) : (tz == FL_IF ? T(0.5) * (phn[q] + phx) : T(0));
                dm += k * (fin[o] - fo[q]);
            }
            T r = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) r += fin[q];
            if constexpr (P::SHIFT) r = T(1) + r;
            const T mn = mc + dm;
            uint8_t st = CV_NONE;
            if (mn > (T(1) + T(prm.eps_c)) * r) st = CV_FILL;
            else if (mn < -T(prm.eps_c) * r) st = CV_EMPTY;
            F.m[i] = R(mn);
            F.rho[i] = R(r);
            F.conv[i] = st;
            if (st != CV_NONE) {
                if (!prm.frozen) atomicAdd(&F.sc->nconv, 1);
                else atomicMin(&F.sc->conv_out_step, F.sc->step);  // the free method would convert here
            }
        }
    }
    relax<P, COLL>(fin, prm);
    push<P>(F, i, fin);
}

// Stream-collide over the fluid bounding box. MODE 0: every fluid cell;
// MODE 1: only liquid cells away from walls (the lean pull, few registers;
// the other fluid cells then go through k_stream_collide_list). Block b
// takes the SC_BLOCK consecutive box cells from SC_BLOCK b; the host sizes the grid
// to the box it last read back, so normally each block has one chunk and
// returns (a box that has grown since is covered by a grid-stride tail).
// Blocks are dispatched in index order, so the blocks in flight at any
// moment work on one narrow window of the box and the 38 distribution
// streams stay within few DRAM pages; blocks that each walk a long share of
// the box drift apart and lose that locality.
template <class P, int COLL, int MODE>
__device__ inline void stream_collide_box(const Batch<P> &B)
{
    const Params &prm = B.p[blockIdx.y];
    if (prm.coll != COLL) return;
    const Fields<P> &F = B.f[blockIdx.y];
    const CellRange box = CellRange::from(F.sc->fbox);
    const int n = box.size();
    for (int c = xcd_chunk(blockIdx.x, gridDim.x, xcd_run<P>()); c * SC_BLOCK < n; c += gridDim.x) {
        const int k = c * SC_BLOCK + (int)threadIdx.x;
        if (k >= n) continue;
        // unsigned: the signed division costs twice the instructions
        const unsigned uk = unsigned(k), uex = unsigned(box.ex), uey = unsigned(box.ey);
        const unsigned r = uk / uex;
        const int bx = int(uk - r * uex), by = int(r % uey), bz = int(r / uey);
        const Nbr nb(box.x0 + bx, box.y0 + by, box.z0 + bz, F.nx, F.ny, F.nz);
        const int i = nb.at(0, 0, 0);
        const uint8_t fl = F.flags[i];
        if (!(fl & FL_FLUID)) continue;
        if (MODE == 1) {
            if (fl == FL_LIQ) liquid_cell<P, COLL>(F, prm, i, nb);
        } else {
            fluid_cell<P, COLL>(F, prm, i, nb, fl);
        }
    }
}

// FP32 storage: 4 waves per SIMD (the boundary path then fits in 128
// VGPRs). 16-bit storage: 3 waves per SIMD, where the boundary path takes
// 134 VGPRs without spilling (at 4 waves it spilled 6-8; the droplet
// sweep's merged pass took 102 us there against 94 us now). The lean pass
// takes 37-60 VGPRs either way. FP64 keeps the compiler's register choice
// (it would spill).
template <class P, int COLL, int MODE>
__global__ __launch_bounds__(SC_BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(typename P::S) == 2 ? 3 : 4))) void k_stream_collide(const Batch<P> B)
{
    stream_collide_box<P, COLL, MODE>(B);
}
template <int COLL, int MODE>
__global__ __launch_bounds__(SC_BLOCK) void k_stream_collide_f64(const Batch<Prec<P_F64>> B)
{
    stream_collide_box<Prec<P_F64>, COLL, MODE>(B);
}
template <class P, int COLL, int MODE>
inline void launch_stream_collide(dim3 grid, hipStream_t st, const Batch<P> &A)
{
    if constexpr (P::SHIFT == false && sizeof(typename P::T) == 8)
        k_stream_collide_f64<COLL, MODE><<<grid, SC_BLOCK, 0, st>>>(A);
    else
        k_stream_collide<P, COLL, MODE><<<grid, SC_BLOCK, 0, st>>>(A);
}

// The fluid cells that the lean box pass (MODE 1) leaves out, one thread
// per cell: the interface cells from the interface list, then the liquid
// cells of the static wall list (interface cells on that list are skipped
// there, gas cells have no update). Wavefronts hold cells of one kind, so
// the long boundary path does not stall liquid cells.
template <class P, int COLL>
__global__ __launch_bounds__(256) void k_stream_collide_list(const Batch<P> B)
{
    const Params &prm = B.p[blockIdx.y];
    if (prm.coll != COLL) return;
    const Fields<P> &F = B.f[blockIdx.y];
    const int ni = *(volatile const int *)&F.sc->icount;
    const int n = ni + F.sc->wcount;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = k < ni ? F.ilist[k] : F.wlist[k - ni];
        const Nbr nb(i, F.nx, F.ny, F.nz);
        if (k < ni) boundary_cell<P, COLL, true>(F, prm, i, nb);
        else if ((F.flags[i] & FL_TYPE) == FL_LIQ) boundary_cell<P, COLL, false>(F, prm, i, nb);
    }
}

}  // namespace fslbm
