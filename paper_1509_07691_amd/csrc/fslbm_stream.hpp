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
//   - fill / empty classification of interface cells.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

template <class T>
__device__ inline T feq(int q, T rho, T ux, T uy, T uz, T usq)
{
    const T cu = T(dir_x(q)) * ux + T(dir_y(q)) * uy + T(dir_z(q)) * uz;
    return weight<T>(q) * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
}

// Moments of 19 values: rho in fixed q order, momentum over the directions
// with a non-zero component.
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
    ux = jx / r;
    uy = jy / r;
    uz = jz / r;
}

template <class T, int COLL>
__device__ inline void collide(T (&f)[NQ], const Params &p)
{
    T rho, ux, uy, uz;
    moments(f, rho, ux, uy, uz);
    const T usq = ux * ux + uy * uy + uz * uz;
    const T we = T(p.omega);
    if constexpr (COLL == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) f[q] = f[q] - we * (f[q] - feq<T>(q, rho, ux, uy, uz, usq));
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

template <class P, int Q>
__device__ inline const typename P::S *plane(const typename P::S *base, int N)
{
    return base + (size_t)Q * (size_t)N;
}
template <class P, int Q>
__device__ inline typename P::S *plane(typename P::S *base, int N)
{
    return base + (size_t)Q * (size_t)N;
}

template <class P, int COLL>
__global__ __launch_bounds__(256) void k_stream_collide(Fields<P> F, Params prm)
{
    using T = typename P::T;
    using R = typename P::R;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    const uint8_t fl = F.flags[i];
    if (!(fl & FL_FLUID)) return;
    const int N = F.N;
    const Nbr nb(i, F.nx, F.ny, F.nz);
    T fin[NQ];

    if (fl == FL_LIQ) {
        // Liquid cell away from walls: all D3Q19 neighbours are fluid (a
        // liquid cell never touches gas), plain pull.
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int j = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
            switch (q) {
#define FSLBM_PULL(QQ) case QQ: fin[q] = load_f<P, QQ>(plane<P, QQ>(F.fsrc, N), j); break;
                FSLBM_PULL(0) FSLBM_PULL(1) FSLBM_PULL(2) FSLBM_PULL(3) FSLBM_PULL(4)
                FSLBM_PULL(5) FSLBM_PULL(6) FSLBM_PULL(7) FSLBM_PULL(8) FSLBM_PULL(9)
                FSLBM_PULL(10) FSLBM_PULL(11) FSLBM_PULL(12) FSLBM_PULL(13) FSLBM_PULL(14)
                FSLBM_PULL(15) FSLBM_PULL(16) FSLBM_PULL(17) FSLBM_PULL(18)
#undef FSLBM_PULL
            }
        }
    } else {
        const bool is_if = (fl & FL_IF) != 0;
        T fo[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            switch (q) {
#define FSLBM_OWN(QQ) case QQ: fo[q] = load_f<P, QQ>(plane<P, QQ>(F.fsrc, N), i); break;
                FSLBM_OWN(0) FSLBM_OWN(1) FSLBM_OWN(2) FSLBM_OWN(3) FSLBM_OWN(4)
                FSLBM_OWN(5) FSLBM_OWN(6) FSLBM_OWN(7) FSLBM_OWN(8) FSLBM_OWN(9)
                FSLBM_OWN(10) FSLBM_OWN(11) FSLBM_OWN(12) FSLBM_OWN(13) FSLBM_OWN(14)
                FSLBM_OWN(15) FSLBM_OWN(16) FSLBM_OWN(17) FSLBM_OWN(18)
#undef FSLBM_OWN
            }
        }
        // types of the upstream neighbours x - c_q
        uint8_t nt[NQ];
        bool has_gas = false;
        int nwx = 0, nwy = 0, nwz = 0;  // sum of c_q towards obstacle neighbours
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            nt[q] = F.flags[nb.at(-dir_x(q), -dir_y(q), -dir_z(q))] & FL_TYPE;
            has_gas |= nt[q] == FL_GAS;
            if (nt[q] == FL_OBST) { nwx -= dir_x(q); nwy -= dir_y(q); nwz -= dir_z(q); }
        }
        // boundary values of eq. reconstruct
        T rb0, ubx, uby, ubz;
        moments(fo, rb0, ubx, uby, ubz);
        const T ubsq = ubx * ubx + uby * uby + ubz * ubz;
        const T Kc = is_if ? T(F.K[i]) : T(0);
        const T rhob = T(3) * (T(prm.rho_gas) / T(3) + T(prm.sigma) * Kc);
        // corner rule: the outgoing link c_o = -c_q takes the free-surface rule
        // when c_o . (P n) < 0, P the projection onto the wall plane; evaluated
        // as (P c_o) . n with P c_o |nw|^2 = c_o |nw|^2 - (c_o . nw) nw in exact
        // integers, so the link normal to the wall tests exactly zero.
        const bool corner = is_if && has_gas && (nwx | nwy | nwz) != 0;
        const int ww = nwx * nwx + nwy * nwy + nwz * nwz;
        T cnx = 0, cny = 0, cnz = 0;
        if (corner) {
            cnx = T(F.nrm[i]);
            cny = T(F.nrm[(size_t)N + i]);
            cnz = T(F.nrm[2 * (size_t)N + i]);
        }
        fin[0] = fo[0];
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
            const int o = opp(q);
            const uint8_t t = nt[q];
            bool rec = false;
            if (t & FL_FLUID) {
                const int j = nb.at(-dir_x(q), -dir_y(q), -dir_z(q));
                switch (q) {
#define FSLBM_PULL(QQ) case QQ: fin[q] = load_f<P, QQ>(plane<P, QQ>(F.fsrc, N), j); break;
                    FSLBM_PULL(1) FSLBM_PULL(2) FSLBM_PULL(3) FSLBM_PULL(4)
                    FSLBM_PULL(5) FSLBM_PULL(6) FSLBM_PULL(7) FSLBM_PULL(8) FSLBM_PULL(9)
                    FSLBM_PULL(10) FSLBM_PULL(11) FSLBM_PULL(12) FSLBM_PULL(13) FSLBM_PULL(14)
                    FSLBM_PULL(15) FSLBM_PULL(16) FSLBM_PULL(17) FSLBM_PULL(18)
#undef FSLBM_PULL
                }
            } else if (t == FL_GAS) {
                rec = true;
            } else {
                const int cox = -dir_x(q), coy = -dir_y(q), coz = -dir_z(q);
                const int cw = cox * nwx + coy * nwy + coz * nwz;
                const T s = T(cox * ww - cw * nwx) * cnx + T(coy * ww - cw * nwy) * cny + T(coz * ww - cw * nwz) * cnz;
                if (corner && s < T(0)) rec = true;
                else fin[q] = fo[o];
            }
            if (rec)
                fin[q] = feq<T>(q, rhob, ubx, uby, ubz, ubsq) + feq<T>(o, rhob, ubx, uby, ubz, ubsq) - fo[o];
        }
        if (is_if) {
            // mass exchange: the neighbour x + c_q is the upstream node of o = qbar
            const T phx = T(F.phi[i]);
            T dm = 0;
#pragma unroll
            for (int q = 1; q < NQ; ++q) {
                const int o = opp(q);
                const uint8_t tz = nt[o];
                T k;
                if (tz == FL_LIQ) k = T(1);
                else if (tz == FL_IF) k = T(0.5) * (T(F.phi[nb.at(dir_x(q), dir_y(q), dir_z(q))]) + phx);
                else k = T(0);
                dm += k * (fin[o] - fo[q]);
            }
            T r = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) r += fin[q];
            const T mn = T(F.m[i]) + dm;
            uint8_t st = CV_NONE;
            if (mn > (T(1) + T(prm.eps_c)) * r) st = CV_FILL;
            else if (mn < -T(prm.eps_c) * r) st = CV_EMPTY;
            F.m[i] = R(mn);
            F.rho[i] = R(r);
            F.conv[i] = st;
            if (st != CV_NONE) atomicAdd(&F.sc->nconv, 1);
        }
    }
    collide<T, COLL>(fin, prm);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        switch (q) {
#define FSLBM_STORE(QQ) case QQ: store_f<P, QQ>(plane<P, QQ>(F.fdst, N), i, fin[q]); break;
            FSLBM_STORE(0) FSLBM_STORE(1) FSLBM_STORE(2) FSLBM_STORE(3) FSLBM_STORE(4)
            FSLBM_STORE(5) FSLBM_STORE(6) FSLBM_STORE(7) FSLBM_STORE(8) FSLBM_STORE(9)
            FSLBM_STORE(10) FSLBM_STORE(11) FSLBM_STORE(12) FSLBM_STORE(13) FSLBM_STORE(14)
            FSLBM_STORE(15) FSLBM_STORE(16) FSLBM_STORE(17) FSLBM_STORE(18)
#undef FSLBM_STORE
        }
    }
}

}  // namespace fslbm
