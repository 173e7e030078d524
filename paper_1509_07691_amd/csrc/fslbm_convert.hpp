// Cell-type conversion, interface-list compaction, obstacle fill reflection.
//
// The paper keeps the liquid / interface / gas classification of Sec. II
// (an interface cell has liquid and gas D3Q19 neighbours, only interface
// cells hold 0 < phi < 1) and defers the conversion rules to Koerner et al.
// This library uses the following rules, per step:
//   1  interface cells fill when m > (1 + eps) rho and empty when
//      m < -eps rho (classified in the stream-collide kernel);
//   2  filling wins: an emptying cell with a filling D3Q19 neighbour stays;
//   3  gas neighbours of filling cells and liquid neighbours of emptying
//      cells become interface cells; those from gas get
//      f' = feq(mean rho, mean u) of their liquid/interface neighbours and
//      m = 0, those from liquid keep f' and get m = rho;
//   4  closure of the interface layer (Sec. II.D: an interface cell has gas
//      and liquid D3Q19 neighbours): on the types after rules 1-3, a layer
//      cell without a gas neighbour becomes liquid; then, on the updated
//      types, one without a liquid neighbour becomes gas;
//   5  every cell that leaves the layer hands on m - rho (to liquid) or m
//      (to gas), split equally over its D3Q19 neighbours that are interface
//      cells after the step; with no such neighbour the amount goes to a
//      reservoir;
//   6  the cells take their new types.
// Rule 4 starts from a closed layer (creation closes it), so only cells of
// the step's layer (old interface cells and new cells) can break it.
// Every kernel runs over the interface list of the step (grid-stride) and is
// written as a gather: each output value has one writer, or several writers
// storing the identical value (new cells reached from several converting
// neighbours). New cells are tagged in `mark` with the step number, so no
// clearing pass is needed. Kernels return at once when no cell converts.
#pragma once

#include "fslbm_device.hpp"
#include "fslbm_stream.hpp"

namespace fslbm {

constexpr int LIST_GRID = 256;  // blocks per lattice of the grid-stride list kernels

__device__ inline int list_count(const DevScalars *sc) { return *(volatile const int *)&sc->icount; }

// A cell of the step's layer: an interface cell of the old list or a new
// cell tagged in this step (its conv status is reset when it is tagged).
template <class P>
__device__ inline bool in_layer(const Fields<P> &F, int j, uint32_t tag)
{
    return (F.flags[j] & FL_IF) || (F.mark[j] & ~3u) == tag;
}

// A cell that leaves the layer in this step. From k_conv_share_keep on,
// every such cell carries the step's tag: new cells from their tagging,
// and old-list cells that convert get tag | 3 there. The test reads no
// flags, so k_conv_gather can rewrite flags while it runs.
template <class P>
__device__ inline bool is_converter(const Fields<P> &F, int j, uint32_t tag)
{
    return (F.mark[j] & ~3u) == tag && F.conv[j] != CV_NONE;
}

// A new cell of this step (tagged 1 from gas or 2 from liquid; 3 marks an
// old-list cell that leaves the layer).
__device__ inline bool is_new(uint32_t mk, uint32_t tag) { return (mk & ~3u) == tag && (mk & 3u) != 3u; }

// Rule 2 for cell i: an emptying cell next to a filling cell does not
// empty. Returns the cell's status after it. Readers of other cells' status
// only test for CV_FILL, which this never writes or clears.
template <class P>
__device__ inline uint8_t prune_own(const Fields<P> &F, int i)
{
    uint8_t st = F.conv[i];
    if (st != CV_EMPTY) return st;
    const Nbr nb(i, F.nx, F.ny, F.nz);
    bool near_fill = false;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const int j = nb.at(dir_x(q), dir_y(q), dir_z(q));
        near_fill |= (F.flags[j] & FL_IF) && F.conv[j] == CV_FILL;
    }
    if (near_fill) {
        F.conv[i] = CV_NONE;
        st = CV_NONE;
    }
    return st;
}

__device__ inline int wrap_any(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Rules 2 and 3: prune the cell's own emptying (it reads only its
// neighbours' filling, which pruning never changes), then tag the new
// interface cells and initialise them. Cells reached from several
// converting neighbours are written identically by each. A filling or
// emptying cell also stamps the 7x7x7 box around it in `near` with the low
// byte of the step number: the closure of rule 4 can only change a cell
// within two cells of one (the layer was closed before the step), and
// the excess of rule 5 moves one cell further. A stale stamp that happens
// to match only makes a cell be checked.
template <class P>
__global__ __launch_bounds__(256) void k_conv_mark_init(const Batch<P> B)
{
    const Fields<P> &F = B.f[blockIdx.y];
    using T = typename P::T;
    using R = typename P::R;
    if (F.sc->nconv == 0) return;
    const uint32_t tag = F.sc->step << 2;
    const int n = list_count(F.sc);
    const int N = F.N;
    const int n_round = (n + 255) / 256 * 256;  // whole wavefronts iterate together
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n_round; k += gridDim.x * 256) {
        int fresh[NQ];
        int nfresh = 0;
        const int i = k < n ? F.ilist[k] : 0;
        const uint8_t st = k < n ? prune_own(F, i) : CV_NONE;
        if (st != CV_NONE) {
            const uint8_t s8 = uint8_t(tag >> 2);
            const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
            for (int dz = -3; dz <= 3; ++dz)
                for (int dy = -3; dy <= 3; ++dy) {
                    const int row = F.nx * (wrap_any(y + dy, F.ny) + F.ny * wrap_any(z + dz, F.nz));
                    for (int dx = -3; dx <= 3; ++dx) F.near[row + wrap_any(x + dx, F.nx)] = s8;
                }
        }
        const Nbr nb(i, F.nx, F.ny, F.nz);
        for (int q = 1; q < NQ && st != CV_NONE; ++q) {
            const int j = nb.at(dir_x(q), dir_y(q), dir_z(q));
            const uint8_t tj = F.flags[j] & FL_TYPE;
            if (st == CV_FILL && tj == FL_GAS) {
                // the first thread to tag j lists it as a new interface cell
                if ((atomicExch(&F.mark[j], tag | 1u) & ~3u) != tag) fresh[nfresh++] = j;
                F.conv[j] = CV_NONE;
                // mean rho and u over the liquid / interface neighbours of j
                const Nbr nj(j, F.nx, F.ny, F.nz);
                T rs = 0, usx = 0, usy = 0, usz = 0;
                int cnt = 0;
                for (int p = 1; p < NQ; ++p) {
                    const int w = nj.at(dir_x(p), dir_y(p), dir_z(p));
                    if (!(F.flags[w] & FL_FLUID)) continue;
                    T fw[NQ];
#pragma unroll
                    for (int s = 0; s < NQ; ++s) {
                        switch (s) {
#define FSLBM_LD(QQ) case QQ: fw[s] = load_f<P, QQ>(plane<P, QQ>((const typename P::S *)F.fdst, F.NS), w); break;
                            FSLBM_LD(0) FSLBM_LD(1) FSLBM_LD(2) FSLBM_LD(3) FSLBM_LD(4) FSLBM_LD(5)
                            FSLBM_LD(6) FSLBM_LD(7) FSLBM_LD(8) FSLBM_LD(9) FSLBM_LD(10) FSLBM_LD(11)
                            FSLBM_LD(12) FSLBM_LD(13) FSLBM_LD(14) FSLBM_LD(15) FSLBM_LD(16)
                            FSLBM_LD(17) FSLBM_LD(18)
#undef FSLBM_LD
                        }
                    }
                    T r, ux, uy, uz;
                    moments(fw, r, ux, uy, uz);
                    rs += r; usx += ux; usy += uy; usz += uz;
                    ++cnt;
                }
                const T rm = rs / T(cnt), ux = usx / T(cnt), uy = usy / T(cnt), uz = usz / T(cnt);
                const T usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
                for (int s = 0; s < NQ; ++s) {
                    const T v = feq<T>(s, rm, ux, uy, uz, usq);
                    switch (s) {
#define FSLBM_ST(QQ) case QQ: store_f<P, QQ>(plane<P, QQ>(F.fdst, F.NS), j, v); break;
                        FSLBM_ST(0) FSLBM_ST(1) FSLBM_ST(2) FSLBM_ST(3) FSLBM_ST(4) FSLBM_ST(5)
                        FSLBM_ST(6) FSLBM_ST(7) FSLBM_ST(8) FSLBM_ST(9) FSLBM_ST(10) FSLBM_ST(11)
                        FSLBM_ST(12) FSLBM_ST(13) FSLBM_ST(14) FSLBM_ST(15) FSLBM_ST(16)
                        FSLBM_ST(17) FSLBM_ST(18)
#undef FSLBM_ST
                    }
                }
                F.rho[j] = R(rm);
                F.m[j] = R(0);
            } else if (st == CV_EMPTY && tj == FL_LIQ) {
                if ((atomicExch(&F.mark[j], tag | 2u) & ~3u) != tag) fresh[nfresh++] = j;
                F.conv[j] = CV_NONE;
                T fw[NQ];
#pragma unroll
                for (int s = 0; s < NQ; ++s) {
                    switch (s) {
#define FSLBM_LD(QQ) case QQ: fw[s] = load_f<P, QQ>(plane<P, QQ>((const typename P::S *)F.fdst, F.NS), j); break;
                        FSLBM_LD(0) FSLBM_LD(1) FSLBM_LD(2) FSLBM_LD(3) FSLBM_LD(4) FSLBM_LD(5)
                        FSLBM_LD(6) FSLBM_LD(7) FSLBM_LD(8) FSLBM_LD(9) FSLBM_LD(10) FSLBM_LD(11)
                        FSLBM_LD(12) FSLBM_LD(13) FSLBM_LD(14) FSLBM_LD(15) FSLBM_LD(16)
                        FSLBM_LD(17) FSLBM_LD(18)
#undef FSLBM_LD
                    }
                }
                T r = 0;
#pragma unroll
                for (int s = 0; s < NQ; ++s) r += fw[s];
                F.rho[j] = R(r);
                F.m[j] = R(r);
            }
        }
        // one atomic per wavefront for the new cells found by its lanes
        const int lane = threadIdx.x & 63;
        int incl = nfresh;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        const int total = __shfl(incl, 63, 64);
        int base = 0;
        if (lane == 63 && total > 0) base = atomicAdd(&F.sc->nnew, total);
        base = __shfl(base, 63, 64) + incl - nfresh;
        for (int s = 0; s < nfresh; ++s) F.newlist[base + s] = fresh[s];
    }
}

// Cell types after rules 1-3 (CLOSE_* codes read as interface): the
// classification rule 4 starts from.
template <class P>
__device__ inline uint8_t type_after_conversion(const Fields<P> &F, int j, uint32_t tag)
{
    const uint8_t f = F.flags[j];
    if ((F.mark[j] & ~3u) == tag) return FL_IF;
    if (!(f & FL_IF)) return f & FL_TYPE;
    const uint8_t st = F.conv[j];
    return st == CV_FILL ? FL_LIQ : (st == CV_EMPTY ? FL_GAS : FL_IF);
}

// Cell k of the step's layer: the old list, then the new cells.
template <class P>
__device__ inline int layer_cell(const Fields<P> &F, int k, int n)
{
    return k < n ? F.ilist[k] : F.newlist[k - n];
}

// Rule 4 for layer cell c (types after rules 1-3, CLOSE_* codes read as
// interface): without a gas neighbour c becomes liquid; otherwise, without
// a neighbour that is liquid after the first pass (liquid, or a layer cell
// without a gas neighbour) c becomes gas.
template <class P>
__device__ inline bool lacks_gas_neighbour(const Fields<P> &F, int c, uint32_t tag)
{
    const Nbr nb(c, F.nx, F.ny, F.nz);
    bool found = false;
#pragma unroll
    for (int q = 1; q < NQ; ++q) found |= type_after_conversion(F, nb.at(dir_x(q), dir_y(q), dir_z(q)), tag) == FL_GAS;
    return !found;
}

// Rule 4, both passes in one launch: each cell writes only its own status,
// and a neighbour's first-pass result is evaluated, not read, so no thread
// depends on another's write. The second pass looks two cells out only for
// a cell without a liquid neighbour after rules 1-3, which is rare.
template <class P>
__global__ __launch_bounds__(256) void k_conv_close(const Batch<P> B)
{
    const Fields<P> &F = B.f[blockIdx.y];
    if (F.sc->nconv == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // counters of the list rebuild in k_conv_share_keep
        F.sc->nkeep = 0;
        F.sc->bbox[0] = F.nx; F.sc->bbox[1] = F.ny; F.sc->bbox[2] = F.nz;
        F.sc->bbox[3] = -1; F.sc->bbox[4] = -1; F.sc->bbox[5] = -1;
    }
    const uint32_t tag = F.sc->step << 2;
    const uint8_t s8 = uint8_t(tag >> 2);
    const int n = list_count(F.sc), nn = F.sc->nnew;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n + nn; k += gridDim.x * 256) {
        const int i = layer_cell(F, k, n);
        if (F.near[i] != s8 || F.conv[i] != CV_NONE) continue;
        // most cells have both a gas and a liquid neighbour: stop at the
        // first of each
        const Nbr nb(i, F.nx, F.ny, F.nz);
        bool gas = false, liquid = false;
        for (int q = 1; q < NQ && !(gas && liquid); ++q) {
            const uint8_t t = type_after_conversion(F, nb.at(dir_x(q), dir_y(q), dir_z(q)), tag);
            gas |= t == FL_GAS;
            liquid |= t == FL_LIQ;
        }
        if (!gas) {
            F.conv[i] = CV_CLOSE_LIQ;
            continue;
        }
        for (int q = 1; q < NQ && !liquid; ++q) {
            const int j = nb.at(dir_x(q), dir_y(q), dir_z(q));
            liquid = type_after_conversion(F, j, tag) == FL_IF && lacks_gas_neighbour(F, j, tag);
        }
        if (!liquid) F.conv[i] = CV_CLOSE_GAS;
    }
}

template <class P>
__device__ inline bool is_receiver(const Fields<P> &F, int j, uint32_t tag)
{
    return in_layer(F, j, tag) && F.conv[j] == CV_NONE;
}

// Rule 5, first half: a cell that leaves the layer computes its share
// (run by k_conv_share_keep); an old-list cell is tagged tag | 3 (its own
// thread writes it; the neighbours' receiver test reads flags or the tag,
// both of which mark it as a layer cell).
template <class P>
__device__ inline void conv_share_cell(const Fields<P> &F, int i, uint32_t tag, bool old_list)
{
    using R = typename P::R;
    const uint8_t st = F.conv[i];
    if (st == CV_NONE) return;
    if (old_list) F.mark[i] = tag | 3u;
    const R mex = cv_to_liquid(st) ? F.m[i] - F.rho[i] : F.m[i];
    const Nbr nb(i, F.nx, F.ny, F.nz);
    int cnt = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q) cnt += is_receiver(F, nb.at(dir_x(q), dir_y(q), dir_z(q)), tag);
    if (cnt > 0) {
        F.share[i] = mex / R(cnt);
    } else {
        F.share[i] = R(0);
        reservoir_add(F.sc, (double)mex);
    }
}

template <class P>
__device__ inline typename P::R gathered_excess(const Fields<P> &F, int j, uint32_t tag)
{
    using R = typename P::R;
    const Nbr nb(j, F.nx, F.ny, F.nz);
    R acc = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
        const int w = nb.at(dir_x(q), dir_y(q), dir_z(q));
        if (is_converter(F, w, tag)) acc += F.share[w];
    }
    return acc;
}

// Rule 5, second half, and rule 6: receivers gather their neighbours'
// shares in fixed direction order, and the cells that leave the layer and
// the new cells take their types. This kernel also sets phi = m / rho of
// every interface cell for the new time level, so it runs in every step.
// Every new cell is next to a filling or emptying cell of the old list,
// whose thread sets it (several threads may write the same values).
template <class P>
__global__ __launch_bounds__(256) void k_conv_gather(const Batch<P> B)
{
    const Fields<P> &F = B.f[blockIdx.y];
    const bool frozen = B.p[blockIdx.y].frozen != 0;
    using R = typename P::R;
    const bool any = F.sc->nconv != 0;
    const uint32_t tag = F.sc->step << 2;
    const uint8_t s8 = uint8_t(tag >> 2);
    const int n = list_count(F.sc);
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        const uint8_t st = any ? F.conv[i] : CV_NONE;
        if (st == CV_NONE) {
            // only a cell near a filling or emptying cell can receive
            const R acc = any && F.near[i] == s8 ? gathered_excess(F, i, tag) : R(0);
            const R mn = F.m[i] + acc;
            const R ph = mn / F.rho[i];
            F.m[i] = mn;
            F.phi[i] = ph;
            // a frozen window stays on one smooth piece of the step only while
            // every interface fill lies strictly inside (0, 1)
            if (frozen && !(ph > R(0) && ph < R(1))) {
                atomicAdd(&F.sc->fill_out, 1);
                atomicMin(&F.sc->fill_out_step, F.sc->step);
            }
            continue;
        }
        F.phi[i] = cv_to_liquid(st) ? R(1) : R(0);
        F.flags[i] = (F.flags[i] & FL_NEAR_OBST) | (cv_to_liquid(st) ? FL_LIQ : FL_GAS);
        // a new neighbour of a closing cell is also next to the filling or
        // emptying cell that made it, whose thread sets it
        if (st == CV_CLOSE_LIQ || st == CV_CLOSE_GAS) continue;
        const Nbr nb(i, F.nx, F.ny, F.nz);
        for (int q = 1; q < NQ; ++q) {
            const int j = nb.at(dir_x(q), dir_y(q), dir_z(q));
            const uint32_t mk = F.mark[j];
            if (!is_new(mk, tag)) continue;
            const uint8_t sj = F.conv[j];
            const uint8_t tj = sj == CV_NONE ? FL_IF : (cv_to_liquid(sj) ? FL_LIQ : FL_GAS);
            F.flags[j] = (F.flags[j] & FL_NEAR_OBST) | tj;
            if (sj != CV_NONE) {
                F.phi[j] = cv_to_liquid(sj) ? R(1) : R(0);
                continue;
            }
            const R base = (mk & 3u) == 1u ? R(0) : F.rho[j];
            const R mn = base + gathered_excess(F, j, tag);
            F.m[j] = mn;
            F.phi[j] = mn / F.rho[j];
        }
    }
}

// ------------------------------------------------ interface-list update
// After a step with conversions the list becomes the cells of the step's
// layer (old list, then new cells) that are interface cells. The order of
// the list does not enter any result (every per-cell computation is
// independent), so kept cells are appended with an atomic counter; the
// interface bounding box is recomputed on the way.
__device__ inline int block_exclusive_scan(int v, int *lds_wave, int &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds_wave[wave] = x;
    __syncthreads();
    int off = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) off += lds_wave[w];
        tot += lds_wave[w];
    }
    total = tot;
    __syncthreads();
    return off + x - v;
}

// Block-wide min / max of a box contribution; thread 0 issues the atomics.
__device__ inline void block_box_update(int (&lo)[3], int (&hi)[3], int *box)
{
    __shared__ int red[6][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = min(lo[c], __shfl_xor(lo[c], d, 64));
            hi[c] = max(hi[c], __shfl_xor(hi[c], d, 64));
        }
    if (lane == 0)
        for (int c = 0; c < 3; ++c) {
            red[c][wave] = lo[c];
            red[3 + c][wave] = hi[c];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w)
            for (int c = 0; c < 3; ++c) {
                red[c][0] = min(red[c][0], red[c][w]);
                red[3 + c][0] = max(red[3 + c][0], red[3 + c][w]);
            }
        if (red[3][0] >= 0)
            for (int c = 0; c < 3; ++c) {
                atomicMin(&box[c], red[c][0]);
                atomicMax(&box[3 + c], red[3 + c][0]);
            }
    }
    __syncthreads();
}

template <class P>
__device__ inline void box_add(const Fields<P> &F, int i, int (&lo)[3], int (&hi)[3])
{
    const int yz = i / F.nx, z = yz / F.ny, y = yz - z * F.ny, x = i - yz * F.nx;
    lo[0] = min(lo[0], x); lo[1] = min(lo[1], y); lo[2] = min(lo[2], z);
    hi[0] = max(hi[0], x); hi[1] = max(hi[1], y); hi[2] = max(hi[2], z);
}

// Shares of the cells that leave the layer (rule 5, first half), and the
// cells of the step's layer that stay interface cells (status CV_NONE after
// rule 4, old or new), written in layer order within each block: a counting
// pass, one atomic for the block's base, then the ordered write with a
// block prefix sum. Each block takes one contiguous range of the layer.
template <class P>
__global__ __launch_bounds__(256) void k_conv_share_keep(const Batch<P> B)
{
    const Fields<P> &F = B.f[blockIdx.y];
    if (F.sc->nconv == 0) return;
    const uint32_t tag = F.sc->step << 2;
    const int n = list_count(F.sc), nl = n + F.sc->nnew;
    int k0, k1;
    block_share(nl, k0, k1);
    for (int k = k0 + threadIdx.x; k < k1; k += 256) conv_share_cell(F, layer_cell(F, k, n), tag, k < n);
    __shared__ int lw[4];
    __shared__ int base_s;
    int cnt = 0;
    for (int k = k0 + threadIdx.x; k < k1; k += 256) cnt += F.conv[layer_cell(F, k, n)] == CV_NONE;
    int total;
    block_exclusive_scan(cnt, lw, total);
    if (threadIdx.x == 0) base_s = total > 0 ? atomicAdd(&F.sc->nkeep, total) : 0;
    __syncthreads();
    int pos = base_s;
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int kk = k0; kk < k1; kk += 256) {
        const int k = kk + threadIdx.x;
        const int i = k < k1 ? layer_cell(F, k, n) : 0;
        const bool keep = k < k1 && F.conv[i] == CV_NONE;
        int tot;
        const int ex = block_exclusive_scan(keep ? 1 : 0, lw, tot);
        if (keep) {
            F.ilist_tmp[pos + ex] = i;
            box_add(F, i, lo, hi);
        }
        pos += tot;
    }
    block_box_update(lo, hi, F.sc->bbox);
}

// New list = the kept cells. The fluid box grows by every new cell (a new
// cell from gas is fluid whether it stays in the layer or closes to
// liquid); the interface box came from k_conv_share_keep.
template <class P>
__global__ __launch_bounds__(256) void k_list_finish(const Batch<P> B)
{
    const Fields<P> &F = B.f[blockIdx.y];
    if (F.sc->nconv == 0) return;
    const int nk = F.sc->nkeep, nn = F.sc->nnew;
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int k = blockIdx.x * 256 + threadIdx.x; k < nk + nn; k += gridDim.x * 256) {
        if (k < nk) F.ilist[k] = F.ilist_tmp[k];
        else box_add(F, F.newlist[k - nk], lo, hi);
    }
    block_box_update(lo, hi, F.sc->fbox);
    if (blockIdx.x == 0 && threadIdx.x == 0) F.sc->icount = nk;
}

// ----------------------------------------------------------- compaction
// Ascending list of the cells whose flags match `want`: each block covers
// 1024 consecutive cells (4 per thread); per-block counts, one scan block,
// then the write pass with a wavefront-ballot / shuffle prefix sum.
constexpr int CMP_CELLS = 1024;


// Cells k = base .. base+3 of a range (x fastest): hit[s] and their indices.
__device__ inline int cells_matching(const uint8_t *flags, const CellRange &r, int nx, int ny, int base,
                                     uint8_t want, bool (&hit)[4], int (&idx)[4])
{
    const int n = r.size();
    int c = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = base + s;
        idx[s] = k < n ? r.cell(k, nx, ny) : 0;
        hit[s] = k < n && (flags[idx[s]] & want);
        c += hit[s];
    }
    return c;
}

// which = 0: interface cells (flags & FL_IF) into ilist / icount (at
// creation); which = 1: the static list of obstacle cells next to
// non-obstacle cells (conv bit 0) into olist / ocount; which = 2: the static
// list of non-obstacle cells next to obstacle cells (conv bit 1) into
// wlist / wcount.
template <class P>
__device__ inline void compact_source(const Fields<P> &F, int which, const uint8_t *&src, uint8_t &want,
                                      int32_t *&list, int *&count, CellRange &range)
{
    range = which == 0 ? CellRange::from(F.sc->fbox) : CellRange::whole(F.nx, F.ny, F.nz);
    src = which == 0 ? F.flags : F.conv;
    want = which == 0 ? FL_IF : (which == 1 ? 1 : 2);
    list = which == 0 ? F.ilist : (which == 1 ? F.olist : F.wlist);
    count = which == 0 ? &F.sc->icount : (which == 1 ? &F.sc->ocount : &F.sc->wcount);
}

// A fixed grid of CMP_GRID blocks per lattice; block b owns a contiguous run
// of 1024-cell tiles, so the list stays in ascending order.
constexpr int CMP_GRID = 256;

__device__ inline void tile_range(int N, int &t0, int &t1)
{
    const int ntiles = (N + CMP_CELLS - 1) / CMP_CELLS;  // N: cells of the range
    const int per = (ntiles + gridDim.x - 1) / gridDim.x;
    t0 = min(ntiles, (int)blockIdx.x * per);
    t1 = min(ntiles, t0 + per);
}

template <class P>
__global__ __launch_bounds__(256) void k_compact_count(const Batch<P> B, int which, int force)
{
    const Fields<P> &F = B.f[blockIdx.y];
    if (!force && F.sc->nconv == 0) return;
    const uint8_t *src; uint8_t want; int32_t *list; int *count; CellRange range;
    compact_source(F, which, src, want, list, count, range);
    __shared__ int lw[4];
    int t0, t1;
    tile_range(range.size(), t0, t1);
    int sum = 0;
    for (int t = t0; t < t1; ++t) {
        bool hit[4];
        int idx[4];
        const int c = cells_matching(src, range, F.nx, F.ny, t * CMP_CELLS + threadIdx.x * 4, want, hit, idx);
        int total;
        block_exclusive_scan(c, lw, total);
        sum += total;
    }
    if (threadIdx.x == 0) F.counts[blockIdx.x] = sum;
}

// One block per lattice: exclusive scan of the block counts, list length;
// the interface bounding box is reset for the write pass.
template <class P>
__global__ __launch_bounds__(1024) void k_compact_scan(const Batch<P> B, int which, int force, int nblocks)
{
    const Fields<P> &F = B.f[blockIdx.y];
    if (!force && F.sc->nconv == 0) return;
    const uint8_t *src; uint8_t want; int32_t *list; int *count; CellRange range;
    compact_source(F, which, src, want, list, count, range);
    __shared__ int lw[16];
    int carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const int v = b < nblocks ? F.counts[b] : 0;
        int total;
        const int ex = block_exclusive_scan(v, lw, total);
        if (b < nblocks) F.counts[b] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *count = carry;
        if (which == 0) {
            F.sc->bbox[0] = F.nx; F.sc->bbox[1] = F.ny; F.sc->bbox[2] = F.nz;
            F.sc->bbox[3] = -1; F.sc->bbox[4] = -1; F.sc->bbox[5] = -1;
        }
    }
}

template <class P>
__global__ __launch_bounds__(256) void k_compact_write(const Batch<P> B, int which, int force)
{
    const Fields<P> &F = B.f[blockIdx.y];
    if (!force && F.sc->nconv == 0) return;
    const uint8_t *src; uint8_t want; int32_t *list; int *count; CellRange range;
    compact_source(F, which, src, want, list, count, range);
    __shared__ int lw[4];
    int t0, t1;
    tile_range(range.size(), t0, t1);
    int base = F.counts[blockIdx.x];
    int lo[3] = {F.nx, F.ny, F.nz}, hi[3] = {-1, -1, -1};
    for (int t = t0; t < t1; ++t) {
        bool hit[4];
        int idx[4];
        const int c = cells_matching(src, range, F.nx, F.ny, t * CMP_CELLS + threadIdx.x * 4, want, hit, idx);
        int total;
        int pos = base + block_exclusive_scan(c, lw, total);
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (hit[s]) {
                const int i = idx[s];
                list[pos++] = i;
                const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
                lo[0] = min(lo[0], x); lo[1] = min(lo[1], y); lo[2] = min(lo[2], z);
                hi[0] = max(hi[0], x); hi[1] = max(hi[1], y); hi[2] = max(hi[2], z);
            }
        base += total;
    }
    if (which == 0 && hi[0] >= 0) {
        for (int k = 0; k < 3; ++k) {
            atomicMin(&F.sc->bbox[k], lo[k]);
            atomicMax(&F.sc->bbox[3 + k], hi[k]);
        }
    }
}

// Static wall lists: bit 0 marks obstacle cells with a non-obstacle D3Q19
// neighbour, bit 1 non-obstacle cells with an obstacle D3Q19 neighbour.
__global__ __launch_bounds__(256) void k_mark_wall_cells(const uint8_t *flags, uint8_t *out, int nx, int ny,
                                                         int nz, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const bool obst = flags[i] & FL_OBST;
    const Nbr nb(i, nx, ny, nz);
    bool other = false;
#pragma unroll
    for (int q = 1; q < NQ; ++q) other |= ((flags[nb.at(dir_x(q), dir_y(q), dir_z(q))] & FL_OBST) != 0) != obst;
    out[i] = other ? (obst ? 1 : 2) : 0;
}

// ------------------------------------------------ obstacle fill (Sec. II.A)
// phi(x_o) = sum |nw.c^_q| phi(x_o + c_q) / sum |nw.c^_q| over fluid
// neighbours with aperture |nw.c^_q| > sqrt(2)/2 (strict; the 45-degree
// links are excluded), nw the normalised sum of the directions from x_o to
// its non-obstacle neighbours.
template <class P>
__global__ __launch_bounds__(256) void k_obstacle_fill(const Batch<P> B)
{
    const Fields<P> &F = B.f[blockIdx.y];
    using R = typename P::R;
    const int n = F.sc->ocount;
    const double alpha = 0.70710678118654752440 + 1e-12;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.olist[k];
        const Nbr nb(i, F.nx, F.ny, F.nz);
        int sx = 0, sy = 0, sz = 0;
#pragma unroll
        for (int q = 1; q < NQ; ++q)
            if (!(F.flags[nb.at(dir_x(q), dir_y(q), dir_z(q))] & FL_OBST)) {
                sx += dir_x(q); sy += dir_y(q); sz += dir_z(q);
            }
        const double len = sqrt(double(sx * sx + sy * sy + sz * sz));
        double num = 0, den = 0;
        if (len > 0) {
            const double wx = sx / len, wy = sy / len, wz = sz / len;
#pragma unroll
            for (int q = 1; q < NQ; ++q) {
                const int j = nb.at(dir_x(q), dir_y(q), dir_z(q));
                if (!(F.flags[j] & FL_FLUID)) continue;
                const double cl = sqrt(double(dir_len2(q)));
                const double w = fabs((wx * dir_x(q) + wy * dir_y(q) + wz * dir_z(q)) / cl);
                if (w > alpha) {
                    num += w * double(F.phi[j]);
                    den += w;
                }
            }
        }
        F.phi[i] = R(den > 0 ? num / den : 0.0);
        if (F.snap) F.snap[(size_t)SNAP * F.sc->icount + k] = R(den > 0 ? num / den : 0.0);
    }
}

// ------------------------------------------------ bubble model (Sec. III.A.1)
// The whole gas of a lattice is one bubble with isothermal pressure,
// p_g(t) V(t) = p_g(0) V(0), so rho_gas(t) = rho_gas V0 / V(t) with the gas
// volume V = (non-obstacle cells) - (liquid cells + sum of phi over
// interface cells). The liquid volume is summed over the fluid box in a
// fixed partition (VOL_BLOCKS blocks, fixed order within each), after the
// step's conversions.
constexpr int VOL_BLOCKS = 1024;

template <class P>
__global__ __launch_bounds__(256) void k_bubble_partial(const Batch<P> B)
{
    const Params &prm = B.p[blockIdx.y];
    if (!prm.bubble) return;
    const Fields<P> &F = B.f[blockIdx.y];
    __shared__ double s[256];
    const CellRange box = CellRange::from(F.sc->fbox);
    const int n = box.size();
    const int chunk = (n + gridDim.x - 1) / gridDim.x;
    const int b0 = min(n, (int)blockIdx.x * chunk), b1 = min(n, b0 + chunk);
    double acc = 0.0;
    for (int k = b0 + threadIdx.x; k < b1; k += 256) {
        const int i = box.cell(k, F.nx, F.ny);
        const uint8_t fl = F.flags[i];
        if (fl & FL_LIQ) acc += 1.0;
        else if (fl & FL_IF) acc += double(F.phi[i]);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) F.part[blockIdx.x] = s[0];
}

template <class P>
__global__ __launch_bounds__(1024) void k_bubble_final(const Batch<P> B, int nblocks)
{
    const Params &prm = B.p[blockIdx.y];
    if (!prm.bubble) return;
    const Fields<P> &F = B.f[blockIdx.y];
    __shared__ double s[1024];
    s[threadIdx.x] = (int)threadIdx.x < nblocks ? F.part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = prm.n_free - s[0];
        if (F.sc->bubble_init) {
            F.sc->gas_v0 = v;
            F.sc->bubble_init = 0;
        }
        F.sc->rho_gas_t = v > 0.0 ? prm.rho_gas * F.sc->gas_v0 / v : prm.rho_gas;
    }
}

}  // namespace fslbm
