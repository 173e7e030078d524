// Host driver and C ABI of libfslbm (declared in include/fslbm.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <mutex>
#include <vector>

#include "fslbm.h"
#include "fslbm_adjoint.hpp"
#include "fslbm_convert.hpp"
#include "fslbm_device.hpp"
#include "fslbm_geometry.hpp"
#include "fslbm_pullcopy.hpp"
#include "fslbm_stream.hpp"

using namespace fslbm;

// ------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(FSLBM_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------ layout
namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t fbytes(int prec)
{
    switch (prec) {
    case P_F64: return 8;
    case P_F32: return 4;
    default: return 2;
    }
}
size_t rbytes(int prec) { return prec == P_F64 ? 8 : 4; }

struct Layout {
    size_t fA, fB, flags, conv, near, mark, m, rho, phi, K, nrm, plic, share, phis, nmol, cnrm, ilist, olist, wlist, newlist,
        ilist_tmp,
        staging,
        counts, part, sc, total;
};

constexpr int MASS_BLOCKS = 1024;
constexpr int DIAG_VALUES = 5;  // partial sums per block of the diagnostics

// Plane stride of the distribution buffers (elements): N rounded up to 64
// elements, so that every plane starts on a 128-byte boundary, plus 1024
// elements, so that the 19 planes' streams do not start a power of two
// apart in HBM. Measured on the 512^3 probe: the FP32 stream-collide takes
// 3514 us with the 1024-element gap and 3562 without (F16 1877 and 1891; a
// 4096-element gap slowed F16 to 1976).
long long plane_stride(long long N) { return (N + 63) / 64 * 64 + 1024; }

Layout make_layout(int nx, int ny, int nz, int prec)
{
    const long long N = (long long)nx * ny * nz;
    const long long NS = plane_stride(N);
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t fb = fbytes(prec), rb = rbytes(prec);
    L.fA = take(19 * NS * fb);
    L.fB = take(19 * NS * fb);
    L.flags = take(N);
    L.near = take(N);
    L.conv = take(N);
    L.mark = take(4 * N);
    L.m = take(N * rb);
    L.rho = take(N * rb);
    L.phi = take(N * rb);
    L.K = take(N * rb);
    L.nrm = take(3 * N * rb);
    L.plic = take(N * rb);
    L.share = take(N * rb);
    L.phis = take(N * rb);
    L.nmol = take(3 * N * rb);
    L.cnrm = take(3 * N * rb);
    L.ilist = take(4 * N);
    L.olist = take(4 * N);
    L.wlist = take(4 * N);
    L.newlist = take(4 * N);
    L.ilist_tmp = take(4 * N);
    L.staging = take(8 * N + 512);  // N doubles for read-outs; the ordered interface list (count + N ints)
    L.counts = take(4 * (size_t)CMP_GRID);  // one count per compaction block (fixed grid)
    L.part = take(8 * (DIAG_VALUES * MASS_BLOCKS + 8));  // mass, bubble volume and diagnostics partials
    L.sc = take(sizeof(DevScalars));
    L.total = off;
    return L;
}

bool shape_ok(int nx, int ny, int nz)
{
    if (nx < 3 || ny < 3 || nz < 3) return false;
    const long long N = (long long)nx * ny * nz;
    return plane_stride(N) <= 2147483647LL;  // cell indices and the plane stride are 32-bit
}

}  // namespace

// What the closure of the interface layer at creation did to the input fill.
struct LayerClosure {
    long long against = 0;  // cells rounded to the phase that fills less than half of them
    long long to_liquid = 0, to_gas = 0;
    double fill_added = 0.0, fill_removed = 0.0;
};

struct fslbm_lattice;

// A recorded frozen-topology window: checkpoints of the state every K steps
// (and at the end) in a caller-owned device workspace, plus the adjoint
// fields and a ring of K-1 states recomputed per segment in the reverse
// sweep.
struct AdjWindow {
    int recorded = 0;
    long long T = 0;
    int K = 0;
    long long fill_events = 0;     // (step, interface cell) events with a fill outside (0, 1)
    long long inside_steps = 0;    // steps before the first such event (T if none)
    long long unconverted_steps = 0;  // steps before a cell would first fill or empty (T if none)
    int icount = 0, ocount = 0;
    long long t_end = 0;     // steps taken at the end of the window
    unsigned start_step = 0;  // the device step number of the window's first step
    unsigned long long epoch = 0;  // state epoch at the end of the window
    char *ws = nullptr;
    size_t bytes = 0;
    std::vector<long long> ck;  // checkpoint times 0, K, 2K, ..., T
    size_t f_bytes = 0, snap_bytes = 0, slot_bytes = 0;
    size_t off_ck = 0, off_ring[2] = {0, 0}, off_shadow = 0;
    size_t off_gin[2] = {0, 0}, off_own[2] = {0, 0}, off_refl = 0, off_scal = 0, off_gb = 0, off_contrib = 0, off_pos = 0,
           off_part = 0, total = 0;
};

// A set of lattices advanced together: each kernel of the step is launched
// once for all of them (blockIdx.y selects the lattice). Every handle also
// owns an implicit batch holding only itself.
struct fslbm_batch {
    std::vector<fslbm_lattice *> hs;
    std::vector<unsigned> versions;  // handle versions the graphs were captured at
    int prec;
    // optional phase timing: events around stream-collide, conversion,
    // compaction and obstacle fill + curvature of every step
    int timing;
    std::vector<hipEvent_t> ev;
    int ev_used;  // steps recorded in ev since the last fold
    double tacc[5];
    long long tsteps;
    // optional replay of one step as a HIP graph (one per buffer parity)
    int use_graph;
    hipGraphExec_t gexec[2];
    // interface and wall cells: 0 = in the bulk stream-collide kernel, 1 =
    // own list kernel, -1 = chosen per step (split_now)
    int split_interface;
    int split_last;  // 1 if the last step ran the split passes
};

struct fslbm_lattice {
    int nx, ny, nz;
    int N;
    int NS;  // plane stride of the distribution buffers
    int box_blocks;  // SC_BLOCK-cell chunks of the fluid box when last read back (grid of the bulk stream-collide)
    long long box_cells, boundary_cells;  // fluid-box cells, interface + wall-list cells (last read back)
    int device;      // device that holds the workspace
    int strong_wetting;  // 1: contact angles below 45 deg are accepted (FSLBM_OPT_STRONG_WETTING)
    LayerClosure closure;  // what the closure of the interface layer did to the input fill
    int prec, curv, coll;
    double sigma, tau, theta, rho_gas, eps_c, trt_magic;
    hipStream_t stream;
    char *ws;
    Layout L;
    int cur;  // 0: current f' in fA, 1: in fB
    long long steps;
    unsigned version;  // bumped whenever launch arguments change
    unsigned long long epoch;  // bumped whenever the state changes other than by stepping
    int frozen;        // 1 inside a frozen-topology window
    int icount0;       // interface cells at creation (sizes the list-kernel grids)
    int ocount0;       // obstacle cells next to the fluid (sizes the reflection grid)
    int bubble;        // bubble model on (FSLBM_OPT_BUBBLE)
    double n_free;     // non-obstacle cells
    fslbm_batch self;
    AdjWindow adj;
    // while the reverse sweep enqueues a segment's recompute: the copy of the
    // non-distribution fields (from Layout::flags on) that those steps work
    // on, so that they can run beside the reverse steps (make_fields)
    char *scal_base = nullptr;
};

namespace {
constexpr int TIMING_CAP = 512;  // steps held in the event pool before folding
constexpr int TIMING_EV = 6;     // events per step
constexpr int NPHASE = TIMING_EV - 1;
}

namespace {

Params make_params(const fslbm_lattice *h)
{
    Params p;
    p.sigma = h->sigma;
    p.tau = h->tau;
    p.omega = 1.0 / h->tau;
    p.omega_odd = 1.0 / (0.5 + h->trt_magic / (h->tau - 0.5));
    p.cos_theta = cos(h->theta);
    p.sin_theta = sin(h->theta);
    p.rho_gas = h->rho_gas;
    p.eps_c = h->eps_c;
    p.curv = h->curv;
    p.coll = h->coll;
    p.frozen = h->frozen;
    p.bubble = h->bubble;
    p.n_free = h->n_free;
    return p;
}

template <class P>
Fields<P> make_fields(const fslbm_lattice *h)
{
    using S = typename P::S;
    using R = typename P::R;
    Fields<P> F;
    char *w = h->ws;
    const Layout &L = h->L;
    // every field after the two distribution buffers: in the workspace, or
    // in the copy h->scal_base holds
    auto at = [&](size_t off) { return h->scal_base ? h->scal_base + (off - L.flags) : w + off; };
    F.fsrc = (const S *)(w + (h->cur == 0 ? L.fA : L.fB));
    F.fdst = (S *)(w + (h->cur == 0 ? L.fB : L.fA));
    F.flags = (uint8_t *)at(L.flags);
    F.conv = (uint8_t *)at(L.conv);
    F.near = (uint8_t *)at(L.near);
    F.mark = (uint32_t *)at(L.mark);
    F.m = (R *)at(L.m);
    F.rho = (R *)at(L.rho);
    F.phi = (R *)at(L.phi);
    F.K = (R *)at(L.K);
    F.nrm = (R *)at(L.nrm);
    F.plic = (R *)at(L.plic);
    F.share = (R *)at(L.share);
    F.phis = (R *)at(L.phis);
    F.nmol = (R *)at(L.nmol);
    F.cnrm = (R *)at(L.cnrm);
    F.ilist = (int32_t *)at(L.ilist);
    F.olist = (int32_t *)at(L.olist);
    F.wlist = (int32_t *)at(L.wlist);
    F.newlist = (int32_t *)at(L.newlist);
    F.ilist_tmp = (int32_t *)at(L.ilist_tmp);
    F.counts = (int *)at(L.counts);
    F.part = (double *)at(L.part);
    F.sc = (DevScalars *)at(L.sc);
    F.snap = nullptr;
    F.nx = h->nx;
    F.ny = h->ny;
    F.nz = h->nz;
    F.N = h->N;
    F.NS = h->NS;
    return F;
}

inline int cell_blocks(int N) { return (N + 255) / 256; }
inline int list_blocks(int N) { return std::min(LIST_GRID, std::max(1, (N + 255) / 256)); }
inline int cmp_blocks(int N) { return std::min(CMP_GRID, (N + CMP_CELLS - 1) / CMP_CELLS); }
constexpr int GEOM_GRID = 1024;  // blocks per lattice of the tiled geometry kernels
constexpr int SC_LIST_GRID = 1024;  // blocks per lattice of the interface / wall-list stream-collide

// ------------------------------------------------------ init kernels
__global__ void k_fill_bytes(uint8_t *p, size_t n, uint8_t v)
{
    for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = v;
}

__global__ void k_init_scalars(DevScalars *sc)
{
    sc->icount = 0;
    sc->ocount = 0;
    sc->nconv = 0;
    sc->nnew = 0;
    sc->nkeep = 0;
    sc->step = 1;
    sc->res_hi = 0;
    sc->res_lo = 0;
    sc->mass = 0.0;
    sc->bad = 0;
    sc->wcount = 0;
    sc->gas_v0 = 0.0;
    sc->rho_gas_t = 0.0;
    sc->bubble_init = 0;
    sc->fill_out = 0;
    sc->fill_out_step = 0xffffffffu;
    sc->conv_out_step = 0xffffffffu;
    for (int k = 0; k < 6; ++k) sc->bbox[k] = 0;
    sc->fbox[0] = sc->fbox[1] = sc->fbox[2] = 1 << 30;
    sc->fbox[3] = sc->fbox[4] = sc->fbox[5] = -1;
}

// Types from fill level and obstacle mask (obstacle input in `types` on entry).
__global__ void k_init_types(const double *fill, uint8_t *types, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double f = fill[i];
    types[i] = types[i] ? FL_OBST : (f >= 1.0 ? FL_LIQ : (f <= 0.0 ? FL_GAS : FL_IF));
}

// Initial interface layer, one pass per stage over all cells (in -> out):
// STAGE 0: a liquid cell with a gas D3Q19 neighbour becomes an interface
// cell (phi = 1); STAGE 1: an interface cell without a gas neighbour
// becomes liquid; STAGE 2: an interface cell without a liquid neighbour
// becomes gas. Stages 1-2 close the layer (Sec. II.D: an interface cell has
// both gas and liquid neighbours).
template <int STAGE>
__global__ void k_init_layer(const uint8_t *in, uint8_t *out, int nx, int ny, int nz, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    uint8_t t = in[i];
    const uint8_t from = STAGE == 0 ? FL_LIQ : FL_IF;
    if (t == from) {
        const uint8_t want = STAGE == 2 ? FL_LIQ : FL_GAS;
        const Nbr nb(i, nx, ny, nz);
        bool found = false;
#pragma unroll
        for (int q = 1; q < NQ; ++q) found |= in[nb.at(dir_x(q), dir_y(q), dir_z(q))] == want;
        if (STAGE == 0 && found) t = FL_IF;
        if (STAGE == 1 && !found) t = FL_LIQ;
        if (STAGE == 2 && !found) t = FL_GAS;
    }
    out[i] = t;
}

// Final flags and fields from the closed layer's types: f' = feq(1, 0);
// interface cells m = phi (at most 1), rho = 1.
template <class P>
__global__ void k_init_fields(Fields<P> F, const double *fill, const uint8_t *types, uint8_t *out_flags)
{
    using R = typename P::R;
    using T = typename P::T;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    const Nbr nb(i, F.nx, F.ny, F.nz);
    const uint8_t t = types[i];
    bool obst_nb = false;
#pragma unroll
    for (int q = 1; q < NQ; ++q) obst_nb |= types[nb.at(dir_x(q), dir_y(q), dir_z(q))] == FL_OBST;
    out_flags[i] = t | (obst_nb ? FL_NEAR_OBST : 0);
    R phi = 0, m = 0, rho = 0;
    if (t == FL_LIQ) phi = 1;
    if (t == FL_IF) {
        phi = R(fill[i] < 1.0 ? fill[i] : 1.0);
        m = phi;
        rho = 1;
    }
    F.phi[i] = phi;
    F.m[i] = m;
    F.rho[i] = rho;
    F.K[i] = 0;
    F.plic[i] = 0;
    F.share[i] = 0;
    F.phis[i] = 0;
    const size_t N = F.N;
    for (int c = 0; c < 3; ++c) {
        F.nrm[c * N + i] = 0;
        F.nmol[c * N + i] = 0;
        F.cnrm[c * N + i] = 0;
    }
    F.mark[i] = 0;
    F.near[i] = 0;
    typename P::S *dst = F.fdst;
    typename P::S *src = const_cast<typename P::S *>(F.fsrc);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const T v = t == FL_OBST ? T(0) : weight<T>(q);
        switch (q) {
#define FSLBM_ST(QQ)                                 \
    case QQ:                                         \
        store_f<P, QQ>(plane<P, QQ>(src, F.NS), i, v); \
        store_f<P, QQ>(plane<P, QQ>(dst, F.NS), i, v); \
        break;
            FSLBM_ST(0) FSLBM_ST(1) FSLBM_ST(2) FSLBM_ST(3) FSLBM_ST(4) FSLBM_ST(5) FSLBM_ST(6)
            FSLBM_ST(7) FSLBM_ST(8) FSLBM_ST(9) FSLBM_ST(10) FSLBM_ST(11) FSLBM_ST(12) FSLBM_ST(13)
            FSLBM_ST(14) FSLBM_ST(15) FSLBM_ST(16) FSLBM_ST(17) FSLBM_ST(18)
#undef FSLBM_ST
        }
    }
}

// Bounding box of the fluid cells (block min / max, then atomics).
__global__ __launch_bounds__(256) void k_fluid_box(const uint8_t *flags, int nx, int ny, int N, DevScalars *sc)
{
    __shared__ int red[6][256];
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) {
        if (!(flags[i] & FL_FLUID)) continue;
        const int yz = i / nx, x = i - yz * nx, z = yz / ny, y = yz - z * ny;
        lo[0] = min(lo[0], x); lo[1] = min(lo[1], y); lo[2] = min(lo[2], z);
        hi[0] = max(hi[0], x); hi[1] = max(hi[1], y); hi[2] = max(hi[2], z);
    }
    for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = lo[k];
        red[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 3; ++k) {
                red[k][threadIdx.x] = min(red[k][threadIdx.x], red[k][threadIdx.x + w]);
                red[3 + k][threadIdx.x] = max(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[3][0] >= 0)
        for (int k = 0; k < 3; ++k) {
            atomicMin(&sc->fbox[k], red[k][0]);
            atomicMax(&sc->fbox[3 + k], red[3 + k][0]);
        }
}

__global__ void k_copy_bytes(const uint8_t *src, uint8_t *dst, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) dst[i] = src[i];
}

// f' = feq(rho, u) at fluid cells; u read from three planes of doubles.
template <class P>
__global__ void k_set_equilibrium(Fields<P> F, const double *rho_in, const double *u_in)
{
    using T = typename P::T;
    using R = typename P::R;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    const uint8_t fl = F.flags[i];
    if (!(fl & FL_FLUID)) return;
    const size_t N = F.N;
    const T r = T(rho_in[i]), ux = T(u_in[i]), uy = T(u_in[N + i]), uz = T(u_in[2 * N + i]);
    const T usq = ux * ux + uy * uy + uz * uz;
    typename P::S *dst = const_cast<typename P::S *>(F.fsrc);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const T v = feq<T>(q, r, ux, uy, uz, usq);
        switch (q) {
#define FSLBM_ST(QQ) case QQ: store_f<P, QQ>(plane<P, QQ>(dst, F.NS), i, v); break;
            FSLBM_ST(0) FSLBM_ST(1) FSLBM_ST(2) FSLBM_ST(3) FSLBM_ST(4) FSLBM_ST(5) FSLBM_ST(6)
            FSLBM_ST(7) FSLBM_ST(8) FSLBM_ST(9) FSLBM_ST(10) FSLBM_ST(11) FSLBM_ST(12) FSLBM_ST(13)
            FSLBM_ST(14) FSLBM_ST(15) FSLBM_ST(16) FSLBM_ST(17) FSLBM_ST(18)
#undef FSLBM_ST
        }
    }
    if (fl & FL_IF) {
        F.rho[i] = R(r);
        F.m[i] = F.phi[i] * R(r);
    }
}

// ----------------------------------------------------------- read-outs
template <class P>
__device__ inline void load_all(const Fields<P> &F, int i, typename P::T (&f)[NQ])
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        switch (q) {
#define FSLBM_LD(QQ) case QQ: f[q] = load_f<P, QQ>(plane<P, QQ>(F.fsrc, F.NS), i); break;
            FSLBM_LD(0) FSLBM_LD(1) FSLBM_LD(2) FSLBM_LD(3) FSLBM_LD(4) FSLBM_LD(5) FSLBM_LD(6)
            FSLBM_LD(7) FSLBM_LD(8) FSLBM_LD(9) FSLBM_LD(10) FSLBM_LD(11) FSLBM_LD(12) FSLBM_LD(13)
            FSLBM_LD(14) FSLBM_LD(15) FSLBM_LD(16) FSLBM_LD(17) FSLBM_LD(18)
#undef FSLBM_LD
        }
    }
}

// Density (FP64) and velocity of a fluid cell from its stored
// distributions: for the shifted forms rho = 1 + sum d with the deviations
// summed in FP64 (a sum of the f_q in FP32 would round at 1e-7 of rho).
template <class P>
__device__ inline void cell_moments(const Fields<P> &F, int i, double &rho, typename P::T &ux, typename P::T &uy,
                                    typename P::T &uz)
{
    using T = typename P::T;
    T f[NQ];
    if constexpr (P::SHIFT) {
        int own[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) own[q] = i;
        load_dirs_dev<P>(F, own, f);
        T dr;
        moments_dev(f, dr, ux, uy, uz);
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) s += double(f[q]);
        rho = 1.0 + s;
    } else {
        load_all(F, i, f);
        T r;
        moments(f, r, ux, uy, uz);
        rho = double(r);
    }
}

enum ReadWhat { RD_FILL, RD_PRESSURE, RD_CURV, RD_VEL, RD_NORMAL, RD_PLIC, RD_MASS };

template <class P>
__global__ void k_read(Fields<P> F, double rho_gas, int bubble, int what, int comp, double *out)
{
    using T = typename P::T;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    const uint8_t fl = F.flags[i];
    const bool fluid = fl & FL_FLUID, ifc = fl & FL_IF;
    const size_t N = F.N;
    double v = 0.0;
    switch (what) {
    case RD_FILL: v = double(F.phi[i]); break;
    case RD_CURV: v = ifc ? double(F.K[i]) : 0.0; break;
    case RD_NORMAL: v = ifc ? double(F.nrm[comp * N + i]) : 0.0; break;
    case RD_PLIC: v = ifc ? double(F.plic[i]) : 0.0; break;
    case RD_MASS: v = ifc ? double(F.m[i]) : 0.0; break;
    case RD_PRESSURE:
    case RD_VEL:
        if (fluid) {
            double r;
            T ux, uy, uz;
            cell_moments(F, i, r, ux, uy, uz);
            if (what == RD_PRESSURE) v = r / 3.0;
            else v = double(comp == 0 ? ux : (comp == 1 ? uy : uz));
        } else if (what == RD_PRESSURE) {
            v = (fl & FL_GAS) ? (bubble ? F.sc->rho_gas_t : rho_gas) / 3.0 : 0.0;
        }
        break;
    }
    out[i] = v;
}

// Ascending list of the interface cells (read-out): CMP_GRID blocks, each
// owning a contiguous run of 1024-cell tiles of the fluid box; per-block
// counts, one scan block, then every block writes its run in order. The
// scratch holds the block counts, the total and up to `cap` list entries;
// the write pass never writes past `cap` (the host rejects a longer list).
struct ListScratch {
    int *counts;    // CMP_GRID ints
    int *total;     // one int
    int32_t *list;  // cap ints
    int cap;
};

__global__ __launch_bounds__(256) void k_ilist_count(const uint8_t *flags, const DevScalars *sc, int nx, int ny,
                                                     ListScratch s)
{
    const CellRange range = CellRange::from(sc->fbox);
    __shared__ int lw[4];
    int t0, t1;
    tile_range(range.size(), t0, t1);
    int sum = 0;
    for (int t = t0; t < t1; ++t) {
        bool hit[4];
        int idx[4];
        const int c = cells_matching(flags, range, nx, ny, t * CMP_CELLS + threadIdx.x * 4, FL_IF, hit, idx);
        int total;
        block_exclusive_scan(c, lw, total);
        sum += total;
    }
    if (threadIdx.x == 0) s.counts[blockIdx.x] = sum;
}

__global__ __launch_bounds__(1024) void k_ilist_scan(ListScratch s, int nblocks)
{
    __shared__ int lw[16];
    int carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += 1024) {
        const int b = b0 + threadIdx.x;
        const int v = b < nblocks ? s.counts[b] : 0;
        int total;
        const int ex = block_exclusive_scan(v, lw, total);
        if (b < nblocks) s.counts[b] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *s.total = carry;
}

__global__ __launch_bounds__(256) void k_ilist_write(const uint8_t *flags, const DevScalars *sc, int nx, int ny,
                                                     ListScratch s)
{
    const CellRange range = CellRange::from(sc->fbox);
    __shared__ int lw[4];
    int t0, t1;
    tile_range(range.size(), t0, t1);
    int base = s.counts[blockIdx.x];
    for (int t = t0; t < t1; ++t) {
        bool hit[4];
        int idx[4];
        const int c = cells_matching(flags, range, nx, ny, t * CMP_CELLS + threadIdx.x * 4, FL_IF, hit, idx);
        int total;
        int pos = base + block_exclusive_scan(c, lw, total);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (hit[k]) {
                if (pos < s.cap) s.list[pos] = idx[k];
                ++pos;
            }
        base += total;
    }
}

__global__ void k_read_flags(const uint8_t *flags, uint8_t *out, int N)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const uint8_t t = flags[i] & FL_TYPE;
    out[i] = t == FL_GAS ? 0 : (t == FL_LIQ ? 1 : (t == FL_IF ? 2 : 3));
}

// Mass: fixed partition of the cells over MASS_BLOCKS blocks, fixed
// per-thread order and fixed tree inside each block, then one block adds the
// partial sums in a fixed tree. The result does not depend on scheduling.
template <class P>
__global__ __launch_bounds__(256) void k_mass_partial(Fields<P> F, double *part)
{
    using T = typename P::T;
    __shared__ double s[256];
    const int chunk = (F.N + MASS_BLOCKS - 1) / MASS_BLOCKS;
    const int b0 = blockIdx.x * chunk, b1 = min(F.N, b0 + chunk);
    double acc = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += 256) {
        const uint8_t fl = F.flags[i];
        if (fl & FL_LIQ) {
            double r;
            T ux, uy, uz;
            cell_moments(F, i, r, ux, uy, uz);
            acc += r;
        } else if (fl & FL_IF) {
            acc += double(F.m[i]);
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void k_mass_final(const double *part, DevScalars *sc)
{
    __shared__ double s[1024];
    s[threadIdx.x] = threadIdx.x < MASS_BLOCKS ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sc->mass = s[0] + reservoir_value(sc->res_hi, sc->res_lo);
}

// Diagnostics (the measures of Sec. III.A.1: spurious currents and the
// pressure jump), over the same fixed partition and with fixed trees like
// the mass. Per block: max |u| and sum |u| over the fluid cells, their
// count, and the density sum and count of the inner liquid cells, those with
// no gas or interface cell within a Euclidean distance of 2.5 cells
// (periodic). part holds DIAG_VALUES rows of MASS_BLOCKS entries.
template <class P>
__device__ inline bool near_surface(const Fields<P> &F, int i)
{
    const int yz = i / F.nx, x = i - yz * F.nx, z = yz / F.ny, y = yz - z * F.ny;
    for (int dz = -2; dz <= 2; ++dz)
        for (int dy = -2; dy <= 2; ++dy) {
            const int row = F.nx * (wrap_any(y + dy, F.ny) + F.ny * wrap_any(z + dz, F.nz));
            for (int dx = -2; dx <= 2; ++dx) {
                if (dx * dx + dy * dy + dz * dz > 6) continue;
                const uint8_t t = F.flags[row + wrap_any(x + dx, F.nx)] & FL_TYPE;
                if (t == FL_GAS || t == FL_IF) return true;
            }
        }
    return false;
}

template <class P>
__global__ __launch_bounds__(256) void k_diag_partial(Fields<P> F, double *part)
{
    using T = typename P::T;
    __shared__ double s[DIAG_VALUES][256];
    const int chunk = (F.N + MASS_BLOCKS - 1) / MASS_BLOCKS;
    const int b0 = blockIdx.x * chunk, b1 = min(F.N, b0 + chunk);
    double umax = 0.0, usum = 0.0, nfl = 0.0, rsum = 0.0, nin = 0.0;
    for (int i = b0 + threadIdx.x; i < b1; i += 256) {
        const uint8_t fl = F.flags[i];
        if (!(fl & FL_FLUID)) continue;
        double r;
        T ux, uy, uz;
        cell_moments(F, i, r, ux, uy, uz);
        const double a = double(ux), b = double(uy), c = double(uz);
        const double sp = sqrt(a * a + b * b + c * c);
        umax = fmax(umax, sp);
        usum += sp;
        nfl += 1.0;
        if ((fl & FL_TYPE) == FL_LIQ && !near_surface(F, i)) {
            rsum += r;
            nin += 1.0;
        }
    }
    s[0][threadIdx.x] = umax;
    s[1][threadIdx.x] = usum;
    s[2][threadIdx.x] = nfl;
    s[3][threadIdx.x] = rsum;
    s[4][threadIdx.x] = nin;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            for (int v = 1; v < DIAG_VALUES; ++v) s[v][threadIdx.x] += s[v][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < DIAG_VALUES) part[threadIdx.x * MASS_BLOCKS + blockIdx.x] = s[threadIdx.x][0];
}

// One block: the block values in a fixed tree, then the results and the
// current gas density after the partial rows.
__global__ __launch_bounds__(1024) void k_diag_final(double *part, const DevScalars *sc)
{
    __shared__ double s[DIAG_VALUES][1024];
    for (int v = 0; v < DIAG_VALUES; ++v)
        s[v][threadIdx.x] = threadIdx.x < MASS_BLOCKS ? part[v * MASS_BLOCKS + threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            for (int v = 1; v < DIAG_VALUES; ++v) s[v][threadIdx.x] += s[v][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < DIAG_VALUES) part[DIAG_VALUES * MASS_BLOCKS + threadIdx.x] = s[threadIdx.x][0];
    if (threadIdx.x == 0) part[DIAG_VALUES * MASS_BLOCKS + DIAG_VALUES] = sc->rho_gas_t;
}

template <class P>
__global__ void k_check_numeric(Fields<P> F)
{
    using T = typename P::T;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= F.N) return;
    if (!(F.flags[i] & FL_FLUID)) return;
    double r;
    T ux, uy, uz;
    cell_moments(F, i, r, ux, uy, uz);
    if (!(r > 0.0) || !isfinite(r)) atomicOr(&F.sc->bad, 1);
}

// ------------------------------------------------------ host sequences
template <class P>
Batch<P> make_batch(const fslbm_batch *b, int &maxN, bool &any_srt, bool &any_trt)
{
    Batch<P> A;
    maxN = 0;
    any_srt = any_trt = false;
    const int n = (int)b->hs.size();
    for (int i = 0; i < MAXB; ++i) {
        const fslbm_lattice *h = b->hs[i < n ? i : 0];
        A.f[i] = make_fields<P>(h);
        A.p[i] = make_params(h);
    }
    for (int i = 0; i < n; ++i) {
        maxN = std::max(maxN, b->hs[i]->N);
        any_srt |= b->hs[i]->coll == FSLBM_SRT;
        any_trt |= b->hs[i]->coll == FSLBM_TRT;
    }
    return A;
}

inline hipStream_t bstream(const fslbm_batch *b) { return b->hs[0]->stream; }

// Grid of the interface-list kernels of a batch: about one thread per
// interface cell at creation (the loops are grid-stride, so later growth is
// still covered), at least 8 and at most 512 blocks per lattice.
inline int batch_list_blocks(const fslbm_batch *b, int cells_per_block)
{
    int m = 0;
    for (auto *h : b->hs) m = std::max(m, h->icount0);
    return std::min(512, std::max(8, (m + cells_per_block - 1) / cells_per_block));
}

template <class P>
int enqueue_compaction(const fslbm_batch *b, const Batch<P> &A, int maxN, int which, int force)
{
    const unsigned n = (unsigned)b->hs.size();
    const hipStream_t st = bstream(b);
    k_compact_count<P><<<dim3(cmp_blocks(maxN), n), 256, 0, st>>>(A, which, force);
    k_compact_scan<P><<<dim3(1, n), 1024, 0, st>>>(A, which, force, cmp_blocks(maxN));
    k_compact_write<P><<<dim3(cmp_blocks(maxN), n), 256, 0, st>>>(A, which, force);
    HIP_OK(hipGetLastError());
    return 0;
}

// Curvature of every lattice of the batch. With eos = 1 the first launch
// also closes the step's device bookkeeping (end_of_step).
template <class P>
int enqueue_geometry(const fslbm_batch *b, const Batch<P> &A, int maxN, int eos = 0)
{
    const unsigned n = (unsigned)b->hs.size();
    const hipStream_t st = bstream(b);
    const dim3 tg(std::min(GEOM_GRID, std::max(1, maxN / 512)), n);
    bool any_fd = false, any_fd_wall = false, any_lsqr = false, any_tr = false;
    for (auto *h : b->hs) {
        any_fd |= h->curv == FSLBM_CURV_FD;
        any_fd_wall |= h->curv == FSLBM_CURV_FD && h->ocount0 > 0;
        any_lsqr |= h->curv == FSLBM_CURV_LSQR;
        any_tr |= h->curv == FSLBM_CURV_TR;
    }
    const bool any_plic = any_lsqr || any_tr;
    const dim3 cg4(batch_list_blocks(b, 64), n), cgt(batch_list_blocks(b, 256 / TR_LANES), n);
    // FD contact normals exist only next to walls
    if (any_fd_wall) {
        k_fd_contact_normals<P><<<dim3(list_blocks(maxN), n), 256, 0, st>>>(A, eos);
        eos = 0;
    }
    if (any_fd && any_plic) k_geometry_mixed<P><<<tg, 256, 0, st>>>(A, eos);
    else if (any_fd) k_geometry_fd<P><<<tg, 256, 0, st>>>(A, eos);
    else k_normals_plic<P><<<dim3(batch_list_blocks(b, 256), n), 256, 0, st>>>(A, eos);
    if (any_lsqr) k_curv_lsqr4<P><<<cg4, 256, 0, st>>>(A);
    if (any_tr) k_curv_tr<P><<<cgt, 256, 0, st>>>(A);
    HIP_OK(hipGetLastError());
    return 0;
}

template <class P>
int enqueue_geometry_one(fslbm_lattice *h)
{
    int maxN;
    bool s_, t_;
    const Batch<P> A = make_batch<P>(&h->self, maxN, s_, t_);
    return enqueue_geometry<P>(&h->self, A, maxN);
}

// Whether this step runs the lean liquid pass plus the list kernel (split)
// or the merged pass: forced by FSLBM_OPT_SPLIT_INTERFACE = 0 / 1; by
// default (-1) split for the 16-bit storage forms when the interface and
// wall cells are under 1/64 of the fluid box, so that nearly every
// wavefront of the lean pass holds liquid cells only (measured on the 512^3
// probe: F16 split 1.95 ms against merged 2.56 ms; FP32 merged is the
// faster, 3.56 against 3.79 ms, and droplet boxes are full of interface
// cells).
template <class P>
bool split_now(const fslbm_batch *b)
{
    if (b->split_interface >= 0) return b->split_interface == 1;
    if (sizeof(typename P::S) != 2) return false;
    for (auto *h : b->hs)
        if (h->boundary_cells * 64 >= h->box_cells) return false;
    return true;
}

// Kernels of one time step of every lattice of the batch.
// With fsrc / fdst given (a single lattice), the step reads and writes those
// distribution buffers instead of the lattice's pair, and records no timing;
// with snap given too, the kernels that finish the interface-list and
// obstacle-list values also write them there (Fields::snap; LSQR model).
template <class P>
int enqueue_step_kernels(fslbm_batch *b, const void *fsrc = nullptr, void *fdst = nullptr, void *snap = nullptr)
{
    int maxN;
    bool any_srt, any_trt;
    Batch<P> A = make_batch<P>(b, maxN, any_srt, any_trt);
    const bool over = fsrc != nullptr;
    if (over)
        for (int k = 0; k < MAXB; ++k) {
            A.f[k].fsrc = (const typename P::S *)fsrc;
            A.f[k].fdst = (typename P::S *)fdst;
            A.f[k].snap = (typename P::R *)snap;
        }
    auto mark = [&](fslbm_batch *bb, int k) {
        if (!over && bb->timing) (void)hipEventRecord(bb->ev[(size_t)bb->ev_used * TIMING_EV + k], bstream(bb));
    };
    const unsigned n = (unsigned)b->hs.size();
    const hipStream_t st = bstream(b);
    // bulk stream-collide: one block per 256 cells of the largest fluid box
    int boxb = 1;
    for (auto *h : b->hs) boxb = std::max(boxb, h->box_blocks);
    const dim3 cg(boxb, n), sg(std::min(SC_LIST_GRID, cell_blocks(maxN)), n),
        lg(batch_list_blocks(b, 256), n);
    mark(b, 0);
    b->split_last = split_now<P>(b) ? 1 : 0;
    if (b->split_last) {
        if (any_srt) launch_stream_collide<P, 0, 1>(cg, st, A);
        if (any_trt) launch_stream_collide<P, 1, 1>(cg, st, A);
        mark(b, 1);
        if (any_srt) k_stream_collide_list<P, 0><<<sg, 256, 0, st>>>(A);
        if (any_trt) k_stream_collide_list<P, 1><<<sg, 256, 0, st>>>(A);
    } else {
        if (any_srt) launch_stream_collide<P, 0, 0>(cg, st, A);
        if (any_trt) launch_stream_collide<P, 1, 0>(cg, st, A);
        mark(b, 1);
    }
    // with frozen cell types no cell converts: only phi = m / rho remains
    bool frozen = true;
    for (auto *h : b->hs) frozen &= h->frozen != 0;
    mark(b, 2);
    if (!frozen) k_conv_mark_init<P><<<lg, 256, 0, st>>>(A);
    if (!frozen) k_conv_close<P><<<lg, 256, 0, st>>>(A);
    if (!frozen) k_conv_share_keep<P><<<lg, 256, 0, st>>>(A);
    k_conv_gather<P><<<lg, 256, 0, st>>>(A);
    mark(b, 3);
    HIP_OK(hipGetLastError());
    if (!frozen) k_list_finish<P><<<lg, 256, 0, st>>>(A);
    HIP_OK(hipGetLastError());
    int rc = 0;
    mark(b, 4);
    // grid-stride over the static obstacle list (none without walls)
    int maxo = 0;
    for (auto *h : b->hs) maxo = std::max(maxo, h->ocount0);
    if (maxo > 0) k_obstacle_fill<P><<<dim3(std::min(list_blocks(maxN), (maxo + 255) / 256), n), 256, 0, st>>>(A);
    bool any_bubble = false;
    for (auto *h : b->hs) any_bubble |= h->bubble != 0;
    if (any_bubble) {
        k_bubble_partial<P><<<dim3(VOL_BLOCKS, n), 256, 0, st>>>(A);
        k_bubble_final<P><<<dim3(1, n), 1024, 0, st>>>(A, VOL_BLOCKS);
    }
    rc = enqueue_geometry<P>(b, A, maxN, 1);
    if (rc) return rc;
    mark(b, 5);
    return 0;
}

int fold_timing(fslbm_batch *b)
{
    if (!b->timing || b->ev_used == 0) return 0;
    HIP_OK(hipEventSynchronize(b->ev[(size_t)(b->ev_used - 1) * TIMING_EV + TIMING_EV - 1]));
    for (int s = 0; s < b->ev_used; ++s)
        for (int k = 0; k < NPHASE; ++k) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, b->ev[(size_t)s * TIMING_EV + k], b->ev[(size_t)s * TIMING_EV + k + 1]));
            b->tacc[k] += ms;
        }
    b->tsteps += b->ev_used;
    b->ev_used = 0;
    return 0;
}

void drop_graphs(fslbm_batch *b)
{
    for (int c = 0; c < 2; ++c)
        if (b->gexec[c]) {
            (void)hipGraphExecDestroy(b->gexec[c]);
            b->gexec[c] = nullptr;
        }
}

void batch_init(fslbm_batch *b)
{
    b->prec = 0;
    b->timing = 0;
    b->ev_used = 0;
    b->tsteps = 0;
    for (int k = 0; k < NPHASE; ++k) b->tacc[k] = 0.0;
    b->use_graph = 0;
    b->gexec[0] = b->gexec[1] = nullptr;
    b->split_interface = -1;
    b->split_last = 0;
}

void batch_release(fslbm_batch *b)
{
    drop_graphs(b);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    b->ev.clear();
}

int batch_set_timing(fslbm_batch *b, int on)
{
    if (on && b->ev.empty()) {
        b->ev.resize((size_t)TIMING_CAP * TIMING_EV, nullptr);
        for (auto &e : b->ev) HIP_OK(hipEventCreate(&e));
    }
    if (!on) {
        const int rc = fold_timing(b);
        if (rc) return rc;
    }
    b->timing = on;
    return 0;
}

bool graphs_stale(const fslbm_batch *b)
{
    if (b->versions.size() != b->hs.size()) return true;
    for (size_t i = 0; i < b->hs.size(); ++i)
        if (b->versions[i] != b->hs[i]->version) return true;
    return false;
}

template <class P>
int batch_step_once(fslbm_batch *b)
{
    const int cur = b->hs[0]->cur;
    for (auto *h : b->hs)
        if (h->cur != cur) return fail(FSLBM_E_STATE, "lattices of a batch must have taken the same number of steps");
    const hipStream_t st = bstream(b);
    if (b->use_graph && !b->timing && st != nullptr) {
        if (graphs_stale(b)) {
            drop_graphs(b);
            b->versions.clear();
            for (auto *h : b->hs) b->versions.push_back(h->version);
        }
        hipGraphExec_t &ge = b->gexec[cur];
        if (!ge) {
            hipGraph_t g = nullptr;
            HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue_step_kernels<P>(b);
            const hipError_t e = hipStreamEndCapture(st, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(FSLBM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            const hipError_t e2 = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e2 != hipSuccess) {
                ge = nullptr;
                return fail(FSLBM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
            }
        }
        HIP_OK(hipGraphLaunch(ge, st));
    } else {
        if (b->timing && b->ev_used == TIMING_CAP) {
            const int rc = fold_timing(b);
            if (rc) return rc;
        }
        const int rc = enqueue_step_kernels<P>(b);
        if (rc) return rc;
        if (b->timing) b->ev_used += 1;
    }
    for (auto *h : b->hs) {
        h->cur ^= 1;  // f'(t+1) is now current
        h->steps += 1;
    }
    return 0;
}

template <class P>
int enqueue_init(fslbm_lattice *h, const double *fill, const uint8_t *obstacle)
{
    Fields<P> F = make_fields<P>(h);
    const int N = h->N;
    double *staging = (double *)(h->ws + h->L.staging);
    HIP_OK(hipMemcpyAsync(staging, fill, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
    if (obstacle) {
        HIP_OK(hipMemcpyAsync(F.conv, obstacle, N, hipMemcpyHostToDevice, h->stream));
    } else {
        k_fill_bytes<<<std::min(4096, cell_blocks(N)), 256, 0, h->stream>>>(F.conv, N, 0);
    }
    k_init_scalars<<<1, 1, 0, h->stream>>>(F.sc);
    k_init_types<<<cell_blocks(N), 256, 0, h->stream>>>(staging, F.conv, N);
    // the layer stages rotate over conv -> flags -> mark (as bytes) -> conv;
    // k_init_fields then resets mark and writes the final flags
    uint8_t *mark_bytes = (uint8_t *)F.mark;
    k_init_layer<0><<<cell_blocks(N), 256, 0, h->stream>>>(F.conv, F.flags, h->nx, h->ny, h->nz, N);
    k_init_layer<1><<<cell_blocks(N), 256, 0, h->stream>>>(F.flags, mark_bytes, h->nx, h->ny, h->nz, N);
    k_init_layer<2><<<cell_blocks(N), 256, 0, h->stream>>>(mark_bytes, F.conv, h->nx, h->ny, h->nz, N);
    k_init_fields<P><<<cell_blocks(N), 256, 0, h->stream>>>(F, staging, F.conv, F.flags);
    k_fluid_box<<<std::min(1024, cell_blocks(N)), 256, 0, h->stream>>>(F.flags, h->nx, h->ny, N, F.sc);
    // static list of obstacle cells next to non-obstacle cells
    k_mark_wall_cells<<<cell_blocks(N), 256, 0, h->stream>>>(F.flags, F.conv, h->nx, h->ny, h->nz, N);
    HIP_OK(hipGetLastError());
    int maxN;
    bool s_, t_;
    const Batch<P> A = make_batch<P>(&h->self, maxN, s_, t_);
    int rc = enqueue_compaction<P>(&h->self, A, maxN, 1, 1);
    if (!rc) rc = enqueue_compaction<P>(&h->self, A, maxN, 2, 1);
    if (rc) return rc;
    k_fill_bytes<<<std::min(4096, cell_blocks(N)), 256, 0, h->stream>>>(F.conv, N, 0);
    rc = enqueue_compaction<P>(&h->self, A, maxN, 0, 1);
    if (rc) return rc;
    k_obstacle_fill<P><<<dim3(list_blocks(N), 1), 256, 0, h->stream>>>(A);
    HIP_OK(hipGetLastError());
    return enqueue_geometry<P>(&h->self, A, maxN);
}

template <class P>
int do_read(fslbm_lattice *h, int what, double *out, int out_is_device)
{
    const Fields<P> F = make_fields<P>(h);
    const int N = h->N;
    const int comps = (what == RD_VEL || what == RD_NORMAL) ? 3 : 1;
    double *staging = (double *)(h->ws + h->L.staging);
    for (int c = 0; c < comps; ++c) {
        double *dst = out_is_device ? out + (size_t)c * N : staging;
        k_read<P><<<cell_blocks(N), 256, 0, h->stream>>>(F, h->rho_gas, h->bubble, what, c, dst);
        HIP_OK(hipGetLastError());
        if (!out_is_device)
            HIP_OK(hipMemcpyAsync(out + (size_t)c * N, staging, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream));
    }
    HIP_OK(hipStreamSynchronize(h->stream));
    return 0;
}

template <class P>
int do_mass(fslbm_lattice *h, double *total)
{
    const Fields<P> F = make_fields<P>(h);
    double *part = (double *)(h->ws + h->L.part);
    k_mass_partial<P><<<MASS_BLOCKS, 256, 0, h->stream>>>(F, part);
    k_mass_final<<<1, 1024, 0, h->stream>>>(part, F.sc);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(total, &F.sc->mass, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return 0;
}

template <class P>
int do_diagnostics(fslbm_lattice *h, double *out)
{
    const Fields<P> F = make_fields<P>(h);
    double *part = (double *)(h->ws + h->L.part);
    k_diag_partial<P><<<MASS_BLOCKS, 256, 0, h->stream>>>(F, part);
    k_diag_final<<<1, 1024, 0, h->stream>>>(part, F.sc);
    HIP_OK(hipGetLastError());
    double v[DIAG_VALUES + 1];
    HIP_OK(hipMemcpyAsync(v, part + DIAG_VALUES * MASS_BLOCKS, sizeof(v), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    const double rho_gas = h->bubble ? v[DIAG_VALUES] : h->rho_gas;
    out[0] = v[0];
    out[1] = v[2] > 0.0 ? v[1] / v[2] : 0.0;
    out[2] = v[4] > 0.0 ? (v[3] / v[4] - rho_gas) / 3.0 : 0.0;
    out[3] = v[4];
    return 0;
}

template <class P>
int do_check(fslbm_lattice *h)
{
    const Fields<P> F = make_fields<P>(h);
    int zero = 0, bad = 0;
    HIP_OK(hipMemcpyAsync(&F.sc->bad, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream));
    k_check_numeric<P><<<cell_blocks(h->N), 256, 0, h->stream>>>(F);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(&bad, &F.sc->bad, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return bad ? fail(FSLBM_E_NUMERIC, "non-finite or non-positive density in a fluid cell") : 0;
}

template <class P>
int do_set_equilibrium(fslbm_lattice *h, const double *rho, const double *u3)
{
    const Fields<P> F = make_fields<P>(h);
    const int N = h->N;
    double *staging = (double *)(h->ws + h->L.staging);
    // the velocity goes through the (scratch) destination PDF buffer, whose
    // 19 planes hold at least 3 planes of doubles for every precision
    double *ubuf = (double *)(h->ws + (h->cur == 0 ? h->L.fB : h->L.fA));
    HIP_OK(hipMemcpyAsync(staging, rho, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
    HIP_OK(hipMemcpyAsync(ubuf, u3, sizeof(double) * 3 * N, hipMemcpyHostToDevice, h->stream));
    k_set_equilibrium<P><<<cell_blocks(N), 256, 0, h->stream>>>(F, staging, ubuf);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(h->stream));
    return 0;
}

// ------------------------------------------- interface fill, state copies
template <class P>
__global__ void k_set_interface_fill(Fields<P> F, const double *fill)
{
    using R = typename P::R;
    const int n = F.sc->icount;
    for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
        const int i = F.ilist[k];
        const R phi = R(fill[i]);
        F.phi[i] = phi;
        F.m[i] = phi * F.rho[i];
    }
}

template <class P>
int do_set_interface_fill(fslbm_lattice *h, const double *fill, int is_device)
{
    const Fields<P> F = make_fields<P>(h);
    const int N = h->N;
    const double *src = fill;
    if (!is_device) {
        double *staging = (double *)(h->ws + h->L.staging);
        HIP_OK(hipMemcpyAsync(staging, fill, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
        src = staging;
    }
    k_set_interface_fill<P><<<list_blocks(N), 256, 0, h->stream>>>(F, src);
    HIP_OK(hipGetLastError());
    int maxN;
    bool s_, t_;
    const Batch<P> A = make_batch<P>(&h->self, maxN, s_, t_);
    k_obstacle_fill<P><<<dim3(list_blocks(N), 1), 256, 0, h->stream>>>(A);
    HIP_OK(hipGetLastError());
    const int rc = enqueue_geometry<P>(&h->self, A, maxN);
    if (rc) return rc;
    if (!is_device) HIP_OK(hipStreamSynchronize(h->stream));
    return 0;
}

// Parts of the workspace that make up the state (offset, bytes); the first
// entry is the current distribution buffer.
std::vector<std::pair<size_t, size_t>> state_regions(const fslbm_lattice *h)
{
    const Layout &L = h->L;
    const size_t N = h->N, fb = fbytes(h->prec), rb = rbytes(h->prec);
    return {{h->cur == 0 ? L.fA : L.fB, 19 * (size_t)h->NS * fb},
            {L.flags, N},
            {L.mark, 4 * N},
            {L.m, N * rb},
            {L.rho, N * rb},
            {L.phi, N * rb},
            {L.K, N * rb},
            {L.nrm, 3 * N * rb},
            {L.plic, N * rb},
            {L.ilist, 4 * N},
            {L.olist, 4 * N},
            {L.wlist, 4 * N},
            {L.sc, sizeof(DevScalars)}};
}

struct StateHeader {
    uint64_t magic;
    int32_t nx, ny, nz, prec, curv, pad;
    int64_t steps;
};
// state blob tag, layout version 2 (distribution planes 1024 elements apart)
constexpr uint64_t STATE_MAGIC = 0x32564d42534c5346ull;

size_t state_bytes(const fslbm_lattice *h)
{
    size_t b = 256;
    for (auto &r : state_regions(h)) b += align256(r.second);
    return b;
}

// ------------------------------------------------ frozen-topology window
size_t adj_layout(AdjWindow &w, const fslbm_lattice *h)
{
    const size_t N = h->N;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    for (int b = 0; b < 2; ++b) {
        w.off_gin[b] = take(19 * N * 8);
        w.off_own[b] = take(19 * N * 8);
    }
    w.off_refl = take((size_t)(NQ - 1) * std::max(1, w.icount) * 8);
    w.off_scal = take(8 * N * 8);  // mbar phib rhob kbar sacc tacc ms msb
    w.off_gb = take(3 * N * 8);
    w.off_contrib = take((size_t)CONTRIB * std::max(1, w.icount) * 8);
    w.off_pos = take(4 * N);
    w.off_part = take(8 * (MASS_BLOCKS + 4));
    w.f_bytes = align256(19 * (size_t)h->NS * fbytes(h->prec));
    w.snap_bytes = align256(((size_t)SNAP * w.icount + w.ocount) * rbytes(h->prec));
    w.slot_bytes = w.f_bytes + w.snap_bytes;
    w.ck.clear();
    for (long long t = 0; t < w.T; t += w.K) w.ck.push_back(t);
    w.ck.push_back(w.T);
    w.off_ck = take(w.ck.size() * w.slot_bytes);
    // two rings: the reverse steps of one segment read one while the
    // recompute of the segment before it fills the other
    const long long ring = std::max(0LL, std::min<long long>(w.K, w.T) - 1);
    for (int r = 0; r < 2; ++r) w.off_ring[r] = take((size_t)ring * w.slot_bytes);
    w.off_shadow = take(h->L.total - h->L.flags);
    w.total = off;
    return off;
}

// Adjoint fields; gin / own of the previous reverse step are read from
// buffer `par` and written to buffer 1 - par.
Adj adj_fields(const AdjWindow &w, const fslbm_lattice *h, int par)
{
    const size_t N = h->N;
    char *b = w.ws;
    Adj A;
    A.gin_in = (const double *)(b + w.off_gin[par]);
    A.own_in = (const double *)(b + w.off_own[par]);
    A.gin = (double *)(b + w.off_gin[1 - par]);
    A.own = (double *)(b + w.off_own[1 - par]);
    A.refl = (double *)(b + w.off_refl);
    double *s = (double *)(b + w.off_scal);
    A.mbar = s;
    A.phib = s + N;
    A.rhob = s + 2 * N;
    A.kbar = s + 3 * N;
    A.sacc = s + 4 * N;
    A.tacc = s + 5 * N;
    A.ms = s + 6 * N;
    A.msb = s + 7 * N;
    A.gb = (double *)(b + w.off_gb);
    A.contrib = (double *)(b + w.off_contrib);
    A.pos = (int *)(b + w.off_pos);
    return A;
}

// Reads the fluid box back (synchronises the stream) and sizes the bulk
// stream-collide grid to it; a changed grid invalidates captured graphs.
int refresh_box(fslbm_lattice *h)
{
    const DevScalars *scd = (const DevScalars *)(h->ws + h->L.sc);
    DevScalars sc;
    HIP_OK(hipMemcpyAsync(&sc, scd, sizeof sc, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    const int *b = sc.fbox;
    long long cells = 0;
    if (b[3] >= b[0] && b[4] >= b[1] && b[5] >= b[2])
        cells = (long long)(b[3] - b[0] + 1) * (b[4] - b[1] + 1) * (b[5] - b[2] + 1);
    const int blocks = xcd_grid((cells + SC_BLOCK - 1) / SC_BLOCK);
    h->boundary_cells = (long long)sc.icount + sc.wcount;
    h->box_cells = cells;
    if (blocks != h->box_blocks) {
        h->box_blocks = blocks;
        h->version += 1;
    }
    return 0;
}

int read_counts(fslbm_lattice *h, int &icount, int &ocount)
{
    const DevScalars *sc = (const DevScalars *)(h->ws + h->L.sc);
    int v[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(v, &sc->icount, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    icount = v[0];
    ocount = v[1];
    return 0;
}

// Slot (distributions, snapshot) of the state at time t of the segment
// [t0, t1] with checkpoint index s at t0.
struct Slot {
    char *f;
    char *snap;
};
inline Slot ck_slot(const AdjWindow &w, size_t s)
{
    char *b = w.ws + w.off_ck + s * w.slot_bytes;
    return {b, b + w.f_bytes};
}
inline Slot seg_slot(const AdjWindow &w, size_t s, long long t)
{
    const long long t0 = w.ck[s], t1 = w.ck[s + 1];
    if (t == t0) return ck_slot(w, s);
    if (t == t1) return ck_slot(w, s + 1);
    char *b = w.ws + w.off_ring[s & 1] + (size_t)(t - t0 - 1) * w.slot_bytes;
    return {b, b + w.f_bytes};
}

template <class P>
int save_slot(fslbm_lattice *h, const Slot &sl, bool with_f)
{
    const Fields<P> F = make_fields<P>(h);
    if (with_f)
        HIP_OK(hipMemcpyAsync(sl.f, F.fsrc, 19 * (size_t)h->NS * fbytes(h->prec), hipMemcpyDeviceToDevice, h->stream));
    k_snap<P><<<list_blocks(h->N), 256, 0, h->stream>>>(F, (typename P::R *)sl.snap, 1);
    HIP_OK(hipGetLastError());
    return 0;
}

template <class P>
int load_snap(fslbm_lattice *h, const char *snap)
{
    const Fields<P> F = make_fields<P>(h);
    k_snap<P><<<list_blocks(h->N), 256, 0, h->stream>>>(F, (typename P::R *)snap, 0);
    HIP_OK(hipGetLastError());
    return 0;
}

// The device step number (it seeds the stochastic 16-bit stores).
__global__ void k_set_step(DevScalars *sc, unsigned step) { sc->step = step; }

__global__ void k_reset_fill_out(DevScalars *sc)
{
    sc->fill_out = 0;
    sc->fill_out_step = 0xffffffffu;
    sc->conv_out_step = 0xffffffffu;
}

template <class P>
int do_adj_forward(fslbm_lattice *h, long long T, int K, void *ws, size_t bytes)
{
    AdjWindow &w = h->adj;
    w.recorded = 0;
    int rc = read_counts(h, w.icount, w.ocount);
    if (rc) return rc;
    w.T = T;
    w.K = K;
    adj_layout(w, h);
    if (bytes < w.total) return fail(FSLBM_E_SHAPE, "adjoint workspace has %zu bytes, %zu needed", bytes, w.total);
    w.ws = (char *)ws;
    w.bytes = bytes;
    DevScalars *sc = (DevScalars *)(h->ws + h->L.sc);
    unsigned start_step = 0;
    HIP_OK(hipMemcpyAsync(&start_step, &sc->step, sizeof start_step, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    w.start_step = start_step;
    k_reset_fill_out<<<1, 1, 0, h->stream>>>(sc);
    HIP_OK(hipGetLastError());
    h->frozen = 1;
    h->version += 1;
    rc = save_slot<P>(h, ck_slot(w, 0), true);
    size_t next = 1;
    for (long long t = 1; t <= T && !rc; ++t) {
        rc = batch_step_once<P>(&h->self);
        if (!rc && t == w.ck[next]) rc = save_slot<P>(h, ck_slot(w, next++), true);
    }
    h->frozen = 0;
    h->version += 1;
    if (rc) return rc;
    unsigned out[3] = {0, 0, 0};  // fill_out, fill_out_step, conv_out_step
    HIP_OK(hipMemcpyAsync(out, &sc->fill_out, sizeof out, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    w.fill_events = (int)out[0];
    // the window's step t (1..T) runs with step number start_step + t - 1
    w.inside_steps = out[0] == 0 ? T : (long long)(out[1] - start_step);
    w.unconverted_steps = out[2] == 0xffffffffu ? T : (long long)(out[2] - start_step);
    w.t_end = h->steps;
    w.epoch = h->epoch;
    w.recorded = 1;
    return 0;
}

template <class P>
int enqueue_geometry_adjoint(fslbm_lattice *h, const Fields<P> &F, const Adj &A, const Params &prm)
{
    const hipStream_t st = h->stream;
    const int N = h->N;
    const int cg = std::min(4096, cell_blocks(N)), lg = list_blocks(N);
    if (h->curv == FSLBM_CURV_FD) {
        k_adj_fd_mol<P><<<cg, 256, 0, st>>>(F, A);
        k_adj_fd_nbar<P><<<cg, 256, 0, st>>>(F, A, prm);
        k_adj_fd_msb<P><<<cg, 256, 0, st>>>(F, A);
        k_adj_fd_phib<P><<<cg, 256, 0, st>>>(F, A);
    } else {
        const int cpb = 256 / ADJ_LANES;  // interface cells per block
        const int l8 = std::min(2048, std::max(1, (h->adj.icount + cpb - 1) / cpb));
        k_adj_lsqr_cell<P><<<l8 + lg, 256, 0, st>>>(F, A, prm, l8);
        k_adj_lsqr_plic<P><<<l8, 256, 0, st>>>(F, A);
        k_adj_lsqr_phib<P><<<lg, 256, 0, st>>>(F, A);
    }
    HIP_OK(hipGetLastError());
    return 0;
}

template <class P>
int do_adj_backward(fslbm_lattice *h, const double *dphi, int in_dev, double *dsig, double *dth, double *dfill0,
                    int out_dev)
{
    AdjWindow &w = h->adj;
    const hipStream_t st = h->stream;
    const int N = h->N;
    const int cg = std::min(4096, cell_blocks(N)), lg = list_blocks(N);
    int par = 0;
    Adj A = adj_fields(w, h, par);
    // adjoint state at T: lam = 0 (gin = own = 0), mbar = 0, phib = dL/dphi_T
    for (int b = 0; b < 2; ++b) {
        k_adj_zero<<<4096, 256, 0, st>>>((double *)(w.ws + w.off_gin[b]), 19 * (size_t)N);
        k_adj_zero<<<4096, 256, 0, st>>>((double *)(w.ws + w.off_own[b]), 19 * (size_t)N);
    }
    k_adj_zero<<<4096, 256, 0, st>>>((double *)(w.ws + w.off_scal), 8 * (size_t)N);
    k_adj_zero<<<4096, 256, 0, st>>>(A.gb, 3 * (size_t)N);
    HIP_OK(hipGetLastError());
    double *staging = (double *)(h->ws + h->L.staging);
    const double *src = dphi;
    if (!in_dev) {
        HIP_OK(hipMemcpyAsync(staging, dphi, sizeof(double) * N, hipMemcpyHostToDevice, st));
        src = staging;
    }
    {
        const Fields<P> F = make_fields<P>(h);
        k_adj_begin<P><<<lg, 256, 0, st>>>(F, A, src);
        k_adj_reflect_setup<P><<<lg, 256, 0, st>>>(F, A);
        HIP_OK(hipGetLastError());
    }
    h->frozen = 1;
    const Params prm = make_params(h);
    const size_t nseg = w.ck.size() - 1;
    // Segment s is recomputed on a second stream, on the copy of the
    // non-distribution fields at off_shadow and into ring s % 2, while the
    // reverse steps of segment s + 1 run on the handle's stream from the
    // other ring and the handle's own fields: both chains are latency-bound
    // launches of a few thousand wavefronts, so they overlap. Events order
    // the rings: ev[s] = recompute of s done, ev[nseg + s] = reverse of s
    // done, ev[2 nseg] = the copy of the fields done.
    int rc = 0;
    auto hip = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && !rc) rc = fail(FSLBM_E_HIP, "%s: %s", what, hipGetErrorString(e));
    };
    hipStream_t st2 = nullptr;
    std::vector<hipEvent_t> ev(2 * nseg + 1, nullptr);
    auto cleanup = [&]() {
        h->stream = st;
        h->scal_base = nullptr;
        if (st2) (void)hipStreamSynchronize(st2);
        (void)hipStreamSynchronize(st);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
        if (st2) (void)hipStreamDestroy(st2);
    };
    // the stream and events belong to the lattice's device, whichever device
    // is current
    int dev0 = 0;
    hip(hipGetDevice(&dev0), "hipGetDevice");
    if (!rc && dev0 != h->device) hip(hipSetDevice(h->device), "hipSetDevice");
    if (!rc) hip(hipStreamCreateWithFlags(&st2, hipStreamNonBlocking), "hipStreamCreateWithFlags");
    for (auto &e : ev)
        if (!rc) hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
    if (dev0 != h->device) (void)hipSetDevice(dev0);
    char *shadow = w.ws + w.off_shadow;
    if (!rc)
        hip(hipMemcpyAsync(shadow, h->ws + h->L.flags, h->L.total - h->L.flags, hipMemcpyDeviceToDevice, st),
            "copy of the fields");
    if (!rc) hip(hipEventRecord(ev[2 * nseg], st), "hipEventRecord");
    if (!rc) hip(hipStreamWaitEvent(st2, ev[2 * nseg], 0), "hipStreamWaitEvent");
    const bool lsqr = h->curv == FSLBM_CURV_LSQR;
    // the states t0+1 .. t1-1 of segment s into its ring, with the step
    // numbers the window ran them with (the 16-bit forms draw their rounding
    // bits from them); the LSQR step writes the snapshot itself, FD takes
    // k_snap
    auto recompute = [&](size_t sg) {
        if (sg + 2 < nseg && !rc) hip(hipStreamWaitEvent(st2, ev[nseg + sg + 2], 0), "hipStreamWaitEvent");
        // the step functions enqueue on h->stream and take their fields from
        // make_fields(h): both point at the second stream and the copy while
        // this segment's steps are enqueued (host code, one thread per handle)
        h->stream = st2;
        h->scal_base = shadow;
        const long long t0 = w.ck[sg], t1 = w.ck[sg + 1];
        if (!rc) rc = load_snap<P>(h, ck_slot(w, sg).snap);
        if (!rc) {
            k_set_step<<<1, 1, 0, st2>>>(make_fields<P>(h).sc, w.start_step + (unsigned)t0);
            hip(hipGetLastError(), "k_set_step");
        }
        for (long long t = t0; t + 1 < t1 && !rc; ++t) {
            const Slot a = seg_slot(w, sg, t), b = seg_slot(w, sg, t + 1);
            rc = enqueue_step_kernels<P>(&h->self, a.f, b.f, lsqr ? b.snap : nullptr);
            if (!rc && !lsqr) {
                const Fields<P> F = make_fields<P>(h);
                k_snap<P><<<lg, 256, 0, st2>>>(F, (typename P::R *)b.snap, 1);
                hip(hipGetLastError(), "k_snap");
            }
        }
        h->stream = st;
        h->scal_base = nullptr;
        if (!rc) hip(hipEventRecord(ev[sg], st2), "hipEventRecord");
    };
    if (!rc && nseg > 0) recompute(nseg - 1);
    for (size_t s = nseg; s-- > 0 && !rc;) {
        if (s > 0) recompute(s - 1);
        if (!rc) hip(hipStreamWaitEvent(st, ev[s], 0), "hipStreamWaitEvent");
        const long long t0 = w.ck[s], t1 = w.ck[s + 1];
        // reverse steps t1-1 .. t0
        for (long long t = t1 - 1; t >= t0 && !rc; --t) {
            const Slot cur = seg_slot(w, s, t), nxt = seg_slot(w, s, t + 1);
            Fields<P> F = make_fields<P>(h);
            k_adj_prepass<P><<<lg, 256, 0, st>>>(F, A, (const typename P::R *)nxt.snap,
                                                 (const typename P::R *)cur.snap);
            F.fsrc = (const typename P::S *)cur.f;
            A = adj_fields(w, h, par);
            if (h->coll == FSLBM_SRT) k_adj_stream<P, 0><<<cg, 256, 0, st>>>(F, A, prm);
            else k_adj_stream<P, 1><<<cg, 256, 0, st>>>(F, A, prm);
            par ^= 1;
            hip(hipGetLastError(), "k_adj_stream");
            if (!rc) rc = enqueue_geometry_adjoint<P>(h, F, A, prm);
        }
        if (!rc) hip(hipEventRecord(ev[nseg + s], st), "hipEventRecord");
    }
    cleanup();
    h->frozen = 0;
    if (rc) return rc;
    // dL/dphi_0, dL/dsigma, dL/dtheta
    double *out = out_dev ? dfill0 : staging;
    k_adj_zero<<<cg, 256, 0, st>>>(out, (size_t)N);
    {
        const Fields<P> F = make_fields<P>(h);
        k_adj_finish<P><<<lg, 256, 0, st>>>(F, A, (const typename P::R *)ck_slot(w, 0).snap, out);
    }
    double *part = (double *)(w.ws + w.off_part);
    double *res = part + MASS_BLOCKS;
    k_adj_sum_partial<<<MASS_BLOCKS, 256, 0, st>>>(A.sacc, N, part, MASS_BLOCKS);
    k_adj_sum_final<<<1, 1024, 0, st>>>(part, MASS_BLOCKS, res);
    k_adj_sum_partial<<<MASS_BLOCKS, 256, 0, st>>>(A.tacc, N, part, MASS_BLOCKS);
    k_adj_sum_final<<<1, 1024, 0, st>>>(part, MASS_BLOCKS, res + 1);
    HIP_OK(hipGetLastError());
    if (!out_dev) HIP_OK(hipMemcpyAsync(dfill0, staging, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    double g[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(g, res, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    // back to the state at the end of the window
    {
        const Slot last = ck_slot(w, nseg);
        rc = load_snap<P>(h, last.snap);
        if (rc) return rc;
        const Fields<P> F = make_fields<P>(h);
        HIP_OK(hipMemcpyAsync((void *)F.fsrc, last.f, 19 * (size_t)h->NS * fbytes(h->prec), hipMemcpyDeviceToDevice, st));
        k_set_step<<<1, 1, 0, st>>>(F.sc, w.start_step + (unsigned)w.T);
        HIP_OK(hipGetLastError());
    }
    HIP_OK(hipStreamSynchronize(st));
    if (dsig) *dsig = g[0];
    if (dth) *dth = g[1];
    return 0;
}

// Dispatch on the precision of the handle.
template <template <class> class Op, class... A>
int dispatch(fslbm_lattice *h, A... a)
{
    switch (h->prec) {
    case P_F64: return Op<Prec<P_F64>>::run(h, a...);
    case P_F32: return Op<Prec<P_F32>>::run(h, a...);
    case P_F16: return Op<Prec<P_F16>>::run(h, a...);
    default: return Op<Prec<P_BF16>>::run(h, a...);
    }
}
template <class P> struct OpInit { static int run(fslbm_lattice *h, const double *f, const uint8_t *o) { return enqueue_init<P>(h, f, o); } };
template <class P> struct OpGeom { static int run(fslbm_lattice *h) { return enqueue_geometry_one<P>(h); } };

int batch_step(fslbm_batch *b, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc;
        switch (b->prec) {
        case P_F64: rc = batch_step_once<Prec<P_F64>>(b); break;
        case P_F32: rc = batch_step_once<Prec<P_F32>>(b); break;
        case P_F16: rc = batch_step_once<Prec<P_F16>>(b); break;
        default: rc = batch_step_once<Prec<P_BF16>>(b); break;
        }
        if (rc) return rc;
    }
    return 0;
}
template <class P> struct OpRead { static int run(fslbm_lattice *h, int w, double *o, int d) { return do_read<P>(h, w, o, d); } };
template <class P> struct OpMass { static int run(fslbm_lattice *h, double *t) { return do_mass<P>(h, t); } };
template <class P> struct OpCheck { static int run(fslbm_lattice *h) { return do_check<P>(h); } };
template <class P> struct OpDiag { static int run(fslbm_lattice *h, double *o) { return do_diagnostics<P>(h, o); } };
template <class P> struct OpEq { static int run(fslbm_lattice *h, const double *r, const double *u) { return do_set_equilibrium<P>(h, r, u); } };

__global__ void k_bubble_arm(DevScalars *sc) { sc->bubble_init = 1; }

template <class P>
int do_bubble_start(fslbm_lattice *h)
{
    int maxN;
    bool s_, t_;
    const Batch<P> A = make_batch<P>(&h->self, maxN, s_, t_);
    const Fields<P> F = make_fields<P>(h);
    k_bubble_arm<<<1, 1, 0, h->stream>>>(F.sc);
    k_bubble_partial<P><<<dim3(VOL_BLOCKS, 1), 256, 0, h->stream>>>(A);
    k_bubble_final<P><<<dim3(1, 1), 1024, 0, h->stream>>>(A, VOL_BLOCKS);
    HIP_OK(hipGetLastError());
    return 0;
}
template <class P> struct OpBubble { static int run(fslbm_lattice *h) { return do_bubble_start<P>(h); } };

template <class P> struct OpFill { static int run(fslbm_lattice *h, const double *f, int d) { return do_set_interface_fill<P>(h, f, d); } };
template <class P> struct OpAdjF { static int run(fslbm_lattice *h, long long T, int K, void *w, size_t b) { return do_adj_forward<P>(h, T, K, w, b); } };
template <class P> struct OpAdjB {
    static int run(fslbm_lattice *h, const double *g, int gd, double *ds, double *dt, double *d0, int od)
    {
        return do_adj_backward<P>(h, g, gd, ds, dt, d0, od);
    }
};

}  // namespace

// ================================================================ C ABI
extern "C" {

const char *fslbm_last_error(void) { return g_err.c_str(); }

int fslbm_required_bytes(int nx, int ny, int nz, int precision, size_t *bytes)
{
    if (!bytes) return fail(FSLBM_E_ARG, "bytes is NULL");
    if (precision < 0 || precision > 3) return fail(FSLBM_E_ARG, "unknown precision %d", precision);
    if (!shape_ok(nx, ny, nz)) return fail(FSLBM_E_SHAPE, "lattice %dx%dx%d out of range", nx, ny, nz);
    *bytes = make_layout(nx, ny, nz, precision).total;
    return 0;
}

int fslbm_pull_copy_bytes(int nx, int ny, int nz, int precision, size_t *bytes)
{
    if (!bytes) return fail(FSLBM_E_ARG, "bytes is NULL");
    if (precision < 0 || precision > 3) return fail(FSLBM_E_ARG, "unknown precision %d", precision);
    if (!shape_ok(nx, ny, nz)) return fail(FSLBM_E_SHAPE, "lattice %dx%dx%d out of range", nx, ny, nz);
    *bytes = 19 * (size_t)plane_stride((long long)nx * ny * nz) * fbytes(precision);
    return 0;
}

int fslbm_pull_copy_time(int nx, int ny, int nz, int precision, const void *src, void *dst, size_t buffer_bytes,
                         void *hip_stream, int launches, double *us_per_launch)
{
    size_t need = 0;
    const int rc = fslbm_pull_copy_bytes(nx, ny, nz, precision, &need);
    if (rc) return rc;
    if (!src || !dst || !us_per_launch) return fail(FSLBM_E_ARG, "src, dst or us_per_launch is NULL");
    if (src == dst) return fail(FSLBM_E_ARG, "src and dst must be different buffers");
    if (buffer_bytes < need) return fail(FSLBM_E_SHAPE, "buffers of %zu bytes, %zu needed", buffer_bytes, need);
    if (launches < 1 || launches > 100000) return fail(FSLBM_E_ARG, "launches %d out of range", launches);
    const long long N = (long long)nx * ny * nz;
    const int NS = (int)plane_stride(N);
    const int blocks = xcd_grid((N + SC_BLOCK - 1) / SC_BLOCK);
    hipStream_t st = (hipStream_t)hip_stream;
    auto launch = [&]() {
        switch (precision) {
        case P_F64:
            k_pull_copy<double><<<blocks, SC_BLOCK, 0, st>>>((const double *)src, (double *)dst, nx, ny, nz, NS, 1);
            break;
        case P_F32:
            k_pull_copy<float><<<blocks, SC_BLOCK, 0, st>>>((const float *)src, (float *)dst, nx, ny, nz, NS,
                                                             xcd_run<Prec<P_F32>>());
            break;
        default:
            k_pull_copy<uint16_t><<<blocks, SC_BLOCK, 0, st>>>((const uint16_t *)src, (uint16_t *)dst, nx, ny, nz, NS,
                                                                xcd_run<Prec<P_F16>>());
        }
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(FSLBM_E_HIP, "hipEventCreate failed");
    }
    launch();  // untimed
    hipError_t e = hipEventRecord(e0, st);
    for (int k = 0; k < launches && e == hipSuccess; ++k) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(FSLBM_E_HIP, "pull copy: %s", hipGetErrorString(e));
    *us_per_launch = 1000.0 * ms / launches;
    return 0;
}

}  // extern "C"

namespace {
// What the closure of the interface layer at creation does to the input
// (Sec. II.D: an interface cell has both gas and liquid D3Q19 neighbours;
// the device closes the layer in two passes, see k_init_layer): a partly
// filled cell without a gas neighbour closes to liquid; a cell of the layer
// that keeps a gas neighbour but has no neighbour that ends the first pass
// liquid closes to gas. A cell is thus rounded to one phase. Rounded to the
// phase that fills less than half of it (a fill >= 1/2 closing to gas, or
// <= 1/2 closing to liquid), it belonged to a liquid film or gas layer
// thinner than one cell: the configuration of Fig. limitation, which the
// method does not support. Host code, run before any device call; periodic
// wrap on every axis as on the device.
LayerClosure layer_closure(int nx, int ny, int nz, const double *fill, const uint8_t *obst)
{
    auto is_obst = [&](long long j) { return obst && obst[j]; };
    auto gas0 = [&](long long j) { return !is_obst(j) && fill[j] <= 0.0; };
    auto wrap = [](long long v, long long n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
    auto nbr = [&](long long x, long long y, long long z, int q) {
        return wrap(x + dir_x(q), nx) + nx * (wrap(y + dir_y(q), ny) + (long long)ny * wrap(z + dir_z(q), nz));
    };
    auto has_gas = [&](long long j) {
        const long long x = j % nx, y = (j / nx) % ny, z = j / ((long long)nx * ny);
        for (int q = 1; q < NQ; ++q)
            if (gas0(nbr(x, y, z, q))) return true;
        return false;
    };
    // rows (y, z) that hold a gas cell: a liquid cell can touch gas only if
    // its own or a neighbouring row does
    std::vector<uint8_t> row_gas((size_t)ny * nz, 0);
    for (long long r = 0; r < (long long)ny * nz; ++r)
        for (long long x = 0; x < nx; ++x)
            if (gas0(r * nx + x)) {
                row_gas[r] = 1;
                break;
            }
    LayerClosure c;
    for (long long z = 0; z < nz; ++z)
        for (long long y = 0; y < ny; ++y) {
            bool near_gas = false;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy) near_gas |= row_gas[wrap(y + dy, ny) + ny * wrap(z + dz, nz)] != 0;
            for (long long x = 0; x < nx; ++x) {
                const long long i = x + nx * (y + (long long)ny * z);
                const double f = fill[i];
                if (is_obst(i) || f <= 0.0) continue;
                if (f >= 1.0 && !near_gas) continue;  // liquid far from gas
                const bool g = near_gas && has_gas(i);
                if (f >= 1.0 && !g) continue;  // liquid, not on the layer
                if (!g) {  // a partly filled cell without a gas neighbour closes to liquid
                    c.against += f <= 0.5;
                    c.to_liquid += 1;
                    c.fill_added += 1.0 - f;
                    continue;
                }
                // on the layer after the first pass: closes to gas without a liquid neighbour
                bool liquid_nbr = false;
                for (int q = 1; q < NQ && !liquid_nbr; ++q) {
                    const long long j = nbr(x, y, z, q);
                    liquid_nbr = !is_obst(j) && fill[j] > 0.0 && !has_gas(j);
                }
                if (!liquid_nbr) {  // closes to gas (fill 1 for a liquid cell on the layer)
                    c.against += f >= 0.5;
                    c.to_gas += 1;
                    c.fill_removed += std::min(f, 1.0);
                }
            }
        }
    return c;
}
}  // namespace

extern "C" {

int fslbm_create(int nx, int ny, int nz, int precision, int curv_model, const double *fill,
                 const uint8_t *obstacle, void *workspace, size_t workspace_bytes, void *hip_stream,
                 fslbm_t *out)
{
    if (!out) return fail(FSLBM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!fill) return fail(FSLBM_E_ARG, "fill is NULL");
    if (!workspace) return fail(FSLBM_E_ARG, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(FSLBM_E_ARG, "workspace not 256-byte aligned");
    if (precision < 0 || precision > 3) return fail(FSLBM_E_ARG, "unknown precision %d", precision);
    if (curv_model != FSLBM_CURV_FD && curv_model != FSLBM_CURV_LSQR && curv_model != FSLBM_CURV_TR)
        return fail(FSLBM_E_ARG, "unknown curvature model %d", curv_model);
    if (!shape_ok(nx, ny, nz)) return fail(FSLBM_E_SHAPE, "lattice %dx%dx%d out of range", nx, ny, nz);
    // the FD model's 8^3 tiles read from 3 cells below to 10 cells above a
    // tile origin; one periodic wrap covers that only for extents >= 10
    if (curv_model == FSLBM_CURV_FD && (nx < 10 || ny < 10 || nz < 10))
        return fail(FSLBM_E_SHAPE, "the FD curvature model needs every extent >= 10 (lattice %dx%dx%d)", nx, ny, nz);
    const long long N = (long long)nx * ny * nz;
    const Layout L = make_layout(nx, ny, nz, precision);
    if (workspace_bytes < L.total)
        return fail(FSLBM_E_SHAPE, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
    const LayerClosure closure = layer_closure(nx, ny, nz, fill, obstacle);
    if (closure.against > 0)
        return fail(FSLBM_E_TOPOLOGY,
                    "%lld cells belong to a liquid film or gas layer thinner than one cell (the interface layer's "
                    "closure would turn a fill >= 1/2 into gas or <= 1/2 into liquid); Sec. II.D calls this unsupported",
                    closure.against);
    fslbm_lattice *h = new (std::nothrow) fslbm_lattice();
    if (!h) return fail(FSLBM_E_STATE, "out of host memory");
    h->nx = nx; h->ny = ny; h->nz = nz;
    h->N = (int)N;
    h->NS = (int)plane_stride(N);
    h->prec = precision;
    h->curv = curv_model;
    h->coll = FSLBM_SRT;
    h->sigma = 0.0; h->tau = 1.0; h->theta = M_PI / 2; h->rho_gas = 1.0;
    h->eps_c = 1e-3; h->trt_magic = 3.0 / 16.0;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char *)workspace;
    {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, workspace) == hipSuccess && attr.device >= 0) {
            h->device = attr.device;
        } else {
            (void)hipGetLastError();
            if (hipGetDevice(&h->device) != hipSuccess) {
                delete h;
                return fail(FSLBM_E_HIP, "cannot determine the device of the workspace");
            }
        }
    }
    h->L = L;
    h->cur = 0;
    h->steps = 0;
    h->version = 0;
    h->epoch = 0;
    h->frozen = 0;
    h->bubble = 0;
    h->strong_wetting = 0;
    h->closure = closure;
    {
        long long nf = N;
        if (obstacle)
            for (long long i = 0; i < N; ++i) nf -= obstacle[i] != 0;
        h->n_free = double(nf);
    }
    batch_init(&h->self);
    h->self.hs.push_back(h);
    h->self.prec = precision;
    h->icount0 = 1 << 20;  // large until counted: the creation's own geometry launch
    h->ocount0 = 1 << 20;
    h->box_blocks = xcd_grid(((long long)N + SC_BLOCK - 1) / SC_BLOCK);
    h->box_cells = N;
    h->boundary_cells = N;
    int rc = dispatch<OpInit>(h, fill, obstacle);
    if (!rc) {
        int ic = 0, oc = 0;
        rc = read_counts(h, ic, oc);
        h->icount0 = ic;
        h->ocount0 = oc;
    }
    if (!rc) rc = refresh_box(h);
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return 0;
}

// Smallest contact angle accepted by default (Sec. II.D): 45 degrees, with a
// margin for the rounding of a converted 45.
constexpr double THETA_MIN = M_PI / 4.0 - 1e-12;

int fslbm_layer_closure(fslbm_t h, int64_t *to_liquid, int64_t *to_gas, double *fill_added, double *fill_removed)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!to_liquid || !to_gas || !fill_added || !fill_removed) return fail(FSLBM_E_ARG, "an output is NULL");
    *to_liquid = h->closure.to_liquid;
    *to_gas = h->closure.to_gas;
    *fill_added = h->closure.fill_added;
    *fill_removed = h->closure.fill_removed;
    return 0;
}

int fslbm_set_params(fslbm_t h, double sigma, double tau, double theta_rad, double rho_gas)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(FSLBM_E_ARG, "sigma must be >= 0");
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(FSLBM_E_ARG, "tau must be > 1/2");
    if (!(theta_rad > 0.0 && theta_rad < M_PI)) return fail(FSLBM_E_ARG, "theta must lie in (0, pi)");
    if (!(rho_gas > 0.0) || !std::isfinite(rho_gas)) return fail(FSLBM_E_ARG, "rho_gas must be > 0");
    if (theta_rad < THETA_MIN && !h->strong_wetting)
        return fail(FSLBM_E_TOPOLOGY,
                    "theta = %.4g deg is below 45 deg: Sec. II.D calls contact angles below 45 deg unsupported "
                    "(FSLBM_OPT_STRONG_WETTING = 1 allows them)",
                    theta_rad * 180.0 / M_PI);
    h->sigma = sigma; h->tau = tau; h->theta = theta_rad; h->rho_gas = rho_gas;
    h->version += 1;
    h->epoch += 1;
    return dispatch<OpGeom>(h);
}

int fslbm_set_option(fslbm_t h, int key, double value)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    switch (key) {
    case FSLBM_OPT_EPS_C:
        if (!(value >= 0.0 && value < 0.5)) return fail(FSLBM_E_ARG, "eps_c must lie in [0, 0.5)");
        h->eps_c = value;
        h->version += 1;
        h->epoch += 1;
        return 0;
    case FSLBM_OPT_COLLISION:
        if (value != FSLBM_SRT && value != FSLBM_TRT) return fail(FSLBM_E_ARG, "collision must be SRT or TRT");
        h->coll = (int)value;
        h->version += 1;
        h->epoch += 1;
        return 0;
    case FSLBM_OPT_TRT_MAGIC:
        if (!(value > 0.0) || !std::isfinite(value)) return fail(FSLBM_E_ARG, "TRT Lambda must be > 0");
        h->trt_magic = value;
        h->version += 1;
        h->epoch += 1;
        return 0;
    case FSLBM_OPT_BUBBLE:
        h->version += 1;
        h->epoch += 1;
        h->bubble = value != 0.0;
        return h->bubble ? dispatch<OpBubble>(h) : 0;
    case FSLBM_OPT_STRONG_WETTING:
        if (value != 0.0 && value != 1.0) return fail(FSLBM_E_ARG, "strong wetting must be 0 or 1");
        if (value == 0.0 && h->theta < THETA_MIN)
            return fail(FSLBM_E_TOPOLOGY, "the current theta is below 45 deg; set theta >= 45 deg first");
        h->strong_wetting = (int)value;
        return 0;
    case FSLBM_OPT_TIMING:
    case FSLBM_OPT_GRAPH:
    case FSLBM_OPT_SPLIT_INTERFACE: return fslbm_batch_set_option(&h->self, key, value);
    default: return fail(FSLBM_E_ARG, "unknown option %d", key);
    }
}

int fslbm_set_stream(fslbm_t h, void *hip_stream)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    const int rc = fold_timing(&h->self);
    if (rc) return rc;
    h->version += 1;
    h->stream = (hipStream_t)hip_stream;
    return 0;
}

int fslbm_set_equilibrium(fslbm_t h, const double *rho, const double *u3)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!rho || !u3) return fail(FSLBM_E_ARG, "rho and u must be given");
    h->epoch += 1;
    return dispatch<OpEq>(h, rho, u3);
}

int fslbm_step(fslbm_t h, int64_t nsteps)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (nsteps < 0) return fail(FSLBM_E_ARG, "nsteps must be >= 0");
    return batch_step(&h->self, nsteps);
}

int fslbm_batch_create(const fslbm_t *handles, int count, fslbm_batch_t *out)
{
    if (!out) return fail(FSLBM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!handles || count < 1 || count > MAXB) return fail(FSLBM_E_ARG, "a batch holds 1..%d lattices", MAXB);
    for (int i = 0; i < count; ++i) {
        if (!handles[i]) return fail(FSLBM_E_ARG, "handle %d is NULL", i);
        if (handles[i]->prec != handles[0]->prec) return fail(FSLBM_E_ARG, "lattices of a batch share the precision");
        if (handles[i]->stream != handles[0]->stream) return fail(FSLBM_E_ARG, "lattices of a batch share the stream");
        if (handles[i]->cur != handles[0]->cur) return fail(FSLBM_E_STATE, "lattices of a batch must be at the same step parity");
        for (int j = 0; j < i; ++j)
            if (handles[j] == handles[i]) return fail(FSLBM_E_ARG, "handle %d appears twice", i);
    }
    fslbm_batch *b = new (std::nothrow) fslbm_batch();
    if (!b) return fail(FSLBM_E_STATE, "out of host memory");
    batch_init(b);
    b->prec = handles[0]->prec;
    for (int i = 0; i < count; ++i) b->hs.push_back(handles[i]);
    *out = b;
    return 0;
}

int fslbm_batch_step(fslbm_batch_t b, int64_t nsteps)
{
    if (!b) return fail(FSLBM_E_STATE, "null batch");
    if (nsteps < 0) return fail(FSLBM_E_ARG, "nsteps must be >= 0");
    for (auto *h : b->hs)
        if (h->stream != b->hs[0]->stream) return fail(FSLBM_E_STATE, "lattices of a batch share the stream");
    return batch_step(b, nsteps);
}

int fslbm_batch_set_option(fslbm_batch_t b, int key, double value)
{
    if (!b) return fail(FSLBM_E_STATE, "null batch");
    switch (key) {
    case FSLBM_OPT_TIMING: return batch_set_timing(b, value != 0.0);
    case FSLBM_OPT_GRAPH:
        b->use_graph = value != 0.0;
        if (!b->use_graph) drop_graphs(b);
        return 0;
    case FSLBM_OPT_SPLIT_INTERFACE:
        if (value != 0.0 && value != 1.0 && value != -1.0) return fail(FSLBM_E_ARG, "split must be 0, 1 or -1");
        b->split_interface = (int)value;
        drop_graphs(b);
        return 0;
    default: return fail(FSLBM_E_ARG, "option %d does not apply to a batch", key);
    }
}

int fslbm_batch_split_active(fslbm_batch_t b, int *active)
{
    if (!b) return fail(FSLBM_E_STATE, "null batch");
    if (!active) return fail(FSLBM_E_ARG, "active is NULL");
    *active = b->split_last;
    return 0;
}

int fslbm_split_active(fslbm_t h, int *active)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    return fslbm_batch_split_active(&h->self, active);
}

int fslbm_batch_read_timing(fslbm_batch_t b, double *phase_ms, int64_t *steps)
{
    if (!b) return fail(FSLBM_E_STATE, "null batch");
    if (!phase_ms || !steps) return fail(FSLBM_E_ARG, "null output");
    HIP_OK(hipStreamSynchronize(bstream(b)));
    const int rc = fold_timing(b);
    if (rc) return rc;
    for (int k = 0; k < NPHASE; ++k) phase_ms[k] = b->tacc[k];
    *steps = b->tsteps;
    return 0;
}

int fslbm_batch_reset_timing(fslbm_batch_t b)
{
    if (!b) return fail(FSLBM_E_STATE, "null batch");
    HIP_OK(hipStreamSynchronize(bstream(b)));
    const int rc = fold_timing(b);
    if (rc) return rc;
    for (int k = 0; k < NPHASE; ++k) b->tacc[k] = 0.0;
    b->tsteps = 0;
    return 0;
}

void fslbm_batch_destroy(fslbm_batch_t b)
{
    if (!b) return;
    (void)hipStreamSynchronize(bstream(b));
    batch_release(b);
    delete b;
}

// After a call that has synchronised the stream anyway, the fluid box is
// read back so that the next steps' grid fits it.
static int then_refresh(fslbm_t h, int rc) { return rc ? rc : refresh_box(h); }

static int read_common(fslbm_t h, int what, double *out, int dev)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!out) return fail(FSLBM_E_ARG, "out is NULL");
    return then_refresh(h, dispatch<OpRead>(h, what, out, dev));
}

int fslbm_read_fill(fslbm_t h, double *out, int d) { return read_common(h, RD_FILL, out, d); }
int fslbm_read_pressure(fslbm_t h, double *out, int d) { return read_common(h, RD_PRESSURE, out, d); }
int fslbm_read_curvature(fslbm_t h, double *out, int d) { return read_common(h, RD_CURV, out, d); }
int fslbm_read_velocity(fslbm_t h, double *out3, int d) { return read_common(h, RD_VEL, out3, d); }
int fslbm_read_normal(fslbm_t h, double *out3, int d) { return read_common(h, RD_NORMAL, out3, d); }
int fslbm_read_plic(fslbm_t h, double *out, int d) { return read_common(h, RD_PLIC, out, d); }
int fslbm_read_mass_field(fslbm_t h, double *out, int d) { return read_common(h, RD_MASS, out, d); }

int fslbm_read_flags(fslbm_t h, uint8_t *out, int out_is_device)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!out) return fail(FSLBM_E_ARG, "out is NULL");
    const int N = h->N;
    uint8_t *flags = (uint8_t *)(h->ws + h->L.flags);
    uint8_t *dst = out_is_device ? out : (uint8_t *)(h->ws + h->L.staging);
    k_read_flags<<<cell_blocks(N), 256, 0, h->stream>>>(flags, dst, N);
    HIP_OK(hipGetLastError());
    if (!out_is_device) HIP_OK(hipMemcpyAsync(out, dst, N, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return refresh_box(h);
}

// Runs the ordered compaction of the interface cells with the given
// scratch and copies the count (and, with out, the list) to the host.
static int read_ilist(fslbm_t h, const ListScratch &s, int32_t *out, int64_t capacity, int64_t *count)
{
    const uint8_t *flags = (const uint8_t *)(h->ws + h->L.flags);
    const DevScalars *sc = (const DevScalars *)(h->ws + h->L.sc);
    k_ilist_count<<<CMP_GRID, 256, 0, h->stream>>>(flags, sc, h->nx, h->ny, s);
    k_ilist_scan<<<1, 1024, 0, h->stream>>>(s, CMP_GRID);
    k_ilist_write<<<CMP_GRID, 256, 0, h->stream>>>(flags, sc, h->nx, h->ny, s);
    HIP_OK(hipGetLastError());
    int n = 0;
    HIP_OK(hipMemcpyAsync(&n, s.total, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    if (n > s.cap)
        return fail(FSLBM_E_SHAPE, "interface list has %d cells; the scratch of this call holds at most %d", n, s.cap);
    *count = n;
    if (!out) return 0;
    if (n > capacity) return fail(FSLBM_E_SHAPE, "interface list has %d entries, capacity %lld", n, (long long)capacity);
    if (n > 0) {
        HIP_OK(hipMemcpyAsync(out, s.list, sizeof(int32_t) * n, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(hipStreamSynchronize(h->stream));
    }
    return 0;
}

int fslbm_read_interface_list(fslbm_t h, int32_t *out, int64_t capacity, int64_t *count)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!count) return fail(FSLBM_E_ARG, "count is NULL");
    // scratch inside the workspace: the compaction counts and the staging area
    char *stg = h->ws + h->L.staging;
    ListScratch s;
    s.counts = (int *)(h->ws + h->L.counts);
    s.total = (int *)stg;
    s.list = (int32_t *)(stg + 256);
    s.cap = h->N;
    return read_ilist(h, s, out, capacity, count);
}

// ------------------------------------------- allocation-free read-out
// Scratch of fslbm_read_interface_list_noalloc: a file-scope device array
// of fixed size (block counts, total, up to NOALLOC_LIST_CAP list entries).
// Every device the library runs on holds its own copy until the process
// ends. Host code never passes the symbol itself to a kernel: it uses the
// per-device address that hipGetSymbolAddress returns on that device.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
constexpr int NOALLOC_LIST_CAP = int((NOALLOC_SCRATCH_BYTES - 2048) / 4);
static_assert(CMP_GRID * sizeof(int) <= 1024, "block counts must fit below the total at byte 1024");
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES];

// Address of `scratch` on device dev, which must be current; looked up once
// per device.
int scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(FSLBM_E_STATE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FSLBM_E_HIP, "hipGetSymbolAddress returned a null address");
        g_scratch[dev] = (char *)p;
    }
    *out = g_scratch[dev];
    return 0;
}
}  // namespace

int fslbm_read_interface_list_noalloc(fslbm_t h, int32_t *out, int64_t capacity, int64_t *count)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!count) return fail(FSLBM_E_ARG, "count is NULL");
    int cur = 0;
    HIP_OK(hipGetDevice(&cur));
    if (cur != h->device) HIP_OK(hipSetDevice(h->device));
    char *base = nullptr;
    int rc = scratch_address(h->device, &base);
    if (!rc) {
        ListScratch s;
        s.counts = (int *)base;  // CMP_GRID ints
        s.total = (int *)(base + 1024);
        s.list = (int32_t *)(base + 2048);
        s.cap = NOALLOC_LIST_CAP;
        rc = read_ilist(h, s, out, capacity, count);
    }
    if (cur != h->device) (void)hipSetDevice(cur);
    return rc;
}

int fslbm_gas_density(fslbm_t h, double *rho_gas)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!rho_gas) return fail(FSLBM_E_ARG, "rho_gas is NULL");
    if (!h->bubble) {
        *rho_gas = h->rho_gas;
        return 0;
    }
    const DevScalars *sc = (const DevScalars *)(h->ws + h->L.sc);
    HIP_OK(hipMemcpyAsync(rho_gas, &sc->rho_gas_t, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    return 0;
}

int fslbm_mass(fslbm_t h, double *total)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!total) return fail(FSLBM_E_ARG, "total is NULL");
    return then_refresh(h, dispatch<OpMass>(h, total));
}

int fslbm_diagnostics(fslbm_t h, double *out)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!out) return fail(FSLBM_E_ARG, "out is NULL");
    return then_refresh(h, dispatch<OpDiag>(h, out));
}

int fslbm_check_numeric(fslbm_t h)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    return then_refresh(h, dispatch<OpCheck>(h));
}

int fslbm_steps_taken(fslbm_t h, int64_t *steps)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!steps) return fail(FSLBM_E_ARG, "steps is NULL");
    *steps = h->steps;
    return 0;
}

int fslbm_read_timing(fslbm_t h, double *phase_ms, int64_t *steps)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    return fslbm_batch_read_timing(&h->self, phase_ms, steps);
}

int fslbm_reset_timing(fslbm_t h)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    return fslbm_batch_reset_timing(&h->self);
}

int fslbm_set_interface_fill(fslbm_t h, const double *fill, int in_is_device)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!fill) return fail(FSLBM_E_ARG, "fill is NULL");
    h->epoch += 1;
    return dispatch<OpFill>(h, fill, in_is_device);
}

int fslbm_state_bytes(fslbm_t h, size_t *bytes)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!bytes) return fail(FSLBM_E_ARG, "bytes is NULL");
    *bytes = state_bytes(h);
    return 0;
}

int fslbm_save_state(fslbm_t h, void *dst, size_t bytes)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!dst) return fail(FSLBM_E_ARG, "dst is NULL");
    if (bytes < state_bytes(h)) return fail(FSLBM_E_SHAPE, "state buffer has %zu bytes, %zu needed", bytes, state_bytes(h));
    StateHeader hd{STATE_MAGIC, h->nx, h->ny, h->nz, h->prec, h->curv, 0, h->steps};
    char *d = (char *)dst;
    HIP_OK(hipMemcpyAsync(d, &hd, sizeof hd, hipMemcpyHostToDevice, h->stream));
    size_t off = 256;
    for (auto &r : state_regions(h)) {
        HIP_OK(hipMemcpyAsync(d + off, h->ws + r.first, r.second, hipMemcpyDeviceToDevice, h->stream));
        off += align256(r.second);
    }
    HIP_OK(hipStreamSynchronize(h->stream));
    return 0;
}

int fslbm_load_state(fslbm_t h, const void *src, size_t bytes)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!src) return fail(FSLBM_E_ARG, "src is NULL");
    if (bytes < state_bytes(h)) return fail(FSLBM_E_SHAPE, "state buffer has %zu bytes, %zu needed", bytes, state_bytes(h));
    StateHeader hd;
    const char *s = (const char *)src;
    HIP_OK(hipMemcpyAsync(&hd, s, sizeof hd, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(hipStreamSynchronize(h->stream));
    if (hd.magic != STATE_MAGIC || hd.nx != h->nx || hd.ny != h->ny || hd.nz != h->nz || hd.prec != h->prec ||
        hd.curv != h->curv)
        return fail(FSLBM_E_ARG, "state buffer does not belong to a lattice of this shape, precision and model");
    size_t off = 256;
    for (auto &r : state_regions(h)) {
        HIP_OK(hipMemcpyAsync(h->ws + r.first, s + off, r.second, hipMemcpyDeviceToDevice, h->stream));
        off += align256(r.second);
    }
    h->steps = hd.steps;
    h->epoch += 1;
    h->version += 1;
    HIP_OK(hipStreamSynchronize(h->stream));
    // the loaded state brings its own obstacle list (launch sizing only)
    int ic = 0, oc = 0;
    const int rc = read_counts(h, ic, oc);
    if (rc) return rc;
    h->ocount0 = oc;
    return refresh_box(h);
}

int fslbm_adjoint_required_bytes(fslbm_t h, int64_t nsteps, int K, size_t *bytes)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!bytes) return fail(FSLBM_E_ARG, "bytes is NULL");
    if (nsteps < 1 || K < 1) return fail(FSLBM_E_ARG, "nsteps and K must be >= 1");
    AdjWindow w;
    const int rc = read_counts(h, w.icount, w.ocount);
    if (rc) return rc;
    w.T = nsteps;
    w.K = K;
    *bytes = adj_layout(w, h);
    return 0;
}

int fslbm_adjoint_forward(fslbm_t h, int64_t nsteps, int K, void *workspace, size_t workspace_bytes)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (nsteps < 1 || K < 1) return fail(FSLBM_E_ARG, "nsteps and K must be >= 1");
    if (!workspace) return fail(FSLBM_E_ARG, "workspace is NULL");
    if (h->bubble) return fail(FSLBM_E_STATE, "the adjoint does not cover the bubble model");
    if (h->curv == FSLBM_CURV_TR) return fail(FSLBM_E_STATE, "the adjoint covers the FD and LSQR models");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(FSLBM_E_ARG, "workspace not 256-byte aligned");
    return dispatch<OpAdjF>(h, (long long)nsteps, K, workspace, workspace_bytes);
}

int fslbm_adjoint_status(fslbm_t h, int64_t *inside_steps, int64_t *fill_events, int64_t *unconverted_steps)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!inside_steps || !fill_events || !unconverted_steps) return fail(FSLBM_E_ARG, "an output is NULL");
    if (!h->adj.recorded) return fail(FSLBM_E_STATE, "no differentiation window recorded");
    *inside_steps = h->adj.inside_steps;
    *fill_events = h->adj.fill_events;
    *unconverted_steps = h->adj.unconverted_steps;
    return 0;
}

int fslbm_adjoint_backward(fslbm_t h, const double *dL_dfill_T, int in_is_device, double *dL_dsigma,
                           double *dL_dtheta, double *dL_dfill_0, int out_is_device)
{
    if (!h) return fail(FSLBM_E_STATE, "null handle");
    if (!dL_dfill_T || !dL_dfill_0) return fail(FSLBM_E_ARG, "dL_dfill_T and dL_dfill_0 must be given");
    const AdjWindow &w = h->adj;
    if (!w.recorded) return fail(FSLBM_E_STATE, "no window recorded (call fslbm_adjoint_forward first)");
    if (h->steps != w.t_end || h->epoch != w.epoch)
        return fail(FSLBM_E_STATE, "the lattice changed since the window was recorded");
    if (h->bubble) return fail(FSLBM_E_STATE, "the adjoint does not cover the bubble model");
    return dispatch<OpAdjB>(h, dL_dfill_T, in_is_device, dL_dsigma, dL_dtheta, dL_dfill_0, out_is_device);
}

void fslbm_destroy(fslbm_t h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    batch_release(&h->self);
    delete h;
}

}  // extern "C"
