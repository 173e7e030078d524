// Device-side definitions shared by the FSLBM kernels: D3Q19 lattice,
// precision traits, cell flags and the field bundle handed to every kernel.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fslbm {

// ---------------------------------------------------------------- lattice
// D3Q19 (Sec. II): rest, the 6 face and the 12 edge directions. Directions
// 2k-1 and 2k are opposite. Weights 1/3, 1/18, 1/36 (Qian et al. 1992).
constexpr int NQ = 19;
// Components are encoded as bit masks over q (bit q set: component +1 or
// -1), which folds to constants in unrolled loops and stays a few integer
// operations for a run-time q.
constexpr unsigned XP = (1u << 1) | (1u << 7) | (1u << 9) | (1u << 11) | (1u << 13);
constexpr unsigned XM = (1u << 2) | (1u << 8) | (1u << 10) | (1u << 12) | (1u << 14);
constexpr unsigned YP = (1u << 3) | (1u << 7) | (1u << 10) | (1u << 15) | (1u << 17);
constexpr unsigned YM = (1u << 4) | (1u << 8) | (1u << 9) | (1u << 16) | (1u << 18);
constexpr unsigned ZP = (1u << 5) | (1u << 11) | (1u << 14) | (1u << 15) | (1u << 18);
constexpr unsigned ZM = (1u << 6) | (1u << 12) | (1u << 13) | (1u << 16) | (1u << 17);
__host__ __device__ constexpr int dir_x(int q) { return int((XP >> q) & 1u) - int((XM >> q) & 1u); }
__host__ __device__ constexpr int dir_y(int q) { return int((YP >> q) & 1u) - int((YM >> q) & 1u); }
__host__ __device__ constexpr int dir_z(int q) { return int((ZP >> q) & 1u) - int((ZM >> q) & 1u); }
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
__host__ __device__ constexpr int dir_len2(int q)
{
    return dir_x(q) * dir_x(q) + dir_y(q) * dir_y(q) + dir_z(q) * dir_z(q);
}
template <class T>
__host__ __device__ constexpr T weight(int q)
{
    return dir_len2(q) == 0 ? T(1) / T(3) : (dir_len2(q) == 1 ? T(1) / T(18) : T(1) / T(36));
}

// ------------------------------------------------------------- cell flags
// Low nibble: cell type (exactly one bit). Bit 4 (static): the cell has an
// obstacle among its D3Q19 neighbours.
enum : uint8_t {
    FL_GAS = 1,
    FL_LIQ = 2,
    FL_IF = 4,
    FL_OBST = 8,
    FL_TYPE = 15,
    FL_FLUID = FL_LIQ | FL_IF,
    FL_NEAR_OBST = 16,
};
// Conversion status of an interface cell within one step.
// Conversion status of a cell in a step: fills / empties (rules 1-2 of the
// conversion), or leaves the interface layer by its closure (to liquid /
// to gas).
enum : uint8_t { CV_NONE = 0, CV_FILL = 1, CV_EMPTY = 2, CV_CLOSE_LIQ = 3, CV_CLOSE_GAS = 4 };
__host__ __device__ inline bool cv_to_liquid(uint8_t st) { return st == CV_FILL || st == CV_CLOSE_LIQ; }

// ------------------------------------------------------- precision traits
// S: stored type of a distribution, T: arithmetic type of the collide,
// R: type of the scalar fields m, rho, phi, K, normals and PLIC offsets,
// G: arithmetic type of normals, PLIC offsets and FD curvature (the LSQR
// normal equations are always FP64). Shifted storage keeps
// g_q = (f_q - w_q) * SCALE, and the stream-collide of a shifted form works
// on the deviations d_q = f_q - w_q throughout (fslbm_stream.hpp): they are
// O(|u| + |rho - 1|), so FP32 rounds them far more finely than f_q ~ w_q.
// The 16-bit forms round stochastically (store_d).
enum Precision { P_F64 = 0, P_F32 = 1, P_F16 = 2, P_BF16 = 3 };

template <int P> struct Prec;
template <> struct Prec<P_F64> {
    using S = double; using T = double; using R = double; using G = double;
    static constexpr bool SHIFT = false;
    static constexpr double SCALE = 1.0;
};
template <> struct Prec<P_F32> {
    using S = float; using T = float; using R = float; using G = float;
    static constexpr bool SHIFT = true;
    static constexpr double SCALE = 1.0;
};
template <> struct Prec<P_F16> {
    using S = __half; using T = float; using R = float; using G = float;
    static constexpr bool SHIFT = true;
    static constexpr double SCALE = 4096.0;
};
template <> struct Prec<P_BF16> {
    using S = __hip_bfloat16; using T = float; using R = float; using G = float;
    static constexpr bool SHIFT = true;
    static constexpr double SCALE = 1.0;
};

__device__ inline float to_float(float v) { return v; }
__device__ inline float to_float(__half v) { return __half2float(v); }
__device__ inline float to_float(__hip_bfloat16 v) { return __bfloat162float(v); }
// Round-to-nearest-even stores (a truncating conversion would bias the
// stored distributions and show up as mass drift); FP32 is stored as is.
__device__ inline void store_rn(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ inline void store_rn(__half *p, float v) { *p = __float2half_rn(v); }
__device__ inline void store_rn(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }
// Stochastic rounding to 16 bits with gfx950's conversion instructions: the
// top bits of the uniform word `bits` are added below the kept mantissa
// bits and the rest is dropped (13 bits for F16 in its normal range, 16 for
// BF16), so |v| is rounded up with the probability of the dropped fraction
// and the expected stored value is v. Rounding to nearest is exact in
// expectation only for values spread over many quanta; a nearly uniform
// fluid stores the same few values in every cell, the nearest-rounding
// errors then all have one sign, and the total mass drifts by a fixed amount
// every step.
typedef _Float16 fslbm_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 fslbm_bf2 __attribute__((ext_vector_type(2)));
// The 16-bit code of v in the low half of the result. The conversion keeps
// the other half of its destination; only the low half is stored, so the
// destination starts as v's own bits (any value would do; this one needs no
// extra register).
__device__ inline uint32_t sr_code(__half, float v, uint32_t bits)
{
    return __builtin_bit_cast(uint32_t,
                              __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(fslbm_h2, v), v, bits, false));
}
__device__ inline uint32_t sr_code(__hip_bfloat16, float v, uint32_t bits)
{
    return __builtin_bit_cast(uint32_t,
                              __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(fslbm_bf2, v), v, bits, false));
}
__device__ inline void store_sr(float *p, float v, uint32_t) { __builtin_nontemporal_store(v, p); }
// Streaming stores (non-temporal), as FP32: the written planes are not read
// again in the step, and leaving them out of L2 keeps the pulled lines there.
__device__ inline void store_sr(__half *p, float v, uint32_t bits)
{
    __builtin_nontemporal_store((unsigned short)sr_code(__half(), v, bits), (unsigned short *)p);
}
__device__ inline void store_sr(__hip_bfloat16 *p, float v, uint32_t bits)
{
    __builtin_nontemporal_store((unsigned short)sr_code(__hip_bfloat16(), v, bits), (unsigned short *)p);
}

// Counter-based random bits for the stochastic stores: one hash of (cell,
// step) per cell (the low-bias 32-bit integer hash of Wellons' "prospecting
// for hash functions") gives a word s that is uniform over cells and steps,
// and direction q takes s + q phi (phi = 0x9e3779b9, 2^32 times the
// fractional part of the golden ratio: a Weyl sequence). Each direction's
// word is then uniform on its own, which is what makes the stochastic
// rounding unbiased; the 19 words of a cell are spread evenly instead of
// being independent, which changes the spread of the cell's summed rounding
// error but not its mean. One add per direction. Deterministic: a run is
// reproduced bit for bit.
__device__ inline uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ inline uint32_t cell_seed(int i, uint32_t step) { return hash32(uint32_t(i) ^ hash32(step * 0x9e3779b9u)); }
struct SrBits {
    uint32_t s;
    __device__ inline explicit SrBits(uint32_t seed) : s(seed) {}
    // the word for direction q
    __device__ inline uint32_t at(int q) const { return s + uint32_t(q) * 0x9e3779b9u; }
};

// f_q from storage (any form).
template <class P, int Q>
__device__ inline typename P::T load_f(const typename P::S *__restrict__ plane, int i)
{
    using T = typename P::T;
    if constexpr (P::SHIFT) {
        return weight<T>(Q) + to_float(plane[i]) * T(1.0 / P::SCALE);
    } else {
        return plane[i];
    }
}
// Stores f_q (any form; nearest rounding).
template <class P, int Q>
__device__ inline void store_f(typename P::S *__restrict__ plane, int i, typename P::T v)
{
    if constexpr (P::SHIFT) {
        store_rn(plane + i, (v - weight<typename P::T>(Q)) * typename P::T(P::SCALE));
    } else {
        __builtin_nontemporal_store(v, plane + i);
    }
}
// Stored value of a shifted form in the units of the store (d_q SCALE) and
// its inverse, with stochastic rounding in the 16-bit forms. The 16-bit
// forms address a plane with a 32-bit byte offset (a plane of at most
// 2^31 cells), which the loads and stores take as is.
template <class P>
__device__ inline constexpr int scale_log2()
{
    static_assert(P::SCALE == 1.0 || P::SCALE == 4096.0, "power-of-two scales only");
    return P::SCALE == 4096.0 ? 12 : 0;
}
template <class P>
__device__ inline typename P::T load_raw(const typename P::S *__restrict__ plane, int i)
{
    using S = typename P::S;
    if constexpr (sizeof(S) == 2) return to_float(*(const S *)((const char *)plane + uint32_t(i) * 2u));
    else return to_float(plane[i]);
}
// The 16-bit stores go through a buffer resource per plane (base and size
// in scalar registers, the byte offset 2 i the only per-lane operand), so
// the 19 stores need no 64-bit address arithmetic; a store past the plane's
// `plane_cells` is dropped by the hardware.
template <class P>
__device__ inline void store_raw(typename P::S *__restrict__ plane, int i, typename P::T v, uint32_t bits,
                                 int plane_cells)
{
    using S = typename P::S;
    if constexpr (sizeof(S) == 2) {
        // the byte size as an unsigned 32-bit value (a plane of up to 2^31 - 1 cells)
        const __amdgpu_buffer_rsrc_t r =
            __builtin_amdgcn_make_buffer_rsrc(plane, 0, int(uint32_t(plane_cells) * 2u), 0x00020000);
        // cache policy 2: non-temporal, as the global stores of store_sr
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)sr_code(S(), v, bits), r, int(uint32_t(i) * 2u), 0, 2);
    } else {
        store_sr(plane + i, v, bits);
    }
}
// Deviation d_q = f_q - w_q from shifted storage.
template <class P, int Q>
__device__ inline typename P::T load_d(const typename P::S *__restrict__ plane, int i)
{
    static_assert(P::SHIFT, "deviations are stored by the shifted forms only");
    return to_float(plane[i]) * typename P::T(1.0 / P::SCALE);
}
// Stores a deviation d_q into shifted storage (stochastic rounding in the
// 16-bit forms, with the given random bits).
template <class P, int Q>
__device__ inline void store_d(typename P::S *__restrict__ plane, int i, typename P::T d, uint32_t bits)
{
    static_assert(P::SHIFT, "deviations are stored by the shifted forms only");
    store_sr(plane + i, d * typename P::T(P::SCALE), bits);
}

// ------------------------------------------------------ per-step scalars
struct DevScalars {
    int icount;         // number of interface cells in ilist
    int ocount;         // number of obstacle cells in olist (static)
    int nconv;          // interface cells that fill or empty in this step
    int nnew;           // new interface cells of this step (in newlist)
    int nkeep;          // interface cells that stay (rebuilding the list)
    unsigned step;      // completed steps + 1 (conversion tag, never 0)
    // excess mass that found no receiving cell, as a 128-bit fixed-point
    // number res_hi + res_lo 2^-64: integer additions are associative, so
    // the sum does not depend on the order of the atomic updates
    long long res_hi;
    unsigned long long res_lo;
    double mass;        // result of the last mass reduction
    int bad;            // numeric check result
    int wcount;         // number of cells in wlist (static)
    int bbox[6];        // min x, y, z and max x, y, z of the interface cells
    int fbox[6];        // the same for the fluid cells; never shrinks
    double gas_v0;      // bubble model: gas volume when it was switched on
    double rho_gas_t;   // bubble model: gas density rho_gas V0 / V(t)
    int bubble_init;    // 1: the next volume reduction sets gas_v0
    int fill_out;       // frozen window: (step, interface cell) events with a fill outside (0, 1)
    unsigned fill_out_step;  // frozen window: step number of the first such event (UINT_MAX: none)
    unsigned conv_out_step;  // frozen window: step number of the first would-be fill or empty (UINT_MAX: none)
};

// A box of cells [x0, x0+ex) x [y0, y0+ey) x [z0, z0+ez) enumerated with x
// fastest, so consecutive box cells are consecutive in memory along rows and
// the enumeration follows ascending linear index.
struct CellRange {
    int x0, y0, z0, ex, ey, ez;
    __device__ inline int size() const { return ex * ey * ez; }
    __device__ inline int cell(int k, int nx, int ny) const
    {
        const int x = k % ex, r = k / ex, y = r % ey, z = r / ey;
        return (x0 + x) + nx * ((y0 + y) + ny * (z0 + z));
    }
    __device__ static inline CellRange whole(int nx, int ny, int nz) { return {0, 0, 0, nx, ny, nz}; }
    __device__ static inline CellRange from(const int *b)
    {
        if (b[3] < b[0] || b[4] < b[1] || b[5] < b[2]) return {0, 0, 0, 0, 0, 0};
        return {b[0], b[1], b[2], b[3] - b[0] + 1, b[4] - b[1] + 1, b[5] - b[2] + 1};
    }
};

// XCD-aware order of the 256-cell chunks of a one-shot grid. The hardware
// hands workgroups to the 8 XCDs in turn (workgroup b to XCD b mod 8), and
// each XCD has its own L2. The x-shifted pulls of a chunk read one cache
// line of every such plane that the neighbouring chunk also reads; with
// chunk = b that neighbour runs on another XCD and the line is fetched from
// HBM twice (about 1/8 more reads in FP32, 1/4 in the 16-bit forms, over
// the 10 directions with c_x != 0). Here `run` consecutive chunks go to one
// XCD, so only one chunk boundary in `run` crosses XCDs, and successive
// runs go to successive XCDs, so the blocks in flight still cover one
// narrow window of the box. Measured on the 512^3 probe: the 16-bit lean
// pass gains 6 % with runs of 8 (2.02 -> 1.89 ms); FP32 does not gain and
// runs of 4 or 8 slow it by 5-25 % (the access pattern across HBM channels
// changes), so it keeps runs of 1. The host rounds such grids up to a
// multiple of XCD_GRID (so that blockIdx.y does not shift the XCD of a
// block); the map is a bijection of [0, gridDim.x).
constexpr int XCDS = 8, XCD_GRID = 64;
// Cells per block (one chunk) of the bulk stream-collide over the box.
// Measured on the 512^3 probe and the droplet workloads: 512 is equal on
// the probe and 10-15 % slower on droplets, 1024 slower everywhere.
constexpr int SC_BLOCK = 256;
template <class P>
__host__ __device__ constexpr int xcd_run()
{
    return sizeof(typename P::S) == 2 ? 8 : 1;
}
__host__ __device__ inline int xcd_chunk(int b, int grid, int run)
{
    const int period = XCDS * run;
    if (b >= grid / period * period) return b;
    return b / period * period + (b % XCDS) * run + (b / XCDS) % run;
}
__host__ inline int xcd_grid(long long chunks)
{
    const long long g = (chunks + XCD_GRID - 1) / XCD_GRID * XCD_GRID;
    return (int)std::max<long long>(XCD_GRID, g);
}

// Contiguous share [k0, k1) of n items for block blockIdx.x of gridDim.x,
// in whole 256-item strides.
__device__ inline void block_share(int n, int &k0, int &k1)
{
    const int strides = (n + 255) / 256;
    const int per = (strides + gridDim.x - 1) / gridDim.x;
    k0 = min(n, (int)blockIdx.x * per * 256);
    k1 = min(n, k0 + per * 256);
}

// Adds x to the fixed-point reservoir. |x| = a + b 2^-64 with a = floor|x|
// and b the first 64 bits of the fraction (|x| - floor|x| is exact in FP64
// and scaling by 2^64 is exact; bits below 2^-64 are dropped); a negative x
// adds the two's complement. The carry out of the low word is taken from
// the value its atomic returns, so concurrent additions in any order give
// the same 128-bit sum.
__device__ inline void reservoir_add(DevScalars *sc, double x)
{
    const double ax = fabs(x);
    const double a = floor(ax);
    unsigned long long lo = (unsigned long long)((ax - a) * 18446744073709551616.0);
    long long hi = (long long)a;
    if (x < 0.0) {
        hi = -hi - (lo != 0ull ? 1 : 0);
        lo = ~lo + 1ull;
    }
    const unsigned long long old = atomicAdd(&sc->res_lo, lo);
    const long long carry = old + lo < old ? 1 : 0;
    if (hi + carry != 0) atomicAdd((unsigned long long *)&sc->res_hi, (unsigned long long)(hi + carry));
}
__host__ __device__ inline double reservoir_value(long long hi, unsigned long long lo)
{
    return double(hi) + double(lo) * 5.421010862427522e-20;  // 2^-64
}

// Closes a time step's device bookkeeping (conversion counters, the step
// number that tags new cells). The first geometry launch of a step does it,
// by thread 0 of block (0, lattice), when asked; no kernel of that launch
// reads these counters.
__device__ inline void end_of_step(DevScalars *sc, int eos)
{
    if (eos && blockIdx.x == 0 && threadIdx.x == 0) {
        sc->nconv = 0;
        sc->nnew = 0;
        sc->step += 1;
    }
}

// Model parameters (Sec. II): rho_b = 3 (p_g + sigma K), p_g = rho_gas / 3.
struct Params {
    double sigma;
    double tau;
    double omega;      // 1/tau
    double omega_odd;  // TRT odd rate
    double cos_theta, sin_theta;
    double rho_gas;
    double eps_c;
    int curv;          // 0 FD, 1 LSQR
    int coll;          // 0 SRT, 1 TRT
    int frozen;        // 1: cell types stay fixed (no fill / empty conversion)
    int bubble;        // 1: the gas pressure follows the gas volume (one bubble)
    double n_free;     // number of non-obstacle cells
};

// Gas density of the reconstruction: rho_gas, or the bubble model's
// rho_gas V0 / V(t) (Sec. III.A.1).
__device__ inline double gas_density(const Params &p, const DevScalars *sc)
{
    return p.bubble ? sc->rho_gas_t : p.rho_gas;
}

template <class P> struct Fields {
    using S = typename P::S;
    using R = typename P::R;
    const S *fsrc;     // f'(t), 19 planes of N cells, NS elements apart
    S *fdst;           // f'(t+1)
    uint8_t *flags;
    uint8_t *conv;
    uint8_t *near;  // low byte of the step number when within 2 cells of a filling or emptying cell
    uint32_t *mark;
    R *m, *rho, *phi, *K, *nrm, *plic, *share, *phis, *nmol;
    R *cnrm;           // FD wetting: contact normal of obstacle cells (3 planes, 0 = none)
    int32_t *ilist, *olist;
    int32_t *wlist;    // static: non-obstacle cells with an obstacle D3Q19 neighbour
    int32_t *newlist, *ilist_tmp;  // new interface cells; scratch for the list rebuild
    int *counts;       // per-block counts of the list compaction
    double *part;      // per-block partial sums of reductions
    DevScalars *sc;
    // when set (the recompute steps of the reverse sweep, LSQR model): the
    // step's end state of the interface-list entries (SNAP values each: m,
    // rho, phi, K, n, PLIC offset) and the obstacle-list fill levels after
    // them, written by the kernels that finish those values
    R *snap;
    int nx, ny, nz;
    int N;
    int NS;            // plane stride of the distribution buffers (elements, >= N)
};
constexpr int SNAP = 8;

// Up to MAXB lattices advanced by one launch per kernel: lattice b is
// handled by the blocks with blockIdx.y == b. Passed by value as the kernel
// argument (about 1.8 KB), so no device-side descriptor memory is needed.
constexpr int MAXB = 8;
template <class P> struct Batch {
    Fields<P> f[MAXB];
    Params p[MAXB];
};

// Periodic neighbour offsets of one cell: index of (x+dx, y+dy, z+dz) is
// ox[dx+1] + oy[dy+1] + oz[dz+1].
struct Nbr {
    int ox[3], oy[3], oz[3];
    int x, y, z;
    __device__ inline Nbr(int i, int nx, int ny, int nz)
    {
        const int yz = i / nx;
        const int zz = yz / ny;
        set(i - yz * nx, yz - zz * ny, zz, nx, ny, nz);
    }
    __device__ inline Nbr(int x_, int y_, int z_, int nx, int ny, int nz) { set(x_, y_, z_, nx, ny, nz); }
    __device__ inline void set(int x_, int y_, int z_, int nx, int ny, int nz)
    {
        x = x_;
        y = y_;
        z = z_;
        const int nxy = nx * ny;
        ox[0] = x == 0 ? nx - 1 : x - 1; ox[1] = x; ox[2] = x == nx - 1 ? 0 : x + 1;
        // the wrapped row and plane offsets as sums around y nx and z nx ny
        // (a product of a selected index would be multiplied out by the
        // compiler for each of the nine (dy, dz) combinations)
        const int ry = y * nx, wy = nxy - nx, rz = z * nxy, wz = nxy * (nz - 1);
        oy[0] = y == 0 ? ry + wy : ry - nx; oy[1] = ry; oy[2] = y == ny - 1 ? ry - wy : ry + nx;
        oz[0] = z == 0 ? rz + wz : rz - nxy; oz[1] = rz; oz[2] = z == nz - 1 ? rz - wz : rz + nxy;
    }
    __device__ inline int at(int dx, int dy, int dz) const
    {
        return ox[dx + 1] + oy[dy + 1] + oz[dz + 1];
    }
};

}  // namespace fslbm
