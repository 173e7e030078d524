/*
 * fslbm.h -- C ABI of the MI355X (gfx950) free surface lattice Boltzmann
 * library libfslbm.so.
 *
 * The library advances the free surface lattice Boltzmann method (FSLBM) of
 * Bogner, Ruede and Harting, "Curvature estimation from a volume of fluid
 * indicator function for the simulation of surface tension and wetting with a
 * free surface lattice Boltzmann method" (arXiv:1509.07691), Sec. II: D3Q19
 * stream-collide (eqs. lbe1, lbe2), fill-level advection by mass exchange
 * (eqs. advection1, advection2), free-surface reconstruction at gas links with
 * the Laplace pressure jump (eq. reconstruct, rho_b = (p_g + p_s)/c_s^2,
 * p_s = 2 sigma kappa), curvature by finite differences (Sec. II.A, eqs.
 * curvature, normal) or by the least-squares fit of PLIC points with the
 * wetting condition (Sec. II.C, eqs. LSQR-model, LSQR-error, anacurv,
 * contactNormal, contactConstraint), and cell-type conversion.
 *
 * Conventions for every function:
 *  - Return 0 (FSLBM_OK) or a negative FSLBM_E_* code; fslbm_last_error()
 *    then holds a message (per thread). No exception crosses the ABI.
 *  - An argument error leaves the handle unchanged.
 *  - Arrays over the lattice have nx*ny*nz entries with linear index
 *    i = x + nx*(y + ny*z) (x fastest); vector fields are component-major
 *    (all x components, then all y, then all z). All axes wrap periodically;
 *    walls are obstacle cells.
 *  - Ownership: the caller owns every host and device buffer, including the
 *    device workspace handed to fslbm_create; the library keeps raw pointers
 *    into it and never frees them. The library owns only its handle.
 *  - Work is enqueued on the HIP stream given at creation (or by
 *    fslbm_set_stream). fslbm_step does not synchronise; every read function
 *    synchronises that stream before it returns.
 *  - Curvature is reported as K = -div(n) = 2 kappa (2/R for a sphere,
 *    positive for a droplet); the pressure jump is p_s = sigma*K, i.e.
 *    2 sigma kappa with kappa the mean curvature.
 */
#ifndef FSLBM_H
#define FSLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fslbm_lattice *fslbm_t;
typedef struct fslbm_batch *fslbm_batch_t;

enum fslbm_status {
    FSLBM_OK = 0,
    FSLBM_E_ARG = -1,      /* invalid argument value */
    FSLBM_E_SHAPE = -2,    /* lattice or buffer size out of range */
    FSLBM_E_HIP = -3,      /* a HIP runtime call failed */
    FSLBM_E_STATE = -4,    /* handle not usable for this call */
    FSLBM_E_NUMERIC = -5,  /* non-finite or non-positive density found */
    FSLBM_E_TOPOLOGY = -6  /* a configuration the method does not support (Sec. II.D) */
};

/* Storage and arithmetic precision of the distributions. F16/BF16 store
 * (f_q - w_q) * S in 16 bits (S = 2^12 for F16, 1 for BF16) and compute in
 * FP32; m, phi, rho and K are FP64 in F64 mode and FP32 otherwise. In the
 * F32, F16 and BF16 modes the normals, PLIC offsets and FD curvature are
 * computed and stored in FP32 as well; the least-squares normal equations of
 * the LSQR fit and the mass and volume sums are FP64 in every mode. */
enum fslbm_precision { FSLBM_F64 = 0, FSLBM_F32 = 1, FSLBM_F16_STORE = 2, FSLBM_BF16_STORE = 3 };
/* Curvature models: FD (Sec. II.A, mollified finite differences, wetting
 * by the extrapolated contact normal), LSQR (Sec. II.C, least-squares
 * quadric of the PLIC points, wetting by the contact constraint), TR
 * (Sec. II.B, triangle fan of the PLIC points with Taubin's estimate; no
 * wetting, and not covered by the adjoint). */
enum fslbm_curv_model { FSLBM_CURV_FD = 0, FSLBM_CURV_LSQR = 1, FSLBM_CURV_TR = 2 };
enum fslbm_collision { FSLBM_SRT = 0, FSLBM_TRT = 1 };
/* Cell types reported by fslbm_read_flags. */
enum fslbm_cell { FSLBM_GAS = 0, FSLBM_LIQUID = 1, FSLBM_INTERFACE = 2, FSLBM_OBSTACLE = 3 };
/* Keys of fslbm_set_option. */
enum fslbm_option {
    FSLBM_OPT_EPS_C = 0,      /* conversion offset eps: fill if m > (1+eps) rho,
                                 empty if m < -eps rho (default 1e-3) */
    FSLBM_OPT_COLLISION = 1,  /* FSLBM_SRT (default) or FSLBM_TRT */
    FSLBM_OPT_TRT_MAGIC = 2,  /* TRT Lambda = (tau-1/2)(tau_odd-1/2), default 3/16 */
    FSLBM_OPT_TIMING = 3,     /* 1: record HIP events around the phases of every
                                 step (read with fslbm_read_timing), 0: off */
    FSLBM_OPT_GRAPH = 4,      /* 1: replay each step as a captured HIP graph
                                 (ignored while timing is on or on the null
                                 stream), 0: plain launches (default) */
    FSLBM_OPT_SPLIT_INTERFACE = 5, /* 1: two stream-collide passes, a lean one
                                 for liquid cells away from walls and one for
                                 interface and wall-adjacent cells; 0: one pass for all fluid cells; -1
                                 (default): the two passes for the 16-bit
                                 storage forms when interface and wall cells
                                 are under 1/64 of the fluid box, else one.
                                 Results are identical either way. */
    FSLBM_OPT_BUBBLE = 6,     /* 1: bubble model (Sec. III.A.1): the whole gas
                                 of the lattice is one bubble whose pressure
                                 follows its volume isothermally,
                                 rho_gas(t) = rho_gas V0 / V(t), with V the
                                 gas volume (non-obstacle cells minus liquid
                                 cells minus the fill of interface cells) and
                                 V0 its value when the option is set; 0
                                 (default): constant rho_gas. Not covered by
                                 the adjoint (FSLBM_E_STATE there). */
    FSLBM_OPT_STRONG_WETTING = 7 /* 1: accept contact angles below 45 deg,
                                 which Sec. II.D calls unsupported (the
                                 curvature at the contact line then tends to
                                 oscillate); 0 (default): fslbm_set_params
                                 rejects them with FSLBM_E_TOPOLOGY. Setting 0
                                 while theta < 45 deg is FSLBM_E_TOPOLOGY. */
};

/* Device workspace needed for a lattice (bytes, written to *bytes).
 * FSLBM_E_SHAPE if any extent is < 3 or the cell count exceeds 2^31 - 1. */
int fslbm_required_bytes(int nx, int ny, int nz, int precision, size_t *bytes);

/*
 * Create a lattice (Sec. II: fill level and cell types).
 *  fill     host, n doubles: liquid volume fraction per cell. Cell types are
 *           derived as obstacle where obstacle[i] != 0, else liquid for
 *           fill >= 1, gas for fill <= 0, interface otherwise; a liquid cell
 *           with a gas D3Q19 neighbour becomes an interface cell with fill 1.
 *           Then the interface layer is closed (Sec. II.D: an interface cell
 *           has gas and liquid D3Q19 neighbours): interface cells without a
 *           gas neighbour become liquid (fill 1), then those without a
 *           liquid neighbour gas (fill 0). The step keeps this invariant.
 *  obstacle host, n bytes, may be NULL (no walls).
 *  workspace device memory of at least fslbm_required_bytes() bytes, 256-byte
 *           aligned, owned by the caller and kept alive until fslbm_destroy.
 *  hip_stream a hipStream_t (NULL = the null stream).
 * The distributions start at equilibrium with rho = 1, u = 0, the interface
 * mass at m = fill. Parameters start at sigma = 0, tau = 1, theta = pi/2,
 * rho_gas = 1 until fslbm_set_params. Copies fill and obstacle; returns with
 * the initialisation enqueued on the stream. FSLBM_E_ARG for a NULL fill,
 * workspace or out, a misaligned workspace, or an unknown precision or
 * model; FSLBM_E_SHAPE for an extent out of range (as fslbm_required_bytes),
 * a workspace below fslbm_required_bytes(), or, with the FD model, any
 * extent below 10 (its 8^3 tiles read a periodic halo of 3 + 10 cells).
 * The closure rounds each rewritten cell to one phase; FSLBM_E_TOPOLOGY if it
 * would have to round a cell to the phase that fills less than half of it
 * (a fill >= 1/2 closing to gas or <= 1/2 closing to liquid): the input then
 * holds a liquid film or gas layer thinner than one cell, which Sec. II.D
 * (Fig. limitation) calls unsupported. Films thinner than half a cell close
 * to gas without an error; fslbm_layer_closure reports every rewrite.
 * All of these are checked on the host before any device call.
 */
int fslbm_create(int nx, int ny, int nz, int precision, int curv_model, const double *fill,
                 const uint8_t *obstacle, void *workspace, size_t workspace_bytes,
                 void *hip_stream, fslbm_t *out);

/* What the closure of the interface layer did to the input fill at
 * creation: the number of cells closed to liquid (fill set to 1) and to gas
 * (fill set to 0), the fill they gained and the fill they lost (sums over
 * those cells, in cell volumes). FSLBM_E_ARG if an output is NULL. */
int fslbm_layer_closure(fslbm_t h, int64_t *to_liquid, int64_t *to_gas, double *fill_added, double *fill_removed);

/* sigma >= 0 (surface tension, lattice units), tau > 1/2 (relaxation time,
 * nu = (tau - 1/2)/3), 0 < theta < pi (equilibrium contact angle, radians),
 * rho_gas > 0 (gas pressure p_g = rho_gas/3) (Sec. II). Recomputes the
 * curvature field (it depends on theta at walls). FSLBM_E_ARG for a value
 * out of range or not finite; FSLBM_E_TOPOLOGY for theta below 45 degrees,
 * which Sec. II.D calls unsupported, unless FSLBM_OPT_STRONG_WETTING is set.
 * The handle is unchanged on any error. */
int fslbm_set_params(fslbm_t h, double sigma, double tau, double theta_rad, double rho_gas);
/* One option (enum fslbm_option). FSLBM_E_ARG for an unknown key or a value
 * out of its range (eps_c in [0, 0.5), collision SRT or TRT, TRT Lambda > 0). */
int fslbm_set_option(fslbm_t h, int key, double value);
/* Later work of this lattice goes to hip_stream (a hipStream_t; NULL = the
 * null stream). */
int fslbm_set_stream(fslbm_t h, void *hip_stream);

/* Overwrite the distributions of all fluid cells with feq(rho, u) (eq.
 * lbe2's equilibrium; host arrays: rho n doubles, u 3n component-major);
 * interface masses become m = fill * rho. Used to start flows with a
 * prescribed velocity. The values are not checked (fslbm_check_numeric
 * reports a non-positive or non-finite density). FSLBM_E_ARG if rho or u3
 * is NULL. */
int fslbm_set_equilibrium(fslbm_t h, const double *rho, const double *u3);

/* Advance nsteps >= 0 time steps (Sec. II); enqueued, no synchronisation.
 * FSLBM_E_ARG if nsteps < 0. */
int fslbm_step(fslbm_t h, int64_t nsteps);

/* Read-outs (n doubles; 3n for velocity and normal). out_is_device = 1 if
 * out is device memory, 0 for host memory. Synchronise the stream.
 *  fill: phi (1 liquid, 0 gas, m/rho interface, reflected value at walls);
 *  pressure: rho/3 at fluid cells, rho_gas/3 at gas cells, 0 at obstacles;
 *  curvature: K at interface cells, 0 elsewhere;
 *  velocity: u at fluid cells, 0 elsewhere;
 *  normal / plic: unit normal of the raw fill level and (LSQR model only)
 *  PLIC plane offset (point p = cell centre + a n) at interface cells,
 *  0 elsewhere;
 *  mass_field: interface mass m (0 at other cells). */
/* FSLBM_E_ARG if out is NULL. */
int fslbm_read_fill(fslbm_t h, double *out, int out_is_device);
int fslbm_read_pressure(fslbm_t h, double *out, int out_is_device);
int fslbm_read_curvature(fslbm_t h, double *out, int out_is_device);
int fslbm_read_velocity(fslbm_t h, double *out3, int out_is_device);
int fslbm_read_normal(fslbm_t h, double *out3, int out_is_device);
int fslbm_read_plic(fslbm_t h, double *out, int out_is_device);
int fslbm_read_mass_field(fslbm_t h, double *out, int out_is_device);
/* Cell types (enum fslbm_cell), n bytes; FSLBM_E_ARG if out is NULL. */
int fslbm_read_flags(fslbm_t h, uint8_t *out, int out_is_device);
/* Interface cells (Sec. II: cells whose D3Q19 neighbourhood holds both gas
 * and liquid) as ascending linear indices into host out[capacity], found by
 * an ordered compaction of the cell types on the device; *count receives
 * their number (FSLBM_E_SHAPE if it exceeds capacity; out may be NULL to
 * query the count). Uses scratch inside the lattice's workspace and
 * synchronises the stream. FSLBM_E_ARG if count is NULL. */
int fslbm_read_interface_list(fslbm_t h, int32_t *out, int64_t capacity, int64_t *count);
/* The same read-out for callers that cannot allocate device memory (code
 * under graph capture, serving loops, harnesses that forbid hipMalloc): the
 * compaction's scratch (block counts, total and the staged list) lives in a
 * file-scope device array of 16 MiB that each device holds until the
 * process ends, so this call allocates nothing. It holds at most 4,193,792
 * interface cells: a longer list is rejected with FSLBM_E_SHAPE (nothing is
 * copied to out). Every call on a device shares that device's array and
 * leaves its contents behind; calls that overlap on one device (other
 * streams or threads) race and must be serialised by the caller. Arguments,
 * result and other errors as fslbm_read_interface_list. */
int fslbm_read_interface_list_noalloc(fslbm_t h, int32_t *out, int64_t capacity, int64_t *count);
/* Gas density used by the step (rho_gas, or rho_gas(t) of the bubble
 * model); synchronises. FSLBM_E_ARG if rho_gas is NULL. */
int fslbm_gas_density(fslbm_t h, double *rho_gas);
/* Total mass: sum of rho over liquid cells + sum of m over interface cells +
 * excess mass that found no receiving cell; FP64, fixed summation order
 * (the invariant of eqs. advection1/2). Synchronises. FSLBM_E_ARG if total
 * is NULL. */
int fslbm_mass(fslbm_t h, double *total);
/* Diagnostics of the current state: the measures of the paper's
 * equilibrium tests (spurious currents, Laplace law; Sec. III.A.1). FP64
 * device reductions over a fixed partition of the cells in a fixed order, so
 * that calls on the same state agree bit for bit. out is a host array of 4
 * doubles:
 *   out[0]  max |u| over the fluid (liquid and interface) cells,
 *   out[1]  mean |u| over the fluid cells (0 if there are none),
 *   out[2]  the pressure jump (rho_in - rho_gas(t)) / 3, rho_in the mean
 *           density of the inner liquid cells: liquid cells with no gas or
 *           interface cell within a Euclidean distance of 2.5 cells
 *           (periodic). 2 sigma / R for a droplet at equilibrium, minus
 *           that for a bubble; 0 if there are no inner cells,
 *   out[3]  the number of inner liquid cells.
 * u = j / rho as in fslbm_read_velocity. Uses the lattice's reduction
 * scratch (inside its workspace) and synchronises the stream. FSLBM_E_ARG
 * if out is NULL. */
int fslbm_diagnostics(fslbm_t h, double *out);
/* FSLBM_E_NUMERIC if any fluid cell has a non-finite or non-positive
 * density, else 0. Synchronises. */
int fslbm_check_numeric(fslbm_t h);
/* Number of time steps taken since creation. */
int fslbm_steps_taken(fslbm_t h, int64_t *steps);

/* Batches: 1..8 lattices of the same precision, on the same stream and at
 * the same step count, advanced together; each kernel of a step is launched
 * once for all of them (the lattice index is the second grid dimension), so
 * small lattices fill the device and a step is one graph when
 * FSLBM_OPT_GRAPH is set on the batch. The batch holds the handles (not
 * their memory); destroy it before its handles. Stepping a batch advances
 * each lattice exactly as fslbm_step would. Only FSLBM_OPT_TIMING,
 * FSLBM_OPT_GRAPH and FSLBM_OPT_SPLIT_INTERFACE apply to a batch. */
int fslbm_batch_create(const fslbm_t *handles, int count, fslbm_batch_t *out);
int fslbm_batch_step(fslbm_batch_t b, int64_t nsteps);
int fslbm_batch_set_option(fslbm_batch_t b, int key, double value);
int fslbm_batch_read_timing(fslbm_batch_t b, double *phase_ms, int64_t *steps);
/* *active = 1 if the last step of the batch (of the lattice) ran the two
 * stream-collide passes of FSLBM_OPT_SPLIT_INTERFACE, else 0. */
int fslbm_batch_split_active(fslbm_batch_t b, int *active);
int fslbm_split_active(fslbm_t h, int *active);
int fslbm_batch_reset_timing(fslbm_batch_t b);
void fslbm_batch_destroy(fslbm_batch_t b);

/* Accumulated device time (ms) of the five phases of a step while
 * FSLBM_OPT_TIMING is on, phase_ms[5]: [0] stream-collide of liquid cells,
 * [1] stream-collide with mass exchange of interface cells, [2] cell
 * conversion, [3] interface-list compaction, [4] obstacle fill and
 * curvature; *steps receives the number of timed steps. Synchronises. */
int fslbm_read_timing(fslbm_t h, double *phase_ms, int64_t *steps);
int fslbm_reset_timing(fslbm_t h);

/* Set the fill level of the interface cells (cell types unchanged): phi =
 * fill[i] and m = fill[i] * rho at every interface cell i, where rho is the
 * cell's current density; the obstacle fill reflection and the curvature
 * are recomputed (Sec. II.A, II.C). fill holds n doubles (host, or device
 * memory when in_is_device = 1); entries at other cells are ignored. This
 * is the input phi_0 of the differentiation window below. */
int fslbm_set_interface_fill(fslbm_t h, const double *fill, int in_is_device);

/* Checkpoint and resume: the whole lattice state (distributions, cell
 * flags, m, rho, phi, K, normals, PLIC offsets, lists, step count) as an
 * opaque device buffer of fslbm_state_bytes() bytes owned by the caller.
 * fslbm_load_state checks that the buffer was saved from a lattice of the
 * same shape, precision and curvature model (FSLBM_E_ARG otherwise).
 * Both synchronise the stream. */
int fslbm_state_bytes(fslbm_t h, size_t *bytes);
int fslbm_save_state(fslbm_t h, void *dst, size_t bytes);
int fslbm_load_state(fslbm_t h, const void *src, size_t bytes);

/*
 * Differentiation window with frozen cell types (discrete adjoint).
 *
 * fslbm_adjoint_forward advances nsteps >= 1 steps from the current state
 * with the cell types, the interface list and the obstacle list held fixed
 * (no fill / empty conversion), so that the step is a smooth map of
 * (f', m, phi) for given sigma and theta. It stores the state at t = 0, K,
 * 2K, ... and at t = nsteps in `workspace` (device memory of at least
 * fslbm_adjoint_required_bytes() bytes, 256-byte aligned, owned by the
 * caller and kept unchanged until the last backward call; its size depends
 * on the number of interface cells, so query it in the state the window
 * starts from). The lattice ends at the state of step nsteps.
 *
 * fslbm_adjoint_backward takes dL/dphi_T (n doubles, host or device; only
 * interface cells are used: the fill level of liquid and gas cells is
 * constant and the value at obstacle cells is derived) and returns
 *   *dL_dsigma  dL/dsigma (through rho_b = rho_gas + 3 sigma K, Sec. II),
 *   *dL_dtheta  dL/dtheta (radians; through the contact condition of the
 *               LSQR model, eqs. contactNormal, contactConstraint; 0 for FD),
 *   dL_dfill_0  n doubles (host or device): dL/dphi_0 at interface cells for
 *               phi_0 as set by fslbm_set_interface_fill (m_0 = phi_0 rho_0
 *               with the distributions of the window start held fixed),
 *               0 elsewhere.
 * It recomputes each K-step segment from its checkpoint into one of two
 * rings of K-1 states, on a second HIP stream that it creates for the call
 * (default priority) and on a copy of the lattice's fields in the
 * workspace, while the transposed steps of the segment after it run in
 * reverse order on the handle's stream from the other ring; it leaves the
 * lattice at the state of step nsteps, so it may be called again with
 * another dL/dphi_T. FSLBM_E_STATE if no window was recorded or the
 * lattice has been stepped or modified since. Synchronises the stream.
 */
int fslbm_adjoint_required_bytes(fslbm_t h, int64_t nsteps, int K, size_t *bytes);
int fslbm_adjoint_forward(fslbm_t h, int64_t nsteps, int K, void *workspace, size_t workspace_bytes);
int fslbm_adjoint_backward(fslbm_t h, const double *dL_dfill_T, int in_is_device, double *dL_dsigma,
                           double *dL_dtheta, double *dL_dfill_0, int out_is_device);
/* Validity of the recorded window. The frozen step is a smooth map only
 * while every interface fill stays strictly inside (0, 1): at 0 and 1 the
 * PLIC offset is clamped, and near the cell corners its derivative -1/A
 * (A the area of the plane section) diverges. *inside_steps receives the
 * number of window steps before the first step in which an interface fill
 * left (0, 1) (nsteps if none did), *fill_events the number of (step,
 * interface cell) pairs with a fill outside (0, 1), and *unconverted_steps
 * the number of steps before the first step in which the method with free
 * cell types would have filled or emptied a cell (m > (1 + eps) rho or
 * m < -eps rho): up to there the frozen window is the method's own
 * trajectory. Gradients of a window with fill_events > 0 belong to a
 * piecewise-smooth map (each clamped cell contributes the derivative of its
 * clamped piece) and do not describe changes that move a fill across 0 or 1.
 * FSLBM_E_STATE if no window was recorded, FSLBM_E_ARG for a NULL output. */
int fslbm_adjoint_status(fslbm_t h, int64_t *inside_steps, int64_t *fill_events, int64_t *unconverted_steps);

/* Measurement aid: the bound that memory sets for the stream-collide. The
 * streaming half of eq. lbe1 (Sec. II) alone, as a copy: on a periodic
 * nx x ny x nz lattice every cell x writes dst_q(x) = src_q(x - c_q) for the
 * 19 directions, with no collision and no cell types, in the library's
 * distribution layout for `precision` (19 planes, q-major, the plane stride
 * a lattice of that shape uses; elements of 8, 4 or 2 bytes copied as raw
 * bits) and with the grid, chunk order and launch bounds of the bulk
 * stream-collide. src and dst are caller-owned device buffers on the
 * current device, of at least fslbm_pull_copy_bytes() bytes each (the
 * padding between planes is neither read nor written). The call enqueues
 * one untimed and then `launches` (1 .. 100000) timed launches on
 * hip_stream (NULL: the null stream), waits for them, and writes their
 * average duration from HIP events recorded on that stream to
 * *us_per_launch; it moves 38 s N bytes per launch (s the element size,
 * N = nx ny nz). FSLBM_E_ARG for an unknown precision, NULL pointers,
 * src == dst or launches out of range, FSLBM_E_SHAPE for an extent < 3, a
 * cell count above 2^31 - 1 or buffers that are too small, FSLBM_E_HIP if
 * a HIP call fails. */
int fslbm_pull_copy_bytes(int nx, int ny, int nz, int precision, size_t *bytes);
int fslbm_pull_copy_time(int nx, int ny, int nz, int precision, const void *src, void *dst, size_t buffer_bytes,
                         void *hip_stream, int launches, double *us_per_launch);

/* Synchronises the handle's stream and frees the handle (not the caller's
 * workspace). */
void fslbm_destroy(fslbm_t h);
const char *fslbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
