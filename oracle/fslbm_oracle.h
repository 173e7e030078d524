/*
 * fslbm_oracle.h -- slow, plain FP64 CPU reference of the free surface
 * lattice Boltzmann time step (Bogner, Ruede, Harting, "Curvature estimation
 * from a volume of fluid indicator function ...", Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the checker of the GPU library:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it. It shares no source, header, table or helper with the GPU path.
 *
 * Fields are dense arrays over nx*ny*nz cells, linear index
 * i = x + nx*(y + ny*z), every axis wraps periodically (walls are explicit
 * obstacle cells). Cell-type codes: 0 gas, 1 liquid, 2 interface, 3 obstacle.
 */
#ifndef FSLBM_ORACLE_H
#define FSLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GAS = 0, ORC_LIQUID = 1, ORC_INTERFACE = 2, ORC_OBSTACLE = 3 };
enum { ORC_CURV_FD = 0, ORC_CURV_LSQR = 1, ORC_CURV_TR = 2 };
enum { ORC_SRT = 0, ORC_TRT = 1 };

typedef struct {
    double sigma;      /* surface tension (lattice units) */
    double tau;        /* relaxation time, nu = (tau - 1/2)/3 */
    double theta;      /* equilibrium contact angle [rad] */
    double rho_gas;    /* gas pressure as a density: p_g = rho_gas / 3 */
    double eps_c;      /* conversion offset of the fill/empty thresholds */
    double trt_magic;  /* TRT Lambda = (tau_e - 1/2)(tau_o - 1/2) */
    int curv_model;    /* ORC_CURV_FD, ORC_CURV_LSQR or ORC_CURV_TR */
    int collision;     /* ORC_SRT or ORC_TRT */
    int frozen;        /* 1: cell types stay fixed (no fill/empty conversion) */
    int bubble;        /* 1: the gas pressure follows the gas volume (one bubble) */
} orc_params;

typedef struct orc_lattice orc_lattice;

/* Build the initial state from fill levels and an obstacle mask (both n
 * cells, copied). Returns NULL on bad arguments. */
orc_lattice *orc_create(int nx, int ny, int nz, const double *fill,
                        const unsigned char *obstacle, const orc_params *p);
void orc_destroy(orc_lattice *L);
void orc_step(orc_lattice *L, long nsteps);

/* Read-outs (n values, 3n component-major for vectors). */
void orc_get_fill(const orc_lattice *L, double *out);
void orc_get_flags(const orc_lattice *L, unsigned char *out);
void orc_get_density(const orc_lattice *L, double *out);
void orc_get_velocity(const orc_lattice *L, double *out3);
void orc_get_curvature(const orc_lattice *L, double *out);
void orc_get_normal(const orc_lattice *L, double *out3);
void orc_get_plic(const orc_lattice *L, double *out);
void orc_get_mass_field(const orc_lattice *L, double *out);
double orc_get_mass(const orc_lattice *L);
double orc_get_reservoir(const orc_lattice *L);
/* Gas density rho_gas(t) of the bubble model (rho_gas when it is off). */
double orc_get_gas_density(const orc_lattice *L);
long orc_interface_list(const orc_lattice *L, int *out);
void orc_get_pdf(const orc_lattice *L, double *out19n);
void orc_set_pdf(orc_lattice *L, const double *in19n);
void orc_set_equilibrium(orc_lattice *L, const double *rho, const double *u3);

/* Building blocks exposed for the pin tests. */
double orc_cut_volume(const double nhat[3], double a);
double orc_plic_offset(const double nhat[3], double phi);
int orc_lsq_solve(int rows, int cols, const double *M, const double *b, double *x);
double orc_quadric_curvature(double A, double B, double C, double H, double I);
int orc_lsqr_fit_points(int npts, const double *pts, const double nhat[3],
                        double *coef5);
/* TR curvature K (= 2 x mean curvature) at a point with unit normal nhat
 * from its neighbours' offsets d (npts x 3, block order). */
double orc_tr_curvature_points(int npts, const double *d, const double nhat[3]);

#ifdef __cplusplus
}
#endif
#endif
