/*
 * lbpf_oracle.h -- plain FP64 CPU oracle for the lattice-Boltzmann phase-field
 * scheme of Cartalade, Younsi & Plapp, "Lattice Boltzmann simulations of 3D
 * crystal growth: numerical schemes for a phase-field model with anti-trapping
 * current" (arXiv:1602.07483).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test-suite, the package's smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no header, table, helper or
 * constant with the GPU library.
 *
 * Storage: every field is a double array [nz][ny][nx] (x fastest); the
 * populations of one field are [Q][nz][ny][nx].
 */
#ifndef LBPF_ORACLE_H
#define LBPF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Walls, one per domain face in the order -x,+x,-y,+y,-z,+z. */
#define ORC_WALL_NOFLUX   0   /* bounce-back, Sec. 3.4 "Algorithm implementation" */
#define ORC_WALL_SYMMETRY 1   /* mirror plane at the half link */

#define ORC_ANISO_CUBIC  0    /* Sec. 2, eq. (Anisotropic-Function_As) */
#define ORC_ANISO_K41K61 1    /* Sec. 4.3, eq. (As_K41-K61) */

typedef struct {
    int32_t nx, ny, nz;
    int32_t lattice;          /* 7, 15 or 19 (Sec. 3.4, Tables 1-2) */
    int32_t wall[6];
    double dx, dt;            /* space and time steps */
    double W0, tau0;          /* interface width, relaxation time scale */
    double lambda, Mcinf;     /* coupling constant, scaled liquidus slope x c_inf */
    double k, D, kappa;       /* partition coefficient, solute and heat diffusivity */
    int32_t aniso;
    double eps, delta;        /* anisotropy strengths */
    double vel[3];            /* uniform advective velocity of the heat equation
                                 (advection-diffusion equilibrium, Sec. 3.1) */
    int32_t skip_theta;       /* 1: isothermal (Sec. 4.2 benchmark): theta is
                                 held at its initial value, the heat equation
                                 is not solved */
    int32_t lattice_ut;       /* lattice of the U and theta schemes (7, 15 or
                                 19); 0: the phase field's.  Sec. 4.1 runs its
                                 2D validation with D2Q9 for phi and D2Q5 for
                                 theta */
    int32_t skip_U;           /* 1: pure substance (M c_inf = 0, where U acts
                                 on nothing): U is held at its initial value,
                                 its scheme is not run */
    int32_t grad_stencil;     /* gradients of phi: 0 = central differences
                                 along the axes (reading R5); 1 = the
                                 isotropic lattice gradient
                                 (e^2 dx)^-1 sum_i w_i e_i phi(x + e_i) over
                                 the phase field's lattice, mirror ghosts */
} orc_params;

typedef struct orc_ctx orc_ctx;

/* Reduction record layout (orc_reduce output, 12 doubles). */
enum {
    ORC_R_SOLID = 0,   /* mean of (1+phi)/2 */
    ORC_R_MASS,        /* sum of zeta(phi)(1+(1-k)U) dx^3 */
    ORC_R_ENTHALPY,    /* sum of (theta - phi/2) dx^3 */
    ORC_R_TIPX, ORC_R_TIPY, ORC_R_TIPZ,   /* phi=0 crossing, lattice units from centre */
    ORC_R_PHIMIN, ORC_R_PHIMAX,
    ORC_R_NONFINITE,
    ORC_R_SUMU,        /* sum of U dx^3 */
    ORC_R_SUMPHI,      /* sum of phi dx^3 */
    ORC_R_COUNT
};

orc_ctx* orc_create(const orc_params* p);
void     orc_destroy(orc_ctx* c);
/* Initial populations = equilibria of the given fields. */
int      orc_init(orc_ctx* c, const double* phi, const double* U, const double* theta);
/* Per-node advective velocity of the heat equation (three arrays of n
 * values, physical units, copied), used instead of p->vel; all three NULL
 * clears it.  Returns 0, or -1 (some but not all NULL, out of memory). */
int      orc_set_velocity_field(orc_ctx* c, const double* vx, const double* vy, const double* vz);
/* nsteps full time steps (phi first, then U and theta). */
int      orc_step(orc_ctx* c, int64_t nsteps);
/* Streaming only (collision = identity), used to check the permutation. */
int      orc_stream_only(orc_ctx* c, int64_t nsteps);
void     orc_fields(const orc_ctx* c, double* phi, double* U, double* theta);
/* field: 0 = g (phi), 1 = h (U), 2 = f (theta) */
void     orc_get_pops(const orc_ctx* c, int field, double* out);
void     orc_set_pops(orc_ctx* c, int field, const double* in);
void     orc_reduce(const orc_ctx* c, const double centre[3], double* out);
int64_t  orc_step_count(const orc_ctx* c);
/* OpenMP threads the oracle's loops use. */
int      orc_num_threads(void);

/* Pieces exposed for the pins. */
int      orc_lattice(int q, int32_t* e /* q*3 */, double* w, double* A, double* B, double* e2);
void     orc_anisotropy(int aniso, double eps, double delta, const double p[3],
                        double* a, double N[3]);
void     orc_geq(int q, double phi, const double N[3], double cphi, double* out);
void     orc_heq(int q, double U, double r, const double J[3], double dt_over_dx, double* out);

#ifdef __cplusplus
}
#endif
#endif
