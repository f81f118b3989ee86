/*
 * pulbm_oracle.h -- plain FP64 CPU reference ("the oracle") for the coupled
 * phase-field + P-u lattice Boltzmann time step of Otomo et al.,
 * "Lattice Boltzmann models for the hydrodynamic equations in multiphase flow
 * with high density ratio" (arXiv 2512.01027), Sec. II.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library: only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py use it.  It shares no code, header, table or
 * helper with the HIP library under paper_2512_01027_amd/csrc.
 *
 * Conventions (all host memory, caller-owned, copied on entry/exit):
 *   node index  n = x + nx*(y + ny*z), x fastest; 2D runs use nz = 1;
 *   vector fields are SoA: u[a*N + n] for a in 0..dim-1;
 *   every call returns 0 on success, a negative code on error.
 */
#ifndef PULBM_ORACLE_H
#define PULBM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim, nx, ny, nz;      /* nz = 1 in 2D                                  */
    int32_t q_hydro, q_phase;     /* 2D: 9/9; 3D: hydro 19|27, phase 19|27         */
    int32_t wall[3];              /* per axis: 0 periodic, 1 halfway bounce-back at
                                     both ends, 2 (last axis only) bounce-back at
                                     the low end, pressure p_top at the high end   */
    int32_t delta_theta;          /* 1: apply the anti-rarefaction correction      */
    int32_t collision;            /* hydro collision: 0 filter (Eq. LB_filter_col),
                                     1 BGK (Eq. BGK_LBeq_hydroeq)                  */
    double rho_heavy, rho_light;  /* phi = 1 fluid ("water"), phi = 0 fluid ("air") */
    double nu_heavy, nu_light;    /* kinematic viscosities                         */
    double sigma, W, M;           /* surface tension, interface width, mobility    */
    double lambda_bulk;           /* bulk viscosity (1/6 in the paper)             */
    double gravity[3];            /* body force per unit mass: F_ext = rho * g     */
    int32_t block_lo[3], block_hi[3]; /* solid block, nodes lo <= x < hi per axis;
                                     none when lo >= hi on any axis               */
    double p_top;                 /* pressure of an open high end (wall = 2)       */
} pulbm_oracle_params;

typedef struct {
    double phi_sum, u_sum[3], rhou_sum[3], umax;
    int64_t nonfinite, step;
} pulbm_oracle_diag;

typedef struct pulbm_oracle_case pulbm_oracle_case;

int  pulbm_oracle_create(const pulbm_oracle_params* p, pulbm_oracle_case** out);
void pulbm_oracle_destroy(pulbm_oracle_case* c);
/* Equilibrium initialisation from phi0[N], P0[N], u0[dim*N]. */
int  pulbm_oracle_init_fields(pulbm_oracle_case* c, const double* phi, const double* P,
                              const double* u);
int  pulbm_oracle_step(pulbm_oracle_case* c, int64_t nsteps);
/* Moments of the current state (does not change it). */
int  pulbm_oracle_read_fields(const pulbm_oracle_case* c, double* phi, double* P, double* u);
int  pulbm_oracle_diagnostics(const pulbm_oracle_case* c, pulbm_oracle_diag* d);
/* Raw state: h[q_phase*N], g[q_hydro*N] (post-streaming, oracle direction order)
 * and the pressure of the previous step Plag[N].  Any pointer may be NULL. */
int  pulbm_oracle_get_state(const pulbm_oracle_case* c, double* h, double* g, double* Plag,
                            int64_t* step);
int  pulbm_oracle_set_state(pulbm_oracle_case* c, const double* h, const double* g,
                            const double* Plag, int64_t step);
/* Direction table of a lattice in the oracle's own order: c[3*q], w[q]. */
int  pulbm_oracle_lattice(int dim, int q, int32_t* c, double* w);
/* Node-level equilibria for given local macroscopic values and gradients:
 * gradphi[3], gradrho[3], G[9] (G[3a+b] = d u_a / d x_b).  heq[q_phase], geq[q_hydro]. */
int  pulbm_oracle_node_eq(const pulbm_oracle_params* p, double phi, double P, const double* u,
                          const double* gradphi, double lapphi, const double* gradrho,
                          const double* G, double* heq, double* geq);
/* Isotropic central-difference stencils on the hydro lattice, periodic/ghost rules of the
 * case: grad[3*N] of an even field q[N], lap[N]. */
int  pulbm_oracle_stencil(const pulbm_oracle_case* c, const double* q, double* grad, double* lap);
int  pulbm_oracle_num_threads(void);
/* Threads of the node loops from now on (>= 1); the arithmetic does not depend on it. */
int  pulbm_oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
