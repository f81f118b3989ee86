/* Drives every call of the oracle's C interface on small 2D and 3D cases
 * (periodic, walls, open top, solid block, filter and BGK collisions,
 * D3Q27 and D3Q19 hydro) for a few steps.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py: any
 * out-of-bounds access, use after free, leak or undefined operation in the
 * oracle ends the run with a report and a non-zero status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pulbm_oracle.h"

static int run(const pulbm_oracle_params* p, int steps)
{
    pulbm_oracle_case* c = NULL;
    if (pulbm_oracle_create(p, &c) != 0 || !c) return 1;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double* phi = calloc((size_t)N, sizeof(double));
    double* P = calloc((size_t)N, sizeof(double));
    double* u = calloc((size_t)(3 * N), sizeof(double));
    double* h = calloc((size_t)(p->q_phase * N), sizeof(double));
    double* g = calloc((size_t)(p->q_hydro * N), sizeof(double));
    double* Pl = calloc((size_t)N, sizeof(double));
    double* grad = calloc((size_t)(3 * N), sizeof(double));
    double* lap = calloc((size_t)N, sizeof(double));
    int rc = 0;
    /* a droplet of radius n/4 in the middle, moving slowly along x */
    const double R = 0.25 * (p->nx < p->ny ? p->nx : p->ny);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const int64_t n = x + (int64_t)p->nx * (y + (int64_t)p->ny * z);
                const double dx = x + 0.5 - 0.5 * p->nx, dy = y + 0.5 - 0.5 * p->ny;
                const double dz = p->dim == 3 ? z + 0.5 - 0.5 * p->nz : 0.0;
                const double d = sqrt(dx * dx + dy * dy + dz * dz) - R;
                phi[n] = 0.5 - 0.5 * tanh(2.0 * d / p->W);
                u[n] = 0.01 * phi[n];
            }
    rc |= pulbm_oracle_init_fields(c, phi, P, u);
    rc |= pulbm_oracle_step(c, steps);
    rc |= pulbm_oracle_read_fields(c, phi, P, u);
    pulbm_oracle_diag d;
    rc |= pulbm_oracle_diagnostics(c, &d);
    int64_t st = 0;
    rc |= pulbm_oracle_get_state(c, h, g, Pl, &st);
    rc |= pulbm_oracle_set_state(c, h, g, Pl, st);
    rc |= pulbm_oracle_step(c, 1);
    rc |= pulbm_oracle_stencil(c, phi, grad, lap);
    if (!(d.phi_sum == d.phi_sum) || d.nonfinite != 0 || st != steps) rc |= 1;
    free(phi); free(P); free(u); free(h); free(g); free(Pl); free(grad); free(lap);
    pulbm_oracle_destroy(c);
    return rc;
}

static pulbm_oracle_params base(int dim, int nx, int ny, int nz, int qh)
{
    pulbm_oracle_params p;
    memset(&p, 0, sizeof p);
    p.dim = dim; p.nx = nx; p.ny = ny; p.nz = nz;
    p.q_hydro = qh; p.q_phase = dim == 2 ? 9 : 19;
    p.delta_theta = 1;
    p.rho_heavy = 100.0; p.rho_light = 1.0;
    p.nu_heavy = 0.05; p.nu_light = 0.1;
    p.sigma = 1e-3; p.W = 4.0; p.M = 0.166; p.lambda_bulk = 1.0 / 6.0;
    return p;
}

int main(void)
{
    int rc = 0;
    pulbm_oracle_set_num_threads(2);
    pulbm_oracle_params p = base(2, 12, 10, 1, 9);  /* periodic 2D */
    rc |= run(&p, 4);
    p = base(2, 13, 11, 1, 9);                       /* walls, gravity, BGK */
    p.wall[0] = 1; p.wall[1] = 1; p.gravity[1] = -1e-5; p.collision = 1;
    rc |= run(&p, 4);
    p = base(3, 8, 6, 5, 27);                        /* periodic 3D, D3Q27 */
    rc |= run(&p, 3);
    p = base(3, 9, 7, 8, 19);                        /* walls, open top, block, D3Q19 */
    p.wall[0] = 1; p.wall[1] = 1; p.wall[2] = 2; p.gravity[2] = -1e-5;
    p.block_lo[0] = 3; p.block_lo[1] = 2; p.block_lo[2] = 0;
    p.block_hi[0] = 5; p.block_hi[1] = 4; p.block_hi[2] = 3;
    rc |= run(&p, 3);
    int32_t cv[3 * 27];
    double w[27], heq[27], geq[27];
    rc |= pulbm_oracle_lattice(3, 27, cv, w);
    const double u0[3] = {0.01, 0.0, 0.0}, gp[3] = {0.1, 0.0, 0.0}, gr[3] = {1.0, 0.0, 0.0};
    const double G[9] = {0};
    p = base(3, 8, 6, 5, 27);
    rc |= pulbm_oracle_node_eq(&p, 0.5, 0.0, u0, gp, 0.0, gr, G, heq, geq);
    printf("oracle sanitizer run: %s\n", rc ? "FAILED" : "ok");
    return rc ? 1 : 0;
}
