/*
 * pulbm_oracle.c -- plain FP64 CPU reference ("the oracle") of the coupled
 * phase-field + P-u lattice Boltzmann time step (Otomo et al., arXiv 2512.01027,
 * Sec. II "Lattice Boltzmann models").
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  The product path never links or calls it.
 *
 * The code follows the paper's equations in the paper's order, one node at a
 * time, with plain loops: no blocking, no fusion, no algebraic shortcuts.  In
 * particular K_i, the omega term and Pi are evaluated exactly as written (no
 * compact form), and streaming is a plain push into a second buffer.
 *
 * Readings of points the paper leaves open:
 *  R1  one LKS pass with no iteration, in the order the paper writes the two
 *      formulas.  The pressure equation holds P on both sides (through K_i);
 *      its one evaluation starts from the pressure the streamed populations
 *      carry, P* = rho_ref T sum_i g_i: P from K_i of P* and, in the omega
 *      term, the velocity the populations carry, u* = sum_i g_i c_i, at
 *      x - c_i; then u = sum_i (g_i + K_i) c_i with K_i of the new P.  rho in
 *      K_i is the current rho(x).  Starting from the previous step's P instead
 *      couples pressure and velocity by forward Euler and is unstable in the
 *      light fluid below nu ~ 5e-3; from P* the scheme stays stable to
 *      nu ~ 1e-3.
 *  R2  rho, tau and omega use phi clamped to [0,1]; theta, mu, h^eq use raw phi.
 *  R3  the velocity moment sums g_i + K_i (the paper's f_i is read as g_i).
 *  R4  nu in B and sigma_lm is the local T(tau_mix - 1/2).
 *  R5  the delta-theta switch is s = lap(phi)/(|lap(phi)| + eps).
 *  R6  the phase-field LBE is BGK with tau_phi = M/T + 1/2.
 *  R7  every finite-difference stencil and the K_i / omega sums use the hydro
 *      lattice (D2Q9 in 2D, D3Q27 or D3Q19 in 3D).
 *  R8  F_ext = rho * g.
 *  R9  no half-force shift: u is the literal sum.
 *  R10 initial distributions are the equilibria of (phi0, P0, u0); lagged P = P0.
 *  R11 walls: halfway bounce-back; a population reflected at a wall keeps the
 *      body/surface force part of its equilibrium (g_ibar(x) = g*_i(x)
 *      - 2 w_i c_i.F/(rho T)); ghost values one node outside a wall mirror the
 *      nearest fluid node: phi, rho even, u odd (no slip at the half link),
 *      u* odd in its flow part and even in its body-force part,
 *      P extrapolated hydrostatically P(m) + rho(x) g.(ghost - m).
 *  R12 phi = 1 is the heavy fluid; rho_ref = rho_light.
 *  R15 solid block (the dam-break obstacle of Sec. III): its nodes carry no
 *      fluid.  A link from a fluid node into the block bounces back as at a
 *      wall (R11).  A stencil value at a block node mirrors it across each
 *      of its faces that is exposed to fluid (a face node across one, an edge
 *      node across two, a corner node across three), with the parities and
 *      the hydrostatic pressure of R11 counted once per face crossed.
 *  R16 open top at fixed pressure (the dam break's atmospheric top, Sec. III;
 *      the paper gives no scheme): beyond the high end of the last axis,
 *      phi, rho, u and u* take the value of the nearest node (zero normal
 *      gradient) and the pressure the value 2 p_top - P(m), so that P is
 *      p_top on the boundary half a link out.  A hydrodynamic population
 *      leaving through the top is gone, and the opposite one entering the top
 *      node is that node's own equilibrium g^eq of the step.  The phase field
 *      is closed there (h bounces back as at a wall): phi's mass stays exact,
 *      and the sharpening flux theta n of the air side (with delta theta on
 *      wherever phi > 0) cannot pump phi in through the boundary.
 */
#include "pulbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Lattice temperature T (Sec. II, D3Q19 with T = 1/3). */
static const double T = 1.0 / 3.0;
/* epsilon of the interface normal (Sec. II). */
static const double EPS = 1.0e-10;
/* Constants of the delta-theta correction (Sec. II, after Eq. theta). */
static const double GAMMA_DT = -22.5, PHI_N = 0.8, PHI_M = 0.2, D_DT = 1.0e-4;

typedef struct {
    int dim, q, rest;
    int c[27][3];
    double w[27];
    int opp[27];
} lattice;

typedef struct {
    pulbm_oracle_params p;
    lattice G;  /* hydro lattice */
    lattice H;  /* phase-field lattice */
    double tau_a, tau_w, tau_phi, omega_max;
} model;

struct pulbm_oracle_case {
    model m;
    int n[3];
    size_t N;
    double *h, *g;       /* post-streaming distributions [q][N] */
    double *hn, *gn;     /* streaming targets */
    double *Plag;        /* P of the previous moment stage (restart image; the step
                            reads the pressure the populations carry instead) */
    double *J;           /* velocity moment of the populations (work array) */
    double *Ps;          /* pressure the populations carry, rho_ref T sum g (work) */
    double *phi, *rho, *P, *u;
    unsigned char* solid; /* 1 at nodes of the block (R15) */
    int64_t step;
};

/* ---------------------------------------------------------------- lattices */

/* Velocity sets with components in {-1,0,1}; weights by squared speed:
 * D2Q9 {4/9, 1/9, 1/36}, D3Q19 {1/3, 1/18, 1/36}, D3Q27 {8/27, 2/27, 1/54, 1/216}. */
static int build_lattice(lattice* L, int dim, int q)
{
    double wc[4];
    int maxn2;
    if (dim == 2 && q == 9) {
        wc[0] = 4.0 / 9.0; wc[1] = 1.0 / 9.0; wc[2] = 1.0 / 36.0; wc[3] = 0.0; maxn2 = 2;
    } else if (dim == 3 && q == 19) {
        wc[0] = 1.0 / 3.0; wc[1] = 1.0 / 18.0; wc[2] = 1.0 / 36.0; wc[3] = 0.0; maxn2 = 2;
    } else if (dim == 3 && q == 27) {
        wc[0] = 8.0 / 27.0; wc[1] = 2.0 / 27.0; wc[2] = 1.0 / 54.0; wc[3] = 1.0 / 216.0; maxn2 = 3;
    } else {
        return -1;
    }
    int n = 0;
    int zr = dim == 3 ? 1 : 0;
    for (int cz = -zr; cz <= zr; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                int n2 = cx * cx + cy * cy + cz * cz;
                if (n2 > maxn2) continue;
                L->c[n][0] = cx;
                L->c[n][1] = cy;
                L->c[n][2] = cz;
                L->w[n] = wc[n2];
                if (n2 == 0) L->rest = n;
                ++n;
            }
    L->dim = dim;
    L->q = n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
                L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    return n == q ? 0 : -1;
}

static int model_init(model* m, const pulbm_oracle_params* p)
{
    if (p->dim != 2 && p->dim != 3) return -1;
    if (p->dim == 2 && (p->q_hydro != 9 || p->q_phase != 9)) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || (p->dim == 2 && p->nz != 1)) return -1;
    if (!(p->rho_heavy > 0) || !(p->rho_light > 0) || !(p->W > 0) || !(p->M > 0)) return -1;
    if (!(p->nu_heavy > 0) || !(p->nu_light > 0) || p->rho_heavy == p->rho_light) return -1;
    if (p->collision != 0 && p->collision != 1) return -1;
    const int nn[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a) {
        if (p->wall[a] < 0 || p->wall[a] > 2) return -1;
        if (p->wall[a] == 2 && a != p->dim - 1) return -1;  /* open end: last axis only */
    }
    int has_block = 1;
    for (int a = 0; a < 3; ++a)
        if (p->block_lo[a] >= p->block_hi[a]) has_block = 0;
    if (has_block) {
        for (int a = 0; a < 3; ++a) {
            int lo = p->block_lo[a], hi = p->block_hi[a];
            int full = lo == 0 && hi == nn[a];
            if (lo < 0 || hi > nn[a]) return -1;
            if (!full && hi - lo < 2) return -1;  /* faces on both sides need 2 layers */
            if (!full && !p->wall[a] && (lo < 1 || hi > nn[a] - 1)) return -1;  /* no wrap */
            if (p->wall[a] == 2 && hi == nn[a]) return -1;  /* clear of the open end */
        }
    }
    if (build_lattice(&m->G, p->dim, p->q_hydro)) return -1;
    if (build_lattice(&m->H, p->dim, p->q_phase)) return -1;
    m->p = *p;
    /* tau from nu (Sec. II, Eq. tau_interpolate and below); tau_phi from the
     * phase-field LBE denominator M/T + 0.5. */
    m->tau_a = p->nu_light / T + 0.5;
    m->tau_w = p->nu_heavy / T + 0.5;
    m->tau_phi = p->M / T + 0.5;
    /* No LKS iterations: omega_max = rho_water / rho_air. */
    m->omega_max = p->rho_heavy / p->rho_light;
    return 0;
}

/* ------------------------------------------------------------ node access */

static size_t idx3(const pulbm_oracle_case* C, const int x[3])
{
    return (size_t)x[0] + (size_t)C->n[0] * ((size_t)x[1] + (size_t)C->n[1] * (size_t)x[2]);
}

static int in_block(const pulbm_oracle_case* C, const int m[3])
{
    const int32_t *lo = C->m.p.block_lo, *hi = C->m.p.block_hi;
    for (int a = 0; a < 3; ++a)
        if (lo[a] >= hi[a] || m[a] < lo[a] || m[a] >= hi[a]) return 0;
    return 1;
}

/* Target of displacement d from node x.  Periodic axes wrap.  On a wall axis a
 * target outside the box is a ghost: its mirror m is the nearest fluid node on
 * that axis and off = ghost - m.  A target in the solid block is mirrored
 * across each exposed face it lies on (R15).  Returns the number of walls and
 * block faces crossed; *open (if given) is set when the target lies beyond an
 * open top (R16), which is not counted as a crossing. */
static int resolve(const pulbm_oracle_case* C, const int x[3], const int d[3], int m[3], int off[3],
                   int* open)
{
    int crossed = 0;
    if (open) *open = 0;
    for (int a = 0; a < 3; ++a) {
        int t = x[a] + d[a], n = C->n[a];
        off[a] = 0;
        if (t < 0 || t >= n) {
            if (C->m.p.wall[a]) {
                int mm = t < 0 ? 0 : n - 1;
                off[a] = t - mm;
                if (C->m.p.wall[a] == 2 && t >= n) {
                    if (open) *open = 1;
                } else {
                    ++crossed;
                }
                t = mm;
            } else {
                t = ((t % n) + n) % n;
            }
        }
        m[a] = t;
    }
    if (in_block(C, m)) {
        const int32_t *lo = C->m.p.block_lo, *hi = C->m.p.block_hi;
        int r[3] = {m[0], m[1], m[2]};
        for (int a = 0; a < 3; ++a) {
            if (m[a] == lo[a] && lo[a] >= 1) {
                r[a] = lo[a] - 1;
                ++crossed;
            } else if (m[a] == hi[a] - 1 && hi[a] <= C->n[a] - 1) {
                r[a] = hi[a];
                ++crossed;
            }
            off[a] += m[a] - r[a];
        }
        for (int a = 0; a < 3; ++a) m[a] = r[a];
    }
    return crossed;
}

/* Even field (phi, rho): a ghost takes the mirror value. */
static double even_at(const pulbm_oracle_case* C, const double* f, const int x[3], const int d[3])
{
    int m[3], off[3];
    resolve(C, x, d, m, off, NULL);
    return f[idx3(C, m)];
}

/* Velocity component: a ghost takes the mirror value with the sign flipped once
 * per wall crossed (zero velocity on the half-link wall). */
static double odd_at(const pulbm_oracle_case* C, const double* f, const int x[3], const int d[3])
{
    int m[3], off[3];
    int k = resolve(C, x, d, m, off, NULL);
    double v = f[idx3(C, m)];
    return (k & 1) ? -v : v;
}

/* Pressure: a ghost is extrapolated hydrostatically from its mirror; beyond
 * an open top it is 2 p_top - P(m) (R16). */
static double pres_at(const pulbm_oracle_case* C, const double* P, const int x[3], const int d[3],
                      double rho_x)
{
    int m[3], off[3], open;
    int k = resolve(C, x, d, m, off, &open);
    double v = P[idx3(C, m)];
    if (open) return 2.0 * C->m.p.p_top - v;
    if (k) {
        const double* gv = C->m.p.gravity;
        v += rho_x * (gv[0] * off[0] + gv[1] * off[1] + gv[2] * off[2]);
    }
    return v;
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* rho, tau linear in the clamped order parameter (Eq. tau_interpolate; R2). */
static void phase_props(const model* M, double phi, double* rho, double* tau)
{
    double pc = clamp01(phi);
    *rho = M->p.rho_light + pc * (M->p.rho_heavy - M->p.rho_light);
    *tau = M->tau_a + pc * (M->tau_w - M->tau_a);
}

/* ------------------------------------------------------ moment stage (M1-M5) */

/* K_i = w_i / (T rho) [P(x - c_i) - P(x)]  (Eq. Kiterm). */
static double k_term(const pulbm_oracle_case* C, const double* Pf, const int x[3], int i, double r)
{
    const lattice* G = &C->m.G;
    int d[3] = {-G->c[i][0], -G->c[i][1], -G->c[i][2]};
    return G->w[i] / (T * r) * (pres_at(C, Pf, x, d, r) - Pf[idx3(C, x)]);
}

/* Velocity carried by the populations, u* = sum_i g_i c_i, at a ghost node: the
 * flow part is mirrored oddly (no slip at the half-link wall) and the
 * body-force part g of the populations' momentum evenly. */
static double ustar_at(const pulbm_oracle_case* C, const double* J, int a, const int x[3],
                       const int d[3])
{
    int m[3], off[3];
    int k = resolve(C, x, d, m, off, NULL);
    double v = J[(size_t)a * C->N + idx3(C, m)];
    if (k & 1) v = -v + 2.0 * C->m.p.gravity[a];
    return v;
}

/* phi = sum h; P and u from the pressure and velocity formulas of Sec. II,
 * one LKS pass without iteration (reading R1), in the order the paper writes
 * them: P first, with K_i of the pressure the populations carry,
 * P* = rho_ref T sum g, and, in the omega term, the velocity they carry,
 * u* = sum g c, at x - c_i; then u = sum (g_i + K_i) c_i with K_i of the new
 * pressure. */
static void moments(const pulbm_oracle_case* C, double* phi, double* rho, double* P, double* u)
{
    const model* M = &C->m;
    const lattice* G = &M->G;
    const lattice* H = &M->H;
    const int dim = M->p.dim;
    const double ra = M->p.rho_light, rw = M->p.rho_heavy;
    const size_t N = C->N;
    double* J = C->J;
    double* Ps = C->Ps;
    /* pass 1: phi, rho, u*, P*; block nodes hold no fluid (phi = 0, u = 0,
     * P = 0) */
#pragma omp parallel for schedule(static)
    for (size_t n = 0; n < N; ++n) {
        if (C->solid[n]) {
            phi[n] = 0.0;
            rho[n] = ra;
            P[n] = 0.0;
            Ps[n] = 0.0;
            for (int a = 0; a < 3; ++a) {
                J[(size_t)a * N + n] = 0.0;
                if (a < dim) u[(size_t)a * N + n] = 0.0;
            }
            continue;
        }
        double ph = 0.0;
        for (int j = 0; j < H->q; ++j) ph += C->h[(size_t)j * N + n];
        double r, tau;
        phase_props(M, ph, &r, &tau);
        phi[n] = ph;
        rho[n] = r;
        for (int a = 0; a < dim; ++a) {
            double s = 0.0;
            for (int i = 0; i < G->q; ++i) s += C->g[(size_t)i * N + n] * G->c[i][a];
            J[(size_t)a * N + n] = s;
        }
        double sg = 0.0;
        for (int i = 0; i < G->q; ++i) sg += C->g[(size_t)i * N + n];
        Ps[n] = ra * T * sg;
    }
    /* pass 2: P */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < C->n[2]; ++z)
        for (int y = 0; y < C->n[1]; ++y)
            for (int xx = 0; xx < C->n[0]; ++xx) {
                int x[3] = {xx, y, z};
                size_t n = idx3(C, x);
                if (C->solid[n]) continue;
                double r = rho[n];
                double omega = (r - ra) / (rw - ra) * (M->omega_max - 1.0);
                double s1 = 0.0, s2 = 0.0;
                for (int i = 0; i < G->q; ++i) {
                    int d[3] = {-G->c[i][0], -G->c[i][1], -G->c[i][2]};
                    double K = k_term(C, Ps, x, i, r);
                    s1 += C->g[(size_t)i * N + n] + (1.0 + omega) * K;
                    double cu = 0.0;
                    for (int a = 0; a < dim; ++a) cu += G->c[i][a] * ustar_at(C, J, a, x, d);
                    s2 += G->w[i] * cu;
                }
                P[n] = ra * T * s1 + omega * ra * s2;
            }
    /* pass 3: u with K_i of the new pressure */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < C->n[2]; ++z)
        for (int y = 0; y < C->n[1]; ++y)
            for (int xx = 0; xx < C->n[0]; ++xx) {
                int x[3] = {xx, y, z};
                size_t n = idx3(C, x);
                if (C->solid[n]) continue;
                double uu[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < G->q; ++i) {
                    double K = k_term(C, P, x, i, rho[n]);
                    for (int a = 0; a < dim; ++a) uu[a] += (C->g[(size_t)i * N + n] + K) * G->c[i][a];
                }
                for (int a = 0; a < dim; ++a) u[(size_t)a * N + n] = uu[a];
            }
}

/* ------------------------------------------------- equilibria (C2-C4) */

typedef struct {
    double phi, P, u[3], gradphi[3], lapphi, gradrho[3], G[9];
} nodevals;

static double ramp(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* h^eq with the delta-theta correction, and g^eq of the hydrodynamic LBE.
 * Also returns F, rho and tau_mix of the node. */
static void equilibria(const model* M, const nodevals* v, double* heq, double* geq, double F[3],
                       double* rho_out, double* tau_out)
{
    const pulbm_oracle_params* p = &M->p;
    const lattice* G = &M->G;
    const lattice* H = &M->H;
    const int dim = p->dim;
    const double phi = v->phi;

    /* --- phase field: n, theta (+ delta theta), Gamma, h^eq --- */
    double gp2 = 0.0;
    for (int a = 0; a < dim; ++a) gp2 += v->gradphi[a] * v->gradphi[a];
    double gnorm = sqrt(gp2);
    double nvec[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) nvec[a] = v->gradphi[a] / (gnorm + EPS);
    double theta = (p->M / T) * (1.0 - 4.0 * (phi - 0.5) * (phi - 0.5)) / p->W;
    if (p->delta_theta) {
        double s = v->lapphi / (fabs(v->lapphi) + EPS);
        double Y1 = fmin(ramp((phi - PHI_N) / D_DT), ramp(-(phi - 1.0) / D_DT));
        double Y2 = fmin(ramp(phi / D_DT), ramp(-(phi - PHI_M) / D_DT));
        theta += GAMMA_DT * (p->M / (T * p->W)) * gnorm * ((1.0 + s) * Y1 + (1.0 - s) * Y2);
    }
    double u2 = 0.0;
    for (int a = 0; a < dim; ++a) u2 += v->u[a] * v->u[a];
    for (int j = 0; j < H->q; ++j) {
        double cu = 0.0, cn = 0.0;
        for (int a = 0; a < dim; ++a) {
            cu += H->c[j][a] * v->u[a];
            cn += H->c[j][a] * nvec[a];
        }
        double Gam = H->w[j] * (1.0 + cu / T + cu * cu / (2.0 * T * T) - u2 / (2.0 * T));
        heq[j] = phi * Gam + theta * H->w[j] * cn;
    }

    /* --- hydrodynamics: rho, tau, nu, mu, F, sigma, B, g^eq --- */
    double rho, tau;
    phase_props(M, phi, &rho, &tau);
    double nu = T * (tau - 0.5);
    double mu = (48.0 * p->sigma / p->W) * phi * (phi - 1.0) * (phi - 0.5) -
                (3.0 * p->sigma * p->W / 2.0) * v->lapphi;
    for (int a = 0; a < 3; ++a) F[a] = 0.0;
    for (int a = 0; a < dim; ++a) F[a] = rho * p->gravity[a] + mu * v->gradphi[a];
    double div = 0.0;
    for (int a = 0; a < dim; ++a) div += v->G[3 * a + a];
    double sig[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            sig[a][b] = 0.0;
            if (a < dim && b < dim) {
                sig[a][b] = rho * nu * (v->G[3 * a + b] + v->G[3 * b + a]);
                if (a == b) sig[a][b] += rho * (2.0 / 3.0) * (p->lambda_bulk - nu) * div;
            }
        }
    double B = (2.0 / 3.0) * (nu - p->lambda_bulk) + T / 2.0;
    for (int i = 0; i < G->q; ++i) {
        const double w = G->w[i];
        const double dst = (i == G->rest) ? 1.0 : 0.0;
        double cu = 0.0, cF = 0.0, csd = 0.0;
        for (int a = 0; a < dim; ++a) {
            cu += G->c[i][a] * v->u[a];
            cF += G->c[i][a] * F[a];
        }
        for (int l = 0; l < dim; ++l)
            for (int m = 0; m < dim; ++m) csd += G->c[i][l] * sig[l][m] * v->gradrho[m];
        double Gam = w * (1.0 + cu / T + cu * cu / (2.0 * T * T) - u2 / (2.0 * T));
        geq[i] = v->P / (p->rho_light * T) * dst + Gam - w + w * cF / (rho * T) +
                 B * (w - dst) / T * div + w * csd / (rho * rho * T);
    }
    *rho_out = rho;
    *tau_out = tau;
}

/* Central-difference gradient and Laplacian on the hydro lattice (Sec. II,
 * the two stencil formulas after Eq. tau_interpolate).  kind 0 = even field,
 * 1 = velocity component (odd ghosts). */
static void grad_lap(const pulbm_oracle_case* C, const double* f, int kind, const int x[3],
                     double grad[3], double* lap)
{
    const lattice* G = &C->m.G;
    const int dim = C->m.p.dim;
    double g3[3] = {0.0, 0.0, 0.0}, l = 0.0;
    double f0 = f[idx3(C, x)];
    for (int i = 0; i < G->q; ++i) {
        int dp[3] = {G->c[i][0], G->c[i][1], G->c[i][2]};
        int dm[3] = {-G->c[i][0], -G->c[i][1], -G->c[i][2]};
        double fp = kind ? odd_at(C, f, x, dp) : even_at(C, f, x, dp);
        double fm = kind ? odd_at(C, f, x, dm) : even_at(C, f, x, dm);
        for (int a = 0; a < dim; ++a) g3[a] += (fp - fm) * G->c[i][a] * G->w[i];
        l += (fp - f0) * G->w[i];
    }
    for (int a = 0; a < 3; ++a) grad[a] = a < dim ? g3[a] / (2.0 * T) : 0.0;
    if (lap) *lap = 2.0 * l / T;
}

/* Stencils (C1) at node x from the current phi, rho, u fields. */
static void node_values(const pulbm_oracle_case* C, const int x[3], nodevals* v)
{
    const int dim = C->m.p.dim;
    const size_t N = C->N;
    size_t n = idx3(C, x);
    v->phi = C->phi[n];
    v->P = C->P[n];
    for (int a = 0; a < 3; ++a) v->u[a] = a < dim ? C->u[(size_t)a * N + n] : 0.0;
    grad_lap(C, C->phi, 0, x, v->gradphi, &v->lapphi);
    grad_lap(C, C->rho, 0, x, v->gradrho, NULL);
    for (int a = 0; a < 9; ++a) v->G[a] = 0.0;
    for (int a = 0; a < dim; ++a) {
        double gr[3];
        grad_lap(C, C->u + (size_t)a * N, 1, x, gr, NULL);
        for (int b = 0; b < dim; ++b) v->G[3 * a + b] = gr[b];
    }
}

/* ------------------------------------------ collision + streaming (C1-C5, S) */

static void collide_stream(pulbm_oracle_case* C)
{
    const model* M = &C->m;
    const lattice* G = &M->G;
    const lattice* H = &M->H;
    const int dim = M->p.dim;
    const size_t N = C->N;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < C->n[2]; ++z)
        for (int y = 0; y < C->n[1]; ++y)
            for (int xx = 0; xx < C->n[0]; ++xx) {
                int x[3] = {xx, y, z};
                size_t n = idx3(C, x);
                if (C->solid[n]) continue;
                nodevals v;
                node_values(C, x, &v);
                double heq[27], geq[27], F[3], rho, tau;
                equilibria(M, &v, heq, geq, F, &rho, &tau);
                /* Phase field BGK (Eq. LB_phi_filter_col). */
                double hs[27];
                for (int j = 0; j < H->q; ++j) {
                    double hj = C->h[(size_t)j * N + n];
                    hs[j] = hj - (hj - heq[j]) / M->tau_phi;
                }
                /* Filter collision (Eq. LB_filter_col): Pi from Eq. momentum_flux,
                 * Phi_i from Eq. momentum_flux0; or the BGK collision of
                 * Eq. BGK_LBeq_hydroeq with tau_mix. */
                double gs[27];
                if (M->p.collision == 1) {
                    for (int i = 0; i < G->q; ++i) {
                        double gi = C->g[(size_t)i * N + n];
                        gs[i] = gi - (gi - geq[i]) / tau;
                    }
                } else {
                double Pi[3][3] = {{0}};
                for (int k = 0; k < G->q; ++k) {
                    double ne = C->g[(size_t)k * N + n] - geq[k];
                    for (int a = 0; a < dim; ++a)
                        for (int b = 0; b < dim; ++b) Pi[a][b] += G->c[k][a] * G->c[k][b] * ne;
                }
                for (int i = 0; i < G->q; ++i) {
                    double phipi = 0.0;
                    for (int a = 0; a < dim; ++a)
                        for (int b = 0; b < dim; ++b) {
                            double phab = G->w[i] / (2.0 * T * T) *
                                          (G->c[i][a] * G->c[i][b] - (a == b ? T : 0.0));
                            phipi += phab * Pi[a][b];
                        }
                    gs[i] = geq[i] + (1.0 - 1.0 / tau) * phipi;
                }
                }
                /* Streaming: push to x + c; at a wall or the block, reflect into
                 * the opposite slot; through an open top, h reflects (no phi
                 * crosses it) and the opposite g slot takes this node's
                 * equilibrium (R16). */
                for (int j = 0; j < H->q; ++j) {
                    int m[3], off[3], open;
                    int k = resolve(C, x, H->c[j], m, off, &open);
                    if (k || open)
                        C->hn[(size_t)H->opp[j] * N + n] = hs[j];
                    else
                        C->hn[(size_t)j * N + idx3(C, m)] = hs[j];
                }
                for (int i = 0; i < G->q; ++i) {
                    int m[3], off[3], open;
                    int k = resolve(C, x, G->c[i], m, off, &open);
                    if (open) {
                        C->gn[(size_t)G->opp[i] * N + n] = geq[G->opp[i]];
                    } else if (k) {
                        double cF = 0.0;
                        for (int a = 0; a < dim; ++a) cF += G->c[i][a] * F[a];
                        C->gn[(size_t)G->opp[i] * N + n] = gs[i] - 2.0 * G->w[i] * cF / (rho * T);
                    } else {
                        C->gn[(size_t)i * N + idx3(C, m)] = gs[i];
                    }
                }
            }
}

/* ----------------------------------------------------------------- public */

int pulbm_oracle_create(const pulbm_oracle_params* p, pulbm_oracle_case** out)
{
    if (!p || !out) return -1;
    *out = NULL;
    pulbm_oracle_case* C = (pulbm_oracle_case*)calloc(1, sizeof(*C));
    if (!C) return -2;
    if (model_init(&C->m, p)) {
        free(C);
        return -1;
    }
    C->n[0] = p->nx;
    C->n[1] = p->ny;
    C->n[2] = p->nz;
    C->N = (size_t)p->nx * p->ny * p->nz;
    size_t N = C->N;
    int qh = C->m.H.q, qg = C->m.G.q;
    C->h = (double*)calloc((size_t)qh * N, sizeof(double));
    C->hn = (double*)calloc((size_t)qh * N, sizeof(double));
    C->g = (double*)calloc((size_t)qg * N, sizeof(double));
    C->gn = (double*)calloc((size_t)qg * N, sizeof(double));
    C->Plag = (double*)calloc(N, sizeof(double));
    C->J = (double*)calloc(3 * N, sizeof(double));
    C->Ps = (double*)calloc(N, sizeof(double));
    C->phi = (double*)calloc(N, sizeof(double));
    C->rho = (double*)calloc(N, sizeof(double));
    C->P = (double*)calloc(N, sizeof(double));
    C->u = (double*)calloc(3 * N, sizeof(double));
    C->solid = (unsigned char*)calloc(N, 1);
    if (!C->h || !C->hn || !C->g || !C->gn || !C->Plag || !C->J || !C->Ps || !C->phi || !C->rho ||
        !C->P || !C->u || !C->solid) {
        pulbm_oracle_destroy(C);
        return -2;
    }
    for (int z = 0; z < C->n[2]; ++z)
        for (int y = 0; y < C->n[1]; ++y)
            for (int xx = 0; xx < C->n[0]; ++xx) {
                int x[3] = {xx, y, z};
                C->solid[idx3(C, x)] = (unsigned char)in_block(C, x);
            }
    *out = C;
    return 0;
}

void pulbm_oracle_destroy(pulbm_oracle_case* C)
{
    if (!C) return;
    free(C->h);
    free(C->hn);
    free(C->g);
    free(C->gn);
    free(C->Plag);
    free(C->J);
    free(C->Ps);
    free(C->phi);
    free(C->rho);
    free(C->P);
    free(C->u);
    free(C->solid);
    free(C);
}

/* Initial distributions are the equilibria (Sec. I, below Eq. feq_expansion). */
int pulbm_oracle_init_fields(pulbm_oracle_case* C, const double* phi, const double* P,
                             const double* u)
{
    if (!C || !phi || !P || !u) return -1;
    const model* M = &C->m;
    const int dim = M->p.dim;
    const size_t N = C->N;
    for (size_t n = 0; n < N; ++n) {
        double tau;
        const int s = C->solid[n];
        C->phi[n] = s ? 0.0 : phi[n];
        phase_props(M, C->phi[n], &C->rho[n], &tau);
        C->P[n] = s ? 0.0 : P[n];
        C->Plag[n] = C->P[n];
    }
    memset(C->u, 0, 3 * N * sizeof(double));
    for (int a = 0; a < dim; ++a)
        for (size_t n = 0; n < N; ++n) C->u[(size_t)a * N + n] = C->solid[n] ? 0.0 : u[(size_t)a * N + n];
    for (int z = 0; z < C->n[2]; ++z)
        for (int y = 0; y < C->n[1]; ++y)
            for (int xx = 0; xx < C->n[0]; ++xx) {
                int x[3] = {xx, y, z};
                size_t n = idx3(C, x);
                if (C->solid[n]) {  /* block nodes hold no populations */
                    for (int j = 0; j < M->H.q; ++j) C->h[(size_t)j * N + n] = 0.0;
                    for (int i = 0; i < M->G.q; ++i) C->g[(size_t)i * N + n] = 0.0;
                    continue;
                }
                nodevals v;
                node_values(C, x, &v);
                double heq[27], geq[27], F[3], rho, tau;
                equilibria(M, &v, heq, geq, F, &rho, &tau);
                for (int j = 0; j < M->H.q; ++j) C->h[(size_t)j * N + n] = heq[j];
                for (int i = 0; i < M->G.q; ++i) C->g[(size_t)i * N + n] = geq[i];
            }
    C->step = 0;
    return 0;
}

int pulbm_oracle_step(pulbm_oracle_case* C, int64_t nsteps)
{
    if (!C || nsteps < 0) return -1;
    const size_t N = C->N;
    for (int64_t s = 0; s < nsteps; ++s) {
        moments(C, C->phi, C->rho, C->P, C->u);
        collide_stream(C);
        double* t = C->h; C->h = C->hn; C->hn = t;
        t = C->g; C->g = C->gn; C->gn = t;
        memcpy(C->Plag, C->P, N * sizeof(double));
        C->step += 1;
    }
    return 0;
}

int pulbm_oracle_read_fields(const pulbm_oracle_case* C, double* phi, double* P, double* u)
{
    if (!C) return -1;
    const size_t N = C->N;
    double* wphi = (double*)malloc(N * sizeof(double));
    double* wrho = (double*)malloc(N * sizeof(double));
    double* wP = (double*)malloc(N * sizeof(double));
    double* wu = (double*)calloc(3 * N, sizeof(double));
    if (!wphi || !wrho || !wP || !wu) {
        free(wphi); free(wrho); free(wP); free(wu);
        return -2;
    }
    moments(C, wphi, wrho, wP, wu);
    if (phi) memcpy(phi, wphi, N * sizeof(double));
    if (P) memcpy(P, wP, N * sizeof(double));
    if (u) memcpy(u, wu, (size_t)C->m.p.dim * N * sizeof(double));
    free(wphi); free(wrho); free(wP); free(wu);
    return 0;
}

int pulbm_oracle_diagnostics(const pulbm_oracle_case* C, pulbm_oracle_diag* d)
{
    if (!C || !d) return -1;
    const size_t N = C->N;
    const int dim = C->m.p.dim;
    double* wphi = (double*)malloc(N * sizeof(double));
    double* wrho = (double*)malloc(N * sizeof(double));
    double* wP = (double*)malloc(N * sizeof(double));
    double* wu = (double*)calloc(3 * N, sizeof(double));
    if (!wphi || !wrho || !wP || !wu) {
        free(wphi); free(wrho); free(wP); free(wu);
        return -2;
    }
    moments(C, wphi, wrho, wP, wu);
    memset(d, 0, sizeof(*d));
    for (size_t n = 0; n < N; ++n) {
        int bad = !isfinite(wphi[n]) || !isfinite(wP[n]);
        double um2 = 0.0;
        d->phi_sum += wphi[n];
        for (int a = 0; a < dim; ++a) {
            double ua = wu[(size_t)a * N + n];
            bad |= !isfinite(ua);
            d->u_sum[a] += ua;
            d->rhou_sum[a] += wrho[n] * ua;
            um2 += ua * ua;
        }
        if (sqrt(um2) > d->umax) d->umax = sqrt(um2);
        d->nonfinite += bad;
    }
    d->step = C->step;
    free(wphi); free(wrho); free(wP); free(wu);
    return 0;
}

int pulbm_oracle_get_state(const pulbm_oracle_case* C, double* h, double* g, double* Plag,
                           int64_t* step)
{
    if (!C) return -1;
    const size_t N = C->N;
    if (h) memcpy(h, C->h, (size_t)C->m.H.q * N * sizeof(double));
    if (g) memcpy(g, C->g, (size_t)C->m.G.q * N * sizeof(double));
    if (Plag) memcpy(Plag, C->Plag, N * sizeof(double));
    if (step) *step = C->step;
    return 0;
}

int pulbm_oracle_set_state(pulbm_oracle_case* C, const double* h, const double* g,
                           const double* Plag, int64_t step)
{
    if (!C || !h || !g || !Plag) return -1;
    const size_t N = C->N;
    memcpy(C->h, h, (size_t)C->m.H.q * N * sizeof(double));
    memcpy(C->g, g, (size_t)C->m.G.q * N * sizeof(double));
    memcpy(C->Plag, Plag, N * sizeof(double));
    C->step = step;
    return 0;
}

int pulbm_oracle_lattice(int dim, int q, int32_t* c, double* w)
{
    lattice L;
    if (build_lattice(&L, dim, q)) return -1;
    for (int i = 0; i < L.q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        w[i] = L.w[i];
    }
    return 0;
}

int pulbm_oracle_node_eq(const pulbm_oracle_params* p, double phi, double P, const double* u,
                         const double* gradphi, double lapphi, const double* gradrho,
                         const double* G, double* heq, double* geq)
{
    model M;
    if (!p || model_init(&M, p)) return -1;
    nodevals v;
    v.phi = phi;
    v.P = P;
    v.lapphi = lapphi;
    for (int a = 0; a < 3; ++a) {
        v.u[a] = u[a];
        v.gradphi[a] = gradphi[a];
        v.gradrho[a] = gradrho[a];
    }
    for (int a = 0; a < 9; ++a) v.G[a] = G[a];
    double F[3], rho, tau;
    equilibria(&M, &v, heq, geq, F, &rho, &tau);
    return 0;
}

int pulbm_oracle_stencil(const pulbm_oracle_case* C, const double* q, double* grad, double* lap)
{
    if (!C || !q) return -1;
    const size_t N = C->N;
    for (int z = 0; z < C->n[2]; ++z)
        for (int y = 0; y < C->n[1]; ++y)
            for (int xx = 0; xx < C->n[0]; ++xx) {
                int x[3] = {xx, y, z};
                size_t n = idx3(C, x);
                double gr[3], l;
                grad_lap(C, q, 0, x, gr, &l);
                if (grad)
                    for (int a = 0; a < 3; ++a) grad[(size_t)a * N + n] = gr[a];
                if (lap) lap[n] = l;
            }
    return 0;
}

int pulbm_oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int pulbm_oracle_set_num_threads(int n)
{
    if (n < 1) return -1;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return 0;
}
