// Kernels of the coupled phase-field + P-u lattice Boltzmann step
// (Otomo et al., arXiv 2512.01027, Sec. II) for gfx950.
//
// One time step is three launches over every resident case:
//   k_moments  per node, no halo: gathers h and g (AA pattern), writes
//              phi = sum h, u* = sum g c, S = rho_ref T sum g (without the
//              pressure carried by the rest population) and M2 = sum g c c.
//   k_pressure 1-halo LDS tile, FP64 arithmetic: the pressure formula of
//              Sec. II with K_i of the previous-step pressure and, in the
//              omega term, u* at x - c_i.
//   k_collide  LDS tiles (P with a 2-node halo, phi and u* with 1): rebuilds
//              u = u* + sum K_i c_i with the new P, takes the isotropic
//              central differences of phi, rho and u, applies the BGK
//              phase-field collision and the filter collision of the
//              hydrodynamic LBE, and writes back in place (AA pattern).
//
// Memory layout (per case): structure of arrays, x fastest; population i of
// node n at f[i*N + n].  AA pattern: on even steps node x reads slot i of x
// and writes its post-collision f*_i to slot opp(i) of x; on odd steps it reads
// slot opp(i) of x - c_i and writes slot i of x + c_i.  Each node reads and
// writes the same set of slots within a step, so the update is in place with
// no race.  Halfway bounce-back: a population that would leave through a
// wall is written to the slot the node itself reads as the reflected
// direction next step.
//
// The rest population of g is stored as g_0 - P/(rho_ref T): the pressure
// (kept separately as state) never passes through the distribution storage,
// and k_moments needs no pressure at all.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "codec.hpp"
#include "lattice.hpp"

namespace pulbm {

// Per-case descriptor, resident in device memory (one per case of a launch).
struct CaseDev {
    int32_t nx, ny, nz, dim;
    int32_t wall[3];
    int32_t ntx, nty, ntz;  // tiles per axis
    int32_t delta_theta;
    int32_t pad0;
    int64_t N;
    int64_t step;      // steps done
    int64_t step_end;  // the case is advanced while step < step_end
    void* h;           // Q_h * N populations (storage type)
    void* g;           // Q_g * N populations (storage type)
    void* P[2];        // pressure ping-pong: P[step & 1] is the previous-step pressure
    void* phi;         // N      scratch (aux type)
    void* J;           // dim*N  scratch: u* = sum g c
    void* S;           // N      scratch: rho_ref T (sum g without the pressure part)
    void* M2;          // 3 (2D) or 6 (3D) * N scratch: sum g c c
    void* U;           // dim*N  velocity written by a read pass
    double rho_a, rho_w, tau_a, tau_w, tau_phi, M, W, sigma, lambda_b;
    double grav[3];
    double h_scale, h_inv_scale, g_scale, g_inv_scale, phi_ref;
};

// --------------------------------------------------------------- launch map

// Blocks are dealt to the 8 XCDs round-robin; remapping gives each XCD one
// contiguous run of tiles, so tiles that share halo planes share an L2.
// The grid is a multiple of 8.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ int find_case(const int* __restrict__ tstart, int ncases, int tile)
{
    int lo = 0, hi = ncases - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tstart[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct TileCtx {
    int ci;          // case index
    int ox, oy, oz;  // tile origin
    int64_t step;
    bool active;
};

// A launch covers the tiles of every case in a table of case pointers;
// tstart[c] is the first tile of case c.
using CaseTab = CaseDev* const* __restrict__;

template <class Mo>
__device__ __forceinline__ TileCtx tile_ctx(CaseTab cases, const int* __restrict__ tstart,
                                            int ncases, int total_tiles, int step_off)
{
    TileCtx t;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    t.active = tile < total_tiles;
    if (!t.active) return t;
    t.ci = find_case(tstart, ncases, tile);
    const CaseDev& cs = *cases[t.ci];
    t.step = cs.step + step_off;
    t.active = t.step < cs.step_end;
    int lt = tile - tstart[t.ci];
    const int tx = lt % cs.ntx;
    lt /= cs.ntx;
    const int ty = lt % cs.nty;
    const int tz = lt / cs.nty;
    t.ox = tx * Mo::TX;
    t.oy = ty * Mo::TY;
    t.oz = tz * Mo::TZ;
    return t;
}

// Neighbour navigation of one node: linear offsets of a -1/0/+1 step along
// each axis (periodic wrap included) and which steps leave through a wall.
struct Nav {
    int64_t o[3][3];
    uint32_t solid;  // bit 2a: the -1 step on axis a is outside a wall; bit 2a+1: the +1 step
};

__device__ __forceinline__ Nav make_nav(const CaseDev& cs, int x, int y, int z)
{
    Nav v;
    const int p[3] = {x, y, z};
    const int n[3] = {cs.nx, cs.ny, cs.nz};
    const int64_t st[3] = {1, (int64_t)cs.nx, (int64_t)cs.nx * cs.ny};
    v.solid = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.o[a][1] = 0;
        v.o[a][0] = (p[a] == 0) ? (int64_t)(n[a] - 1) * st[a] : -st[a];
        v.o[a][2] = (p[a] == n[a] - 1) ? -(int64_t)(n[a] - 1) * st[a] : st[a];
        if (cs.wall[a]) {
            if (p[a] == 0) v.solid |= 1u << (2 * a);
            if (p[a] == n[a] - 1) v.solid |= 1u << (2 * a + 1);
        }
    }
    return v;
}

template <class L>
__device__ __forceinline__ int64_t nav_off(const Nav& v, int i, int sgn)
{
    return v.o[0][sgn * L::c(i, 0) + 1] + v.o[1][sgn * L::c(i, 1) + 1] + v.o[2][sgn * L::c(i, 2) + 1];
}

template <class L>
__device__ __forceinline__ bool nav_solid(const Nav& v, int i, int sgn)
{
    bool s = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int ca = sgn * L::c(i, a);
        if (ca == -1) s |= (v.solid >> (2 * a)) & 1u;
        if (ca == 1) s |= (v.solid >> (2 * a + 1)) & 1u;
    }
    return s;
}

// Where the population arriving at node n along direction i is stored.
template <class L>
__device__ __forceinline__ int64_t aa_src(const Nav& v, int64_t N, int64_t n, int i, bool odd)
{
    if (!odd) return (int64_t)i * N + n;
    if (nav_solid<L>(v, i, -1)) return (int64_t)i * N + n;  // reflected at the wall last step
    return (int64_t)opp(i) * N + n + nav_off<L>(v, i, -1);
}

// Where node n writes its post-collision population i; *bb tells whether it
// is reflected by a wall (and needs the force correction for g).
template <class L>
__device__ __forceinline__ int64_t aa_dst(const Nav& v, int64_t N, int64_t n, int i, bool odd, bool* bb)
{
    *bb = nav_solid<L>(v, i, +1);
    if (!odd || *bb) return (int64_t)opp(i) * N + n;
    return (int64_t)i * N + n + nav_off<L>(v, i, +1);
}

// ---------------------------------------------------------- tile regions

// Resolve global coordinate t on an axis of n nodes: periodic wrap, or the
// mirror node of a ghost outside a wall (off = t - mirror).
__device__ __forceinline__ int resolve_axis(int t, int n, int wall, int* off, int* crossed)
{
    *off = 0;
    if (t >= 0 && t < n) return t;
    if (wall) {
        const int m = t < 0 ? 0 : n - 1;
        *off = t - m;
        *crossed += 1;
        return m;
    }
    t %= n;
    return t < 0 ? t + n : t;
}

template <int RX, int RY, int RZ>
struct Region {
    static constexpr int N = RX * RY * RZ;
    __device__ static __forceinline__ int idx(int ix, int iy, int iz) { return ix + RX * (iy + RY * iz); }
};

// ------------------------------------------------------------ physics

template <class CT>
struct Phys {
    CT rho_a, drho, tau_a, dtau, inv_tau_phi;
    CT theta0;   // M / (T W)
    CT sig48W;   // 48 sigma / W
    CT sigW15;   // 3 sigma W / 2
    CT lambda_b;
    CT grav[3];
    CT inv_rho_a_T;
    int delta_theta;
};

template <class CT>
__device__ __forceinline__ Phys<CT> make_phys(const CaseDev& cs)
{
    Phys<CT> p;
    p.rho_a = (CT)cs.rho_a;
    p.drho = (CT)(cs.rho_w - cs.rho_a);
    p.tau_a = (CT)cs.tau_a;
    p.dtau = (CT)(cs.tau_w - cs.tau_a);
    p.inv_tau_phi = (CT)(1.0 / cs.tau_phi);
    p.theta0 = (CT)(cs.M / (kT * cs.W));
    p.sig48W = (CT)(48.0 * cs.sigma / cs.W);
    p.sigW15 = (CT)(1.5 * cs.sigma * cs.W);
    p.lambda_b = (CT)cs.lambda_b;
    p.grav[0] = (CT)cs.grav[0];
    p.grav[1] = (CT)cs.grav[1];
    p.grav[2] = (CT)cs.grav[2];
    p.inv_rho_a_T = (CT)(1.0 / (cs.rho_a * kT));
    p.delta_theta = cs.delta_theta;
    return p;
}

template <class CT> __device__ __forceinline__ CT clamp01(CT v) { return v < (CT)0 ? (CT)0 : (v > (CT)1 ? (CT)1 : v); }

// Local macroscopic values and gradients of one node.
template <class CT>
struct NodeVals {
    CT phi, u[3], gphi[3], lphi, grho[3], G[3][3];  // G[a][b] = d u_a / d x_b
};

// Equilibria of both lattices at one node, then (unless INIT) the collisions.
//   h[j]  in: post-streaming h_j; out: post-collision h*_j (INIT: h^eq_j)
//   g[i]  out: post-collision g*_i (INIT: g^eq_i); the rest entry excludes
//         the P / (rho_ref T) part
//   M2    sum g c c of the post-streaming populations (unused with INIT)
//   F     total force (for the wall correction); rho of the node
template <int DIMV, bool INIT, class CT>
__device__ __forceinline__ void node_physics(const Phys<CT>& p, const NodeVals<CT>& v,
                                             CT* __restrict__ h, const CT* __restrict__ M2,
                                             CT* __restrict__ g, CT F[3], CT* rho_out)
{
    using Mo = Model<DIMV>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    constexpr int D = DIMV;
    const CT T = (CT)kT, iT = (CT)3.0, i2T2 = (CT)4.5, i2T = (CT)1.5;
    const CT eps = (CT)1.0e-10;
    const CT phi = v.phi;

    // ---- phase field: normal, theta (+ delta theta), Gamma, h^eq, BGK
    CT gn2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) gn2 += v.gphi[a] * v.gphi[a];
    const CT gn = sqrt(gn2);
    const CT inv_n = (CT)1 / (gn + eps);
    CT nv[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) nv[a] = v.gphi[a] * inv_n;
    const CT dphi = phi - (CT)0.5;
    CT theta = p.theta0 * ((CT)1 - (CT)4 * dphi * dphi);
    if (p.delta_theta) {
        const CT s = v.lphi / (fabs(v.lphi) + eps);
        const CT iD = (CT)1.0e4;
        const CT Y1 = fmin(clamp01((phi - (CT)0.8) * iD), clamp01(-(phi - (CT)1) * iD));
        const CT Y2 = fmin(clamp01(phi * iD), clamp01(-(phi - (CT)0.2) * iD));
        theta += (CT)(-22.5) * p.theta0 * gn * (((CT)1 + s) * Y1 + ((CT)1 - s) * Y2);
    }
    CT u2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) u2 += v.u[a] * v.u[a];
    const CT base = (CT)1 - u2 * i2T;
#pragma unroll
    for (int j = 0; j < H::Q; ++j) {
        CT cu = 0, cn = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (H::c(j, a) == 1) { cu += v.u[a]; cn += nv[a]; }
            if (H::c(j, a) == -1) { cu -= v.u[a]; cn -= nv[a]; }
        }
        const CT wj = (CT)H::w(j);
        const CT gam = wj * (base + cu * iT + cu * cu * i2T2);
        const CT heq = phi * gam + theta * wj * cn;
        if (INIT) h[j] = heq;
        else h[j] = h[j] + (heq - h[j]) * p.inv_tau_phi;
    }

    // ---- hydrodynamics: rho, tau, nu, mu, F, sigma, B, g^eq, filter
    const CT pc = clamp01(phi);
    const CT rho = p.rho_a + pc * p.drho;
    const CT tau = p.tau_a + pc * p.dtau;
    const CT nu = T * (tau - (CT)0.5);
    const CT mu = p.sig48W * phi * (phi - (CT)1) * dphi - p.sigW15 * v.lphi;
    const CT irho = (CT)1 / rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) F[a] = rho * p.grav[a] + mu * v.gphi[a];
    CT div = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) div += v.G[a][a];
    const CT bulk = rho * (CT)(2.0 / 3.0) * (p.lambda_b - nu) * div;
    // a = u + F / rho + sigma . grad rho / rho^2 : first moment of g^eq
    CT av[3] = {0, 0, 0};
#pragma unroll
    for (int l = 0; l < D; ++l) {
        CT sg = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            CT s_lm = rho * nu * (v.G[l][m] + v.G[m][l]);
            if (l == m) s_lm += bulk;
            sg += s_lm * v.grho[m];
        }
        av[l] = v.u[l] + F[l] * irho + sg * irho * irho;
    }
    const CT B = (CT)(2.0 / 3.0) * (nu - p.lambda_b) + T * (CT)0.5;
    const CT Bdiv = B * div;
    // Pi = sum c c (g - g^eq) = M2 - (u u + B div I) on these lattices
    CT Pi[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    CT kf = 0, trPi = 0;
    if (!INIT) {
        if (D == 2) {
            Pi[0][0] = M2[0] - v.u[0] * v.u[0] - Bdiv;
            Pi[1][1] = M2[1] - v.u[1] * v.u[1] - Bdiv;
            Pi[0][1] = Pi[1][0] = M2[2] - v.u[0] * v.u[1];
        } else {
            Pi[0][0] = M2[0] - v.u[0] * v.u[0] - Bdiv;
            Pi[1][1] = M2[1] - v.u[1] * v.u[1] - Bdiv;
            Pi[2][2] = M2[2] - v.u[2] * v.u[2] - Bdiv;
            Pi[0][1] = Pi[1][0] = M2[3] - v.u[0] * v.u[1];
            Pi[0][2] = Pi[2][0] = M2[4] - v.u[0] * v.u[2];
            Pi[1][2] = Pi[2][1] = M2[5] - v.u[1] * v.u[2];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) trPi += Pi[a][a];
        kf = ((CT)1 - (CT)1 / tau) * i2T2;
    }
    const CT gbase = Bdiv * iT - u2 * i2T;
#pragma unroll
    for (int i = 0; i < G::Q; ++i) {
        const CT wi = (CT)G::w(i);
        CT ca = 0, cu = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (G::c(i, a) == 1) { ca += av[a]; cu += v.u[a]; }
            if (G::c(i, a) == -1) { ca -= av[a]; cu -= v.u[a]; }
        }
        CT geq = wi * (ca * iT + cu * cu * i2T2 + gbase);
        if (i == 0) geq -= Bdiv * iT;
        if (!INIT) {
            CT cPc = 0;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    const int cc = G::c(i, a) * G::c(i, b);
                    if (cc == 1) cPc += Pi[a][b];
                    if (cc == -1) cPc -= Pi[a][b];
                }
            geq += wi * kf * (cPc - T * trPi);
        }
        g[i] = geq;
    }
    *rho_out = rho;
}

// Isotropic central differences (Sec. II) of a tile field at cell c0:
// grad_a q = sum_i w_i c_ia (q(+c_i) - q(-c_i)) / (2T), lap q = 2 sum_i w_i (q(+c_i) - q0) / T.
template <class G, class RG, class CT, class F>
__device__ __forceinline__ void stencil(F q, int cx, int cy, int cz, CT grad[3], CT* lap)
{
    CT gr[3] = {0, 0, 0};
    CT l = 0;
    const CT q0 = q(RG::idx(cx, cy, cz));
#pragma unroll
    for (int i = 1; i < G::Q; i += 2) {  // pairs (i, i+1) are opposite
        const CT qp = q(RG::idx(cx + G::c(i, 0), cy + G::c(i, 1), cz + G::c(i, 2)));
        const CT qm = q(RG::idx(cx - G::c(i, 0), cy - G::c(i, 1), cz - G::c(i, 2)));
        const CT d = (qp - qm) * (CT)G::w(i);
#pragma unroll
        for (int a = 0; a < G::DIM; ++a) {
            if (G::c(i, a) == 1) gr[a] += d;
            if (G::c(i, a) == -1) gr[a] -= d;
        }
        if (lap) l += (qp + qm - (CT)2 * q0) * (CT)G::w(i);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) grad[a] = gr[a] * (CT)3.0;  // 2 * (1/(2T)): each pair counted once
    if (lap) *lap = l * (CT)6.0;                             // 2/T
}

// ================================================================ kernels

// --- moments: phi, u* = sum g c, S, M2 (per node; no halo)
template <int DIMV, class S>
__global__ __launch_bounds__(256) void k_moments(CaseTab cases, const int* __restrict__ tstart,
                                                 int ncases, int total_tiles, int step_off)
{
    using Mo = Model<DIMV>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    const TileCtx t = tile_ctx<Mo>(cases, tstart, ncases, total_tiles, step_off);
    if (!t.active) return;
    const CaseDev& cs = *cases[t.ci];
    const int lx = threadIdx.x % Mo::TX, ly = (threadIdx.x / Mo::TX) % Mo::TY,
              lz = threadIdx.x / (Mo::TX * Mo::TY);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    if (x >= cs.nx || y >= cs.ny || z >= cs.nz) return;
    const int64_t N = cs.N;
    const int64_t n = x + (int64_t)cs.nx * (y + (int64_t)cs.ny * z);
    const bool odd = t.step & 1;
    const Nav nv = make_nav(cs, x, y, z);
    const S* __restrict__ hp = (const S*)cs.h;
    const S* __restrict__ gp = (const S*)cs.g;
    const CT hsc = (CT)cs.h_inv_scale, gsc = (CT)cs.g_inv_scale;
    const CT phr = (CT)cs.phi_ref;

    CT phi = 0;
#pragma unroll
    for (int j = 0; j < H::Q; ++j)
        phi += Codec<S>::load(hp, aa_src<H>(nv, N, n, j, odd), hsc, phr * (CT)H::w(j));
    CT sum = 0, J[3] = {0, 0, 0}, m2[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < G::Q; ++i) {
        const CT f = Codec<S>::load(gp, aa_src<G>(nv, N, n, i, odd), gsc, (CT)0);
        sum += f;
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            if (G::c(i, a) == 1) J[a] += f;
            if (G::c(i, a) == -1) J[a] -= f;
        }
        if (i != 0) {
#pragma unroll
            for (int a = 0; a < DIMV; ++a)
                if (G::c(i, a) != 0) m2[a] += f;  // c_a^2 = 1
            if (DIMV == 2) {
                const int xy = G::c(i, 0) * G::c(i, 1);
                if (xy) m2[2] += xy > 0 ? f : -f;
            } else {
                const int xy = G::c(i, 0) * G::c(i, 1), xz = G::c(i, 0) * G::c(i, 2),
                          yz = G::c(i, 1) * G::c(i, 2);
                if (xy) m2[3] += xy > 0 ? f : -f;
                if (xz) m2[4] += xz > 0 ? f : -f;
                if (yz) m2[5] += yz > 0 ? f : -f;
            }
        }
    }
    CT* phiv = (CT*)cs.phi;
    CT* Jv = (CT*)cs.J;
    CT* Sv = (CT*)cs.S;
    CT* M2v = (CT*)cs.M2;
    phiv[n] = phi;
#pragma unroll
    for (int a = 0; a < DIMV; ++a) Jv[a * N + n] = J[a];
    Sv[n] = (CT)(cs.rho_a * kT) * sum;
    constexpr int NM = DIMV == 2 ? 3 : 6;
#pragma unroll
    for (int k = 0; k < NM; ++k) M2v[k * N + n] = m2[k];
}

// --- pressure (Sec. II): P = rho_ref T sum_i (g_i + (1 + omega) K_i)
//     + omega rho_ref sum_i w_i c_i . u*(x - c_i), K_i from the previous
//     pressure.  FP64 arithmetic whatever the storage precision.
template <int DIMV, class AT>
__global__ __launch_bounds__(256) void k_pressure(CaseTab cases, const int* __restrict__ tstart,
                                                  int ncases, int total_tiles, int step_off)
{
    using Mo = Model<DIMV>;
    using G = typename Mo::G;
    constexpr int ZH = DIMV == 3 ? 1 : 0;
    constexpr int RX = Mo::TX + 2, RY = Mo::TY + 2, RZ = Mo::TZ + 2 * ZH;
    using R = Region<RX, RY, RZ>;
    __shared__ double sP[R::N], sGD[R::N], sJ[DIMV][R::N];
    const TileCtx t = tile_ctx<Mo>(cases, tstart, ncases, total_tiles, step_off);
    if (!t.active) return;
    const CaseDev& cs = *cases[t.ci];
    const int64_t N = cs.N;
    const AT* __restrict__ Pl = (const AT*)cs.P[t.step & 1];
    AT* __restrict__ Pn = (AT*)cs.P[(t.step + 1) & 1];
    const AT* __restrict__ Jv = (const AT*)cs.J;
    for (int k = threadIdx.x; k < R::N; k += 256) {
        const int ix = k % RX, iy = (k / RX) % RY, iz = k / (RX * RY);
        int off[3], cr = 0;
        const int mx = resolve_axis(t.ox - 1 + ix, cs.nx, cs.wall[0], &off[0], &cr);
        const int my = resolve_axis(t.oy - 1 + iy, cs.ny, cs.wall[1], &off[1], &cr);
        const int mz = resolve_axis(t.oz - ZH + iz, cs.nz, cs.wall[2], &off[2], &cr);
        const int64_t m = mx + (int64_t)cs.nx * (my + (int64_t)cs.ny * mz);
        sP[k] = (double)Pl[m];
        // ghost pressure = P(mirror) + rho(x) g.(ghost - mirror): keep g.off
        sGD[k] = cs.grav[0] * off[0] + cs.grav[1] * off[1] + cs.grav[2] * off[2];
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            double j = (double)Jv[a * N + m];
            // u* at a ghost: flow part odd, body-force part even
            if (cr & 1) j = -j + 2.0 * cs.grav[a];
            sJ[a][k] = j;
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % Mo::TX, ly = (threadIdx.x / Mo::TX) % Mo::TY,
              lz = threadIdx.x / (Mo::TX * Mo::TY);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    if (x >= cs.nx || y >= cs.ny || z >= cs.nz) return;
    const int64_t n = x + (int64_t)cs.nx * (y + (int64_t)cs.ny * z);
    const double phi = (double)((const AT*)cs.phi)[n];
    const double ra = cs.rho_a, rw = cs.rho_w;
    const double pc = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
    const double rho = ra + pc * (rw - ra);
    const double omega = (rho - ra) / (rw - ra) * (rw / ra - 1.0);
    const int cx = lx + 1, cy = ly + 1, cz = lz + ZH;
    const double P0 = sP[R::idx(cx, cy, cz)];
    double sk = 0.0, su = 0.0;
#pragma unroll
    for (int i = 1; i < G::Q; ++i) {
        const int k = R::idx(cx - G::c(i, 0), cy - G::c(i, 1), cz - G::c(i, 2));
        sk += G::w(i) * (sP[k] + rho * sGD[k] - P0);
        double cu = 0.0;
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            if (G::c(i, a) == 1) cu += sJ[a][k];
            if (G::c(i, a) == -1) cu -= sJ[a][k];
        }
        su += G::w(i) * cu;
    }
    // rho_ref T (1 + omega) K summed = (1 + omega) rho_ref / rho * sum w (dP)
    const double P = P0 + (double)((const AT*)cs.S)[n] + (1.0 + omega) * ra / rho * sk +
                     omega * ra * su;
    Pn[n] = (AT)P;
}

// --- collide + stream.  READ: stop after rebuilding u (read pass).
template <int DIMV, class S, bool READ>
__global__ __launch_bounds__(256) void k_collide(CaseTab cases, const int* __restrict__ tstart,
                                                 int ncases, int total_tiles, int step_off)
{
    using Mo = Model<DIMV>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    constexpr int ZH = DIMV == 3 ? 1 : 0;
    constexpr int R1X = Mo::TX + 2, R1Y = Mo::TY + 2, R1Z = Mo::TZ + 2 * ZH;
    constexpr int R2X = Mo::TX + 4, R2Y = Mo::TY + 4, R2Z = Mo::TZ + 4 * ZH;
    using R1 = Region<R1X, R1Y, R1Z>;
    using R2 = Region<R2X, R2Y, R2Z>;
    __shared__ CT sP[R2::N], sGD[R2::N], sPhi[R1::N], sU[DIMV][R1::N];
    const TileCtx t = tile_ctx<Mo>(cases, tstart, ncases, total_tiles, step_off);
    if (!t.active) return;
    const CaseDev& cs = *cases[t.ci];
    const int64_t N = cs.N;
    const CT* __restrict__ Pn = (const CT*)cs.P[(t.step + 1) & 1];
    const CT* __restrict__ phiv = (const CT*)cs.phi;
    const CT* __restrict__ Jv = (const CT*)cs.J;
    const Phys<CT> ph = make_phys<CT>(cs);

    // A: new pressure on the 2-halo region, phi and u* on the 1-halo region
    for (int k = threadIdx.x; k < R2::N; k += 256) {
        const int ix = k % R2X, iy = (k / R2X) % R2Y, iz = k / (R2X * R2Y);
        int off[3], cr = 0;
        const int mx = resolve_axis(t.ox - 2 + ix, cs.nx, cs.wall[0], &off[0], &cr);
        const int my = resolve_axis(t.oy - 2 + iy, cs.ny, cs.wall[1], &off[1], &cr);
        const int mz = resolve_axis(t.oz - 2 * ZH + iz, cs.nz, cs.wall[2], &off[2], &cr);
        const int64_t m = mx + (int64_t)cs.nx * (my + (int64_t)cs.ny * mz);
        sP[k] = Pn[m];
        sGD[k] = (CT)(cs.grav[0] * off[0] + cs.grav[1] * off[1] + cs.grav[2] * off[2]);
    }
    for (int k = threadIdx.x; k < R1::N; k += 256) {
        const int ix = k % R1X, iy = (k / R1X) % R1Y, iz = k / (R1X * R1Y);
        int off[3], cr = 0;
        const int mx = resolve_axis(t.ox - 1 + ix, cs.nx, cs.wall[0], &off[0], &cr);
        const int my = resolve_axis(t.oy - 1 + iy, cs.ny, cs.wall[1], &off[1], &cr);
        const int mz = resolve_axis(t.oz - ZH + iz, cs.nz, cs.wall[2], &off[2], &cr);
        const int64_t m = mx + (int64_t)cs.nx * (my + (int64_t)cs.ny * mz);
        sPhi[k] = phiv[m];
#pragma unroll
        for (int a = 0; a < DIMV; ++a) sU[a][k] = Jv[a * N + m];
    }
    __syncthreads();

    // B: u = u* - D P / rho at every 1-halo cell.  A ghost cell takes the
    // velocity of its mirror node with the sign flipped once per wall.
    for (int k = threadIdx.x; k < R1::N; k += 256) {
        const int ix = k % R1X, iy = (k / R1X) % R1Y, iz = k / (R1X * R1Y);
        const int gx = t.ox - 1 + ix, gy = t.oy - 1 + iy, gz = t.oz - ZH + iz;
        int sx = 0, sy = 0, sz = 0, cr = 0;
        if (cs.wall[0]) { if (gx < 0) { sx = 1; ++cr; } else if (gx >= cs.nx) { sx = -1; ++cr; } }
        if (cs.wall[1]) { if (gy < 0) { sy = 1; ++cr; } else if (gy >= cs.ny) { sy = -1; ++cr; } }
        if (cs.wall[2]) { if (gz < 0) { sz = 1; ++cr; } else if (gz >= cs.nz) { sz = -1; ++cr; } }
        const int mx = ix + sx + 1, my = iy + sy + 1, mz = iz + sz + ZH;  // mirror in R2 coordinates
        const CT rho = ph.rho_a + clamp01(sPhi[k]) * ph.drho;
        const CT irho = (CT)1 / rho;
        CT gr[3] = {0, 0, 0};
#pragma unroll
        for (int i = 1; i < G::Q; i += 2) {
            const int kp = R2::idx(mx + G::c(i, 0), my + G::c(i, 1), mz + G::c(i, 2));
            const int km = R2::idx(mx - G::c(i, 0), my - G::c(i, 1), mz - G::c(i, 2));
            const CT d = ((sP[kp] + rho * sGD[kp]) - (sP[km] + rho * sGD[km])) * (CT)G::w(i);
#pragma unroll
            for (int a = 0; a < DIMV; ++a) {
                if (G::c(i, a) == 1) gr[a] += d;
                if (G::c(i, a) == -1) gr[a] -= d;
            }
        }
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            CT ua = sU[a][k] - gr[a] * (CT)3.0 * irho;
            sU[a][k] = (cr & 1) ? -ua : ua;
        }
    }
    __syncthreads();

    const int lx = threadIdx.x % Mo::TX, ly = (threadIdx.x / Mo::TX) % Mo::TY,
              lz = threadIdx.x / (Mo::TX * Mo::TY);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    if (x >= cs.nx || y >= cs.ny || z >= cs.nz) return;
    const int64_t n = x + (int64_t)cs.nx * (y + (int64_t)cs.ny * z);
    const int cx = lx + 1, cy = ly + 1, cz = lz + ZH;
    const int c0 = R1::idx(cx, cy, cz);
    if (READ) {
        CT* U = (CT*)cs.U;
#pragma unroll
        for (int a = 0; a < DIMV; ++a) U[a * N + n] = sU[a][c0];
        return;
    }

    // C: gradients, collisions, AA write
    NodeVals<CT> v;
    v.phi = sPhi[c0];
#pragma unroll
    for (int a = 0; a < 3; ++a) v.u[a] = a < DIMV ? sU[a][c0] : (CT)0;
    stencil<G, R1, CT>([&](int k) { return sPhi[k]; }, cx, cy, cz, v.gphi, &v.lphi);
    stencil<G, R1, CT>([&](int k) { return ph.rho_a + clamp01(sPhi[k]) * ph.drho; }, cx, cy, cz,
                       v.grho, (CT*)nullptr);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) v.G[a][b] = 0;
#pragma unroll
    for (int a = 0; a < DIMV; ++a) {
        CT gr[3];
        stencil<G, R1, CT>([&](int k) { return sU[a][k]; }, cx, cy, cz, gr, (CT*)nullptr);
#pragma unroll
        for (int b = 0; b < DIMV; ++b) v.G[a][b] = gr[b];
    }

    const bool odd = t.step & 1;
    const Nav nv = make_nav(cs, x, y, z);
    S* __restrict__ hp = (S*)cs.h;
    S* __restrict__ gp = (S*)cs.g;
    const CT hisc = (CT)cs.h_inv_scale, hsc = (CT)cs.h_scale;
    const CT gsc = (CT)cs.g_scale;
    const CT phr = (CT)cs.phi_ref;
    CT hv[H::Q];
#pragma unroll
    for (int j = 0; j < H::Q; ++j)
        hv[j] = Codec<S>::load(hp, aa_src<H>(nv, N, n, j, odd), hisc, phr * (CT)H::w(j));
    constexpr int NM = DIMV == 2 ? 3 : 6;
    CT m2[NM];
    const CT* __restrict__ M2v = (const CT*)cs.M2;
#pragma unroll
    for (int k = 0; k < NM; ++k) m2[k] = M2v[k * N + n];
    CT gv[G::Q];
    CT F[3], rho;
    node_physics<DIMV, false, CT>(ph, v, hv, m2, gv, F, &rho);
#pragma unroll
    for (int j = 0; j < H::Q; ++j) {
        bool bb;
        const int64_t d = aa_dst<H>(nv, N, n, j, odd, &bb);
        Codec<S>::store(hp, d, hv[j], hsc, phr * (CT)H::w(j));
    }
    const CT corr = (CT)2 * (CT)3.0 / rho;  // 2 / (rho T)
#pragma unroll
    for (int i = 0; i < G::Q; ++i) {
        bool bb;
        const int64_t d = aa_dst<G>(nv, N, n, i, odd, &bb);
        CT val = gv[i];
        if (bb) {
            CT cF = 0;
#pragma unroll
            for (int a = 0; a < DIMV; ++a) {
                if (G::c(i, a) == 1) cF += F[a];
                if (G::c(i, a) == -1) cF -= F[a];
            }
            val -= (CT)G::w(i) * cF * corr;
        }
        Codec<S>::store(gp, d, val, gsc, (CT)0);
    }
}

// --- initial state: equilibria of (phi0, P0, u0) in the even AA layout,
//     previous-step pressure P[0] = P0.  Inputs are FP64 device arrays.
template <int DIMV, class S>
__global__ __launch_bounds__(256) void k_init(CaseTab cases, const int* __restrict__ tstart, int ncases,
                                              int total_tiles, const double* __restrict__ phi0,
                                              const double* __restrict__ P0,
                                              const double* __restrict__ u0)
{
    using Mo = Model<DIMV>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    constexpr int ZH = DIMV == 3 ? 1 : 0;
    constexpr int R1X = Mo::TX + 2, R1Y = Mo::TY + 2, R1Z = Mo::TZ + 2 * ZH;
    using R1 = Region<R1X, R1Y, R1Z>;
    __shared__ CT sPhi[R1::N], sU[DIMV][R1::N];
    const TileCtx t = tile_ctx<Mo>(cases, tstart, ncases, total_tiles, 0);
    if (!t.active) return;
    const CaseDev& cs = *cases[t.ci];
    const int64_t N = cs.N;
    const Phys<CT> ph = make_phys<CT>(cs);
    for (int k = threadIdx.x; k < R1::N; k += 256) {
        const int ix = k % R1X, iy = (k / R1X) % R1Y, iz = k / (R1X * R1Y);
        int off[3], cr = 0;
        const int mx = resolve_axis(t.ox - 1 + ix, cs.nx, cs.wall[0], &off[0], &cr);
        const int my = resolve_axis(t.oy - 1 + iy, cs.ny, cs.wall[1], &off[1], &cr);
        const int mz = resolve_axis(t.oz - ZH + iz, cs.nz, cs.wall[2], &off[2], &cr);
        const int64_t m = mx + (int64_t)cs.nx * (my + (int64_t)cs.ny * mz);
        sPhi[k] = (CT)phi0[m];
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            const CT ua = (CT)u0[a * N + m];
            sU[a][k] = (cr & 1) ? -ua : ua;
        }
    }
    __syncthreads();
    const int lx = threadIdx.x % Mo::TX, ly = (threadIdx.x / Mo::TX) % Mo::TY,
              lz = threadIdx.x / (Mo::TX * Mo::TY);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    if (x >= cs.nx || y >= cs.ny || z >= cs.nz) return;
    const int64_t n = x + (int64_t)cs.nx * (y + (int64_t)cs.ny * z);
    const int cx = lx + 1, cy = ly + 1, cz = lz + ZH;
    const int c0 = R1::idx(cx, cy, cz);
    NodeVals<CT> v;
    v.phi = sPhi[c0];
#pragma unroll
    for (int a = 0; a < 3; ++a) v.u[a] = a < DIMV ? sU[a][c0] : (CT)0;
    stencil<G, R1, CT>([&](int k) { return sPhi[k]; }, cx, cy, cz, v.gphi, &v.lphi);
    stencil<G, R1, CT>([&](int k) { return ph.rho_a + clamp01(sPhi[k]) * ph.drho; }, cx, cy, cz,
                       v.grho, (CT*)nullptr);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) v.G[a][b] = 0;
#pragma unroll
    for (int a = 0; a < DIMV; ++a) {
        CT gr[3];
        stencil<G, R1, CT>([&](int k) { return sU[a][k]; }, cx, cy, cz, gr, (CT*)nullptr);
#pragma unroll
        for (int b = 0; b < DIMV; ++b) v.G[a][b] = gr[b];
    }
    CT hv[H::Q], gv[G::Q], F[3], rho;
    node_physics<DIMV, true, CT>(ph, v, hv, (const CT*)nullptr, gv, F, &rho);
    S* __restrict__ hp = (S*)cs.h;
    S* __restrict__ gp = (S*)cs.g;
    const CT hsc = (CT)cs.h_scale, gsc = (CT)cs.g_scale, phr = (CT)cs.phi_ref;
#pragma unroll
    for (int j = 0; j < H::Q; ++j) Codec<S>::store(hp, (int64_t)j * N + n, hv[j], hsc, phr * (CT)H::w(j));
#pragma unroll
    for (int i = 0; i < G::Q; ++i) Codec<S>::store(gp, (int64_t)i * N + n, gv[i], gsc, (CT)0);
    ((CT*)cs.P[0])[n] = (CT)P0[n];
}

// --- step counters: every case of a table advances by k (up to its end).
__global__ void k_advance(CaseTab cases, int ncases, int k)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncases) return;
    CaseDev* cs = cases[c];
    const int64_t s = cs->step + k;
    cs->step = s < cs->step_end ? s : cs->step_end;
}

// --- conservation diagnostics of a read pass: per-block FP64 partials
//     (wave64 shuffles, then across the block), reduced in a fixed order.
constexpr int kDiagBlocks = 1024;
constexpr int kDiagVals = 10;  // phi, u[3], rho u[3], umax, nonfinite, spare

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <class AT>
__global__ __launch_bounds__(256) void k_diag(const CaseDev* __restrict__ csp, double* __restrict__ partial)
{
    const CaseDev& cs = *csp;
    const int64_t N = cs.N;
    const AT* phi = (const AT*)cs.phi;
    const AT* P = (const AT*)cs.P[(cs.step + 1) & 1];
    const AT* U = (const AT*)cs.U;
    double acc[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < N; n += (int64_t)gridDim.x * 256) {
        const double f = (double)phi[n];
        const double pc = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
        const double rho = cs.rho_a + pc * (cs.rho_w - cs.rho_a);
        bool bad = !isfinite(f) || !isfinite((double)P[n]);
        double um2 = 0.0;
        acc[0] += f;
        for (int a = 0; a < cs.dim; ++a) {
            const double ua = (double)U[a * N + n];
            bad |= !isfinite(ua);
            acc[1 + a] += ua;
            acc[4 + a] += rho * ua;
            um2 += ua * ua;
        }
        acc[7] = fmax(acc[7], sqrt(um2));
        acc[8] += bad ? 1.0 : 0.0;
    }
    __shared__ double red[4][kDiagVals];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kDiagVals; ++k) {
        const double r = k == 7 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = r;
    }
    __syncthreads();
    if (threadIdx.x < kDiagVals) {
        const int k = threadIdx.x;
        double r = red[0][k];
        for (int w = 1; w < 4; ++w) r = k == 7 ? fmax(r, red[w][k]) : r + red[w][k];
        partial[blockIdx.x * kDiagVals + k] = r;
    }
}

__global__ __launch_bounds__(64) void k_diag_final(const double* __restrict__ partial, int nblocks,
                                                   double* __restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= kDiagVals) return;
    double r = 0.0;
    for (int b = 0; b < nblocks; ++b) r = k == 7 ? fmax(r, partial[b * kDiagVals + k]) : r + partial[b * kDiagVals + k];
    out[k] = r;
}

}  // namespace pulbm
