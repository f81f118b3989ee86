// libpulbm.so: C ABI (include/pulbm.h) around the HIP kernels of kernels.hpp.
//
// Host-side responsibilities: parameter validation, device memory layout of a
// case (library- or caller-owned), kernel dispatch per lattice / storage
// precision, read-back, diagnostics, restart images and the serving batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "pulbm.h"

using namespace pulbm;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPC(expr)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(PULBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

extern "C" const char* pulbm_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------ case layout

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int store_bytes(int store) { return store == PULBM_STORE_FP64 ? 8 : store == PULBM_STORE_FP32 ? 4 : 2; }
int aux_bytes(int store) { return store == PULBM_STORE_FP64 ? 8 : 4; }

struct Layout {
    size_t h, g, P0, P1, phi0, phi1, J, Ps, M2, U0, U1, desc, tab, partial, diag, total;
};

// Row pitch of every field: nx rounded up to 32 nodes, so that a tile row
// (64 nodes, at an x origin that is a multiple of 64) starts on a 128-byte
// line whatever nx is.
int row_pitch(int nx) { return (nx + 31) & ~31; }

Layout make_layout(const pulbm_params& p)
{
    const size_t N = (size_t)row_pitch(p.nx) * p.ny * p.nz;
    const size_t sb = store_bytes(p.store), ab = aux_bytes(p.store);
    const int dim = p.dim, nm = dim == 2 ? 3 : 6;
    Layout L;
    size_t o = 0;
    auto put = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.h = put((size_t)p.q_phase * N * sb);
    L.g = put((size_t)p.q_hydro * N * sb);
    L.P0 = put(N * ab);
    L.P1 = put(N * ab);
    L.phi0 = put(N * ab);
    L.phi1 = put(N * ab);
    L.J = put((size_t)dim * N * ab);
    L.Ps = put(N * ab);
    L.M2 = put((size_t)nm * N * ab);
    L.U0 = put((size_t)dim * N * ab);
    L.U1 = put((size_t)dim * N * ab);
    L.desc = put(sizeof(CaseDev));
    L.tab = put(sizeof(CaseDev*) + 4 * sizeof(int));
    L.partial = put((size_t)kDiagBlocks * kDiagVals * sizeof(double));
    L.diag = put(kDiagVals * sizeof(double));
    L.total = o;
    return L;
}

bool has_block(const pulbm_params& p)
{
    for (int a = 0; a < 3; ++a)
        if (p.block_lo[a] >= p.block_hi[a]) return false;
    return true;
}

int validate(const pulbm_params* p)
{
    if (!p) return fail(PULBM_EINVAL, "params is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(PULBM_EINVAL, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(PULBM_EINVAL, "grid sizes must be >= 1");
    if (p->dim == 2 && p->nz != 1) return fail(PULBM_EINVAL, "2D cases need nz = 1");
    if (p->dim == 2 && (p->q_hydro != 9 || p->q_phase != 9))
        return fail(PULBM_EINVAL, "2D cases use D2Q9 for both lattices (q_hydro = q_phase = 9)");
    if (p->dim == 3 && ((p->q_hydro != 27 && p->q_hydro != 19) || p->q_phase != 19))
        return fail(PULBM_EINVAL, "3D cases use a D3Q27 or D3Q19 hydro lattice and the D3Q19 phase field "
                                  "(q_hydro 27 or 19, q_phase 19)");
    if (p->store < PULBM_STORE_FP64 || p->store > PULBM_STORE_BF16) return fail(PULBM_EINVAL, "bad store %d", p->store);
    // kernels address one field with 32-bit byte offsets (signed for the
    // periodic neighbour steps): N times the widest element must stay below 2^31
    const double nodes = (double)row_pitch(p->nx) * p->ny * p->nz;
    const int widest = std::max(store_bytes(p->store), aux_bytes(p->store));
    if (nodes * widest >= 2147483648.0)
        return fail(PULBM_EINVAL, "grid too large: %.0f nodes x %d bytes per field element must stay below 2^31",
                    nodes, widest);
    if (p->collision != 0 && p->collision != 1)
        return fail(PULBM_EINVAL, "collision must be 0 (filter) or 1 (BGK)");
    for (int a = 0; a < 3; ++a) {
        if (p->wall[a] < 0 || p->wall[a] > 2) return fail(PULBM_EINVAL, "wall[%d] must be 0, 1 or 2", a);
        if (p->wall[a] == 2 && a != p->dim - 1)
            return fail(PULBM_EINVAL, "wall = 2 (open high end) is for the last axis only (axis %d)", p->dim - 1);
    }
    if (p->dim == 2 && p->wall[2]) return fail(PULBM_EINVAL, "2D cases have no z walls");
    if (!std::isfinite(p->p_top)) return fail(PULBM_EINVAL, "p_top must be finite");
    if (has_block(*p)) {
        const int n[3] = {p->nx, p->ny, p->nz};
        for (int a = 0; a < 3; ++a) {
            const int lo = p->block_lo[a], hi = p->block_hi[a];
            const bool full = lo == 0 && hi == n[a];
            if (lo < 0 || hi > n[a]) return fail(PULBM_EINVAL, "block exceeds the grid on axis %d", a);
            if (!full && hi - lo < 2)
                return fail(PULBM_EINVAL, "block must be at least 2 nodes thick on axis %d (or span it)", a);
            if (!full && !p->wall[a] && (lo < 1 || hi > n[a] - 1))
                return fail(PULBM_EINVAL, "block may not touch the periodic boundary of axis %d", a);
            if (p->wall[a] == 2 && hi == n[a])
                return fail(PULBM_EINVAL, "block may not touch the open end of axis %d", a);
        }
    }
    if (!(p->rho_heavy > 0) || !(p->rho_light > 0) || !(p->rho_heavy > p->rho_light))
        return fail(PULBM_EINVAL, "densities must satisfy rho_heavy > rho_light > 0");
    if (!(p->nu_heavy > 0) || !(p->nu_light > 0)) return fail(PULBM_EINVAL, "viscosities must be > 0");
    if (!(p->W > 0) || !(p->M > 0) || !(p->sigma >= 0) || !(p->lambda_bulk >= 0))
        return fail(PULBM_EINVAL, "W, M must be > 0 and sigma, lambda_bulk >= 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->gravity[a])) return fail(PULBM_EINVAL, "gravity must be finite");
    if (p->delta_theta != 0 && p->delta_theta != 1) return fail(PULBM_EINVAL, "delta_theta must be 0 or 1");
    return PULBM_OK;
}

// Multipliers of the tile order's divisors (CaseDev::dvh, dvl): M =
// floor(2^40 / d) + 1 gives floor(n M / 2^40) = n / d for n d < 2^40, since
// M d - 2^40 lies in [1, d].  fastdiv is set when that holds for every
// divisor and its largest dividend, and the tile count is below 2^23.
void tile_divisors(CaseDev& h, int64_t ntiles)
{
    const int64_t nb = (h.nty + h.tband - 1) / h.tband;
    const int64_t d[4] = {h.ntx, (int64_t)h.tband * h.ntz, h.tband, h.nty - (nb - 1) * h.tband};
    const int64_t nmax[4] = {ntiles, ntiles / h.ntx + 1, (int64_t)h.tband * h.ntz, (int64_t)h.tband * h.ntz};
    bool ok = ntiles < (int64_t(1) << 23);
    for (int k = 0; k < 4; ++k) {
        const uint64_t m = (uint64_t(1) << 40) / (uint64_t)d[k] + 1;
        h.dvh[k] = (uint32_t)(m >> 32);
        h.dvl[k] = (uint32_t)m;
        ok = ok && d[k] >= 1 && (uint64_t)nmax[k] * (uint64_t)d[k] < (uint64_t(1) << 40);
    }
    h.fastdiv = ok ? 1 : 0;
}

template <int LS> void tiles_of(const pulbm_params& p, int* ntx, int* nty, int* ntz)
{
    using Mo = Model<LS>;
    *ntx = (p.nx + Mo::TX - 1) / Mo::TX;
    *nty = (p.ny + Mo::TY - 1) / Mo::TY;
    *ntz = (p.nz + Mo::TZ - 1) / Mo::TZ;
}

int grid_of(int tiles) { return ((tiles + 7) / 8) * 8; }

constexpr int kStepKernels = 4;  // moments, pressure, velocity, collide + stream
constexpr int kVelocityKernel = 2;
constexpr int kReadKernels = 3;  // the moment stage only

}  // namespace

struct pulbm_case {
    pulbm_params p;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    bool own = false;
    Layout L;
    CaseDev h;          // host copy of the descriptor
    CaseDev* d = nullptr;
    CaseDev** tab = nullptr;  // device {d}
    int* hdr = nullptr;       // device tile table header {1, ntiles, 0, ntiles}
    int ntiles = 0;
    int64_t step = 0;
    bool ready = false;
    int device = 0;           // device current at pulbm_create
};

// ------------------------------------------------------------ dispatch

namespace {

template <int LS, class S>
void launch_step(hipStream_t st, CaseDev* const* tab, const int* hdr, int blocks, int off, int which, bool bgk,
                 int parity)
{
    using CT = typename Codec<S>::CT;
    const dim3 grid(blocks), block(256);
    if (which == 0) hipLaunchKernelGGL((k_moments<LS, S>), grid, block, 0, st, tab, hdr, off);
    if (which == 1) hipLaunchKernelGGL((k_pressure<LS, CT>), grid, block, 0, st, tab, hdr, off);
    if (which == 2) hipLaunchKernelGGL((k_velocity<LS, CT>), grid, block, 0, st, tab, hdr, off);
    if (which == 3) {
        // the collide kernel of each parity present (each skips the other's tiles)
        if (parity != 1) {
            if (bgk) hipLaunchKernelGGL((k_collide<LS, S, true, 0>), grid, block, 0, st, tab, hdr, off);
            else hipLaunchKernelGGL((k_collide<LS, S, false, 0>), grid, block, 0, st, tab, hdr, off);
        }
        if (parity != 0) {
            if (bgk) hipLaunchKernelGGL((k_collide<LS, S, true, 1>), grid, block, 0, st, tab, hdr, off);
            else hipLaunchKernelGGL((k_collide<LS, S, false, 1>), grid, block, 0, st, tab, hdr, off);
        }
    }
}

template <int LS>
void launch_dim(int store, hipStream_t st, CaseDev* const* tab, const int* hdr, int blocks, int off, int which,
                bool bgk, int parity)
{
    switch (store) {
        case PULBM_STORE_FP64: launch_step<LS, double>(st, tab, hdr, blocks, off, which, bgk, parity); break;
        case PULBM_STORE_FP32: launch_step<LS, float>(st, tab, hdr, blocks, off, which, bgk, parity); break;
        case PULBM_STORE_FP16: launch_step<LS, _Float16>(st, tab, hdr, blocks, off, which, bgk, parity); break;
        default: launch_step<LS, uint16_t>(st, tab, hdr, blocks, off, which, bgk, parity); break;
    }
}

// which: 0 moments, 1 pressure, 2 velocity, 3 collide + stream.  blocks must
// cover the table's tiles (rounded up to a multiple of 8); extra blocks exit.
// parity: the step parity of every case of the table for this launch (its
// device step counter plus off), 0 or 1, when the host knows it (a single
// case); -1 when cases may differ (serving batches): then the collide
// kernels of both parities are launched.
void launch(int ls, int store, bool bgk, hipStream_t st, CaseDev* const* tab, const int* hdr, int blocks, int off,
            int which, int parity = -1)
{
    if (ls == 2) launch_dim<2>(store, st, tab, hdr, blocks, off, which, bgk, parity);
    else if (ls == 4) launch_dim<4>(store, st, tab, hdr, blocks, off, which, bgk, parity);
    else launch_dim<3>(store, st, tab, hdr, blocks, off, which, bgk, parity);
}

template <int LS, class S>
void launch_init_t(hipStream_t st, CaseDev* const* tab, const int* hdr, int blocks, const double* phi,
                   const double* P, const double* u)
{
    hipLaunchKernelGGL((k_init<LS, S>), dim3(blocks), dim3(256), 0, st, tab, hdr, phi, P, u);
}

void launch_init(int ls, int store, hipStream_t st, CaseDev* const* tab, const int* hdr, int blocks,
                 const double* phi, const double* P, const double* u)
{
#define PULBM_INIT_CASE(D)                                                                          \
    switch (store) {                                                                                \
        case PULBM_STORE_FP64: launch_init_t<D, double>(st, tab, hdr, blocks, phi, P, u); break;    \
        case PULBM_STORE_FP32: launch_init_t<D, float>(st, tab, hdr, blocks, phi, P, u); break;     \
        case PULBM_STORE_FP16: launch_init_t<D, _Float16>(st, tab, hdr, blocks, phi, P, u); break;  \
        default: launch_init_t<D, uint16_t>(st, tab, hdr, blocks, phi, P, u); break;                \
    }
    if (ls == 2) { PULBM_INIT_CASE(2) } else if (ls == 4) { PULBM_INIT_CASE(4) } else { PULBM_INIT_CASE(3) }
#undef PULBM_INIT_CASE
}

// Codec constants.  FP16 stores h_j - w_j phi (phi of the reading node one
// step earlier) times 2^14 and g times 2^12; the stored values are small
// (|h_j - w_j phi| < w_j, |g_i| of the order of w_i |u| / T), so the scales
// keep them in FP16's normal range without overflow.  BF16 has FP32's
// exponent range and uses scale 1.
void codec_constants(const pulbm_params& p, CaseDev& h)
{
    h.h_scale = h.h_inv_scale = h.g_scale = h.g_inv_scale = 1.0;
    if (p.store == PULBM_STORE_FP16) {
        h.h_scale = 16384.0;
        h.h_inv_scale = 1.0 / 16384.0;
        h.g_scale = 4096.0;
        h.g_inv_scale = 1.0 / 4096.0;
    }
}

// The collision's derived constants, once on the host, in the expressions
// the kernels used (bitwise the values a thread would compute), and their
// FP32 roundings.
void derived_constants(CaseDev& h)
{
    h.inv_tau_phi = 1.0 / h.tau_phi;
    h.theta0 = h.M / (kT * h.W);
    h.sig48W = 48.0 * h.sigma / h.W;
    h.sigW15 = 1.5 * h.sigma * h.W;
    auto& f = h.f32;
    f.rho_a = (float)h.rho_a;
    f.drho = (float)(h.rho_w - h.rho_a);
    f.tau_a = (float)h.tau_a;
    f.dtau = (float)(h.tau_w - h.tau_a);
    f.inv_tau_phi = (float)h.inv_tau_phi;
    f.theta0 = (float)h.theta0;
    f.sig48W = (float)h.sig48W;
    f.sigW15 = (float)h.sigW15;
    f.lambda_b = (float)h.lambda_b;
    for (int a = 0; a < 3; ++a) f.grav[a] = (float)h.grav[a];
    f.h_scale = (float)h.h_scale;
    f.h_inv_scale = (float)h.h_inv_scale;
    f.g_scale = (float)h.g_scale;
    f.g_inv_scale = (float)h.g_inv_scale;
}

int upload_desc(pulbm_case* c)
{
    HIPC(hipMemcpyAsync(c->d, &c->h, sizeof(CaseDev), hipMemcpyHostToDevice, c->stream));
    return PULBM_OK;
}

// The moment stage on the current state without changing it.  Launched in
// read mode (step offset -1): it runs whatever the case's step limit, so a
// case that has finished its steps in a serving batch can be read while its
// descriptor stays untouched.
int read_pass(pulbm_case* c)
{
    for (int w = 0; w < kReadKernels; ++w)
        launch(lattice_set(c->p.dim, c->p.q_hydro), c->p.store, c->p.collision == 1, c->stream, c->tab, c->hdr, grid_of(c->ntiles), -1, w);
    HIPC(hipGetLastError());
    return PULBM_OK;
}

// Padded device rows of sx values -> compact host rows of nx doubles.
template <class AT>
void to_double(const std::vector<char>& raw, double* out, size_t rows, size_t nx, size_t sx)
{
    const AT* src = (const AT*)raw.data();
    for (size_t r = 0; r < rows; ++r)
        for (size_t i = 0; i < nx; ++i) out[r * nx + i] = (double)src[r * sx + i];
}

// Copy `comps` fields (each of N padded nodes) from the device into compact
// host rows of nx doubles: one contiguous copy (a strided copy to pageable
// memory goes row by row), then the rows are compacted on the host.
int fetch(pulbm_case* c, const void* dev, double* out, int comps)
{
    if (!out) return PULBM_OK;
    const size_t ab = aux_bytes(c->p.store);
    const size_t nx = (size_t)c->p.nx, sx = (size_t)c->h.sx, rows = (size_t)comps * c->p.ny * c->p.nz;
    std::vector<char> raw(rows * sx * ab);
    HIPC(hipMemcpyAsync(raw.data(), dev, raw.size(), hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    if (ab == 8) to_double<double>(raw, out, rows, nx, sx);
    else to_double<float>(raw, out, rows, nx, sx);
    return PULBM_OK;
}

}  // namespace

// ================================================================ case API

extern "C" int pulbm_required_bytes(const pulbm_params* p, size_t* bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return fail(PULBM_EINVAL, "bytes is NULL");
    *bytes = make_layout(*p).total;
    return PULBM_OK;
}

extern "C" int pulbm_create(const pulbm_params* p, void* dev_arena, size_t arena_bytes, void* hip_stream,
                            pulbm_case** out)
{
    if (!out) return fail(PULBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    pulbm_case* c = new (std::nothrow) pulbm_case();
    if (!c) return fail(PULBM_ENOMEM, "host allocation failed");
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    c->L = make_layout(*p);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(PULBM_EDEVICE, "hipGetDevice failed");
    }
    if (dev_arena) {
        if (arena_bytes < c->L.total) {
            delete c;
            return fail(PULBM_ENOMEM, "arena of %zu bytes is smaller than the %zu required", arena_bytes,
                        c->L.total);
        }
        if (((uintptr_t)dev_arena) % kAlign) {
            delete c;
            return fail(PULBM_EINVAL, "arena must be 256-byte aligned");
        }
        c->base = (char*)dev_arena;
    } else {
        hipError_t e = hipMalloc((void**)&c->base, c->L.total);
        if (e != hipSuccess) {
            delete c;
            return fail(PULBM_ENOMEM, "hipMalloc(%zu) failed: %s", c->L.total, hipGetErrorString(e));
        }
        c->own = true;
    }
    const Layout& L = c->L;
    CaseDev& h = c->h;
    std::memset(&h, 0, sizeof h);
    h.nx = p->nx; h.ny = p->ny; h.nz = p->nz; h.dim = p->dim;
    for (int a = 0; a < 3; ++a) { h.wall[a] = p->wall[a]; h.grav[a] = p->gravity[a]; }
    if (p->dim == 2) tiles_of<2>(*p, &h.ntx, &h.nty, &h.ntz);
    else tiles_of<3>(*p, &h.ntx, &h.nty, &h.ntz);
    c->ntiles = h.ntx * h.nty * h.ntz;
    // y bands of at least 64 tiles per z layer, and of 16 tile rows while a
    // layer's band stays within 128 tiles: z neighbours then run within what
    // one XCD holds at once (measured against plain x-y-z order: 128^3 +1%,
    // 256^3 +6%; 16 rows rather than 8 on the 512-wide dam break: +1.7%)
    h.tband = std::max(4, std::min(32, std::max(64 / h.ntx, std::min(16, 128 / h.ntx))));
    tile_divisors(h, c->ntiles);
    h.delta_theta = p->delta_theta;
    h.sx = row_pitch(p->nx);
    h.N = (int64_t)h.sx * p->ny * p->nz;
    // odd-step streamed loads in k_moments for wide populations of up to
    // 1 GiB (measured, FP32: 128^3 4% faster with them, the 256^3 bubble and
    // the 512x256x256 dam break 1-3% faster without)
    h.nt_odd_moments = (int64_t)(p->q_phase + p->q_hydro) * h.N * store_bytes(p->store) <= (int64_t(1) << 30);
    h.step = 0;
    h.step_end = INT64_MAX;
    h.h = c->base + L.h; h.g = c->base + L.g;
    h.P[0] = c->base + L.P0; h.P[1] = c->base + L.P1;
    h.phi[0] = c->base + L.phi0; h.phi[1] = c->base + L.phi1;
    h.J = c->base + L.J; h.Ps = c->base + L.Ps;
    h.M2 = c->base + L.M2; h.U[0] = c->base + L.U0; h.U[1] = c->base + L.U1;
    h.rho_a = p->rho_light; h.rho_w = p->rho_heavy;
    h.tau_a = p->nu_light / kT + 0.5;
    h.tau_w = p->nu_heavy / kT + 0.5;
    h.tau_phi = p->M / kT + 0.5;
    h.M = p->M; h.W = p->W; h.sigma = p->sigma; h.lambda_b = p->lambda_bulk;
    h.p_top = p->p_top;
    h.has_block = has_block(*p);
    for (int a = 0; a < 3; ++a) {
        h.blk_lo[a] = h.has_block ? p->block_lo[a] : 0;
        h.blk_hi[a] = h.has_block ? p->block_hi[a] : 0;
    }
    // the collide kernel rebuilds u from a 2-node halo of the new P where
    // every tile is clear of walls, the open end and the block, and one
    // +-n wraps two nodes past either end of every axis.  Measured at 128^3:
    // with D3Q19 and D2Q9 hydro (9 and 4 direction pairs) this saves more
    // than it adds to the collide kernel; with D3Q27 (13 pairs) the two
    // cancel, and the separate velocity kernel is kept.
    h.fuse_u = !h.has_block && !p->wall[0] && !p->wall[1] && !p->wall[2] && store_bytes(p->store) >= 4 &&
               p->nx >= 3 && p->ny >= 3 && (p->dim == 2 || (p->nz >= 3 && p->q_hydro == 19));
    codec_constants(*p, h);
    derived_constants(h);
    c->d = (CaseDev*)(c->base + L.desc);
    c->tab = (CaseDev**)(c->base + L.tab);
    c->hdr = (int*)(c->base + L.tab + sizeof(CaseDev*));
    struct { CaseDev* d; int hdr[4]; } tabh = {c->d, {1, c->ntiles, 0, c->ntiles}};
    hipError_t e = hipMemcpyAsync(c->tab, &tabh, sizeof tabh, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d, &c->h, sizeof(CaseDev), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        pulbm_destroy(c);
        return fail(PULBM_EDEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
    }
    *out = c;
    return PULBM_OK;
}

extern "C" void pulbm_destroy(pulbm_case* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->own && c->base) (void)hipFree(c->base);
    delete c;
}

extern "C" int pulbm_init_fields(pulbm_case* c, const double* phi, const double* P, const double* u)
{
    if (!c || !phi || !P || !u) return fail(PULBM_EINVAL, "NULL argument");
    const size_t N = (size_t)c->h.N;  // padded
    const size_t nx = (size_t)c->p.nx, rows = (size_t)c->p.ny * c->p.nz, Nc = nx * rows;
    const int dim = c->p.dim;
    for (size_t n = 0; n < Nc; ++n)
        if (!std::isfinite(phi[n]) || !std::isfinite(P[n]))
            return fail(PULBM_EDIVERGED, "non-finite initial phi or P at node %zu", n);
    for (size_t n = 0; n < (size_t)dim * Nc; ++n)
        if (!std::isfinite(u[n])) return fail(PULBM_EDIVERGED, "non-finite initial u at entry %zu", n);
    c->h.step = 0;
    c->h.step_end = INT64_MAX;
    int rc = upload_desc(c);
    if (rc) return rc;
    // stage the FP64 inputs in the case's own scratch fields (u*, P*, M2,
    // U[0]), which k_init does not touch (it writes U[1]); no allocation on
    // this path
    // (u*, P*, M2 and U[0] hold at least (dim + 1 + 3 + dim) * N auxiliary
    // values of 4 or 8 bytes, which covers (2 + dim) * N doubles whenever
    // dim <= 3; checked anyway)
    const size_t bytes = (2 + (size_t)dim) * N * sizeof(double);
    double* tmp = (double*)(c->base + c->L.J);
    if (bytes > c->L.U1 - c->L.J) return fail(PULBM_EDEVICE, "internal: init staging does not fit the scratch fields");
    // compact host rows of nx padded to rows of sx on the host (the padding is
    // never read), then one contiguous copy
    const size_t sx = (size_t)c->h.sx;
    std::vector<double> staged((2 + (size_t)dim) * N, 0.0);
    auto pad = [&](const double* src, double* dst, size_t nrows) {
        for (size_t r = 0; r < nrows; ++r) std::memcpy(dst + r * sx, src + r * nx, nx * sizeof(double));
    };
    pad(phi, staged.data(), rows);
    pad(P, staged.data() + N, rows);
    pad(u, staged.data() + 2 * N, (size_t)dim * rows);
    hipError_t e = hipMemcpyAsync(tmp, staged.data(), bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        launch_init(lattice_set(dim, c->p.q_hydro), c->p.store, c->stream, c->tab, c->hdr, grid_of(c->ntiles), tmp, tmp + N, tmp + 2 * N);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(PULBM_EDEVICE, "init failed: %s", hipGetErrorString(e));
    c->step = 0;
    c->ready = true;
    return PULBM_OK;
}

// count steps: kernels at step offsets 0 .. count-1, then the step counter.
// (Replaying captured graphs instead was measured: 5% slower on a 128^3 case,
// 3% faster on an 80k-node 2D case; direct launches are kept.)
static void queue_direct(pulbm_case* c, int64_t first, int count)
{
    for (int k = 0; k < count; ++k)
        for (int w = 0; w < kStepKernels; ++w)
            if (w != kVelocityKernel || !c->h.fuse_u)
                launch(lattice_set(c->p.dim, c->p.q_hydro), c->p.store, c->p.collision == 1, c->stream, c->tab,
                       c->hdr, grid_of(c->ntiles), k, w, (int)((first + k) & 1));
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, c->stream, c->tab, c->hdr, count);
}

static int queue_steps(pulbm_case* c, int64_t nsteps)
{
    int64_t s = 0;
    for (; s < nsteps;) {
        const int chunk = (int)std::min<int64_t>(nsteps - s, 1 << 20);
        queue_direct(c, c->step + s, chunk);
        HIPC(hipGetLastError());
        s += chunk;
    }
    c->step += nsteps;
    c->h.step = c->step;
    return PULBM_OK;
}

extern "C" int pulbm_step(pulbm_case* c, int64_t nsteps)
{
    if (!c) return fail(PULBM_EINVAL, "case is NULL");
    if (!c->ready) return fail(PULBM_ESTATE, "pulbm_step before pulbm_init_fields");
    if (nsteps < 0) return fail(PULBM_EINVAL, "nsteps < 0");
    return queue_steps(c, nsteps);
}

extern "C" int pulbm_step_timed(pulbm_case* c, int64_t nsteps, double* ms)
{
    if (!c || !ms) return fail(PULBM_EINVAL, "NULL argument");
    if (!c->ready) return fail(PULBM_ESTATE, "pulbm_step_timed before pulbm_init_fields");
    hipEvent_t ev[kStepKernels + 1];
    for (int k = 0; k <= kStepKernels; ++k) HIPC(hipEventCreate(&ev[k]));
    int rc = PULBM_OK;
    for (int64_t s = 0; s < nsteps && rc == PULBM_OK; ++s) {
        (void)hipEventRecord(ev[0], c->stream);
        for (int w = 0; w < kStepKernels; ++w) {
            if (w != kVelocityKernel || !c->h.fuse_u)
                launch(lattice_set(c->p.dim, c->p.q_hydro), c->p.store, c->p.collision == 1, c->stream, c->tab,
                       c->hdr, grid_of(c->ntiles), 0, w, (int)(c->step & 1));
            (void)hipEventRecord(ev[w + 1], c->stream);
        }
        hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, c->stream, c->tab, c->hdr, 1);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipEventSynchronize(ev[kStepKernels]);
        if (e != hipSuccess) {
            rc = fail(PULBM_EDEVICE, "timed step failed: %s", hipGetErrorString(e));
            break;
        }
        for (int w = 0; w < kStepKernels; ++w) {
            float t = 0.f;
            (void)hipEventElapsedTime(&t, ev[w], ev[w + 1]);
            ms[w] += t;
        }
        c->step += 1;
    }
    c->h.step = c->step;
    for (int k = 0; k <= kStepKernels; ++k) (void)hipEventDestroy(ev[k]);
    if (rc == PULBM_OK) HIPC(hipStreamSynchronize(c->stream));
    return rc;
}

extern "C" int pulbm_read_fields(pulbm_case* c, double* phi, double* P, double* u)
{
    if (!c) return fail(PULBM_EINVAL, "case is NULL");
    if (!c->ready) return fail(PULBM_ESTATE, "read before init");
    int rc = read_pass(c);
    if (rc) return rc;
    if ((rc = fetch(c, c->h.phi[c->step & 1], phi, 1))) return rc;
    if ((rc = fetch(c, c->h.P[(c->step + 1) & 1], P, 1))) return rc;
    if ((rc = fetch(c, c->h.U[c->step & 1], u, c->p.dim))) return rc;
    return PULBM_OK;
}

// ============================================= allocation-free read-back

namespace {

// Device staging of pulbm_read_fields_noalloc: the compact FP64 phi, P and u
// of one case.  Each GPU the library runs on holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress gives on that device (scratch_ptr).
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
struct ScratchDev {
    std::mutex lock;       // one call at a time uses a device's array
    void* ptr = nullptr;   // its device address, once looked up
};
ScratchDev g_scratch[kMaxDevices];

// Device address of `scratch` on device dev (which must be current).
int scratch_ptr(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(PULBM_EDEVICE, "device %d out of range", dev);
    ScratchDev& sd = g_scratch[dev];
    if (!sd.ptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PULBM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        sd.ptr = p;
    }
    *out = sd.ptr;
    return PULBM_OK;
}

// Compact FP64 copies of phi, P and the dim velocity components (padded rows
// of sx nodes in the auxiliary type -> rows of nx doubles), field after field.
template <class AT>
__global__ __launch_bounds__(256) void k_pack_fields(const AT* __restrict__ phi, const AT* __restrict__ P,
                                                     const AT* __restrict__ U, int64_t N, int nx, int sx,
                                                     int64_t nc, int comps, double* __restrict__ out)
{
    const int64_t total = nc * comps;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        const int64_t f = k / nc, n = k - f * nc;
        const int64_t m = (n % nx) + (int64_t)sx * (n / nx);
        const AT* src = f == 0 ? phi : (f == 1 ? P : U + (f - 2) * N);
        out[k] = (double)src[m];
    }
}

}  // namespace

extern "C" int pulbm_read_fields_noalloc(pulbm_case* c, double* phi, double* P, double* u)
{
    if (!c || !phi || !P || !u) return fail(PULBM_EINVAL, "NULL argument");
    if (!c->ready) return fail(PULBM_ESTATE, "read before init");
    const int dim = c->p.dim, comps = 2 + dim;
    const size_t nc = (size_t)c->p.nx * c->p.ny * c->p.nz;
    if ((size_t)comps * nc * sizeof(double) > kScratchBytes)
        return fail(PULBM_EINVAL, "case of %zu nodes exceeds the allocation-free read-back (at most %zu nodes in %dD)",
                    nc, kScratchBytes / (sizeof(double) * comps), dim);
    int cur = 0;
    HIPC(hipGetDevice(&cur));
    if (cur != c->device) HIPC(hipSetDevice(c->device));
    int rc = PULBM_OK;
    {
        std::lock_guard<std::mutex> hold(g_scratch[c->device < kMaxDevices && c->device >= 0 ? c->device : 0].lock);
        void* sp = nullptr;
        rc = scratch_ptr(c->device, &sp);
        if (!rc) rc = read_pass(c);
        if (!rc) {
            double* out = (double*)sp;
            const void* fphi = c->h.phi[c->step & 1];
            const void* fP = c->h.P[(c->step + 1) & 1];
            const void* fU = c->h.U[c->step & 1];
            const int64_t total = (int64_t)nc * comps;
            const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
            if (c->p.store == PULBM_STORE_FP64)
                hipLaunchKernelGGL(k_pack_fields<double>, dim3(blocks), dim3(256), 0, c->stream, (const double*)fphi,
                                   (const double*)fP, (const double*)fU, c->h.N, c->p.nx, c->h.sx, (int64_t)nc,
                                   comps, out);
            else
                hipLaunchKernelGGL(k_pack_fields<float>, dim3(blocks), dim3(256), 0, c->stream, (const float*)fphi,
                                   (const float*)fP, (const float*)fU, c->h.N, c->p.nx, c->h.sx, (int64_t)nc,
                                   comps, out);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(phi, out, nc * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(P, out + nc, nc * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(u, out + 2 * nc, (size_t)dim * nc * sizeof(double), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) rc = fail(PULBM_EDEVICE, "allocation-free read-back failed: %s", hipGetErrorString(e));
        }
    }
    if (cur != c->device) (void)hipSetDevice(cur);
    return rc;
}

extern "C" int pulbm_diagnostics(pulbm_case* c, pulbm_diag* d)
{
    if (!c || !d) return fail(PULBM_EINVAL, "NULL argument");
    if (!c->ready) return fail(PULBM_ESTATE, "diagnostics before init");
    int rc = read_pass(c);
    if (rc) return rc;
    double* partial = (double*)(c->base + c->L.partial);
    double* dd = (double*)(c->base + c->L.diag);
    if (c->p.store == PULBM_STORE_FP64)
        hipLaunchKernelGGL(k_diag<double>, dim3(kDiagBlocks), dim3(256), 0, c->stream, c->d, partial);
    else
        hipLaunchKernelGGL(k_diag<float>, dim3(kDiagBlocks), dim3(256), 0, c->stream, c->d, partial);
    hipLaunchKernelGGL(k_diag_final, dim3(kDiagVals), dim3(64), 0, c->stream, partial, kDiagBlocks, dd);
    HIPC(hipGetLastError());
    double r[kDiagVals];
    HIPC(hipMemcpyAsync(r, dd, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    std::memset(d, 0, sizeof *d);
    d->phi_sum = r[0];
    for (int a = 0; a < 3; ++a) { d->u_sum[a] = r[1 + a]; d->rhou_sum[a] = r[4 + a]; }
    d->umax = r[7];
    d->nonfinite = (int64_t)r[8];
    d->step = c->step;
    if (d->nonfinite > 0) return fail(PULBM_EDIVERGED, "%lld nodes hold non-finite values", (long long)d->nonfinite);
    return PULBM_OK;
}

// Restart image: header, h, g, previous-step pressure, previous-step phi and
// u (the references of the 2-byte codecs).
namespace {
constexpr char kCkptMagic[9] = "PULBMCK4";
constexpr int32_t kCkptVersion = 4;
struct CkptHeader {
    char magic[8];
    int32_t version, store;
    pulbm_params p;
    int64_t step;
    uint64_t h_bytes, g_bytes, P_bytes;
};
}  // namespace

extern "C" int pulbm_checkpoint_bytes(const pulbm_case* c, size_t* bytes)
{
    if (!c || !bytes) return fail(PULBM_EINVAL, "NULL argument");
    const size_t N = (size_t)c->h.N, sb = store_bytes(c->p.store), ab = aux_bytes(c->p.store);
    *bytes = sizeof(CkptHeader) + (size_t)(c->p.q_phase + c->p.q_hydro) * N * sb + (2 + (size_t)c->p.dim) * N * ab;
    return PULBM_OK;
}

extern "C" int pulbm_checkpoint(pulbm_case* c, void* buf, size_t bytes)
{
    size_t need = 0;
    int rc = pulbm_checkpoint_bytes(c, &need);
    if (rc) return rc;
    if (!buf || bytes < need) return fail(PULBM_EINVAL, "checkpoint buffer needs %zu bytes", need);
    if (!c->ready) return fail(PULBM_ESTATE, "checkpoint before init");
    const size_t N = (size_t)c->h.N, sb = store_bytes(c->p.store), ab = aux_bytes(c->p.store);
    CkptHeader hd;
    std::memset(&hd, 0, sizeof hd);
    std::memcpy(hd.magic, kCkptMagic, 8);
    hd.version = kCkptVersion;
    hd.store = c->p.store;
    hd.p = c->p;
    hd.step = c->step;
    hd.h_bytes = (uint64_t)c->p.q_phase * N * sb;
    hd.g_bytes = (uint64_t)c->p.q_hydro * N * sb;
    hd.P_bytes = N * ab;
    char* o = (char*)buf;
    std::memcpy(o, &hd, sizeof hd);
    o += sizeof hd;
    HIPC(hipMemcpyAsync(o, c->h.h, hd.h_bytes, hipMemcpyDeviceToHost, c->stream));
    o += hd.h_bytes;
    HIPC(hipMemcpyAsync(o, c->h.g, hd.g_bytes, hipMemcpyDeviceToHost, c->stream));
    o += hd.g_bytes;
    HIPC(hipMemcpyAsync(o, c->h.P[c->step & 1], hd.P_bytes, hipMemcpyDeviceToHost, c->stream));
    o += hd.P_bytes;
    HIPC(hipMemcpyAsync(o, c->h.phi[(c->step + 1) & 1], hd.P_bytes, hipMemcpyDeviceToHost, c->stream));
    o += hd.P_bytes;
    HIPC(hipMemcpyAsync(o, c->h.U[(c->step + 1) & 1], (size_t)c->p.dim * hd.P_bytes, hipMemcpyDeviceToHost,
                        c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    return PULBM_OK;
}

extern "C" int pulbm_restore(pulbm_case* c, const void* buf, size_t bytes)
{
    if (!c || !buf) return fail(PULBM_EINVAL, "NULL argument");
    if (bytes < sizeof(CkptHeader)) return fail(PULBM_EINVAL, "restart image too short");
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof hd);
    if (std::memcmp(hd.magic, kCkptMagic, 8) || hd.version != kCkptVersion) return fail(PULBM_EINVAL, "not a restart image");
    const pulbm_params& q = hd.p;
    const pulbm_params& p = c->p;
    if (q.dim != p.dim || q.nx != p.nx || q.ny != p.ny || q.nz != p.nz || q.store != p.store ||
        hd.store != p.store || q.q_hydro != p.q_hydro || q.q_phase != p.q_phase)
        return fail(PULBM_EINVAL, "restart image is for a different grid or precision");
    // the boundaries and the collision shape the stored state (bounce-back
    // slots, block nodes, the rest population of BGK), so they must match too;
    // fluid properties and body force are taken from the target case
    bool same_geometry = q.collision == p.collision && q.p_top == p.p_top;
    for (int a = 0; a < 3; ++a)
        same_geometry = same_geometry && q.wall[a] == p.wall[a] && q.block_lo[a] == p.block_lo[a] &&
                        q.block_hi[a] == p.block_hi[a];
    if (!same_geometry) return fail(PULBM_EINVAL, "restart image is for different boundaries or collision");
    // section sizes are checked against the case, never trusted from the image
    const size_t N = (size_t)c->h.N, sb = store_bytes(p.store), ab = aux_bytes(p.store);
    if (hd.h_bytes != (uint64_t)p.q_phase * N * sb || hd.g_bytes != (uint64_t)p.q_hydro * N * sb ||
        hd.P_bytes != (uint64_t)N * ab)
        return fail(PULBM_EINVAL, "restart image section sizes do not match the case");
    if (hd.step < 0) return fail(PULBM_EINVAL, "restart image has a negative step count");
    size_t need = 0;
    pulbm_checkpoint_bytes(c, &need);
    if (bytes < need) return fail(PULBM_EINVAL, "restart image too short");
    c->step = hd.step;
    c->h.step = hd.step;
    c->h.step_end = INT64_MAX;
    int rc = upload_desc(c);
    if (rc) return rc;
    const char* o = (const char*)buf + sizeof hd;
    HIPC(hipMemcpyAsync(c->h.h, o, hd.h_bytes, hipMemcpyHostToDevice, c->stream));
    o += hd.h_bytes;
    HIPC(hipMemcpyAsync(c->h.g, o, hd.g_bytes, hipMemcpyHostToDevice, c->stream));
    o += hd.g_bytes;
    HIPC(hipMemcpyAsync(c->h.P[c->step & 1], o, hd.P_bytes, hipMemcpyHostToDevice, c->stream));
    o += hd.P_bytes;
    HIPC(hipMemcpyAsync(c->h.phi[(c->step + 1) & 1], o, hd.P_bytes, hipMemcpyHostToDevice, c->stream));
    o += hd.P_bytes;
    HIPC(hipMemcpyAsync(c->h.U[(c->step + 1) & 1], o, (size_t)c->p.dim * hd.P_bytes, hipMemcpyHostToDevice,
                        c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    c->ready = true;
    return PULBM_OK;
}

extern "C" int pulbm_sync(pulbm_case* c)
{
    if (!c) return fail(PULBM_EINVAL, "case is NULL");
    HIPC(hipStreamSynchronize(c->stream));
    return PULBM_OK;
}

extern "C" int64_t pulbm_steps_done(const pulbm_case* c) { return c ? c->step : -1; }

extern "C" int pulbm_set_tile_order(pulbm_case* c, int32_t order)
{
    if (!c) return fail(PULBM_EINVAL, "case is NULL");
    if (order != 0 && order != 1) return fail(PULBM_EINVAL, "order must be 0 or 1");
    c->h.tile_rev = order;
    return upload_desc(c);
}

// ============================================================= measurement

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy: each block moves 1024 16-byte vectors (16 KiB), every load
// of a thread issued before its first store.  NTL / NTS: non-temporal loads /
// stores, the access hints the step kernels choose per storage width.
template <bool NTL, bool NTS>
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     uint64_t n16)
{
    const uint64_t base = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i = base + 256 * k;
        if (i < n16) {
            if constexpr (NTL) v[k] = __builtin_nontemporal_load(src + i);
            else v[k] = src[i];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t i = base + 256 * k;
        if (i < n16) {
            if constexpr (NTS) __builtin_nontemporal_store(v[k], dst + i);
            else dst[i] = v[k];
        }
    }
}

}  // namespace

extern "C" int pulbm_stream_copy(void* dst, const void* src, size_t bytes, int32_t mode, int32_t reps,
                                 void* hip_stream, double* ms)
{
    if (!dst || !src || !ms) return fail(PULBM_EINVAL, "NULL argument");
    if (bytes == 0 || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
        return fail(PULBM_EINVAL, "bytes and both pointers must be non-zero multiples of 16");
    if (mode < 0 || mode > 3) return fail(PULBM_EINVAL, "mode must be 0..3");
    if (reps < 1) return fail(PULBM_EINVAL, "reps must be >= 1");
    const char* s = (const char*)src;
    const char* d = (const char*)dst;
    if (s < d + bytes && d < s + bytes) return fail(PULBM_EINVAL, "source and destination overlap");
    hipStream_t st = (hipStream_t)hip_stream;
    const uint64_t n16 = bytes / 16;
    const uint64_t blocks = (n16 + 1023) / 1024;
    if (blocks > 0x7fffffffull) return fail(PULBM_EINVAL, "copy too large");
    const u32x4* a = (const u32x4*)src;
    u32x4* b = (u32x4*)dst;
    auto go = [&]() {
        const dim3 grid((unsigned)blocks), block(256);
        switch (mode) {
            case 0: hipLaunchKernelGGL((k_stream_copy<false, false>), grid, block, 0, st, a, b, n16); break;
            case 1: hipLaunchKernelGGL((k_stream_copy<true, false>), grid, block, 0, st, a, b, n16); break;
            case 2: hipLaunchKernelGGL((k_stream_copy<false, true>), grid, block, 0, st, a, b, n16); break;
            default: hipLaunchKernelGGL((k_stream_copy<true, true>), grid, block, 0, st, a, b, n16); break;
        }
    };
    go();  // warm
    HIPC(hipGetLastError());
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) go();
    (void)hipEventRecord(e1, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(PULBM_EDEVICE, "stream copy failed: %s", hipGetErrorString(e));
    *ms = (double)t / reps;
    return PULBM_OK;
}

// ============================================================= serving batch

struct pulbm_batch {
    size_t budget = 0, used = 0;
    int store = 0, max_slots = 0;
    hipStream_t stream = nullptr;  // advances
    hipStream_t side = nullptr;    // admissions and read-backs
    bool own_stream = false;
    // one device arena of the whole budget; cases are carved from it
    // (first fit, 256-byte granules, neighbouring holes merged on release)
    char* arena = nullptr;
    std::map<size_t, size_t> holes;  // offset -> bytes
    struct Release {
        int64_t after;  // advances up to this one may still read the block
        size_t off, bytes;
    };
    std::vector<Release> retiring;
    // graphs replaced while advances that replay them may still be queued
    std::vector<std::pair<int64_t, hipGraphExec_t>> old_graphs;
    struct Slot {
        pulbm_case* c = nullptr;
        int64_t end = 0;
        int64_t finish = -1;  // advance that takes the case to its end
        size_t bytes = 0, off = 0;
    };
    std::vector<Slot> slots;
    // advances in flight: sequence number -> completion event
    int64_t enqueued = 0, completed = 0;
    std::deque<std::pair<int64_t, hipEvent_t>> inflight;
    std::vector<hipEvent_t> spare_events;
    // per lattice dimension: device table of case pointers + its header,
    // filled by stream-ordered copies from pinned host staging (two buffers,
    // each reused once its previous copy has executed)
    struct Tab {
        CaseDev** dtab = nullptr;
        int* dhdr = nullptr;  // {ncases, tiles, tstart[0..ncases]}
        char* stage[2] = {nullptr, nullptr};
        hipEvent_t staged[2] = {nullptr, nullptr};
        int which = 0;
        int cap = 0, ncases = 0, tiles = 0, grid = 0;
        std::map<int, hipGraphExec_t> graphs;  // by 4 ksteps + parity (0, 1; 2 mixed), captured for `grid` blocks
    } tab[6];  // index (lattice set - 2) + 3 * collision
    bool dirty = true;
};

namespace {

bool arena_take(pulbm_batch* b, size_t bytes, size_t* off)
{
    for (auto it = b->holes.begin(); it != b->holes.end(); ++it) {
        if (it->second < bytes) continue;
        *off = it->first;
        const size_t rest = it->second - bytes;
        b->holes.erase(it);
        if (rest) b->holes[*off + bytes] = rest;
        return true;
    }
    return false;
}

void arena_give(pulbm_batch* b, size_t off, size_t bytes)
{
    auto it = b->holes.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != b->holes.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->holes.erase(nx);
    }
    if (it != b->holes.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->holes.erase(it);
        }
    }
}

// Retire completed advances (wait_upto: block until that one is done too)
// and release the arena blocks no advance can read any more.
int sync_advances(pulbm_batch* b, int64_t wait_upto)
{
    while (!b->inflight.empty()) {
        auto& f = b->inflight.front();
        if (f.first <= wait_upto) {
            HIPC(hipEventSynchronize(f.second));
        } else {
            const hipError_t q = hipEventQuery(f.second);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return fail(PULBM_EDEVICE, "advance failed: %s", hipGetErrorString(q));
        }
        b->completed = f.first;
        b->spare_events.push_back(f.second);
        b->inflight.pop_front();
    }
    if (b->inflight.empty()) b->completed = b->enqueued;
    for (size_t i = 0; i < b->old_graphs.size();) {
        if (b->old_graphs[i].first <= b->completed) {
            (void)hipGraphExecDestroy(b->old_graphs[i].second);
            b->old_graphs[i] = b->old_graphs.back();
            b->old_graphs.pop_back();
        } else {
            ++i;
        }
    }
    for (size_t i = 0; i < b->retiring.size();) {
        if (b->retiring[i].after <= b->completed) {
            arena_give(b, b->retiring[i].off, b->retiring[i].bytes);
            b->used -= b->retiring[i].bytes;
            b->retiring[i] = b->retiring.back();
            b->retiring.pop_back();
        } else {
            ++i;
        }
    }
    return PULBM_OK;
}

// Graphs of the old grid are destroyed once the advances queued so far, which
// may replay them, have completed.
void drop_graphs(pulbm_batch* b, pulbm_batch::Tab& t)
{
    for (auto& kv : t.graphs) b->old_graphs.emplace_back(b->enqueued, kv.second);
    t.graphs.clear();
}

int rebuild_tables(pulbm_batch* b)
{
    for (int di = 0; di < 6; ++di) {
        const int ls = di % 3 + 2, coll = di / 3;
        pulbm_batch::Tab& t = b->tab[di];
        if (t.cap == 0) {  // sized once for every slot
            t.cap = b->max_slots;
            HIPC(hipMalloc((void**)&t.dtab, t.cap * sizeof(CaseDev*)));
            HIPC(hipMalloc((void**)&t.dhdr, (t.cap + 3) * sizeof(int)));
            for (int k = 0; k < 2; ++k) {
                HIPC(hipHostMalloc((void**)&t.stage[k], t.cap * sizeof(CaseDev*) + (t.cap + 3) * sizeof(int),
                                   hipHostMallocDefault));
                HIPC(hipEventCreateWithFlags(&t.staged[k], hipEventDisableTiming));
            }
        }
        t.which ^= 1;
        HIPC(hipEventSynchronize(t.staged[t.which]));  // its last copy has executed
        CaseDev** ptr = (CaseDev**)t.stage[t.which];
        int* hdr = (int*)(t.stage[t.which] + t.cap * sizeof(CaseDev*));
        int n = 0;
        hdr[2] = 0;
        for (auto& s : b->slots)
            if (s.c && lattice_set(s.c->p.dim, s.c->p.q_hydro) == ls && s.c->p.collision == coll) {
                ptr[n] = s.c->d;
                hdr[3 + n] = hdr[2 + n] + s.c->ntiles;
                ++n;
            }
        t.ncases = n;
        t.tiles = hdr[2 + n];
        hdr[0] = n;
        hdr[1] = t.tiles;
        // every block of a launch that finds no tile still costs a dispatch,
        // so the captured grid follows the tile count: recapture when it no
        // longer covers the tiles or exceeds them by more than a quarter
        const int g = grid_of(t.tiles);
        if (n && (g > t.grid || 4 * t.grid > 5 * g)) {
            drop_graphs(b, t);
            t.grid = g;
        }
        if (n) HIPC(hipMemcpyAsync(t.dtab, ptr, n * sizeof(CaseDev*), hipMemcpyHostToDevice, b->stream));
        HIPC(hipMemcpyAsync(t.dhdr, hdr, (3 + n) * sizeof(int), hipMemcpyHostToDevice, b->stream));
        HIPC(hipEventRecord(t.staged[t.which], b->stream));
    }
    b->dirty = false;
    return PULBM_OK;
}

}  // namespace

extern "C" int pulbm_batch_create(size_t budget, int32_t store, int32_t max_slots, void* hip_stream,
                                  pulbm_batch** out)
{
    if (!out) return fail(PULBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (store < PULBM_STORE_FP64 || store > PULBM_STORE_BF16) return fail(PULBM_EINVAL, "bad store");
    if (max_slots < 1 || max_slots > 4096) return fail(PULBM_EINVAL, "max_slots must be in [1, 4096]");
    pulbm_batch* b = new (std::nothrow) pulbm_batch();
    if (!b) return fail(PULBM_ENOMEM, "host allocation failed");
    b->budget = budget;
    b->store = store;
    b->max_slots = max_slots;
    b->slots.resize(max_slots);
    hipError_t e = hipSuccess;
    if (budget) {
        e = hipMalloc((void**)&b->arena, budget);
        if (e != hipSuccess) {
            b->arena = nullptr;
            pulbm_batch_destroy(b);
            return fail(PULBM_ENOMEM, "batch arena of %zu bytes: %s", budget, hipGetErrorString(e));
        }
        b->holes[0] = budget;
    }
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {  // graph capture needs a stream other than the null stream
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        b->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e != hipSuccess) {
        pulbm_batch_destroy(b);
        return fail(PULBM_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return PULBM_OK;
}

extern "C" int pulbm_batch_admit(pulbm_batch* b, const pulbm_params* p, const double* phi, const double* P,
                                 const double* u, int64_t nsteps, int32_t* slot)
{
    if (!b || !slot) return fail(PULBM_EINVAL, "NULL argument");
    int rc = validate(p);
    if (rc) return rc;
    if (p->store != b->store) return fail(PULBM_EINVAL, "case store %d differs from the batch's %d", p->store, b->store);
    if (nsteps < 0) return fail(PULBM_EINVAL, "nsteps < 0");
    if ((rc = sync_advances(b, 0))) return rc;  // picks up released blocks
    const size_t bytes = align_up(make_layout(*p).total);
    int free_slot = -1;
    for (int i = 0; i < b->max_slots; ++i)
        if (!b->slots[i].c) { free_slot = i; break; }
    if (free_slot < 0) return fail(PULBM_EAGAIN, "no free slot");
    size_t off = 0;
    if (b->used + bytes > b->budget || !arena_take(b, bytes, &off))
        return fail(PULBM_EAGAIN, "needs %zu bytes, %zu of %zu free", bytes, b->budget - b->used, b->budget);
    // the case works on the side stream: its set-up overlaps the advances
    pulbm_case* c = nullptr;
    if ((rc = pulbm_create(p, b->arena + off, bytes, b->side, &c))) {
        arena_give(b, off, bytes);
        return rc;
    }
    rc = pulbm_init_fields(c, phi, P, u);
    if (!rc) {
        c->h.step_end = nsteps;
        rc = upload_desc(c);
    }
    if (!rc && hipStreamSynchronize(b->side) != hipSuccess) rc = fail(PULBM_EDEVICE, "case set-up failed");
    if (rc) {
        pulbm_destroy(c);
        arena_give(b, off, bytes);
        return rc;
    }
    pulbm_batch::Slot& s = b->slots[free_slot];
    s.c = c;
    s.end = nsteps;
    s.finish = nsteps == 0 ? 0 : -1;
    s.bytes = bytes;
    s.off = off;
    b->used += bytes;
    b->dirty = true;
    *slot = free_slot;
    return PULBM_OK;
}

extern "C" int pulbm_batch_advance(pulbm_batch* b, int32_t ksteps)
{
    if (!b) return fail(PULBM_EINVAL, "batch is NULL");
    if (ksteps < 1 || ksteps > 4096) return fail(PULBM_EINVAL, "ksteps must be in [1, 4096]");
    int rc = sync_advances(b, 0);
    if (rc) return rc;
    if (b->dirty && (rc = rebuild_tables(b))) return rc;
    for (int di = 0; di < 6; ++di) {
        pulbm_batch::Tab& t = b->tab[di];
        if (t.ncases == 0) continue;
        // the step parity of the table's unfinished cases at this advance's
        // first step: when they all agree (the usual case: cases start at step
        // 0 and advance by the same k), each step launches the collide kernel
        // of its parity only; when they differ, both (each skips the other's
        // tiles).  Finished cases run nothing, whatever their parity.
        int par = -2;
        for (auto& s : b->slots)
            if (s.c && s.c->step < s.end && lattice_set(s.c->p.dim, s.c->p.q_hydro) == di % 3 + 2 &&
                s.c->p.collision == di / 3) {
                const int p = (int)(s.c->step & 1);
                par = par == -2 ? p : (par == p ? p : -1);
            }
        if (par == -2) par = 0;
        const int key = ksteps * 4 + (par < 0 ? 2 : par);
        auto it = t.graphs.find(key);
        if (it == t.graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            HIPC(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < ksteps; ++k)
                for (int w = 0; w < kStepKernels; ++w)
                    launch(di % 3 + 2, b->store, di / 3 == 1, b->stream, t.dtab, t.dhdr, t.grid, k, w,
                           par < 0 ? -1 : (par + k) & 1);
            hipLaunchKernelGGL(k_advance, dim3((t.cap + 63) / 64), dim3(64), 0, b->stream, t.dtab, t.dhdr, ksteps);
            HIPC(hipStreamEndCapture(b->stream, &g));
            HIPC(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            (void)hipGraphDestroy(g);
            it = t.graphs.emplace(key, ge).first;
        }
        HIPC(hipGraphLaunch(it->second, b->stream));
    }
    hipEvent_t ev = nullptr;
    if (!b->spare_events.empty()) {
        ev = b->spare_events.back();
        b->spare_events.pop_back();
    } else {
        HIPC(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    HIPC(hipEventRecord(ev, b->stream));
    const int64_t seq = ++b->enqueued;
    b->inflight.emplace_back(seq, ev);
    // host bookkeeping of every resident case
    for (auto& s : b->slots)
        if (s.c) {
            const int64_t was = s.c->step;
            s.c->step = std::min<int64_t>(s.c->step + ksteps, s.end);
            s.c->h.step = s.c->step;
            if (was < s.end && s.c->step >= s.end) s.finish = seq;
        }
    return PULBM_OK;
}

extern "C" int pulbm_batch_poll(pulbm_batch* b, int32_t* done, int32_t cap, int32_t* ndone)
{
    if (!b || !ndone) return fail(PULBM_EINVAL, "NULL argument");
    // keep the newest advance queued while other cases still have steps to
    // run; wait for the ones before it
    bool pending = false;
    for (auto& s : b->slots)
        if (s.c && s.c->step < s.end) pending = true;
    int rc = sync_advances(b, pending ? b->enqueued - 1 : b->enqueued);
    if (rc) return rc;
    int k = 0;
    for (int i = 0; i < b->max_slots; ++i) {
        const pulbm_batch::Slot& s = b->slots[i];
        if (s.c && s.finish >= 0 && s.finish <= b->completed) {
            if (done && k < cap) done[k] = i;
            ++k;
        }
    }
    *ndone = k;
    return PULBM_OK;
}

extern "C" int pulbm_batch_take(pulbm_batch* b, int32_t slot, double* phi, double* P, double* u)
{
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].c) return fail(PULBM_EINVAL, "bad slot");
    pulbm_batch::Slot& s = b->slots[slot];
    int rc = PULBM_OK;
    if (s.finish < 0) {  // not finished: wait for everything queued
        if ((rc = sync_advances(b, b->enqueued))) return rc;
    } else if ((rc = sync_advances(b, s.finish))) {
        return rc;
    }
    // read on the side stream while later advances run (the case is idle in
    // them: its descriptor caps its steps)
    rc = pulbm_read_fields(s.c, phi, P, u);
    if (rc) return rc;
    pulbm_destroy(s.c);
    // advances already queued may still read the case's descriptor
    b->retiring.push_back({b->enqueued, s.off, s.bytes});
    s = pulbm_batch::Slot();
    b->dirty = true;
    return sync_advances(b, 0);
}

extern "C" int pulbm_batch_usage(const pulbm_batch* b, size_t* used, int32_t* active)
{
    if (!b) return fail(PULBM_EINVAL, "batch is NULL");
    if (used) *used = b->used;
    if (active) {
        int a = 0;
        for (auto& s : b->slots) a += s.c != nullptr;
        *active = a;
    }
    return PULBM_OK;
}

extern "C" void pulbm_batch_destroy(pulbm_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    for (auto& s : b->slots)
        if (s.c) pulbm_destroy(s.c);
    for (auto& t : b->tab) {
        for (auto& kv : t.graphs) (void)hipGraphExecDestroy(kv.second);
        if (t.dtab) (void)hipFree(t.dtab);
        if (t.dhdr) (void)hipFree(t.dhdr);
        for (int k = 0; k < 2; ++k) {
            if (t.stage[k]) (void)hipHostFree(t.stage[k]);
            if (t.staged[k]) (void)hipEventDestroy(t.staged[k]);
        }
    }
    for (auto& g : b->old_graphs) (void)hipGraphExecDestroy(g.second);
    for (auto& f : b->inflight) (void)hipEventDestroy(f.second);
    for (auto ev : b->spare_events) (void)hipEventDestroy(ev);
    if (b->arena) (void)hipFree(b->arena);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
}
