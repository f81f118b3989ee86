// Kernels of the coupled phase-field + P-u lattice Boltzmann step
// (Otomo et al., arXiv 2512.01027, Sec. II) for gfx950.
//
// One time step is four launches over every resident case:
//   k_moments  per node, no halo: gathers h and g (AA pattern) and writes
//              phi = sum h, u* = sum g c, P* = rho_ref T sum g (the pressure
//              the populations carry; the stored rest population lacks the
//              previous P, which is added back) and M2 = sum g c c (in
//              2-byte storage as 2-byte codes, two to a 32-bit word).
//   k_pressure 1-halo LDS tile: the pressure formula of Sec. II with K_i of
//              P* and, in the omega term, u* at x - c_i.  Link terms are
//              summed per shell in the auxiliary type (FP64 in FP64 storage,
//              FP32 otherwise); the shell-weighted sum and the final
//              combination are FP64.
//   k_velocity 1-halo LDS tile: u = sum_i (g_i + K_i) c_i with K_i of the new
//              pressure, i.e. u = u* - D P / rho.
//   k_collide  1-halo LDS tile of phi and u: the isotropic central
//              differences of phi, rho and u, the BGK phase-field collision
//              and the filter collision of the hydrodynamic LBE, written back
//              in place (AA pattern).  Cases without walls, open end or block
//              on D3Q19 or D2Q9 hydro (with 4- or 8-byte storage) rebuild u
//              here from u* and a 2-node halo of the new P, and a step skips
//              k_velocity.
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
//
// Addressing: case descriptors and tile tables are read through the
// constant address space (scalar loads, values in SGPRs); arrays are used
// through global-address-space pointers with 32-bit node indices.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "codec.hpp"
#include "lattice.hpp"

namespace pulbm {

// Per-case descriptor, resident in device memory (one per case of a launch).
struct CaseDev {
    int32_t nx, ny, nz, dim;
    int32_t wall[3];
    int32_t ntx, nty, ntz;  // tiles per axis
    int32_t delta_theta;
    int32_t sx;        // row pitch in nodes: nx rounded up to 32, so that every row of a
                       // tile starts on a 128-byte line (node n = x + sx (y + ny z))
    int64_t N;         // nodes per field including the row padding (sx ny nz)
    int64_t step;      // steps done
    int64_t step_end;  // the case is advanced while step < step_end
    void* h;           // Q_h * N populations (storage type)
    void* g;           // Q_g * N populations (storage type)
    void* P[2];        // pressure ping-pong: P[step & 1] is the previous-step pressure
    void* phi[2];      // N each: phi of this step's moments at phi[step & 1]; phi[(step + 1) & 1]
                       // keeps the previous step's, the reference of the 2-byte h codec
    void* J;           // dim*N  scratch: u* = sum g c
    void* Ps;          // N      scratch: P* = previous P + rho_ref T sum g, the pressure the
                       //        streamed populations carry (the rest population holds
                       //        g_0 - P/(rho_ref T), so the previous P is added back)
    void* M2;          // 3 (2D) or 6 (3D) * N scratch: sum g c c
    void* U[2];        // dim*N each: velocity of this step at U[step & 1]; U[(step + 1) & 1]
                       // keeps the previous step's, the second reference of the 2-byte codecs
    double rho_a, rho_w, tau_a, tau_w, tau_phi, M, W, sigma, lambda_b;
    double grav[3];
    double h_scale, h_inv_scale, g_scale, g_inv_scale;
    double p_top;           // pressure of an open high end (wall = 2 on the last axis)
    int32_t blk_lo[3], blk_hi[3];  // solid block, nodes lo <= x < hi (has_block)
    int32_t has_block;
    int32_t tband;  // tile rows per y band of the tile order (>= 1)
    int32_t fuse_u; // 1: the collide kernel rebuilds u itself and a step skips k_velocity
                    // (no wall, open end or block, 4- or 8-byte storage, every axis >= 3,
                    // D2Q9 or D3Q19 hydro)
    // The tile order's divisors -- ntx, tband ntz, tband and the last band's
    // rows -- as multipliers M = floor(2^40 / d) + 1 split into high and low
    // words, so that a block takes its tile apart with scalar multiplies:
    // n / d = (n Mh + mulhi(n, Ml)) >> 8, exact while n d < 2^40 (fastdiv
    // = 1, checked for every divisor against its largest dividend when the
    // case is created; otherwise the kernels divide).
    int32_t fastdiv;
    uint32_t dvh[4], dvl[4];
    int32_t tile_rev;  // 1: the case's tiles are taken in reverse order (a race check, pulbm_set_tile_order)
    int32_t nt_odd_moments;  // 1: k_moments streams its 4- and 8-byte loads on odd steps too
    // Constants of the collision derived once on the host (so no thread
    // divides in FP64): 1 / tau_phi, M / (T W), 48 sigma / W, 1.5 sigma W;
    // and every constant the FP32 kernels use, rounded once to FP32.
    double inv_tau_phi, theta0, sig48W, sigW15;
    struct {
        float rho_a, drho, tau_a, dtau, inv_tau_phi, theta0, sig48W, sigW15, lambda_b, grav[3];
        float h_scale, h_inv_scale, g_scale, g_inv_scale;
    } f32;
};

using CDesc = const PULBM_CST CaseDev;

template <class T> __device__ __forceinline__ PULBM_GLB T* glb(void* p) { return (PULBM_GLB T*)p; }

// A launch covers the tiles of every case in a table of case pointers.  The
// table's header lives in device memory next to it -- hdr[0] cases,
// hdr[1] tiles in all, hdr[2 + c] the first tile of case c -- so a captured
// graph stays valid while cases join and leave, as long as the grid has a
// block for every tile.
using CaseTab = CaseDev* const*;

// --------------------------------------------------------------- launch map

// Blocks are dealt to the 8 XCDs round-robin; remapping gives each XCD one
// contiguous run of tiles, so tiles that share halo planes share an L2.
// The grid is a multiple of 8.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// n / d for the multiplier (mh, ml) of d (CaseDev::dvh, dvl): the high word
// of n times the 40-bit multiplier, shifted down by 8.  n mh stays below 2^32
// for n < 2^23 (mh <= 256).
__device__ __forceinline__ uint32_t udiv_m(uint32_t n, uint32_t mh, uint32_t ml)
{
    return (n * mh + __umulhi(n, ml)) >> 8;
}

__device__ __forceinline__ int find_case(const PULBM_CST int* tstart, int ncases, int tile)
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
    CDesc* cs;
    int ox, oy, oz;  // tile origin
    int64_t step;
    bool active;
};

template <class Mo>
__device__ __forceinline__ TileCtx tile_ctx(CaseTab cases, const int* hdr_, int step_off)
{
    TileCtx t;
    const PULBM_CST int* hdr = (const PULBM_CST int*)hdr_;
    const int ncases = hdr[0], total_tiles = hdr[1];
    // the first blocks (a multiple of 8) take the tiles; the XCD remap runs
    // over them only, so every XCD gets its share however large the grid
    const int used = (total_tiles + 7) & ~7;
    t.active = (int)blockIdx.x < used;
    if (!t.active) return t;
    const int tile = xcd_tile(blockIdx.x, used);
    t.active = tile < total_tiles;
    if (!t.active) return t;
    const PULBM_CST int* tstart = hdr + 2;
    const int ci = find_case(tstart, ncases, tile);
    const PULBM_CST uint64_t* tab = (const PULBM_CST uint64_t*)(const void*)cases;
    t.cs = (CDesc*)(uintptr_t)tab[ci];
    CDesc& cs = *t.cs;
    // step_off < 0: read mode (the moment stage of the current state, run
    // whatever the case's step limit)
    t.step = cs.step + (step_off > 0 ? step_off : 0);
    t.active = step_off < 0 || t.step < cs.step_end;
    // tile order: x fastest, then z within a band of tband tile rows, then
    // the bands along y.  Tiles that share z-halo rows then run close together
    // (a band's width of tiles apart), while each plane is still read in runs
    // of whole rows.
    int lt = tile - tstart[ci];
    if (cs.tile_rev) lt = tstart[ci + 1] - tstart[ci] - 1 - lt;
    int tx, ty, tz;
    if (cs.fastdiv) {
        const uint32_t l = (uint32_t)lt;
        const uint32_t r = udiv_m(l, cs.dvh[0], cs.dvl[0]);
        tx = (int)(l - r * (uint32_t)cs.ntx);
        const uint32_t yb = udiv_m(r, cs.dvh[1], cs.dvl[1]);
        const uint32_t rem = r - yb * (uint32_t)(cs.tband * cs.ntz);
        const int rows = cs.nty - (int)yb * cs.tband;  // rows of this band: tband, or fewer in the last
        const int k = rows < cs.tband ? 3 : 2;
        const uint32_t tq = udiv_m(rem, cs.dvh[k], cs.dvl[k]);
        tz = (int)tq;
        ty = (int)yb * cs.tband + (int)(rem - tq * (uint32_t)min(cs.tband, rows));
    } else {
        tx = lt % cs.ntx;
        lt /= cs.ntx;
        const int yb = lt / (cs.tband * cs.ntz);
        const int rem = lt - yb * cs.tband * cs.ntz;
        const int by = min(cs.tband, cs.nty - yb * cs.tband);
        tz = rem / by;
        ty = yb * cs.tband + rem % by;
    }
    t.ox = tx * Mo::TX;
    t.oy = ty * Mo::TY;
    t.oz = tz * Mo::TZ;
    return t;
}

// Q slots of N elements of T (structure of arrays).  Addresses are formed as
// a uniform slot base (SGPRs) plus a 32-bit per-node byte offset, which maps
// onto the saddr + voffset form of the global memory instructions.
// Buffer load / store of populations: the slot's base and length sit in a
// buffer resource (SGPRs) and each lane supplies only its 32-bit byte offset.
// Through plain pointers the compiler forms every population address as a
// per-lane 64-bit sum; through buffer resources the collision kernel issues
// about 12% fewer vector instructions and keeps fewer registers live.  An
// offset past the slot would read 0 and write nothing (none is formed: every
// target node lies in the grid).  aux 2 marks the access non-temporal.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(PULBM_GLB char* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
template <bool NT, class T> __device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t boff)
{
    constexpr int aux = NT ? 2 : 0;
    if constexpr (sizeof(T) == 2) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)boff, 0, aux));
    else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, 0, aux));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)boff, 0, aux));
}
template <bool NT, class T> __device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t boff, T v)
{
    constexpr int aux = NT ? 2 : 0;
    if constexpr (sizeof(T) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)boff, 0, aux);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)boff, 0, aux);
    } else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)boff, 0, aux);
    }
}

template <class T>
struct Slots {
    PULBM_GLB char* base;
    uint64_t slot_bytes;  // N * sizeof(T), below 2^31
    __device__ __forceinline__ PULBM_GLB T* at(int slot, uint32_t boff) const
    {
        return (PULBM_GLB T*)(base + (uint64_t)slot * slot_bytes + boff);
    }
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int slot) const
    {
        return buf_rsrc(base + (uint64_t)slot * slot_bytes, (uint32_t)slot_bytes);
    }
};

template <class T> __device__ __forceinline__ Slots<T> slots(void* p, int64_t N)
{
    Slots<T> s;
    s.base = (PULBM_GLB char*)p;
    s.slot_bytes = (uint64_t)N * sizeof(T);
    return s;
}

// M2, the second moment of g that the moment stage writes and the collision
// reads once, is kept in the compute type, except in 2-byte storage: there
// each component is encoded with g's codec and scale (no shift) and two of
// them share a 32-bit word (word j holds components 2j and 2j + 1, the first
// in the low half), so a node's six values take three loads and three
// registers.
template <class S> __device__ __forceinline__ uint32_t m2_pack(S lo, S hi)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}
template <class S> __device__ __forceinline__ S m2_half(uint32_t w, int k)
{
    return __builtin_bit_cast(S, (uint16_t)(k ? w >> 16 : w & 0xffffu));
}

template <class T> __device__ __forceinline__ PULBM_GLB T* at_node(void* p, uint32_t n)
{
    return (PULBM_GLB T*)((PULBM_GLB char*)p + n * (uint32_t)sizeof(T));
}

// Neighbour navigation of one node: byte offsets (elements of ESZ bytes) of a
// -1/0/+1 step along each axis (periodic wrap included) and which steps
// leave through a wall.
struct Nav {
    int o[3][3];
    uint32_t solid;  // bit 2a: the -1 step on axis a is outside a wall; bit 2a+1: the +1 step
    uint32_t open;   // the same bits for a step out through an open end
    uint32_t blk[3]; // bit k: coordinate + k - 1 on axis a lies in the block's range
};

// Is node (x, y, z) inside the solid block?
__device__ __forceinline__ bool in_block(CDesc& cs, int x, int y, int z)
{
    return cs.has_block && x >= cs.blk_lo[0] && x < cs.blk_hi[0] && y >= cs.blk_lo[1] && y < cs.blk_hi[1] &&
           z >= cs.blk_lo[2] && z < cs.blk_hi[2];
}

__device__ __forceinline__ Nav make_nav(CDesc& cs, int x, int y, int z, int esz)
{
    Nav v;
    const int p[3] = {x, y, z};
    const int n[3] = {cs.nx, cs.ny, cs.nz};
    const int st[3] = {esz, esz * cs.sx, esz * cs.sx * cs.ny};
    v.solid = 0;
    v.open = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.o[a][1] = 0;
        v.o[a][0] = (p[a] == 0) ? (n[a] - 1) * st[a] : -st[a];
        v.o[a][2] = (p[a] == n[a] - 1) ? -(n[a] - 1) * st[a] : st[a];
        if (cs.wall[a]) {
            if (p[a] == 0) v.solid |= 1u << (2 * a);
            if (p[a] == n[a] - 1) {
                if (cs.wall[a] == 2) v.open |= 1u << (2 * a + 1);
                else v.solid |= 1u << (2 * a + 1);
            }
        }
        // a block spanning a whole periodic axis holds every coordinate
        const bool full = cs.blk_lo[a] == 0 && cs.blk_hi[a] == n[a];
        v.blk[a] = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int q = p[a] + k - 1;
            if (cs.has_block && (full || (q >= cs.blk_lo[a] && q < cs.blk_hi[a]))) v.blk[a] |= 1u << k;
        }
    }
    return v;
}

// Nav of a node whose neighbours all lie inside the grid (no wall, block or
// wrap within one node): the offsets are the strides, the same for every
// node of the workgroup.
__device__ __forceinline__ Nav make_nav_inner(CDesc& cs, int esz)
{
    Nav v;
    const int st[3] = {esz, esz * cs.sx, esz * cs.sx * cs.ny};
    v.solid = 0;
    v.open = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.o[a][0] = -st[a];
        v.o[a][1] = 0;
        v.o[a][2] = st[a];
        v.blk[a] = 0;
    }
    return v;
}

template <class L>
__device__ __forceinline__ int nav_off(const Nav& v, int i, int sgn)
{
    return v.o[0][sgn * L::c(i, 0) + 1] + v.o[1][sgn * L::c(i, 1) + 1] + v.o[2][sgn * L::c(i, 2) + 1];
}

template <class L> __device__ __forceinline__ uint32_t nav_mask(int i, int sgn)
{
    uint32_t m = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int ca = sgn * L::c(i, a);
        if (ca == -1) m |= 1u << (2 * a);
        if (ca == 1) m |= 1u << (2 * a + 1);
    }
    return m;
}

// Does the step along sgn c_i leave through the open end?
template <class L>
__device__ __forceinline__ bool nav_open(const Nav& v, int i, int sgn)
{
    return (v.open & nav_mask<L>(i, sgn)) != 0;
}

// Does the step along sgn c_i leave the fluid (through a wall or the open
// end, or into the block)?  Its population then stays at the node, in the
// slot of the opposite direction.
template <class L>
__device__ __forceinline__ bool nav_solid(const Nav& v, int i, int sgn)
{
    const bool blk = ((v.blk[0] >> (sgn * L::c(i, 0) + 1)) & (v.blk[1] >> (sgn * L::c(i, 1) + 1)) &
                      (v.blk[2] >> (sgn * L::c(i, 2) + 1)) & 1u) != 0;
    return ((v.solid | v.open) & nav_mask<L>(i, sgn)) != 0 || blk;
}

// Does the tile (or its ghost layer) touch a wall, the open end or the
// block?  Uniform per block; tiles that do not skip every boundary test.
template <class Mo>
__device__ __forceinline__ bool tile_at_wall(CDesc& cs, int ox, int oy, int oz)
{
    const bool blk = cs.has_block && ox - 1 < cs.blk_hi[0] && ox + Mo::TX >= cs.blk_lo[0] && oy - 1 < cs.blk_hi[1] &&
                     oy + Mo::TY >= cs.blk_lo[1] && oz - 1 < cs.blk_hi[2] && oz + Mo::TZ >= cs.blk_lo[2];
    return (cs.wall[0] && (ox == 0 || ox + Mo::TX >= cs.nx)) || (cs.wall[1] && (oy == 0 || oy + Mo::TY >= cs.ny)) ||
           (cs.wall[2] && (oz == 0 || oz + Mo::TZ >= cs.nz)) || blk;
}

// Population loads and stores.  The populations of a step are read once and
// written once, and at the sizes that matter the state is far larger than the
// caches, so accesses can be marked non-temporal.  Which accesses gain from it
// was measured per storage width (bit 0: loads in k_moments, bit 1: loads in
// k_collide, bit 2: stores in k_collide, bit 3: loads in k_moments on even
// steps only): populations of every width stream the collide's loads, the
// collide's stores on even steps (odd-step stores stay in L2, see
// collide_tile) and k_moments' loads on even steps: on odd steps, shifted by
// one node in x, a line is read partly by one tile and partly by its x
// neighbour, and streamed past L2 it is fetched twice.  Wide populations of
// a small grid stream on odd steps too (CaseDev::nt_odd_moments): the
// second fetch then hits the last-level cache.
// The per-node fields a kernel reads only at its own nodes (the codecs'
// previous-step phi and u, the previous P, u*, phi and M2 where no halo of
// them is taken) are loaded non-temporal too (FP16 step 3.03 -> 2.99 ms).
enum PopAccess { kLoadMoments = 1, kLoadCollide = 2, kStoreCollide = 4, kLoadMomentsEven = 8 };
constexpr int kNtWide = kLoadMomentsEven | kLoadCollide | kStoreCollide, kNtHalf = kNtWide;
template <class S, int A> constexpr bool nt_access() { return ((sizeof(S) >= 4 ? kNtWide : kNtHalf) & A) != 0; }

// Population arriving at the node (byte offset nb) along direction i.
template <class L, bool WALL, bool NT, class S>
__device__ __forceinline__ S aa_load(const Slots<S>& f, uint32_t nb, const Nav& v, int i, bool odd)
{
    if (!odd) return buf_ld<NT, S>(f.rsrc(i), nb);
    if (WALL && nav_solid<L>(v, i, -1)) return buf_ld<NT, S>(f.rsrc(i), nb);  // reflected at a wall last step
    return buf_ld<NT, S>(f.rsrc(opp(i)), nb + (uint32_t)nav_off<L>(v, i, -1));
}

// Store the node's post-collision population i where it streams to; a
// population leaving through a wall goes to the slot the node reads back as
// the reflected direction.
template <class L, bool WALL, bool NT, class S>
__device__ __forceinline__ void aa_store(const Slots<S>& f, uint32_t nb, const Nav& v, int i, bool odd, S val,
                                         bool bb)
{
    if (!odd || (WALL && bb)) buf_st<NT, S>(f.rsrc(opp(i)), nb, val);
    else buf_st<NT, S>(f.rsrc(i), nb + (uint32_t)nav_off<L>(v, i, +1), val);
}

// ---------------------------------------------------------- tile regions

// Resolve global coordinate t on an axis of n nodes: periodic wrap, or the
// mirror node of a ghost outside a wall (off = t - mirror).  A ghost beyond
// an open end (wall = 2, high side) takes the nearest node too, marked by
// kOpenGhost in *crossed instead of counting as a wall crossing.
// Branch-free, without division: a 1-node halo reaches at most one node past
// either end, where one +-n wraps exactly.  Cells further out belong only to
// the halo of nodes outside the grid (a ragged last tile); they are kept
// inside the grid by the clamp and their values are never used.
constexpr int kOpenGhost = 256;
__device__ __forceinline__ int resolve_axis(int t, int n, int wall, int* off, int* crossed)
{
    const bool lo = t < 0, hi = t >= n;
    const int near = lo ? 0 : (hi ? n - 1 : t);
    const int wrapped = min(lo ? t + n : (hi ? t - n : t), n - 1);
    *off = wall ? t - near : 0;
    *crossed += (wall && (lo || hi)) ? ((wall == 2 && hi) ? kOpenGhost : 1) : 0;
    return wall ? near : wrapped;
}

template <int RX, int RY, int RZ>
struct Region {
    static constexpr int N = RX * RY * RZ;
    __device__ static __forceinline__ int idx(int ix, int iy, int iz) { return ix + RX * (iy + RY * iz); }
    // The 3x3(x3) neighbourhood of cell (cx, cy, cz): its lowest corner
    // (cx - 1, cy - 1, cz - ZL) as a base index, and each cell of it at a
    // constant offset from there that is never negative, which LDS reads
    // take as their immediate (DS offsets are unsigned).
    template <int ZL>
    __device__ static __forceinline__ int nb_base(int cx, int cy, int cz) { return idx(cx - 1, cy - 1, cz - ZL); }
    template <int ZL>
    static constexpr int nb(int dx, int dy, int dz) { return (1 + dx) + RX * ((1 + dy) + RY * (ZL + dz)); }
};

// 1-halo region of a tile: cell k -> mirror node index, wall offsets, crossings.
template <class Mo, int DIMV>
struct Halo1 {
    static constexpr int D = 1;  // halo depth
    static constexpr int ZH = DIMV == 3 ? 1 : 0;
    static constexpr int RX = Mo::TX + 2, RY = Mo::TY + 2, RZ = Mo::TZ + 2 * ZH;
    using R = Region<RX, RY, RZ>;
    // BND: the tile touches a wall, the open end or the block (tiles that do
    // not never meet the block, and skip its test)
    template <bool BND = true>
    __device__ static __forceinline__ uint32_t cell(CDesc& cs, const TileCtx& t, int k, int off[3], int* cr)
    {
        const int ix = k % RX, iy = (k / RX) % RY, iz = k / (RX * RY);
        *cr = 0;
        int m[3];
        m[0] = resolve_axis(t.ox - 1 + ix, cs.nx, cs.wall[0], &off[0], cr);
        m[1] = resolve_axis(t.oy - 1 + iy, cs.ny, cs.wall[1], &off[1], cr);
        m[2] = resolve_axis(t.oz - ZH + iz, cs.nz, cs.wall[2], &off[2], cr);
        if (BND && in_block(cs, m[0], m[1], m[2])) {
            // a block node mirrors across each exposed face it lies on
            const int n[3] = {cs.nx, cs.ny, cs.nz};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (m[a] == cs.blk_lo[a] && cs.blk_lo[a] >= 1) {
                    m[a] -= 1;
                    off[a] += 1;
                    *cr += 1;
                } else if (m[a] == cs.blk_hi[a] - 1 && cs.blk_hi[a] <= n[a] - 1) {
                    m[a] += 1;
                    off[a] -= 1;
                    *cr += 1;
                }
            }
        }
        return (uint32_t)m[0] + (uint32_t)cs.sx * ((uint32_t)m[1] + (uint32_t)cs.ny * (uint32_t)m[2]);
    }
};

// 2-halo region of a tile on a grid without walls, open end or block and
// with every axis of at least 3 nodes, so that one +-n wraps a coordinate
// two nodes past either end.
template <class Mo, int DIMV>
struct Halo2 {
    static constexpr int D = 2;
    static constexpr int ZH = DIMV == 3 ? 2 : 0;
    static constexpr int RX = Mo::TX + 4, RY = Mo::TY + 4, RZ = Mo::TZ + 2 * ZH;
    using R = Region<RX, RY, RZ>;
    template <bool BND = false>
    __device__ static __forceinline__ uint32_t cell(CDesc& cs, const TileCtx& t, int k, int off[3], int* cr)
    {
        static_assert(!BND, "periodic grids only");
        const int ix = k % RX, iy = (k / RX) % RY, iz = k / (RX * RY);
        *cr = 0;
        const int x = resolve_axis(t.ox - 2 + ix, cs.nx, 0, &off[0], cr);
        const int y = resolve_axis(t.oy - 2 + iy, cs.ny, 0, &off[1], cr);
        const int z = resolve_axis(t.oz - ZH + iz, cs.nz, 0, &off[2], cr);
        return (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
    }
};

// Fills a tile's halo region in LDS (HR: Halo1, or Halo2 two nodes deep)
// from NV arrays (src[j]: node-indexed array of CT).  store(k, cr, off, v)
// writes cell k from the NV values v of its node, with the crossing flags and
// wall offsets of HR::cell.
//
// A tile clear of walls, the open end and the block whose x range lies in the
// grid takes the row path: each halo row's TX interior cells are read as
// aligned 4-element vectors (tile origins and row pitches are multiples of 32
// nodes), its D end cells on either side one by one.  Only y and z wrap, once
// per row.
//
// Other tiles take the cell path: each thread takes the cells
// k = threadIdx.x + 256 it, resolves all of them and issues all their loads
// before the first LDS write, so they are in flight together.  Cells past the
// region repeat its last cell, and write it too, with the same values as its
// owner: control flow stays uniform, so no load is sunk into a conditional
// store.
//
// Tiles at a wall or the open end (WALL) take the row path too, as long as
// their halo region keeps clear of the block: a halo row beyond a wall or the
// open end is the mirror row (resolve_axis, with the row's offsets and
// crossings), and so is an end cell beyond a wall in x; the cells within a
// row share the row's y and z resolution.
template <class HR, bool WALL, int NV, class CT, class StoreF>
__device__ __forceinline__ void halo_rows(CDesc& cs, const TileCtx& t, void* const* src, StoreF store)
{
    using R = typename HR::R;
    constexpr int DH = HR::D, TX = HR::RX - 2 * DH, ROWS = HR::RY * HR::RZ, LPR = TX / 4;
    constexpr int NVEC = ROWS * LPR, NEDGE = 2 * DH * ROWS;
    constexpr int PV = (NVEC + 255) / 256, PE = (NEDGE + 255) / 256;
    static_assert(TX % 4 == 0, "rows of 4-element vectors");
    static_assert(!WALL || DH == 1, "walls mirror one ghost layer");
    typedef CT V4 __attribute__((ext_vector_type(4)));
    const int tid = (int)threadIdx.x;
    // node index of the start of halo row r, its first LDS cell, and (at
    // walls) the row's wall offsets and crossings
    auto row_of = [&](int r, int* kr, int* off, int* cr) {
        const int iy = r % HR::RY, iz = r / HR::RY;
        int y = t.oy - DH + iy, z = t.oz - HR::ZH + iz;
        off[0] = off[1] = off[2] = 0;
        *cr = 0;
        if constexpr (WALL) {
            y = resolve_axis(y, cs.ny, cs.wall[1], &off[1], cr);
            z = resolve_axis(z, cs.nz, cs.wall[2], &off[2], cr);
        } else {
            y += y < 0 ? cs.ny : (y >= cs.ny ? -cs.ny : 0);
            y = min(y, cs.ny - 1);
            z += z < 0 ? cs.nz : (z >= cs.nz ? -cs.nz : 0);
            z = min(z, cs.nz - 1);
        }
        *kr = R::idx(0, iy, iz);
        return (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
    };
    // items past the last one repeat it (same loads, same LDS cells, same
    // values), so every load is unconditional and issued before any store
    V4 v[PV][NV];
    int kv[PV], crv[PV], offv[PV][3];
#pragma unroll
    for (int p = 0; p < PV; ++p) {
        const int it = min(tid + 256 * p, NVEC - 1);
        const int q = it % LPR;
        int kr;
        const uint32_t m = row_of(it / LPR, &kr, offv[p], &crv[p]) + (uint32_t)(t.ox + 4 * q);
        kv[p] = kr + DH + 4 * q;
#pragma unroll
        for (int j = 0; j < NV; ++j) v[p][j] = *(const PULBM_GLB V4*)at_node<CT>(src[j], m);
    }
    CT e[PE][NV];
    int ke[PE], cre[PE], offe[PE][3];
#pragma unroll
    for (int p = 0; p < PE; ++p) {
        const int it = min(tid + 256 * p, NEDGE - 1);
        const int side = it % (2 * DH);  // 0 .. DH-1 before the row, DH .. 2DH-1 after it
        int kr;
        const uint32_t row = row_of(it / (2 * DH), &kr, offe[p], &cre[p]);
        int x = side < DH ? t.ox - DH + side : t.ox + TX + side - DH;
        if constexpr (WALL) {
            x = resolve_axis(x, cs.nx, cs.wall[0], &offe[p][0], &cre[p]);
        } else {
            x += x < 0 ? cs.nx : (x >= cs.nx ? -cs.nx : 0);
            x = min(x, cs.nx - 1);
        }
        ke[p] = kr + (side < DH ? side : TX + side);
#pragma unroll
        for (int j = 0; j < NV; ++j) e[p][j] = *at_node<CT>(src[j], row + (uint32_t)x);
    }
#pragma unroll
    for (int p = 0; p < PV; ++p)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            CT w[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) w[j] = v[p][j][c];
            store(kv[p] + c, crv[p], offv[p], w);
        }
#pragma unroll
    for (int p = 0; p < PE; ++p) store(ke[p], cre[p], offe[p], e[p]);
}

// Does the halo region of a tile reach a node of the block?
template <class HR>
__device__ __forceinline__ bool halo_near_block(CDesc& cs, const TileCtx& t)
{
    constexpr int DH = HR::D, TX = HR::RX - 2 * DH, TY = HR::RY - 2 * DH, TZ = HR::RZ - 2 * HR::ZH;
    return cs.has_block && t.ox - DH < cs.blk_hi[0] && t.ox + TX + DH > cs.blk_lo[0] &&
           t.oy - DH < cs.blk_hi[1] && t.oy + TY + DH > cs.blk_lo[1] && t.oz - HR::ZH < cs.blk_hi[2] &&
           t.oz + TZ + HR::ZH > cs.blk_lo[2];
}

template <class HR, bool WALL, int NV, class CT, class StoreF>
__device__ __forceinline__ void halo_stage(CDesc& cs, const TileCtx& t, void* const* src, StoreF store)
{
    if (t.ox + HR::RX - 2 * HR::D <= cs.nx) {
        if constexpr (!WALL) {
            halo_rows<HR, false, NV, CT>(cs, t, src, store);
            return;
        } else {
            if (!halo_near_block<HR>(cs, t)) {
                halo_rows<HR, true, NV, CT>(cs, t, src, store);
                return;
            }
        }
    }
    constexpr int RN = HR::R::N;
    constexpr int NIT = (RN + 255) / 256;
    CT v[NIT][NV];
    int cr[NIT], off[NIT][3];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int k = min((int)threadIdx.x + 256 * it, RN - 1);
        const uint32_t m = HR::template cell<WALL>(cs, t, k, off[it], &cr[it]);
#pragma unroll
        for (int j = 0; j < NV; ++j) v[it][j] = *at_node<CT>(src[j], m);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) store(min((int)threadIdx.x + 256 * it, RN - 1), cr[it], off[it], v[it]);
}

// ------------------------------------------------------------ physics

template <class CT> __device__ __forceinline__ CT rcp(CT x) { return (CT)1 / x; }
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <class CT> __device__ __forceinline__ CT sqrt_(CT x) { return sqrt(x); }
template <> __device__ __forceinline__ float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

template <class CT>
struct Phys {
    CT rho_a, drho, tau_a, dtau, inv_tau_phi;
    CT theta0;   // M / (T W)
    CT sig48W;   // 48 sigma / W
    CT sigW15;   // 3 sigma W / 2
    CT lambda_b;
    CT grav[3];
    int delta_theta;
};

// A case constant in the compute type: the host's FP32 copy for FP32
// arithmetic, the FP64 value otherwise.
template <class CT> __device__ __forceinline__ CT cconst(double d, float f)
{
    if constexpr (std::is_same_v<CT, float>) return f;
    else return (CT)d;
}

template <class CT>
__device__ __forceinline__ Phys<CT> make_phys(CDesc& cs)
{
    Phys<CT> p;
    p.rho_a = cconst<CT>(cs.rho_a, cs.f32.rho_a);
    p.drho = cconst<CT>(cs.rho_w - cs.rho_a, cs.f32.drho);
    p.tau_a = cconst<CT>(cs.tau_a, cs.f32.tau_a);
    p.dtau = cconst<CT>(cs.tau_w - cs.tau_a, cs.f32.dtau);
    p.inv_tau_phi = cconst<CT>(cs.inv_tau_phi, cs.f32.inv_tau_phi);
    p.theta0 = cconst<CT>(cs.theta0, cs.f32.theta0);
    p.sig48W = cconst<CT>(cs.sig48W, cs.f32.sig48W);
    p.sigW15 = cconst<CT>(cs.sigW15, cs.f32.sigW15);
    p.lambda_b = cconst<CT>(cs.lambda_b, cs.f32.lambda_b);
#pragma unroll
    for (int a = 0; a < 3; ++a) p.grav[a] = cconst<CT>(cs.grav[a], cs.f32.grav[a]);
    p.delta_theta = cs.delta_theta;
    return p;
}

template <class CT> __device__ __forceinline__ CT clamp01(CT v) { return v < (CT)0 ? (CT)0 : (v > (CT)1 ? (CT)1 : v); }

// Local macroscopic values and gradients of one node.
template <class CT>
struct NodeVals {
    CT phi, u[3], gphi[3], lphi, grho[3], G[3][3];  // G[a][b] = d u_a / d x_b
};

// Macroscopic part of the collision of one node (everything but the
// per-direction loops): phase-field theta and normal, hydrodynamic force,
// first moment of g^eq, B div u and the non-equilibrium momentum flux Pi.
template <int DIMV, class CT>
struct NodeCoef {
    CT theta, nv[3];     // phase field
    CT base_h;           // 1 - u^2 / (2T)
    CT rho, F[3];        // for the wall correction
    CT av[3];            // u + F / rho + sigma . grad rho / rho^2
    CT gbase;            // B div / T - u^2 / (2T)
    CT Bdiv;
    // (1 - 1/tau) / (2 T^2) * Pi: its diagonal, twice its off-diagonal
    // entries (xy, xz, yz), and * T tr(Pi)
    CT kPi[3], kPi2[3], kTr;
};

template <int DIMV, bool INIT, class CT>
__device__ __forceinline__ NodeCoef<DIMV, CT> node_coef(const Phys<CT>& p, const NodeVals<CT>& v,
                                                        const CT* __restrict__ M2)
{
    constexpr int D = DIMV;
    const CT T = (CT)kT, i2T2 = (CT)4.5, i2T = (CT)1.5, iT = (CT)3.0;
    const CT eps = (CT)1.0e-10;
    NodeCoef<DIMV, CT> k;
    const CT phi = v.phi;
    // phase field: normal, theta (+ delta theta)
    CT gn2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) gn2 += v.gphi[a] * v.gphi[a];
    const CT gn = sqrt_(gn2);
    const CT inv_n = rcp(gn + eps);
#pragma unroll
    for (int a = 0; a < 3; ++a) k.nv[a] = a < D ? v.gphi[a] * inv_n : (CT)0;
    const CT dphi = phi - (CT)0.5;
    CT theta = p.theta0 * ((CT)1 - (CT)4 * dphi * dphi);
    if (p.delta_theta) {
        const CT s = v.lphi * rcp(fabs(v.lphi) + eps);
        const CT iD = (CT)1.0e4;
        const CT Y1 = fmin(clamp01((phi - (CT)0.8) * iD), clamp01(-(phi - (CT)1) * iD));
        const CT Y2 = fmin(clamp01(phi * iD), clamp01(-(phi - (CT)0.2) * iD));
        theta += (CT)(-22.5) * p.theta0 * gn * (((CT)1 + s) * Y1 + ((CT)1 - s) * Y2);
    }
    k.theta = theta;
    CT u2 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) u2 += v.u[a] * v.u[a];
    k.base_h = (CT)1 - u2 * i2T;
    // hydrodynamics
    const CT pc = clamp01(phi);
    const CT rho = p.rho_a + pc * p.drho;
    const CT tau = p.tau_a + pc * p.dtau;
    const CT nu = T * (tau - (CT)0.5);
    const CT mu = p.sig48W * phi * (phi - (CT)1) * dphi - p.sigW15 * v.lphi;
    const CT irho = rcp(rho);
    k.rho = rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) k.F[a] = a < D ? rho * p.grav[a] + mu * v.gphi[a] : (CT)0;
    CT div = v.G[0][0];
#pragma unroll
    for (int a = 1; a < D; ++a) div += v.G[a][a];
    const CT bulk = rho * (CT)(2.0 / 3.0) * (p.lambda_b - nu) * div;
    const CT rnu = rho * nu;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l >= D) { k.av[l] = 0; continue; }
        CT sg = 0;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            CT s_lm = rnu * (v.G[l][m] + v.G[m][l]);
            if (l == m) s_lm += bulk;
            sg += s_lm * v.grho[m];
        }
        k.av[l] = v.u[l] + (k.F[l] + sg * irho) * irho;
    }
    const CT B = (CT)(2.0 / 3.0) * (nu - p.lambda_b) + T * (CT)0.5;
    k.Bdiv = B * div;
    k.gbase = k.Bdiv * iT - u2 * i2T;
#pragma unroll
    for (int a = 0; a < 3; ++a) k.kPi[a] = k.kPi2[a] = 0;
    k.kTr = 0;
    if (!INIT) {
        // Pi = sum c c (g - g^eq) = M2 - (u u + B div I) on these lattices;
        // diagonal entries, then xy, xz, yz (M2 holds xx, yy, [zz,] xy[, xz, yz])
        CT Pd[3] = {0, 0, 0}, Po[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < D; ++a) Pd[a] = M2[a] - v.u[a] * v.u[a] - k.Bdiv;
        Po[0] = M2[D] - v.u[0] * v.u[1];
        if (D == 3) {
            Po[1] = M2[4] - v.u[0] * v.u[2];
            Po[2] = M2[5] - v.u[1] * v.u[2];
        }
        const CT kf = ((CT)1 - rcp(tau)) * i2T2;
        CT tr = Pd[0];
#pragma unroll
        for (int a = 1; a < D; ++a) tr += Pd[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            k.kPi[a] = kf * Pd[a];
            k.kPi2[a] = (kf + kf) * Po[a];
        }
        k.kTr = kf * T * tr;
    }
    return k;
}

// c_i . x over the axes where direction j of lattice L is nonzero, started
// from the first such term: an accumulator started at zero costs one more
// add per sum (0 + x is not x when x is -0, so the compiler keeps the add).
template <class L, int D, class CT>
__device__ __forceinline__ CT c_dot(int j, const CT* x)
{
    CT s = 0;
    bool first = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int c = L::c(j, a);
        if (c == 0) continue;
        s = first ? (c == 1 ? x[a] : -x[a]) : (c == 1 ? s + x[a] : s - x[a]);
        first = false;
    }
    return s;
}

// h^eq_j (INIT) or the BGK post-collision h*_j from the incoming h_j.
template <class H, int D, bool INIT, class CT>
__device__ __forceinline__ CT h_out(const Phys<CT>& p, const NodeVals<CT>& v, const NodeCoef<D, CT>& k, int j,
                                    CT hj)
{
    const CT cu = c_dot<H, D>(j, v.u), cn = c_dot<H, D>(j, k.nv);
    const CT wj = (CT)H::w(j);
    const CT heq = wj * (v.phi * (k.base_h + cu * (CT)3.0 + cu * cu * (CT)4.5) + k.theta * cn);
    return INIT ? heq : hj + (heq - hj) * p.inv_tau_phi;
}

// The part of g^eq_i (INIT) or of the filtered g*_i that is even in c_i,
// before the weight: 4.5 (c_i.u)^2 + B div u / T - u^2 / (2T), and when
// filtered c_i.kPi.c_i - T tr(kPi).  c_i.kPi.c_i is summed as the diagonal
// entries of the axes c_i spans, then the off-diagonal ones (kPi2 = 2 kPi),
// so that directions spanning the same axes share one diagonal sum.
template <class G, int D, bool INIT, class CT>
__device__ __forceinline__ CT g_even(const NodeCoef<D, CT>& k, int i, CT cu)
{
    CT e = k.gbase;
    if (!INIT) {
        e = e - k.kTr;
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (G::c(i, a) != 0) e = e + k.kPi[a];
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a + 1; b < D; ++b) {
                const int cc = G::c(i, a) * G::c(i, b);
                const CT p2 = k.kPi2[a + b - 1];  // (0,1) -> 0, (0,2) -> 1, (1,2) -> 2
                if (cc == 1) e = e + p2;
                if (cc == -1) e = e - p2;
            }
    }
    return cu * cu * (CT)4.5 + e;
}

// g^eq_i (INIT) or the filtered post-collision g*_i; the rest entry excludes
// the P / (rho_ref T) part.
template <class G, int D, bool INIT, class CT>
__device__ __forceinline__ CT g_out(const NodeVals<CT>& v, const NodeCoef<D, CT>& k, int i)
{
    const CT wi = (CT)G::w(i);
    const CT ca = c_dot<G, D>(i, k.av), cu = c_dot<G, D>(i, v.u);
    CT geq = wi * (g_even<G, D, INIT>(k, i, cu) + ca * (CT)3.0);
    if (i == 0) geq -= k.Bdiv * (CT)3.0;
    return geq;
}

// Opposite directions i and i+1 (i odd) have c_{i+1} = -c_i: the terms odd in
// c change sign and the even ones do not, so each pair shares one evaluation.
// The products of the weight with per-node values (w phi, w theta, ...) are
// written alike in every pair, so directions of one weight share them.
// h^eq (INIT) or the BGK post-collision h* for the pair (j, j+1).
template <class H, int D, bool INIT, class CT>
__device__ __forceinline__ void h_pair(const Phys<CT>& p, const NodeVals<CT>& v, const NodeCoef<D, CT>& k,
                                       int j, CT hj, CT hk, CT* oj, CT* ok)
{
    const CT cu = c_dot<H, D>(j, v.u), cn = c_dot<H, D>(j, k.nv);
    const CT pw = (CT)H::w(j) * v.phi;
    const CT even = cu * cu * (pw * (CT)4.5) + pw * k.base_h;
    const CT odd = cu * (pw * (CT)3.0) + ((CT)H::w(j) * k.theta) * cn;
    const CT ej = even + odd, ek = even - odd;
    *oj = INIT ? ej : hj + (ej - hj) * p.inv_tau_phi;
    *ok = INIT ? ek : hk + (ek - hk) * p.inv_tau_phi;
}

// g^eq (INIT) or the filtered post-collision g* for the pair (i, i+1).
template <class G, int D, bool INIT, class CT>
__device__ __forceinline__ void g_pair(const NodeVals<CT>& v, const NodeCoef<D, CT>& k, int i, CT* oi, CT* ok)
{
    const CT wi = (CT)G::w(i);
    const CT ca = c_dot<G, D>(i, k.av), cu = c_dot<G, D>(i, v.u);
    const CT we = wi * g_even<G, D, INIT>(k, i, cu);
    const CT w3 = wi * (CT)3.0;
    *oi = ca * w3 + we;
    *ok = we - ca * w3;
}

// Isotropic central differences (Sec. II) of a tile field at cell (cx,cy,cz):
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


template <class Mo>
__device__ __forceinline__ void local_xyz(int* lx, int* ly, int* lz)
{
    *lx = threadIdx.x % Mo::TX;
    *ly = (threadIdx.x / Mo::TX) % Mo::TY;
    *lz = threadIdx.x / (Mo::TX * Mo::TY);
}

// ================================================================ kernels

// phi of this node one step earlier: the reference of the incoming h in
// 2-byte storage (wider storage keeps h as it is and reads nothing).
template <class S, class CT = typename Codec<S>::CT>
__device__ __forceinline__ CT h_reference(void* phi_prev, uint32_t n)
{
    if constexpr (sizeof(S) == 2) return __builtin_nontemporal_load(at_node<CT>(phi_prev, n));
    else return (CT)0;
}

// Shifts of the 2-byte codecs: a population is stored less the part of its
// equilibrium that the node reading it rebuilds from its own values of the
// step before: w_j phi for h, w_i c_i.u / T for g (T = 1/3).  Writer and
// reader evaluate one expression on the same FP32 values, so the reader's
// decode of a value equals the writer's own decode of it.
template <class CT> __device__ __forceinline__ CT g_shift(CT w, CT cu) { return (w * (CT)3) * cu; }
// shift of an incoming g_i read by a node whose previous-step velocity is u
template <class G, int D, class CT>
__device__ __forceinline__ CT g_ref(int i, const CT* u)
{
    return g_shift((CT)G::w(i), c_dot<G, D>(i, u));
}

// previous-step velocity of node n in 2-byte storage (wider storage: zero, unread)
template <class S, int D, class CT = typename Codec<S>::CT>
__device__ __forceinline__ void u_reference(void* u_prev, int64_t N, uint32_t n, CT* ur)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) ur[a] = 0;
    if constexpr (sizeof(S) == 2) {
        const Slots<CT> Up = slots<CT>(u_prev, N);
#pragma unroll
        for (int a = 0; a < D; ++a) ur[a] = __builtin_nontemporal_load(Up.at(a, n * (uint32_t)sizeof(CT)));
    }
}

// --- moments: phi, u* = sum g c, P*, M2 (per node; no halo).  NTL: the
// population loads stream past L2 (non-temporal); odd is the step parity,
// a constant in every instantiation the kernel calls.
template <int LS, class S, bool WALL, bool NTL>
__device__ __forceinline__ void moments_node(CDesc& cs, int x, int y, int z, bool odd)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    const uint32_t n = (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
    const uint32_t nb = n * (uint32_t)sizeof(S);
    const Nav nv = make_nav(cs, x, y, z, (int)sizeof(S));
    const Slots<S> hs = slots<S>(cs.h, cs.N), gs = slots<S>(cs.g, cs.N);
    const CT hsc = cconst<CT>(cs.h_inv_scale, cs.f32.h_inv_scale), gsc = cconst<CT>(cs.g_inv_scale, cs.f32.g_inv_scale);
    // 2-byte storage holds the populations less shifts made of phi (h) and
    // u (g) of this node one step earlier
    const CT php = h_reference<S>(cs.phi[odd ? 0 : 1], n);
    CT ur[3];
    u_reference<S, DIMV>(cs.U[odd ? 0 : 1], cs.N, n, ur);
    CT phi = 0;
#pragma unroll
    for (int j = 0; j < H::Q; ++j)
        phi += Codec<S>::dec(aa_load<H, WALL, NTL>(hs, nb, nv, j, odd), hsc,
                             php * (CT)H::w(j));
    CT sum = 0, J[3] = {0, 0, 0}, m2[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < G::Q; ++i) {
        const CT f = Codec<S>::dec(aa_load<G, WALL, NTL>(gs, nb, nv, i, odd), gsc,
                                   g_ref<G, DIMV>(i, ur));
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
    const uint32_t na = n * (uint32_t)sizeof(CT);
    // the moment fields are written once and read by the next kernels after
    // the whole grid has been written: stored non-temporal (FP16 moments 3%
    // faster, the kernels reading them unchanged)
    __builtin_nontemporal_store(phi, at_node<CT>(cs.phi[odd ? 1 : 0], n));
    const Slots<CT> Js = slots<CT>(cs.J, cs.N);
#pragma unroll
    for (int a = 0; a < DIMV; ++a) __builtin_nontemporal_store(J[a], Js.at(a, na));
    using AT = CT;
    const double Pprev = (double)__builtin_nontemporal_load(at_node<AT>(cs.P[odd ? 1 : 0], n));
    __builtin_nontemporal_store((AT)(Pprev + cs.rho_a * kT * (double)sum), at_node<AT>(cs.Ps, n));
    constexpr int NM = DIMV == 2 ? 3 : 6;
    if constexpr (sizeof(S) == 2) {
        const Slots<uint32_t> Ms = slots<uint32_t>(cs.M2, cs.N);
        const CT gsc_out = cconst<CT>(cs.g_scale, cs.f32.g_scale);
#pragma unroll
        for (int j = 0; j < (NM + 1) / 2; ++j) {
            const S lo = Codec<S>::enc(m2[2 * j], gsc_out, (CT)0);
            const S hi = 2 * j + 1 < NM ? Codec<S>::enc(m2[2 * j + 1], gsc_out, (CT)0) : (S)0;
            __builtin_nontemporal_store(m2_pack<S>(lo, hi), Ms.at(j, n * 4u));
        }
    } else {
        const Slots<CT> Ms = slots<CT>(cs.M2, cs.N);
#pragma unroll
        for (int k = 0; k < NM; ++k) __builtin_nontemporal_store(m2[k], Ms.at(k, na));
    }
}

template <int LS, class S>
__global__ __launch_bounds__(256) void k_moments(CaseTab cases, const int* hdr, int step_off)
{
    using Mo = Model<LS>;
    const TileCtx t = tile_ctx<Mo>(cases, hdr, step_off);
    if (!t.active) return;
    CDesc& cs = *t.cs;
    int lx, ly, lz;
    local_xyz<Mo>(&lx, &ly, &lz);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    if (x >= cs.nx || y >= cs.ny || z >= cs.nz) return;
    const bool odd = t.step & 1;
    constexpr bool nt_odd = nt_access<S, kLoadMoments>();
    constexpr bool nt_even = nt_odd || nt_access<S, kLoadMomentsEven>();
    constexpr bool nt_odd_wide = !nt_odd && sizeof(S) >= 4;
    if (tile_at_wall<Mo>(cs, t.ox, t.oy, t.oz)) {
        if (in_block(cs, x, y, z)) {
            // block nodes carry no fluid: phi, u*, P*, M2 = 0
            using CT = typename Codec<S>::CT;
            constexpr int DIMV = Model<LS>::DIM;
            const uint32_t n = (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
            const uint32_t na = n * (uint32_t)sizeof(CT);
            *at_node<CT>(cs.phi[odd ? 1 : 0], n) = 0;
            *at_node<CT>(cs.Ps, n) = 0;
            const Slots<CT> Js = slots<CT>(cs.J, cs.N);
#pragma unroll
            for (int a = 0; a < DIMV; ++a) *Js.at(a, na) = 0;
            constexpr int NM = DIMV == 2 ? 3 : 6;
            if constexpr (sizeof(S) == 2) {
                const Slots<uint32_t> Ms = slots<uint32_t>(cs.M2, cs.N);
#pragma unroll
                for (int j = 0; j < (NM + 1) / 2; ++j) *Ms.at(j, n * 4u) = 0u;  // +0 in both halves
            } else {
                const Slots<CT> Ms = slots<CT>(cs.M2, cs.N);
#pragma unroll
                for (int k = 0; k < NM; ++k) *Ms.at(k, na) = 0;
            }
            return;
        }
        if (!odd) moments_node<LS, S, true, nt_even>(cs, x, y, z, false);
        else if (nt_odd_wide && cs.nt_odd_moments) moments_node<LS, S, true, true>(cs, x, y, z, true);
        else moments_node<LS, S, true, nt_odd>(cs, x, y, z, true);
    } else {
        if (!odd) moments_node<LS, S, false, nt_even>(cs, x, y, z, false);
        else if (nt_odd_wide && cs.nt_odd_moments) moments_node<LS, S, false, true>(cs, x, y, z, true);
        else moments_node<LS, S, false, nt_odd>(cs, x, y, z, true);
    }
}

// --- pressure (Sec. II): P = rho_ref T sum_i (g_i + (1 + omega) K_i)
//     + omega rho_ref sum_i w_i c_i . u*(x - c_i), one evaluation of this
//     equation (which holds P on both sides, through K_i) started from the
//     pressure the streamed populations carry, P* = rho_ref T sum g: K_i from
//     P*.  Difference form: opposite links enter as
//     (P(x - c) - P0) + (P(x + c) - P0) and as u*(x - c) - u*(x + c), each
//     formed in the auxiliary type and so rounded relative to itself (the
//     single differences exact for P within a factor 2); the sums within a
//     shell are in the auxiliary type, the sum over shells and the final
//     combination FP64.
template <int LS, class AT, bool WALL, class R>
__device__ __forceinline__ void pressure_tile(CDesc& cs, const TileCtx& t, AT* sP, AT* sGD, AT (*sJ)[R::N])
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using G = typename Mo::G;
    using HR = Halo1<Mo, DIMV>;
    const Slots<AT> Js = slots<AT>(cs.J, cs.N);
    int lx, ly, lz;
    local_xyz<Mo>(&lx, &ly, &lz);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    const bool live = x < cs.nx && y < cs.ny && z < cs.nz;
    const uint32_t n = (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
    // the node's own phi is loaded first, so its latency overlaps the halo's
    const AT phi = live ? __builtin_nontemporal_load(at_node<AT>(cs.phi[t.step & 1], n)) : (AT)0;
    void* src[1 + DIMV];
    src[0] = cs.Ps;
#pragma unroll
    for (int a = 0; a < DIMV; ++a) src[1 + a] = (void*)Js.at(a, 0);
    halo_stage<HR, WALL, 1 + DIMV, AT>(
        cs, t, src,
        [&](int k, int cr, const int* off, const AT* v) {
            AT p = v[0], gd = 0;
            // ghost pressure = P(mirror) + rho(x) g.(ghost - mirror): keep g.off;
            // beyond the open end 2 p_top - P(mirror), p_top half a link out
            if (WALL) gd = (AT)(cs.grav[0] * off[0] + cs.grav[1] * off[1] + cs.grav[2] * off[2]);
            if (WALL && (cr & kOpenGhost)) {
                p = (AT)(2.0 * cs.p_top - (double)p);
                gd = 0;
            }
            sP[k] = p;
            if (WALL) sGD[k] = gd;
#pragma unroll
            for (int a = 0; a < DIMV; ++a) {
                AT j = v[1 + a];
                // u* at a ghost: flow part odd, body-force part even
                if (WALL && (cr & 1)) j = (AT)(-(double)j + 2.0 * cs.grav[a]);
                sJ[a][k] = j;
            }
        });
    __syncthreads();
    if (!live) return;
    if (WALL && in_block(cs, x, y, z)) {
        *at_node<AT>(cs.P[(t.step + 1) & 1], n) = 0;
        return;
    }
    // omega = (rho - rho_ref) / rho_ref with omega_max = rho_w / rho_ref, so
    // (1 + omega) rho_ref / rho = 1 and omega rho_ref = rho - rho_ref, which
    // weights the u* term by up to the density ratio: the shell-weighted sums
    // and this combination are taken in FP64 (the per-shell sums below are in
    // the auxiliary type)
    const double drho = (double)clamp01(phi) * (cs.rho_w - cs.rho_a);
    const double rho = cs.rho_a + drho;
    const int kb = R::template nb_base<HR::ZH>(lx + 1, ly + 1, lz + HR::ZH);
    const AT P0 = sP[kb + R::template nb<HR::ZH>(0, 0, 0)];
    // The weight of a link depends on its shell alone, so the link terms are
    // summed per shell, unweighted, in the auxiliary type (a handful of terms
    // of one magnitude class, each a difference rounded relative to itself);
    // the weighted sum over shells and the combination are FP64.
    constexpr int NS = shell<G>(G::Q - 1) + 1;
    AT sks[NS], sgs[NS], dus[3][NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sks[s] = sgs[s] = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) dus[a][s] = 0;
    }
#pragma unroll
    for (int i = 1; i < G::Q; i += 2) {  // pairs (i, i+1) are opposite
        const int s = shell<G>(i);
        const int km = kb + R::template nb<HR::ZH>(-G::c(i, 0), -G::c(i, 1), -G::c(i, 2));
        const int kp = kb + R::template nb<HR::ZH>(G::c(i, 0), G::c(i, 1), G::c(i, 2));
        // the pair's second difference of P
        sks[s] += (sP[km] - P0) + (sP[kp] - P0);
        if (WALL) sgs[s] += sGD[km] + sGD[kp];
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            if (G::c(i, a) == 0) continue;
            const AT d = sJ[a][km] - sJ[a][kp];
            if (G::c(i, a) == 1) dus[a][s] += d;
            else dus[a][s] -= d;
        }
    }
    double sk = 0, sg = 0, su = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double w = shell_w<G>(s);
        sk += w * (double)sks[s];
        if (WALL) sg += w * (double)sgs[s];
#pragma unroll
        for (int a = 0; a < DIMV; ++a) su += w * (double)dus[a][s];
    }
    if (WALL) sk += rho * sg;
    // rho_ref T (1 + omega) sum K = (1 + omega) rho_ref / rho * sum w dP = sk
    *at_node<AT>(cs.P[(t.step + 1) & 1], n) = (AT)((double)P0 + (sk + drho * su));
}

template <int LS, class AT>
__global__ __launch_bounds__(256) void k_pressure(CaseTab cases, const int* hdr, int step_off)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using R = typename Halo1<Mo, DIMV>::R;
    __shared__ AT sP[R::N], sGD[R::N], sJ[DIMV][R::N];
    const TileCtx t = tile_ctx<Mo>(cases, hdr, step_off);
    if (!t.active) return;
    CDesc& cs = *t.cs;
    if (tile_at_wall<Mo>(cs, t.ox, t.oy, t.oz)) pressure_tile<LS, AT, true, R>(cs, t, sP, sGD, sJ);
    else pressure_tile<LS, AT, false, R>(cs, t, sP, sGD, sJ);
}

// --- velocity: u = u* + sum_i K_i c_i with K_i of the new pressure.
template <int LS, class CT, bool WALL, class R>
__device__ __forceinline__ void velocity_tile(CDesc& cs, const TileCtx& t, CT* sP, CT* sGD)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using G = typename Mo::G;
    using HR = Halo1<Mo, DIMV>;
    void* Pn = cs.P[(t.step + 1) & 1];
    int lx, ly, lz;
    local_xyz<Mo>(&lx, &ly, &lz);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    const bool live = x < cs.nx && y < cs.ny && z < cs.nz;
    const uint32_t n = (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
    const uint32_t na = n * (uint32_t)sizeof(CT);
    // the node's own operands are loaded first, so their latency overlaps the halo's
    const Slots<CT> Js = slots<CT>(cs.J, cs.N), Us = slots<CT>(cs.U[t.step & 1], cs.N);
    CT phi = 0, J[3] = {0, 0, 0};
    if (live) {
        phi = __builtin_nontemporal_load(at_node<CT>(cs.phi[t.step & 1], n));
#pragma unroll
        for (int a = 0; a < DIMV; ++a) J[a] = __builtin_nontemporal_load(Js.at(a, na));
    }
    void* src[1] = {Pn};
    halo_stage<HR, WALL, 1, CT>(
        cs, t, src,
        [&](int k, int cr, const int* off, const CT* v) {
            CT p = v[0], gd = 0;
            if (WALL) gd = (CT)(cs.grav[0] * off[0] + cs.grav[1] * off[1] + cs.grav[2] * off[2]);
            if (WALL && (cr & kOpenGhost)) {
                p = (CT)(2.0 * cs.p_top - (double)p);
                gd = 0;
            }
            sP[k] = p;
            if (WALL) sGD[k] = gd;
        });
    __syncthreads();
    if (!live) return;
    if (WALL && in_block(cs, x, y, z)) {
#pragma unroll
        for (int a = 0; a < DIMV; ++a) *Us.at(a, na) = 0;
        return;
    }
    const CT ra = cconst<CT>(cs.rho_a, cs.f32.rho_a), dr = cconst<CT>(cs.rho_w - cs.rho_a, cs.f32.drho);
    const CT rho = ra + clamp01(phi) * dr;
    const CT irho = rcp(rho);
    const int kb = R::template nb_base<HR::ZH>(lx + 1, ly + 1, lz + HR::ZH);
    CT gr[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < G::Q; i += 2) {
        const int kp = kb + R::template nb<HR::ZH>(G::c(i, 0), G::c(i, 1), G::c(i, 2));
        const int km = kb + R::template nb<HR::ZH>(-G::c(i, 0), -G::c(i, 1), -G::c(i, 2));
        const CT d = (WALL ? (sP[kp] + rho * sGD[kp]) - (sP[km] + rho * sGD[km]) : sP[kp] - sP[km]) * (CT)G::w(i);
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            if (G::c(i, a) == 1) gr[a] += d;
            if (G::c(i, a) == -1) gr[a] -= d;
        }
    }
#pragma unroll
    for (int a = 0; a < DIMV; ++a) *Us.at(a, na) = J[a] - gr[a] * (CT)3.0 * irho;
}

template <int LS, class CT>
__global__ __launch_bounds__(256) void k_velocity(CaseTab cases, const int* hdr, int step_off)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using R = typename Halo1<Mo, DIMV>::R;
    __shared__ CT sP[R::N], sGD[R::N];
    const TileCtx t = tile_ctx<Mo>(cases, hdr, step_off);
    if (!t.active) return;
    CDesc& cs = *t.cs;
    // a fused case's collide rebuilds u itself; the read pass (step_off < 0) still needs it here
    if (cs.fuse_u && step_off >= 0) return;
    if (tile_at_wall<Mo>(cs, t.ox, t.oy, t.oz)) velocity_tile<LS, CT, true, R>(cs, t, sP, sGD);
    else velocity_tile<LS, CT, false, R>(cs, t, sP, sGD);
}

// Gradients of phi, rho and u at interior cell (cx, cy, cz) of a 1-halo tile.
template <int LS, class R, class CT>
__device__ __forceinline__ void tile_gradients(const CT* sPhi, const CT* sRho, const CT (*sU)[R::N], int cx,
                                               int cy, int cz, NodeVals<CT>& v)
{
    constexpr int DIMV = Model<LS>::DIM;
    using G = typename Model<LS>::G;
    const int c0 = R::idx(cx, cy, cz);
    v.phi = sPhi[c0];
#pragma unroll
    for (int a = 0; a < 3; ++a) v.u[a] = a < DIMV ? sU[a][c0] : (CT)0;
    stencil<G, R, CT>([&](int k) { return sPhi[k]; }, cx, cy, cz, v.gphi, &v.lphi);
    stencil<G, R, CT>([&](int k) { return sRho[k]; }, cx, cy, cz, v.grho, (CT*)nullptr);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) v.G[a][b] = 0;
#pragma unroll
    for (int a = 0; a < DIMV; ++a) {
        CT gr[3];
        stencil<G, R, CT>([&](int k) { return sU[a][k]; }, cx, cy, cz, gr, (CT*)nullptr);
#pragma unroll
        for (int b = 0; b < DIMV; ++b) v.G[a][b] = gr[b];
    }
}

// --- collide + stream.  A tile first issues the loads of its own nodes'
// incoming h (parked in LDS until the direction loop) and M2,
// together with the halo loads of phi and u, so that their latencies overlap;
// then it takes the gradients from LDS and collides one direction at a time.
// The tile's step read again from the descriptor (a volatile load, so the
// compiler cannot take it for the value a branch already tested).
__device__ __forceinline__ int64_t step_parity(CDesc& cs, const TileCtx& t)
{
    return *(const volatile PULBM_CST int64_t*)&cs.step + (t.step - cs.step);
}

template <int LS, class S, bool WALL, bool BGK, class R, int PAR>
__device__ __forceinline__ void collide_tile(CDesc& cs, const TileCtx& t, typename Codec<S>::CT* sPhi,
                                             typename Codec<S>::CT* sRho,
                                             typename Codec<S>::CT (*sU)[R::N], S (*sH)[256],
                                             typename Codec<S>::CT* sP2)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    using HR = Halo1<Mo, DIMV>;
    constexpr int NM = DIMV == 2 ? 3 : 6;
    const Phys<CT> ph = make_phys<CT>(cs);
    int lx, ly, lz;
    local_xyz<Mo>(&lx, &ly, &lz);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    // block nodes carry no fluid and are skipped like nodes past the grid
    const bool inside = x < cs.nx && y < cs.ny && z < cs.nz && !(WALL && in_block(cs, x, y, z));
    const uint32_t n = inside ? (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z) : 0u;
    const uint32_t nb = n * (uint32_t)sizeof(S), na = n * (uint32_t)(sizeof(S) == 2 ? 4 : sizeof(CT));
    // the step's parity, which decides the slots the AA pattern reads and
    // writes.  PAR 0: even, fixed at compile time.  PAR 1: odd, read again at
    // run time (step_parity), so that each load and store decides its slot
    // as it runs: a copy with the odd slots fixed keeps a node's neighbour
    // offsets in registers and spills past the 3-waves budget.  PAR 2: odd,
    // fixed, for a tile whose nodes have every neighbour inside the grid,
    // whose offsets are then the strides (scalars).
    const bool odd = PAR == 0 ? false : (PAR == 2 ? true : (bool)(step_parity(cs, t) & 1));
    const Nav nv = PAR == 2 ? make_nav_inner(cs, (int)sizeof(S))
                            : make_nav(cs, inside ? x : 0, inside ? y : 0, inside ? z : 0, (int)sizeof(S));
    // stores stream past L2 on even steps (FP32 even collide 3% faster); on
    // odd steps, shifted by one node in x, each line is written partly by
    // this tile and partly by its x neighbour, and kept in L2 the parts merge
    // (measured, FP16: the odd steps' writes 123 -> 92 B/node)
    constexpr bool nts = PAR == 0 && nt_access<S, kStoreCollide>();
    const Slots<S> hs = slots<S>(cs.h, cs.N), gs = slots<S>(cs.g, cs.N);
    // own-node loads first
    S hraw[H::Q];
    // M2 as loaded: compute-type values, or words of two 2-byte codes
    using M2L = std::conditional_t<sizeof(S) == 2, uint32_t, CT>;
    constexpr int NL = sizeof(S) == 2 ? (NM + 1) / 2 : NM;
    M2L m2l[NL];
    CT php = 0;  // reference of the incoming h (2-byte storage)
    CT dP = 0;   // BGK: (previous P - new P) / (rho_ref T), restores the stored rest population
    CT ur[3] = {0, 0, 0};  // BGK, 2-byte storage: reference of the incoming g
    if (inside) {
        php = h_reference<S>(cs.phi[(t.step + 1) & 1], n);
        if constexpr (BGK) u_reference<S, DIMV>(cs.U[(t.step + 1) & 1], cs.N, n, ur);
#pragma unroll
        for (int j = 0; j < H::Q; ++j) hraw[j] = aa_load<H, WALL, nt_access<S, kLoadCollide>()>(hs, nb, nv, j, odd);
        if constexpr (BGK) {
            dP = (CT)(((double)*at_node<CT>(cs.P[t.step & 1], n) - (double)*at_node<CT>(cs.P[(t.step + 1) & 1], n)) *
                      (3.0 / cs.rho_a));
        } else {
            const Slots<M2L> Ms = slots<M2L>(cs.M2, cs.N);
#pragma unroll
            for (int k = 0; k < NL; ++k) m2l[k] = __builtin_nontemporal_load(Ms.at(k, na));
        }
    }
    // 2-byte storage parks h in LDS before the halo loads: the codec's extra
    // registers leave no room to hold h and every halo value at once
    if constexpr (sizeof(S) == 2) {
        if (inside) {
#pragma unroll
            for (int j = 0; j < H::Q; ++j) sH[j][threadIdx.x] = hraw[j];
        }
    }
    // halo of phi, rho and u; a fused case (no wall, open end or block)
    // loads u* instead of u and the new P two nodes deep, and rebuilds u
    // itself below
    bool fused = false;
    if constexpr (!WALL && sizeof(S) >= 4) fused = cs.fuse_u;
    const Slots<CT> Us = slots<CT>(fused ? cs.J : cs.U[t.step & 1], cs.N);
    void* src[1 + DIMV];
    src[0] = cs.phi[t.step & 1];
#pragma unroll
    for (int a = 0; a < DIMV; ++a) src[1 + a] = (void*)Us.at(a, 0);
    halo_stage<HR, WALL, 1 + DIMV, CT>(
        cs, t, src,
        [&](int k, int cr, const int*, const CT* v) {
            sPhi[k] = v[0];
            sRho[k] = ph.rho_a + clamp01(v[0]) * ph.drho;
#pragma unroll
            for (int a = 0; a < DIMV; ++a) sU[a][k] = (WALL && (cr & 1)) ? -v[1 + a] : v[1 + a];  // no slip
        });
    if constexpr (!WALL && sizeof(S) >= 4) {
        if (fused) {
            void* psrc[1] = {cs.P[(t.step + 1) & 1]};
            halo_stage<Halo2<Mo, DIMV>, false, 1, CT>(cs, t, psrc,
                                                      [&](int k, int, const int*, const CT* v) { sP2[k] = v[0]; });
        }
    }
    if constexpr (sizeof(S) != 2) {
        if (inside) {
#pragma unroll
            for (int j = 0; j < H::Q; ++j) sH[j][threadIdx.x] = hraw[j];
        }
    }
    __syncthreads();
    if constexpr (!WALL && sizeof(S) >= 4) {
        if (fused) {
            // u = u* - D P / rho at every cell of the 1-halo region, the
            // expression of k_velocity term by term
            using R2 = typename Halo2<Mo, DIMV>::R;
            constexpr int DZ = Halo2<Mo, DIMV>::ZH - HR::ZH;
#pragma unroll
            for (int it = 0; it < (R::N + 255) / 256; ++it) {
                const int k = (int)threadIdx.x + 256 * it;
                if (k < R::N) {
                    const int ix = k % HR::RX, iy = (k / HR::RX) % HR::RY, iz = k / (HR::RX * HR::RY);
                    const int cx2 = ix + 1, cy2 = iy + 1, cz2 = iz + DZ;
                    CT gr[3] = {0, 0, 0};
#pragma unroll
                    for (int i = 1; i < G::Q; i += 2) {
                        const int kp = R2::idx(cx2 + G::c(i, 0), cy2 + G::c(i, 1), cz2 + G::c(i, 2));
                        const int km = R2::idx(cx2 - G::c(i, 0), cy2 - G::c(i, 1), cz2 - G::c(i, 2));
                        const CT d = (sP2[kp] - sP2[km]) * (CT)G::w(i);
#pragma unroll
                        for (int a = 0; a < DIMV; ++a) {
                            if (G::c(i, a) == 1) gr[a] += d;
                            if (G::c(i, a) == -1) gr[a] -= d;
                        }
                    }
                    const CT irho = rcp(sRho[k]);
#pragma unroll
                    for (int a = 0; a < DIMV; ++a) sU[a][k] = sU[a][k] - gr[a] * (CT)3.0 * irho;
                }
            }
            __syncthreads();
        }
    }
    if (!inside) return;

    CT m2[NM];
    if constexpr (!BGK) {
        if constexpr (sizeof(S) == 2) {
            const CT gsc_m = cconst<CT>(cs.g_inv_scale, cs.f32.g_inv_scale);
#pragma unroll
            for (int k = 0; k < NM; ++k) m2[k] = Codec<S>::dec(m2_half<S>(m2l[k / 2], k & 1), gsc_m, (CT)0);
        } else {
#pragma unroll
            for (int k = 0; k < NM; ++k) m2[k] = m2l[k];
        }
    }
    NodeVals<CT> v;
    tile_gradients<LS, R, CT>(sPhi, sRho, sU, lx + 1, ly + 1, lz + HR::ZH, v);
    // the BGK collision needs the equilibria alone (no Pi: the INIT form)
    const NodeCoef<DIMV, CT> kc = node_coef<DIMV, BGK, CT>(ph, v, m2);
    const CT omf = BGK ? (CT)1 - rcp(ph.tau_a + clamp01(v.phi) * ph.dtau) : (CT)0;  // 1 - 1/tau_mix
    const CT hisc = cconst<CT>(cs.h_inv_scale, cs.f32.h_inv_scale), hsc = cconst<CT>(cs.h_scale, cs.f32.h_scale);
    const CT gsc = cconst<CT>(cs.g_scale, cs.f32.g_scale), gsc_in = cconst<CT>(cs.g_inv_scale, cs.f32.g_inv_scale);
    const CT corr = (CT)6.0 * rcp(kc.rho);  // 2 / (rho T)
    // shifts of an outgoing g_i and h_i in 2-byte storage, from phi and u
    // (this step) of the node that reads it next step: x + c_i, or x itself
    // for a population reflected at a wall, which that node reads as moving
    // along -c_i
    const int cx = lx + 1, cy = ly + 1, cz = lz + HR::ZH, c0 = R::idx(cx, cy, cz);
    // (each taken where it is used, which keeps the register budget)
    auto gref_out = [&](int i, bool reflected) -> CT {
        if constexpr (sizeof(S) != 2) {
            return (CT)0;
        } else {
            const int k = reflected ? c0 : R::idx(cx + G::c(i, 0), cy + G::c(i, 1), cz + G::c(i, 2));
            CT ud[3] = {0, 0, 0};
#pragma unroll
            for (int a = 0; a < DIMV; ++a)
                if (G::c(i, a) != 0) ud[a] = sU[a][k];
            CT cu = c_dot<G, DIMV>(i, ud);
            if (reflected) cu = -cu;
            return g_shift((CT)G::w(i), cu);
        }
    };
    auto href_out = [&](int i, bool reflected) -> CT {
        if constexpr (sizeof(S) != 2) {
            return (CT)0;
        } else {
            const int k = reflected ? c0 : R::idx(cx + H::c(i, 0), cy + H::c(i, 1), cz + H::c(i, 2));
            return (CT)H::w(i) * sPhi[k];
        }
    };
    // rest direction of g, the opposite pairs, then the rest direction of h;
    // both lattices share the direction order, so h_i and g_i stream to the
    // same node
    {
        CT g0 = g_out<G, DIMV, BGK>(v, kc, 0);
        if constexpr (BGK) {
            // BGK (Eq. BGK_LBeq_hydroeq) on the full rest population; both the
            // stored incoming value and the equilibrium lack their P / (rho_ref T)
            const CT gin = Codec<S>::dec(aa_load<G, WALL, false>(gs, nb, nv, 0, odd), gsc_in,
                                         g_ref<G, DIMV>(0, ur)) + dP;
            g0 += omf * (gin - g0);
        }
        aa_store<G, WALL, nts>(gs, nb, nv, 0, odd, Codec<S>::enc(g0, gsc, (CT)0), false);
    }
    // sum over j != 0 of the incoming h_j less the outgoing h*_j as its reader
    // will decode it (the rest population balances it below)
    CT hmoved = 0;
#pragma unroll
    for (int i = 1; i < G::Q; i += 2) {
        // BF16 storage: keep the scheduler from interleaving pairs (its
        // codec's integer rounding, hoisted across pairs, pushes the D3Q27
        // kernel past its register budget into scratch spills; FP16 storage
        // runs faster without the barrier)
        if constexpr (std::is_same_v<S, uint16_t>) __builtin_amdgcn_sched_barrier(0);
        const bool bi = WALL && nav_solid<G>(nv, i, +1);
        const bool bk = WALL && nav_solid<G>(nv, i + 1, +1);
        CT gi, gk;
        g_pair<G, DIMV, BGK>(v, kc, i, &gi, &gk);
        if constexpr (BGK) {
            // incoming g_i, g_i+1: within a step a node reads and writes one set
            // of slots (AA), and the slots of this pair are written just below
            const CT ai = Codec<S>::dec(aa_load<G, WALL, false>(gs, nb, nv, i, odd), gsc_in,
                                        g_ref<G, DIMV>(i, ur));
            const CT ak = Codec<S>::dec(aa_load<G, WALL, false>(gs, nb, nv, i + 1, odd), gsc_in,
                                        g_ref<G, DIMV>(i + 1, ur));
            gi += omf * (ai - gi);
            gk += omf * (ak - gk);
        }
        if (WALL) {
            const bool oi = nav_open<G>(nv, i, +1), ok = nav_open<G>(nv, i + 1, +1);
            CT cF = 0;
#pragma unroll
            for (int a = 0; a < DIMV; ++a) {
                if (G::c(i, a) == 1) cF += kc.F[a];
                if (G::c(i, a) == -1) cF -= kc.F[a];
            }
            // a reflected population keeps the force part of its equilibrium
            const CT fc = (CT)G::w(i) * cF * corr;
            gi -= (bi && !oi) ? fc : (CT)0;
            gk += (bk && !ok) ? fc : (CT)0;
            // through the open end: the population leaves, and the opposite
            // one entering this node is the node's own equilibrium
            if (oi || ok) {
                CT ei, ek;
                g_pair<G, DIMV, true>(v, kc, i, &ei, &ek);
                if (oi) gi = ek;
                if (ok) gk = ei;
            }
        }
        aa_store<G, WALL, nts>(gs, nb, nv, i, odd, Codec<S>::enc(gi, gsc, gref_out(i, bi)),
                                                         bi);
        aa_store<G, WALL, nts>(gs, nb, nv, i + 1, odd,
                                                         Codec<S>::enc(gk, gsc, gref_out(i + 1, bk)), bk);
        if (i < H::Q) {
            const CT hi = Codec<S>::dec(sH[i][threadIdx.x], hisc, php * (CT)H::w(i));
            const CT hk = Codec<S>::dec(sH[i + 1][threadIdx.x], hisc, php * (CT)H::w(i + 1));
            CT oi, ok;
            h_pair<H, DIMV, false>(ph, v, kc, i, hi, hk, &oi, &ok);
            const CT ri = href_out(i, bi), rk = href_out(i + 1, bk);
            const S ei = Codec<S>::enc(oi, hsc, ri), ek = Codec<S>::enc(ok, hsc, rk);
            hmoved += (hi - Codec<S>::dec(ei, hisc, ri)) + (hk - Codec<S>::dec(ek, hisc, rk));
            aa_store<H, WALL, nts>(hs, nb, nv, i, odd, ei, bi);
            aa_store<H, WALL, nts>(hs, nb, nv, i + 1, odd, ek, bk);
        }
    }
    // rest population of h: BGK conserves phi (sum_j h^eq_j = phi), so
    // h*_0 = h_0 + sum_{j != 0} (h_j - h*_j).  Taking it in that form, with the
    // outgoing values as stored, keeps the weights' rounding (their FP32
    // values sum to 1 + 1.5e-8 on D3Q19) and the rounding of identical bulk
    // nodes from drifting phi's mass step after step.
    {
        const CT h0 = Codec<S>::dec(sH[0][threadIdx.x], hisc, php * (CT)H::w(0));
        aa_store<H, WALL, nts>(hs, nb, nv, 0, odd,
                                                         Codec<S>::enc(h0 + hmoved, hsc, href_out(0, true)), false);
    }
}

// Occupancy target of the collision kernel: 3 waves per SIMD.  Left alone
// the compiler takes ~175-195 VGPRs (2 waves); a budget of 168 (3 waves)
// costs a few dwords of spill and hides enough more memory latency to run
// 10% (FP32) to 18% (FP16) faster; 128 (4 waves) spills too much.
#define PULBM_COLLIDE_ATTR __attribute__((amdgpu_waves_per_eu(3, 3)))
// One kernel per step parity: PAR 0 takes the tiles of cases at an even
// step, with every load and store on its fixed slot (no branch: the FP16
// collide's even steps run 17% faster than with the parity read at run
// time); PAR 1 takes the tiles of cases at an odd step, with fixed slots
// on tiles clear of the grid's edges (PAR 2 of collide_tile, 6% faster)
// and slots decided at run time on the others.  A single case
// launches the kernel of its step's parity, a serving batch (whose cases may
// differ in parity) both, each skipping the other's tiles, so a case runs the
// same code alone and in a batch, bitwise.
template <int LS, class S, bool BGK, int PAR>
__global__ __launch_bounds__(256) PULBM_COLLIDE_ATTR void k_collide(CaseTab cases, const int* hdr, int step_off)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    using R = typename Halo1<Mo, DIMV>::R;
    __shared__ CT sPhi[R::N], sRho[R::N], sU[DIMV][R::N];
    __shared__ S sH[H::Q][256];
    // the new P two nodes deep, for cases whose collide rebuilds u (4- and 8-byte storage)
    __shared__ CT sP2[sizeof(S) >= 4 ? Halo2<Mo, DIMV>::R::N : 1];
    const TileCtx t = tile_ctx<Mo>(cases, hdr, step_off);
    if (!t.active || (int)(t.step & 1) != PAR) return;
    CDesc& cs = *t.cs;
    if (tile_at_wall<Mo>(cs, t.ox, t.oy, t.oz)) {
        collide_tile<LS, S, true, BGK, R, PAR>(cs, t, sPhi, sRho, sU, sH, sP2);
    } else if (PAR == 1 && t.ox >= 1 && t.ox + Mo::TX < cs.nx && t.oy >= 1 && t.oy + Mo::TY < cs.ny &&
               (DIMV == 2 || (t.oz >= 1 && t.oz + Mo::TZ < cs.nz))) {
        // every node of the tile has its neighbours inside the grid
        collide_tile<LS, S, false, BGK, R, 2>(cs, t, sPhi, sRho, sU, sH, sP2);
    } else {
        collide_tile<LS, S, false, BGK, R, PAR>(cs, t, sPhi, sRho, sU, sH, sP2);
    }
}

// --- initial state: equilibria of (phi0, P0, u0) in the even AA layout,
//     previous-step pressure P[0] = P0.  Inputs are FP64 device arrays.
template <int LS, class S>
__global__ __launch_bounds__(256) void k_init(CaseTab cases, const int* hdr,
                                              const double* __restrict__ phi0, const double* __restrict__ P0,
                                              const double* __restrict__ u0)
{
    constexpr int DIMV = Model<LS>::DIM;
    using Mo = Model<LS>;
    using G = typename Mo::G;
    using H = typename Mo::H;
    using CT = typename Codec<S>::CT;
    using HR = Halo1<Mo, DIMV>;
    using R = typename HR::R;
    __shared__ CT sPhi[R::N], sRho[R::N], sU[DIMV][R::N];
    const TileCtx t = tile_ctx<Mo>(cases, hdr, 0);
    if (!t.active) return;
    CDesc& cs = *t.cs;
    const uint32_t N = (uint32_t)cs.N;
    const Phys<CT> ph = make_phys<CT>(cs);
    // the halo cell by cell (initialisation runs once; the step kernels use
    // halo_stage)
#pragma unroll
    for (int it = 0; it < (R::N + 255) / 256; ++it) {
        const int k = threadIdx.x + 256 * it;
        if (k >= R::N) break;
        int off[3], cr;
        const uint32_t m = HR::cell(cs, t, k, off, &cr);
        const CT f = (CT)phi0[m];
        sPhi[k] = f;
        sRho[k] = ph.rho_a + clamp01(f) * ph.drho;
#pragma unroll
        for (int a = 0; a < DIMV; ++a) {
            const CT ua = (CT)u0[(size_t)a * N + m];
            sU[a][k] = (cr & 1) ? -ua : ua;
        }
    }
    __syncthreads();
    int lx, ly, lz;
    local_xyz<Mo>(&lx, &ly, &lz);
    const int x = t.ox + lx, y = t.oy + ly, z = t.oz + lz;
    if (x >= cs.nx || y >= cs.ny || z >= cs.nz) return;
    const uint32_t n = (uint32_t)x + (uint32_t)cs.sx * ((uint32_t)y + (uint32_t)cs.ny * (uint32_t)z);
    const Slots<S> hs = slots<S>(cs.h, cs.N), gs = slots<S>(cs.g, cs.N);
    const uint32_t nb = n * (uint32_t)sizeof(S);
    const Slots<CT> U1 = slots<CT>(cs.U[1], cs.N);
    if (in_block(cs, x, y, z)) {
        // block nodes hold no populations and no fluid
#pragma unroll
        for (int j = 0; j < H::Q; ++j) *hs.at(j, nb) = Codec<S>::enc((CT)0, (CT)1, (CT)0);
#pragma unroll
        for (int i = 0; i < G::Q; ++i) *gs.at(i, nb) = Codec<S>::enc((CT)0, (CT)1, (CT)0);
        *at_node<CT>(cs.P[0], n) = 0;
        *at_node<CT>(cs.P[1], n) = 0;
        *at_node<CT>(cs.phi[1], n) = 0;
#pragma unroll
        for (int a = 0; a < DIMV; ++a) *U1.at(a, n * (uint32_t)sizeof(CT)) = 0;
        return;
    }
    NodeVals<CT> v;
    tile_gradients<LS, R, CT>(sPhi, sRho, sU, lx + 1, ly + 1, lz + HR::ZH, v);
    const NodeCoef<DIMV, CT> kc = node_coef<DIMV, true, CT>(ph, v, (const CT*)nullptr);
    const CT hsc = cconst<CT>(cs.h_scale, cs.f32.h_scale), gsc = cconst<CT>(cs.g_scale, cs.f32.g_scale);
    // 2-byte storage: h_j - w_j phi0 (the previous-step phi of step 0 is phi0)
    const CT phr = sizeof(S) == 2 ? v.phi : (CT)0;
    CT hmoved = 0;
#pragma unroll
    for (int j = 1; j < H::Q; ++j) {
        const CT hj = h_out<H, DIMV, true>(ph, v, kc, j, (CT)0);
        hmoved += hj;
        *hs.at(j, nb) = Codec<S>::enc(hj, hsc, phr * (CT)H::w(j));
    }
    // rest population as the remainder, so that sum_j h_j = phi0 exactly
    *hs.at(0, nb) = Codec<S>::enc(v.phi - hmoved, hsc, phr * (CT)H::w(0));
    // 2-byte storage: g_i - w_i c_i.u0 / T (the previous-step u of step 0 is u0)
#pragma unroll
    for (int i = 0; i < G::Q; ++i)
        *gs.at(i, nb) = Codec<S>::enc(g_out<G, DIMV, true>(v, kc, i), gsc,
                                      sizeof(S) == 2 ? g_ref<G, DIMV>(i, v.u) : (CT)0);
    *at_node<CT>(cs.P[0], n) = (CT)P0[n];
    *at_node<CT>(cs.phi[1], n) = v.phi;
#pragma unroll
    for (int a = 0; a < DIMV; ++a) *U1.at(a, n * (uint32_t)sizeof(CT)) = v.u[a];
}

// --- step counters: every case of a table advances by k (up to its end).
__global__ void k_advance(CaseTab cases, const int* hdr, int k)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= hdr[0]) return;
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
    const AT* phi = (const AT*)cs.phi[cs.step & 1];
    const AT* P = (const AT*)cs.P[(cs.step + 1) & 1];
    const AT* U = (const AT*)cs.U[cs.step & 1];
    double acc[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < N; n += (int64_t)gridDim.x * 256) {
        if (n % cs.sx >= cs.nx) continue;  // row padding
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

// one wave per value: lane l takes blocks l, l + 64, ... in order, then a
// fixed shuffle tree (the result does not depend on scheduling)
__global__ __launch_bounds__(64) void k_diag_final(const double* __restrict__ partial, int nblocks,
                                                   double* __restrict__ out)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    double r = 0.0;
    for (int b = lane; b < nblocks; b += 64) r = k == 7 ? fmax(r, partial[b * kDiagVals + k]) : r + partial[b * kDiagVals + k];
    r = k == 7 ? wave_max(r) : wave_sum(r);
    if (lane == 0) out[k] = r;
}

}  // namespace pulbm
