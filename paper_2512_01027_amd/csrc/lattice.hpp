// Velocity sets of the solver, as compile-time tables (every loop over
// directions is fully unrolled, so c and w become immediates).
//
// Direction order: 0 is the rest direction; i and i+1 (i odd) are opposite.
// The 3D phase-field set D3Q19 is the first 19 directions of D3Q27 (rest,
// 6 faces, 12 edges) with its own weights.  Lattice temperature T = 1/3
// (Sec. II of the paper).
#pragma once

namespace pulbm {

constexpr double kT = 1.0 / 3.0;

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int DIM = 2;
    __host__ __device__ static constexpr int c(int i, int a)
    {
        constexpr int t[9][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
        return t[i][a];
    }
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
};

struct D3Q27 {
    static constexpr int Q = 27;
    static constexpr int DIM = 3;
    __host__ __device__ static constexpr int c(int i, int a)
    {
        constexpr int t[27][3] = {
            {0, 0, 0},   {1, 0, 0},    {-1, 0, 0},   {0, 1, 0},   {0, -1, 0},  {0, 0, 1},
            {0, 0, -1},  {1, 1, 0},    {-1, -1, 0},  {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},
            {-1, 0, -1}, {1, 0, -1},   {-1, 0, 1},   {0, 1, 1},   {0, -1, -1}, {0, 1, -1},
            {0, -1, 1},  {1, 1, 1},    {-1, -1, -1}, {1, 1, -1},  {-1, -1, 1}, {1, -1, 1},
            {-1, 1, -1}, {1, -1, -1},  {-1, 1, 1}};
        return t[i][a];
    }
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 8.0 / 27.0 : (i < 7 ? 2.0 / 27.0 : (i < 19 ? 1.0 / 54.0 : 1.0 / 216.0));
    }
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int DIM = 3;
    __host__ __device__ static constexpr int c(int i, int a) { return D3Q27::c(i, a); }
    __host__ __device__ static constexpr double w(int i)
    {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
};

// Shell of link i: its number of non-zero components less one (axis links 0,
// face diagonals 1, cube diagonals 2).  In D2Q9, D3Q19 and D3Q27 a link's
// weight depends on its shell alone, which lets a weighted sum over links be
// taken as a weighted sum over shells of plain sums.
template <class G> __host__ __device__ constexpr int shell(int i)
{
    return (G::c(i, 0) != 0) + (G::c(i, 1) != 0) + (G::c(i, 2) != 0) - 1;
}
template <class G> __host__ __device__ constexpr double shell_w(int s)
{
    for (int i = 1; i < G::Q; ++i)
        if (shell<G>(i) == s) return G::w(i);
    return 0.0;
}
template <class G> constexpr bool weight_by_shell()
{
    for (int i = 1; i < G::Q; ++i)
        if (G::w(i) != shell_w<G>(shell<G>(i))) return false;
    return true;
}
static_assert(weight_by_shell<D2Q9>() && weight_by_shell<D3Q19>() && weight_by_shell<D3Q27>(),
              "link weights depend on the shell alone");

// Lattice sets: hydro lattice G, phase-field lattice H, dimension and the
// workgroup tile.  Set 2: D2Q9 / D2Q9; set 3: D3Q27 / D3Q19; set 4: D3Q19 /
// D3Q19 (the lattice the paper uses in 3D, Sec. II).  Tiles are 256 threads
// (four 64-wide wavefronts), x fastest so that a wavefront reads a whole
// 256-byte row of a 4-byte population.  The 3D tile is 64 x 2 x 2: against
// 32 x 4 x 2 its longer rows halve the cache lines that odd-step x-shifted
// reads and writes share with the neighbouring tile (moments and collide
// ran 12-14% faster at 128^3), at a larger halo (66 x 4 x 4 cells).
template <int LS> struct Model;
template <> struct Model<2> {
    using G = D2Q9;
    using H = D2Q9;
    static constexpr int DIM = 2;
    static constexpr int TX = 64, TY = 4, TZ = 1;
};
struct Tile3 {
    static constexpr int TX = 64, TY = 2, TZ = 2;
};
template <> struct Model<3> : Tile3 {
    using G = D3Q27;
    using H = D3Q19;
    static constexpr int DIM = 3;
};
template <> struct Model<4> : Tile3 {
    using G = D3Q19;
    using H = D3Q19;
    static constexpr int DIM = 3;
};

// Lattice set of a case: dimension and hydro lattice size.
__host__ __device__ constexpr int lattice_set(int dim, int q_hydro) { return dim == 2 ? 2 : (q_hydro == 19 ? 4 : 3); }

}  // namespace pulbm
