// hb_tile.hip -- LDS-tiled kernels of the tensor viscous problem for the
// multigrid levels (gfx950), templated on the storage and arithmetic type R
// (double, or float in the mixed-precision correction cycles):
//   k_tsmooth       one component's red AND black Gauss-Seidel half sweeps in
//                   one launch: the tile plus a 2-cell halo of every component
//                   is staged in LDS, red cells are updated on the tile and its
//                   1-cell ring, black cells on the tile; the result goes to
//                   the other buffer of a double-buffered iterate, so blocks
//                   never read values another block has already written;
//   k_tresid        r = b - A x (max-norm reduced) or y = A x, halo 1;
//   k_tresid_restr  fine residual and its restriction (mean of children).
// Boundary values (odd wall reflection, periodic wrap) are produced once, when
// the tile is filled; the stencil then reads plain LDS offsets.
// For R = double the arithmetic per cell is the same sequence as the
// global-memory operator, so results do not depend on the tiling.
#include "hb_internal.h"
#include "hb_stencil.h"

#include <hip/hip_ext.h>

#include <tuple>

namespace hb {

template <int TX_, int TY_, int TZ_, int TH_>
struct TileShape {
    static constexpr int TX = TX_, TY = TY_, TZ = TZ_, THREADS = TH_;
};
template <int DIM> struct TileCfg;
template <> struct TileCfg<2> : TileShape<64, 8, 1, 256> {};
template <> struct TileCfg<3> : TileShape<32, 4, 4, 512> {};
// tile of the 3D fused MAC sweep (k_mac_sweep)
using Mac3Tile = TileShape<32, 8, 8, 1024>;
// tile of the 3D coarse-level tensor smoother (k_tsmooth): a deeper tile
// than TileCfg<3> stages fewer halo cells per updated cell
using Tsm3Tile = TileShape<16, 8, 8, 1024>;
// tile of the one-colour 3D tensor sweep (k_trb3): one thread per cell of
// the colour; 8 rows deep, it stages 2.0 cells per updated cell against
// 2.4 for a 32x4x4 tile, and its FP64 stage (64 KB) still lets two blocks
// share a CU
using Trb3Tile = TileShape<32, 8, 4, 512>;
// Candidates of the 2D fused tensor sweep, chosen per level by the
// autotuner (index 0 is the default): the tile with its thread count, the
// most sweeps one launch may run (NSW), and whether b and the face
// viscosities are staged in LDS (k_tsweepN) or held in registers (k_tsweep2,
// one sweep per launch).
template <class CF_, int NSW_, bool STAGED_>
struct SweepCand {
    using CF = CF_;
    static constexpr int NSW = NSW_;
    static constexpr bool STAGED = STAGED_;
};
using Sweep2Cands = std::tuple<SweepCand<TileShape<64, 8, 1, 256>, 1, false>, SweepCand<TileShape<32, 16, 1, 256>, 1, false>,
                               SweepCand<TileShape<128, 4, 1, 256>, 1, false>, SweepCand<TileShape<32, 16, 1, 512>, 2, true>,
                               SweepCand<TileShape<64, 16, 1, 512>, 2, true>, SweepCand<TileShape<32, 16, 1, 1024>, 2, true>,
                               SweepCand<TileShape<16, 8, 1, 256>, 2, true>, SweepCand<TileShape<16, 8, 1, 1024>, 2, true>>;
static_assert(std::tuple_size_v<Sweep2Cands> == kSweep2Cands, "candidate count");


// Source of a tile position (i, j, k) that may lie outside the box:
// periodic axes wrap; across a wall the odd reflection about the wall reads
// the mirrored cell with the opposite sign (homogeneous ghost; arrays filled
// with `mirror` take the mirrored value itself, as the viscosity tile does);
// positions outside along two or more wall axes (never used by the stencil)
// read as 0.  Returns an in-range index always, with valid = false for the
// zero positions, so the loads of a fill issue without branches around them;
// src (optional) receives the source cell's coordinates.
template <int DIM>
__device__ inline long tile_src(const GridD& g, int i, int j, int k, bool& valid, bool& neg, int* src = nullptr)
{
    int p[3] = {i, j, k};
    int out = 0;
    valid = true;
    neg = false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int n = g.n[a];
        int v = p[a];
        const bool lo = v < 0, hi = v >= n;
        if (g.per[a]) {
            v = lo ? v + n : (hi ? v - n : v);
        } else if (lo || hi) {
            v = lo ? -1 - v : 2 * n - 1 - v;
            ++out;
            neg = !neg;
        }
        if (v < 0 || v >= n) {
            valid = false;
            v = 0;
        }
        p[a] = v;
    }
    if (out > 1) valid = false;
    if (src)
        for (int a = 0; a < 3; ++a) src[a] = p[a];
    return cid(g, p[0], p[1], p[2]);   // every p[a] is in range
}

// LDS tile with halo H around the interior box starting at (ox, oy, oz);
// array q at local (lx, ly, lz) is s[q * NS + (lz * SY + ly) * SX + lx]
template <int DIM, int H, class CF = TileCfg<DIM>>
struct Tile {
    static constexpr int TX = CF::TX, TY = CF::TY, TZ = CF::TZ;
    static constexpr int HZ = DIM == 3 ? H : 0;
    static constexpr int SX = TX + 2 * H, SY = TY + 2 * H, SZ = TZ + 2 * HZ;
    static constexpr int NS = SX * SY * SZ;
    __device__ static inline int at(int lx, int ly, int lz) { return (lz * SY + ly) * SX + lx; }
};

// Stage NA arrays (tile plus halo H) in LDS.  Every thread first issues all
// of its global loads into registers, then stores them, so the loads of a
// block are in flight together instead of one round trip per element.
template <int DIM, int H, int NA, typename R, class CF = TileCfg<DIM>>
__device__ inline void fill_batched(const GridD& g, const R* const* q, const bool* mirror, R* s, int ox, int oy,
                                    int oz)
{
    using T = Tile<DIM, H, CF>;
    constexpr int TH = CF::THREADS;
    constexpr int K = (T::NS + TH - 1) / TH;
    // tiles away from every domain face need no boundary logic
    const bool inner = ox - H >= 0 && ox + T::TX + H <= g.n[0] && oy - H >= 0 && oy + T::TY + H <= g.n[1] &&
                       (DIM == 2 || (oz - H >= 0 && oz + T::TZ + H <= g.n[2]));
    R v[NA][K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * TH;
        const int tt = t < T::NS ? t : 0;
        const int lx = tt % T::SX, ly = (tt / T::SX) % T::SY, lz = tt / (T::SX * T::SY);
        const int i = ox - H + lx, j = oy - H + ly, k = DIM == 3 ? oz - H + lz : 0;
        bool ok = true, ng = false;
        const long idx = inner ? cid(g, i, j, k) : tile_src<DIM>(g, i, j, k, ok, ng);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const R x = q[a] ? q[a][idx] : R(0);   // a null array reads as zeros
            v[a][u] = ok ? ((ng && !mirror[a]) ? -x : x) : R(0);
        }
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * TH;
        if (t < T::NS)
#pragma unroll
            for (int a = 0; a < NA; ++a) s[a * T::NS + t] = v[a][u];
    }
}

// fill of the 3D halo-1 tile for k_trb3: all arrays present, so no load is
// guarded
template <bool FINE, typename R, class CF>
__device__ inline void fill_tile1(const GridD& g, const R* const* q, const bool* mirror, R* s, int ox, int oy, int oz)
{
    using T = Tile<3, 1, CF>;
    constexpr int TH = CF::THREADS;
    constexpr int NA = FINE ? 4 : 3;
    constexpr int K = (T::NS + TH - 1) / TH;
    const bool inner = ox - 1 >= 0 && ox + T::TX + 1 <= g.n[0] && oy - 1 >= 0 && oy + T::TY + 1 <= g.n[1] &&
                       oz - 1 >= 0 && oz + T::TZ + 1 <= g.n[2];
    R v[NA][K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * TH;
        const int tt = t < T::NS ? t : 0;
        const int lx = tt % T::SX, ly = (tt / T::SX) % T::SY, lz = tt / (T::SX * T::SY);
        const int i = ox - 1 + lx, j = oy - 1 + ly, k = oz - 1 + lz;
        bool ok = true, ng = false;
        const long idx = inner ? cid(g, i, j, k) : tile_src<3>(g, i, j, k, ok, ng);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const R x = q[a][idx];
            v[a][u] = ok ? ((ng && !mirror[a]) ? -x : x) : R(0);
        }
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * TH;
        if (t < T::NS)
#pragma unroll
            for (int a = 0; a < NA; ++a) s[a * T::NS + t] = v[a][u];
    }
}

// the stencil above on a Tile<DIM, H> (compile-time strides)
template <int DIM, int H, bool FINE, typename R, class CF = TileCfg<DIM>>
__device__ inline R tile_visc_div(const GridD& g, const R* bfc, const R* s, const R* e, int c, const int G[3], int wm,
                                  int l0, R dt, R* diag)
{
    using T = Tile<DIM, H, CF>;
    (void)G;
    return visc_div_lds<DIM, FINE, R>(g, bfc, s, T::NS, T::SX, T::SX * T::SY, e, c, wm, l0, dt, diag);
}

// ---------------------------------------------------------------------------
// fused red-black sweep of component c
// ---------------------------------------------------------------------------

// cell of the active colour walked by thread slot t of a region (the tile
// plus `ring` cells); returns false when t is past the region or the cell lies
// beyond a wall.  Cells across a periodic boundary are the wrapped cells.
template <int DIM, class CF = TileCfg<DIM>>
__device__ inline bool colour_cell(const GridD& g, int t, int ring, int colour, int ox, int oy, int oz, int G[3],
                                   int L[3])
{
    using T = Tile<DIM, 2, CF>;
    const int RX = T::TX + 2 * ring, RY = T::TY + 2 * ring, RZ = DIM == 3 ? T::TZ + 2 * ring : 1;
    const int HX = RX / 2;
    if (t >= HX * RY * RZ) {
        // no cell: the tile's first cell, so that the slot's loads stay in range
        G[0] = ox;
        G[1] = oy;
        G[2] = oz;
        L[0] = L[1] = 2;
        L[2] = DIM == 3 ? 2 : 0;
        return false;
    }
    const int px = t % HX, ry = (t / HX) % RY, rz = t / (HX * RY);
    const int y0 = oy - ring + ry, z0 = DIM == 3 ? oz - ring + rz : 0, x0 = ox - ring;
    const int rx = 2 * px + ((x0 + y0 + z0 + colour) & 1);
    G[0] = x0 + rx;
    G[1] = y0;
    G[2] = z0;
    L[0] = rx - ring + 2;
    L[1] = ry - ring + 2;
    L[2] = DIM == 3 ? rz - ring + 2 : 0;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (G[a] >= 0 && G[a] < g.n[a]) continue;
        if (g.per[a]) G[a] = G[a] < 0 ? G[a] + g.n[a] : G[a] - g.n[a];
        if (G[a] < 0 || G[a] >= g.n[a]) inside = false;
    }
    return inside;
}

// dynamic LDS of the tile kernels, viewed as an array of R
extern __shared__ __align__(16) unsigned char tile_lds[];

// Batched launches: block z = cavity * zb + z-tile.  Each kernel finds its
// cavity's grid and array offsets in the level's tables (the arenas hold the
// cavities back to back, components of a cavity contiguous), returns when
// the cavity takes no part or the tile lies outside it, and then runs the
// single-grid body on that cavity's arrays.
#define TILE_ENTER(DIM, T)                                                                  \
    int cav, bz, tbx, tby, tbz;                                                             \
    GridD g;                                                                                \
    xcd_tile(tbx, tby, tbz);                                                                \
    if (!bv_enter_at(v, tbz, cav, bz, g)) return;                                           \
    const int ox = tbx * T::TX, oy = tby * T::TY, oz = (DIM == 3) ? bz * T::TZ : 0;          \
    if (ox >= g.n[0] || oy >= g.n[1] || oz >= g.n[2]) return;                               \
    const long cell0 = bv_o(v, cav);

template <int DIM, bool FINE, int c, typename R, class CF = TileCfg<DIM>>
__global__ void __launch_bounds__(CF::THREADS)
k_tsmooth(BV v, const R* __restrict__ coefa, const double* __restrict__ scb, const R* __restrict__ xcura,
          const R* xnext_ina, R* xnexta, const R* __restrict__ ba)
{
    using T = Tile<DIM, 2, CF>;
    TILE_ENTER(DIM, T);
    const R dt = (R)vload(scb + (long)cav * S_NSLOT + S_DT);
    const R* coef = FINE ? coefa + cell0 : coefa + bv_of(v, cav);
    const R* xcur = xcura + DIM * cell0;
    const R* xnext_in = xnext_ina + DIM * cell0;
    R* xnext = xnexta + DIM * cell0;
    const R* b = ba + DIM * cell0;
    constexpr int TH = CF::THREADS;
    constexpr int RZ1 = DIM == 3 ? T::TZ + 2 : 1;
    constexpr int KR = ((T::TX + 2) / 2 * (T::TY + 2) * RZ1 + TH - 1) / TH;   // red slots per thread
    constexpr int KB = (T::TX / 2 * T::TY * T::TZ + TH - 1) / TH;            // black slots per thread
    R* s = reinterpret_cast<R*>(tile_lds);
    R* e = s + DIM * T::NS;     // eta/Re tile (FINE)
    const long N = ncells(g);
    const R* bc = b + c * N;
    // this thread's cells of each colour, and their right-hand sides
    constexpr int NF = FINE ? 1 : 2 * DIM;
    int rG[KR][3], rL[KR];
    bool rOk[KR];
    R rB[KR], rF[KR][NF];
#pragma unroll
    for (int u = 0; u < KR; ++u) {
        int L[3];
        rOk[u] = colour_cell<DIM, CF>(g, threadIdx.x + u * TH, 1, 0, ox, oy, oz, rG[u], L);
        rL[u] = T::at(L[0], L[1], L[2]);
        rB[u] = bc[cid_clamped(g, rG[u])];
        if (!FINE) load_faces<DIM, R>(g, coef, rG[u], rF[u]);
    }
    int kG[KB][3], kL[KB];
    bool kOk[KB];
    R kB[KB], kF[KB][NF];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
        int L[3];
        kOk[u] = colour_cell<DIM, CF>(g, threadIdx.x + u * TH, 0, 1, ox, oy, oz, kG[u], L);
        kL[u] = T::at(L[0], L[1], L[2]);
        kB[u] = bc[cid_clamped(g, kG[u])];
        if (!FINE) load_faces<DIM, R>(g, coef, kG[u], kF[u]);
    }
    // components already swept in this sweep live in the next buffer
    {
        const R* q[DIM + 1];
        bool mir[DIM + 1];
        for (int a = 0; a < DIM; ++a) { q[a] = (a < c ? xnext_in : xcur) + a * N; mir[a] = false; }
        q[DIM] = coef;
        mir[DIM] = true;
        fill_batched<DIM, 2, DIM + (FINE ? 1 : 0), R, CF>(g, q, mir, s, ox, oy, oz);
    }
    __syncthreads();
    R* sc = s + c * T::NS;
    // red cells of the tile and its 1-cell ring, then black cells of the
    // tile; a cell of one colour reads only the other colour of component c
    // (face neighbours) and the other components, so each colour is updated
    // in place.  Every slot within the colour's region is evaluated (region
    // positions beyond the box on an in-range cell) and only real cells are
    // stored, so a phase is straight-line code whose LDS reads issue
    // together; slots past the region (whole waves, but for one) skip it.
    constexpr int NR = (T::TX + 2) / 2 * (T::TY + 2) * RZ1, NB = T::TX / 2 * T::TY * T::TZ;
    {
        R nv[KR];
#pragma unroll
        for (int u = 0; u < KR; ++u) {
            if (threadIdx.x + u * TH >= NR) continue;
            R dg;
            const R vd =
                tile_visc_div<DIM, 2, FINE, R, CF>(g, rF[u], s, e, c, rG[u], wall_mask<DIM>(g, rG[u]), rL[u], dt, &dg);
            const R xc = sc[rL[u]];
            const R Au = xc - dt * vd;
            nv[u] = xc + (rB[u] - Au) / dg;
        }
#pragma unroll
        for (int u = 0; u < KR; ++u)
            if (rOk[u]) sc[rL[u]] = nv[u];
    }
    __syncthreads();
    {
        R nv[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            if (threadIdx.x + u * TH >= NB) continue;
            R dg;
            const R vd =
                tile_visc_div<DIM, 2, FINE, R, CF>(g, kF[u], s, e, c, kG[u], wall_mask<DIM>(g, kG[u]), kL[u], dt, &dg);
            const R xc = sc[kL[u]];
            const R Au = xc - dt * vd;
            nv[u] = xc + (kB[u] - Au) / dg;
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (kOk[u]) sc[kL[u]] = nv[u];
    }
    __syncthreads();
    // write the tile's cells of component c
    R* xo = xnext + c * N;
    for (int t = threadIdx.x; t < T::TX * T::TY * T::TZ; t += blockDim.x) {
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        const int G[3] = {ox + rx, oy + ry, DIM == 3 ? oz + rz : 0};
        if (G[0] >= g.n[0] || G[1] >= g.n[1] || G[2] >= g.n[2]) continue;
        xo[cid(g, G[0], G[1], G[2])] = sc[T::at(rx + 2, ry + 2, DIM == 3 ? rz + 2 : 0)];
    }
}

// ---------------------------------------------------------------------------
// 2D: both components of a sweep in one launch.  The sweep's four half
// steps (component 0 red, black, component 1 red, black) run on the tile
// grown by 3, 2, 1 and 0 rings: each half step reads values of the previous
// ones at most one cell away (face neighbours of its own component, the
// other component at face and diagonal neighbours), so a halo of 4 cells
// covers the sweep.  Component 1 reads component 0 at the wall ghosts as
// well, so each update of a wall cell also writes its odd reflection into
// the ghost position.  Every cell sees the values of the one-component-per-
// launch order, so the result is the same bit for bit.
// ---------------------------------------------------------------------------

// cell of colour `colour` for slot t of the tile grown by `ring` (halo H
// layout); as colour_cell
template <int H, class CF>
__device__ inline bool colour_cell2(const GridD& g, int t, int ring, int colour, int ox, int oy, int G[3], int& L)
{
    using T = Tile<2, H, CF>;
    const int RX = T::TX + 2 * ring, RY = T::TY + 2 * ring, HX = RX / 2;
    if (t >= HX * RY) {
        G[0] = ox;
        G[1] = oy;
        G[2] = 0;
        L = T::at(H, H, 0);
        return false;
    }
    const int px = t % HX, ry = t / HX;
    const int y0 = oy - ring + ry, x0 = ox - ring;
    const int rx = 2 * px + ((x0 + y0 + colour) & 1);
    G[0] = x0 + rx;
    G[1] = y0;
    G[2] = 0;
    L = T::at(rx - ring + H, ry - ring + H, 0);
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (G[a] >= 0 && G[a] < g.n[a]) continue;
        if (g.per[a]) G[a] = G[a] < 0 ? G[a] + g.n[a] : G[a] - g.n[a];
        if (G[a] < 0 || G[a] >= g.n[a]) inside = false;
    }
    return inside;
}

// one half step of the fused sweep: K slots per thread
template <int C, int COLOUR, int RING, int K, bool FINE, typename R, class CF>
struct HalfStep {
    static constexpr int NF = FINE ? 1 : 4;
    int G[K][3], L[K];
    bool ok[K];
    R bq[K], bf[K][NF];

    __device__ inline void setup(const GridD& g, int ox, int oy, const R* __restrict__ bc, const R* __restrict__ coef)
    {
        constexpr int TH = CF::THREADS;
#pragma unroll
        for (int u = 0; u < K; ++u) {
            ok[u] = colour_cell2<4, CF>(g, threadIdx.x + u * TH, RING, COLOUR, ox, oy, G[u], L[u]);
            bq[u] = bc[cid_clamped(g, G[u])];
            if (!FINE) load_faces<2, R>(g, coef, G[u], bf[u]);
        }
    }

    __device__ inline void run(const GridD& g, R* s, const R* e, R dt)
    {
        using T = Tile<2, 4, CF>;
        R* sc = s + C * T::NS;
        R nv[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            R dg;
            const R vd =
                tile_visc_div<2, 4, FINE, R, CF>(g, bf[u], s, e, C, G[u], wall_mask<2>(g, G[u]), L[u], dt, &dg);
            const R xc = sc[L[u]];
            const R Au = xc - dt * vd;
            nv[u] = xc + (bq[u] - Au) / dg;
        }
        const int off[2] = {1, T::SX};
#pragma unroll
        for (int u = 0; u < K; ++u) {
            if (!ok[u]) continue;
            sc[L[u]] = nv[u];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (g.per[a]) continue;
                if (G[u][a] == 0) sc[L[u] - off[a]] = -nv[u];
                else if (G[u][a] == g.n[a] - 1) sc[L[u] + off[a]] = -nv[u];
            }
        }
    }
};

template <bool FINE, typename R, class CF>
__global__ void __launch_bounds__(CF::THREADS)
k_tsweep2(BV v, const R* __restrict__ coefa, const double* __restrict__ scb, const R* __restrict__ xcura,
          R* __restrict__ xnexta, const R* __restrict__ ba)
{
    using T = Tile<2, 4, CF>;
    constexpr int TH = CF::THREADS;
    constexpr int K0 = ((T::TX + 6) / 2 * (T::TY + 6) + TH - 1) / TH;
    constexpr int K1 = ((T::TX + 4) / 2 * (T::TY + 4) + TH - 1) / TH;
    constexpr int K2 = ((T::TX + 2) / 2 * (T::TY + 2) + TH - 1) / TH;
    constexpr int K3 = (T::TX / 2 * T::TY + TH - 1) / TH;
    TILE_ENTER(2, T);
    const R dt = (R)vload(scb + (long)cav * S_NSLOT + S_DT);
    const R* coef = FINE ? coefa + cell0 : coefa + bv_of(v, cav);
    // xcura == nullptr: the sweep starts from zeros
    const R* xcur = xcura ? xcura + 2 * cell0 : nullptr;
    R* xnext = xnexta + 2 * cell0;
    const R* b = ba + 2 * cell0;
    const long N = ncells(g);
    R* s = reinterpret_cast<R*>(tile_lds);
    R* e = s + 2 * T::NS;
    HalfStep<0, 0, 3, K0, FINE, R, CF> h0;
    HalfStep<0, 1, 2, K1, FINE, R, CF> h1;
    HalfStep<1, 0, 1, K2, FINE, R, CF> h2;
    HalfStep<1, 1, 0, K3, FINE, R, CF> h3;
    h0.setup(g, ox, oy, b, coef);
    h1.setup(g, ox, oy, b, coef);
    h2.setup(g, ox, oy, b + N, coef);
    h3.setup(g, ox, oy, b + N, coef);
    {
        const R* q[3] = {xcur, xcur ? xcur + N : nullptr, coef};
        const bool mir[3] = {false, false, true};
        fill_batched<2, 4, FINE ? 3 : 2, R, CF>(g, q, mir, s, ox, oy, 0);
    }
    __syncthreads();
    h0.run(g, s, e, dt);
    __syncthreads();
    h1.run(g, s, e, dt);
    __syncthreads();
    h2.run(g, s, e, dt);
    __syncthreads();
    h3.run(g, s, e, dt);
    __syncthreads();
    for (int t = threadIdx.x; t < 2 * T::TX * T::TY; t += TH) {
        const int q = t / (T::TX * T::TY), r = t - q * (T::TX * T::TY);
        const int rx = r % T::TX, ry = r / T::TX;
        const int G[2] = {ox + rx, oy + ry};
        if (G[0] >= g.n[0] || G[1] >= g.n[1]) continue;
        xnext[q * N + cid(g, G[0], G[1], 0)] = s[q * T::NS + T::at(rx + 4, ry + 4, 0)];
    }
}

// ---------------------------------------------------------------------------
// 2D: NSW whole sweeps (both components) in one launch, everything staged.
// The 4 NSW half steps run on the tile grown by 4 NSW - 1, ..., 1, 0 rings
// (the ring argument above, applied once per half step), on a tile with a
// halo of 4 NSW.  Besides both components of x, the fill stages both
// components of b and the face viscosities (coarse levels: beta on the low x
// and the low y face of each position; finest level: eta/Re) in LDS, so a
// half step reads no global memory and holds nothing in registers across
// the barriers.  The arithmetic per cell is that of k_tsweep2, so NSW = 2
// gives bit for bit the result of two launches of one sweep.  A periodic
// extent must be at least the halo (positions wrap once).
// ---------------------------------------------------------------------------

// LDS arrays of the staged tile, each Tile<2, H, CF>::NS long
enum { ST_X0 = 0, ST_X1 = 1, ST_B0 = 2, ST_B1 = 3, ST_E = 4, ST_FX = 4, ST_FY = 5 };

// Prolongation correction (P e)_q at fine cell (si, sj) from the coarse
// iterate e (components Nc apart) on grid gc: the 2^2 nearest coarse cells
// with axis weights 3/4 and 1/4; a coarse neighbour beyond a wall is the
// cell itself with the homogeneous ghost sign wsign (tensor problem -1,
// MAC problem +1).  Same terms, order and
// rounding as the prolongation kernel.
// Prolongation correction (P e)_q at fine cell (si, sj) from the coarse
// iterate e (components Nc apart) on grid gc: the 2^2 nearest coarse cells
// with axis weights 3/4 and 1/4; a coarse neighbour beyond a wall is the
// cell itself with the homogeneous ghost sign wsign (tensor problem -1,
// MAC problem +1).  Same terms, order and rounding as the prolongation
// kernel.  Split in two so that a fill can issue every load before it adds
// anything: prolong_src gives the four coarse indices (order: the cell, its
// x neighbour, its y neighbour, the diagonal) and the signs per axis,
// prolong_sum the correction from the four loaded values.
template <typename R>
__device__ inline void prolong_src(const GridD& gc, int si, int sj, R wsign, long q[4], R sgn[2])
{
    const int C[2] = {si >> 1, sj >> 1}, ch[2] = {si & 1, sj & 1};
    int J[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        int J2 = C[a] + (ch[a] ? 1 : -1);
        R sg = 1;
        if (J2 < 0 || J2 >= gc.n[a]) {
            if (gc.per[a]) J2 = J2 < 0 ? J2 + gc.n[a] : J2 - gc.n[a];
            else { J2 = C[a]; sg = wsign; }
        }
        J[a] = J2;
        sgn[a] = sg;
    }
    q[0] = (long)C[1] * gc.n[0] + C[0];
    q[1] = (long)C[1] * gc.n[0] + J[0];
    q[2] = (long)J[1] * gc.n[0] + C[0];
    q[3] = (long)J[1] * gc.n[0] + J[0];
}

template <typename R>
__device__ inline R prolong_sum(const R nb[4], const R sgn[2])
{
    R s = 0;
#pragma unroll
    for (int bits = 0; bits < 4; ++bits) {
        R w = 1, sg = 1;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (!((bits >> a) & 1)) { w *= R(0.75); continue; }
            w *= R(0.25);
            sg *= sgn[a];
        }
        s += w * sg * nb[bits];
    }
    return s;
}

template <typename R>
__device__ inline R prolong_at(const GridD& gc, const R* __restrict__ e, int si, int sj, R wsign)
{
    long q[4];
    R sgn[2], nb[4];
    prolong_src<R>(gc, si, sj, wsign, q, sgn);
#pragma unroll
    for (int k = 0; k < 4; ++k) nb[k] = e[q[k]];
    return prolong_sum<R>(nb, sgn);
}

// coarse patch of a tile whose prolonged positions need no coarse cell
// beyond the grid: PW x PH coarse cells per component, from (cx0, cy0)
template <int H, class CF>
struct CoarsePatch {
    static constexpr int PW = (CF::TX + 2 * H) / 2 + 2, PH = (CF::TY + 2 * H) / 2 + 2, PN = PW * PH;
};

// PRO: x of the fill is x + P e (the coarse correction of a V-cycle folded
// into the first sweep after it): pe the coarse iterate, gc its grid.  Where
// every coarse value the tile's positions read lies inside the coarse grid
// (no wall image, no periodic wrap), the block first stages that coarse
// patch in LDS (patch: 2 PN values after the staged arrays) and reads the
// four values of each position from it; elsewhere each position reads them
// from global memory after its other loads.  Either way a position adds the
// same four values in the same order as the prolongation kernel.
template <bool FINE, int H, typename R, class CF, bool PRO>
__device__ inline void fill_staged(const GridD& g, const R* __restrict__ x, const R* __restrict__ b,
                                   const R* __restrict__ coef, R* s, int ox, int oy, long N,
                                   const R* __restrict__ pe, const GridD& gc)
{
    using T = Tile<2, H, CF>;
    constexpr int TH = CF::THREADS;
    constexpr int K = (T::NS + TH - 1) / TH;
    constexpr int NA = FINE ? 5 : 6;
    const bool inner = ox - H >= 0 && ox + T::TX + H <= g.n[0] && oy - H >= 0 && oy + T::TY + H <= g.n[1];
    const long fo1 = FINE ? 0 : foffset(g, 1);
    R v[NA][K];
    bool pok[K], png[K];
    constexpr int KP = PRO ? K : 1;
    int sx[KP], sy[KP];   // PRO: the source cell of each position
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * TH;
        const int tt = t < T::NS ? t : 0;
        const int lx = tt % T::SX, ly = tt / T::SX;
        const int i = ox - H + lx, j = oy - H + ly;
        bool ok = true, ng = false;
        int src[3] = {i, j, 0};
        const long idx = inner ? cid(g, i, j, 0) : tile_src<2>(g, i, j, 0, ok, ng, src);
        pok[u] = ok;
        png[u] = ng;
        if constexpr (PRO) {
            sx[u] = src[0];
            sy[u] = src[1];
        }
        v[ST_X0][u] = x ? x[idx] : R(0);
        v[ST_X1][u] = x ? x[N + idx] : R(0);
        // b is read only at cells that are updated, which lie in the box
        v[ST_B0][u] = b[idx];
        v[ST_B1][u] = b[N + idx];
        if (FINE) {
            v[ST_E][u] = coef[idx];
        } else {
            // position (i, j) holds the faces on its low x and low y side:
            // wrapped once along periodic axes, then clamped to the face
            // range (clamped values are read only by cells outside the box
            // or beyond the one wrap, whose results are not kept)
            int wi = i, wj = j;
            if (g.per[0]) wi = i < 0 ? i + g.n[0] : (i >= g.n[0] ? i - g.n[0] : i);
            if (g.per[1]) wj = j < 0 ? j + g.n[1] : (j >= g.n[1] ? j - g.n[1] : j);
            const int ax = min(max(wi, 0), g.n[0] - g.per[0]);
            const int ay = min(max(wj, 0), g.n[1] - 1);
            const int bx = min(max(wi, 0), g.n[0] - 1);
            const int by = min(max(wj, 0), g.n[1] - g.per[1]);
            v[ST_FX][u] = coef[fid(g, 0, ax, ay, 0)];
            v[ST_FY][u] = coef[fo1 + fid(g, 1, bx, by, 0)];
        }
    }
    if constexpr (PRO) {
        const long Nc = ncells(gc);
        // positions 2 .. n - 3 along both axes: coarse cells C and C +- 1
        // inside the coarse grid
        const bool in_patch = ox - H >= 2 && ox + T::TX + H <= g.n[0] - 2 && oy - H >= 2 &&
                              oy + T::TY + H <= g.n[1] - 2;
        if (in_patch) {
            using P = CoarsePatch<H, CF>;
            R* patch = s + NA * T::NS;
            const int cx0 = (ox - H) / 2 - 1, cy0 = (oy - H) / 2 - 1;
            constexpr int KQ = (2 * P::PN + TH - 1) / TH;
            R cp[KQ];
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const int t = threadIdx.x + q * TH;
                const int tt = t < 2 * P::PN ? t : 0;
                const int c = tt / P::PN, r = tt - c * P::PN;
                const int py = r / P::PW, px = r - py * P::PW;
                cp[q] = pe[c * Nc + cid(gc, cx0 + px, cy0 + py, 0)];
            }
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                const int t = threadIdx.x + q * TH;
                if (t < 2 * P::PN) patch[t] = cp[q];
            }
            __syncthreads();
            const R one[2] = {R(1), R(1)};
#pragma unroll
            for (int u = 0; u < K; ++u) {
                const int C0 = sx[u] >> 1, C1 = sy[u] >> 1;
                const int J0 = C0 + ((sx[u] & 1) ? 1 : -1), J1 = C1 + ((sy[u] & 1) ? 1 : -1);
                const int at[4] = {(C1 - cy0) * P::PW + (C0 - cx0), (C1 - cy0) * P::PW + (J0 - cx0),
                                   (J1 - cy0) * P::PW + (C0 - cx0), (J1 - cy0) * P::PW + (J0 - cx0)};
                R n0[4], n1[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    n0[k] = patch[at[k]];
                    n1[k] = patch[P::PN + at[k]];
                }
                v[ST_X0][u] = v[ST_X0][u] + prolong_sum<R>(n0, one);
                v[ST_X1][u] = v[ST_X1][u] + prolong_sum<R>(n1, one);
            }
        } else {
#pragma unroll
            for (int u = 0; u < K; ++u) {
                long q[4];
                R sg[2], n0[4], n1[4];
                prolong_src<R>(gc, sx[u], sy[u], R(-1), q, sg);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    n0[k] = pe[q[k]];
                    n1[k] = pe[Nc + q[k]];
                }
                v[ST_X0][u] = v[ST_X0][u] + prolong_sum<R>(n0, sg);
                v[ST_X1][u] = v[ST_X1][u] + prolong_sum<R>(n1, sg);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const R x0 = v[ST_X0][u], x1 = v[ST_X1][u];
        v[ST_X0][u] = pok[u] ? (png[u] ? -x0 : x0) : R(0);
        v[ST_X1][u] = pok[u] ? (png[u] ? -x1 : x1) : R(0);
        if (FINE) v[ST_E][u] = pok[u] ? v[ST_E][u] : R(0);
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * TH;
        if (t < T::NS)
#pragma unroll
            for (int a = 0; a < NA; ++a) s[a * T::NS + t] = v[a][u];
    }
}

// one half step (component C, colour COLOUR, tile grown by RING) of the
// staged sweep; the same per-cell arithmetic and ghost updates as HalfStep
template <int C, int COLOUR, int RING, int H, bool FINE, typename R, class CF>
__device__ inline void staged_half(const GridD& g, R* s, R dt, R ihh, int ox, int oy)
{
    using T = Tile<2, H, CF>;
    constexpr int TH = CF::THREADS;
    constexpr int K = ((T::TX + 2 * RING) / 2 * (T::TY + 2 * RING) + TH - 1) / TH;
    R* sc = s + C * T::NS;
    const R* sb = s + (ST_B0 + C) * T::NS;
    const R* e = s + ST_E * T::NS;
    const R* fx = s + ST_FX * T::NS;
    const R* fy = s + ST_FY * T::NS;
    int G[K][3], L[K];
    bool ok[K];
    R nv[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        ok[u] = colour_cell2<H, CF>(g, threadIdx.x + u * TH, RING, COLOUR, ox, oy, G[u], L[u]);
        const int l = L[u];
        R bf[4];
        if (!FINE) {
            bf[0] = fx[l];
            bf[1] = fx[l + 1];
            bf[2] = fy[l];
            bf[3] = fy[l + T::SX];
        }
        R dg;
        const R vd = visc_div_ih<2, FINE, R>(bf, s, T::NS, T::SX, T::SX * T::SY, e, C, wall_mask<2>(g, G[u]), l, dt,
                                             ihh, &dg);
        const R xc = sc[l];
        const R Au = xc - dt * vd;
        nv[u] = xc + (sb[l] - Au) / dg;
    }
    const int off[2] = {1, T::SX};
#pragma unroll
    for (int u = 0; u < K; ++u) {
        if (!ok[u]) continue;
        sc[L[u]] = nv[u];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (g.per[a]) continue;
            if (G[u][a] == 0) sc[L[u] - off[a]] = -nv[u];
            else if (G[u][a] == g.n[a] - 1) sc[L[u] + off[a]] = -nv[u];
        }
    }
}

// sweep SW of NSW on a tile with halo H: its four half steps, each
// followed by a barrier (rings H - 1 - 4 SW down to H - 4 - 4 SW)
template <int SW, int NSW, int H, bool FINE, typename R, class CF>
__device__ inline void staged_sweeps(const GridD& g, R* s, R dt, R ihh, int ox, int oy)
{
    if constexpr (SW < NSW) {
        constexpr int R0 = H - 1 - 4 * SW;
        staged_half<0, 0, R0, H, FINE, R, CF>(g, s, dt, ihh, ox, oy);
        __syncthreads();
        staged_half<0, 1, R0 - 1, H, FINE, R, CF>(g, s, dt, ihh, ox, oy);
        __syncthreads();
        staged_half<1, 0, R0 - 2, H, FINE, R, CF>(g, s, dt, ihh, ox, oy);
        __syncthreads();
        staged_half<1, 1, R0 - 3, H, FINE, R, CF>(g, s, dt, ihh, ox, oy);
        __syncthreads();
        staged_sweeps<SW + 1, NSW, H, FINE, R, CF>(g, s, dt, ihh, ox, oy);
    }
}

// RES: the launch ends a pre-smoothing; it also forms the residual of the
// tile's cells and restricts it to the coarse level (coarse b = mean of the
// 2x2 children, coarse x = 0), as the residual-restriction kernel would
// after it.  The sweeps then run one ring wider (halo 4 NSW + 1, last half
// step on ring 1), so every value the residual reads is final.
// waves per SIMD asked of the register allocator: the finest level's launch
// that folds in the prolongation is held to two workgroups per compute unit
// where its LDS fits twice (160 KB per CU), so a launch over twice as many
// tiles as compute units runs in one round
template <bool FINE, typename R, class CF, int NSW, bool PRO, bool RES>
constexpr int tsweep_waves()
{
    constexpr size_t lds = sizeof(R) * ((FINE ? 5 : 6) * Tile<2, 4 * NSW + (RES ? 1 : 0), CF>::NS +
                                        (PRO ? 2 * CoarsePatch<4 * NSW, CF>::PN : 0));
    return FINE && PRO && 2 * lds <= 160 * 1024 ? 2 * CF::THREADS / 256 : 1;
}

template <bool FINE, typename R, class CF, int NSW, bool PRO, bool RES>
__global__ void __launch_bounds__(CF::THREADS, (tsweep_waves<FINE, R, CF, NSW, PRO, RES>()))
k_tsweepN(BV v, const R* __restrict__ coefa, const double* __restrict__ scb, const R* __restrict__ xcura,
          R* __restrict__ xnexta, const R* __restrict__ ba, const R* __restrict__ pea, const GridD* __restrict__ gct,
          const long* __restrict__ oct, R* __restrict__ bca, R* __restrict__ xca)
{
    static_assert(!(PRO && RES), "a launch either starts a post-smoothing or ends a pre-smoothing");
    constexpr int H = 4 * NSW + (RES ? 1 : 0);
    using T = Tile<2, H, CF>;
    constexpr int TH = CF::THREADS;
    TILE_ENTER(2, T);
    const R dt = (R)vload(scb + (long)cav * S_NSLOT + S_DT);
    const R* coef = FINE ? coefa + cell0 : coefa + bv_of(v, cav);
    // xcura == nullptr: the sweeps start from zeros
    const R* xcur = xcura ? xcura + 2 * cell0 : nullptr;
    R* xnext = xnexta + 2 * cell0;
    const R* b = ba + 2 * cell0;
    const long N = ncells(g);
    R* s = reinterpret_cast<R*>(tile_lds);
    GridD gc = g;
    const R* pe = nullptr;
    if (PRO || RES) gc = bv_g2(v, gct, cav);
    if (PRO) pe = pea + 2 * bv_o2(v, oct, cav);
    fill_staged<FINE, H, R, CF, PRO>(g, xcur, b, coef, s, ox, oy, N, pe, gc);
    const R h = (R)g.h;
    const R ihh = R(1) / (h * h);
    __syncthreads();
    staged_sweeps<0, NSW, H, FINE, R, CF>(g, s, dt, ihh, ox, oy);
    for (int t = threadIdx.x; t < 2 * T::TX * T::TY; t += TH) {
        const int q = t / (T::TX * T::TY), r = t - q * (T::TX * T::TY);
        const int rx = r % T::TX, ry = r / T::TX;
        const int G[2] = {ox + rx, oy + ry};
        if (G[0] >= g.n[0] || G[1] >= g.n[1]) continue;
        xnext[q * N + cid(g, G[0], G[1], 0)] = s[q * T::NS + T::at(rx + H, ry + H, 0)];
    }
    if constexpr (RES) {
        // residual of the tile's cells (both components), then the 2x2 means
        constexpr int NT = T::TX * T::TY;
        R* rr = s + (FINE ? 5 : 6) * T::NS;
        const R* e = s + ST_E * T::NS;
        const R* fx = s + ST_FX * T::NS;
        const R* fy = s + ST_FY * T::NS;
        for (int t = threadIdx.x; t < NT; t += TH) {
            const int rx = t % T::TX, ry = t / T::TX;
            const int G[3] = {ox + rx, oy + ry, 0};
            if (G[0] >= g.n[0] || G[1] >= g.n[1]) continue;
            const int l = T::at(rx + H, ry + H, 0);
            R bf[4];
            if (!FINE) {
                bf[0] = fx[l];
                bf[1] = fx[l + 1];
                bf[2] = fy[l];
                bf[3] = fy[l + T::SX];
            }
            const int wm = wall_mask<2>(g, G);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const R vd = visc_div_ih<2, FINE, R>(bf, s, T::NS, T::SX, T::SX * T::SY, e, c, wm, l, dt, ihh, nullptr);
                const R Ax = s[c * T::NS + l] - dt * vd;
                rr[c * NT + t] = s[(ST_B0 + c) * T::NS + l] - Ax;
            }
        }
        __syncthreads();
        R* bcoarse = bca + 2 * bv_o2(v, oct, cav);
        R* xcoarse = xca + 2 * bv_o2(v, oct, cav);
        const long Nc = ncells(gc);
        constexpr int CX = T::TX / 2, CY = T::TY / 2;
        for (int t = threadIdx.x; t < CX * CY; t += TH) {
            const int cx = t % CX, cy = t / CX;
            const int C[2] = {ox / 2 + cx, oy / 2 + cy};
            if (C[0] >= gc.n[0] || C[1] >= gc.n[1]) continue;
            const long qc = cid(gc, C[0], C[1], 0);
            for (int c = 0; c < 2; ++c) {
                R sum = 0;
                for (int bits = 0; bits < 4; ++bits) {
                    const int fxc = 2 * cx + (bits & 1), fyc = 2 * cy + ((bits >> 1) & 1);
                    sum += rr[c * NT + fyc * T::TX + fxc];
                }
                bcoarse[c * Nc + qc] = sum / R(4);
                xcoarse[c * Nc + qc] = R(0);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// MAC problem: both colours of a red-black sweep in one launch.  Red cells
// of the tile and its 1-cell ring, then black cells of the tile, on the tile
// plus a 2-cell halo staged in LDS (read from cur; the tile is written to
// next).  A neighbour beyond a wall is masked (zero flux), as in the
// one-colour kernel, whose per-cell arithmetic this repeats, so the result
// is the same bit for bit.
// ---------------------------------------------------------------------------
template <int DIM, typename R, class CF = TileCfg<DIM>>
__global__ void __launch_bounds__(CF::THREADS)
k_mac_sweep(BV v, const R* __restrict__ cura, R* __restrict__ nexta, const R* __restrict__ ba)
{
    using T = Tile<DIM, 2, CF>;
    TILE_ENTER(DIM, T);
    constexpr int TH = CF::THREADS;
    constexpr int RZ1 = DIM == 3 ? T::TZ + 2 : 1;
    constexpr int KR = ((T::TX + 2) / 2 * (T::TY + 2) * RZ1 + TH - 1) / TH;
    constexpr int KB = (T::TX / 2 * T::TY * T::TZ + TH - 1) / TH;
    const R* cur = cura + cell0;
    R* next = nexta + cell0;
    const R* b = ba + cell0;
    R* s = reinterpret_cast<R*>(tile_lds);
    const R h = (R)g.h;
    const R ih2 = R(1) / (h * h);
    const int off[3] = {1, T::SX, T::SX * T::SY};
    // a colour's slots: LDS index, neighbour mask (bit 2a + side), diagonal, b
    auto setup = [&](int t, int ring, int colour, int& L, int& m, R& dg, R& bq) {
        int G[3], Lc[3];
        const bool ok = colour_cell<DIM, CF>(g, t, ring, colour, ox, oy, oz, G, Lc);
        L = T::at(Lc[0], Lc[1], Lc[2]);
        int cnt = 0;
        m = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const bool okl = g.per[a] || G[a] > 0, okh = g.per[a] || G[a] + 1 < g.n[a];
            m |= (okl ? 1 : 0) << (2 * a);
            m |= (okh ? 2 : 0) << (2 * a);
            cnt += (okl ? 1 : 0) + (okh ? 1 : 0);
        }
        dg = -(R)cnt * ih2;
        bq = b[cid_clamped(g, G)];
        return ok;
    };
    int rL[KR], rM[KR], kL[KB], kM[KB];
    bool rOk[KR], kOk[KB];
    R rD[KR], rB[KR], kD[KB], kB[KB];
#pragma unroll
    for (int u = 0; u < KR; ++u) rOk[u] = setup(threadIdx.x + u * TH, 1, 0, rL[u], rM[u], rD[u], rB[u]);
#pragma unroll
    for (int u = 0; u < KB; ++u) kOk[u] = setup(threadIdx.x + u * TH, 0, 1, kL[u], kM[u], kD[u], kB[u]);
    {
        const R* q[1] = {cur};
        const bool mir[1] = {false};
        fill_batched<DIM, 2, 1, R, CF>(g, q, mir, s, ox, oy, oz);
    }
    __syncthreads();
    auto update = [&](int l, int m, R dg, R bq) {
        const R xq = s[l];
        R xn[DIM][2];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            xn[a][0] = s[l - off[a]];
            xn[a][1] = s[l + off[a]];
        }
        R Lx = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool ok = (m >> (2 * a + side)) & 1;
                Lx += ok ? (xn[a][side] - xq) * ih2 : R(0);
            }
        return xq + (bq - Lx) / dg;
    };
    {
        R nv[KR];
#pragma unroll
        for (int u = 0; u < KR; ++u) nv[u] = update(rL[u], rM[u], rD[u], rB[u]);
#pragma unroll
        for (int u = 0; u < KR; ++u)
            if (rOk[u]) s[rL[u]] = nv[u];
    }
    __syncthreads();
    {
        R nv[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) nv[u] = update(kL[u], kM[u], kD[u], kB[u]);
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (kOk[u]) s[kL[u]] = nv[u];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < T::TX * T::TY * T::TZ; t += TH) {
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        const int G[3] = {ox + rx, oy + ry, DIM == 3 ? oz + rz : 0};
        if (G[0] >= g.n[0] || G[1] >= g.n[1] || G[2] >= g.n[2]) continue;
        next[cid(g, G[0], G[1], G[2])] = s[T::at(rx + 2, ry + 2, DIM == 3 ? rz + 2 : 0)];
    }
}

// ---------------------------------------------------------------------------
// MAC problem, 2D: NSW whole red-black sweeps in one launch.  x and b of the
// tile plus a halo of 2 NSW are staged in LDS; the half steps (red, black,
// ...) walk the tile grown by 2 NSW - 1, ..., 0 rings (each reads face
// neighbours only), so NSW = 2 gives bit for bit the result of two one-sweep
// launches.  PRO: the fill adds the prolongation of the coarse correction
// (wall sign +1), as the prolongation kernel would have before the sweep.
// Per-cell arithmetic as k_mac_sweep.
// ---------------------------------------------------------------------------
template <int COLOUR, int RING, int H, typename R, class CF>
__device__ inline void mac_half(const GridD& g, R* s, R ih2, int ox, int oy)
{
    using T = Tile<2, H, CF>;
    constexpr int TH = CF::THREADS;
    constexpr int K = ((T::TX + 2 * RING) / 2 * (T::TY + 2 * RING) + TH - 1) / TH;
    const R* sb = s + T::NS;
    const int off[2] = {1, T::SX};
    int L[K];
    bool ok[K];
    R nv[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        int G[3];
        ok[u] = colour_cell2<H, CF>(g, threadIdx.x + u * TH, RING, COLOUR, ox, oy, G, L[u]);
        const int l = L[u];
        int m = 0, cnt = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const bool okl = g.per[a] || G[a] > 0, okh = g.per[a] || G[a] + 1 < g.n[a];
            m |= (okl ? 1 : 0) << (2 * a);
            m |= (okh ? 2 : 0) << (2 * a);
            cnt += (okl ? 1 : 0) + (okh ? 1 : 0);
        }
        const R dg = -(R)cnt * ih2;
        const R xq = s[l];
        R xn[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            xn[a][0] = s[l - off[a]];
            xn[a][1] = s[l + off[a]];
        }
        R Lx = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const bool okf = (m >> (2 * a + side)) & 1;
                Lx += okf ? (xn[a][side] - xq) * ih2 : R(0);
            }
        nv[u] = xq + (sb[l] - Lx) / dg;
    }
#pragma unroll
    for (int u = 0; u < K; ++u)
        if (ok[u]) s[L[u]] = nv[u];
}

template <int SW, int NSW, int H, typename R, class CF>
__device__ inline void mac_sweeps(const GridD& g, R* s, R ih2, int ox, int oy)
{
    if constexpr (SW < NSW) {
        constexpr int R0 = H - 1 - 2 * SW;
        mac_half<0, R0, H, R, CF>(g, s, ih2, ox, oy);
        __syncthreads();
        mac_half<1, R0 - 1, H, R, CF>(g, s, ih2, ox, oy);
        __syncthreads();
        mac_sweeps<SW + 1, NSW, H, R, CF>(g, s, ih2, ox, oy);
    }
}

// RES: the launch ends a pre-smoothing and also restricts the residual to
// the coarse level (coarse b = mean of the children's b - L x, coarse x = 0,
// as the residual-restriction kernel); the sweeps run one ring wider (halo
// 2 NSW + 1) so the values the residual reads are final.
template <typename R, class CF, int NSW, bool PRO, bool RES>
__global__ void __launch_bounds__(CF::THREADS)
k_mac_sweepN(BV v, const R* __restrict__ cura, R* __restrict__ nexta, const R* __restrict__ ba,
             const R* __restrict__ pea, const GridD* __restrict__ gct, const long* __restrict__ oct,
             R* __restrict__ bca, R* __restrict__ xca)
{
    static_assert(!(PRO && RES), "a launch either starts a post-smoothing or ends a pre-smoothing");
    constexpr int H = 2 * NSW + (RES ? 1 : 0);
    using T = Tile<2, H, CF>;
    constexpr int TH = CF::THREADS;
    TILE_ENTER(2, T);
    const R* cur = cura + cell0;
    R* next = nexta + cell0;
    const R* b = ba + cell0;
    R* s = reinterpret_cast<R*>(tile_lds);
    GridD gc = g;
    const R* pe = nullptr;
    if (PRO || RES) gc = bv_g2(v, gct, cav);
    if (PRO) pe = pea + bv_o2(v, oct, cav);
    {
        constexpr int K = (T::NS + TH - 1) / TH;
        const bool inner = ox - H >= 0 && ox + T::TX + H <= g.n[0] && oy - H >= 0 && oy + T::TY + H <= g.n[1];
        R vx[K], vb[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int t = threadIdx.x + u * TH;
            const int tt = t < T::NS ? t : 0;
            const int i = ox - H + tt % T::SX, j = oy - H + tt / T::SX;
            bool ok = true, ng = false;
            int src[3] = {i, j, 0};
            const long idx = inner ? cid(g, i, j, 0) : tile_src<2>(g, i, j, 0, ok, ng, src);
            R x = cur[idx];
            if (PRO) x = x + prolong_at<R>(gc, pe, src[0], src[1], R(1));
            vx[u] = ok ? (ng ? -x : x) : R(0);
            vb[u] = b[idx];
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int t = threadIdx.x + u * TH;
            if (t < T::NS) {
                s[t] = vx[u];
                s[T::NS + t] = vb[u];
            }
        }
    }
    const R h = (R)g.h;
    const R ih2 = R(1) / (h * h);
    __syncthreads();
    mac_sweeps<0, NSW, H, R, CF>(g, s, ih2, ox, oy);
    for (int t = threadIdx.x; t < T::TX * T::TY; t += TH) {
        const int rx = t % T::TX, ry = t / T::TX;
        if (ox + rx >= g.n[0] || oy + ry >= g.n[1]) continue;
        next[cid(g, ox + rx, oy + ry, 0)] = s[T::at(rx + H, ry + H, 0)];
    }
    if constexpr (RES) {
        R* bcoarse = bca + bv_o2(v, oct, cav);
        R* xcoarse = xca + bv_o2(v, oct, cav);
        const R* sb = s + T::NS;
        const int off[2] = {1, T::SX};
        constexpr int CX = T::TX / 2, CY = T::TY / 2;
        for (int t = threadIdx.x; t < CX * CY; t += TH) {
            const int cx = t % CX, cy = t / CX;
            const int C[2] = {ox / 2 + cx, oy / 2 + cy};
            if (C[0] >= gc.n[0] || C[1] >= gc.n[1]) continue;
            R sum = 0;
#pragma unroll
            for (int bits = 0; bits < 4; ++bits) {
                const int fx = 2 * cx + (bits & 1), fy = 2 * cy + ((bits >> 1) & 1);
                const int G[2] = {ox + fx, oy + fy};
                const int l = T::at(fx + H, fy + H, 0);
                const R xc = s[l];
                R lap = 0;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const bool okl = g.per[a] || G[a] > 0, okh = g.per[a] || G[a] + 1 < g.n[a];
                    const R Fhi = okh ? s[l + off[a]] - xc : R(0);
                    const R Flo = okl ? xc - s[l - off[a]] : R(0);
                    lap += Fhi - Flo;
                }
                sum += sb[l] - lap * ih2;
            }
            const long qc = cid(gc, C[0], C[1], 0);
            bcoarse[qc] = sum / R(4);
            xcoarse[qc] = R(0);
        }
    }
}

using MacSweepTile = TileShape<32, 16, 1, 1024>;

// ---------------------------------------------------------------------------
// residual / operator application (FP64, halo 1) and residual + restriction
// ---------------------------------------------------------------------------

template <int DIM>
__global__ void __launch_bounds__(TileCfg<DIM>::THREADS)
k_tresid(BV v, const double* __restrict__ coefa, const double* __restrict__ scb, const double* __restrict__ xa,
         const double* __restrict__ ba, double* __restrict__ outa, unsigned long long* __restrict__ mp, int slot)
{
    using T = Tile<DIM, 1>;
    __shared__ unsigned long long red[16];
    TILE_ENTER(DIM, T);
    const double dt = vload(scb + (long)cav * S_NSLOT + S_DT);
    const double* coef = coefa + cell0;
    const double* x = xa + DIM * cell0;
    const double* b = ba ? ba + DIM * cell0 : nullptr;
    double* out = outa ? outa + DIM * cell0 : nullptr;
    double* s = reinterpret_cast<double*>(tile_lds);
    double* e = s + DIM * T::NS;
    const long N = ncells(g);
    constexpr int NT = T::TX * T::TY * T::TZ, TH = TileCfg<DIM>::THREADS, KT = (NT + TH - 1) / TH;
    // this thread's cells and, for the residual, their right-hand sides
    // (loaded with the tile fill)
    int tG[KT][3];
    bool tOk[KT];
    long tq[KT];
    double tb[KT][DIM];
#pragma unroll
    for (int u = 0; u < KT; ++u) {
        const int t = threadIdx.x + u * TH;
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        tG[u][0] = ox + rx;
        tG[u][1] = oy + ry;
        tG[u][2] = DIM == 3 ? oz + rz : 0;
        tOk[u] = t < NT && tG[u][0] < g.n[0] && tG[u][1] < g.n[1] && tG[u][2] < g.n[2];
        tq[u] = cid_clamped(g, tG[u]);
        if (b)
#pragma unroll
            for (int c = 0; c < DIM; ++c) tb[u][c] = b[c * N + tq[u]];
    }
    {
        const double* q[DIM + 1];
        bool mir[DIM + 1];
        for (int a = 0; a < DIM; ++a) { q[a] = x + a * N; mir[a] = false; }
        q[DIM] = coef;
        mir[DIM] = true;
        fill_batched<DIM, 1, DIM + 1, double>(g, q, mir, s, ox, oy, oz);
    }
    __syncthreads();
    unsigned long long m = 0ull;
#pragma unroll
    for (int u = 0; u < KT; ++u) {
        if (!tOk[u]) continue;
        const int t = threadIdx.x + u * TH;
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        const int* G = tG[u];
        const int l = T::at(rx + 1, ry + 1, DIM == 3 ? rz + 1 : 0);
        const int wm = wall_mask<DIM>(g, G);
        const long q0 = tq[u];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double vd = tile_visc_div<DIM, 1, true, double>(g, nullptr, s, e, c, G, wm, l, dt, nullptr);
            const double Ax = s[c * T::NS + l] - dt * vd;
            if (b) {
                const double rv = tb[u][c] - Ax;
                if (out) out[c * N + q0] = rv;
                const unsigned long long bv = abits(rv);
                m = bv > m ? bv : m;
            } else {
                out[c * N + q0] = Ax;
            }
        }
    }
    if (slot >= 0) {
        m = block_umax(m, red);
        if (threadIdx.x == 0) max_partial(mp, cav, ((long)bz * gridDim.y + tby) * gridDim.x + tbx, m);
    }
}

template <int DIM, bool FINE, typename R>
__global__ void __launch_bounds__(TileCfg<DIM>::THREADS)
k_tresid_restr(BV v, const GridD* __restrict__ gct, const long* __restrict__ oct, const R* __restrict__ coefa,
               const double* __restrict__ scb, const R* __restrict__ xa, const R* __restrict__ ba,
               R* __restrict__ bcoarsea, R* __restrict__ xcoarsea)
{
    using T = Tile<DIM, 1>;
    TILE_ENTER(DIM, T);
    const R dt = (R)vload(scb + (long)cav * S_NSLOT + S_DT);
    const GridD gc = bv_g2(v, gct, cav);
    const R* coef = FINE ? coefa + cell0 : coefa + bv_of(v, cav);
    const R* x = xa + DIM * cell0;
    const R* b = ba + DIM * cell0;
    R* bcoarse = bcoarsea + DIM * bv_o2(v, oct, cav);
    R* xcoarse = xcoarsea + DIM * bv_o2(v, oct, cav);
    R* s = reinterpret_cast<R*>(tile_lds);
    R* e = s + DIM * T::NS;
    R* r = e + T::NS;   // residual of the tile, [c][tile cell]
    constexpr int NT = T::TX * T::TY * T::TZ, TH = TileCfg<DIM>::THREADS, KT = (NT + TH - 1) / TH;
    constexpr int NF = FINE ? 1 : 2 * DIM;
    const long N = ncells(g), Nc = ncells(gc);
    // this thread's cells, their right-hand sides and (coarse levels) face
    // viscosities, loaded with the tile fill
    int tG[KT][3];
    bool tOk[KT];
    R tb[KT][DIM], tF[KT][NF];
#pragma unroll
    for (int u = 0; u < KT; ++u) {
        const int t = threadIdx.x + u * TH;
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        tG[u][0] = ox + rx;
        tG[u][1] = oy + ry;
        tG[u][2] = DIM == 3 ? oz + rz : 0;
        tOk[u] = t < NT && tG[u][0] < g.n[0] && tG[u][1] < g.n[1] && tG[u][2] < g.n[2];
        const long q0 = cid_clamped(g, tG[u]);
#pragma unroll
        for (int c = 0; c < DIM; ++c) tb[u][c] = b[c * N + q0];
        if (!FINE) load_faces<DIM, R>(g, coef, tG[u], tF[u]);
    }
    {
        const R* q[DIM + 1];
        bool mir[DIM + 1];
        for (int a = 0; a < DIM; ++a) { q[a] = x + a * N; mir[a] = false; }
        q[DIM] = coef;
        mir[DIM] = true;
        fill_batched<DIM, 1, DIM + (FINE ? 1 : 0), R>(g, q, mir, s, ox, oy, oz);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < KT; ++u) {
        if (!tOk[u]) continue;
        const int t = threadIdx.x + u * TH;
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        const int* G = tG[u];
        const int l = T::at(rx + 1, ry + 1, DIM == 3 ? rz + 1 : 0);
        const int wm = wall_mask<DIM>(g, G);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const R vd = tile_visc_div<DIM, 1, FINE, R>(g, tF[u], s, e, c, G, wm, l, dt, nullptr);
            const R Ax = s[c * T::NS + l] - dt * vd;
            r[c * NT + t] = tb[u][c] - Ax;
        }
    }
    __syncthreads();
    constexpr int CX = T::TX / 2, CY = T::TY / 2, CZ = DIM == 3 ? T::TZ / 2 : 1;
    constexpr int nch = 1 << DIM;
    for (int t = threadIdx.x; t < CX * CY * CZ; t += blockDim.x) {
        const int cx = t % CX, cy = (t / CX) % CY, cz = t / (CX * CY);
        const int C[3] = {ox / 2 + cx, oy / 2 + cy, DIM == 3 ? oz / 2 + cz : 0};
        if (C[0] >= gc.n[0] || C[1] >= gc.n[1] || C[2] >= gc.n[2]) continue;
        const long qc = cid(gc, C[0], C[1], C[2]);
        for (int c = 0; c < DIM; ++c) {
            R sum = 0;
            for (int bits = 0; bits < nch; ++bits) {
                const int fx = 2 * cx + (bits & 1), fy = 2 * cy + ((bits >> 1) & 1), fz = DIM == 3 ? 2 * cz + ((bits >> 2) & 1) : 0;
                sum += r[c * NT + (fz * T::TY + fy) * T::TX + fx];
            }
            bcoarse[c * Nc + qc] = sum / R(nch);
            xcoarse[c * Nc + qc] = R(0);
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: one colour of one component per launch, updated in place.  The cells
// of one colour read only the other colour of component c and the other
// components, none of which change in the launch, so blocks can update their
// tiles in place without a second buffer; the tile needs a 1-cell halo only.
// In 3D this needs fewer operator evaluations and less LDS than the fused
// two-colour sweep (whose 2-cell halo is large relative to a 3D tile).
// ---------------------------------------------------------------------------

template <bool FINE, typename R, class CF = Trb3Tile>
__global__ void __launch_bounds__(CF::THREADS)
k_trb3(BV v, const R* __restrict__ coefa, const double* __restrict__ scb, int c, int colour, R* xa,
       const R* __restrict__ ba)
{
    using T = Tile<3, 1, CF>;
    static_assert(T::TX * T::TY * T::TZ / 2 == CF::THREADS, "one cell of the colour per thread");
    TILE_ENTER(3, T);
    const R dt = (R)vload(scb + (long)cav * S_NSLOT + S_DT);
    const R* coef = FINE ? coefa + cell0 : coefa + bv_of(v, cav);
    R* x = xa + 3 * cell0;
    const R* b = ba + 3 * cell0;
    R* s = reinterpret_cast<R*>(tile_lds);
    R* e = s + 3 * T::NS;
    const long N = ncells(g);
    // this thread's cell of the colour and its right-hand side
    const int t = threadIdx.x;
    const int px = t % (T::TX / 2), ry = (t / (T::TX / 2)) % T::TY, rz = t / (T::TX / 2 * T::TY);
    const int G[3] = {ox + 2 * px + ((ox + oy + ry + oz + rz + colour) & 1), oy + ry, oz + rz};
    const bool ok = G[0] < g.n[0] && G[1] < g.n[1] && G[2] < g.n[2];
    const long q0 = cid_clamped(g, G);
    const R bv = b[c * N + q0];
    constexpr int NF = FINE ? 1 : 6;
    R bf[NF];
    if (!FINE) load_faces<3, R>(g, coef, G, bf);
    {
        const R* q[4] = {x, x + N, x + 2 * N, coef};
        const bool mir[4] = {false, false, false, true};
        fill_tile1<FINE, R, CF>(g, q, mir, s, ox, oy, oz);
    }
    __syncthreads();
    if (!ok) return;
    const int l = T::at(G[0] - ox + 1, ry + 1, rz + 1);
    R dg;
    const R vd = tile_visc_div<3, 1, FINE, R, CF>(g, bf, s, e, c, G, wall_mask<3>(g, G), l, dt, &dg);
    const R xc = s[c * T::NS + l];
    const R Au = xc - dt * vd;
    x[c * N + q0] = xc + (bv - Au) / dg;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// tile grid over the largest cavity of the level, z-tiles times cavities
template <int DIM, class CF = TileCfg<DIM>>
static dim3 tile_grid(const Ctx* c, const Level& L, BV& v)
{
    using T = Tile<DIM, 1, CF>;
    const GridD& g = L.gmax;
    v.zb = DIM == 3 ? (g.n[2] + T::TZ - 1) / T::TZ : 1;
    return dim3((g.n[0] + T::TX - 1) / T::TX, (g.n[1] + T::TY - 1) / T::TY, v.zb * c->nb);
}

static double level_cells(const Level& L)
{
    double n = 0.0;
    for (const GridD& g : L.hg)
        if (g.dim) n += (double)ncells(g);
    return n;
}

static double level_faces(const Level& L)
{
    double n = 0.0;
    for (const GridD& g : L.hg)
        if (g.dim)
            for (int a = 0; a < g.dim; ++a) n += (double)fcount(g, a);
    return n;
}

// Launch kernel k on the context's stream.  With the kernel timer on, the
// launch goes through hipExtLaunchKernelGGL with the timer's next event
// pair, which the runtime records at the kernel's own start and end (so the
// timing does not include the cost of separate event commands); bytes is the
// launch's algorithmic traffic.
template <typename K, typename... A>
static void tlaunch(Ctx* c, bool timed, double bytes, K k, dim3 grid, dim3 block, size_t lds, A... args)
{
    if (timed) {
        hipEvent_t e0, e1;
        kt_pair(c, &e0, &e1, bytes);
        hipExtLaunchKernelGGL(k, grid, block, (std::uint32_t)lds, c->s, e0, e1, 0u, args...);
    } else {
        k<<<grid, block, lds, c->s>>>(args...);
    }
}

template <int DIM, bool FINE, typename R, class CF = TileCfg<DIM>>
static void tsmooth_impl(Ctx* c, const Level& L, BV v, const R* coef, int comp, const R* xcur, R* xnext, const R* b,
                         bool timed, double bytes)
{
    const size_t lds = sizeof(R) * (DIM + (FINE ? 1 : 0)) * Tile<DIM, 2, CF>::NS;
    const dim3 grid = tile_grid<DIM, CF>(c, L, v);
    constexpr int TH = CF::THREADS;
    const R* xin = xnext;
    if (comp == 0)
        tlaunch(c, timed, bytes, k_tsmooth<DIM, FINE, 0, R, CF>, grid, dim3(TH), lds, v, coef, (const double*)c->sc,
                xcur, xin, xnext, b);
    else if (comp == 1)
        tlaunch(c, timed, bytes, k_tsmooth<DIM, FINE, 1, R, CF>, grid, dim3(TH), lds, v, coef, (const double*)c->sc,
                xcur, xin, xnext, b);
    else
        tlaunch(c, timed, bytes, k_tsmooth<DIM, FINE, (DIM == 3 ? 2 : 1), R, CF>, grid, dim3(TH), lds, v, coef,
                (const double*)c->sc, xcur, xin, xnext, b);
}

template <typename R>
void launch_tsmooth(Ctx* c, const Level& L, const BV& v, const R* coef, bool fine, int comp, const R* xcur, R* xnext,
                    const R* b)
{
    const bool timed = fine && kt_take(c);
    // algorithmic bytes counted per red-black sweep of all components (every
    // component of x, the coefficients and every component of b read once,
    // x written once); a launch sweeps one component, 1/dim of a sweep
    const double N = level_cells(L);
    const double coefw = fine ? N : level_faces(L);
    const double dim = L.gmax.dim;
    const double bytes = sizeof(R) * (3.0 * dim * N + coefw) / dim;
    if (L.gmax.dim == 2) {
        if (fine) tsmooth_impl<2, true, R>(c, L, v, coef, comp, xcur, xnext, b, timed, bytes);
        else tsmooth_impl<2, false, R>(c, L, v, coef, comp, xcur, xnext, b, timed, bytes);
    } else if (fine) {
        tsmooth_impl<3, true, R>(c, L, v, coef, comp, xcur, xnext, b, timed, bytes);
    } else {
        tsmooth_impl<3, false, R, Tsm3Tile>(c, L, v, coef, comp, xcur, xnext, b, timed, bytes);
    }
}

// the 3D coarse-level tile stages more than the default 64 KB of LDS in FP64
void tsmooth_allow_lds(size_t bytes)
{
    auto allow = [&](const void* k) {
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    };
    allow(reinterpret_cast<const void*>(&k_tsmooth<3, false, 0, double, Tsm3Tile>));
    allow(reinterpret_cast<const void*>(&k_tsmooth<3, false, 1, double, Tsm3Tile>));
    allow(reinterpret_cast<const void*>(&k_tsmooth<3, false, 2, double, Tsm3Tile>));
    allow(reinterpret_cast<const void*>(&k_tsmooth<3, false, 0, float, Tsm3Tile>));
    allow(reinterpret_cast<const void*>(&k_tsmooth<3, false, 1, float, Tsm3Tile>));
    allow(reinterpret_cast<const void*>(&k_tsmooth<3, false, 2, float, Tsm3Tile>));
}

template <int DIM>
static void tresid_impl(Ctx* c, const Level& L, BV v, const double* coef, const double* x, const double* b, double* out,
                        int slot)
{
    const size_t lds = sizeof(double) * (DIM + 1) * Tile<DIM, 1>::NS;
    const dim3 grid = tile_grid<DIM>(c, L, v);
    k_tresid<DIM><<<grid, TileCfg<DIM>::THREADS, lds, c->s>>>(v, coef, c->sc, x, b, out, c->mpart, slot);
    if (slot >= 0) launch_max_final(c, v.act, slot);
}

void launch_tresid(Ctx* c, const Level& L, const BV& v, const double* coef, const double* x, const double* b, double* out,
                   int slot)
{
    if (L.gmax.dim == 2) tresid_impl<2>(c, L, v, coef, x, b, out, slot);
    else tresid_impl<3>(c, L, v, coef, x, b, out, slot);
}

template <int DIM, bool FINE, typename R>
static void tresid_restr_impl(Ctx* c, const Level& L, BV v, const GridD* gc, const long* oc, const R* coef, const R* x,
                              const R* b, R* bc, R* xc)
{
    using T = Tile<DIM, 1>;
    const size_t lds = sizeof(R) * (DIM * (T::NS + T::TX * T::TY * T::TZ) + T::NS);
    const dim3 grid = tile_grid<DIM>(c, L, v);
    k_tresid_restr<DIM, FINE, R><<<grid, TileCfg<DIM>::THREADS, lds, c->s>>>(v, gc, oc, coef, c->sc, x, b, bc, xc);
}

template <typename R>
void launch_tresid_restr(Ctx* c, const Level& L, const BV& v, const GridD* gc, const long* oc, const R* coef, bool fine,
                         const R* x, const R* b, R* bc, R* xc)
{
    if (L.gmax.dim == 2) {
        if (fine) tresid_restr_impl<2, true, R>(c, L, v, gc, oc, coef, x, b, bc, xc);
        else tresid_restr_impl<2, false, R>(c, L, v, gc, oc, coef, x, b, bc, xc);
    } else {
        if (fine) tresid_restr_impl<3, true, R>(c, L, v, gc, oc, coef, x, b, bc, xc);
        else tresid_restr_impl<3, false, R>(c, L, v, gc, oc, coef, x, b, bc, xc);
    }
}

// dynamic LDS of a staged launch (PRO: with the coarse patch)
template <bool FINE, typename R, class CF, int NSW, bool RES, bool PRO = false>
constexpr size_t staged_lds()
{
    return sizeof(R) * ((FINE ? 5 : 6) * Tile<2, 4 * NSW + (RES ? 1 : 0), CF>::NS + (RES ? 2 * CF::TX * CF::TY : 0) +
                        (PRO ? 2 * CoarsePatch<4 * NSW, CF>::PN : 0));
}

// the largest of a candidate's launches (coarse level, FP64)
template <class CF, int NSW>
constexpr size_t staged_lds_max()
{
    const size_t r = staged_lds<false, double, CF, NSW, true>(), p = staged_lds<false, double, CF, NSW, false, true>();
    return r > p ? r : p;
}

template <bool FINE, bool PRO, bool RES, typename R, class CF, int NSW>
static void staged_launch(Ctx* c, bool timed, double bytes, dim3 grid, const BV& vv, const R* coef, const R* xcur,
                          R* xnext, const R* b, const R* pe, const GridD* gct, const long* oct, R* bc, R* xc)
{
    tlaunch(c, timed, bytes, k_tsweepN<FINE, R, CF, NSW, PRO, RES>, grid, dim3(CF::THREADS),
            staged_lds<FINE, R, CF, NSW, RES, PRO>(), vv, coef, (const double*)c->sc, xcur, xnext, b, pe, gct, oct, bc, xc);
}

template <bool FINE, typename R, class CAND>
static void tsweep2_impl(Ctx* c, const Level& L, const BV& v, const R* coef, const R* xcur, R* xnext, const R* b,
                         int nsw, const R* pe, const GridD* gct, const long* oct, R* bc, R* xc)
{
    using CF = typename CAND::CF;
    const bool timed = FINE && kt_take(c);
    BV vv = v;
    const dim3 grid = tile_grid<2, CF>(c, L, vv);
    // algorithmic bytes of a launch, counted per red-black sweep of both
    // components (both components of x, eta/Re and both components of b
    // read once, x written once: 7 words per cell) times the sweeps the
    // launch runs; with a folded prolongation also both components of the
    // coarse iterate read, with a folded restriction both components of the
    // coarse right-hand side and iterate written (N/4 cells each)
    const double N = level_cells(L);
    const int sweeps = (CAND::STAGED && CAND::NSW >= 2 && nsw == 2) ? 2 : 1;
    // (a launch that starts from zeros does not read x: 2 words fewer)
    const double bytes = sizeof(R) * (7.0 * N * sweeps - (xcur ? 0.0 : 2.0 * N) + (pe ? 2.0 * N / 4.0 : 0.0) +
                                      (bc ? 4.0 * N / 4.0 : 0.0));
    if constexpr (!CAND::STAGED) {
        using T = Tile<2, 4, CF>;
        const size_t lds = sizeof(R) * (FINE ? 3 : 2) * T::NS;
        if (pe) launch_prolong_cells<R>(c, L, v, gct, oct, 2, -1.0, pe, const_cast<R*>(xcur));
        tlaunch(c, timed, bytes, k_tsweep2<FINE, R, CF>, grid, dim3(CF::THREADS), lds, vv, coef, (const double*)c->sc,
                xcur, xnext, b);
        if (bc) launch_tresid_restr<R>(c, L, v, gct, oct, coef, FINE, xnext, b, bc, xc);
    } else if (CAND::NSW >= 2 && nsw == 2) {
        if (pe) staged_launch<FINE, true, false, R, CF, 2>(c, timed, bytes, grid, vv, coef, xcur, xnext, b, pe, gct, oct, bc, xc);
        else if (bc) staged_launch<FINE, false, true, R, CF, 2>(c, timed, bytes, grid, vv, coef, xcur, xnext, b, pe, gct, oct, bc, xc);
        else staged_launch<FINE, false, false, R, CF, 2>(c, timed, bytes, grid, vv, coef, xcur, xnext, b, pe, gct, oct, bc, xc);
    } else {
        if (pe) staged_launch<FINE, true, false, R, CF, 1>(c, timed, bytes, grid, vv, coef, xcur, xnext, b, pe, gct, oct, bc, xc);
        else if (bc) staged_launch<FINE, false, true, R, CF, 1>(c, timed, bytes, grid, vv, coef, xcur, xnext, b, pe, gct, oct, bc, xc);
        else staged_launch<FINE, false, false, R, CF, 1>(c, timed, bytes, grid, vv, coef, xcur, xnext, b, pe, gct, oct, bc, xc);
    }
}

template <bool FINE, typename R, size_t... I>
static void tsweep2_pick(Ctx* c, const Level& L, const BV& v, const R* coef, const R* xcur, R* xnext, const R* b,
                         int k, int nsw, const R* pe, const GridD* gct, const long* oct, R* bc, R* xc,
                         std::index_sequence<I...>)
{
    ((k == (int)I ? tsweep2_impl<FINE, R, std::tuple_element_t<I, Sweep2Cands>>(c, L, v, coef, xcur, xnext, b, nsw, pe,
                                                                                gct, oct, bc, xc)
                  : void()),
     ...);
}

template <typename R>
void launch_tsweep2(Ctx* c, const Level& L, const BV& v, const R* coef, bool fine, const R* xcur, R* xnext, const R* b,
                    int tile, int nsw, const R* pe, const GridD* gct, const long* oct, R* bc, R* xc)
{
    const int k = tile >= 0 && tile < kSweep2Cands ? tile : 0;
    constexpr auto seq = std::make_index_sequence<kSweep2Cands>{};
    if (fine) tsweep2_pick<true, R>(c, L, v, coef, xcur, xnext, b, k, nsw, pe, gct, oct, bc, xc, seq);
    else tsweep2_pick<false, R>(c, L, v, coef, xcur, xnext, b, k, nsw, pe, gct, oct, bc, xc, seq);
}

template <size_t... I>
static SweepShape sweep2_shape_of(int k, std::index_sequence<I...>)
{
    SweepShape out{};
    ((k == (int)I ? (void)(out = SweepShape{std::tuple_element_t<I, Sweep2Cands>::CF::TX,
                                            std::tuple_element_t<I, Sweep2Cands>::CF::TY,
                                            std::tuple_element_t<I, Sweep2Cands>::CF::THREADS,
                                            std::tuple_element_t<I, Sweep2Cands>::NSW,
                                            std::tuple_element_t<I, Sweep2Cands>::STAGED})
                  : void()),
     ...);
    return out;
}

SweepShape sweep2_shape(int k) { return sweep2_shape_of(k, std::make_index_sequence<kSweep2Cands>{}); }

// the staged sweeps may use more dynamic LDS than the default limit
template <class CF, typename R, int NSW>
static void allow_one(size_t bytes)
{
    const void* k[6] = {reinterpret_cast<const void*>(&k_tsweepN<true, R, CF, NSW, false, false>),
                        reinterpret_cast<const void*>(&k_tsweepN<false, R, CF, NSW, false, false>),
                        reinterpret_cast<const void*>(&k_tsweepN<true, R, CF, NSW, true, false>),
                        reinterpret_cast<const void*>(&k_tsweepN<false, R, CF, NSW, true, false>),
                        reinterpret_cast<const void*>(&k_tsweepN<true, R, CF, NSW, false, true>),
                        reinterpret_cast<const void*>(&k_tsweepN<false, R, CF, NSW, false, true>)};
    for (const void* f : k) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <class CAND, typename R>
static void allow_staged(size_t bytes)
{
    if constexpr (CAND::STAGED) {
        using CF = typename CAND::CF;
        allow_one<CF, R, 1>(bytes);
        if constexpr (CAND::NSW >= 2) allow_one<CF, R, 2>(bytes);
    }
}

template <size_t... I>
static void allow_all(size_t bytes, std::index_sequence<I...>)
{
    (allow_staged<std::tuple_element_t<I, Sweep2Cands>, double>(bytes), ...);
    (allow_staged<std::tuple_element_t<I, Sweep2Cands>, float>(bytes), ...);
}

void sweep2_allow_lds(size_t bytes) { allow_all(bytes, std::make_index_sequence<kSweep2Cands>{}); }

// dynamic LDS bytes of candidate k running nsw sweeps per launch (FP64,
// coarse level: the larger of the launches with the residual epilogue and
// with the coarse patch)
template <size_t... I>
static size_t sweep2_lds_of(int k, int nsw, std::index_sequence<I...>)
{
    size_t out = 0;
    ((k == (int)I ? (void)(out = std::tuple_element_t<I, Sweep2Cands>::STAGED
                                     ? (nsw == 2 ? staged_lds_max<typename std::tuple_element_t<I, Sweep2Cands>::CF, 2>()
                                                 : staged_lds_max<typename std::tuple_element_t<I, Sweep2Cands>::CF, 1>())
                                     : sizeof(double) * 3 *
                                           Tile<2, 4, typename std::tuple_element_t<I, Sweep2Cands>::CF>::NS)
                  : void()),
     ...);
    return out;
}

size_t sweep2_lds(int k, int nsw) { return sweep2_lds_of(k, nsw, std::make_index_sequence<kSweep2Cands>{}); }

template <typename R>
void launch_trb3(Ctx* c, const Level& L, const BV& v, const R* coef, bool fine, int comp, int colour, R* x, const R* b)
{
    using CF = Trb3Tile;
    using T = Tile<3, 1, CF>;
    const bool timed = fine && kt_take(c);
    const size_t lds = sizeof(R) * (3 + (fine ? 1 : 0)) * T::NS;
    BV vv = v;
    const dim3 grid = tile_grid<3, CF>(c, L, vv);
    // algorithmic bytes counted per red-black sweep of all three components
    // (every component of x, eta/Re and every component of b read once, x
    // written once: 10 words per cell); a launch runs one colour of one
    // component, a sixth of a sweep
    const double N = level_cells(L);
    const double bytes = sizeof(R) * 10.0 * N / 6.0;
    const dim3 blk(CF::THREADS);
    if (fine) tlaunch(c, timed, bytes, k_trb3<true, R, CF>, grid, blk, lds, vv, coef, (const double*)c->sc, comp, colour, x, b);
    else tlaunch(c, timed, bytes, k_trb3<false, R, CF>, grid, blk, lds, vv, coef, (const double*)c->sc, comp, colour, x, b);
}


template <typename R>
void launch_mac_sweep(Ctx* c, const Level& L, const BV& v, const R* cur, R* next, const R* b, int nsw, const R* pe,
                      const GridD* gct, const long* oct, R* bc, R* xc)
{
    BV vv = v;
    if (L.gmax.dim == 2) {
        // staged: nsw sweeps per launch, the prolongation folded in with pe,
        // the residual restriction with bc
        using CF = MacSweepTile;
        const dim3 grid = tile_grid<2, CF>(c, L, vv);
        auto go = [&](auto kern, int halo) {
            kern<<<grid, CF::THREADS, sizeof(R) * 2 * (CF::TX + 2 * halo) * (CF::TY + 2 * halo), c->s>>>(
                vv, cur, next, b, pe, gct, oct, bc, xc);
        };
        if (nsw == 2) {
            if (pe) go(k_mac_sweepN<R, CF, 2, true, false>, 4);
            else if (bc) go(k_mac_sweepN<R, CF, 2, false, true>, 5);
            else go(k_mac_sweepN<R, CF, 2, false, false>, 4);
        } else {
            if (pe) go(k_mac_sweepN<R, CF, 1, true, false>, 2);
            else if (bc) go(k_mac_sweepN<R, CF, 1, false, true>, 3);
            else go(k_mac_sweepN<R, CF, 1, false, false>, 2);
        }
        return;
    }
    if (pe) launch_prolong_cells<R>(c, L, v, gct, oct, 1, 1.0, pe, const_cast<R*>(cur));
    if (L.gmax.dim == 2) {
        const dim3 grid = tile_grid<2>(c, L, vv);
        k_mac_sweep<2, R><<<grid, TileCfg<2>::THREADS, sizeof(R) * Tile<2, 2>::NS, c->s>>>(vv, cur, next, b);
    } else {
        // 3D: a 32x8x8 tile with 1024 threads stages 2.5 positions per cell
        // (halo 2) where the 32x4x4 default tile stages 4.5
        using CF = Mac3Tile;
        const dim3 grid = tile_grid<3, CF>(c, L, vv);
        k_mac_sweep<3, R, CF><<<grid, CF::THREADS, sizeof(R) * Tile<3, 2, CF>::NS, c->s>>>(vv, cur, next, b);
    }
}

#define HB_TILE_INST(R)                                                                                             \
    template void launch_tsmooth<R>(Ctx*, const Level&, const BV&, const R*, bool, int, const R*, R*, const R*);     \
    template void launch_trb3<R>(Ctx*, const Level&, const BV&, const R*, bool, int, int, R*, const R*);             \
    template void launch_tsweep2<R>(Ctx*, const Level&, const BV&, const R*, bool, const R*, R*, const R*, int, int, \
                                     const R*, const GridD*, const long*, R*, R*);  \
    template void launch_mac_sweep<R>(Ctx*, const Level&, const BV&, const R*, R*, const R*, int, const R*,         \
                                      const GridD*, const long*, R*, R*);                                           \
    template void launch_tresid_restr<R>(Ctx*, const Level&, const BV&, const GridD*, const long*, const R*, bool, \
                                         const R*, const R*, R*, R*);
HB_TILE_INST(double)
HB_TILE_INST(float)
#undef HB_TILE_INST

}  // namespace hb
