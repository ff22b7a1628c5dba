// hb_nodal.hip -- LDS-tiled kernels of the nodal projection problem K x = b
// (Q1 stiffness, natural boundary on walls): multi-colour Gauss-Seidel and
// residual.  gfx950; templated on the storage and arithmetic type R (double,
// or float in the mixed-precision correction cycles).
//
// The assembled stencil is written per node from the element stiffness: the
// weight of neighbour node+delta is Ke(|delta|_0) times the number of
// existing elements that contain both nodes, which factors per axis into
// cnt_a(delta_a) (2 or 1 in the interior and on periodic axes, fewer on a
// wall).  Ke by the number of differing coordinates: 2D {2/3, -1/6, -1/3},
// 3D h {1/3, 0, -1/12, -1/12}.
#include "hb_internal.h"
#include "hb_ops.h"

#include <tuple>
#include <utility>

namespace hb {

template <int DIM> struct NodalCfg;
// threads per block (one per node of the active colour); node tile = 2x that
template <> struct NodalCfg<2> { static constexpr int BX = 64, BY = 4, BZ = 1; };
template <> struct NodalCfg<3> { static constexpr int BX = 32, BY = 4, BZ = 2; };

template <int DIM>
struct NTile {
    static constexpr int TX = 2 * NodalCfg<DIM>::BX, TY = 2 * NodalCfg<DIM>::BY, TZ = DIM == 3 ? 2 * NodalCfg<DIM>::BZ : 1;
    static constexpr int SX = TX + 2, SY = TY + 2, SZ = DIM == 3 ? TZ + 2 : 1;
    static constexpr int NS = SX * SY * SZ;
    static constexpr int THREADS = NodalCfg<DIM>::BX * NodalCfg<DIM>::BY * NodalCfg<DIM>::BZ;
    __device__ static inline int at(int lx, int ly, int lz) { return (lz * SY + ly) * SX + lx; }
};

// the same on an NTile
template <int DIM, typename R>
__device__ inline R tile_K(const GridD& g, const R* s, const int G[3], int l, R* diag)
{
    using T = NTile<DIM>;
    return block_K<DIM, R>(g, s, T::SX, T::SX * T::SY, G, l, diag);
}

// stage the node tile plus a 1-node halo; all loads of a thread are issued
// before any store so they are in flight together.  Positions beyond a
// wall read as 0 (their stencil weight is zero); periodic axes wrap.  The
// load always uses an in-range index, so no branch separates the loads.
template <int DIM, typename R>
__device__ inline void fill_nodes(const GridD& g, const R* __restrict__ x, R* s, int ox, int oy, int oz)
{
    using T = NTile<DIM>;
    constexpr int K = (T::NS + T::THREADS - 1) / T::THREADS;
    R v[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * T::THREADS;
        const int tt = t < T::NS ? t : 0;
        const int lx = tt % T::SX, ly = (tt / T::SX) % T::SY, lz = tt / (T::SX * T::SY);
        int p[3] = {ox - 1 + lx, oy - 1 + ly, DIM == 3 ? oz - 1 + lz : 0};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int nn = nnode(g, a);
            int q = p[a];
            if (g.per[a]) q = q < 0 ? q + nn : (q >= nn ? q - nn : q);
            if (q < 0 || q >= nn) {
                ok = false;
                q = 0;
            }
            p[a] = q;
        }
        const R val = x[nid(g, p[0], p[1], p[2])];   // every p[a] is in range
        v[u] = ok ? val : R(0);
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int t = threadIdx.x + u * T::THREADS;
        if (t < T::NS) s[t] = v[u];
    }
}

// Batched launches: block z = cavity * zb + z-tile; each block takes its
// cavity's grid and node offset from the level tables and returns when the
// cavity takes no part or the tile lies outside it.
#define NTILE_ENTER(DIM, T)                                                                 \
    int cav, bz, tbx, tby, tbz;                                                             \
    GridD g;                                                                                \
    xcd_tile(tbx, tby, tbz);                                                                \
    if (!bv_enter_at(v, tbz, cav, bz, g)) return;                                           \
    const int ox = tbx * T::TX, oy = tby * T::TY, oz = DIM == 3 ? bz * T::TZ : 0;            \
    if (ox >= nnode(g, 0) || oy >= nnode(g, 1) || oz >= nnode(g, 2)) return;                \
    const long node0 = bv_o(v, cav);

// one colour (i&1) + 2(j&1) + 4(k&1) of the Gauss-Seidel sweep, in place:
// nodes of one colour share no element
template <int DIM, typename R>
__global__ void __launch_bounds__(NTile<DIM>::THREADS)
k_nodal_gs_tile(BV v, int colour, R* __restrict__ xa, const R* __restrict__ ba)
{
    using T = NTile<DIM>;
    __shared__ R s[T::NS];
    NTILE_ENTER(DIM, T);
    R* x = xa + node0;
    const R* b = ba + node0;
    const int tx = threadIdx.x % NodalCfg<DIM>::BX, ty = (threadIdx.x / NodalCfg<DIM>::BX) % NodalCfg<DIM>::BY,
              tz = threadIdx.x / (NodalCfg<DIM>::BX * NodalCfg<DIM>::BY);
    const int G[3] = {ox + 2 * tx + (colour & 1), oy + 2 * ty + ((colour >> 1) & 1),
                      DIM == 3 ? oz + 2 * tz + ((colour >> 2) & 1) : 0};
    const bool ok = G[0] < nnode(g, 0) && G[1] < nnode(g, 1) && G[2] < nnode(g, 2);
    const long q = nid(g, G[0] < nnode(g, 0) ? G[0] : 0, G[1] < nnode(g, 1) ? G[1] : 0, G[2] < nnode(g, 2) ? G[2] : 0);
    const R bq = b[q];   // in flight with the tile fill
    fill_nodes<DIM, R>(g, x, s, ox, oy, oz);
    __syncthreads();
    if (!ok) return;
    const int l = T::at(G[0] - ox + 1, G[1] - oy + 1, DIM == 3 ? G[2] - oz + 1 : 0);
    R dg;
    const R Kx = tile_K<DIM, R>(g, s, G, l, &dg);
    x[q] = s[l] + (bq - Kx) / dg;
}

// r = b - K x (and, FP64, its max-norm into the cavity's slot) or y = K x
template <int DIM, typename R>
__global__ void __launch_bounds__(NTile<DIM>::THREADS)
k_nodal_resid_tile(BV v, const R* __restrict__ xa, const R* __restrict__ ba, R* __restrict__ outa,
                   unsigned long long* __restrict__ mp, int slot)
{
    using T = NTile<DIM>;
    __shared__ R s[T::NS];
    __shared__ unsigned long long red[16];
    NTILE_ENTER(DIM, T);
    const R* x = xa + node0;
    const R* b = ba ? ba + node0 : nullptr;
    R* out = outa ? outa + node0 : nullptr;
    // this thread's nodes and their right-hand sides, loaded with the fill
    constexpr int NT = T::TX * T::TY * T::TZ, KT = NT / T::THREADS;
    static_assert(NT % T::THREADS == 0, "whole node slots per thread");
    bool tOk[KT];
    long tq[KT];
    R tb[KT];
#pragma unroll
    for (int u = 0; u < KT; ++u) {
        const int t = threadIdx.x + u * T::THREADS;
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        const int G[3] = {ox + rx, oy + ry, DIM == 3 ? oz + rz : 0};
        tOk[u] = G[0] < nnode(g, 0) && G[1] < nnode(g, 1) && G[2] < nnode(g, 2);
        tq[u] = nid(g, G[0] < nnode(g, 0) ? G[0] : 0, G[1] < nnode(g, 1) ? G[1] : 0, G[2] < nnode(g, 2) ? G[2] : 0);
        if (b) tb[u] = b[tq[u]];
    }
    fill_nodes<DIM, R>(g, x, s, ox, oy, oz);
    __syncthreads();
    unsigned long long m = 0ull;
#pragma unroll
    for (int u = 0; u < KT; ++u) {
        if (!tOk[u]) continue;
        const int t = threadIdx.x + u * T::THREADS;
        const int rx = t % T::TX, ry = (t / T::TX) % T::TY, rz = t / (T::TX * T::TY);
        const int G[3] = {ox + rx, oy + ry, DIM == 3 ? oz + rz : 0};
        const int l = T::at(rx + 1, ry + 1, DIM == 3 ? rz + 1 : 0);
        const R Kx = tile_K<DIM, R>(g, s, G, l, nullptr);
        const long q = tq[u];
        if (b) {
            const R rv = tb[u] - Kx;
            if (out) out[q] = rv;
            const unsigned long long bv = abits((double)rv);
            m = bv > m ? bv : m;
        } else {
            out[q] = Kx;
        }
    }
    if (slot >= 0) {
        m = block_umax(m, red);
        if (threadIdx.x == 0) max_partial(mp, cav, ((long)bz * gridDim.y + tby) * gridDim.x + tbx, m);
    }
}

// ---------------------------------------------------------------------------
// Fused colour sweep.  The 2^d colours (i&1) + 2(j&1) + 4(k&1) of a sweep run
// in order; the four in-plane colours of the planes of one z parity depend
// only on each other and on the planes of the other parity.  One launch
// therefore runs all four in-plane colours on the planes of one parity (2D:
// the whole sweep; 3D: even planes, then odd planes).  Within the tile's
// planes colour c is updated on the tile grown by the rings its successors
// read (x by 3, 2, 1, 0 and y by 1, 1, 0, 0 for c = 0..3, since colour 1
// neighbours colour 0 along x, colour 2 neighbours it along y and colour 1
// diagonally, colour 3 neighbours all three), so the staged block needs a
// halo of 4 nodes in x and 2 in y.  Blocks read `cur` and write the planes
// they update to `next` (other blocks still read the old values); in 3D the
// odd-parity launch reads the even planes from `next`.  Every node sees the
// same neighbour values as in the one-colour-per-launch order, so the result
// is the same bit for bit.
// ---------------------------------------------------------------------------
// tile of the fused sweep: TX x TY nodes of PZ planes of one parity, TH
// threads; candidates per dimension, chosen per level by the autotuner
// (index 0 is the default)
template <int TX_, int TY_, int PZ_, int TH_>
struct NG4 {
    static constexpr int TX = TX_, TY = TY_, PZ = PZ_, TH = TH_;
};
using NG4Tiles2 = std::tuple<NG4<64, 16, 1, 256>, NG4<128, 8, 1, 256>, NG4<32, 32, 1, 256>, NG4<64, 16, 1, 1024>>;
using NG4Tiles3 = std::tuple<NG4<64, 8, 2, 512>, NG4<32, 16, 2, 512>, NG4<64, 4, 4, 512>, NG4<64, 8, 2, 1024>>;
constexpr int kNG4Tiles = 4;
static_assert(kNG4Tiles == kNodalCands && std::tuple_size_v<NG4Tiles2> == kNG4Tiles &&
                  std::tuple_size_v<NG4Tiles3> == kNG4Tiles,
              "nodal candidate count");

// 2D, NSW = 2: two whole sweeps in one launch.  Colour c of sweep w runs on
// the tile grown by 4 (NSW - 1 - w) + 3 - c in x and 2 (NSW - 1 - w) + (1 for
// c <= 1) in y (the rings above, widened by what the later sweep reads), so
// the halo is 4 NSW by 2 NSW nodes; again every node sees the values of the
// one-colour-per-launch order.
// EXT = 2 (a launch that ends a pre-smoothing and restricts the residual):
// every ring two nodes wider, so x is final two nodes around the tile.
template <int DIM, class CF, int NSW = 1, int EXT = 0>
struct NG4Tile {
    static_assert(DIM == 2 || (NSW == 1 && EXT == 0), "two sweeps and folded transfers in 2D only");
    using C = CF;
    static constexpr int HX = 4 * NSW + EXT, HY = 2 * NSW + EXT;   // halo of x
    static constexpr int SX = C::TX + 2 * HX, SY = C::TY + 2 * HY, SZ = DIM == 3 ? 2 * C::PZ + 1 : 1;
    static constexpr int NS = SX * SY * SZ;
    // b on the first colour's region
    static constexpr int BX = C::TX + 2 * (HX - 1), BY = C::TY + 2 * (HY - 1);
    static constexpr int NB = BX * BY * C::PZ;
};

// Nodal interpolation (P e) at fine node (i, j) from the coarse iterate e
// on grid gc: the mean of the coarse nodes of its coarse edge or cell; same
// terms, order and rounding as the prolongation kernel.
template <typename R>
__device__ inline R nodal_prolong_at(const GridD& gc, const R* __restrict__ e, int i, int j)
{
    const int F[2] = {i, j};
    R s = 0;
#pragma unroll
    for (int bits = 0; bits < 4; ++bits) {
        int p[2] = {0, 0};
        R w = 1;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int hi = (bits >> a) & 1;
            if (!(F[a] & 1)) {
                if (hi) ok = false;
                p[a] = F[a] >> 1;
            } else {
                w *= R(0.5);
                int C = ((F[a] - 1) >> 1) + hi;
                if (gc.per[a] && C == nnode(gc, a)) C = 0;
                p[a] = C;
            }
        }
        const R val = e[nid(gc, p[0], p[1], 0)];
        s = ok ? s + w * val : s;
    }
    return s;
}

// PRO (2D): the fill adds the interpolated coarse correction pe to x (a
// V-cycle's prolongation folded into the first sweep after it).  RES (2D):
// the launch ends a pre-smoothing; it also forms the residual b - K x of
// the tile's nodes and a ring of one below them, and restricts it by full
// weighting to the tile's coarse nodes (coarse b, coarse x = 0), as the
// residual and restriction kernels would after it.
template <int DIM, typename R, class CF, int NSW = 1, bool PRO = false, bool RES = false>
__global__ void __launch_bounds__(CF::TH)
k_nodal_gs_fused(BV v, int zpar, const R* __restrict__ cura, const R* fixa, R* nexta, const R* __restrict__ ba,
                 const R* __restrict__ pea = nullptr, const GridD* __restrict__ gct = nullptr,
                 const long* __restrict__ oct = nullptr, R* __restrict__ bca = nullptr, R* __restrict__ xca = nullptr)
{
    static_assert(!(PRO && RES), "a launch either starts a post-smoothing or ends a pre-smoothing");
    using T = NG4Tile<DIM, CF, NSW, RES ? 2 : 0>;
    constexpr int TH = CF::TH;
    __shared__ R s[T::NS];
    __shared__ R sb[T::NB];
    constexpr int RX = CF::TX + 1, RY = CF::TY + 1;   // residual positions: the tile and a ring below
    __shared__ R rr[RES ? RX * RY : 1];
    int cav, bz, tbx, tby, tbz;
    GridD g;
    xcd_tile(tbx, tby, tbz);
    if (!bv_enter_at(v, tbz, cav, bz, g)) return;
    const int nn[3] = {nnode(g, 0), nnode(g, 1), nnode(g, 2)};
    const int ox = tbx * CF::TX, oy = tby * CF::TY;
    const int kb = DIM == 3 ? zpar + 2 * bz * CF::PZ : 0;   // first updated plane
    if (ox >= nn[0] || oy >= nn[1] || kb >= nn[2]) return;
    const long node0 = bv_o(v, cav);
    const R* cur = cura + node0;
    const R* fix = fixa + node0;
    R* next = nexta + node0;
    const R* b = ba + node0;
    GridD gc = g;
    const R* pe = nullptr;
    if (PRO || RES) gc = bv_g2(v, gct, cav);
    if (PRO) pe = pea + bv_o2(v, oct, cav);
    // stage x (all planes kb-1 .. kb+2PZ-1; halo 4 in x, 2 in y) and b (the
    // updated planes on the colour-0 region); positions beyond a wall are 0,
    // periodic axes wrap; every load uses an in-range index
    {
        constexpr int K = (T::NS + TH - 1) / TH;
        R vx[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int t = threadIdx.x + u * TH;
            const int tt = t < T::NS ? t : 0;
            const int lx = tt % T::SX, ly = (tt / T::SX) % T::SY, lz = tt / (T::SX * T::SY);
            int p[3] = {ox - T::HX + lx, oy - T::HY + ly, DIM == 3 ? kb - 1 + lz : 0};
            bool ok = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                int q = p[a];
                if (g.per[a]) q = q < 0 ? q + nn[a] : (q >= nn[a] ? q - nn[a] : q);
                if (q < 0 || q >= nn[a]) { ok = false; q = 0; }
                p[a] = q;
            }
            const bool upd = DIM == 2 || ((p[2] & 1) == zpar);
            const R* src = upd ? cur : fix;
            R val = src[nid(g, p[0], p[1], p[2])];
            if (PRO) val = val + nodal_prolong_at<R>(gc, pe, p[0], p[1]);
            vx[u] = ok ? val : R(0);
        }
        constexpr int KB = (T::NB + TH - 1) / TH;
        R vb[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int t = threadIdx.x + u * TH;
            const int tt = t < T::NB ? t : 0;
            const int lx = tt % T::BX, ly = (tt / T::BX) % T::BY, lz = tt / (T::BX * T::BY);
            int p[3] = {ox - (T::HX - 1) + lx, oy - (T::HY - 1) + ly, DIM == 3 ? kb + 2 * lz : 0};
            bool ok = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                int q = p[a];
                if (g.per[a]) q = q < 0 ? q + nn[a] : (q >= nn[a] ? q - nn[a] : q);
                if (q < 0 || q >= nn[a]) { ok = false; q = 0; }
                p[a] = q;
            }
            const R val = b[nid(g, p[0], p[1], p[2])];
            vb[u] = ok ? val : R(0);
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int t = threadIdx.x + u * TH;
            if (t < T::NS) s[t] = vx[u];
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int t = threadIdx.x + u * TH;
            if (t < T::NB) sb[t] = vb[u];
        }
    }
    __syncthreads();
    // the four in-plane colours (of each sweep), each on its region of every
    // updated plane
#pragma unroll
    for (int q = 0; q < 4 * NSW; ++q) {
        const int cc = q & 3, w = q >> 2;
        const int gx = 4 * (NSW - 1 - w) + 3 - cc + (RES ? 2 : 0);
        const int gy = 2 * (NSW - 1 - w) + (cc <= 1 ? 1 : 0) + (RES ? 2 : 0);
        const int px = cc & 1, py = (cc >> 1) & 1;
        // region [ox - gx, ox + TX + gx) x [oy - gy, oy + TY + gy); the first
        // node of colour parity px along x, py along y
        const int x0 = ox - gx, y0 = oy - gy;
        const int fx = x0 + (((x0 & 1) != px) ? 1 : 0), fy = y0 + (((y0 & 1) != py) ? 1 : 0);
        const int wx = (ox + CF::TX + gx - fx + 1) / 2, wy = (oy + CF::TY + gy - fy + 1) / 2;
        const int cnt = wx * wy * CF::PZ;
        for (int t = threadIdx.x; t < cnt; t += TH) {
            const int ix = t % wx, iy = (t / wx) % wy, m = t / (wx * wy);
            int G[3] = {fx + 2 * ix, fy + 2 * iy, DIM == 3 ? kb + 2 * m : 0};
            const int lx = G[0] - ox + T::HX, ly = G[1] - oy + T::HY, lz = DIM == 3 ? 1 + 2 * m : 0;
            const int lb = (m * T::BY + (G[1] - oy + T::HY - 1)) * T::BX + (G[0] - ox + T::HX - 1);
            bool inside = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                if (G[a] >= 0 && G[a] < nn[a]) continue;
                if (g.per[a]) G[a] = G[a] < 0 ? G[a] + nn[a] : G[a] - nn[a];
                else inside = false;
            }
            if (!inside) continue;
            const int l = (lz * T::SY + ly) * T::SX + lx;
            R dg;
            const R Kx = block_K<DIM, R>(g, s, T::SX, T::SX * T::SY, G, l, &dg);
            s[l] = s[l] + (sb[lb] - Kx) / dg;
        }
        __syncthreads();
    }
    // the tile's nodes of the updated planes
    for (int t = threadIdx.x; t < CF::TX * CF::TY * CF::PZ; t += TH) {
        const int rx = t % CF::TX, ry = (t / CF::TX) % CF::TY, m = t / (CF::TX * CF::TY);
        const int G[3] = {ox + rx, oy + ry, DIM == 3 ? kb + 2 * m : 0};
        if (G[0] >= nn[0] || G[1] >= nn[1] || G[2] >= nn[2]) continue;
        next[nid(g, G[0], G[1], G[2])] = s[((DIM == 3 ? 1 + 2 * m : 0) * T::SY + ry + T::HY) * T::SX + rx + T::HX];
    }
    if constexpr (RES) {
        // residual at tile offsets [-1, TX) x [-1, TY) (periodic positions
        // are the wrapped nodes; positions beyond a wall are never read)
        for (int t = threadIdx.x; t < RX * RY; t += TH) {
            const int rx = t % RX - 1, ry = t / RX - 1;
            int G[3] = {ox + rx, oy + ry, 0};
            bool in = true;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                if (G[a] >= 0 && G[a] < nn[a]) continue;
                if (g.per[a]) G[a] = G[a] < 0 ? G[a] + nn[a] : G[a] - nn[a];
                else in = false;
            }
            R rv = R(0);
            if (in) {
                const int l = (ry + T::HY) * T::SX + rx + T::HX;
                const R Kx = block_K<DIM, R>(g, s, T::SX, T::SX * T::SY, G, l, nullptr);
                rv = sb[(ry + T::HY - 1) * T::BX + rx + T::HX - 1] - Kx;
            }
            rr[t] = rv;
        }
        __syncthreads();
        R* bcoarse = bca + bv_o2(v, oct, cav);
        R* xcoarse = xca + bv_o2(v, oct, cav);
        constexpr int CX = CF::TX / 2, CY = CF::TY / 2;
        for (int t = threadIdx.x; t < CX * CY; t += TH) {
            const int I[2] = {ox / 2 + t % CX, oy / 2 + t / CX};
            if (I[0] >= nnode(gc, 0) || I[1] >= nnode(gc, 1)) continue;
            R sum = 0;
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                int tt = u, lr[2];
                bool ok = true;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int del = tt % 3 - 1;
                    tt /= 3;
                    const int F = 2 * I[a] + del;
                    if ((F < 0 || F >= nn[a]) && !g.per[a]) ok = false;
                    lr[a] = F - (a == 0 ? ox : oy) + 1;
                }
                tt = u;
                R w = 1;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    if (tt % 3 != 1) w *= R(0.5);
                    tt /= 3;
                }
                const R val = rr[lr[1] * RX + lr[0]];
                sum = ok ? sum + w * val : sum;
            }
            const long qc = nid(gc, I[0], I[1], 0);
            bcoarse[qc] = sum;
            xcoarse[qc] = R(0);
        }
    }
}

template <int DIM>
static dim3 ntile_grid(const Ctx* c, const Level& L, BV& v)
{
    using T = NTile<DIM>;
    const GridD& g = L.gmax;
    v.zb = DIM == 3 ? (nnode(g, 2) + T::TZ - 1) / T::TZ : 1;
    return dim3((nnode(g, 0) + T::TX - 1) / T::TX, (nnode(g, 1) + T::TY - 1) / T::TY, v.zb * c->nb);
}

template <typename R>
void launch_nodal_gs(Ctx* c, const Level& L, const BV& v, int colour, R* x, const R* b)
{
    BV vv = v;
    if (L.gmax.dim == 2) {
        const dim3 grid = ntile_grid<2>(c, L, vv);
        k_nodal_gs_tile<2, R><<<grid, NTile<2>::THREADS, 0, c->s>>>(vv, colour, x, b);
    } else {
        const dim3 grid = ntile_grid<3>(c, L, vv);
        k_nodal_gs_tile<3, R><<<grid, NTile<3>::THREADS, 0, c->s>>>(vv, colour, x, b);
    }
}

template <int DIM, typename R, class CF>
static void nodal_sweep_impl(Ctx* c, const Level& L, const BV& v, const R* cur, R* next, const R* b, int nsw,
                             const R* pe, const GridD* gct, const long* oct, R* bc, R* xc)
{
    BV vv = v;
    if (DIM == 2) {
        vv.zb = 1;
        const dim3 grid((nnode(L.gmax, 0) + CF::TX - 1) / CF::TX, (nnode(L.gmax, 1) + CF::TY - 1) / CF::TY, c->nb);
        auto go = [&](auto kern) { kern<<<grid, CF::TH, 0, c->s>>>(vv, 0, cur, cur, next, b, pe, gct, oct, bc, xc); };
        if (nsw == 2) {
            if (pe) go(k_nodal_gs_fused<2, R, CF, 2, true, false>);
            else if (bc) go(k_nodal_gs_fused<2, R, CF, 2, false, true>);
            else go(k_nodal_gs_fused<2, R, CF, 2, false, false>);
        } else {
            if (pe) go(k_nodal_gs_fused<2, R, CF, 1, true, false>);
            else if (bc) go(k_nodal_gs_fused<2, R, CF, 1, false, true>);
            else go(k_nodal_gs_fused<2, R, CF, 1, false, false>);
        }
    } else {
        const int planes = (nnode(L.gmax, 2) + 1) / 2;   // even planes (at least as many as odd)
        vv.zb = (planes + CF::PZ - 1) / CF::PZ;
        const dim3 grid((nnode(L.gmax, 0) + CF::TX - 1) / CF::TX, (nnode(L.gmax, 1) + CF::TY - 1) / CF::TY,
                        vv.zb * c->nb);
        k_nodal_gs_fused<3, R, CF><<<grid, CF::TH, 0, c->s>>>(vv, 0, cur, cur, next, b);
        k_nodal_gs_fused<3, R, CF><<<grid, CF::TH, 0, c->s>>>(vv, 1, cur, next, next, b);
    }
}

template <int DIM, typename R, class Tiles, size_t... I>
static void nodal_sweep_pick(Ctx* c, const Level& L, const BV& v, const R* cur, R* next, const R* b, int k, int nsw,
                             const R* pe, const GridD* gct, const long* oct, R* bc, R* xc, std::index_sequence<I...>)
{
    ((k == (int)I ? nodal_sweep_impl<DIM, R, std::tuple_element_t<I, Tiles>>(c, L, v, cur, next, b, nsw, pe, gct, oct,
                                                                             bc, xc)
                  : void()),
     ...);
}

// nsw Gauss-Seidel sweeps (all 2^d colours; two in 2D only) from cur into
// next, with tile candidate `tile`; 2D: pe folds in the prolongation, bc/xc
// the residual restriction
template <typename R>
void launch_nodal_sweep(Ctx* c, const Level& L, const BV& v, const R* cur, R* next, const R* b, int tile, int nsw,
                        const R* pe, const GridD* gct, const long* oct, R* bc, R* xc)
{
    const int k = tile >= 0 && tile < kNG4Tiles ? tile : 0;
    constexpr auto seq = std::make_index_sequence<kNG4Tiles>{};
    if (L.gmax.dim == 2) nodal_sweep_pick<2, R, NG4Tiles2>(c, L, v, cur, next, b, k, nsw, pe, gct, oct, bc, xc, seq);
    else nodal_sweep_pick<3, R, NG4Tiles3>(c, L, v, cur, next, b, k, 1, nullptr, nullptr, nullptr, nullptr, nullptr, seq);
}

template <class TILES, size_t... I>
static void nodal_tile_of(int k, int* tx, int* ty, int* th, std::index_sequence<I...>)
{
    ((k == (int)I ? (void)(*tx = std::tuple_element_t<I, TILES>::TX, *ty = std::tuple_element_t<I, TILES>::TY,
                           *th = std::tuple_element_t<I, TILES>::TH)
                  : void()),
     ...);
}

void nodal_sweep_tile(int dim, int k, int* tx, int* ty, int* th)
{
    constexpr auto seq = std::make_index_sequence<kNG4Tiles>{};
    if (dim == 2) nodal_tile_of<NG4Tiles2>(k, tx, ty, th, seq);
    else nodal_tile_of<NG4Tiles3>(k, tx, ty, th, seq);
}

template <typename R>
void launch_nodal_resid(Ctx* c, const Level& L, const BV& v, const R* x, const R* b, R* r, int slot)
{
    BV vv = v;
    if (L.gmax.dim == 2) {
        const dim3 grid = ntile_grid<2>(c, L, vv);
        k_nodal_resid_tile<2, R><<<grid, NTile<2>::THREADS, 0, c->s>>>(vv, x, b, r, c->mpart, slot);
    } else {
        const dim3 grid = ntile_grid<3>(c, L, vv);
        k_nodal_resid_tile<3, R><<<grid, NTile<3>::THREADS, 0, c->s>>>(vv, x, b, r, c->mpart, slot);
    }
    if (slot >= 0) launch_max_final(c, vv.act, slot);
}

template void launch_nodal_sweep<double>(Ctx*, const Level&, const BV&, const double*, double*, const double*, int, int,
                                         const double*, const GridD*, const long*, double*, double*);
template void launch_nodal_sweep<float>(Ctx*, const Level&, const BV&, const float*, float*, const float*, int, int,
                                        const float*, const GridD*, const long*, float*, float*);
template void launch_nodal_gs<double>(Ctx*, const Level&, const BV&, int, double*, const double*);
template void launch_nodal_gs<float>(Ctx*, const Level&, const BV&, int, float*, const float*);
template void launch_nodal_resid<double>(Ctx*, const Level&, const BV&, const double*, const double*, double*, int);
template void launch_nodal_resid<float>(Ctx*, const Level&, const BV&, const float*, const float*, float*, int);

// dense coarsest matrix with the same assembled stencil (global reads)
template <int DIM>
__global__ void k_nodal_dense(GridD g, int N, const double* __restrict__ E, double* __restrict__ A)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (row >= N) return;
    const int nx = nnode(g, 0), ny = nnode(g, 1);
    const int G[3] = {row % nx, (row / nx) % ny, row / (nx * ny)};
    const double acc = K_glob<DIM>(g, E + (long)col * N, G[0], G[1], G[2], nullptr);
    A[(long)row * N + col] = acc;
}

void launch_nodal_dense(Ctx* c, const GridD& g, int N, const double* E, double* A)
{
    if (g.dim == 2) k_nodal_dense<2><<<dim3((N + 255) / 256, N), 256, 0, c->s>>>(g, N, E, A);
    else k_nodal_dense<3><<<dim3((N + 255) / 256, N), 256, 0, c->s>>>(g, N, E, A);
}

}  // namespace hb
