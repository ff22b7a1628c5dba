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

// K x at node G from the LDS tile (local index l), and the diagonal
template <int DIM, typename R>
__device__ inline R tile_K(const GridD& g, const R* s, const int G[3], int l, R* diag)
{
    using T = NTile<DIM>;
    int cnt[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) cnt[a][d] = a < DIM ? node_cnt(g, a, G[a], d - 1) : (d == 1 ? 1 : 0);
    R acc = 0;
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int k = (dx != 0) + (dy != 0) + (dz != 0);
                const R w = (R)(q1_ke(DIM, g.h, k) * (double)(cnt[0][dx + 1] * cnt[1][dy + 1] * cnt[2][dz + 1]));
                acc += w * s[l + (dz * T::SY + dy) * T::SX + dx];
            }
    if (diag) *diag = (R)(q1_ke(DIM, g.h, 0) * (double)(cnt[0][1] * cnt[1][1] * cnt[2][1]));
    return acc;
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
        const R val = x[ok ? nid(g, p[0], p[1], p[2]) : 0];
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
    const long node0 = v.o[cav];

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
    const long q = ok ? nid(g, G[0], G[1], G[2]) : 0;
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
                   double* __restrict__ scb, int slot)
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
        tq[u] = tOk[u] ? nid(g, G[0], G[1], G[2]) : 0;
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
        if (threadIdx.x == 0) atomic_max_bits(scb + (long)cav * S_NSLOT + slot, m);
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

template <typename R>
void launch_nodal_resid(Ctx* c, const Level& L, const BV& v, const R* x, const R* b, R* r, int slot)
{
    BV vv = v;
    if (L.gmax.dim == 2) {
        const dim3 grid = ntile_grid<2>(c, L, vv);
        k_nodal_resid_tile<2, R><<<grid, NTile<2>::THREADS, 0, c->s>>>(vv, x, b, r, c->sc, slot);
    } else {
        const dim3 grid = ntile_grid<3>(c, L, vv);
        k_nodal_resid_tile<3, R><<<grid, NTile<3>::THREADS, 0, c->s>>>(vv, x, b, r, c->sc, slot);
    }
}

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
