// hb_tail.hip -- the coarse end of a V-cycle in one launch (gfx950).
//
// Below some level every multigrid kernel is a handful of workgroups, and a
// launch costs more than its work.  Here one workgroup per cavity runs all
// levels from `lt` down to the cavity's coarsest and back up, with every
// level's iterate (plus a 1-cell halo), right-hand side and coefficients
// resident in LDS and barriers in place of launches.  The arithmetic per
// cell or node is the one of the per-level kernels (same stencil functions,
// same summation orders).  Cell problems (tensor viscous, MAC): red-black
// Gauss-Seidel component by component, residual restricted by the mean of
// the 2^d children, the coarsest system solved by its FP64 inverse,
// (bi/tri)linear prolongation.  Nodal problem: 2^d-colour Gauss-Seidel,
// full-weighting restriction, nodal interpolation, FP64 coarsest solve.  The coarse iterate at `lt`
// starts from zero (the restriction above zeroes it); the result is written
// to the level's current buffer.
//
// The halo holds the boundary images of the iterate: periodic axes wrap,
// walls take the odd reflection (homogeneous coarse problems), positions
// beyond two walls stay zero (the stencil never reads them).  The thread
// that writes a cell writes its images in the same pass, so no separate
// halo pass is needed: on smoothing levels every extent is even, and the
// image of a cell of one colour is read only by cells of the other colour.
#include "hb_internal.h"
#include "hb_ops.h"
#include "hb_stencil.h"

#include <cstdint>

namespace hb {

constexpr int kTailThreads = 512;   // tensor tail
// MAC tail: threads and cells of one colour per thread (2D: 1024 x 2, 3D:
// 512 x 4, where 1024 threads would spill); both cover 4096 cells
template <int DIM> struct MacTail {
    static constexpr int TH = DIM == 2 ? 1024 : 512, KC = DIM == 2 ? 2 : 4;
};
constexpr long kMacTailCells = 2L * MacTail<2>::TH * MacTail<2>::KC;
static_assert(kMacTailCells == 2L * MacTail<3>::TH * MacTail<3>::KC, "same first-level limit");

// LDS block of one level: `dim` components of (n0+2)(n1+2)[(n2+2)] cells
struct TailLay {
    int sx, sy, sxy, ns, hz;   // strides, positions per component, z halo (0 in 2D)
    __device__ inline int at(int i, int j, int k) const { return ((k + hz) * sy + j + 1) * sx + i + 1; }
};

__device__ inline TailLay tail_lay(const GridD& g)
{
    TailLay t;
    t.hz = g.dim == 3 ? 1 : 0;
    t.sx = g.n[0] + 2;
    t.sy = g.n[1] + 2;
    t.sxy = t.sx * t.sy;
    t.ns = t.sxy * (g.dim == 3 ? g.n[2] + 2 : 1);
    return t;
}

// The boundary images of cell G: up to 2^DIM - 1 halo positions (-1: none)
// and whether each takes -v.  Periodic axes wrap; a wall reflects with a
// sign; positions beyond two walls are never read and get no image.
template <int DIM>
struct Images {
    int pos[(1 << DIM) - 1];
    int neg;   // bit m - 1 set: image m takes -v
};

template <int DIM>
__device__ inline Images<DIM> cell_images(const GridD& g, const TailLay& t, const int G[3], bool walls = true)
{
    Images<DIM> im;
    im.neg = 0;
    int ic[3] = {0, 0, 0};
    bool has[3] = {false, false, false}, wall[3] = {false, false, false};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int n = g.n[a];
        wall[a] = !g.per[a];
        if (wall[a] && !walls) continue;
        if (G[a] == 0) { has[a] = true; ic[a] = g.per[a] ? n : -1; }
        else if (G[a] == n - 1) { has[a] = true; ic[a] = g.per[a] ? -1 : n; }
    }
#pragma unroll
    for (int m = 1; m < (1 << DIM); ++m) {
        int p[3] = {G[0], G[1], G[2]};
        int nw = 0;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (!((m >> a) & 1)) continue;
            ok = ok && has[a];
            p[a] = ic[a];
            if (wall[a]) ++nw;
        }
        im.pos[m - 1] = (ok && nw <= 1) ? t.at(p[0], p[1], p[2]) : -1;
        if (nw & 1) im.neg |= 1 << (m - 1);
    }
    return im;
}

// store v at LDS position l of one component and at the cell's images
template <int DIM, typename R>
__device__ inline void put_images(R* xq, int l, const Images<DIM>& im, R v)
{
    xq[l] = v;
#pragma unroll
    for (int m = 0; m < (1 << DIM) - 1; ++m)
        if (im.pos[m] >= 0) xq[im.pos[m]] = ((im.neg >> m) & 1) ? -v : v;
}

// Store v at cell G of one component and at each of its boundary images
// (walls = false: periodic images only).
template <int DIM, typename R>
__device__ inline void put_cell(const GridD& g, const TailLay& t, R* xq, const int G[3], R v, bool walls = true)
{
    put_images<DIM, R>(xq, t.at(G[0], G[1], G[2]), cell_images<DIM>(g, t, G, walls), v);
}

struct TailArgs {
    int nu1, nu2;                    // sweeps before / after the coarse correction
    const TailPlan* plan;            // per cavity: levels, LDS layout, offsets
    const void* beta[kMaxTail];      // level lt + i: face viscosities (storage type)
    void* x;                         // level lt iterate (current buffer)
    const void* b;                   // level lt right-hand side
    const CoarseD* cs;               // coarsest systems
    const double* Ainv;
    const int* act;
    const double* scb;               // scalar slots (dt)
};

extern __shared__ __align__(16) unsigned char tail_lds[];

// grid of tail level i (the fields the stencils use; uniform, so it lives in
// scalar registers)
template <int DIM>
__device__ inline GridD tail_grid(const TailPlan* __restrict__ P, int i)
{
    GridD g;
    g.dim = DIM;
    const TailLevel& T = P->lv[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.n[a] = T.n[a];
        g.per[a] = T.per[a];
    }
    g.h = T.h;
    return g;
}

template <int DIM, typename R>
__global__ void __launch_bounds__(kTailThreads) k_visc_tail(TailArgs A)
{
    const int cav = blockIdx.x, tid = threadIdx.x;
    if (A.act && !A.act[cav]) return;
    const TailPlan* __restrict__ P = A.plan + cav;
    const int nl = P->nl;   // levels of this cavity in the tail
    if (nl <= 0) return;
    R* lds = reinterpret_cast<R*>(tail_lds);
    const R dt = (R)A.scb[(long)cav * S_NSLOT + S_DT];
    // coefficients of every level, the right-hand side at lt, zero iterates
    for (int i = 0; i < nl; ++i) {
        const TailLevel& T = P->lv[i];
        const R* gb = reinterpret_cast<const R*>(A.beta[i]) + T.gofs;
        R* F = lds + T.foff;
        for (int t = tid; t < T.nf; t += kTailThreads) F[t] = gb[t];
        R* X = lds + T.xoff;
        for (int t = tid; t < DIM * T.ns; t += kTailThreads) X[t] = R(0);
    }
    {
        const TailLevel& T = P->lv[0];
        const R* gb = reinterpret_cast<const R*>(A.b) + DIM * P->o0;
        R* B = lds + T.boff;
        for (int t = tid; t < DIM * T.nc; t += kTailThreads) B[t] = gb[t];
    }
    __syncthreads();

    // red-black sweeps of level i, component by component.  Each thread
    // owns at most one cell of each colour (the host keeps a tail level's
    // cells within 2 * kTailThreads); its faces, diagonals, right-hand sides
    // and indices are set up once per visit, so a pass is the stencil and
    // the update only.
    auto smooth = [&](int i, int sweeps) {
        const GridD g = tail_grid<DIM>(P, i);
        const TailLevel& T = P->lv[i];
        const TailLay L = tail_lay(g);
        const int N = T.nc, H = N / 2;
        const R h = (R)g.h;
        const R ihh = R(1) / (h * h);
        R* X = lds + T.xoff;
        const R* B = lds + T.boff;
        const R* F = lds + T.foff;
        bool on[2];
        int l0[2], wm[2], G[2][3];
        Images<DIM> im[2];
        R bf[2][2 * DIM], dg[2][DIM], bq[2][DIM];
#pragma unroll
        for (int colour = 0; colour < 2; ++colour) {
            const int t = tid < H ? tid : 0;
            on[colour] = tid < H;
            const int hx = g.n[0] / 2;
            const int px = t % hx, j = (t / hx) % g.n[1], k = t / (hx * g.n[1]);
            G[colour][0] = 2 * px + ((j + k + colour) & 1);
            G[colour][1] = j;
            G[colour][2] = k;
            load_faces<DIM, R>(g, F, G[colour], bf[colour]);
            l0[colour] = L.at(G[colour][0], j, k);
            wm[colour] = wall_mask<DIM>(g, G[colour]);
            im[colour] = cell_images<DIM>(g, L, G[colour]);
            const int q0 = (int)cid(g, G[colour][0], j, k);
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                (void)visc_div_ih<DIM, false, R>(bf[colour], X, L.ns, L.sx, L.sxy, nullptr, q, wm[colour], l0[colour],
                                                 dt, ihh, &dg[colour][q]);
                bq[colour][q] = B[q * N + q0];
            }
        }
        for (int s = 0; s < sweeps; ++s)
#pragma unroll
            for (int q = 0; q < DIM; ++q)
#pragma unroll
                for (int colour = 0; colour < 2; ++colour) {
                    if (on[colour]) {
                        const R vd = visc_div_ih<DIM, false, R>(bf[colour], X, L.ns, L.sx, L.sxy, nullptr, q,
                                                                wm[colour], l0[colour], dt, ihh, nullptr);
                        const R xc = X[q * L.ns + l0[colour]];
                        const R Au = xc - dt * vd;
                        put_images<DIM, R>(X + q * L.ns, l0[colour], im[colour],
                                           xc + (bq[colour][q] - Au) / dg[colour][q]);
                    }
                    __syncthreads();
                }
    };

    // descend: smooth, residual, restriction (coarse iterate stays zero)
    for (int i = 0; i + 1 < nl; ++i) {
        smooth(i, A.nu1);
        const GridD g = tail_grid<DIM>(P, i);
        const TailLevel& T = P->lv[i];
        const TailLay L = tail_lay(g);
        const int N = T.nc;
        const R h = (R)g.h;
        const R ihh = R(1) / (h * h);
        const R* X = lds + T.xoff;
        const R* B = lds + T.boff;
        const R* F = lds + T.foff;
        R* Rr = lds + P->roff;
        for (int t = tid; t < N; t += kTailThreads) {
            const int G[3] = {t % g.n[0], (t / g.n[0]) % g.n[1], t / (g.n[0] * g.n[1])};
            R bf[2 * DIM];
            load_faces<DIM, R>(g, F, G, bf);
            const int l0 = L.at(G[0], G[1], G[2]);
            const int wm = wall_mask<DIM>(g, G);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const R vd = visc_div_ih<DIM, false, R>(bf, X, L.ns, L.sx, L.sxy, nullptr, c, wm, l0, dt, ihh, nullptr);
                const R Ax = X[c * L.ns + l0] - dt * vd;
                Rr[c * N + t] = B[c * N + t] - Ax;
            }
        }
        __syncthreads();
        const GridD gc = tail_grid<DIM>(P, i + 1);
        const int Nc = P->lv[i + 1].nc;
        R* Bc = lds + P->lv[i + 1].boff;
        constexpr int nch = 1 << DIM;
        for (int t = tid; t < Nc; t += kTailThreads) {
            const int C[3] = {t % gc.n[0], (t / gc.n[0]) % gc.n[1], t / (gc.n[0] * gc.n[1])};
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                R sum = 0;
#pragma unroll
                for (int bits = 0; bits < nch; ++bits) {
                    const int fx = 2 * C[0] + (bits & 1), fy = 2 * C[1] + ((bits >> 1) & 1),
                              fz = DIM == 3 ? 2 * C[2] + ((bits >> 2) & 1) : 0;
                    sum += Rr[c * N + cid(g, fx, fy, fz)];
                }
                Bc[c * Nc + t] = sum / R(nch);
            }
        }
        __syncthreads();
    }

    // coarsest: x = A^{-1} b, accumulated in FP64
    {
        const int i = nl - 1;
        const CoarseD cd = A.cs[cav];
        const GridD g = tail_grid<DIM>(P, i);
        const TailLevel& T = P->lv[i];
        const TailLay L = tail_lay(g);
        const int N = T.nc;
        const R* B = lds + T.boff;
        R* X = lds + T.xoff;
        for (int r = tid; r < cd.N; r += kTailThreads) {
            const double* row = A.Ainv + cd.aoff + (long)r * cd.N;
            double s = 0.0;
            for (int jj = 0; jj < cd.N; ++jj) s += row[jj] * (double)B[jj];
            const int c = r / N, t = r - c * N;
            const int G[3] = {t % g.n[0], (t / g.n[0]) % g.n[1], t / (g.n[0] * g.n[1])};
            put_cell<DIM, R>(g, L, X + c * L.ns, G, (R)s);
        }
        __syncthreads();
    }

    // ascend: prolongation (coarse neighbour beyond a wall: -e of the cell
    // itself), then smoothing
    for (int i = nl - 2; i >= 0; --i) {
        const GridD gf = tail_grid<DIM>(P, i);
        const GridD gc = tail_grid<DIM>(P, i + 1);
        const TailLay Lf = tail_lay(gf), Lc = tail_lay(gc);
        R* X = lds + P->lv[i].xoff;
        const R* E = lds + P->lv[i + 1].xoff;
        const int Nc = P->lv[i + 1].nc;
        for (int t = tid; t < Nc; t += kTailThreads) {
            const int C[3] = {t % gc.n[0], (t / gc.n[0]) % gc.n[1], t / (gc.n[0] * gc.n[1])};
            int src[3][3];
            R sgn[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    int J2 = C[a] + o - 1;
                    R sv = 1;
                    if (a < DIM && (J2 < 0 || J2 >= gc.n[a])) {
                        if (gc.per[a]) J2 = J2 < 0 ? J2 + gc.n[a] : J2 - gc.n[a];
                        else { J2 = C[a]; sv = R(-1); }
                    }
                    if (a >= DIM) J2 = 0;
                    src[a][o] = J2;
                    sgn[a][o] = sv;
                }
            constexpr int nz = DIM == 3 ? 2 : 1;
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                const R* e = E + q * Lc.ns;
                R nb[3][3][3];
#pragma unroll
                for (int oz = 0; oz < 3; ++oz)
#pragma unroll
                    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
                        for (int ox = 0; ox < 3; ++ox)
                            if (DIM == 3 || oz == 1) nb[oz][oy][ox] = e[Lc.at(src[0][ox], src[1][oy], src[2][oz])];
#pragma unroll
                for (int cz = 0; cz < nz; ++cz)
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 2; ++cx) {
                            const int ch[3] = {cx, cy, cz};
                            R s = 0;
#pragma unroll
                            for (int bits = 0; bits < (1 << DIM); ++bits) {
                                int o[3] = {1, 1, 1};
                                R w = 1, sv = 1;
#pragma unroll
                                for (int a = 0; a < DIM; ++a) {
                                    if (!((bits >> a) & 1)) { w *= R(0.75); continue; }
                                    w *= R(0.25);
                                    o[a] = ch[a] ? 2 : 0;
                                    sv *= sgn[a][o[a]];
                                }
                                s += w * sv * nb[o[2]][o[1]][o[0]];
                            }
                            const int G[3] = {2 * C[0] + cx, 2 * C[1] + cy, DIM == 3 ? 2 * C[2] + cz : 0};
                            R* xq = X + q * Lf.ns;
                            put_cell<DIM, R>(gf, Lf, xq, G, xq[Lf.at(G[0], G[1], G[2])] + s);
                        }
            }
        }
        __syncthreads();
        smooth(i, A.nu2);
    }

    // result of level lt
    {
        const GridD g = tail_grid<DIM>(P, 0);
        const TailLay L = tail_lay(g);
        const int N = P->lv[0].nc;
        const R* X = lds + P->lv[0].xoff;
        R* gx = reinterpret_cast<R*>(A.x) + DIM * P->o0;
        for (int t = tid; t < DIM * N; t += kTailThreads) {
            const int c = t / N, u = t - c * N;
            gx[t] = X[c * L.ns + L.at(u % g.n[0], (u / g.n[0]) % g.n[1], u / (g.n[0] * g.n[1]))];
        }
    }
}

// ---------------------------------------------------------------------------
// MAC problem (cell Poisson, zero flux through walls).  The halo holds the
// periodic images only: a neighbour beyond a wall is masked, as in the
// per-level kernels.  Each thread owns up to KC cells of each colour.
// ---------------------------------------------------------------------------

// L_mac x at cell G of an LDS level block (as mac_lap_at)
template <int DIM, typename R>
__device__ inline R tail_mac_lap(const GridD& g, const TailLay& L, const R* X, const int G[3], R ihh)
{
    const int off[3] = {1, L.sx, L.sxy};
    const int l0 = L.at(G[0], G[1], G[2]);
    const R xc = X[l0];
    R s = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const bool okh = g.per[a] || G[a] + 1 < g.n[a], okl = g.per[a] || G[a] > 0;
        const R xh = X[l0 + off[a]], xl = X[l0 - off[a]];
        const R Fhi = okh ? xh - xc : R(0);
        const R Flo = okl ? xc - xl : R(0);
        s += Fhi - Flo;
    }
    return s * ihh;
}

template <int DIM, typename R, int KC = MacTail<DIM>::KC, int TH = MacTail<DIM>::TH>
__global__ void __launch_bounds__(TH) k_mac_tail(TailArgs A)
{
    const int cav = blockIdx.x, tid = threadIdx.x;
    if (A.act && !A.act[cav]) return;
    const TailPlan* __restrict__ P = A.plan + cav;
    const int nl = P->nl;
    if (nl <= 0) return;
    R* lds = reinterpret_cast<R*>(tail_lds);
    for (int i = 0; i < nl; ++i) {
        const TailLevel& T = P->lv[i];
        R* X = lds + T.xoff;
        for (int t = tid; t < T.ns; t += TH) X[t] = R(0);
    }
    {
        const TailLevel& T = P->lv[0];
        const R* gb = reinterpret_cast<const R*>(A.b) + P->o0;
        R* B = lds + T.boff;
        for (int t = tid; t < T.nc; t += TH) B[t] = gb[t];
    }
    __syncthreads();

    // red-black sweeps of level i; per owned cell: LDS index, neighbour mask,
    // diagonal, right-hand side and periodic images, set up once per visit
    auto smooth = [&](int i, int sweeps) {
        const GridD g = tail_grid<DIM>(P, i);
        const TailLevel& T = P->lv[i];
        const TailLay L = tail_lay(g);
        const int off[3] = {1, L.sx, L.sxy};
        const int H = T.nc / 2, hx = g.n[0] / 2;
        const R h = (R)g.h;
        const R ih2 = R(1) / (h * h);
        R* X = lds + T.xoff;
        const R* B = lds + T.boff;
        bool on[2][KC];
        int l0[2][KC], okm[2][KC];
        R dg[2][KC], bq[2][KC];
        Images<DIM> im[2][KC];
#pragma unroll
        for (int colour = 0; colour < 2; ++colour)
#pragma unroll
            for (int u = 0; u < KC; ++u) {
                const int t0 = tid + u * TH;
                on[colour][u] = t0 < H;
                const int t = t0 < H ? t0 : 0;
                const int px = t % hx, j = (t / hx) % g.n[1], k = t / (hx * g.n[1]);
                const int G[3] = {2 * px + ((j + k + colour) & 1), j, k};
                l0[colour][u] = L.at(G[0], j, k);
                int m = 0, cnt = 0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const bool okl = g.per[a] || G[a] > 0, okh = g.per[a] || G[a] + 1 < g.n[a];
                    m |= (okl ? 1 : 0) << (2 * a);
                    m |= (okh ? 2 : 0) << (2 * a);
                    cnt += (okl ? 1 : 0) + (okh ? 1 : 0);
                }
                okm[colour][u] = m;
                dg[colour][u] = -(R)cnt * ih2;
                bq[colour][u] = B[cid(g, G[0], j, k)];
                im[colour][u] = cell_images<DIM>(g, L, G, false);
            }
        for (int s = 0; s < sweeps; ++s)
#pragma unroll
            for (int colour = 0; colour < 2; ++colour) {
#pragma unroll
                for (int u = 0; u < KC; ++u) {
                    if (!on[colour][u]) continue;
                    const int l = l0[colour][u];
                    const R xq = X[l];
                    R xn[DIM][2];
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        xn[a][0] = X[l - off[a]];
                        xn[a][1] = X[l + off[a]];
                    }
                    R Lx = 0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a)
#pragma unroll
                        for (int side = 0; side < 2; ++side) {
                            const bool ok = (okm[colour][u] >> (2 * a + side)) & 1;
                            Lx += ok ? (xn[a][side] - xq) * ih2 : R(0);
                        }
                    put_images<DIM, R>(X, l, im[colour][u], xq + (bq[colour][u] - Lx) / dg[colour][u]);
                }
                __syncthreads();
            }
    };

    // descend: smooth, then each coarse cell restricts the residuals of its
    // children (as the per-level residual-restriction kernel)
    for (int i = 0; i + 1 < nl; ++i) {
        smooth(i, A.nu1);
        const GridD g = tail_grid<DIM>(P, i);
        const TailLay L = tail_lay(g);
        const R h = (R)g.h;
        const R ihh = R(1) / (h * h);
        const R* X = lds + P->lv[i].xoff;
        const R* B = lds + P->lv[i].boff;
        const GridD gc = tail_grid<DIM>(P, i + 1);
        const int Nc = P->lv[i + 1].nc;
        R* Bc = lds + P->lv[i + 1].boff;
        constexpr int nch = 1 << DIM;
        for (int t = tid; t < Nc; t += TH) {
            const int C[3] = {t % gc.n[0], (t / gc.n[0]) % gc.n[1], t / (gc.n[0] * gc.n[1])};
            R sum = 0;
#pragma unroll
            for (int bits = 0; bits < nch; ++bits) {
                const int F[3] = {2 * C[0] + (bits & 1), 2 * C[1] + ((bits >> 1) & 1),
                                  DIM == 3 ? 2 * C[2] + ((bits >> 2) & 1) : 0};
                sum += B[cid(g, F[0], F[1], F[2])] - tail_mac_lap<DIM, R>(g, L, X, F, ihh);
            }
            Bc[t] = sum / R(nch);
        }
        __syncthreads();
    }

    // coarsest: x = A^{-1} b, accumulated in FP64
    {
        const int i = nl - 1;
        const CoarseD cd = A.cs[cav];
        const GridD g = tail_grid<DIM>(P, i);
        const TailLay L = tail_lay(g);
        const R* B = lds + P->lv[i].boff;
        R* X = lds + P->lv[i].xoff;
        for (int r = tid; r < cd.N; r += TH) {
            const double* row = A.Ainv + cd.aoff + (long)r * cd.N;
            double s = 0.0;
            for (int jj = 0; jj < cd.N; ++jj) s += row[jj] * (double)B[jj];
            const int G[3] = {r % g.n[0], (r / g.n[0]) % g.n[1], r / (g.n[0] * g.n[1])};
            put_cell<DIM, R>(g, L, X, G, (R)s, false);
        }
        __syncthreads();
    }

    // ascend: prolongation (coarse neighbour beyond a wall: the cell itself),
    // then smoothing
    for (int i = nl - 2; i >= 0; --i) {
        const GridD gf = tail_grid<DIM>(P, i);
        const GridD gc = tail_grid<DIM>(P, i + 1);
        const TailLay Lf = tail_lay(gf), Lc = tail_lay(gc);
        R* X = lds + P->lv[i].xoff;
        const R* E = lds + P->lv[i + 1].xoff;
        const int Nc = P->lv[i + 1].nc;
        for (int t = tid; t < Nc; t += TH) {
            const int C[3] = {t % gc.n[0], (t / gc.n[0]) % gc.n[1], t / (gc.n[0] * gc.n[1])};
            int src[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    int J2 = C[a] + o - 1;
                    if (a < DIM && (J2 < 0 || J2 >= gc.n[a])) {
                        if (gc.per[a]) J2 = J2 < 0 ? J2 + gc.n[a] : J2 - gc.n[a];
                        else J2 = C[a];
                    }
                    if (a >= DIM) J2 = 0;
                    src[a][o] = J2;
                }
            R nb[3][3][3];
#pragma unroll
            for (int oz = 0; oz < 3; ++oz)
#pragma unroll
                for (int oy = 0; oy < 3; ++oy)
#pragma unroll
                    for (int ox = 0; ox < 3; ++ox)
                        if (DIM == 3 || oz == 1) nb[oz][oy][ox] = E[Lc.at(src[0][ox], src[1][oy], src[2][oz])];
            constexpr int nz = DIM == 3 ? 2 : 1;
#pragma unroll
            for (int cz = 0; cz < nz; ++cz)
#pragma unroll
                for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                    for (int cx = 0; cx < 2; ++cx) {
                        const int ch[3] = {cx, cy, cz};
                        R s = 0;
#pragma unroll
                        for (int bits = 0; bits < (1 << DIM); ++bits) {
                            int o[3] = {1, 1, 1};
                            R w = 1, sv = 1;
#pragma unroll
                            for (int a = 0; a < DIM; ++a) {
                                if (!((bits >> a) & 1)) { w *= R(0.75); continue; }
                                w *= R(0.25);
                                o[a] = ch[a] ? 2 : 0;
                                sv *= R(1);
                            }
                            s += w * sv * nb[o[2]][o[1]][o[0]];
                        }
                        const int G[3] = {2 * C[0] + cx, 2 * C[1] + cy, DIM == 3 ? 2 * C[2] + cz : 0};
                        put_cell<DIM, R>(gf, Lf, X, G, X[Lf.at(G[0], G[1], G[2])] + s, false);
                    }
        }
        __syncthreads();
        smooth(i, A.nu2);
    }

    {
        const GridD g = tail_grid<DIM>(P, 0);
        const TailLay L = tail_lay(g);
        const int N = P->lv[0].nc;
        const R* X = lds + P->lv[0].xoff;
        R* gx = reinterpret_cast<R*>(A.x) + P->o0;
        for (int t = tid; t < N; t += TH)
            gx[t] = X[L.at(t % g.n[0], (t / g.n[0]) % g.n[1], t / (g.n[0] * g.n[1]))];
    }
}

// ---------------------------------------------------------------------------
// Nodal problem (Q1 stiffness K, natural boundary on walls).  Each level's
// nodes sit in a block with a 1-node halo that holds the periodic images;
// halo positions beyond a wall stay zero (their stencil weights are zero,
// as in the tiled kernels, which read zeros there).  A sweep runs the 2^d
// colours (i&1) + 2(j&1) + 4(k&1) in order, as the per-level sweeps; the
// residual is stored for the full-weighting restriction; prolongation is the
// (bi/tri)linear interpolation; the coarsest system is solved by its FP64
// inverse.  Same per-node arithmetic and summation order as the per-level
// kernels.  The first level holds at most 2^d * kNodalTailThreads *
// kNodalTailKN nodes: one CU runs the whole tail, and on a larger level a
// colour pass costs it more than the level's own launches cost the chip.
// ---------------------------------------------------------------------------
constexpr int kNodalTailThreads = 1024;
constexpr int kNodalTailKN = 1;

// the level's node lattice as a grid of "cells" (node counts per axis), for
// the LDS layout and the periodic images
__device__ inline GridD node_grid(const GridD& g)
{
    GridD q = g;
#pragma unroll
    for (int a = 0; a < 3; ++a) q.n[a] = nnode(g, a);
    return q;
}

__device__ inline void node_of(const GridD& gn, int t, int G[3])
{
    G[0] = t % gn.n[0];
    G[1] = (t / gn.n[0]) % gn.n[1];
    G[2] = t / (gn.n[0] * gn.n[1]);
}

template <int DIM, typename R>
__global__ void __launch_bounds__(kNodalTailThreads) k_nodal_tail(TailArgs A)
{
    constexpr int TH = kNodalTailThreads;
    const int cav = blockIdx.x, tid = threadIdx.x;
    if (A.act && !A.act[cav]) return;
    const TailPlan* __restrict__ P = A.plan + cav;
    const int nl = P->nl;
    if (nl <= 0) return;
    R* lds = reinterpret_cast<R*>(tail_lds);
    for (int i = 0; i < nl; ++i) {
        const TailLevel& T = P->lv[i];
        R* X = lds + T.xoff;
        for (int t = tid; t < T.ns; t += TH) X[t] = R(0);
    }
    {
        const TailLevel& T = P->lv[0];
        const R* gb = reinterpret_cast<const R*>(A.b) + P->o0;
        R* B = lds + T.boff;
        for (int t = tid; t < T.nc; t += TH) B[t] = gb[t];
    }
    __syncthreads();

    // Gauss-Seidel sweeps of level i: the nodes of one colour share no
    // element, and a node's periodic image is read only by nodes of other
    // colours (periodic node counts are even on smoothing levels)
    auto smooth = [&](int i, int sweeps) {
        const GridD g = tail_grid<DIM>(P, i);
        const GridD gn = node_grid(g);
        const TailLay L = tail_lay(gn);
        const TailLevel& T = P->lv[i];
        R* X = lds + T.xoff;
        const R* B = lds + T.boff;
        for (int s = 0; s < sweeps; ++s)
            for (int colour = 0; colour < (1 << DIM); ++colour) {
                int par[3], cn[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    par[a] = a < DIM ? (colour >> a) & 1 : 0;
                    cn[a] = a < DIM ? (gn.n[a] + 1 - par[a]) / 2 : 1;
                }
                const int cnt = cn[0] * cn[1] * cn[2];
                for (int t = tid; t < cnt; t += TH) {
                    const int G[3] = {2 * (t % cn[0]) + par[0], 2 * ((t / cn[0]) % cn[1]) + par[1],
                                      DIM == 3 ? 2 * (t / (cn[0] * cn[1])) + par[2] : 0};
                    const int l = L.at(G[0], G[1], G[2]);
                    R dg;
                    const R Kx = block_K<DIM, R>(g, X, L.sx, L.sxy, G, l, &dg);
                    put_cell<DIM, R>(gn, L, X, G, X[l] + (B[nid(g, G[0], G[1], G[2])] - Kx) / dg, false);
                }
                __syncthreads();
            }
    };

    // descend: smooth, residual, full-weighting restriction (the coarse
    // iterate stays zero)
    for (int i = 0; i + 1 < nl; ++i) {
        smooth(i, A.nu1);
        const GridD g = tail_grid<DIM>(P, i);
        const GridD gn = node_grid(g);
        const TailLay L = tail_lay(gn);
        const TailLevel& T = P->lv[i];
        const R* X = lds + T.xoff;
        const R* B = lds + T.boff;
        R* Rr = lds + P->roff;
        for (int t = tid; t < T.nc; t += TH) {
            int G[3];
            node_of(gn, t, G);
            const R Kx = block_K<DIM, R>(g, X, L.sx, L.sxy, G, L.at(G[0], G[1], G[2]), nullptr);
            Rr[t] = B[t] - Kx;
        }
        __syncthreads();
        const GridD gcn = node_grid(tail_grid<DIM>(P, i + 1));
        const TailLevel& Tc = P->lv[i + 1];
        R* Bc = lds + Tc.boff;
        constexpr int nt = DIM == 3 ? 27 : 9;
        for (int t = tid; t < Tc.nc; t += TH) {
            int I[3];
            node_of(gcn, t, I);
            R s = 0;
#pragma unroll
            for (int u = 0; u < nt; ++u) {
                int tt = u, p[3] = {0, 0, 0};
                bool ok = true;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const int del = tt % 3 - 1;
                    tt /= 3;
                    int F = 2 * I[a] + del;
                    const int nf = gn.n[a];
                    if (F < 0 || F >= nf) {
                        if (g.per[a]) F = F < 0 ? F + nf : F - nf;
                        else { ok = false; F = 0; }
                    }
                    p[a] = F;
                }
                tt = u;
                R w = 1;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    if (tt % 3 != 1) w *= R(0.5);
                    tt /= 3;
                }
                const R val = Rr[nid(g, p[0], p[1], p[2])];
                s = ok ? s + w * val : s;
            }
            Bc[t] = s;
        }
        __syncthreads();
    }

    // coarsest: x = A^{-1} b, accumulated in FP64
    {
        const int i = nl - 1;
        const CoarseD cd = A.cs[cav];
        const GridD gn = node_grid(tail_grid<DIM>(P, i));
        const TailLay L = tail_lay(gn);
        const R* B = lds + P->lv[i].boff;
        R* X = lds + P->lv[i].xoff;
        for (int r = tid; r < cd.N; r += TH) {
            const double* row = A.Ainv + cd.aoff + (long)r * cd.N;
            double s = 0.0;
            for (int jj = 0; jj < cd.N; ++jj) s += row[jj] * (double)B[jj];
            int G[3];
            node_of(gn, r, G);
            put_cell<DIM, R>(gn, L, X, G, (R)s, false);
        }
        __syncthreads();
    }

    // ascend: x_f += P e_c (a fine node takes the mean of the coarse nodes
    // of its coarse edge, face or cell), then smoothing
    for (int i = nl - 2; i >= 0; --i) {
        const GridD gc = tail_grid<DIM>(P, i + 1);
        const GridD gfn = node_grid(tail_grid<DIM>(P, i)), gcn = node_grid(gc);
        const TailLay Lf = tail_lay(gfn), Lc = tail_lay(gcn);
        R* X = lds + P->lv[i].xoff;
        const R* E = lds + P->lv[i + 1].xoff;
        for (int t = tid; t < P->lv[i].nc; t += TH) {
            int F[3];
            node_of(gfn, t, F);
            R s = 0;
#pragma unroll
            for (int bits = 0; bits < (1 << DIM); ++bits) {
                int p[3] = {0, 0, 0};
                R w = 1;
                bool ok = true;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const int hi = (bits >> a) & 1;
                    if (!(F[a] & 1)) {
                        if (hi) ok = false;
                        p[a] = F[a] >> 1;
                    } else {
                        w *= R(0.5);
                        int C = ((F[a] - 1) >> 1) + hi;
                        if (gc.per[a] && C == gcn.n[a]) C = 0;
                        p[a] = C;
                    }
                }
                const R val = E[Lc.at(p[0], p[1], p[2])];
                s = ok ? s + w * val : s;
            }
            const int l = Lf.at(F[0], F[1], F[2]);
            put_cell<DIM, R>(gfn, Lf, X, F, X[l] + s, false);
        }
        __syncthreads();
        smooth(i, A.nu2);
    }

    // result of level lt
    {
        const GridD gn = node_grid(tail_grid<DIM>(P, 0));
        const TailLay L = tail_lay(gn);
        const R* X = lds + P->lv[0].xoff;
        R* gx = reinterpret_cast<R*>(A.x) + P->o0;
        for (int t = tid; t < P->lv[0].nc; t += TH) {
            int G[3];
            node_of(gn, t, G);
            gx[t] = X[L.at(G[0], G[1], G[2])];
        }
    }
}

// Tail plan of one cavity from its levels lt..lc for problem op (grids gl,
// face offsets in the level arenas gofs (tensor problem), component-array
// offset o0 at lt): the LDS layout (per level the iterate with its halo, the
// right-hand side and, tensor problem, the face viscosities; then, tensor
// and nodal problems, one residual array of the first level).  Returns the
// LDS bytes for storage size elem, or SIZE_MAX when the first level has
// more unknowns per colour than the kernel's threads cover (tensor: one cell
// per thread, MAC: kMacTailCells at the first level, nodal: kNodalTailKN
// nodes).
size_t tail_plan(int op, const std::vector<GridD>& gl, const std::vector<long>& gofs, long o0, size_t elem,
                 TailPlan* out)
{
    TailPlan P{};
    if (gl.empty()) {
        if (out) *out = P;
        return 0;
    }
    const bool visc = op == HB_OP_VISC, nodal = op == HB_OP_NODAL;
    const int d = gl[0].dim;
    // unknowns per level: cells, or nodes (node counts per axis nn)
    auto count = [&](const GridD& g) {
        return nodal ? (long)nnode(g, 0) * nnode(g, 1) * nnode(g, 2) : ncells(g);
    };
    const long limit = nodal ? (1L << d) * kNodalTailThreads * kNodalTailKN
                             : (visc ? 2L * kTailThreads : kMacTailCells);
    if (gl.size() > (size_t)kMaxTail || (gl.size() > 1 && count(gl[0]) > limit)) return SIZE_MAX;
    const int nc = visc ? d : 1;
    long o = 0;
    for (size_t i = 0; i < gl.size(); ++i) {
        const GridD& g = gl[i];
        TailLevel& T = P.lv[i];
        for (int a = 0; a < 3; ++a) {
            T.n[a] = g.n[a];
            T.per[a] = g.per[a];
        }
        T.h = g.h;
        T.nc = (int)count(g);
        const int e[3] = {nodal ? nnode(g, 0) : g.n[0], nodal ? nnode(g, 1) : g.n[1], nodal ? nnode(g, 2) : g.n[2]};
        T.ns = (e[0] + 2) * (e[1] + 2) * (d == 3 ? e[2] + 2 : 1);
        long nf = 0;
        if (visc)
            for (int a = 0; a < d; ++a) nf += fcount(g, a);
        T.nf = (int)nf;
        T.gofs = visc ? gofs[i] : 0;
        T.xoff = (int)o;
        o += (long)nc * T.ns;
        T.boff = (int)o;
        o += (long)nc * T.nc;
        T.foff = (int)o;
        o += nf;
    }
    P.roff = (int)o;
    if (visc) o += (long)d * P.lv[0].nc;
    if (nodal && gl.size() > 1) o += P.lv[0].nc;
    P.nl = (int)gl.size();
    P.o0 = o0;
    if (out) *out = P;
    return (size_t)o * elem;
}

template <typename R>
void launch_mac_tail(Ctx* c, const MG& m, int lt, int nu1, int nu2, size_t lds, const int* act)
{
    TailArgs A{};
    A.nu1 = nu1;
    A.nu2 = nu2;
    A.plan = m.tplan;
    A.x = LB<R>::x(m.L[lt]);
    A.b = LB<R>::b(m.L[lt]);
    A.cs = m.cs;
    A.Ainv = m.Ainv;
    A.act = act;
    A.scb = c->sc;
    if (c->dim == 2) k_mac_tail<2, R><<<c->nb, MacTail<2>::TH, lds, c->s>>>(A);
    else k_mac_tail<3, R><<<c->nb, MacTail<3>::TH, lds, c->s>>>(A);
}

template <typename R>
void launch_nodal_tail(Ctx* c, const MG& m, int lt, int nu1, int nu2, size_t lds, const int* act)
{
    TailArgs A{};
    A.nu1 = nu1;
    A.nu2 = nu2;
    A.plan = m.tplan;
    A.x = LB<R>::x(m.L[lt]);
    A.b = LB<R>::b(m.L[lt]);
    A.cs = m.cs;
    A.Ainv = m.Ainv;
    A.act = act;
    A.scb = c->sc;
    if (c->dim == 2) k_nodal_tail<2, R><<<c->nb, kNodalTailThreads, lds, c->s>>>(A);
    else k_nodal_tail<3, R><<<c->nb, kNodalTailThreads, lds, c->s>>>(A);
}

template <typename R>
void launch_visc_tail(Ctx* c, const MG& m, int lt, int nu1, int nu2, size_t lds, const int* act)
{
    TailArgs A{};
    A.nu1 = nu1;
    A.nu2 = nu2;
    A.plan = m.tplan;
    for (int i = 0; i < kMaxTail && lt + i < m.nlev; ++i) A.beta[i] = LB<R>::beta(m.L[lt + i]);
    A.x = LB<R>::x(m.L[lt]);
    A.b = LB<R>::b(m.L[lt]);
    A.cs = m.cs;
    A.Ainv = m.Ainv;
    A.act = act;
    A.scb = c->sc;
    if (c->dim == 2) k_visc_tail<2, R><<<c->nb, kTailThreads, lds, c->s>>>(A);
    else k_visc_tail<3, R><<<c->nb, kTailThreads, lds, c->s>>>(A);
}

// allow the tail kernels dynamic LDS up to `bytes`
void tail_allow_lds(size_t bytes)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mac_tail<2, double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mac_tail<3, double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mac_tail<2, float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mac_tail<3, float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nodal_tail<2, double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nodal_tail<3, double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nodal_tail<2, float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nodal_tail<3, float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_visc_tail<2, double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_visc_tail<3, double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_visc_tail<2, float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_visc_tail<3, float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template void launch_visc_tail<double>(Ctx*, const MG&, int, int, int, size_t, const int*);
template void launch_visc_tail<float>(Ctx*, const MG&, int, int, int, size_t, const int*);
template void launch_mac_tail<double>(Ctx*, const MG&, int, int, int, size_t, const int*);
template void launch_nodal_tail<double>(Ctx*, const MG&, int, int, int, size_t, const int*);
template void launch_nodal_tail<float>(Ctx*, const MG&, int, int, int, size_t, const int*);
template void launch_mac_tail<float>(Ctx*, const MG&, int, int, int, size_t, const int*);

}  // namespace hb
