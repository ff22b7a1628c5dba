// hb_mg.hip -- multigrid kernels of the cell-centred scalar (MAC) problem
// and the nodal Q1 projection problem, cell prolongation shared with the
// tensor problem, and the dense coarsest-level solve.  gfx950; the cycle
// kernels are templated on the storage and arithmetic type R (double, or
// float in the mixed-precision correction cycles).
#include "hb_internal.h"
#include "hb_ops.h"

namespace hb {

static const dim3 kBlk(64, 4, 1);

// ---------------------------------------------------------------------------
// MAC problem: L_mac = D_mac G_mac, zero flux through wall faces
// ---------------------------------------------------------------------------

// Batched launches: block z = cavity * zb + z index within the cavity; each
// block takes its cavity's grid and offsets from the level tables (see
// hb_internal.h) and returns when the cavity takes no part.
#define PT_ENTER(k)                                \
    int cav, k;                                    \
    GridD g;                                       \
    if (!bv_enter(v, cav, k, g)) return;

template <int DIM, typename R>
__global__ void k_mac_rb(BV v, int colour, R* __restrict__ xa, const R* __restrict__ ba)
{
    PT_ENTER(k);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int i = 2 * t + ((j + k + colour) & 1);
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return;
    R* x = xa + bv_o(v, cav);
    const R* b = ba + bv_o(v, cav);
    const long q = cid(g, i, j, k);
    const R h = (R)g.h;
    const R ih2 = R(1) / (h * h);
    // all loads first (neighbours beyond a wall read the cell itself and are
    // masked), then the sum in the order lo, hi per axis
    const R xq = x[q], bq = b[q];
    R xn[DIM][2];
    bool ok[DIM][2];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int side = 0; side < 2; ++side) xn[a][side] = x[nb_cell<DIM>(g, i, j, k, a, side ? 1 : -1, ok[a][side])];
    R Lx = 0;
    int cnt = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            Lx += ok[a][side] ? (xn[a][side] - xq) * ih2 : R(0);
            cnt += ok[a][side] ? 1 : 0;
        }
    const R dg = -(R)cnt * ih2;
    x[q] = xq + (bq - Lx) / dg;
}

template <typename R>
void launch_mac_rb(Ctx* c, const Level& L, const BV& v, int colour, R* x, const R* b)
{
    BV vv = v;
    vv.zb = L.gmax.n[2];
    const dim3 grid = grid3((L.gmax.n[0] + 1) / 2, L.gmax.n[1], vv.zb * c->nb, kBlk);
    if (L.gmax.dim == 2) k_mac_rb<2, R><<<grid, kBlk, 0, c->s>>>(vv, colour, x, b);
    else k_mac_rb<3, R><<<grid, kBlk, 0, c->s>>>(vv, colour, x, b);
}

// r = b - L x (max-norm into each cavity's slot) or y = L x (b null); FP64
template <int DIM>
__global__ void k_mac_resid(BV v, const double* __restrict__ xa, const double* __restrict__ ba, double* __restrict__ ra,
                            unsigned long long* __restrict__ mp, int slot)
{
    __shared__ unsigned long long sh[16];
    PT_ENTER(k);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const long o = bv_o(v, cav);
    unsigned long long m = 0ull;
    if (i < g.n[0] && j < g.n[1] && k < g.n[2]) {
        const long q = cid(g, i, j, k);
        const double Lx = mac_lap_at<DIM, double>(g, xa + o, i, j, k);
        if (ba) {
            const double rv = ba[o + q] - Lx;
            if (ra) ra[o + q] = rv;
            m = abits(rv);
        } else {
            ra[o + q] = Lx;
        }
    }
    if (slot >= 0) {
        m = block_umax(m, sh);
        if (threadIdx.x + threadIdx.y == 0)
            max_partial(mp, cav, ((long)k * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, m);
    }
}

void launch_mac_resid(Ctx* c, const Level& L, const BV& v, const double* x, const double* b, double* r, int slot)
{
    BV vv = v;
    vv.zb = L.gmax.n[2];
    const dim3 grid = grid3(L.gmax.n[0], L.gmax.n[1], vv.zb * c->nb, kBlk);
    if (L.gmax.dim == 2) k_mac_resid<2><<<grid, kBlk, 0, c->s>>>(vv, x, b, r, c->mpart, slot);
    else k_mac_resid<3><<<grid, kBlk, 0, c->s>>>(vv, x, b, r, c->mpart, slot);
    if (slot >= 0) launch_max_final(c, vv.act, slot);
}

// coarse right-hand side = mean of the fine residuals of the 2^d children;
// the coarse iterate starts from zero.  One thread per coarse cell.
template <int DIM, typename R>
__global__ void __launch_bounds__(256) k_mac_resid_restrict(BV v, const GridD* __restrict__ gft, const long* __restrict__ oft,
                                     const R* __restrict__ xfa, const R* __restrict__ bfa, R* __restrict__ bca,
                                     R* __restrict__ xca)
{
    PT_ENTER(k);
    const GridD& gc = g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= gc.n[0] || j >= gc.n[1] || k >= gc.n[2]) return;
    const GridD gf = bv_g2(v, gft, cav);
    const R* xf = xfa + bv_o2(v, oft, cav);
    const R* bf = bfa + bv_o2(v, oft, cav);
    constexpr int nch = 1 << DIM;
    R s = 0;
#pragma unroll
    for (int bits = 0; bits < nch; ++bits) {
        const int fi = 2 * i + (bits & 1), fj = 2 * j + ((bits >> 1) & 1), fk = DIM == 3 ? 2 * k + ((bits >> 2) & 1) : 0;
        s += bf[cid(gf, fi, fj, fk)] - mac_lap_at<DIM, R>(gf, xf, fi, fj, fk);
    }
    const long qc = bv_o(v, cav) + cid(gc, i, j, k);
    bca[qc] = s / (R)nch;
    xca[qc] = R(0);
}

template <typename R>
void launch_mac_resid_restrict(Ctx* c, const Level& C, const BV& vc, const GridD* gf, const long* of_, const R* xf,
                               const R* bf, R* bc, R* xc)
{
    BV vv = vc;
    vv.zb = C.gmax.n[2];
    const dim3 grid = grid3(C.gmax.n[0], C.gmax.n[1], vv.zb * c->nb, kBlk);
    if (C.gmax.dim == 2) k_mac_resid_restrict<2, R><<<grid, kBlk, 0, c->s>>>(vv, gf, of_, xf, bf, bc, xc);
    else k_mac_resid_restrict<3, R><<<grid, kBlk, 0, c->s>>>(vv, gf, of_, xf, bf, bc, xc);
}

__global__ void k_mac_dense(GridD g, int N, const double* __restrict__ E, double* __restrict__ A)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (row >= N) return;
    const int i = row % g.n[0], j = (row / g.n[0]) % g.n[1], k = row / (g.n[0] * g.n[1]);
    A[(long)row * N + col] = g.dim == 2 ? mac_lap_at<2, double>(g, E + (long)col * N, i, j, k)
                                        : mac_lap_at<3, double>(g, E + (long)col * N, i, j, k);
}

void launch_mac_dense(Ctx* c, const GridD& g, int N, const double* E, double* A)
{
    k_mac_dense<<<dim3((N + 255) / 256, N), 256, 0, c->s>>>(g, N, E, A);
}

// ---------------------------------------------------------------------------
// cell prolongation x_f += P e_c: (bi/tri)linear, 3/4 - 1/4 per axis; a coarse
// neighbour beyond a wall takes the homogeneous ghost value wall_sign * e.
// ---------------------------------------------------------------------------

// One thread per coarse cell: the 3^d coarse neighbourhood is read once
// and the 2^d children are corrected (each child's sum in the same order
// as a per-child evaluation: the 2^d nearest coarse cells, axis weights 3/4
// and 1/4).  The block's launch covers the coarse cells of the cavities
// that smooth on the fine level.
template <int DIM, typename R>
__global__ void __launch_bounds__(256) k_prolong_cells(BV v, const GridD* __restrict__ gct, const long* __restrict__ oct, int ncomp,
                                R wall_sign, const R* __restrict__ ea, R* __restrict__ xa)
{
    PT_ENTER(K);
    const GridD& gf = g;
    const GridD gc = bv_g2(v, gct, cav);
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I >= gc.n[0] || J >= gc.n[1] || K >= gc.n[2]) return;
    constexpr int d = DIM;   // every loop below unrolls, so the neighbourhood stays in registers
    const int C[3] = {I, J, K};
    // per axis: source index and sign of the coarse neighbour at offset -1, 0, +1
    int src[3][3];
    R sgn[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            int J2 = C[a] + o - 1;
            R sg = 1;
            if (a < d && (J2 < 0 || J2 >= gc.n[a])) {
                if (gc.per[a]) J2 = J2 < 0 ? J2 + gc.n[a] : J2 - gc.n[a];
                else { J2 = C[a]; sg = wall_sign; }
            }
            if (a >= d) J2 = 0;
            src[a][o] = J2;
            sgn[a][o] = sg;
        }
    const R* e0 = ea + ncomp * bv_o2(v, oct, cav);
    R* x0 = xa + ncomp * bv_o(v, cav);
    const long Nf = ncells(gf), Nc = ncells(gc);
    constexpr int nz = d == 3 ? 2 : 1;
    for (int q = 0; q < ncomp; ++q) {
        const R* e = e0 + q * Nc;
        R* x = x0 + q * Nf;
        R nb[3][3][3];
#pragma unroll
        for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy)
#pragma unroll
                for (int ox = 0; ox < 3; ++ox)
                    if (d == 3 || oz == 1) nb[oz][oy][ox] = e[cid(gc, src[0][ox], src[1][oy], src[2][oz])];
#pragma unroll
        for (int cz = 0; cz < nz; ++cz)
#pragma unroll
            for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                for (int cx = 0; cx < 2; ++cx) {
                    const int ch[3] = {cx, cy, cz};
                    R s = 0;
#pragma unroll
                    for (int bits = 0; bits < (1 << d); ++bits) {
                        int o[3] = {1, 1, 1};
                        R w = 1, sg = 1;
#pragma unroll
                        for (int a = 0; a < d; ++a) {
                            if (!((bits >> a) & 1)) { w *= R(0.75); continue; }
                            w *= R(0.25);
                            o[a] = ch[a] ? 2 : 0;   // the neighbour on the child's side
                            sg *= sgn[a][o[a]];
                        }
                        s += w * sg * nb[o[2]][o[1]][o[0]];
                    }
                    x[cid(gf, 2 * I + cx, 2 * J + cy, d == 3 ? 2 * K + cz : 0)] += s;
                }
    }
}

// grid over the coarse cells of the cavities that smooth on level L
template <typename R>
void launch_prolong_cells(Ctx* c, const Level& L, const BV& v, const GridD* gc, const long* oc, int ncomp,
                          double wall_sign, const R* e, R* x)
{
    BV vv = v;
    const int ex = (L.gmax.n[0] + 1) / 2, ey = (L.gmax.n[1] + 1) / 2, ez = L.gmax.dim == 3 ? (L.gmax.n[2] + 1) / 2 : 1;
    vv.zb = ez;
    if (L.gmax.dim == 2)
        k_prolong_cells<2, R><<<grid3(ex, ey, vv.zb * c->nb, kBlk), kBlk, 0, c->s>>>(vv, gc, oc, ncomp, (R)wall_sign, e, x);
    else
        k_prolong_cells<3, R><<<grid3(ex, ey, vv.zb * c->nb, kBlk), kBlk, 0, c->s>>>(vv, gc, oc, ncomp, (R)wall_sign, e, x);
}

// ---------------------------------------------------------------------------
// nodal problem: Q1 stiffness K (natural boundary on walls)
// ---------------------------------------------------------------------------

// full weighting R = P^T from the fine residual r_f; coarse iterate zeroed.
// One thread per coarse node; the 3^d fine neighbours (x fastest) are loaded
// first (beyond a wall: an in-range index, masked), then summed in order.
template <int DIM, typename R>
__global__ void k_nodal_restrict(BV v, const GridD* __restrict__ gft, const long* __restrict__ oft,
                                 const R* __restrict__ rfa, R* __restrict__ bca, R* __restrict__ xca)
{
    PT_ENTER(k);
    const GridD& gc = g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nnode(gc, 0) || j >= nnode(gc, 1) || k >= nnode(gc, 2)) return;
    const GridD gf = bv_g2(v, gft, cav);
    const R* rf = rfa + bv_o2(v, oft, cav);
    const int I[3] = {i, j, k};
    constexpr int nt = DIM == 3 ? 27 : 9;
    R val[nt];
    bool okv[nt];
#pragma unroll
    for (int t = 0; t < nt; ++t) {
        int tt = t, p[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int del = tt % 3 - 1;
            tt /= 3;
            int F = 2 * I[a] + del;
            const int nf = nnode(gf, a);
            if (F < 0 || F >= nf) {
                if (gf.per[a]) F = F < 0 ? F + nf : F - nf;
                else { ok = false; F = 0; }
            }
            p[a] = F;
        }
        okv[t] = ok;
        val[t] = rf[nid(gf, p[0], p[1], p[2])];
    }
    R s = 0;
#pragma unroll
    for (int t = 0; t < nt; ++t) {
        int tt = t;
        R w = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (tt % 3 != 1) w *= R(0.5);
            tt /= 3;
        }
        s = okv[t] ? s + w * val[t] : s;
    }
    const long q = bv_o(v, cav) + nid(gc, i, j, k);
    bca[q] = s;
    xca[q] = R(0);
}

template <typename R>
void launch_nodal_restrict(Ctx* c, const Level& C, const BV& vc, const GridD* gf, const long* of_, const R* rf, R* bc,
                           R* xc)
{
    BV vv = vc;
    vv.zb = nnode(C.gmax, 2);
    const dim3 grid = grid3(nnode(C.gmax, 0), nnode(C.gmax, 1), vv.zb * c->nb, kBlk);
    if (C.gmax.dim == 2) k_nodal_restrict<2, R><<<grid, kBlk, 0, c->s>>>(vv, gf, of_, rf, bc, xc);
    else k_nodal_restrict<3, R><<<grid, kBlk, 0, c->s>>>(vv, gf, of_, rf, bc, xc);
}

// x_f += P e_c, P the (bi/tri)linear nodal interpolation: a fine node takes
// the mean of the coarse nodes of its coarse edge, face or cell.  One thread
// per fine node; the 2^d candidate coarse nodes are loaded first, then
// summed in order.
template <int DIM, typename R>
__global__ void k_nodal_prolong(BV v, const GridD* __restrict__ gct, const long* __restrict__ oct,
                                const R* __restrict__ ea, R* __restrict__ xa)
{
    PT_ENTER(k);
    const GridD& gf = g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nnode(gf, 0) || j >= nnode(gf, 1) || k >= nnode(gf, 2)) return;
    const GridD gc = bv_g2(v, gct, cav);
    const R* e = ea + bv_o2(v, oct, cav);
    const int F[3] = {i, j, k};
    constexpr int nt = 1 << DIM;
    R val[nt], wv[nt];
    bool okv[nt];
#pragma unroll
    for (int bits = 0; bits < nt; ++bits) {
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
                if (gc.per[a] && C == nnode(gc, a)) C = 0;
                p[a] = C;
            }
        }
        okv[bits] = ok;
        wv[bits] = w;
        val[bits] = e[nid(gc, p[0], p[1], p[2])];
    }
    R s = 0;
#pragma unroll
    for (int bits = 0; bits < nt; ++bits) s = okv[bits] ? s + wv[bits] * val[bits] : s;
    xa[bv_o(v, cav) + nid(gf, i, j, k)] += s;
}

template <typename R>
void launch_nodal_prolong(Ctx* c, const Level& L, const BV& v, const GridD* gc, const long* oc, const R* e, R* x)
{
    BV vv = v;
    vv.zb = nnode(L.gmax, 2);
    const dim3 grid = grid3(nnode(L.gmax, 0), nnode(L.gmax, 1), vv.zb * c->nb, kBlk);
    if (L.gmax.dim == 2) k_nodal_prolong<2, R><<<grid, kBlk, 0, c->s>>>(vv, gc, oc, e, x);
    else k_nodal_prolong<3, R><<<grid, kBlk, 0, c->s>>>(vv, gc, oc, e, x);
}

// ---------------------------------------------------------------------------
// dense coarsest level: A + 1 1^T / N for the singular problems, LU with
// partial pivoting in one workgroup, then the explicit inverse
// ---------------------------------------------------------------------------

__global__ void k_add_ones(int N, double* A)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (long)N * N) A[t] += 1.0 / (double)N;
}

void launch_add_ones(Ctx* c, int N, double* A)
{
    const long n = (long)N * N;
    k_add_ones<<<(unsigned)((n + 255) / 256), 256, 0, c->s>>>(N, A);
}

__global__ void __launch_bounds__(256) k_lu_factor(int N, double* __restrict__ A, int* __restrict__ piv)
{
    __shared__ int sp;
    for (int k = 0; k < N; ++k) {
        if (threadIdx.x == 0) {
            int p = k;
            double best = fabs(A[(long)k * N + k]);
            for (int i = k + 1; i < N; ++i) {
                const double v = fabs(A[(long)i * N + k]);
                if (v > best) { best = v; p = i; }
            }
            piv[k] = p;
            sp = p;
        }
        __syncthreads();
        const int p = sp;
        if (p != k)
            for (int jj = threadIdx.x; jj < N; jj += blockDim.x) {
                const double t = A[(long)k * N + jj];
                A[(long)k * N + jj] = A[(long)p * N + jj];
                A[(long)p * N + jj] = t;
            }
        __syncthreads();
        const double akk = A[(long)k * N + k];
        for (int i = k + 1 + threadIdx.x; i < N; i += blockDim.x) {
            const double f = A[(long)i * N + k] / akk;
            A[(long)i * N + k] = f;
            for (int jj = k + 1; jj < N; ++jj) A[(long)i * N + jj] -= f * A[(long)k * N + jj];
        }
        __syncthreads();
    }
}

void launch_lu_factor(Ctx* c, int N, double* A, int* piv)
{
    k_lu_factor<<<1, 256, 0, c->s>>>(N, A, piv);
}

// column j of A^{-1} from the LU factors (thread j: permutation, forward
// and back substitution of e_j), so the coarsest solve of every V-cycle is a
// parallel matrix-vector product
__global__ void k_lu_inverse(int N, const double* __restrict__ LU, const int* __restrict__ piv, double* __restrict__ Ainv)
{
    const int jcol = blockIdx.x * blockDim.x + threadIdx.x;
    if (jcol >= N) return;
    // work in the output column (stride N): Ainv[i * N + jcol]
    double* y = Ainv + jcol;
    for (int i = 0; i < N; ++i) y[(long)i * N] = (i == jcol) ? 1.0 : 0.0;
    for (int k = 0; k < N; ++k) {
        const int p = piv[k];
        if (p != k) {
            const double t = y[(long)k * N];
            y[(long)k * N] = y[(long)p * N];
            y[(long)p * N] = t;
        }
    }
    for (int i = 0; i < N; ++i) {
        double v = y[(long)i * N];
        for (int jj = 0; jj < i; ++jj) v -= LU[(long)i * N + jj] * y[(long)jj * N];
        y[(long)i * N] = v;
    }
    for (int i = N - 1; i >= 0; --i) {
        double v = y[(long)i * N];
        for (int jj = i + 1; jj < N; ++jj) v -= LU[(long)i * N + jj] * y[(long)jj * N];
        y[(long)i * N] = v / LU[(long)i * N + i];
    }
}

void launch_lu_inverse(Ctx* c, int N, const double* LU, const int* piv, double* Ainv)
{
    k_lu_inverse<<<(N + 63) / 64, 64, 0, c->s>>>(N, LU, piv, Ainv);
}

// Inverse of a dense N x N matrix, N <= kDenseMax, whose symmetric part is
// positive definite (the coarsest tensor viscous operator I - dt
// div(eta (grad u + grad u^T)), slightly unsymmetric at walls), by one
// workgroup: Gauss-Jordan elimination in place, without pivoting, which such
// matrices do not need.  The matrix lives in registers: thread t holds
// column t % 128 of rows 16 (t / 128) + m, m = 0..15 (contiguous, so the
// pivot column's entries a thread needs are read from LDS in wide loads).  Step k passes column k
// and row k through LDS (double-buffered by the parity of k, so one barrier
// per step), every thread forms the scaled pivot row itself, and the update
// of its sixteen elements touches registers only.
constexpr int kGJThreads = 1024, kGJCols = 128, kGJRows = kGJThreads / kGJCols;
constexpr int kGJPer = kDenseMax / kGJRows;
static_assert(kGJCols >= kDenseMax && kGJPer * kGJRows == kDenseMax, "register layout covers the largest system");

__global__ void __launch_bounds__(kGJThreads) k_gj_inverse(const CoarseD* __restrict__ cs, const double* __restrict__ Aa,
                                                           double* __restrict__ Ainva)
{
    // one workgroup per cavity; larger systems take the LU path
    const CoarseD cd = cs[blockIdx.x];
    const int N = cd.N;
    if (N > kDenseMax) return;
    const double* __restrict__ A = Aa + cd.aoff;
    double* __restrict__ Ainv = Ainva + cd.aoff;
    __shared__ double ck[2][kDenseMax];   // column k before step k
    __shared__ double rw[2][kDenseMax];   // row k before step k
    // a wave's 64 lanes share their row group (128 threads per group), so
    // the group index is a scalar
    const int tid = threadIdx.x, j = tid % kGJCols, rg = __builtin_amdgcn_readfirstlane(tid / kGJCols);
    // rows and columns from N to kDenseMax - 1 hold zeros and stay zero
    // (their pivot-column and pivot-row entries are zero), so every thread
    // runs the same branch-free update
    double v[kGJPer];
#pragma unroll
    for (int m = 0; m < kGJPer; ++m) {
        const int i = kGJPer * rg + m;
        v[m] = (j < N && i < N) ? A[(long)i * N + j] : 0.0;
    }
    for (int k = 0; k < N; ++k) {
        double* cc = ck[k & 1];
        double* rr = rw[k & 1];
        if (j == k)
#pragma unroll
            for (int m = 0; m < kGJPer; ++m) cc[kGJPer * rg + m] = v[m];
        if (rg == k / kGJPer) {
            double a = 0.0;
#pragma unroll
            for (int m = 0; m < kGJPer; ++m)
                if (m == k % kGJPer) a = v[m];
            rr[j] = a;
        }
        __syncthreads();
        const double d = 1.0 / cc[k];
        const double r = (j == k ? 1.0 : rr[j]) * d;
        // only the wave whose 64 columns hold column k needs the pivot
        // column's select; every other wave runs the plain update
        if (((tid % kGJCols) >> 6) == (k >> 6)) {
            const bool pc = j == k;
#pragma unroll
            for (int m = 0; m < kGJPer; ++m) v[m] = (pc ? 0.0 : v[m]) - cc[kGJPer * rg + m] * r;
        } else {
#pragma unroll
            for (int m = 0; m < kGJPer; ++m) v[m] = v[m] - cc[kGJPer * rg + m] * r;
        }
        // row k (held by one row group, element k % kGJPer) becomes the
        // scaled pivot row
        if (rg == k / kGJPer) {
            const int mk = k % kGJPer;
#pragma unroll
            for (int m = 0; m < kGJPer; ++m)
                if (m == mk) v[m] = r;
        }
    }
    if (j < N)
#pragma unroll
        for (int m = 0; m < kGJPer; ++m) {
            const int i = kGJPer * rg + m;
            if (i < N) Ainv[(long)i * N + j] = v[m];
        }
}

// explicit inverse of a dense coarsest matrix by LU with partial pivoting
// (A is overwritten by its factors)
void launch_dense_inverse(Ctx* c, int N, double* A, int* piv, double* Ainv)
{
    launch_lu_factor(c, N, A, piv);
    launch_lu_inverse(c, N, A, piv, Ainv);
}

// explicit inverses of the tensor problem's coarsest matrices of every
// cavity (positive definite symmetric part): one workgroup per cavity in
// registers, LU for the few systems above kDenseMax
void launch_gj_inverse_batch(Ctx* c, const MG& m)
{
    k_gj_inverse<<<c->nb, kGJThreads, 0, c->s>>>(m.cs, m.A, m.Ainv);
    for (int b = 0; b < c->nb; ++b) {
        const CoarseD& d = m.hcs[b];
        if (d.N > kDenseMax) {
            launch_lu_factor(c, d.N, m.A + d.aoff, m.piv + d.poff);
            launch_lu_inverse(c, d.N, m.A + d.aoff, m.piv + d.poff, m.Ainv + d.aoff);
        }
    }
}

// x = A^{-1} b for the cavities whose coarsest level is lev; one row per
// thread (block y = cavity), accumulated in FP64
template <typename R>
__global__ void k_coarse_solve(const CoarseD* __restrict__ cs, int lev, const int* __restrict__ act,
                               const double* __restrict__ Ainv, const R* __restrict__ b, R* __restrict__ x)
{
    const int cav = blockIdx.y;
    if (act && !act[cav]) return;
    const CoarseD d = cs[cav];
    if (d.lev != lev) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.N) return;
    const double* row = Ainv + d.aoff + (long)i * d.N;
    const R* bb = b + d.xoff;
    double s = 0.0;
    for (int jj = 0; jj < d.N; ++jj) s += row[jj] * (double)bb[jj];
    x[d.xoff + i] = (R)s;
}

template <typename R>
void launch_coarse_solve(Ctx* c, const MG& m, int lev, const int* act, const R* b, R* x)
{
    k_coarse_solve<R><<<dim3((m.ncmax + 255) / 256, c->nb), 256, 0, c->s>>>(m.cs, lev, act, m.Ainv, b, x);
}

__global__ void k_identity(int N, double* E)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)N * N) return;
    E[t] = (t / N == t % N) ? 1.0 : 0.0;
}

void launch_identity(Ctx* c, int N, double* E)
{
    const long nn = (long)N * N;
    k_identity<<<(unsigned)((nn + 255) / 256), 256, 0, c->s>>>(N, E);
}

#define HB_MG_INST(R)                                                                                          \
    template void launch_mac_rb<R>(Ctx*, const Level&, const BV&, int, R*, const R*);                          \
    template void launch_mac_resid_restrict<R>(Ctx*, const Level&, const BV&, const GridD*, const long*,       \
                                               const R*, const R*, R*, R*);                                    \
    template void launch_prolong_cells<R>(Ctx*, const Level&, const BV&, const GridD*, const long*, int, double, \
                                          const R*, R*);                                                       \
    template void launch_nodal_restrict<R>(Ctx*, const Level&, const BV&, const GridD*, const long*, const R*, \
                                           R*, R*);                                                            \
    template void launch_nodal_prolong<R>(Ctx*, const Level&, const BV&, const GridD*, const long*, const R*, R*); \
    template void launch_coarse_solve<R>(Ctx*, const MG&, int, const int*, const R*, R*);
HB_MG_INST(double)
HB_MG_INST(float)
#undef HB_MG_INST

}  // namespace hb
