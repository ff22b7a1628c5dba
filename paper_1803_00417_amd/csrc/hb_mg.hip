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

template <typename R>
__global__ void k_mac_rb(GridD g, int colour, R* __restrict__ x, const R* __restrict__ b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    const int i = 2 * t + ((j + k + colour) & 1);
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long q = cid(g, i, j, k);
    const R h = (R)g.h;
    const R ih2 = R(1) / (h * h);
    R Lx = 0;
    int cnt = 0;
    for (int a = 0; a < g.dim; ++a)
        for (int side = 0; side < 2; ++side) {
            int p[3] = {i, j, k};
            p[a] += side ? 1 : -1;
            if (!wrap(g, p)) continue;
            Lx += (x[cid(g, p[0], p[1], p[2])] - x[q]) * ih2;
            ++cnt;
        }
    const R dg = -(R)cnt * ih2;
    x[q] += (b[q] - Lx) / dg;
}

template <typename R>
void launch_mac_rb(Ctx* c, const GridD& g, int colour, R* x, const R* b)
{
    k_mac_rb<R><<<grid3((g.n[0] + 1) / 2, g.n[1], g.n[2], kBlk), kBlk, 0, c->s>>>(g, colour, x, b);
}

__global__ void k_mac_resid(GridD g, const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ r,
                            double* __restrict__ mx)
{
    __shared__ unsigned long long sh[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    unsigned long long m = 0ull;
    if (i < g.n[0] && j < g.n[1]) {
        const long q = cid(g, i, j, k);
        const double rv = b[q] - mac_lap_at<double>(g, x, i, j, k);
        if (r) r[q] = rv;
        m = abits(rv);
    }
    if (mx) {
        m = block_umax(m, sh);
        if (threadIdx.x + threadIdx.y == 0) atomic_max_bits(mx, m);
    }
}

void launch_mac_resid(Ctx* c, const GridD& g, const double* x, const double* b, double* r, int slot)
{
    k_mac_resid<<<grid3(g.n[0], g.n[1], g.n[2], kBlk), kBlk, 0, c->s>>>(g, x, b, r, slot >= 0 ? c->sc + slot : nullptr);
}

__global__ void k_mac_apply(GridD g, const double* __restrict__ x, double* __restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    y[cid(g, i, j, k)] = mac_lap_at<double>(g, x, i, j, k);
}

void launch_mac_apply(Ctx* c, const GridD& g, const double* x, double* y)
{
    k_mac_apply<<<grid3(g.n[0], g.n[1], g.n[2], kBlk), kBlk, 0, c->s>>>(g, x, y);
}

template <typename R>
__global__ void k_mac_resid_restrict(GridD gf, GridD gc, const R* __restrict__ xf, const R* __restrict__ bf,
                                     R* __restrict__ bc, R* __restrict__ xc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= gc.n[0] || j >= gc.n[1]) return;
    const int nch = 1 << gf.dim;
    R s = 0;
    for (int bits = 0; bits < nch; ++bits) {
        const int fi = 2 * i + (bits & 1), fj = 2 * j + ((bits >> 1) & 1), fk = gf.dim == 3 ? 2 * k + ((bits >> 2) & 1) : 0;
        s += bf[cid(gf, fi, fj, fk)] - mac_lap_at<R>(gf, xf, fi, fj, fk);
    }
    const long qc = cid(gc, i, j, k);
    bc[qc] = s / (R)nch;
    xc[qc] = R(0);
}

template <typename R>
void launch_mac_resid_restrict(Ctx* c, const GridD& gf, const GridD& gc, const R* xf, const R* bf, R* bc, R* xc)
{
    k_mac_resid_restrict<R><<<grid3(gc.n[0], gc.n[1], gc.n[2], kBlk), kBlk, 0, c->s>>>(gf, gc, xf, bf, bc, xc);
}

__global__ void k_mac_dense(GridD g, int N, const double* __restrict__ E, double* __restrict__ A)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (row >= N) return;
    const int i = row % g.n[0], j = (row / g.n[0]) % g.n[1], k = row / (g.n[0] * g.n[1]);
    A[(long)row * N + col] = mac_lap_at<double>(g, E + (long)col * N, i, j, k);
}

void launch_mac_dense(Ctx* c, const Level& l, int N, double* E, double* A)
{
    k_mac_dense<<<dim3((N + 255) / 256, N), 256, 0, c->s>>>(l.g, N, E, A);
}

// ---------------------------------------------------------------------------
// cell prolongation x_f += P e_c: (bi/tri)linear, 3/4 - 1/4 per axis; a coarse
// neighbour beyond a wall takes the homogeneous ghost value wall_sign * e
// ---------------------------------------------------------------------------

template <typename R>
__global__ void k_prolong_cells(GridD gf, GridD gc, int ncomp, R wall_sign, const R* __restrict__ e, R* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= gf.n[0] || j >= gf.n[1]) return;
    const int d = gf.dim;
    const int fi[3] = {i, j, k};
    const long Nf = ncells(gf), Nc = ncells(gc);
    for (int q = 0; q < ncomp; ++q) {
        R s = 0;
        for (int bits = 0; bits < (1 << d); ++bits) {
            int p[3] = {0, 0, 0};
            R w = 1, sg = 1;
            for (int a = 0; a < d; ++a) {
                const int I = fi[a] >> 1;
                if (!((bits >> a) & 1)) { p[a] = I; w *= R(0.75); continue; }
                int J = (fi[a] & 1) ? I + 1 : I - 1;
                w *= R(0.25);
                if (J < 0 || J >= gc.n[a]) {
                    if (gc.per[a]) J = J < 0 ? J + gc.n[a] : J - gc.n[a];
                    else { J = I; sg *= wall_sign; }
                }
                p[a] = J;
            }
            s += w * sg * e[q * Nc + cid(gc, p[0], p[1], p[2])];
        }
        x[q * Nf + cid(gf, i, j, k)] += s;
    }
}

template <typename R>
void launch_prolong_cells(Ctx* c, const GridD& gf, const GridD& gc, int ncomp, double wall_sign, const R* e, R* x)
{
    k_prolong_cells<R><<<grid3(gf.n[0], gf.n[1], gf.n[2], kBlk), kBlk, 0, c->s>>>(gf, gc, ncomp, (R)wall_sign, e, x);
}

// ---------------------------------------------------------------------------
// nodal problem: Q1 stiffness K (natural boundary on walls)
// ---------------------------------------------------------------------------

// full weighting R = P^T from the fine residual r_f; coarse iterate zeroed
template <typename R>
__global__ void k_nodal_restrict(GridD gf, GridD gc, const R* __restrict__ rf, R* __restrict__ bc, R* __restrict__ xc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nnode(gc, 0) || j >= nnode(gc, 1)) return;
    const int d = gf.dim;
    const int I[3] = {i, j, k};
    int nt = 1;
    for (int a = 0; a < d; ++a) nt *= 3;
    R s = 0;
    for (int t = 0; t < nt; ++t) {
        int tt = t, p[3] = {0, 0, 0};
        R w = 1;
        bool ok = true;
        for (int a = 0; a < d; ++a) {
            const int del = tt % 3 - 1;
            tt /= 3;
            if (del != 0) w *= R(0.5);
            int F = 2 * I[a] + del;
            const int nf = nnode(gf, a);
            if (F < 0 || F >= nf) {
                if (gf.per[a]) F = F < 0 ? F + nf : F - nf;
                else ok = false;
            }
            p[a] = F;
        }
        if (ok) s += w * rf[nid(gf, p[0], p[1], p[2])];
    }
    const long q = nid(gc, i, j, k);
    bc[q] = s;
    xc[q] = R(0);
}

template <typename R>
void launch_nodal_restrict(Ctx* c, const GridD& gf, const GridD& gc, const R* rf, R* bc, R* xc)
{
    k_nodal_restrict<R><<<grid3(nnode(gc, 0), nnode(gc, 1), nnode(gc, 2), kBlk), kBlk, 0, c->s>>>(gf, gc, rf, bc, xc);
}

// (bi/tri)linear nodal prolongation x_f += P e_c
template <typename R>
__global__ void k_nodal_prolong(GridD gf, GridD gc, const R* __restrict__ e, R* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nnode(gf, 0) || j >= nnode(gf, 1)) return;
    const int d = gf.dim;
    const int F[3] = {i, j, k};
    R s = 0;
    for (int bits = 0; bits < (1 << d); ++bits) {
        int p[3] = {0, 0, 0};
        R w = 1;
        bool ok = true;
        for (int a = 0; a < d; ++a) {
            const int hi = (bits >> a) & 1;
            if (!(F[a] & 1)) {
                if (hi) { ok = false; break; }
                p[a] = F[a] >> 1;
            } else {
                w *= R(0.5);
                int C = ((F[a] - 1) >> 1) + hi;
                if (gc.per[a] && C == nnode(gc, a)) C = 0;
                p[a] = C;
            }
        }
        if (ok) s += w * e[nid(gc, p[0], p[1], p[2])];
    }
    x[nid(gf, i, j, k)] += s;
}

template <typename R>
void launch_nodal_prolong(Ctx* c, const GridD& gf, const GridD& gc, const R* e, R* x)
{
    k_nodal_prolong<R><<<grid3(nnode(gf, 0), nnode(gf, 1), nnode(gf, 2), kBlk), kBlk, 0, c->s>>>(gf, gc, e, x);
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

// x = A^{-1} b, one row per thread, accumulated in FP64
template <typename R>
__global__ void k_coarse_solve(int N, const double* __restrict__ Ainv, const R* __restrict__ b, R* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double* row = Ainv + (long)i * N;
    double s = 0.0;
    for (int jj = 0; jj < N; ++jj) s += row[jj] * (double)b[jj];
    x[i] = (R)s;
}

template <typename R>
void launch_coarse_solve(Ctx* c, int N, const double* Ainv, const R* b, R* x)
{
    k_coarse_solve<R><<<(N + 255) / 256, 256, 0, c->s>>>(N, Ainv, b, x);
}

#define HB_MG_INST(R)                                                                                     \
    template void launch_mac_rb<R>(Ctx*, const GridD&, int, R*, const R*);                                \
    template void launch_mac_resid_restrict<R>(Ctx*, const GridD&, const GridD&, const R*, const R*, R*, R*); \
    template void launch_prolong_cells<R>(Ctx*, const GridD&, const GridD&, int, double, const R*, R*);   \
    template void launch_nodal_restrict<R>(Ctx*, const GridD&, const GridD&, const R*, R*, R*);           \
    template void launch_nodal_prolong<R>(Ctx*, const GridD&, const GridD&, const R*, R*);                \
    template void launch_coarse_solve<R>(Ctx*, int, const double*, const R*, R*);
HB_MG_INST(double)
HB_MG_INST(float)
#undef HB_MG_INST

}  // namespace hb
