// hb_mg.hip -- multigrid kernels of the cell-centred scalar (MAC) problem
// and the nodal Q1 projection problem, cell prolongation shared with the
// tensor problem, and the dense LU of the coarsest level.  gfx950, FP64.
#include "hb_internal.h"
#include "hb_ops.h"

namespace hb {

static const dim3 kBlk(64, 4, 1);

// ---------------------------------------------------------------------------
// MAC problem: L_mac = D_mac G_mac, zero flux through wall faces
// ---------------------------------------------------------------------------

__global__ void k_mac_rb(GridD g, int colour, double* __restrict__ x, const double* __restrict__ b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    const int i = 2 * t + ((j + k + colour) & 1);
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long q = cid(g, i, j, k);
    const double ih2 = 1.0 / (g.h * g.h);
    double Lx = 0.0;
    int cnt = 0;
    for (int a = 0; a < g.dim; ++a)
        for (int side = 0; side < 2; ++side) {
            int p[3] = {i, j, k};
            p[a] += side ? 1 : -1;
            if (!wrap(g, p)) continue;
            Lx += (x[cid(g, p[0], p[1], p[2])] - x[q]) * ih2;
            ++cnt;
        }
    const double dg = -(double)cnt * ih2;
    x[q] += (b[q] - Lx) / dg;
}

void launch_mac_rb(Ctx* c, const Level& l, int colour)
{
    k_mac_rb<<<grid3((l.g.n[0] + 1) / 2, l.g.n[1], l.g.n[2], kBlk), kBlk, 0, c->s>>>(l.g, colour, l.X(), l.b);
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
        const double rv = b[q] - mac_lap_at(g, x, i, j, k);
        if (r) r[q] = rv;
        m = abits(rv);
    }
    if (mx) {
        m = block_umax(m, sh);
        if (threadIdx.x + threadIdx.y == 0) atomic_max_bits(mx, m);
    }
}

void launch_mac_resid(Ctx* c, const Level& l, const double* x, const double* b, double* r, int slot)
{
    k_mac_resid<<<grid3(l.g.n[0], l.g.n[1], l.g.n[2], kBlk), kBlk, 0, c->s>>>(l.g, x, b, r, slot >= 0 ? c->sc + slot : nullptr);
}

__global__ void k_mac_apply(GridD g, const double* __restrict__ x, double* __restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    y[cid(g, i, j, k)] = mac_lap_at(g, x, i, j, k);
}

void launch_mac_apply(Ctx* c, const Level& l, const double* x, double* y)
{
    k_mac_apply<<<grid3(l.g.n[0], l.g.n[1], l.g.n[2], kBlk), kBlk, 0, c->s>>>(l.g, x, y);
}

__global__ void k_mac_resid_restrict(GridD gf, GridD gc, const double* __restrict__ xf, const double* __restrict__ bf,
                                     double* __restrict__ bc, double* __restrict__ xc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= gc.n[0] || j >= gc.n[1]) return;
    const int nch = 1 << gf.dim;
    double s = 0.0;
    for (int bits = 0; bits < nch; ++bits) {
        const int fi = 2 * i + (bits & 1), fj = 2 * j + ((bits >> 1) & 1), fk = gf.dim == 3 ? 2 * k + ((bits >> 2) & 1) : 0;
        s += bf[cid(gf, fi, fj, fk)] - mac_lap_at(gf, xf, fi, fj, fk);
    }
    const long qc = cid(gc, i, j, k);
    bc[qc] = s / (double)nch;
    xc[qc] = 0.0;
}

void launch_mac_resid_restrict(Ctx* c, const Level& f, const Level& cl)
{
    k_mac_resid_restrict<<<grid3(cl.g.n[0], cl.g.n[1], cl.g.n[2], kBlk), kBlk, 0, c->s>>>(f.g, cl.g, f.X(), f.b, cl.b, cl.X());
}

__global__ void k_mac_dense(GridD g, int N, const double* __restrict__ E, double* __restrict__ A)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (row >= N) return;
    const int i = row % g.n[0], j = (row / g.n[0]) % g.n[1], k = row / (g.n[0] * g.n[1]);
    A[(long)row * N + col] = mac_lap_at(g, E + (long)col * N, i, j, k);
}

void launch_mac_dense(Ctx* c, const Level& l, int N, double* E, double* A)
{
    k_mac_dense<<<dim3((N + 255) / 256, N), 256, 0, c->s>>>(l.g, N, E, A);
}

// ---------------------------------------------------------------------------
// cell prolongation x_f += P e_c: (bi/tri)linear, 3/4 - 1/4 per axis; a coarse
// neighbour beyond a wall takes the homogeneous ghost value wall_sign * e
// ---------------------------------------------------------------------------

__global__ void k_prolong_cells(GridD gf, GridD gc, int ncomp, double wall_sign, const double* __restrict__ e,
                                double* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= gf.n[0] || j >= gf.n[1]) return;
    const int d = gf.dim;
    const int fi[3] = {i, j, k};
    const long Nf = ncells(gf), Nc = ncells(gc);
    for (int q = 0; q < ncomp; ++q) {
        double s = 0.0;
        for (int bits = 0; bits < (1 << d); ++bits) {
            int p[3] = {0, 0, 0};
            double w = 1.0, sg = 1.0;
            for (int a = 0; a < d; ++a) {
                const int I = fi[a] >> 1;
                if (!((bits >> a) & 1)) { p[a] = I; w *= 0.75; continue; }
                int J = (fi[a] & 1) ? I + 1 : I - 1;
                w *= 0.25;
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

void launch_prolong_cells(Ctx* c, const Level& f, const Level& cl, int ncomp, double wall_sign)
{
    k_prolong_cells<<<grid3(f.g.n[0], f.g.n[1], f.g.n[2], kBlk), kBlk, 0, c->s>>>(f.g, cl.g, ncomp, wall_sign, cl.X(), f.X());
}

// ---------------------------------------------------------------------------
// nodal problem: Q1 stiffness K (natural boundary on walls)
// ---------------------------------------------------------------------------

// full weighting R = P^T from the fine residual r_f; coarse iterate zeroed
__global__ void k_nodal_restrict(GridD gf, GridD gc, const double* __restrict__ rf, double* __restrict__ bc,
                                 double* __restrict__ xc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nnode(gc, 0) || j >= nnode(gc, 1)) return;
    const int d = gf.dim;
    const int I[3] = {i, j, k};
    int nt = 1;
    for (int a = 0; a < d; ++a) nt *= 3;
    double s = 0.0;
    for (int t = 0; t < nt; ++t) {
        int tt = t, p[3] = {0, 0, 0};
        double w = 1.0;
        bool ok = true;
        for (int a = 0; a < d; ++a) {
            const int del = tt % 3 - 1;
            tt /= 3;
            if (del != 0) w *= 0.5;
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
    xc[q] = 0.0;
}

void launch_nodal_restrict(Ctx* c, const Level& f, const Level& cl)
{
    const GridD& g = cl.g;
    k_nodal_restrict<<<grid3(nnode(g, 0), nnode(g, 1), nnode(g, 2), kBlk), kBlk, 0, c->s>>>(f.g, g, f.r, cl.b, cl.X());
}

// (bi/tri)linear nodal prolongation x_f += P e_c
__global__ void k_nodal_prolong(GridD gf, GridD gc, const double* __restrict__ e, double* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nnode(gf, 0) || j >= nnode(gf, 1)) return;
    const int d = gf.dim;
    const int F[3] = {i, j, k};
    double s = 0.0;
    for (int bits = 0; bits < (1 << d); ++bits) {
        int p[3] = {0, 0, 0};
        double w = 1.0;
        bool ok = true;
        for (int a = 0; a < d; ++a) {
            const int hi = (bits >> a) & 1;
            if (!(F[a] & 1)) {
                if (hi) { ok = false; break; }
                p[a] = F[a] >> 1;
            } else {
                w *= 0.5;
                int C = ((F[a] - 1) >> 1) + hi;
                if (gc.per[a] && C == nnode(gc, a)) C = 0;
                p[a] = C;
            }
        }
        if (ok) s += w * e[nid(gc, p[0], p[1], p[2])];
    }
    x[nid(gf, i, j, k)] += s;
}

void launch_nodal_prolong(Ctx* c, const Level& f, const Level& cl)
{
    const GridD& g = f.g;
    k_nodal_prolong<<<grid3(nnode(g, 0), nnode(g, 1), nnode(g, 2), kBlk), kBlk, 0, c->s>>>(g, cl.g, cl.X(), f.X());
}

// ---------------------------------------------------------------------------
// dense coarsest level: A + 1 1^T / N for the singular problems, LU with
// partial pivoting in one workgroup, triangular solves in one thread
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

__global__ void k_lu_solve(int N, const double* __restrict__ A, const int* __restrict__ piv, const double* __restrict__ b,
                           double* __restrict__ x)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < N; ++i) x[i] = b[i];
    for (int k = 0; k < N; ++k) {
        const int p = piv[k];
        if (p != k) { const double t = x[k]; x[k] = x[p]; x[p] = t; }
    }
    for (int i = 0; i < N; ++i)
        for (int jj = 0; jj < i; ++jj) x[i] -= A[(long)i * N + jj] * x[jj];
    for (int i = N - 1; i >= 0; --i) {
        for (int jj = i + 1; jj < N; ++jj) x[i] -= A[(long)i * N + jj] * x[jj];
        x[i] /= A[(long)i * N + i];
    }
}

void launch_lu_solve(Ctx* c, int N, const double* A, const int* piv, const double* b, double* x)
{
    k_lu_solve<<<1, 64, 0, c->s>>>(N, A, piv, b, x);
}

}  // namespace hb
