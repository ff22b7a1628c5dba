// hb_visc.hip -- regularised viscosity and the coupled tensor viscous
// operator (I - dt div(beta gamma_dot(.))): explicit divergence, wall
// right-hand side, face coefficients and the dense coarsest matrix.  gfx950,
// FP64.  One thread per cell; x is the fastest index, so a wavefront reads 64
// consecutive doubles.  (The multigrid sweeps are the LDS-tiled kernels.)
#include "hb_internal.h"
#include "hb_ops.h"

namespace hb {

static const dim3 kBlk(64, 4, 1);

// ---------------------------------------------------------------------------
// apparent viscosity (Sec. III.B, eq:dimensionless:herschel-bulkley)
// ---------------------------------------------------------------------------

__device__ inline double eta_of_g(const FluidD& fl, double g)
{
    const double x = fl.Pa * g;
    // (1 - e^{-x})/x through expm1: no cancellation for small x, 1 at x = 0
    const double phi = (x == 0.0) ? 1.0 : -expm1(-x) / x;
    if (fl.reg == HB_REG_YIELD_ONLY) return pow(g, fl.n - 1.0) + 0.5 * fl.HB * fl.Pa * phi;
    return (pow(g, fl.n) + 0.5 * fl.HB) * fl.Pa * phi;
}

// g = |gamma_dot| of cell (i, j, k): centred differences with wall ghosts,
// |A| = sqrt(sum A_ij^2 / 2) (Sec. II)
__device__ inline double strain_norm_at(const GridD& g, const double* __restrict__ u, int i, int j, int k)
{
    const long N = ncells(g);
    double G[3][3];
    for (int a = 0; a < g.dim; ++a)
        for (int c = 0; c < g.dim; ++c) {
            int p[3] = {i, j, k}, m[3] = {i, j, k};
            p[a] += 1;
            m[a] -= 1;
            const double* q = u + (long)c * N;
            G[a][c] = (cval<false>(g, q, c, p[0], p[1], p[2]) - cval<false>(g, q, c, m[0], m[1], m[2])) / (2.0 * g.h);
        }
    double s = 0.0;
    for (int a = 0; a < g.dim; ++a)
        for (int c = 0; c < g.dim; ++c) {
            const double e = 0.5 * (G[a][c] + G[c][a]);
            s += e * e;
        }
    return sqrt(0.5 * s);
}

__global__ void k_viscosity(GridD g, FluidD fl, const double* __restrict__ u, double* __restrict__ eta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    eta[cid(g, i, j, k)] = eta_of_g(fl, strain_norm_at(g, u, i, j, k));
}

// Yield test (Sec. II, Sec. IV): in the dimensionless variables the stress
// magnitude is 2 eta g and the yield stress HB; a cell is yielded where
// 2 eta g > HB.  mask (nullable): 1 yielded, 0 not.  The number of yielded
// cells is summed into *count (integers, exact in any order) and the largest
// stress magnitude max-reduced into *maxtau.
__global__ void k_yield(GridD g, FluidD fl, const double* __restrict__ u, unsigned char* __restrict__ mask,
                        double* __restrict__ count, double* __restrict__ maxtau)
{
    __shared__ double shs[64];
    __shared__ unsigned long long shm[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    double y = 0.0;
    unsigned long long tb = 0ull;
    if (i < g.n[0] && j < g.n[1]) {
        const double gn = strain_norm_at(g, u, i, j, k);
        const double tau = 2.0 * eta_of_g(fl, gn) * gn;
        const bool yl = tau > fl.HB;
        if (mask) mask[cid(g, i, j, k)] = yl ? 1 : 0;
        y = yl ? 1.0 : 0.0;
        tb = abits(tau);
    }
    y = block_sum(y, shs);
    tb = block_umax(tb, shm);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        if (y != 0.0) atomicAdd(count, y);
        atomic_max_bits(maxtau, tb);
    }
}

void launch_viscosity(Ctx* c, const Cav& v, const double* u, double* eta)
{
    k_viscosity<<<grid3(v.g.n[0], v.g.n[1], v.g.n[2], kBlk), kBlk, 0, c->s>>>(v.g, v.fl, u, eta);
}

void launch_yield(Ctx* c, const Cav& v, const double* u, unsigned char* mask, double* count, double* maxtau)
{
    k_yield<<<grid3(v.g.n[0], v.g.n[1], v.g.n[2], kBlk), kBlk, 0, c->s>>>(v.g, v.fl, u, mask, count, maxtau);
}

// ---------------------------------------------------------------------------
// face viscosity: fine faces from cells, coarse faces from fine faces
// ---------------------------------------------------------------------------

__global__ void k_eta_faces(GridD g, int a, double Re, const double* __restrict__ eta, double* __restrict__ beta)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= fext(g, a, 0) || j >= fext(g, a, 1)) return;
    int R[3] = {i, j, k}, L[3] = {i, j, k};
    L[a] -= 1;
    const bool okL = wrap(g, L), okR = wrap(g, R);
    double v;
    if (okL && okR)
        v = 0.5 * (eta[cid(g, L[0], L[1], L[2])] / Re + eta[cid(g, R[0], R[1], R[2])] / Re);
    else if (okL)
        v = eta[cid(g, L[0], L[1], L[2])] / Re;
    else
        v = eta[cid(g, R[0], R[1], R[2])] / Re;
    beta[foffset(g, a) + fid(g, a, i, j, k)] = v;
}

void launch_eta_faces(Ctx* c, const Cav& v, const GridD& g, const double* eta, double* beta)
{
    for (int a = 0; a < g.dim; ++a)
        k_eta_faces<<<grid3(fext(g, a, 0), fext(g, a, 1), fext(g, a, 2), kBlk), kBlk, 0, c->s>>>(g, a, v.fl.Re, eta, beta);
}

// coarse face = mean of the 2^(d-1) fine faces tiling it
__global__ void k_restrict_faces(GridD gf, GridD gc, int a, const double* __restrict__ bf, double* __restrict__ bc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= fext(gc, a, 0) || j >= fext(gc, a, 1)) return;
    const int I[3] = {i, j, k};
    const double* F = bf + foffset(gf, a);
    double s = 0.0;
    int cnt = 0;
    for (int t = 0; t < (1 << gf.dim); ++t) {
        if ((t >> a) & 1) continue;
        int p[3] = {0, 0, 0};
        for (int b = 0; b < gf.dim; ++b) p[b] = (b == a) ? 2 * I[b] : 2 * I[b] + ((t >> b) & 1);
        s += F[fid(gf, a, p[0], p[1], p[2])];
        ++cnt;
    }
    bc[foffset(gc, a) + fid(gc, a, i, j, k)] = s / (double)cnt;
}

void launch_restrict_faces(Ctx* c, const GridD& gf, const GridD& gc, const double* bf, double* bc)
{
    for (int a = 0; a < gf.dim; ++a)
        k_restrict_faces<<<grid3(fext(gc, a, 0), fext(gc, a, 1), fext(gc, a, 2), kBlk), kBlk, 0, c->s>>>(gf, gc, a, bf, bc);
}

// ---------------------------------------------------------------------------
// tensor flux and divergence
// ---------------------------------------------------------------------------

__global__ void k_visc_div(GridD g, const double* __restrict__ beta, const double* __restrict__ u, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const long N = ncells(g), q = cid(g, i, j, k);
    for (int c = 0; c < g.dim; ++c) out[c * N + q] = visc_div_at<false, false>(g, beta, u, c, i, j, k);
}

void launch_visc_div(Ctx* c, const GridD& g, const double* beta, const double* u, double* out)
{
    k_visc_div<<<grid3(g.n[0], g.n[1], g.n[2], kBlk), kBlk, 0, c->s>>>(g, beta, u, out);
}

// out = rhs + dt div(beta gamma_dot(0 with wall values)): the inhomogeneous
// wall part of the operator moved to the right-hand side.  The stencil of a
// cell reaches one cell along each axis, so only cells in the first layer
// along a wall axis see a wall value; elsewhere the term is zero.  out = rhs
// is copied first, then one thread per boundary-layer cell (block z = wall
// face 2 a + side; a cell on several layers is taken by its lowest axis)
// adds the wall term.
__global__ void k_visc_wall_rhs(GridD g, const double* __restrict__ beta, double dt, const double* __restrict__ rhs,
                                double* __restrict__ out)
{
    const int a = blockIdx.z >> 1, side = blockIdx.z & 1;
    if (a >= g.dim || g.per[a]) return;
    const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
    const int u = blockIdx.x * blockDim.x + threadIdx.x, w = blockIdx.y * blockDim.y + threadIdx.y;
    if (u >= g.n[b0] || w >= g.n[b1]) return;
    int p[3];
    p[a] = side ? g.n[a] - 1 : 0;
    p[b0] = u;
    p[b1] = w;
    for (int b = 0; b < a; ++b)
        if (!g.per[b] && (p[b] == 0 || p[b] == g.n[b] - 1)) return;
    const long N = ncells(g), q = cid(g, p[0], p[1], p[2]);
    for (int c = 0; c < g.dim; ++c)
        out[c * N + q] = rhs[c * N + q] + dt * visc_div_at<false, true>(g, beta, nullptr, c, p[0], p[1], p[2]);
}

void launch_visc_wall_rhs(Ctx* c, const GridD& g, const double* beta, double dt, const double* rhs, double* out)
{
    copy(c, out, rhs, (long)g.dim * ncells(g));
    int e0 = 1, e1 = 1;
    for (int a = 0; a < g.dim; ++a) {
        const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
        e0 = e0 > g.n[b0] ? e0 : g.n[b0];
        e1 = e1 > g.n[b1] ? e1 : g.n[b1];
    }
    k_visc_wall_rhs<<<grid3(e0, e1, 2 * g.dim, kBlk), kBlk, 0, c->s>>>(g, beta, dt, rhs, out);
}

// dense matrix of the homogeneous operator, column j = A e_j (E holds the
// N unit vectors, column-major)
__global__ void k_visc_dense(GridD g, const double* __restrict__ beta, double dt, int N, const double* __restrict__ E,
                             double* __restrict__ A)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (row >= N) return;
    const long Nc = ncells(g);
    const int c = (int)(row / Nc);
    const long q = row % Nc;
    const int i = (int)(q % g.n[0]), j = (int)((q / g.n[0]) % g.n[1]), k = (int)(q / ((long)g.n[0] * g.n[1]));
    const double* x = E + (long)col * N;
    A[(long)row * N + col] = x[row] - dt * visc_div_at<true, false>(g, beta, x, c, i, j, k);
}

void launch_visc_dense(Ctx* c, const GridD& g, const double* beta, double dt, int N, const double* E, double* A)
{
    k_visc_dense<<<dim3((N + 255) / 256, N), 256, 0, c->s>>>(g, beta, dt, N, E, A);
}

// the same for every cavity in one launch (block z = cavity), with the
// cavity's coefficient 2 theta dt from its scalar slot
__global__ void k_visc_dense_batch(const DenseD* __restrict__ dd, const double* __restrict__ sc, double* __restrict__ A)
{
    const int cav = blockIdx.z;
    const DenseD& d = dd[cav];
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (row >= d.N || col >= d.N) return;
    const GridD g = d.g;
    const long Nc = ncells(g);
    const int c = (int)(row / Nc);
    const long q = row % Nc;
    const int i = (int)(q % g.n[0]), j = (int)((q / g.n[0]) % g.n[1]), k = (int)(q / ((long)g.n[0] * g.n[1]));
    const double dt = sc[(long)cav * S_NSLOT + S_DT];
    const double* x = d.E + (long)col * d.N;
    A[d.aoff + (long)row * d.N + col] = x[row] - dt * visc_div_at<true, false>(g, d.beta, x, c, i, j, k);
}

void launch_visc_dense_batch(Ctx* c, const MG& m)
{
    const int n = m.ncmax;
    k_visc_dense_batch<<<dim3((n + 255) / 256, n, c->nb), 256, 0, c->s>>>(m.dd, c->sc, m.A);
}

__global__ void k_eta_over_re(long n, double Re, const double* __restrict__ eta, double* __restrict__ etae)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) etae[i] = eta[i] / Re;
}

void launch_eta_over_re(Ctx* c, const Cav& v, const double* eta, double* etae)
{
    const long n = v.nc;
    k_eta_over_re<<<(unsigned)((n + 255) / 256), 256, 0, c->s>>>(n, v.fl.Re, eta, etae);
}

}  // namespace hb
