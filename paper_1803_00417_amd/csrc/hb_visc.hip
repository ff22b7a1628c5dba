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
template <class GR>
__device__ inline double strain_norm_at(const GR& g, const double* __restrict__ u, int i, int j, int k)
{
    const long N = ncells(g);
    double G[3][3];
#pragma unroll
    for (int a = 0; a < g.dim; ++a)
#pragma unroll
        for (int c = 0; c < g.dim; ++c) {
            int p[3] = {i, j, k}, m[3] = {i, j, k};
            p[a] += 1;
            m[a] -= 1;
            const double* q = u + (long)c * N;
            G[a][c] = (cval<false>(g, q, c, p[0], p[1], p[2]) - cval<false>(g, q, c, m[0], m[1], m[2])) / (2.0 * g.h);
        }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < g.dim; ++a)
#pragma unroll
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

// face (i, j, k) of axis a: the mean of eta/Re of its two cells, or that of
// the interior cell on a wall face (etae: eta/Re per cell, formed by
// k_stage_eta_over_re as eta / Re)
template <class GR>
__device__ __forceinline__ void face_eta(const GR& g, int a, const double* __restrict__ etae,
                                         double* __restrict__ beta, int i, int j, int k)
{
    int R[3] = {i, j, k}, L[3] = {i, j, k};
    L[a] -= 1;
    const bool okL = wrap(g, L), okR = wrap(g, R);
    double v;
    if (okL && okR)
        v = 0.5 * (etae[cid(g, L[0], L[1], L[2])] + etae[cid(g, R[0], R[1], R[2])]);
    else if (okL)
        v = etae[cid(g, L[0], L[1], L[2])];
    else
        v = etae[cid(g, R[0], R[1], R[2])];
    beta[foffset(g, a) + fid(g, a, i, j, k)] = v;
}

// coarse face (i, j, k) of axis a = mean of the 2^(d-1) fine faces tiling it
template <class GR>
__device__ __forceinline__ void restrict_face(const GR& gf, const GR& gc, int a, const double* __restrict__ bf,
                                     double* __restrict__ bc, int i, int j, int k)
{
    const int I[3] = {i, j, k};
    const double* F = bf + foffset(gf, a);
    double s = 0.0;
    int cnt = 0;
#pragma unroll
    for (int t = 0; t < (1 << gf.dim); ++t) {
        if ((t >> a) & 1) continue;
        int p[3] = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < gf.dim; ++b) p[b] = (b == a) ? 2 * I[b] : 2 * I[b] + ((t >> b) & 1);
        s += F[fid(gf, a, p[0], p[1], p[2])];
        ++cnt;
    }
    bc[foffset(gc, a) + fid(gc, a, i, j, k)] = s / (double)cnt;
}

// ---------------------------------------------------------------------------
// tensor flux and divergence
// ---------------------------------------------------------------------------

// out = rhs + dt div(beta gamma_dot(0 with wall values)): the inhomogeneous
// wall part of the operator moved to the right-hand side.  The stencil of a
// cell reaches one cell along each axis, so only cells in the first layer
// along a wall axis see a wall value; elsewhere the term is zero.  out = rhs
// is copied first, then one thread per boundary-layer cell of wall face
// (a, side), at in-face position (u, w), adds the wall term (a cell on
// several layers is taken by its lowest axis).
template <class GR>
__device__ __forceinline__ void visc_wall_at(const GR& g, const double* __restrict__ beta, double dt,
                                    const double* __restrict__ rhs, double* __restrict__ out, int a, int side, int u, int w)
{
    if (a >= g.dim || g.per[a]) return;
    const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
    if (u >= g.n[b0] || w >= g.n[b1]) return;
    int p[3];
    p[a] = side ? g.n[a] - 1 : 0;
    p[b0] = u;
    p[b1] = w;
    for (int b = 0; b < a; ++b)
        if (!g.per[b] && (p[b] == 0 || p[b] == g.n[b] - 1)) return;
    const long N = ncells(g), q = cid(g, p[0], p[1], p[2]);
#pragma unroll
    for (int c = 0; c < g.dim; ++c) {
        out[c * N + q] = rhs[c * N + q] + dt * visc_div_at<false, true>(g, beta, nullptr, c, p[0], p[1], p[2]);
        __builtin_amdgcn_sched_barrier(0);
    }
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
    const GridD& g = d.g;
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

// ---------------------------------------------------------------------------
// the same stages over every cavity in one launch (tables c->ck, c->cio;
// block z = cavity * planes + plane, face loops (cavity * 3 + axis) * planes
// + plane)
// ---------------------------------------------------------------------------

static dim3 cells_of(const Ctx* c) { return dim3((c->cx[0] + kBlk.x - 1) / kBlk.x, (c->cx[1] + kBlk.y - 1) / kBlk.y, c->cx[2] * c->nb); }

// eta = eta(u) of every cavity
template <int DIM>
__global__ void k_stage_viscosity(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int zb)
{
    const int cav = blockIdx.z / zb, k = blockIdx.z - cav * zb;
    const CavK& K = ck[cav];
    const GridS<DIM> g = grid_s<DIM>(K.g);
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return;
    K.eta[cid(g, i, j, k)] = eta_of_g(K.fl, strain_norm_at(g, io[cav].u, i, j, k));
}

void stage_viscosity(Ctx* c)
{
    if (c->dim == 2) k_stage_viscosity<2><<<cells_of(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    else k_stage_viscosity<3><<<cells_of(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
}

// eta/Re at cells and the coefficient slot (the operator's 2 theta dt) of
// every cavity
__global__ void k_stage_eta_over_re(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int zb)
{
    const int cav = blockIdx.z / zb, k = blockIdx.z - cav * zb;
    const CavK& K = ck[cav];
    const CavIO& IO = io[cav];
    const GridD& g = K.g;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i == 0 && j == 0 && k == 0) K.sc[S_DT] = IO.vdt;
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return;
    const long q = cid(g, i, j, k);
    K.etae[q] = IO.eta[q] / K.fl.Re;
}

// level-0 face viscosities of every cavity (after k_stage_eta_over_re)
template <int DIM>
__global__ void k_stage_eta_faces(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int zb)
{
    const int zz = blockIdx.z / zb, k = blockIdx.z - zz * zb;
    const int cav = zz / 3, a = zz - 3 * cav;
    const CavK& K = ck[cav];
    const GridS<DIM> g = grid_s<DIM>(K.g);
    if (a >= g.dim) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= fext(g, a, 0) || j >= fext(g, a, 1) || k >= fext(g, a, 2)) return;
    face_eta(g, a, K.etae, K.beta0, i, j, k);
}

void stage_visc_coef(Ctx* c)
{
    k_stage_eta_over_re<<<cells_of(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    const dim3 fg((c->fx[0] + kBlk.x - 1) / kBlk.x, (c->fx[1] + kBlk.y - 1) / kBlk.y, c->fx[2] * 3 * c->nb);
    if (c->dim == 2) k_stage_eta_faces<2><<<fg, kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
    else k_stage_eta_faces<3><<<fg, kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
}

// face viscosities of level l of every cavity from level l - 1 (entries with
// gc.dim == 0: no such level)
template <int DIM>
__global__ void k_stage_restrict_faces(const RFace* __restrict__ rf, int zb)
{
    const int zz = blockIdx.z / zb, k = blockIdx.z - zz * zb;
    const int cav = zz / 3, a = zz - 3 * cav;
    const RFace& R = rf[cav];
    if (R.gc.dim == 0 || a >= DIM) return;
    const GridS<DIM> gc = grid_s<DIM>(R.gc), gf = grid_s<DIM>(R.gf);
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= fext(gc, a, 0) || j >= fext(gc, a, 1) || k >= fext(gc, a, 2)) return;
    restrict_face(gf, gc, a, R.bf, R.bc, i, j, k);
}

void stage_restrict_faces(Ctx* c, int l)
{
    const int* e = c->rfx[l].data();
    const dim3 fg((e[0] + kBlk.x - 1) / kBlk.x, (e[1] + kBlk.y - 1) / kBlk.y, e[2] * 3 * c->nb);
    if (c->dim == 2) k_stage_restrict_faces<2><<<fg, kBlk, 0, c->s>>>(c->rface + (long)(l - 1) * c->nb, e[2]);
    else k_stage_restrict_faces<3><<<fg, kBlk, 0, c->s>>>(c->rface + (long)(l - 1) * c->nb, e[2]);
}

// E = div(eta_e gamma_dot(u)) of every cavity, level-0 faces (the body
// takes the arrays restrict-qualified: the table says nothing about
// aliasing)
template <class GR>
__device__ __forceinline__ void visc_div_body(const GR& g, const double* __restrict__ beta,
                                              const double* __restrict__ u, double* __restrict__ out, int i, int j,
                                              int k)
{
    const long N = ncells(g), q = cid(g, i, j, k);
    // one component at a time (a scheduling barrier between them keeps the
    // loads of one component's stencil from piling up with the next's)
#pragma unroll
    for (int c = 0; c < g.dim; ++c) {
        out[c * N + q] = visc_div_at<false, false>(g, beta, u, c, i, j, k);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int DIM>
__global__ void k_stage_visc_div(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int zb)
{
    const int cav = blockIdx.z / zb, k = blockIdx.z - cav * zb;
    const CavK& K = ck[cav];
    const GridS<DIM> g = grid_s<DIM>(K.g);
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return;
    visc_div_body(g, K.beta0, io[cav].u, K.E, i, j, k);
}

void stage_visc_div(Ctx* c)
{
    if (c->dim == 2) k_stage_visc_div<2><<<cells_of(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    else k_stage_visc_div<3><<<cells_of(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
}

// the viscous level-0 right-hand side of every cavity: b plus the wall part
// of the operator (coefficient from the slot); block z = cavity * 2 dim +
// wall face 2 a + side, after a copy of b
template <int DIM>
__global__ void k_stage_visc_wall(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int nz)
{
    const int cav = blockIdx.z / nz, w2 = blockIdx.z - cav * nz;
    const CavK& K = ck[cav];
    const int a = w2 >> 1, side = w2 & 1;
    visc_wall_at(grid_s<DIM>(K.g), K.beta0, K.sc[S_DT], io[cav].b, K.viscb, a, side, blockIdx.x * blockDim.x + threadIdx.x,
                 blockIdx.y * blockDim.y + threadIdx.y);
}

__global__ void k_stage_copy_b(const CavK* __restrict__ ck, const CavIO* __restrict__ io)
{
    const CavK& K = ck[blockIdx.y];
    const long n = (long)K.g.dim * K.nc;
    const double* __restrict__ b = io[blockIdx.y].b;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) K.viscb[i] = b[i];
}

void stage_visc_wall_rhs(Ctx* c)
{
    long nmax = 1;
    int e0 = 1, e1 = 1;
    for (const Cav& v : c->cv) {
        nmax = std::max(nmax, (long)v.dim * v.nc);
        for (int a = 0; a < v.g.dim; ++a) {
            const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
            e0 = std::max(e0, v.g.n[b0]);
            e1 = std::max(e1, v.g.n[b1]);
        }
    }
    const long nblk = std::min((nmax + 255) / 256, 8192L);
    k_stage_copy_b<<<dim3((unsigned)nblk, c->nb), 256, 0, c->s>>>(c->ck, c->cio);
    const dim3 wg = grid3(e0, e1, 2 * c->dim * c->nb, kBlk);
    if (c->dim == 2) k_stage_visc_wall<2><<<wg, kBlk, 0, c->s>>>(c->ck, c->cio, 2 * c->dim);
    else k_stage_visc_wall<3><<<wg, kBlk, 0, c->s>>>(c->ck, c->cio, 2 * c->dim);
}



}  // namespace hb
