// hb_step.hip -- kernels of the advection stage (Godunov prediction of face
// states at t^{m+1/2}, MAC divergence/update, convective term and viscous
// right-hand side) and of the approximate nodal projection.  gfx950, FP64.
//
// Layouts: slopes S[a][q][cell], transverse terms T[b][q][cell]; face arrays
// are concatenated per axis (total nf faces): uhat[f], qhat[q][f], qLf[q][f],
// qRf[q][f], uadv[f], umac[f].
#include "hb_internal.h"

namespace hb {

static const dim3 kBlk(64, 4, 1);

__device__ inline double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }
__device__ inline double lesser(double a, double b) { return a < b ? a : b; }

// fourth-order monotonicity-limited slope (Colella 1985), per cell, from the
// five values q[0..4] centred on q[2]
__device__ inline double limited_slope(const double q[5])
{
    double dc[3], dl[3], df[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const double dp = q[t + 2] - q[t + 1], dm = q[t + 1] - q[t];
        dc[t] = 0.5 * (q[t + 2] - q[t]);
        dl[t] = (dp * dm > 0.0) ? 2.0 * lesser(fabs(dp), fabs(dm)) : 0.0;
        df[t] = sgn(dc[t]) * lesser(fabs(dc[t]), dl[t]);
    }
    const double d4 = (4.0 / 3.0) * dc[1] - (1.0 / 6.0) * (df[2] + df[0]);
    return sgn(dc[1]) * lesser(fabs(d4), dl[1]);
}

// Burgers Riemann solution for the normal velocity: uL when the wave moves
// right (uL + uR > delta; 0 for a rarefaction with uL <= 0), uR when it
// moves left, and inside the dead band |uL + uR| <= delta, where a
// stationary shock's side is decided by rounding, the mean of the two
__device__ inline double burgers(double uL, double uR, double delta)
{
    const double s = uL + uR;
    const double l = uL > 0.0 ? uL : 0.0, r = uR < 0.0 ? uR : 0.0;
    if (s > delta) return l;
    if (s < -delta) return r;
    return 0.5 * (l + r);
}

__device__ inline double upwind(double vel, double qL, double qR, double delta)
{
    if (vel > delta) return qL;
    if (vel < -delta) return qR;
    return 0.5 * (qL + qR);
}

__device__ inline double deadband(const double* sc, double ulid)
{
    return 1e-12 * fmax(ulid, sc[S_MAXU]);
}

// ---------------------------------------------------------------------------
// nodal gradient and forcing
// ---------------------------------------------------------------------------

// cell average of the Q1 gradient of a nodal field
template <class GR>
__device__ inline double grad_node_at(const GR& g, const double* __restrict__ p, int a, int i, int j, int k)
{
    const int nc = 1 << g.dim;
    double s = 0.0;
#pragma unroll
    for (int bits = 0; bits < nc; ++bits) {
        if (!((bits >> a) & 1)) continue;
        int hi[3] = {i, j, k}, lo[3] = {i, j, k};
        #pragma unroll
        for (int b = 0; b < g.dim; ++b) {
            hi[b] += (bits >> b) & 1;
            lo[b] += ((bits & ~(1 << a)) >> b) & 1;
            if (g.per[b] && hi[b] == g.n[b]) hi[b] = 0;
            if (g.per[b] && lo[b] == g.n[b]) lo[b] = 0;
        }
        s += (p[nid(g, hi[0], hi[1], hi[2])] - p[nid(g, lo[0], lo[1], lo[2])]) / g.h;
    }
    return s / (double)(nc / 2);
}

// Every stage kernel below runs over all cavities of the context in one
// launch.  Cell and node loops: block z = cavity * planes + z plane; face
// loops: block z = (cavity * 3 + axis) * planes + z plane.  A block whose
// indices fall outside its cavity's extents returns.
#define STAGE_ENTER(zb)                                                   \
    const int cav = blockIdx.z / (zb), k = blockIdx.z - cav * (zb);       \
    const CavK& K = ck[cav];                                               \
    const CavIO& IO = io[cav];                                             \
    (void)IO;                                                              \
    const GridS<DIM> g = grid_s<DIM>(K.g);                                 \
    const int i = blockIdx.x * blockDim.x + threadIdx.x;                   \
    const int j = blockIdx.y * blockDim.y + threadIdx.y;

#define STAGE_CELL(zb)                                                    \
    STAGE_ENTER(zb)                                                        \
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return;

#define STAGE_NODE(zb)                                                    \
    STAGE_ENTER(zb)                                                        \
    if (i >= nnode(g, 0) || j >= nnode(g, 1) || k >= nnode(g, 2)) return;

#define STAGE_FACE(zb)                                                    \
    const int zz_ = blockIdx.z / (zb), k = blockIdx.z - zz_ * (zb);       \
    const int cav = zz_ / 3, a = zz_ - 3 * cav;                            \
    const CavK& K = ck[cav];                                               \
    const CavIO& IO = io[cav];                                             \
    (void)IO;                                                              \
    const GridS<DIM> g = grid_s<DIM>(K.g);                                 \
    if (a >= g.dim) return;                                                \
    const int i = blockIdx.x * blockDim.x + threadIdx.x;                   \
    const int j = blockIdx.y * blockDim.y + threadIdx.y;                   \
    if (i >= fext(g, a, 0) || j >= fext(g, a, 1) || k >= fext(g, a, 2)) return;

#define STAGE_ARGS const CavK* __restrict__ ck, const CavIO* __restrict__ io, int zb

static dim3 cell_grid(const Ctx* c) { return dim3((c->cx[0] + kBlk.x - 1) / kBlk.x, (c->cx[1] + kBlk.y - 1) / kBlk.y, c->cx[2] * c->nb); }
static dim3 node_grid(const Ctx* c) { return dim3((c->nx[0] + kBlk.x - 1) / kBlk.x, (c->nx[1] + kBlk.y - 1) / kBlk.y, c->nx[2] * c->nb); }
static dim3 face_grid(const Ctx* c) { return dim3((c->fx[0] + kBlk.x - 1) / kBlk.x, (c->fx[1] + kBlk.y - 1) / kBlk.y, c->fx[2] * 3 * c->nb); }

// Gp = G p, the cell average of the Q1 gradient of the pressure
// (the bodies take the cavity's arrays as restrict-qualified arguments: the
// table they come from says nothing about aliasing)
template <class GR>
__device__ __forceinline__ void grad_node_body(const GR& g, const double* __restrict__ p, double* __restrict__ Gp,
                                               int i, int j, int k)
{
    const long N = ncells(g), q = cid(g, i, j, k);
    #pragma unroll
    for (int a = 0; a < g.dim; ++a) Gp[a * N + q] = grad_node_at(g, p, a, i, j, k);
}

template <int DIM>
__global__ void k_grad_node(STAGE_ARGS)
{
    STAGE_CELL(zb);
    grad_node_body(g, IO.p, K.Gp, i, j, k);
}

void stage_grad_node(Ctx* c)
{
    if (c->dim == 2) k_grad_node<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    else k_grad_node<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
}

// F = -G p + wF E + f, the forcing of the Taylor prediction: wF = 2 puts
// the whole explicit stress divergence in (as eq:iamr:extrap prints it),
// wF = 0 leaves it out
template <class GR>
__device__ __forceinline__ void forcing_body(const GR& g, const FluidD& fl, double wF, const double* __restrict__ Gp,
                                             const double* __restrict__ E, double* __restrict__ F, int i, int j, int k)
{
    const long N = ncells(g), q0 = cid(g, i, j, k);
    #pragma unroll
    for (int c = 0; c < g.dim; ++c) {
        const long t = c * N + q0;
        F[t] = -Gp[t] + wF * E[t] + fl.f[c];
    }
}

template <int DIM>
__global__ void k_forcing(STAGE_ARGS, double wF)
{
    STAGE_CELL(zb);
    forcing_body(g, K.fl, wF, K.Gp, K.E, K.F, i, j, k);
}

void stage_forcing(Ctx* c)
{
    const double wF = c->opts.pred_visc ? 2.0 : 0.0;
    if (c->dim == 2) k_forcing<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2], wF);
    else k_forcing<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2], wF);
}

// ---------------------------------------------------------------------------
// Godunov prediction
// ---------------------------------------------------------------------------

template <class GR>
__device__ __forceinline__ void slopes_body(const GR& g, const double* __restrict__ u, double* __restrict__ S,
                                            int i, int j, int k)
{
    const long N = ncells(g), q0 = cid(g, i, j, k);
    const int d = g.dim;
    #pragma unroll
    for (int a = 0; a < d; ++a)
        #pragma unroll
        for (int q = 0; q < d; ++q) {
            double st[5];
            for (int t = 0; t < 5; ++t) {
                int p[3] = {i, j, k};
                p[a] += t - 2;
                st[t] = cval<false>(g, u + (long)q * N, q, p[0], p[1], p[2]);
            }
            S[((long)a * d + q) * N + q0] = limited_slope(st);
        }
}

template <int DIM>
__global__ void k_slopes(STAGE_ARGS)
{
    STAGE_CELL(zb);
    slopes_body(g, IO.u, K.S, i, j, k);
}

void stage_slopes(Ctx* c)
{
    if (c->dim == 2) k_slopes<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    else k_slopes<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
}

// normal-only traced states on a-faces, upwinded by their Burgers solution
template <class GR>
__device__ __forceinline__ void trace_normal_body(const GR& g, int a, double dt, double delta, long nf,
                                                  const double* __restrict__ u, const double* __restrict__ S,
                                                  double* __restrict__ uhat, double* __restrict__ qhat, int i, int j,
                                                  int k)
{
    const int d = g.dim;
    const long N = ncells(g);
    const long f = foffset(g, a) + fid(g, a, i, j, k);
    int R[3] = {i, j, k}, L[3] = {i, j, k};
    L[a] -= 1;
    const bool okL = wrap(g, L), okR = wrap(g, R);
    if (!okL || !okR) {
        const int side = okL ? 1 : 0;
        uhat[f] = 0.0;
        #pragma unroll
        for (int q = 0; q < d; ++q) qhat[q * nf + f] = g.wall_u[a][side][q];
        return;
    }
    const long cL = cid(g, L[0], L[1], L[2]), cR = cid(g, R[0], R[1], R[2]);
    double qL[3], qR[3];
    #pragma unroll
    for (int q = 0; q < d; ++q) {
        qL[q] = u[q * N + cL] + (0.5 - dt * u[a * N + cL] / (2.0 * g.h)) * S[((long)a * d + q) * N + cL];
        qR[q] = u[q * N + cR] - (0.5 + dt * u[a * N + cR] / (2.0 * g.h)) * S[((long)a * d + q) * N + cR];
    }
    const double uh = burgers(qL[a], qR[a], delta);
    uhat[f] = uh;
    #pragma unroll
    for (int q = 0; q < d; ++q) qhat[q * nf + f] = (q == a) ? uh : upwind(uh, qL[q], qR[q], delta);
}

template <int DIM>
__global__ void k_trace_normal(STAGE_ARGS)
{
    STAGE_FACE(zb);
    trace_normal_body(g, a, IO.dt, deadband(K.sc, K.ulid), K.nf, IO.u, K.S, K.uhat, K.qhat, i, j, k);
}

void stage_trace_normal(Ctx* c)
{
    if (c->dim == 2) k_trace_normal<2><<<face_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
    else k_trace_normal<3><<<face_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
}

// transverse terms at cells: (u_b dq/dx_b)^ = mean face velocity x difference
template <class GR>
__device__ __forceinline__ void transverse_body(const GR& g, long nf, const double* __restrict__ uhat,
                                                const double* __restrict__ qhat, double* __restrict__ T, int i, int j,
                                                int k)
{
    const int d = g.dim;
    const long N = ncells(g), q0 = cid(g, i, j, k);
    #pragma unroll
    for (int b = 0; b < d; ++b) {
        int hi[3] = {i, j, k};
        hi[b] += 1;
        if (g.per[b] && hi[b] == g.n[b]) hi[b] = 0;
        const long flo = foffset(g, b) + fid(g, b, i, j, k);
        const long fhi = foffset(g, b) + fid(g, b, hi[0], hi[1], hi[2]);
        const double ubar = 0.5 * (uhat[flo] + uhat[fhi]);
        #pragma unroll
        for (int q = 0; q < d; ++q) {
            const double dq = (qhat[q * nf + fhi] - qhat[q * nf + flo]) / g.h;
            T[((long)b * d + q) * N + q0] = ubar * dq;
        }
    }
}

template <int DIM>
__global__ void k_transverse(STAGE_ARGS)
{
    STAGE_CELL(zb);
    transverse_body(g, K.nf, K.uhat, K.qhat, K.trans, i, j, k);
}

void stage_transverse(Ctx* c)
{
    if (c->dim == 2) k_transverse<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    else k_transverse<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
}

// full face states: traced normal part - dt/2 transverse terms + dt/2 forcing;
// the advection velocity is the Burgers solution of the normal component
template <class GR>
__device__ __forceinline__ void trace_full_body(const GR& g, int a, double dt, double delta, long nf,
                                                const double* __restrict__ u, const double* __restrict__ S,
                                                const double* __restrict__ T, const double* __restrict__ F,
                                                double* __restrict__ qLf, double* __restrict__ qRf,
                                                double* __restrict__ uadv, int i, int j, int k)
{
    const int d = g.dim;
    const long N = ncells(g);
    const long f = foffset(g, a) + fid(g, a, i, j, k);
    int R[3] = {i, j, k}, L[3] = {i, j, k};
    L[a] -= 1;
    const bool okL = wrap(g, L), okR = wrap(g, R);
    if (!okL || !okR) {
        const int side = okL ? 1 : 0;
        uadv[f] = 0.0;
        #pragma unroll
        for (int q = 0; q < d; ++q) {
            qLf[q * nf + f] = g.wall_u[a][side][q];
            qRf[q * nf + f] = g.wall_u[a][side][q];
        }
        return;
    }
    const long cL = cid(g, L[0], L[1], L[2]), cR = cid(g, R[0], R[1], R[2]);
    #pragma unroll
    for (int q = 0; q < d; ++q) {
        double tl = 0.0, tr = 0.0;
        #pragma unroll
        for (int b = 0; b < d; ++b) {
            if (b == a) continue;
            tl += T[((long)b * d + q) * N + cL];
            tr += T[((long)b * d + q) * N + cR];
        }
        const double vl = u[q * N + cL] + (0.5 - dt * u[a * N + cL] / (2.0 * g.h)) * S[((long)a * d + q) * N + cL]
                          - 0.5 * dt * tl + 0.5 * dt * F[q * N + cL];
        const double vr = u[q * N + cR] - (0.5 + dt * u[a * N + cR] / (2.0 * g.h)) * S[((long)a * d + q) * N + cR]
                          - 0.5 * dt * tr + 0.5 * dt * F[q * N + cR];
        qLf[q * nf + f] = vl;
        qRf[q * nf + f] = vr;
    }
    uadv[f] = burgers(qLf[a * nf + f], qRf[a * nf + f], delta);
}

template <int DIM>
__global__ void k_trace_full(STAGE_ARGS)
{
    STAGE_FACE(zb);
    trace_full_body(g, a, IO.dt, deadband(K.sc, K.ulid), K.nf, IO.u, K.S, K.trans, K.F, K.qLf, K.qRf, K.uadv, i, j, k);
}

void stage_trace_full(Ctx* c)
{
    if (c->dim == 2) k_trace_full<2><<<face_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
    else k_trace_full<3><<<face_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
}

// ---------------------------------------------------------------------------
// MAC projection of the advection velocity
// ---------------------------------------------------------------------------

// cell divergence of a face field: of u^adv into the MAC right-hand side
// (after = 0), or of u^MAC into macrhs (after = 1)
template <class GR>
__device__ __forceinline__ void mac_div_body(const GR& g, const double* __restrict__ F, double* __restrict__ out,
                                             int i, int j, int k)
{
    double s = 0.0;
    #pragma unroll
    for (int a = 0; a < g.dim; ++a) {
        int hi[3] = {i, j, k};
        hi[a] += 1;
        if (g.per[a] && hi[a] == g.n[a]) hi[a] = 0;
        const long off = foffset(g, a);
        s += (F[off + fid(g, a, hi[0], hi[1], hi[2])] - F[off + fid(g, a, i, j, k)]) / g.h;
    }
    out[cid(g, i, j, k)] = s;
}

template <int DIM>
__global__ void k_mac_div(STAGE_ARGS, int after)
{
    STAGE_CELL(zb);
    mac_div_body(g, after ? K.umac : K.uadv, after ? K.macrhs : K.macb, i, j, k);
}

void stage_mac_div(Ctx* c, int after)
{
    if (c->dim == 2) k_mac_div<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2], after);
    else k_mac_div<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2], after);
}

// u^MAC = u^adv - G_mac phi (the gradient vanishes on wall faces)
template <class GR>
__device__ __forceinline__ void mac_update_body(const GR& g, int a, const double* __restrict__ uadv,
                                                const double* __restrict__ phi, double* __restrict__ umac, int i, int j,
                                                int k)
{
    const long f = foffset(g, a) + fid(g, a, i, j, k);
    int R[3] = {i, j, k}, L[3] = {i, j, k};
    L[a] -= 1;
    double gphi = 0.0;
    if (wrap(g, L) && wrap(g, R)) gphi = (phi[cid(g, R[0], R[1], R[2])] - phi[cid(g, L[0], L[1], L[2])]) / g.h;
    umac[f] = uadv[f] - gphi;
}

template <int DIM>
__global__ void k_mac_update(STAGE_ARGS)
{
    STAGE_FACE(zb);
    mac_update_body(g, a, K.uadv, K.macphi, K.umac, i, j, k);
}

void stage_mac_update(Ctx* c)
{
    if (c->dim == 2) k_mac_update<2><<<face_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
    else k_mac_update<3><<<face_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->fx[2]);
}

// convective term A = sum_a mean(u^MAC_a) (q~_hi - q~_lo)/h with the full
// states upwinded by u^MAC, and b = u - dt A + dt (-G p + wb E + f) with
// wb = 2 (1 - theta) (1 for Crank-Nicolson)
template <class GR>
__device__ __forceinline__ void advect_rhs_body(const GR& g, const FluidD& fl, double dt, double wb, double delta,
                                                long nf, const double* __restrict__ u, const double* __restrict__ umac,
                                                const double* __restrict__ qLf, const double* __restrict__ qRf,
                                                const double* __restrict__ Gp, const double* __restrict__ E,
                                                double* __restrict__ b, double* __restrict__ conv, int i, int j, int k)
{
    const int d = g.dim;
    const long N = ncells(g), q0 = cid(g, i, j, k);
    double A[3] = {0.0, 0.0, 0.0};
    #pragma unroll
    for (int a = 0; a < d; ++a) {
        int hi[3] = {i, j, k};
        hi[a] += 1;
        if (g.per[a] && hi[a] == g.n[a]) hi[a] = 0;
        const long flo = foffset(g, a) + fid(g, a, i, j, k);
        const long fhi = foffset(g, a) + fid(g, a, hi[0], hi[1], hi[2]);
        const double ulo = umac[flo], uhi = umac[fhi];
        #pragma unroll
        for (int q = 0; q < d; ++q) {
            const double tlo = upwind(ulo, qLf[q * nf + flo], qRf[q * nf + flo], delta);
            const double thi = upwind(uhi, qLf[q * nf + fhi], qRf[q * nf + fhi], delta);
            A[q] += 0.5 * (ulo + uhi) * (thi - tlo) / g.h;
        }
    }
    #pragma unroll
    for (int q = 0; q < d; ++q) {
        const long e = q * N + q0;
        b[e] = u[e] - dt * A[q] + dt * (-Gp[e] + wb * E[e] + fl.f[q]);
        if (conv) conv[e] = A[q];
    }
}

template <int DIM>
__global__ void k_advect_rhs(STAGE_ARGS, double wb)
{
    STAGE_CELL(zb);
    advect_rhs_body(g, K.fl, IO.dt, wb, deadband(K.sc, K.ulid), K.nf, IO.u, K.umac, K.qLf, K.qRf, K.Gp, K.E, IO.b,
                    IO.conv, i, j, k);
}

void stage_advect_rhs(Ctx* c)
{
    const double wb = 2.0 * (1.0 - c->opts.theta);
    if (c->dim == 2) k_advect_rhs<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2], wb);
    else k_advect_rhs<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2], wb);
}

// ---------------------------------------------------------------------------
// approximate projection
// ---------------------------------------------------------------------------

// r_k = sum over cells touching node k of sum_a s_a (h/2)^(d-1) V_a, where
// V = ustar/dt + G p into the nodal right-hand side (PROJ), or V = uout into
// rnode
template <bool PROJ, class GR>
__device__ __forceinline__ void weak_div_body(const GR& g, double dt, const double* __restrict__ V,
                                              const double* __restrict__ Gp, double* __restrict__ r, int i, int j,
                                              int k)
{
    const int d = g.dim;
    const long N = ncells(g);
    const double w = d == 2 ? 0.5 * g.h : (0.5 * g.h) * (0.5 * g.h);
    const int node[3] = {i, j, k};
    double s = 0.0;
#pragma unroll
    for (int me = 0; me < (1 << d); ++me) {     // node is corner `me` of the cell
        int cc[3] = {0, 0, 0};
        bool ok = true;
        #pragma unroll
        for (int a = 0; a < d; ++a) {
            int v = node[a] - ((me >> a) & 1);
            if (v < 0) { if (g.per[a]) v += g.n[a]; else ok = false; }
            if (v >= g.n[a]) ok = false;
            cc[a] = v;
        }
        if (!ok) continue;
        const long q = cid(g, cc[0], cc[1], cc[2]);
        double t = 0.0;
        #pragma unroll
        for (int a = 0; a < d; ++a) {
            const double sg = ((me >> a) & 1) ? 1.0 : -1.0;
            const double Va = PROJ ? V[a * N + q] / dt + Gp[a * N + q] : V[a * N + q];
            t += sg * w * Va;
        }
        s += t;
    }
    r[nid(g, i, j, k)] = s;
}

template <bool PROJ, int DIM>
__global__ void k_weak_div(STAGE_ARGS)
{
    STAGE_NODE(zb);
    weak_div_body<PROJ>(g, IO.dt, PROJ ? IO.ustar : IO.uout, K.Gp, PROJ ? K.nodb : K.rnode, i, j, k);
}

void stage_proj_rhs(Ctx* c)
{
    if (c->dim == 2) k_weak_div<true, 2><<<node_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->nx[2]);
    else k_weak_div<true, 3><<<node_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->nx[2]);
}

void stage_weak_div_u(Ctx* c)
{
    if (c->dim == 2) k_weak_div<false, 2><<<node_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->nx[2]);
    else k_weak_div<false, 3><<<node_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->nx[2]);
}

// uout = ustar + dt (G p - G phi)
template <class GR>
__device__ __forceinline__ void proj_update_body(const GR& g, double dt, const double* __restrict__ ustar,
                                                 const double* __restrict__ Gp, const double* __restrict__ phi,
                                                 double* __restrict__ u, int i, int j, int k)
{
    const long N = ncells(g), q = cid(g, i, j, k);
    #pragma unroll
    for (int a = 0; a < g.dim; ++a) {
        const double gphi = grad_node_at(g, phi, a, i, j, k);
        u[a * N + q] = ustar[a * N + q] + dt * (Gp[a * N + q] - gphi);
    }
}

template <int DIM>
__global__ void k_proj_update(STAGE_ARGS)
{
    STAGE_CELL(zb);
    proj_update_body(g, IO.dt, IO.ustar, K.Gp, K.phi, IO.uout, i, j, k);
}

void stage_proj_update(Ctx* c)
{
    if (c->dim == 2) k_proj_update<2><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
    else k_proj_update<3><<<cell_grid(c), kBlk, 0, c->s>>>(c->ck, c->cio, c->cx[2]);
}

}  // namespace hb
