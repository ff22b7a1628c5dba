// hb_tail.hip -- the coarse end of a V-cycle in ONE workgroup: every level
// from the first small one down to the coarsest (smoothing, residual and
// restriction, the dense LU solve, prolongation and post-smoothing) runs in a
// single launch, phases separated by workgroup barriers, with the levels'
// arrays held in LDS for the whole cycle.  The coarse levels are a few
// thousand unknowns at most, so this replaces dozens of tiny, latency-bound
// launches per cycle.  The per-cell arithmetic is the same as
// in the per-level kernels (shared device operators), and the phases run in
// the same order as the level-by-level cycle, so results are identical.
#include <cstring>

#include "hb_internal.h"
#include "hb_ops.h"

namespace hb {

constexpr int kTailThreads = 1024;
constexpr int kTailMaxLev = 10;

struct TailLevel {
    GridD g;
    double* x;
    double* b;
    double* r;
    const double* beta;
};

// static description of a hierarchy's tail, kept in device memory
struct TailArgs {
    int op, nlev, N;
    const double* A;
    const int* piv;
    TailLevel L[kTailMaxLev];
    int nu[kTailMaxLev];       // unknowns per level
    int nbeta[kTailMaxLev];    // face viscosities per level (tensor problem)
    int off[kTailMaxLev];      // LDS offset (doubles) of the level's x, b, r, beta
};

// LDS doubles of one level: x, b, r and (tensor problem) the face viscosities
inline int tail_level_doubles(int nu, int nbeta) { return 3 * nu + nbeta; }

// a level as the tail kernel sees it: the grid stays in kernel-argument
// memory (indexable without private copies), the arrays in LDS
struct TL {
    const GridD* gp;
    double* x;
    double* b;
    double* r;
    const double* beta;
};

// ---- tensor problem ---------------------------------------------------------

__device__ void tail_visc_smooth(const TL& l, double dt, int sweeps)
{
    const GridD& g = *l.gp;
    const long N = ncells(g);
    const int hx = (g.n[0] + 1) / 2;
    const long npair = (long)hx * g.n[1] * g.n[2];
    for (int s = 0; s < sweeps; ++s)
        for (int c = 0; c < g.dim; ++c)
            for (int colour = 0; colour < 2; ++colour) {
                for (long t = threadIdx.x; t < npair; t += blockDim.x) {
                    const int px = (int)(t % hx), j = (int)((t / hx) % g.n[1]), k = (int)(t / ((long)hx * g.n[1]));
                    const int i = 2 * px + ((j + k + colour) & 1);
                    if (i >= g.n[0]) continue;
                    const long q = (long)c * N + cid(g, i, j, k);
                    const double Au = l.x[q] - dt * visc_div_at<true, false>(g, l.beta, l.x, c, i, j, k);
                    const double dg = visc_diag(g, l.beta, dt, c, i, j, k);
                    l.x[q] += (l.b[q] - Au) / dg;
                }
                __syncthreads();
            }
}

__device__ void tail_visc_restrict(const TL& f, const TL& cl, double dt)
{
    const GridD &gf = *f.gp, &gc = *cl.gp;
    const long Nf = ncells(gf), Nc = ncells(gc);
    const int nch = 1 << gf.dim;
    for (long t = threadIdx.x; t < Nc; t += blockDim.x) {
        const int i = (int)(t % gc.n[0]), j = (int)((t / gc.n[0]) % gc.n[1]), k = (int)(t / ((long)gc.n[0] * gc.n[1]));
        for (int c = 0; c < gf.dim; ++c) {
            double s = 0.0;
            for (int bits = 0; bits < nch; ++bits) {
                const int fi = 2 * i + (bits & 1), fj = 2 * j + ((bits >> 1) & 1), fk = gf.dim == 3 ? 2 * k + ((bits >> 2) & 1) : 0;
                const long qf = c * Nf + cid(gf, fi, fj, fk);
                const double Ax = f.x[qf] - dt * visc_div_at<true, false>(gf, f.beta, f.x, c, fi, fj, fk);
                s += f.b[qf] - Ax;
            }
            cl.b[c * Nc + t] = s / (double)nch;
            cl.x[c * Nc + t] = 0.0;
        }
    }
    __syncthreads();
}

// ---- MAC problem ------------------------------------------------------------

__device__ void tail_mac_smooth(const TL& l, int sweeps)
{
    const GridD& g = *l.gp;
    const int hx = (g.n[0] + 1) / 2;
    const long npair = (long)hx * g.n[1] * g.n[2];
    const double ih2 = 1.0 / (g.h * g.h);
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            for (long t = threadIdx.x; t < npair; t += blockDim.x) {
                const int px = (int)(t % hx), j = (int)((t / hx) % g.n[1]), k = (int)(t / ((long)hx * g.n[1]));
                const int i = 2 * px + ((j + k + colour) & 1);
                if (i >= g.n[0]) continue;
                const long q = cid(g, i, j, k);
                double Lx = 0.0;
                int cnt = 0;
                for (int a = 0; a < g.dim; ++a)
                    for (int side = 0; side < 2; ++side) {
                        int p[3] = {i, j, k};
                        p[a] += side ? 1 : -1;
                        if (!wrap(g, p)) continue;
                        Lx += (l.x[cid(g, p[0], p[1], p[2])] - l.x[q]) * ih2;
                        ++cnt;
                    }
                const double dg = -(double)cnt * ih2;
                l.x[q] += (l.b[q] - Lx) / dg;
            }
            __syncthreads();
        }
}

__device__ void tail_mac_restrict(const TL& f, const TL& cl)
{
    const GridD &gf = *f.gp, &gc = *cl.gp;
    const long Nc = ncells(gc);
    const int nch = 1 << gf.dim;
    for (long t = threadIdx.x; t < Nc; t += blockDim.x) {
        const int i = (int)(t % gc.n[0]), j = (int)((t / gc.n[0]) % gc.n[1]), k = (int)(t / ((long)gc.n[0] * gc.n[1]));
        double s = 0.0;
        for (int bits = 0; bits < nch; ++bits) {
            const int fi = 2 * i + (bits & 1), fj = 2 * j + ((bits >> 1) & 1), fk = gf.dim == 3 ? 2 * k + ((bits >> 2) & 1) : 0;
            s += f.b[cid(gf, fi, fj, fk)] - mac_lap_at(gf, f.x, fi, fj, fk);
        }
        cl.b[t] = s / (double)nch;
        cl.x[t] = 0.0;
    }
    __syncthreads();
}

// cell prolongation (both cell problems)
__device__ void tail_prolong_cells(const TL& f, const TL& cl, int ncomp, double wall_sign)
{
    const GridD &gf = *f.gp, &gc = *cl.gp;
    const int d = gf.dim;
    const long Nf = ncells(gf), Nc = ncells(gc);
    for (long t = threadIdx.x; t < Nf; t += blockDim.x) {
        const int fi[3] = {(int)(t % gf.n[0]), (int)((t / gf.n[0]) % gf.n[1]), (int)(t / ((long)gf.n[0] * gf.n[1]))};
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
                s += w * sg * cl.x[q * Nc + cid(gc, p[0], p[1], p[2])];
            }
            f.x[q * Nf + t] += s;
        }
    }
    __syncthreads();
}

// ---- nodal problem ----------------------------------------------------------

template <int DIM>
__device__ void tail_nodal_smooth(const TL& l, int sweeps)
{
    const GridD& g = *l.gp;
    const int nx = nnode(g, 0), ny = nnode(g, 1), nz = nnode(g, 2);
    const int hx = (nx + 1) / 2, hy = (ny + 1) / 2, hz = DIM == 3 ? (nz + 1) / 2 : 1;
    const long nt = (long)hx * hy * hz;
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < (1 << DIM); ++colour) {
            for (long t = threadIdx.x; t < nt; t += blockDim.x) {
                const int i = 2 * (int)(t % hx) + (colour & 1);
                const int j = 2 * (int)((t / hx) % hy) + ((colour >> 1) & 1);
                const int k = DIM == 3 ? 2 * (int)(t / ((long)hx * hy)) + ((colour >> 2) & 1) : 0;
                if (i >= nx || j >= ny || k >= nz) continue;
                double dg;
                const double Kx = K_glob<DIM>(g, l.x, i, j, k, &dg);
                const long q = nid(g, i, j, k);
                l.x[q] += (l.b[q] - Kx) / dg;
            }
            __syncthreads();
        }
}

template <int DIM>
__device__ void tail_nodal_restrict(const TL& f, const TL& cl)
{
    const GridD &gf = *f.gp, &gc = *cl.gp;
    const long nnf = nnodes(gf), nnc = nnodes(gc);
    const int fx = nnode(gf, 0), fy = nnode(gf, 1);
    for (long t = threadIdx.x; t < nnf; t += blockDim.x) {
        const int i = (int)(t % fx), j = (int)((t / fx) % fy), k = (int)(t / ((long)fx * fy));
        f.r[t] = f.b[t] - K_glob<DIM>(gf, f.x, i, j, k, nullptr);
    }
    __syncthreads();
    const int cx = nnode(gc, 0), cy = nnode(gc, 1);
    int ntt = 1;
    for (int a = 0; a < DIM; ++a) ntt *= 3;
    for (long t = threadIdx.x; t < nnc; t += blockDim.x) {
        const int I[3] = {(int)(t % cx), (int)((t / cx) % cy), (int)(t / ((long)cx * cy))};
        double s = 0.0;
        for (int u = 0; u < ntt; ++u) {
            int uu = u, p[3] = {0, 0, 0};
            double w = 1.0;
            bool ok = true;
            for (int a = 0; a < DIM; ++a) {
                const int del = uu % 3 - 1;
                uu /= 3;
                if (del != 0) w *= 0.5;
                int F = 2 * I[a] + del;
                const int nf = nnode(gf, a);
                if (F < 0 || F >= nf) {
                    if (gf.per[a]) F = F < 0 ? F + nf : F - nf;
                    else ok = false;
                }
                p[a] = F;
            }
            if (ok) s += w * f.r[nid(gf, p[0], p[1], p[2])];
        }
        cl.b[t] = s;
        cl.x[t] = 0.0;
    }
    __syncthreads();
}

template <int DIM>
__device__ void tail_nodal_prolong(const TL& f, const TL& cl)
{
    const GridD &gf = *f.gp, &gc = *cl.gp;
    const int fx = nnode(gf, 0), fy = nnode(gf, 1);
    const long nnf = nnodes(gf);
    for (long t = threadIdx.x; t < nnf; t += blockDim.x) {
        const int F[3] = {(int)(t % fx), (int)((t / fx) % fy), (int)(t / ((long)fx * fy))};
        double s = 0.0;
        for (int bits = 0; bits < (1 << DIM); ++bits) {
            int p[3] = {0, 0, 0};
            double w = 1.0;
            bool ok = true;
            for (int a = 0; a < DIM; ++a) {
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
            if (ok) s += w * cl.x[nid(gc, p[0], p[1], p[2])];
        }
        f.x[t] += s;
    }
    __syncthreads();
}

// ---- dense coarsest solve (thread 0), same order as the LU kernel ----------

__device__ void tail_lu_solve(int N, const double* __restrict__ A, const int* __restrict__ piv, const double* b, double* x)
{
    if (threadIdx.x == 0) {
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
    __syncthreads();
}

// level l of the tail with its arrays in LDS
__device__ inline TL lds_level(const TailArgs& t, double* lds, const GridD* sg, int l)
{
    TL L;
    double* base = lds + t.off[l];
    L.gp = &sg[l];
    L.x = base;
    L.b = base + t.nu[l];
    L.r = base + 2 * t.nu[l];
    L.beta = t.nbeta[l] ? base + 3 * t.nu[l] : nullptr;
    return L;
}

template <int DIM>
__global__ void __launch_bounds__(kTailThreads)
k_tail(const TailArgs* __restrict__ tp, double* __restrict__ x0, const double* __restrict__ b0, double dt, int nu1, int nu2)
{
    const TailArgs& t = *tp;
    extern __shared__ double lds[];
    // grids of the levels in LDS: cheap to re-read after the stores to the
    // level arrays, which the compiler cannot tell apart from them
    __shared__ GridD sg[kTailMaxLev];
    if (threadIdx.x < (unsigned)t.nlev) sg[threadIdx.x] = t.L[threadIdx.x].g;
    const int last = t.nlev - 1;
    // the top level's iterate and right-hand side, every level's face
    // viscosities; the coarser levels' x and b are produced in the cycle
    for (int l = 0; l < t.nlev; ++l) {
        double* base = lds + t.off[l];
        if (l == 0) {
            for (int i = threadIdx.x; i < t.nu[0]; i += blockDim.x) {
                base[i] = x0[i];
                base[t.nu[0] + i] = b0[i];
            }
        }
        for (int i = threadIdx.x; i < t.nbeta[l]; i += blockDim.x) base[3 * t.nu[l] + i] = t.L[l].beta[i];
    }
    __syncthreads();
    for (int l = 0; l < last; ++l) {
        const TL L = lds_level(t, lds, sg, l), C = lds_level(t, lds, sg, l + 1);
        if (t.op == HB_OP_VISC) {
            tail_visc_smooth(L, dt, nu1);
            tail_visc_restrict(L, C, dt);
        } else if (t.op == HB_OP_MAC) {
            tail_mac_smooth(L, nu1);
            tail_mac_restrict(L, C);
        } else {
            tail_nodal_smooth<DIM>(L, nu1);
            tail_nodal_restrict<DIM>(L, C);
        }
    }
    {
        const TL C = lds_level(t, lds, sg, last);
        tail_lu_solve(t.N, t.A, t.piv, C.b, C.x);
    }
    for (int l = last - 1; l >= 0; --l) {
        const TL L = lds_level(t, lds, sg, l), C = lds_level(t, lds, sg, l + 1);
        if (t.op == HB_OP_VISC) {
            tail_prolong_cells(L, C, DIM, -1.0);
            tail_visc_smooth(L, dt, nu2);
        } else if (t.op == HB_OP_MAC) {
            tail_prolong_cells(L, C, 1, 1.0);
            tail_mac_smooth(L, nu2);
        } else {
            tail_nodal_prolong<DIM>(L, C);
            tail_nodal_smooth<DIM>(L, nu2);
        }
    }
    for (int i = threadIdx.x; i < t.nu[0]; i += blockDim.x) x0[i] = lds[t.off[0] + i];
}

int tail_max_levels() { return kTailMaxLev; }

static long nbeta_of(const MG& m, int l)
{
    if (m.op != HB_OP_VISC) return 0;
    long n = 0;
    for (int a = 0; a < m.L[l].g.dim; ++a) n += fcount(m.L[l].g, a);
    return n;
}

// LDS bytes of a tail starting at level `first`
size_t tail_lds_bytes(const MG& m, int first)
{
    long d = 0;
    for (int l = first; l < m.nlev; ++l) d += tail_level_doubles((int)m.L[l].nu, (int)nbeta_of(m, l));
    return sizeof(double) * (size_t)d;
}

// write the static tail description of m (levels m.tail..) to device memory
int tail_setup(Ctx* c, MG& m)
{
    TailArgs t;
    memset(&t, 0, sizeof(t));
    const int first = m.tail;
    t.op = m.op;
    t.nlev = m.nlev - first;
    t.N = m.ncoarse;
    t.A = m.A;
    t.piv = m.piv;
    int off = 0;
    for (int l = 0; l < t.nlev; ++l) {
        const Level& L = m.L[first + l];
        t.L[l].g = L.g;
        t.L[l].x = L.xb[0];
        t.L[l].b = L.b;
        t.L[l].r = L.r;
        t.L[l].beta = L.beta;
        t.nu[l] = (int)L.nu;
        t.nbeta[l] = (int)nbeta_of(m, first + l);
        t.off[l] = off;
        off += tail_level_doubles(t.nu[l], t.nbeta[l]);
    }
    m.tail_lds = sizeof(double) * (size_t)off;
    if (hipMalloc(&m.tailargs, sizeof(TailArgs)) != hipSuccess) return HB_ERR_OOM;
    if (hipMemcpy(m.tailargs, &t, sizeof(TailArgs), hipMemcpyHostToDevice) != hipSuccess) return HB_ERR_DEVICE;
    return HB_OK;
}

// V-cycle of levels m.tail.. in one workgroup, from the tail level's current
// iterate and right-hand side
void launch_tail(Ctx* c, const MG& m, int first, int nu1, int nu2)
{
    const Level& L = m.L[first];
    const TailArgs* tp = (const TailArgs*)m.tailargs;
    if (c->g.dim == 2) k_tail<2><<<1, kTailThreads, m.tail_lds, c->s>>>(tp, L.X(), L.b, m.dt, nu1, nu2);
    else k_tail<3><<<1, kTailThreads, m.tail_lds, c->s>>>(tp, L.X(), L.b, m.dt, nu1, nu2);
}

}  // namespace hb
