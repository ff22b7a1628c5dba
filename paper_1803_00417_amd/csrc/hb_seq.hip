// hb_seq.hip -- grid sequencing (Sec. III.C): the state of a run on one grid
// carried to the grid refined by two along every axis, so that a steady
// low-resolution run can continue at the higher resolution.
//
// The paper leaves the interpolation to its framework.  Here the cell-centred
// velocity is interpolated conservatively with central slopes (the mean of
// a coarse cell's children is the coarse value; linear fields are kept),
// with the wall ghost 2 u_wall - u (the step's odd reflection) beyond a wall
// and the wrapped cell beyond a periodic face; the nodal pressure is
// interpolated multilinearly between the coarse nodes.  One thread per fine
// cell or node: the kernels run once per refinement and move a few words per
// point, so plain coalesced loads and stores are all they need.
#include "hb_internal.h"

namespace hb {

static constexpr int kSeqT = 256;

// component q next to cell C along axis a (s = -1 or +1)
__device__ inline double seq_neighbour(const GridD& g, const double* __restrict__ u, long N, int q, const int C[3],
                                       double uC, int a, int s)
{
    int K[3] = {C[0], C[1], C[2]};
    K[a] += s;
    if (K[a] < 0 || K[a] >= g.n[a]) {
        if (!g.per[a]) return 2.0 * g.wall_u[a][s > 0 ? 1 : 0][q] - uC;
        K[a] = K[a] < 0 ? K[a] + g.n[a] : K[a] - g.n[a];
    }
    return u[q * N + cid(g, K[0], K[1], K[2])];
}

// child = u(C) + the sum over the axes, x first, of (+-1/4) (u(C+1) - u(C-1)) / 2,
// with + for the child on the high half of its parent
template <int DIM>
__global__ void __launch_bounds__(kSeqT) k_refine_cells(GridD gc, GridD gf, const double* __restrict__ uc,
                                                        double* __restrict__ uf)
{
    const long Nf = ncells(gf);
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Nf) return;
    const long row = t / gf.n[0];
    const int F[3] = {(int)(t - row * gf.n[0]), (int)(row % gf.n[1]), (int)(row / gf.n[1])};
    const int C[3] = {F[0] >> 1, F[1] >> 1, DIM == 3 ? F[2] >> 1 : 0};
    const long Nc = ncells(gc);
    const long ic = cid(gc, C[0], C[1], C[2]);
#pragma unroll
    for (int q = 0; q < DIM; ++q) {
        const double uC = uc[q * Nc + ic];
        double v = uC;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double lo = seq_neighbour(gc, uc, Nc, q, C, uC, a, -1);
            const double hi = seq_neighbour(gc, uc, Nc, q, C, uC, a, +1);
            const double slope = 0.5 * (hi - lo);
            v = v + ((F[a] & 1) ? 0.25 : -0.25) * slope;
        }
        uf[q * Nf + t] = v;
    }
}

// a fine node at an even index along an axis lies on a coarse node, at an
// odd one halfway between two (the last interval of a periodic axis wraps
// to node 0); the value sums weight (1 or 1/2 per axis) times coarse value
// over those nodes, x choice fastest, low before high
template <int DIM>
__global__ void __launch_bounds__(kSeqT) k_refine_nodes(GridD gc, GridD gf, const double* __restrict__ pc,
                                                        double* __restrict__ pf)
{
    const long Nf = nnodes(gf);
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Nf) return;
    const int m0 = nnode(gf, 0), m1 = nnode(gf, 1);
    const long row = t / m0;
    const int F[3] = {(int)(t - row * m0), (int)(row % m1), (int)(row / m1)};
    const int cn[3] = {nnode(gc, 0), nnode(gc, 1), nnode(gc, 2)};
    double s = 0.0;
#pragma unroll
    for (int bits = 0; bits < (1 << DIM); ++bits) {
        double w = 1.0;
        int I[3] = {0, 0, 0};
        bool skip = false;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int hi = (bits >> a) & 1;
            if (!(F[a] & 1)) {
                if (hi) skip = true;
                I[a] = F[a] >> 1;
            } else {
                w = w * 0.5;
                int k = (F[a] >> 1) + hi;
                if (k >= cn[a]) k -= cn[a];
                I[a] = k;
            }
        }
        if (skip) continue;
        s = s + w * pc[nid(gc, I[0], I[1], I[2])];
    }
    pf[t] = s;
}

void launch_refine_state(Ctx* c, const GridD& gc, const GridD& gf, const double* uc, const double* pc, double* uf,
                         double* pf)
{
    const unsigned bc = (unsigned)((ncells(gf) + kSeqT - 1) / kSeqT);
    const unsigned bn = (unsigned)((nnodes(gf) + kSeqT - 1) / kSeqT);
    if (gf.dim == 2) {
        k_refine_cells<2><<<bc, kSeqT, 0, c->s>>>(gc, gf, uc, uf);
        k_refine_nodes<2><<<bn, kSeqT, 0, c->s>>>(gc, gf, pc, pf);
    } else {
        k_refine_cells<3><<<bc, kSeqT, 0, c->s>>>(gc, gf, uc, uf);
        k_refine_nodes<3><<<bn, kSeqT, 0, c->s>>>(gc, gf, pc, pf);
    }
}

}  // namespace hb
