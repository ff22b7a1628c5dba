// hb_stencil.h -- the tensor viscous stencil on LDS-staged cell blocks,
// shared by the tiled multigrid kernels and the single-workgroup coarse
// V-cycle: wall masks, face viscosity loads and div(beta gamma_dot(x)) with
// its diagonal (Sec. III.A, the coupled viscous solve).
#pragma once
#include "hb_dev.h"

namespace hb {

// bit (2a + side) set when face `side` (0 lo, 1 hi) of the cell along a is a
// wall face
template <int DIM>
__device__ inline int wall_mask(const GridD& g, const int G[3])
{
    int m = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (g.per[a]) continue;
        if (G[a] == 0) m |= 1 << (2 * a);
        if (G[a] == g.n[a] - 1) m |= 2 << (2 * a);
    }
    return m;
}

// The 2*DIM face viscosities of cell G on a coarse level, [2a + side].
// The kernels load them into registers together with the tile fill, so no
// global load waits between the barriers of a sweep.  A cell outside the box
// (taking no part) reads the faces of the nearest cell.
template <int DIM, typename R>
__device__ inline void load_faces(const GridD& g, const R* __restrict__ beta, const int G[3], R* bf)
{
    int C[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) C[a] = G[a] < 0 ? 0 : (G[a] >= g.n[a] ? g.n[a] - 1 : G[a]);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            int F[3] = {C[0], C[1], C[2]};
            F[a] += side;
            if (g.per[a] && F[a] == g.n[a]) F[a] = 0;
            bf[2 * a + side] = beta[foffset(g, a) + fid(g, a, F[0], F[1], F[2])];
        }
    }
}

// div(beta gamma_dot(x))_c at a cell of an LDS block holding every
// component with a halo: component a at s + a * ns, y stride sx, z stride
// sxy; l0 the cell's index.  Returns it and the diagonal of the homogeneous
// operator.  FINE: face viscosities from the eta/Re block `e` (mean of the two
// cells, the interior cell on wall faces); otherwise the cell's face
// viscosities `bfc` as loaded by load_faces.  Same arithmetic sequence per
// face as the global-memory operator.
// ihh = 1/h^2 (computed by the caller as R(1) / (h * h)).
template <int DIM, bool FINE, typename R>
__device__ inline R visc_div_ih(const R* bfc, const R* s, int ns, int sx, int sxy, const R* e, int c, int wm, int l0,
                                R dt, R ihh, R* diag)
{
    // Every flux carries one factor 1/h and the divergence another, so the
    // fluxes are formed in units of h and the sum is scaled by 1/h^2 once
    // (no divisions in the stencil).
    const int off[3] = {1, sx, sxy};
    const R* sc = s + c * ns;
    R acc = 0, coefsum = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        R flux[2];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int lL = l0 + (side - 1) * off[a];
            const int lR = lL + off[a];
            const bool wall = (wm >> (2 * a + side)) & 1;
            // Every value is loaded whether or not the face is a wall (all
            // positions lie in the staged halo) and the wall case is chosen
            // by multiplying with keep = 0 or 1 rather than by a select, so
            // the compiler cannot move loads under a per-lane branch and a
            // stencil's loads issue together.  The products and sums are the
            // ones of the wall and interior formulas (x * 1 = x, x + 0 = x;
            // only the sign of a zero can differ).
            const R keep = wall ? R(0) : R(1);
            R bf;
            if (FINE) {
                const R e0 = e[l0], eL = e[lL], eR = e[lR];
                bf = e0 * (R(1) - keep) + R(0.5) * (eL + eR) * keep;
            } else {
                bf = bfc[2 * a + side];
            }
            const R dn = sc[lR] - sc[lL];
            R f;
            if (a == c) {
                f = bf * dn;
            } else {
                const R* sa = s + a * ns;
                // mean of the two cells' centred transverse differences
                // (dropped on a wall face)
                const R cross = R(0.25) * ((sa[lL + off[c]] - sa[lL - off[c]]) + (sa[lR + off[c]] - sa[lR - off[c]]));
                f = bf * R(0.5) * (dn + cross * keep);
            }
            flux[side] = f;
            coefsum += (wall ? R(2) : R(1)) * ((a == c) ? R(1) : R(0.5)) * bf;
        }
        acc += flux[1] - flux[0];
    }
    if (diag) *diag = R(1) + dt * coefsum * ihh;
    return acc * ihh;
}

// the same with 1/h^2 formed from the grid
template <int DIM, bool FINE, typename R>
__device__ inline R visc_div_lds(const GridD& g, const R* bfc, const R* s, int ns, int sx, int sxy, const R* e, int c,
                                 int wm, int l0, R dt, R* diag)
{
    const R h = (R)g.h;
    return visc_div_ih<DIM, FINE, R>(bfc, s, ns, sx, sxy, e, c, wm, l0, dt, R(1) / (h * h), diag);
}

}  // namespace hb
