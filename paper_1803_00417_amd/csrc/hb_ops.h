// hb_ops.h -- pointwise device operators of the global-memory kernels: the
// tensor viscous flux and divergence, the MAC Laplacian and the assembled Q1
// stiffness, all reading global memory with boundary values produced on the
// fly; and the Q1 stiffness on a staged node block (the tiled and the
// single-workgroup nodal kernels).
#pragma once
#include "hb_internal.h"

namespace hb {

// value of component c; ZI: the interior is zero and only wall values remain
template <bool HOM, bool ZI, class G>
__device__ inline double uval(const G& g, const double* __restrict__ u, int c, int i, int j, int k)
{
    if (!ZI) return cval<HOM>(g, u + (long)c * ncells(g), c, i, j, k);
    int p[3] = {i, j, k};
    for (int a = 0; a < g.dim; ++a) {
        if (p[a] >= 0 && p[a] < g.n[a]) continue;
        if (g.per[a]) continue;
        return 2.0 * g.wall_u[a][p[a] < 0 ? 0 : 1][c];
    }
    return 0.0;
}

// flux of component c through the face normal to a whose hi-side cell is
// (i,j,k): beta (du_c/dx_a + du_a/dx_c)/2 with the transverse derivative
// averaged from the two cells' centred differences (zero on wall faces)
template <bool HOM, bool ZI, class G>
__device__ inline double visc_flux(const G& g, const double* __restrict__ beta, const double* __restrict__ u,
                                   int c, int a, int i, int j, int k)
{
    int R[3] = {i, j, k}, L[3] = {i, j, k};
    L[a] -= 1;
    const bool wall = !g.per[a] && (R[a] == 0 || R[a] == g.n[a]);
    int fp[3] = {i, j, k};
    if (g.per[a] && fp[a] == g.n[a]) fp[a] = 0;
    const double bf = beta[foffset(g, a) + fid(g, a, fp[0], fp[1], fp[2])];
    const double uR = uval<HOM, ZI>(g, u, c, R[0], R[1], R[2]);
    const double uL = uval<HOM, ZI>(g, u, c, L[0], L[1], L[2]);
    const double dn = (uR - uL) / g.h;
    if (a == c) return bf * dn;
    if (wall) return bf * 0.5 * dn;
    wrap(g, R);
    wrap(g, L);
    int Lp[3] = {L[0], L[1], L[2]}, Lm[3] = {L[0], L[1], L[2]};
    int Rp[3] = {R[0], R[1], R[2]}, Rm[3] = {R[0], R[1], R[2]};
    Lp[c] += 1; Lm[c] -= 1; Rp[c] += 1; Rm[c] -= 1;
    const double dL = (uval<HOM, ZI>(g, u, a, Lp[0], Lp[1], Lp[2]) - uval<HOM, ZI>(g, u, a, Lm[0], Lm[1], Lm[2])) / (2.0 * g.h);
    const double dR = (uval<HOM, ZI>(g, u, a, Rp[0], Rp[1], Rp[2]) - uval<HOM, ZI>(g, u, a, Rm[0], Rm[1], Rm[2])) / (2.0 * g.h);
    const double cross = 0.5 * (dL + dR);
    return bf * 0.5 * (dn + cross);
}

template <bool HOM, bool ZI, class G>
__device__ inline double visc_div_at(const G& g, const double* __restrict__ beta, const double* __restrict__ u,
                                     int c, int i, int j, int k)
{
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < g.dim; ++a) {
        int hi[3] = {i, j, k};
        hi[a] += 1;
        s += (visc_flux<HOM, ZI>(g, beta, u, c, a, hi[0], hi[1], hi[2]) - visc_flux<HOM, ZI>(g, beta, u, c, a, i, j, k)) / g.h;
    }
    return s;
}

// diagonal of the homogeneous operator for component c
template <class G>
__device__ inline double visc_diag(const G& g, const double* __restrict__ beta, double dt, int c, int i, int j, int k)
{
    double coef = 0.0;
    for (int a = 0; a < g.dim; ++a)
        for (int side = 0; side < 2; ++side) {
            int q[3] = {i, j, k};
            q[a] += side;
            const bool wall = !g.per[a] && (q[a] == 0 || q[a] == g.n[a]);
            if (g.per[a] && q[a] == g.n[a]) q[a] = 0;
            const double bf = beta[foffset(g, a) + fid(g, a, q[0], q[1], q[2])];
            const double s = (a == c) ? 1.0 : 0.5;
            coef += (wall ? 2.0 : 1.0) * s * bf;
        }
    return 1.0 + dt * coef / (g.h * g.h);
}

// Index of the face neighbour of cell (i,j,k) along axis a, d = -1 or +1,
// wrapped on periodic axes.  Always in range: beyond a wall it is the cell
// itself, with ok = false, so callers load without branching and select.
template <int DIM>
__device__ inline long nb_cell(const GridD& g, int i, int j, int k, int a, int d, bool& ok)
{
    int p[3] = {i, j, k};
    const int n = g.n[a];
    int v = p[a] + d;
    ok = true;
    if (v < 0 || v >= n) {
        if (g.per[a]) v = v < 0 ? v + n : v - n;
        else { ok = false; v = p[a]; }
    }
    p[a] = v;
    return cid(g, p[0], p[1], p[2]);
}

// L_mac x at one cell, as the divergence of face gradients (zero flux
// through walls); the two factors 1/h are applied once, as 1/h^2.  All
// neighbour loads issue before any is used.
template <int DIM, typename R>
__device__ inline R mac_lap_at(const GridD& g, const R* __restrict__ x, int i, int j, int k)
{
    const R h = (R)g.h;
    const R xc = x[cid(g, i, j, k)];
    R xn[DIM][2];
    bool ok[DIM][2];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        xn[a][0] = x[nb_cell<DIM>(g, i, j, k, a, -1, ok[a][0])];
        xn[a][1] = x[nb_cell<DIM>(g, i, j, k, a, +1, ok[a][1])];
    }
    R s = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const R Fhi = ok[a][1] ? xn[a][1] - xc : R(0);
        const R Flo = ok[a][0] ? xc - xn[a][0] : R(0);
        s += Fhi - Flo;
    }
    return s * (R(1) / (h * h));
}

__device__ inline double q1_ke(int dim, double h, int k)
{
    if (dim == 2) return k == 0 ? 2.0 / 3.0 : (k == 1 ? -1.0 / 6.0 : -1.0 / 3.0);
    return (k == 0 ? 1.0 / 3.0 : (k == 1 ? 0.0 : -1.0 / 12.0)) * h;
}

// elements along axis a containing node i and node i + d (d in -1, 0, 1)
__device__ inline int node_cnt(const GridD& g, int a, int i, int d)
{
    if (g.per[a]) return d == 0 ? 2 : 1;
    const int lo = i >= 1, hi = i <= g.n[a] - 1;
    return d == 0 ? lo + hi : (d > 0 ? hi : lo);
}

// K x at node G from an LDS node block with y stride sx and z stride sxy
// (local index l), and the diagonal
template <int DIM, typename R>
__device__ inline R block_K(const GridD& g, const R* s, int sx, int sxy, const int G[3], int l, R* diag)
{
    int cnt[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) cnt[a][d] = a < DIM ? node_cnt(g, a, G[a], d - 1) : (d == 1 ? 1 : 0);
    R acc = 0;
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int k = (dx != 0) + (dy != 0) + (dz != 0);
                if (DIM == 3 && k == 1) continue;   // the 3D Q1 face-neighbour weight is exactly 0
                const R w = (R)(q1_ke(DIM, g.h, k) * (double)(cnt[0][dx + 1] * cnt[1][dy + 1] * cnt[2][dz + 1]));
                acc += w * s[l + dz * sxy + dy * sx + dx];
            }
    if (diag) *diag = (R)(q1_ke(DIM, g.h, 0) * (double)(cnt[0][1] * cnt[1][1] * cnt[2][1]));
    return acc;
}

// value of x at node (i,j,k) (periodic wrap; outside a wall reads 0: its
// stencil weight is zero)
template <int DIM, typename R>
__device__ inline R node_fetch(const GridD& g, const R* __restrict__ x, int i, int j, int k)
{
    int p[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int nn = nnode(g, a);
        if (p[a] >= 0 && p[a] < nn) continue;
        if (!g.per[a]) return R(0);
        p[a] = p[a] < 0 ? p[a] + nn : p[a] - nn;
    }
    return x[nid(g, p[0], p[1], p[2])];
}

// (K x) at node (i,j,k) from global memory, and the diagonal
template <int DIM>
__device__ inline double K_glob(const GridD& g, const double* __restrict__ x, int i, int j, int k, double* diag)
{
    const int G[3] = {i, j, k};
    double acc = 0.0;
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int kk = (dx != 0) + (dy != 0) + (dz != 0);
                const int c0 = node_cnt(g, 0, G[0], dx), c1 = node_cnt(g, 1, G[1], dy);
                const int c2 = DIM == 3 ? node_cnt(g, 2, G[2], dz) : 1;
                const double w = q1_ke(DIM, g.h, kk) * (double)(c0 * c1 * c2);
                acc += w * node_fetch<DIM, double>(g, x, G[0] + dx, G[1] + dy, G[2] + dz);
            }
    if (diag) {
        const int c2 = DIM == 3 ? node_cnt(g, 2, G[2], 0) : 1;
        *diag = q1_ke(DIM, g.h, 0) * (double)(node_cnt(g, 0, G[0], 0) * node_cnt(g, 1, G[1], 0) * c2);
    }
    return acc;
}

}  // namespace hb
