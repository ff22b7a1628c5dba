"""Steady-state driver, grid sequencing and state refinement of the oracle.

TEST INFRASTRUCTURE ONLY: the test suite uses this module to check the HIP
library's steady-state driver and refinement kernels.  The product path never
imports it, and it imports nothing from the product package.

What it follows:
- the steadiness test that closes the description of the projection
  (Sec. III.A): the run is steady once the largest relative change of the
  velocity over one step is below 1e-5.  The printed quotient divides by u^m
  cell by cell, which is undefined where u^m vanishes (at rest, on the axis of
  a symmetric flow); the reading taken here divides the largest change by the
  largest velocity, max|u^(m+1) - u^m| / max|u^m|, the "maximum relative
  change in the velocity field" of Sec. IV;
- grid sequencing (Sec. III.C): a low-resolution run is advanced to steady
  state, the state is carried to a grid refined by two everywhere, and the run
  continues there; repeated once per refinement.  The paper does not name the
  interpolation.  The reading taken here: cell-centred velocity by
  conservative linear interpolation with central slopes (each coarse cell's
  mean is kept, linear fields are reproduced), where a neighbour beyond a wall
  is the wall ghost 2 u_wall - u (the odd reflection of the step's boundary
  treatment) and beyond a periodic face the wrapped cell; nodal pressure by
  multilinear interpolation between the coarse nodes (wrapped on periodic
  axes).

Plain loops over cells and nodes: meant for the small grids of the tests.
"""
import numpy as np

from . import orc


def refined_grid(gc):
    """The grid with every used axis refined by two: half the spacing, the
    same boundaries and wall velocities."""
    n = [2 * gc.n[a] for a in range(gc.dim)]
    bc = [(gc.bc[a][0], gc.bc[a][1]) for a in range(gc.dim)]
    wall = {(a, s): tuple(gc.wall_u[a][s][c] for c in range(3)) for a in range(gc.dim) for s in range(2)}
    return orc.make_grid(gc.dim, n, gc.h / 2.0, bc=bc, wall_u=wall)


def _cell_neighbour(gc, u, comp, C, a, side):
    """u[comp] at the cell next to C along axis a (side -1 or +1): the cell
    itself inside the grid, the wrapped cell across a periodic face, the wall
    ghost 2 u_wall - u(C) across a wall."""
    N = [C[0], C[1], C[2]]
    N[a] += side
    if 0 <= N[a] < gc.n[a]:
        return u[comp, N[2], N[1], N[0]]
    s = 0 if side < 0 else 1
    if gc.bc[a][s] == orc.PERIODIC:
        N[a] %= gc.n[a]
        return u[comp, N[2], N[1], N[0]]
    return 2.0 * gc.wall_u[a][s][comp] - u[comp, C[2], C[1], C[0]]


def refine_cells(gc, u):
    """Velocity on the refined grid (Sec. III.C, reading above).  u: (dim, nz,
    ny, nx) on gc.  Child value = u(C) + sum over axes of (+-1/4) times the
    central slope (u(C+1) - u(C-1)) / 2, + for the child on the high half of
    its parent along that axis, axes taken in order x, y, z."""
    dim = gc.dim
    nf = [2 * gc.n[a] if a < dim else 1 for a in range(3)]
    out = np.zeros((dim, nf[2], nf[1], nf[0]))
    for comp in range(dim):
        for k in range(nf[2]):
            for j in range(nf[1]):
                for i in range(nf[0]):
                    F = (i, j, k)
                    C = [F[a] // 2 if a < dim else 0 for a in range(3)]
                    v = u[comp, C[2], C[1], C[0]]
                    for a in range(dim):
                        lo = _cell_neighbour(gc, u, comp, C, a, -1)
                        hi = _cell_neighbour(gc, u, comp, C, a, +1)
                        slope = 0.5 * (hi - lo)
                        v = v + (0.25 if F[a] % 2 else -0.25) * slope
                    out[comp, k, j, i] = v
    return out


def refine_nodes(gc, p):
    """Pressure on the nodes of the refined grid (Sec. III.C, reading above).
    p: nodal array of gc.  A fine node at an even index along an axis sits on
    a coarse node, at an odd index halfway between two; the value is the sum,
    over the coarse nodes it lies between (combinations taken with the x
    choice varying fastest, low before high), of the product of the weights
    (1 or 1/2) times the coarse value."""
    dim = gc.dim
    ncn = orc.node_shape(gc)[::-1]            # coarse node counts, x first
    gf = refined_grid(gc)
    nfn = orc.node_shape(gf)[::-1]
    out = np.zeros(orc.node_shape(gf))
    for K in range(nfn[2]):
        for J in range(nfn[1]):
            for I in range(nfn[0]):
                F = (I, J, K)
                s = 0.0
                for bits in range(1 << dim):
                    w = 1.0
                    idx = [0, 0, 0]
                    skip = False
                    for a in range(dim):
                        hi = (bits >> a) & 1
                        if F[a] % 2 == 0:
                            if hi:
                                skip = True
                                break
                            idx[a] = F[a] // 2
                        else:
                            w = w * 0.5
                            idx[a] = ((F[a] - 1) // 2 + hi) % ncn[a]
                    if skip:
                        continue
                    s = s + w * p[idx[2], idx[1], idx[0]]
                out[K, J, I] = s
    return out


def state_change(u_old, u_new):
    """max|u_new - u_old| / max|u_old| (Sec. III.A, reading above); infinite
    when u_old is zero everywhere."""
    ref = np.abs(u_old).max()
    d = np.abs(u_new - u_old).max()
    return d / ref if ref > 0.0 else float("inf")


def run_steady(g, fl, o, u, p, tol=1e-5, max_steps=10000, dt=0.0):
    """Step (u, p) in place until the change of one step is below tol
    (Sec. III.A) or max_steps steps have run.  dt <= 0: the CFL step of every
    step.  Returns dict(steps, t, change, steady, rc); a step that returns
    anything but OK ends the run with its code (the time and change of a
    step whose solve hit its cycle limit are counted, those of a step that
    failed otherwise are not)."""
    t = 0.0
    change = float("inf")
    for m in range(max_steps):
        u_old = u.copy()
        rep, rc = orc.step(g, fl, o, u, p, dt)
        if rc not in (orc.OK, orc.ERR_NOCONV):
            return dict(steps=m + 1, t=t, change=change, steady=False, rc=rc)
        t += rep.dt
        change = state_change(u_old, u)
        if rc == orc.ERR_NOCONV:
            # a solve of this step hit its cycle limit: the step ran, the run stops
            return dict(steps=m + 1, t=t, change=change, steady=False, rc=rc)
        if change < tol:
            return dict(steps=m + 1, t=t, change=change, steady=True, rc=orc.OK)
    return dict(steps=max_steps, t=t, change=change, steady=False, rc=orc.ERR_NOCONV)


def sequence(gc, fl, o, levels, tol=1e-5, max_steps=10000):
    """Grid sequencing (Sec. III.C): from rest on gc to steady state, then
    refine the state and continue to steady state, `levels` refinements in
    all.  Returns (grid, u, p, reports) with one report per grid."""
    g = gc
    u = np.zeros(orc.cell_shape(g, g.dim))
    p = np.zeros(orc.node_shape(g))
    reports = []
    for lev in range(levels + 1):
        if lev > 0:
            u = refine_cells(g, u)
            p = refine_nodes(g, p)
            g = refined_grid(g)
        r = run_steady(g, fl, o, u, p, tol, max_steps)
        reports.append(r)
        # a grid not steady within max_steps is refined all the same
        if r["rc"] not in (orc.OK, orc.ERR_NOCONV):
            break
    return g, u, p, reports
