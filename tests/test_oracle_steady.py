"""Pins of the oracle's steady-state driver and grid sequencing (Sec. III.A,
Sec. III.C) against what the mathematics fixes: fields the interpolation
must reproduce exactly, the coarse mean it must keep, the closed-form steady
state of plane Poiseuille flow, and the paper's claim that a sequenced run
needs fewer fine-grid steps."""
import numpy as np
import pytest

from oracle import orc, steady


def _centres(g, a):
    return (np.arange(g.n[a]) + 0.5) * g.h


def _nodes(g, a):
    return np.arange(orc.node_shape(g)[::-1][a]) * g.h


# ------------------------------------------------------------- cell refinement

@pytest.mark.parametrize("dim,wall_axis", [(2, 1), (2, 0), (3, 2), (3, 0)])
def test_refine_cells_couette_exact(dim, wall_axis):
    # a velocity linear across the walls, equal to the wall velocities on
    # them (Couette flow) is linear everywhere including the wall ghosts, so
    # the refined field must be the same linear function at every fine cell
    n = [4] * dim
    bc = [(orc.PERIODIC, orc.PERIODIC)] * dim
    bc[wall_axis] = (orc.WALL, orc.WALL)
    comp = (wall_axis + 1) % dim
    U = 0.75
    top = [0.0, 0.0, 0.0]
    top[comp] = U
    gc = orc.make_grid(dim, n, 0.25, bc=bc, wall_u={(wall_axis, 1): tuple(top)})
    u = np.zeros(orc.cell_shape(gc, dim))
    shape = [1, 1, 1]
    shape[2 - wall_axis] = gc.n[wall_axis]
    u[comp] = (U * _centres(gc, wall_axis)).reshape(shape)
    uf = steady.refine_cells(gc, u)
    gf = steady.refined_grid(gc)
    shape[2 - wall_axis] = gf.n[wall_axis]
    want = np.zeros_like(uf)
    want[comp] = np.broadcast_to((U * _centres(gf, wall_axis)).reshape(shape), want[comp].shape)
    np.testing.assert_allclose(uf, want, rtol=0, atol=1e-15)


def test_refine_cells_keeps_coarse_mean():
    # conservative interpolation: the mean of the 2^d children is the parent
    rng = np.random.default_rng(3)
    for dim in (2, 3):
        gc = orc.lid_cavity(dim, 4)
        u = rng.standard_normal(orc.cell_shape(gc, dim))
        uf = steady.refine_cells(gc, u)
        if dim == 2:
            m = uf.reshape(dim, 1, 4, 2, 4, 2).mean(axis=(3, 5))
        else:
            m = uf.reshape(dim, 4, 2, 4, 2, 4, 2).mean(axis=(2, 4, 6))
        np.testing.assert_allclose(m, u, rtol=0, atol=1e-14)


def test_refine_cells_linear_interior():
    # away from the walls, a linear field is reproduced exactly
    gc = orc.lid_cavity(2, 8)
    x = _centres(gc, 0)[None, :]
    y = _centres(gc, 1)[:, None]
    u = np.zeros(orc.cell_shape(gc, 2))
    u[0, 0] = 0.3 + 1.7 * x - 0.9 * y
    u[1, 0] = -0.2 + 0.4 * x + 2.1 * y
    uf = steady.refine_cells(gc, u)
    gf = steady.refined_grid(gc)
    xf = _centres(gf, 0)[None, :]
    yf = _centres(gf, 1)[:, None]
    want0 = 0.3 + 1.7 * xf - 0.9 * yf
    want1 = -0.2 + 0.4 * xf + 2.1 * yf
    inner = (slice(2, -2), slice(2, -2))   # children of parents off the walls
    np.testing.assert_allclose(uf[0, 0][inner], want0[inner], rtol=0, atol=1e-14)
    np.testing.assert_allclose(uf[1, 0][inner], want1[inner], rtol=0, atol=1e-14)
    # next to a wall the ghost is the odd reflection, not the linear value
    assert abs(uf[0, 0][0, 5] - want0[0, 5]) > 1e-3


# ------------------------------------------------------------- node refinement

@pytest.mark.parametrize("dim", [2, 3])
def test_refine_nodes_multilinear_exact(dim):
    # multilinear interpolation reproduces multilinear functions exactly
    gc = orc.lid_cavity(dim, 4)
    gf = steady.refined_grid(gc)

    def field(g):
        X = _nodes(g, 0)[None, None, :]
        Y = _nodes(g, 1)[None, :, None]
        Z = _nodes(g, 2)[:, None, None] if dim == 3 else np.zeros((1, 1, 1))
        return 0.5 + 1.3 * X - 0.7 * Y + 2.2 * X * Y + 0.9 * Z - 1.1 * X * Z + 0.6 * Y * Z + 1.9 * X * Y * Z
    p = np.ascontiguousarray(np.broadcast_to(field(gc), orc.node_shape(gc)))
    pf = steady.refine_nodes(gc, p)
    want = np.broadcast_to(field(gf), orc.node_shape(gf))
    np.testing.assert_allclose(pf, want, rtol=0, atol=1e-14)


def test_refine_nodes_periodic_axis():
    # x periodic (n nodes, the last interval wraps to node 0), walls in y:
    # a field linear in y and constant in x is exact, and every coarse node
    # carries total weight 2 (itself and half of each of its two intervals),
    # so the sum of the fine values is twice the coarse sum along x
    gc = orc.make_grid(2, [4, 4], 0.25, bc=((orc.PERIODIC, orc.PERIODIC), (orc.WALL, orc.WALL)))
    gf = steady.refined_grid(gc)
    Y = _nodes(gc, 1)[:, None]
    p = np.ascontiguousarray(np.broadcast_to(0.4 - 1.5 * Y, orc.node_shape(gc)))
    pf = steady.refine_nodes(gc, p)
    np.testing.assert_allclose(pf[0], np.broadcast_to(0.4 - 1.5 * _nodes(gf, 1)[:, None], pf[0].shape), atol=1e-15)
    rng = np.random.default_rng(5)
    p = rng.standard_normal(orc.node_shape(gc))
    pf = steady.refine_nodes(gc, p)
    even_rows = pf[0, ::2, :]                  # fine rows on coarse rows
    np.testing.assert_allclose(even_rows.sum(axis=1), 2.0 * p[0].sum(axis=1), rtol=1e-14)


# ------------------------------------------------------------- steadiness

def test_state_change_definition():
    rng = np.random.default_rng(7)
    u = rng.standard_normal((2, 1, 5, 5))
    eps = 3e-6
    assert steady.state_change(u, u * (1.0 + eps)) == pytest.approx(eps, rel=1e-9)
    assert steady.state_change(np.zeros_like(u), u) == float("inf")
    v = u.copy()
    v[1, 0, 2, 3] += 0.5
    assert steady.state_change(u, v) == pytest.approx(0.5 / np.abs(u).max(), rel=1e-15)


@pytest.mark.parametrize("tol,bound", [(1e-5, 1e-3), (1e-10, 1e-8)])
def test_run_steady_reaches_poiseuille(tol, bound):
    # Newtonian plane Poiseuille flow (x periodic, walls at y = 0, 1, body
    # force G): at the discrete steady state the shear stress on every face
    # is -G (y - 1/2) exactly; a run stopped by the steadiness test is that
    # close to it, within the slowest mode's decay over a step
    ny, G, dt = 16, 1.0, 0.02
    g = orc.make_grid(2, [4, ny], 1.0 / ny, bc=((orc.PERIODIC, orc.PERIODIC), (orc.WALL, orc.WALL)))
    fl = orc.make_fluid(Re=1.0, HB=0.0, n=1.0, reg=orc.REG_YIELD_ONLY, f=(G, 0.0, 0.0))
    o = orc.make_step_opts()
    u = np.zeros(orc.cell_shape(g, 2))
    p = np.zeros(orc.node_shape(g))
    # from rest the velocity is zero and the relative change undefined
    r = steady.run_steady(g, fl, o, u, p, tol=tol, max_steps=5000, dt=dt)
    assert r["steady"] and r["rc"] == orc.OK and r["change"] < tol
    assert r["t"] == pytest.approx(r["steps"] * dt)
    ux = u[0, 0, :, 0]
    yf = np.arange(1, ny) / ny
    tau = (ux[1:] - ux[:-1]) * ny
    want = -G * (yf - 0.5)
    assert np.abs(tau - want).max() <= bound * G / 2


def test_run_steady_stops_at_max_steps():
    g = orc.lid_cavity(2, 8)
    fl = orc.make_fluid(Re=100.0, HB=1.0, n=1.0, Pa=1e3)
    u = np.zeros(orc.cell_shape(g, 2))
    p = np.zeros(orc.node_shape(g))
    r = steady.run_steady(g, fl, orc.make_step_opts(), u, p, tol=1e-5, max_steps=7)
    assert r["steps"] == 7 and not r["steady"] and r["rc"] == orc.ERR_NOCONV


def test_sequence_saves_fine_steps():
    # Sec. III.C: started from the refined steady coarse state, the fine grid
    # reaches steady state in fewer steps than from rest, at the same state
    fl = orc.make_fluid(Re=100.0, HB=1.0, n=1.0, Pa=1e3)
    o = orc.make_step_opts()
    g, u, p, reps = steady.sequence(orc.lid_cavity(2, 8), fl, o, 1)
    assert [r["steady"] for r in reps] == [True, True]
    assert g.n[0] == 16
    gd = orc.lid_cavity(2, 16)
    ud = np.zeros(orc.cell_shape(gd, 2))
    pd = np.zeros(orc.node_shape(gd))
    rd = steady.run_steady(gd, fl, o, ud, pd)
    assert rd["steady"]
    assert reps[1]["steps"] < rd["steps"]
    assert np.abs(u - ud).max() <= 1e-3 * np.abs(ud).max()
