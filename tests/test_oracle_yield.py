"""Pins of the oracle's yield diagnostics and cessation protocol (Sec. II,
Sec. IV) against closed forms and physics: simple shear, where the strain
rate and stress are known exactly; the plug of plane Poiseuille flow; rigid
motion, which never yields; and cessation, which stops at rest and stops
sooner under a larger yield stress."""
import math

import numpy as np
import pytest

from oracle import orc, yielding
from tests.test_oracle_pins import _poiseuille_run


def _couette(dim, wall_axis, U):
    n = [4] * dim
    bc = [(orc.PERIODIC, orc.PERIODIC)] * dim
    bc[wall_axis] = (orc.WALL, orc.WALL)
    comp = (wall_axis + 1) % dim
    top = [0.0, 0.0, 0.0]
    top[comp] = U
    g = orc.make_grid(dim, n, 0.25, bc=bc, wall_u={(wall_axis, 1): tuple(top)})
    u = np.zeros(orc.cell_shape(g, dim))
    shape = [1, 1, 1]
    shape[2 - wall_axis] = 4
    u[comp] = (U * (np.arange(4) + 0.5) * 0.25).reshape(shape)
    return g, u


@pytest.mark.parametrize("dim,wall_axis", [(2, 1), (2, 0), (3, 2), (3, 1)])
def test_simple_shear_strain_and_stress(dim, wall_axis):
    # du_c/dx_a = U everywhere (the wall ghosts continue the line): g = U/2,
    # and the stress magnitude is (2 g^n + HB)(1 - exp(-Pa g))
    U, HB, nidx, Pa = 0.5, 1.0, 0.7, 100.0
    g, u = _couette(dim, wall_axis, U)
    gam = yielding.strain_norm(g, u)
    np.testing.assert_allclose(gam, U / 2, rtol=1e-14)
    fl = orc.make_fluid(Re=1.0, HB=HB, n=nidx, Pa=Pa)
    tau = yielding.stress_norm(g, fl, u)
    want = (2 * (U / 2) ** nidx + HB) * (-math.expm1(-Pa * U / 2))
    np.testing.assert_allclose(tau, want, rtol=1e-13)
    mask, _ = yielding.yielded(g, fl, u)
    assert mask.all()
    # a slow shear stays below the yield stress in the regularised law
    g2, u2 = _couette(dim, wall_axis, 1e-4)
    assert not yielding.yielded(g2, fl, u2)[0].any()


def test_rigid_motion_never_yields():
    g = orc.make_grid(2, [8, 8], 1.0 / 8, bc=((orc.PERIODIC, orc.PERIODIC), (orc.PERIODIC, orc.PERIODIC)))
    fl = orc.make_fluid(Re=1.0, HB=0.5, Pa=1e3)
    u = np.zeros(orc.cell_shape(g, 2))
    u[0] = 0.7
    u[1] = -0.2
    assert np.abs(yielding.strain_norm(g, u)).max() == 0.0
    assert not yielding.yielded(g, fl, u)[0].any()


def test_poiseuille_plug_is_the_unyielded_band():
    # plane Poiseuille flow: |tau| = G |y - 1/2|, unyielded where it is below
    # HB, a band of width 2 HB / G about the centre line
    HB, Pa, ny = 0.25, 1e4, 32
    g, fl, u, p = _poiseuille_run(ny, HB, 1.0, Pa, dt=0.02)
    mask, tau = yielding.yielded(g, fl, u)
    col = mask[0, :, 0]
    yc = (np.arange(ny) + 0.5) * g.h
    plug = yc[~col]
    assert (mask == mask[:, :, :1]).all()
    assert abs(plug.max() - plug.min() + g.h - 2 * HB) <= 2 * g.h + 1e-12
    # contiguous band about the centre
    idx = np.nonzero(~col)[0]
    assert (np.diff(idx) == 1).all() and idx.min() < ny // 2 <= idx.max()


def _channel(HB, G=0.0, ny=16):
    g = orc.make_grid(2, [4, ny], 1.0 / ny, bc=((orc.PERIODIC, orc.PERIODIC), (orc.WALL, orc.WALL)))
    return g, orc.make_fluid(Re=1.0, HB=HB, n=1.0, Pa=1e3, f=(G, 0.0, 0.0))


def test_cessation_at_rest_needs_no_step():
    g, fl = _channel(0.5)
    u = np.zeros(orc.cell_shape(g, 2))
    p = np.zeros(orc.node_shape(g))
    r = yielding.run_cessation(g, fl, orc.make_step_opts(), u, p, dt=0.01)
    assert r == dict(steps=0, t=0.0, stopped=True, rc=orc.OK)


def test_cessation_stops_sooner_under_a_larger_yield_stress():
    # from the steady Poiseuille state of a Bingham fluid, the driving force
    # is removed; the flow stops in finite time, sooner for a larger HB
    g, fl, u0, p0 = _poiseuille_run(16, 0.1, 1.0, 1e3, dt=0.02)
    times = []
    for HB in (0.1, 0.3):
        gc, flc = _channel(HB)
        u, p = u0.copy(), p0.copy()
        r = yielding.run_cessation(gc, flc, orc.make_step_opts(), u, p, max_steps=5000, dt=0.005)
        assert r["stopped"] and r["rc"] == orc.OK and r["steps"] > 0
        assert not yielding.yielded(gc, flc, u)[0].any()
        times.append(r["t"])
    assert times[1] < times[0]
