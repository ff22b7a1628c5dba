"""Stability of the step at low Reynolds number (CPU oracle, no GPU).

Sec. IV runs the lid-driven cavity at Re = 1 (Bi = 10, Pa = 400) to a steady
state.  These pins fix the readings of the predictor forcing and of the
viscous time discretisation that the step takes (both options of the step,
shared with the HIP library):

- with the explicit stress divergence in the forcing of the Taylor
  prediction (as eq:iamr:extrap prints it) the face states take
  (dt/2) div tau^m, which amplifies every mode whose diffusion number
  dt eta/(Re h^2) is large: a Newtonian Re = 1 cavity at dt = h/2 on 16^2
  (diffusion number 8) turns non-finite within a few steps;
- without it (the default) the same cavity stays bounded and settles;
- the Crank-Nicolson update of Sec. III.A keeps the Bingham Re = 1 cavity
  bounded but, as it is not L-stable, its stiff modes keep the velocity
  changing by far more than the 1e-5 steadiness bound, while backward Euler
  (theta = 1) damps them and the flow settles.
"""
import numpy as np
import pytest

from oracle import orc


def _run(n, fl, steps, dt_fixed, **opt):
    g = orc.lid_cavity(2, n)
    o = orc.make_step_opts(**opt)
    u = np.zeros(orc.cell_shape(g, 2))
    p = np.zeros(orc.node_shape(g))
    umax, change = 0.0, np.inf
    for s in range(steps):
        uo = u.copy()
        rep, rc = orc.step(g, fl, o, u, p, 0.5 * g.h if dt_fixed else 0.0)
        if rc != orc.OK:
            return rc, s, umax, change
        umax = max(umax, np.abs(u).max())
        change = np.abs(u - uo).max() / np.abs(u).max()
    return orc.OK, steps, umax, change


NEWTONIAN_RE1 = dict(Re=1.0, HB=0.0, n=1.0, Pa=1e3, reg=orc.REG_YIELD_ONLY)
BINGHAM_RE1 = dict(Re=1.0, HB=10.0, n=1.0, Pa=400.0)    # the case of Sec. IV


def test_printed_predictor_forcing_is_unstable_at_re1():
    rc, s, umax, _ = _run(16, orc.make_fluid(**NEWTONIAN_RE1), 30, True, pred_visc=1)
    assert rc == orc.ERR_NONFINITE and s < 30


def test_newtonian_re1_cavity_settles_without_it():
    rc, s, umax, change = _run(16, orc.make_fluid(**NEWTONIAN_RE1), 250, True)
    assert rc == orc.OK
    # the impulsive start overshoots the lid speed in the first step only
    # (cell values next to the moving corner); the flow then stays below it
    assert umax < 1.1
    assert change < 1e-5


def test_newtonian_re1_stays_below_lid_speed_after_start():
    g = orc.lid_cavity(2, 16)
    fl = orc.make_fluid(**NEWTONIAN_RE1)
    o = orc.make_step_opts()
    u = np.zeros(orc.cell_shape(g, 2))
    p = np.zeros(orc.node_shape(g))
    for s in range(60):
        rep, rc = orc.step(g, fl, o, u, p, 0.5 * g.h)
        assert rc == orc.OK
        if s >= 5:
            assert np.abs(u).max() <= 1.0


def test_bingham_re1_cavity_stays_bounded():
    rc, s, umax, change = _run(32, orc.make_fluid(**BINGHAM_RE1), 100, False)
    assert rc == orc.OK and umax <= 1.0


def test_bingham_re1_crank_nicolson_does_not_settle_backward_euler_does():
    fl = orc.make_fluid(**BINGHAM_RE1)
    rc, _, umax_cn, change_cn = _run(16, fl, 300, False)
    assert rc == orc.OK and umax_cn <= 1.0
    assert change_cn > 1e-2
    rc, _, umax_be, change_be = _run(16, fl, 300, False, theta=1.0)
    assert rc == orc.OK and umax_be <= 1.0
    assert change_be < 1e-4
