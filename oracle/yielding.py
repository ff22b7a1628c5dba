"""Yield-surface diagnostics and the cessation protocol of the oracle.

TEST INFRASTRUCTURE ONLY: the test suite uses this module to check the HIP
library's yield diagnostics and cessation driver.  The product path never
imports it, and it imports nothing from the product package.

What it follows:
- the yield criterion (Sec. II, Sec. IV): the material is yielded where the
  stress magnitude exceeds the yield stress.  In the dimensionless variables
  of Sec. IV the deviatoric stress is 2 eta gamma_dot, its magnitude (the
  scaled norm of Sec. II) is 2 eta g with g = |gamma_dot|, and the yield
  stress is HB (the unregularised law gives 2 g^n + HB, which tends to HB as
  g -> 0).  A cell is yielded when 2 eta g > HB, with eta the regularised
  viscosity of the step and g from the same centred differences and wall
  ghosts;
- the cessation experiment (Sec. IV): from a steady state the lid is stopped
  and the run continues until the whole domain is unyielded; the time taken
  is the cessation time.  The stopped lid is a grid whose wall velocities are
  zero; the state carries over.

Plain loops: meant for the small grids of the tests.
"""
import numpy as np

from . import orc


def strain_norm(g, u):
    """g = |gamma_dot| per cell: gamma_dot = (grad u + grad u^T)/2 by centred
    differences, a neighbour beyond a wall being the ghost 2 u_wall - u, beyond
    a periodic face the wrapped cell; |A| = sqrt(sum A_ij^2 / 2) (Sec. II)."""
    dim = g.dim
    n = [g.n[a] for a in range(3)]
    out = np.zeros((n[2], n[1], n[0]))

    def val(comp, C, a, s):
        K = list(C)
        K[a] += s
        if 0 <= K[a] < n[a]:
            return u[comp, K[2], K[1], K[0]]
        side = 0 if s < 0 else 1
        if g.bc[a][side] == orc.PERIODIC:
            K[a] %= n[a]
            return u[comp, K[2], K[1], K[0]]
        return 2.0 * g.wall_u[a][side][comp] - u[comp, C[2], C[1], C[0]]

    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                C = (i, j, k)
                G = [[(val(c, C, a, +1) - val(c, C, a, -1)) / (2.0 * g.h) for c in range(dim)] for a in range(dim)]
                s = 0.0
                for a in range(dim):
                    for c in range(dim):
                        e = 0.5 * (G[a][c] + G[c][a])
                        s += e * e
                out[k, j, i] = np.sqrt(0.5 * s)
    return out


def stress_norm(g, fl, u):
    """2 eta g per cell (eta the regularised viscosity of the oracle)."""
    eta, rc = orc.viscosity(g, fl, u)
    assert rc == orc.OK
    return 2.0 * eta.reshape(g.n[2], g.n[1], g.n[0]) * strain_norm(g, u)


def yielded(g, fl, u):
    """Boolean mask of the yielded cells (2 eta g > HB) and the stress norm."""
    tau = stress_norm(g, fl, u)
    return tau > fl.HB, tau


def run_cessation(g, fl, o, u, p, max_steps=10000, dt=0.0):
    """The cessation protocol (Sec. IV) on a grid whose walls are at rest:
    step (u, p) in place until no cell is yielded (tested before the first
    step and after each), or max_steps steps.  Returns dict(steps, t,
    stopped, rc)."""
    assert fl.HB > 0.0
    t = 0.0
    if not yielded(g, fl, u)[0].any():
        return dict(steps=0, t=0.0, stopped=True, rc=orc.OK)
    for m in range(max_steps):
        rep, rc = orc.step(g, fl, o, u, p, dt)
        if rc not in (orc.OK, orc.ERR_NOCONV):
            return dict(steps=m + 1, t=t, stopped=False, rc=rc)
        t += rep.dt
        if rc == orc.ERR_NOCONV:
            return dict(steps=m + 1, t=t, stopped=False, rc=rc)
        if not yielded(g, fl, u)[0].any():
            return dict(steps=m + 1, t=t, stopped=True, rc=orc.OK)
    return dict(steps=max_steps, t=t, stopped=False, rc=orc.ERR_NOCONV)
