"""Mixed precision (FP32 V-cycles inside FP64 defect correction) against the
FP64 oracle, through the C ABI.

A mixed solve is a different iteration from the FP64 one, so it is compared
at the solver tolerance, not bit for bit: both sides stop at
|b - A x|_inf <= 1e-10 |b|_inf, so each is within kappa * 1e-10 (relative)
of the exact discrete solution, and the two within twice that.  On these
grids (h >= 1/96) the condition numbers are at most ~1e4 (nodal and MAC
Poisson ~ (n/pi)^2, the Helmholtz-type viscous operator far less), which
gives the 2e-6 bound used below; the residual check is the exact criterion.
"""
import numpy as np
import pytest

from oracle import orc
from paper_1803_00417_amd import inputs
from tests.helpers import dev, hip_objs, host, lid_spec, oracle_objs, rel_err, spec

pytestmark = pytest.mark.gpu

hb = pytest.importorskip("paper_1803_00417_amd.hb")

CASES = {
    "lid2d_96x48": lambda: spec(2, [96, 48], h=1.0 / 96, wall_u={(1, 1): (1.0, 0.0, 0.0)}, Re=50.0, HB=2.0,
                                nidx=0.7, Pa=300.0),
    "lid3d_16": lambda: lid_spec(3, 16, Re=100.0, HB=2.0, Pa=1e3),
    "chan2d_8x32": lambda: spec(2, [8, 32], h=1.0 / 32, bc=((1, 1), (0, 0)), Re=1.0, HB=0.2, Pa=1e3,
                                f=(1.0, 0.0, 0.0)),
    "mix3d_12x16x8": lambda: spec(3, [12, 16, 8], h=1.0 / 16, bc=((1, 1), (0, 0), (0, 0)),
                                  wall_u={(2, 1): (1.0, 0.5, 0.0)}, Re=20.0, HB=1.0, nidx=0.6, Pa=200.0),
    # tiles cut in every axis: 24 cells against 32-wide tiles, 12 against
    # 8- and 16-deep ones, 6 against 4 and 8, with a periodic axis across them
    "rag3d_24x12x6": lambda: spec(3, [24, 12, 6], h=1.0 / 24, bc=((0, 0), (0, 0), (1, 1)),
                                  wall_u={(1, 1): (1.0, 0.0, 0.3)}, Re=30.0, HB=1.5, nidx=0.8, Pa=300.0),
}

SOLVE_TOL = 2e-6


def _say(*a):
    print(*a, flush=True)


def _system(s, op, go):
    d = s["dim"]
    eta = None
    if op == hb.OP_VISC:
        sh = orc.cell_shape(go, d)
        eta = inputs.positive_cells(orc.cell_shape(go)[1:], seed=7, lo=0.0, hi=4.5)
    elif op == hb.OP_MAC:
        sh = orc.cell_shape(go)[1:]
    else:
        sh = orc.node_shape(go)
    rhs = inputs.smooth_cells(sh if len(sh) == 4 else (1,) + tuple(sh), seed=8).reshape(sh)
    rhs = rhs + inputs.random_cells(sh, seed=9, scale=0.1)
    return sh, eta, rhs


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("op", [hb.OP_VISC, hb.OP_MAC, hb.OP_NODAL])
@pytest.mark.parametrize("krylov", [0, 1])
def test_mixed_solve_reaches_fp64_tolerance(case, op, krylov):
    _say("mixed solve", case, op, krylov)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    g, fl = hip_objs(s)
    ctx = hb.Context(g, fl, hb.make_step_opts())
    sh, eta, rhs = _system(s, op, go)
    dt = 0.5 * go.h
    xo, rco, repo = orc.mg_solve(go, flo, op, eta, dt, rhs, tol=1e-10, krylov=krylov)
    assert rco == orc.OK
    xd = dev(np.zeros(sh))
    rep, rc = ctx.mg_solve(op, dev(eta) if eta is not None else None, dt, dev(rhs), xd,
                           hb.mg_opts(tol=1e-10, krylov=krylov, precision=hb.PREC_MIXED))
    assert rc == hb.OK and rep.rel_resid <= 1e-10
    # FP32 cycles contract about as well as FP64 ones until the FP64
    # residual reaches the tolerance
    assert rep.cycles <= repo.cycles + 2, (rep.cycles, repo.cycles)
    err = rel_err(host(xd).reshape(sh), xo)
    _say("  cycles mixed/fp64 %d/%d  error vs oracle %.3e" % (rep.cycles, repo.cycles, err))
    assert err < SOLVE_TOL


@pytest.mark.parametrize("case", ["lid2d_96x48", "lid3d_16"])
@pytest.mark.parametrize("op", [hb.OP_VISC, hb.OP_MAC, hb.OP_NODAL])
def test_mixed_cycle_contraction_matches_fp64(case, op):
    # after each of the first cycles the FP64 residual of the mixed solve is
    # within a factor 2 of the FP64 solve's (the FP32 correction is accurate
    # to ~1e-7 relative, far below one cycle's contraction)
    _say("mixed contraction", case, op)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    g, fl = hip_objs(s)
    ctx = hb.Context(g, fl, hb.make_step_opts())
    sh, eta, rhs = _system(s, op, go)
    dt = 0.5 * go.h
    for k in (1, 2, 3):
        res = []
        for prec in (hb.PREC_FP64, hb.PREC_MIXED):
            xd = dev(np.zeros(sh))
            rep, rc = ctx.mg_solve(op, dev(eta) if eta is not None else None, dt, dev(rhs), xd,
                                   hb.mg_opts(max_cycles=k, fixed=1, precision=prec))
            res.append(rep.rel_resid)
        assert res[1] <= 2.0 * res[0] + 1e-12, (k, res)


def _steps(s, nsteps, dt=0.0, u0_seed=None):
    go, flo = oracle_objs(s)
    g, fl = hip_objs(s)
    ctx = hb.Context(g, fl, hb.make_step_opts(precision=hb.PREC_MIXED))
    oo = orc.make_step_opts()
    d = s["dim"]
    u = np.zeros(orc.cell_shape(go, d))
    if u0_seed is not None:
        u = inputs.smooth_cells(u.shape, seed=u0_seed, scale=0.5)
    p = np.zeros(orc.node_shape(go))
    ud, pd = dev(u), dev(p)
    worst = 0.0
    for k in range(nsteps):
        rep_o, rc = orc.step(go, flo, oo, u, p, dt)
        assert rc == orc.OK
        rep = ctx.step(ud, pd, dt)
        assert rep.mac.rel_resid <= 1e-10 and rep.visc.rel_resid <= 1e-10 and rep.proj.rel_resid <= 1e-10
        eu = rel_err(host(ud).reshape(u.shape), u)
        pscale = max(np.abs(p).max(), np.abs(u).max() ** 2)
        ep = np.abs(host(pd).reshape(p.shape) - p).max() / pscale
        worst = max(worst, eu, ep)
    return worst


def test_mixed_step_cavity2d_64_fifty_steps():
    # the 64^2 Bingham cavity (Bi = 1, Re = 100, m = 1e3, CFL 0.5) from rest,
    # every solve in mixed precision, against the FP64 oracle
    _say("mixed step cavity2d_64 x50")
    w = inputs.WORKLOADS["cavity2d_64"]
    s = lid_spec(2, w["n"], Re=w["Re"], HB=w["HB"], nidx=w["nidx"], Pa=w["Pa"])
    worst = _steps(s, w["steps"])
    _say("  worst step error vs oracle %.3e" % worst)
    assert worst < SOLVE_TOL


@pytest.mark.parametrize("case", ["lid3d_16", "mix3d_12x16x8", "rag3d_24x12x6"])
def test_mixed_step_short_runs(case):
    _say("mixed step", case)
    worst = _steps(CASES[case](), 5)
    _say("  worst step error vs oracle %.3e" % worst)
    assert worst < SOLVE_TOL
