"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.

Bars (FP64): single kernels within 1e-13 relative (the two sides differ only
in rounding order and in libm-vs-device expm1/pow); fixed-cycle multigrid
within 1e-12; converged solves within a few times the solver tolerance;
whole steps of the 64^2 cavity within 1e-9 relative in the max norm.
"""
import numpy as np
import pytest

from oracle import orc
from paper_1803_00417_amd import inputs
from tests.helpers import dev, hip_objs, host, lid_spec, oracle_objs, rel_err, spec

pytestmark = pytest.mark.gpu

hb = pytest.importorskip("paper_1803_00417_amd.hb")

CASES = {
    "lid2d_32": lambda: lid_spec(2, 32, Re=100.0, HB=1.0, Pa=1e3),
    "lid2d_96x48": lambda: spec(2, [96, 48], h=1.0 / 96, wall_u={(1, 1): (1.0, 0.0, 0.0)}, Re=50.0, HB=2.0,
                                nidx=0.7, Pa=300.0),
    "per2d_32": lambda: spec(2, 32, bc=((1, 1), (1, 1)), Re=10.0, HB=0.5, nidx=1.3, Pa=100.0),
    "chan2d_8x32": lambda: spec(2, [8, 32], h=1.0 / 32, bc=((1, 1), (0, 0)), Re=1.0, HB=0.2, Pa=1e3,
                                f=(1.0, 0.0, 0.0)),
    "lid3d_16": lambda: lid_spec(3, 16, Re=100.0, HB=2.0, Pa=1e3),
    "mix3d_12x16x8": lambda: spec(3, [12, 16, 8], h=1.0 / 16, bc=((1, 1), (0, 0), (0, 0)),
                                  wall_u={(2, 1): (1.0, 0.5, 0.0)}, Re=20.0, HB=1.0, nidx=0.6, Pa=200.0),
    # tiles cut in every axis: 24 cells against 32-wide tiles, 12 against
    # 8- and 16-deep ones, 6 against 4 and 8, with a periodic axis across them
    "rag3d_24x12x6": lambda: spec(3, [24, 12, 6], h=1.0 / 24, bc=((0, 0), (0, 0), (1, 1)),
                                  wall_u={(1, 1): (1.0, 0.0, 0.3)}, Re=30.0, HB=1.5, nidx=0.8, Pa=300.0),
}


def _ctx(s, **opt):
    g, fl = hip_objs(s)
    return hb.Context(g, fl, hb.make_step_opts(**opt)), g, fl


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("dim,nidx", [(2, 1.5), (3, 1.5), (2, 1.0)])
def test_viscosity_parity_yield_only(dim, nidx):
    # the yield-only regularisation: g^(n-1) + (HB/2)(1 - exp(-Pa g))/g,
    # with n > 1 (the power-law term is not regularised)
    _say("viscosity yield-only", dim, nidx)
    s = lid_spec(dim, 16 if dim == 3 else 48, Re=10.0, HB=3.0, nidx=nidx, Pa=500.0, reg=orc.REG_YIELD_ONLY)
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    u = inputs.random_cells(orc.cell_shape(go, dim), seed=5, scale=0.7)
    u[:, :, :3, :] = 0.0        # a region at rest: g = 0 there
    eta_o, rc = orc.viscosity(go, flo, u)
    assert rc == orc.OK
    eta = dev(np.zeros(orc.cell_shape(go)[1:]))
    ctx.viscosity(dev(u), eta)
    assert rel_err(host(eta), eta_o) < 1e-13


@pytest.mark.parametrize("case", list(CASES))
def test_viscosity_parity(case):
    _say("viscosity", case)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    u = inputs.random_cells(orc.cell_shape(go, s["dim"]), seed=1, scale=0.7)
    eta_o, rc = orc.viscosity(go, flo, u)
    assert rc == orc.OK
    ud = dev(u)
    eta = dev(np.zeros(orc.cell_shape(go)[1:]))
    ctx.viscosity(ud, eta)
    assert rel_err(host(eta), eta_o) < 1e-13


@pytest.mark.parametrize("case", ["lid2d_32", "lid2d_96x48", "per2d_32", "lid3d_16", "mix3d_12x16x8", "rag3d_24x12x6"])
@pytest.mark.parametrize("op", [hb.OP_VISC, hb.OP_MAC, hb.OP_NODAL])
def test_mg_fixed_cycles_parity(case, op):
    _say("mg fixed", case, op)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    d = s["dim"]
    if op == hb.OP_VISC:
        sh = orc.cell_shape(go, d)
        eta = inputs.positive_cells(orc.cell_shape(go)[1:], seed=3, lo=-1.0, hi=4.0)
    elif op == hb.OP_MAC:
        sh = orc.cell_shape(go)[1:]
        eta = None
    else:
        sh = orc.node_shape(go)
        eta = None
    rhs = inputs.random_cells(sh, seed=4)
    x0 = inputs.random_cells(sh, seed=5, scale=0.1)
    dt = 0.3 * go.h
    for krylov in ((0, 1) if op == hb.OP_VISC else (0,)):
        xo, rco, repo = orc.mg_solve(go, flo, op, eta, dt, rhs, x0, max_cycles=3, fixed=1, krylov=krylov)
        xd = dev(x0)
        rep, rc = ctx.mg_solve(op, dev(eta) if eta is not None else None, dt, dev(rhs), xd,
                               hb.mg_opts(max_cycles=3, fixed=1, krylov=krylov))
        assert rep.cycles == repo.cycles == 3
        assert rel_err(host(xd).reshape(sh), xo) < 1e-12, (krylov, rel_err(host(xd).reshape(sh), xo))


@pytest.mark.parametrize("case", ["lid2d_96x48", "lid3d_16", "chan2d_8x32", "rag3d_24x12x6"])
@pytest.mark.parametrize("op", [hb.OP_VISC, hb.OP_MAC, hb.OP_NODAL])
def test_mg_converged_parity(case, op):
    _say("mg converged", case, op)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    d = s["dim"]
    eta = None
    if op == hb.OP_VISC:
        sh = orc.cell_shape(go, d)
        eta = inputs.positive_cells(orc.cell_shape(go)[1:], seed=7, lo=0.0, hi=5.0)
    elif op == hb.OP_MAC:
        sh = orc.cell_shape(go)[1:]
    else:
        sh = orc.node_shape(go)
    rhs = inputs.smooth_cells(sh if len(sh) == 4 else (1,) + tuple(sh), seed=8).reshape(sh)
    dt = 0.5 * go.h
    kry = 1 if op == hb.OP_VISC else 0
    xo, rco, repo = orc.mg_solve(go, flo, op, eta, dt, rhs, tol=1e-10, krylov=kry)
    xd = dev(np.zeros(sh))
    rep, rc = ctx.mg_solve(op, dev(eta) if eta is not None else None, dt, dev(rhs), xd,
                           hb.mg_opts(tol=1e-10, krylov=kry))
    assert rco == orc.OK and rc == hb.OK
    assert rep.rel_resid <= 1e-10 and abs(rep.cycles - repo.cycles) <= 1
    assert rel_err(host(xd).reshape(sh), xo) < 1e-8


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mac_project", [0, 1])
def test_advect_parity(case, mac_project):
    _say("advect", case, mac_project)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s, mac_project=mac_project)
    oo = orc.make_step_opts(mac_project=mac_project)
    d = s["dim"]
    u = inputs.smooth_cells(orc.cell_shape(go, d), seed=11, scale=0.5) + \
        inputs.random_cells(orc.cell_shape(go, d), seed=12, scale=0.05)
    p = inputs.random_cells((1,) + orc.node_shape(go), seed=13, scale=0.1).reshape(orc.node_shape(go))
    eta_o, _ = orc.viscosity(go, flo, u)
    dt = 0.5 * go.h
    b_o, E_o, umac_o, A_o, rep_o, dm_o, rc = orc.advect(go, flo, oo, u, p, eta_o, dt)
    assert rc == orc.OK
    ud, pd = dev(u), dev(p)
    eta = dev(np.zeros(orc.cell_shape(go)[1:]))
    ctx.viscosity(ud, eta)
    b = dev(np.zeros_like(u))
    umac = dev(np.zeros(orc.face_total(go)))
    conv = dev(np.zeros_like(u))
    ctx.advect(ud, pd, eta, dt, b, umac, conv)
    tol = 1e-12 if not mac_project else 2e-9
    assert rel_err(host(umac), umac_o) < tol
    assert rel_err(host(conv).reshape(u.shape), A_o) < tol * 10
    assert rel_err(host(b).reshape(u.shape), b_o) < tol


@pytest.mark.parametrize("case", list(CASES))
def test_project_parity(case):
    _say("project", case)
    s = CASES[case]()
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    oo = orc.make_step_opts()
    d = s["dim"]
    us = inputs.smooth_cells(orc.cell_shape(go, d), seed=21) + inputs.random_cells(orc.cell_shape(go, d), seed=22, scale=0.1)
    p = inputs.random_cells((1,) + orc.node_shape(go), seed=23, scale=0.1).reshape(orc.node_shape(go))
    dt = 0.5 * go.h
    un_o, pn_o, rep_o, rc = orc.project(go, oo, us, p, dt)
    assert rc == orc.OK
    pd = dev(p)
    ud = dev(np.zeros_like(us))
    rep = ctx.project(dev(us), pd, dt, ud)
    assert rep.rel_resid <= 1e-10
    assert rel_err(host(ud).reshape(us.shape), un_o) < 1e-9
    assert rel_err(host(pd).reshape(p.shape), pn_o) < 1e-8


def _run_steps(s, nsteps, dt=0.0, u0_seed=None, **opt):
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s, **opt)
    oo = orc.make_step_opts(**opt)
    d = s["dim"]
    u = np.zeros(orc.cell_shape(go, d))
    if u0_seed is not None:     # boxes without a moving wall start from a smooth field
        u = inputs.smooth_cells(u.shape, seed=u0_seed, scale=0.5)
    p = np.zeros(orc.node_shape(go))
    ud, pd = dev(u), dev(p)
    worst = 0.0
    for k in range(nsteps):
        rep_o, rc = orc.step(go, flo, oo, u, p, dt)
        assert rc == orc.OK
        rep = ctx.step(ud, pd, dt)
        assert abs(rep.dt - rep_o.dt) <= 1e-12 * rep_o.dt
        eu = rel_err(host(ud).reshape(u.shape), u)
        # pressure relative to max(|p|, U^2): a flow with a vanishing pressure
        # (plane channel) is compared on the dynamic-pressure scale
        pscale = max(np.abs(p).max(), np.abs(u).max() ** 2)
        ep = np.abs(host(pd).reshape(p.shape) - p).max() / pscale
        worst = max(worst, eu, ep)
    return worst, rep, rep_o


def test_step_parity_cavity2d_64_fifty_steps():
    # the 64^2 Bingham cavity (Bi = 1, Re = 100, m = 1e3, CFL 0.5) from rest
    _say("step cavity2d_64 x50")
    w = inputs.WORKLOADS["cavity2d_64"]
    s = lid_spec(2, w["n"], Re=w["Re"], HB=w["HB"], nidx=w["nidx"], Pa=w["Pa"])
    worst, rep, rep_o = _run_steps(s, w["steps"])
    assert worst < 1e-9, worst
    assert rep.visc.rel_resid <= 1e-10 and rep.proj.rel_resid <= 1e-10 and rep.div_mac_rel <= 1e-10


@pytest.mark.parametrize("case", ["lid3d_16", "mix3d_12x16x8", "per2d_32", "lid2d_96x48", "rag3d_24x12x6"])
def test_step_parity_short_runs(case):
    _say("step", case)
    s = CASES[case]()
    worst, rep, rep_o = _run_steps(s, 5, u0_seed=31 if case.startswith("per") else None)
    assert worst < 1e-9, worst


def test_step_parity_channel_fixed_dt():
    _say("step channel")
    s = CASES["chan2d_8x32"]()
    worst, rep, rep_o = _run_steps(s, 20, dt=0.01)
    assert worst < 1e-9, worst


@pytest.mark.parametrize("case", ["lid2d_32", "lid3d_16", "chan2d_8x32"])
@pytest.mark.parametrize("opt", [dict(pred_visc=1), dict(theta=1.0), dict(pred_visc=1, theta=0.75)],
                         ids=["pred_visc", "backward_euler", "pred_visc_theta075"])
def test_step_parity_step_options(case, opt):
    # the readings of the predictor forcing and of the viscous update
    _say("step options", case, opt)
    s = CASES[case]()
    worst, rep, rep_o = _run_steps(s, 5, dt=0.01 if case.startswith("chan") else 0.0, **opt)
    assert worst < 1e-9, worst


def test_step_parity_bingham_re1_backward_euler():
    # the Re = 1, Bi = 10, Pa = 400 cavity of Sec. IV under backward Euler
    _say("step bingham Re1 theta=1")
    s = lid_spec(2, 32, Re=1.0, HB=10.0, Pa=400.0)
    worst, rep, rep_o = _run_steps(s, 20, theta=1.0)
    assert worst < 1e-9, worst


def test_step_is_deterministic():
    _say("determinism")
    s = CASES["lid2d_96x48"]()
    ctx, g, fl = _ctx(s)
    outs = []
    for _ in range(2):
        u = dev(np.zeros(orc.cell_shape(oracle_objs(s)[0], 2)))
        p = dev(np.zeros(orc.node_shape(oracle_objs(s)[0])))
        for _ in range(3):
            ctx.step(u, p)
        outs.append((host(u), host(p)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_error_paths():
    _say("errors")
    s = CASES["lid2d_32"]()
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    u = np.zeros(orc.cell_shape(go, 2))
    u[0, 0, 3, 3] = np.nan
    p = np.zeros(orc.node_shape(go))
    with pytest.raises(hb.HBError) as e:
        ctx.step(dev(u), dev(p))
    assert e.value.code == hb.ERR_NONFINITE
    rhs = inputs.random_cells(orc.cell_shape(go)[1:], seed=1)
    x = dev(np.zeros_like(rhs))
    rep, rc = ctx.mg_solve(hb.OP_MAC, None, 0.0, dev(rhs), x, hb.mg_opts(tol=1e-12, max_cycles=1),
                           allow=(hb.ERR_NOCONV,))
    assert rc == hb.ERR_NOCONV and rep.cycles == 1 and rep.rel_resid > 1e-12
    with pytest.raises(hb.HBError) as e:
        ctx.mg_solve(hb.OP_VISC, None, 0.1, dev(np.zeros((2,) + rhs.shape[1:])), dev(np.zeros((2,) + rhs.shape[1:])))
    assert e.value.code == hb.ERR_ARG


@pytest.mark.parametrize("op", [hb.OP_VISC, hb.OP_MAC, hb.OP_NODAL])
def test_zero_rhs_gives_zero_without_cycles(op):
    # |b| = 0: the stopping test holds before the first cycle and x = 0
    # (walls at rest: a moving wall would put its values into the viscous
    # solve's right-hand side)
    _say("zero rhs", op)
    s = spec(2, [96, 48], h=1.0 / 96, Re=50.0, HB=2.0, nidx=0.7, Pa=300.0)
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    sh = {hb.OP_VISC: orc.cell_shape(go, 2), hb.OP_MAC: orc.cell_shape(go)[1:], hb.OP_NODAL: orc.node_shape(go)}[op]
    eta = dev(np.ones(orc.cell_shape(go)[1:])) if op == hb.OP_VISC else None
    x = dev(inputs.random_cells(sh, seed=9))
    rep, rc = ctx.mg_solve(op, eta, 0.01, dev(np.zeros(sh)), x, hb.mg_opts())
    assert rc == hb.OK and rep.cycles == 0
    assert float(x.abs().max()) == 0.0


@pytest.mark.parametrize("dim", [2, 3])
def test_smallest_grid_step_parity(dim):
    # 4 cells per axis, the smallest grid the library takes: less than one
    # tile, two multigrid levels
    _say("smallest grid", dim)
    s = lid_spec(dim, 4, Re=10.0, HB=1.0, Pa=100.0)
    go, flo = oracle_objs(s)
    ctx, g, fl = _ctx(s)
    o = orc.make_step_opts()
    u_o = np.zeros(orc.cell_shape(go, dim))
    p_o = np.zeros(orc.node_shape(go))
    u, p = dev(u_o), dev(p_o)
    for _ in range(3):
        rep_o, rc_o = orc.step(go, flo, o, u_o, p_o)
        assert rc_o == orc.OK
        ctx.step(u, p)
    assert rel_err(host(u), u_o) <= 1e-9
    assert rel_err(host(p), p_o) <= 1e-9


def test_rest_without_lid_needs_a_step():
    # no moving wall and u = 0: the CFL step is undefined, so dt <= 0 is
    # refused before any device work, while a given dt steps (and stays at rest)
    _say("rest without lid")
    s = spec(2, 16, bc=((1, 1), (1, 1)), Re=10.0, HB=0.5, Pa=100.0)
    ctx, g, fl = _ctx(s)
    u = dev(np.zeros(hb.cell_shape(g, 2)))
    p = dev(np.zeros(hb.node_shape(g)))
    with pytest.raises(hb.HBError) as e:
        ctx.step(u, p)
    assert e.value.code == hb.ERR_ARG
    rep = ctx.step(u, p, dt=0.01)
    assert rep.dt == 0.01 and float(u.abs().max()) == 0.0 and float(p.abs().max()) == 0.0
