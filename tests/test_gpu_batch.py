"""Batched sweeps: a context holding several cavities of uneven size and
parameters, stepped together (one launch per multigrid kernel for all
cavities, each cavity stopping at its own tolerance), against each cavity
run alone.  The batched kernels do the same arithmetic per cavity in the
same order, and a cavity's sums use its own fixed blocks, so each cavity of
the batch reproduces its single-context run; the bar is 1e-12 relative.
The single-context runs are themselves held to the oracle by the parity
tests; the first cavity is also compared with the oracle here.
"""
import numpy as np
import pytest

from oracle import orc
from paper_1803_00417_amd import inputs
from tests.helpers import dev, hip_objs, host, lid_spec, oracle_objs, rel_err, spec

pytestmark = pytest.mark.gpu

hb = pytest.importorskip("paper_1803_00417_amd.hb")


def _say(*a):
    print(*a, flush=True)


def _specs2d():
    # sizes from the sweep's set, scaled down; parameters spread like the
    # sweep's distributions (SplitMix64 draws), plus a periodic box
    out = []
    for i, d in enumerate(inputs.batch_cavities(count=5, seed=3, sizes=(16, 24, 32, 48))):
        out.append(lid_spec(2, d["n"], Re=d["Re"], HB=d["HB"], nidx=d["nidx"], Pa=d["Pa"]))
    out.append(spec(2, [32, 16], h=1.0 / 32, bc=((1, 1), (0, 0)), wall_u={(1, 1): (0.5, 0.0, 0.0)}, Re=20.0, HB=0.5,
                    Pa=500.0))
    return out


def _specs3d():
    return [lid_spec(3, 16, Re=100.0, HB=2.0, Pa=1e3),
            spec(3, [12, 16, 8], h=1.0 / 16, bc=((1, 1), (0, 0), (0, 0)), wall_u={(2, 1): (1.0, 0.5, 0.0)},
                 Re=20.0, HB=1.0, nidx=0.6, Pa=200.0),
            lid_spec(3, 8, Re=10.0, HB=0.5, nidx=1.2, Pa=300.0),
            spec(3, [24, 12, 6], h=1.0 / 24, bc=((0, 0), (0, 0), (1, 1)), wall_u={(1, 1): (1.0, 0.0, 0.3)},
                 Re=30.0, HB=1.5, nidx=0.8, Pa=300.0)]


def _zeros(s):
    go, _ = oracle_objs(s)
    return np.zeros(orc.cell_shape(go, s["dim"])), np.zeros(orc.node_shape(go))


def _run(specs, nsteps, **opt):
    objs = [hip_objs(s) for s in specs]
    opts = hb.make_step_opts(**opt)
    bctx = hb.BatchContext([g for g, _ in objs], [f for _, f in objs], opts)
    assert bctx.size() == len(specs)
    us, ps = [], []
    for s in specs:
        u, p = _zeros(s)
        us.append(dev(u))
        ps.append(dev(p))
    breps = []
    for _ in range(nsteps):
        breps.append(bctx.step(us, ps))
    singles = []
    for s, (g, f) in zip(specs, objs):
        ctx = hb.Context(g, f, hb.make_step_opts(**opt))
        u, p = _zeros(s)
        ud, pd = dev(u), dev(p)
        reps = [ctx.step(ud, pd) for _ in range(nsteps)]
        singles.append((ud, pd, reps))
        ctx.close()
    bctx.close()
    return us, ps, breps, singles


def _compare(specs, us, ps, breps, singles):
    worst = 0.0
    for b, s in enumerate(specs):
        ud, pd, reps = singles[b]
        eu = rel_err(host(us[b]), host(ud))
        ep = rel_err(host(ps[b]), host(pd))
        _say("  cavity %d %s: u %.2e p %.2e cycles batch/single %s/%s" % (
            b, s["n"], eu, ep, [breps[-1][b].visc.cycles, breps[-1][b].proj.cycles],
            [reps[-1].visc.cycles, reps[-1].proj.cycles]))
        worst = max(worst, eu, ep)
        for k in range(len(reps)):
            assert breps[k][b].dt == reps[k].dt
            assert breps[k][b].mac.cycles == reps[k].mac.cycles
            assert breps[k][b].visc.cycles == reps[k].visc.cycles
            assert breps[k][b].proj.cycles == reps[k].proj.cycles
    return worst


@pytest.mark.parametrize("precision", [0, 1])
def test_batch2d_matches_single_runs(precision):
    _say("batch 2D, precision", precision)
    specs = _specs2d()
    us, ps, breps, singles = _run(specs, 4, precision=precision)
    assert _compare(specs, us, ps, breps, singles) <= 1e-12


def test_batch3d_matches_single_runs():
    _say("batch 3D")
    specs = _specs3d()
    us, ps, breps, singles = _run(specs, 3)
    assert _compare(specs, us, ps, breps, singles) <= 1e-12


def test_batch_first_cavity_matches_oracle():
    _say("batch vs oracle")
    specs = _specs2d()
    us, ps, breps, singles = _run(specs, 3)
    go, flo = oracle_objs(specs[0])
    u, p = _zeros(specs[0])
    oo = orc.make_step_opts()
    for _ in range(3):
        rep, rc = orc.step(go, flo, oo, u, p)
        assert rc == orc.OK
    assert rel_err(host(us[0]).reshape(u.shape), u) < 1e-9
    assert rel_err(host(ps[0]).reshape(p.shape), p) < 1e-9


def test_batch_of_one_equals_context():
    _say("batch of one")
    s = lid_spec(2, 32, Re=100.0, HB=1.0, Pa=1e3)
    us, ps, breps, singles = _run([s], 3)
    assert np.array_equal(host(us[0]), host(singles[0][0]))
    assert np.array_equal(host(ps[0]), host(singles[0][1]))


def test_batch_rejects_single_cavity_calls():
    _say("batch errors")
    specs = _specs2d()[:2]
    objs = [hip_objs(s) for s in specs]
    bctx = hb.BatchContext([g for g, _ in objs], [f for _, f in objs])
    # the single-cavity entry points refuse a batched context
    rc = hb.load().hb_viscosity(bctx._h, None, None)
    assert rc == hb.ERR_ARG
    with pytest.raises(ValueError):
        bctx.step([dev(np.zeros(3))], [dev(np.zeros(3))])
    bctx.close()
    # mixed dimensions are refused at creation
    g3, f3 = hip_objs(lid_spec(3, 8))
    with pytest.raises(hb.HBError) as e:
        hb.BatchContext([objs[0][0], g3], [objs[0][1], f3])
    assert e.value.code == hb.ERR_ARG
