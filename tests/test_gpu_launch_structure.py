"""Launch structures against the plain per-level, per-colour launches they
replace: the single-workgroup coarse V-cycle (every level below a size limit
in one launch, data in LDS; HB_TAIL=0 turns it off), the fused sweeps (all
colours, or in 2D both tensor components, of a sweep in one launch;
HB_FUSE=0), each candidate tile of the autotuned sweeps (HB_TILE=k
forces candidate k; in 2D, candidates 3.. of the tensor sweep stage
everything in LDS and run two sweeps per launch where the level allows it,
as do the nodal sweeps and the MAC sweeps), and the coarse levels of a
V-cycle replayed as a captured HIP graph (HB_GRAPH=1) instead of launched
one by one.

Each runs the same arithmetic per cell or node in the same order (the same
Gauss-Seidel ordering, residual, restriction, prolongation and FP64
coarsest solve), with FP contraction off, so whole steps agree bit for bit,
cycle counts included.  The plain path is itself held to the oracle by the
parity tests, which run with both on; the cases cover walls, periodic axes,
odd coarsest extents, 2D and 3D, FP64 and mixed precision, and a batch of
uneven cavities.
"""
import os

import numpy as np
import pytest

from oracle import orc
from tests.helpers import dev, hip_objs, host, lid_spec, oracle_objs, spec

pytestmark = pytest.mark.gpu

hb = pytest.importorskip("paper_1803_00417_amd.hb")

CASES = {
    "lid2d_64": lambda: lid_spec(2, 64, Re=100.0, HB=1.0, Pa=1e3),
    "lid2d_96x48": lambda: spec(2, [96, 48], h=1.0 / 96, wall_u={(1, 1): (1.0, 0.0, 0.0)}, Re=50.0, HB=2.0,
                                nidx=0.7, Pa=300.0),
    "per2d_32": lambda: spec(2, 32, bc=((1, 1), (1, 1)), Re=10.0, HB=0.5, nidx=1.3, Pa=100.0),
    "chan2d_8x32": lambda: spec(2, [8, 32], h=1.0 / 32, bc=((1, 1), (0, 0)), Re=1.0, HB=0.2, Pa=1e3,
                                f=(1.0, 0.0, 0.0)),
    "lid3d_16": lambda: lid_spec(3, 16, Re=100.0, HB=2.0, Pa=1e3),
    "mix3d_12x16x8": lambda: spec(3, [12, 16, 8], h=1.0 / 16, bc=((1, 1), (0, 0), (0, 0)),
                                  wall_u={(2, 1): (1.0, 0.5, 0.0)}, Re=20.0, HB=1.0, nidx=0.6, Pa=200.0),
}


def _say(*a):
    print(*a, flush=True)


PLAIN = {"tail": {"HB_TAIL": "0"}, "fuse": {"HB_FUSE": "0"}, "both": {"HB_TAIL": "0", "HB_FUSE": "0"},
         "tile1": {"HB_TILE": "1"}, "tile2": {"HB_TILE": "2"},
         # staged tensor sweeps, two per launch where the level allows it,
         # on every level with the coarse tail off
         "tile3": {"HB_TILE": "3"}, "tile4_notail": {"HB_TILE": "4", "HB_TAIL": "0"},
         "tile5_notail": {"HB_TILE": "5", "HB_TAIL": "0"}, "tile6": {"HB_TILE": "6"},
         "tile6_notail": {"HB_TILE": "6", "HB_TAIL": "0"}, "tile7": {"HB_TILE": "7"},
         # coarse levels replayed as a captured graph
         "graph": {"HB_GRAPH": "1"}, "graph_notail": {"HB_GRAPH": "1", "HB_TAIL": "0"}}


def _context(make, env):
    old = {k: os.environ.get(k) for k in ("HB_TAIL", "HB_FUSE", "HB_TILE", "HB_GRAPH")}
    for k in old:
        os.environ.pop(k, None)
    os.environ.update(env)
    try:
        return make()
    finally:
        for k, v in old.items():
            os.environ.pop(k, None)
            if v is not None:
                os.environ[k] = v


def _start(s):
    go, _ = oracle_objs(s)
    u = np.zeros(orc.cell_shape(go, s["dim"]))
    if s["bc"] is not None and all(b == (1, 1) for b in s["bc"]):
        # a fully periodic box has no moving wall: start from a smooth field
        from paper_1803_00417_amd import inputs
        u = inputs.smooth_cells(u.shape, seed=31, scale=0.5)
    return u, np.zeros(orc.node_shape(go))


def _dt(s):
    # a forced channel at rest has no velocity scale: fixed dt
    return 0.01 if any(f != 0.0 for f in s["f"]) else 0.0


def _steps(s, env, nsteps, **opt):
    g, fl = hip_objs(s)
    ctx = _context(lambda: hb.Context(g, fl, hb.make_step_opts(**opt)), env)
    u0, p0 = _start(s)
    u, p = dev(u0), dev(p0)
    cyc = []
    for _ in range(nsteps):
        rep = ctx.step(u, p, _dt(s))
        cyc.append((rep.mac.cycles, rep.visc.cycles, rep.proj.cycles))
    ctx.close()
    return host(u), host(p), cyc


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("plain", list(PLAIN))
def test_launch_structure_is_bit_identical(case, precision, plain):
    _say("launch structure", plain, case, precision)
    s = CASES[case]()
    opt = {} if precision == "fp64" else {"precision": hb.PREC_MIXED}
    u1, p1, c1 = _steps(s, {}, 4, **opt)
    u0, p0, c0 = _steps(s, PLAIN[plain], 4, **opt)
    _say("  cycles (mac, visc, proj) per step:", c1)
    assert c1 == c0
    assert np.array_equal(u1, u0) and np.array_equal(p1, p0)


def test_launch_structure_in_batch_is_bit_identical():
    _say("launch structure, batch")
    specs = [CASES["lid2d_64"](), CASES["lid2d_96x48"](), lid_spec(2, 16, Re=5.0, HB=3.0, nidx=0.4, Pa=400.0),
             CASES["chan2d_8x32"]()]
    outs = []
    for env in ({}, PLAIN["both"], PLAIN["graph"]):
        objs = [hip_objs(s) for s in specs]
        ctx = _context(lambda: hb.BatchContext([g for g, _ in objs], [f for _, f in objs], hb.make_step_opts()),
                       env)
        us, ps = [], []
        for s in specs:
            u0, p0 = _start(s)
            us.append(dev(u0))
            ps.append(dev(p0))
        for _ in range(3):
            ctx.step(us, ps, [_dt(s) for s in specs])
        outs.append(([host(u) for u in us], [host(p) for p in ps]))
        ctx.close()
    for o in outs[1:]:
        for b in range(len(specs)):
            assert np.array_equal(outs[0][0][b], o[0][b]), b
            assert np.array_equal(outs[0][1][b], o[1][b]), b


def test_autotuner_reports_candidate_tiles():
    _say("tile autotuner")
    s = CASES["lid2d_96x48"]()
    g, fl = hip_objs(s)
    ctx = _context(lambda: hb.Context(g, fl, hb.make_step_opts()), {})
    cand = {"visc": {(64, 8, 256, 1), (32, 16, 256, 1), (128, 4, 256, 1), (32, 16, 512, 1), (32, 16, 512, 2),
                     (64, 16, 512, 1), (64, 16, 512, 2), (32, 16, 1024, 1), (32, 16, 1024, 2), (16, 8, 256, 1),
                     (16, 8, 256, 2), (16, 8, 1024, 1), (16, 8, 1024, 2)},
            "nodal": {(64, 16, 256, 1), (128, 8, 256, 1), (32, 32, 256, 1), (64, 16, 256, 2), (128, 8, 256, 2),
                      (32, 32, 256, 2), (64, 16, 1024, 1), (64, 16, 1024, 2)}}
    tv = [ctx.tile_config(hb.OP_VISC, l) for l in range(8)]
    tn = [ctx.tile_config(hb.OP_NODAL, l) for l in range(8)]
    _say("  tensor", tv, "nodal", tn)
    assert tv[0] in cand["visc"] and tn[0] in cand["nodal"]
    assert all(t is None or t in cand["visc"] for t in tv)
    assert all(t is None or t in cand["nodal"] for t in tn)
    assert ctx.tile_config(hb.OP_MAC, 0) is None
    ctx.close()
    ctx = _context(lambda: hb.Context(g, fl, hb.make_step_opts()), {"HB_TILE": "2"})
    assert ctx.tile_config(hb.OP_VISC, 0) == (128, 4, 256, 1) and ctx.tile_config(hb.OP_NODAL, 0) == (32, 32, 256, 2)
    ctx.close()
    # walls only: the staged candidate runs two sweeps per launch
    ctx = _context(lambda: hb.Context(g, fl, hb.make_step_opts()), {"HB_TILE": "4"})
    assert ctx.tile_config(hb.OP_VISC, 0) == (64, 16, 512, 2) and ctx.tile_config(hb.OP_NODAL, 0) == (64, 16, 256, 2)
    ctx.close()
    ctx = _context(lambda: hb.Context(g, fl, hb.make_step_opts()), {"HB_TILE": "3"})
    assert ctx.tile_config(hb.OP_NODAL, 0) == (64, 16, 1024, 2)
    ctx.close()
    # a periodic extent below 8 allows one sweep per launch only: on an 8x64
    # channel level 1 (4x32) still smooths, level 2 (2x16, 64 unknowns per
    # component pair) is the tensor problem's dense coarsest
    s = spec(2, [8, 64], h=1.0 / 64, bc=((1, 1), (0, 0)), Re=1.0, HB=0.2, Pa=1e3, f=(1.0, 0.0, 0.0))
    g, fl = hip_objs(s)
    ctx = _context(lambda: hb.Context(g, fl, hb.make_step_opts()), {"HB_TILE": "3", "HB_TAIL": "0"})
    assert ctx.tile_config(hb.OP_VISC, 0) == (32, 16, 512, 2)
    assert ctx.tile_config(hb.OP_VISC, 1) == (32, 16, 512, 1)
    assert ctx.tile_config(hb.OP_VISC, 2) is None
    assert ctx.tile_config(hb.OP_NODAL, 0)[3] == 2 and ctx.tile_config(hb.OP_NODAL, 1)[3] == 1
    ctx.close()
