"""The OpenMP timing build of the oracle (liborc_omp.so) gives the serial
build's values bit for bit: its loops split planes and rows over threads
(on grids of at least 4096 cells), and the loops that add into nodes (weak
divergence, Q1 stiffness) gather each node's cells in the order in which
the serial loops add them.  The cases are large enough that the finest
levels run split."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import orc
from tests.helpers import lid_spec, oracle_objs, spec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_RUN = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import orc
from tests.helpers import lid_spec, oracle_objs, spec
s = eval(sys.argv[2])
g, fl = oracle_objs(s)
o = orc.make_step_opts()
u = np.zeros(orc.cell_shape(g, s["dim"]))
if s["bc"] is not None:
    from paper_1803_00417_amd import inputs
    u = inputs.smooth_cells(u.shape, seed=3, scale=0.5)
p = np.zeros(orc.node_shape(g))
for _ in range(int(sys.argv[3])):
    rep, rc = orc.step(g, fl, o, u, p, 0.01 if s["bc"] is not None else 0.0)
    assert rc == orc.OK
np.savez(sys.argv[4], u=u, p=p)
"""

CASES = {
    "lid2d_64": 'lid_spec(2, 64, Re=100.0, HB=1.0, Pa=1e3)',
    "lid3d_16": 'lid_spec(3, 16, Re=50.0, HB=2.0, nidx=0.7, Pa=300.0)',
    "per2d_128x64": 'spec(2, [128, 64], h=1.0 / 128, bc=((1, 1), (0, 0)), Re=5.0, HB=0.5, Pa=100.0)',
}


def _run(case, steps, omp, out):
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = "4"
    if omp:
        env["ORC_OMP"] = "1"
    else:
        env.pop("ORC_OMP", None)
    subprocess.run([sys.executable, "-c", _RUN, ROOT, CASES[case], str(steps), out], env=env, check=True)
    d = np.load(out)
    return d["u"], d["p"]


@pytest.mark.parametrize("case", list(CASES))
def test_openmp_build_equals_serial_build(case, tmp_path):
    orc.build()
    u1, p1 = _run(case, 3, False, str(tmp_path / "a.npz"))
    u2, p2 = _run(case, 3, True, str(tmp_path / "b.npz"))
    np.testing.assert_array_equal(u1, u2)
    np.testing.assert_array_equal(p1, p2)
