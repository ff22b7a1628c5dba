"""hb_cfl_dt_noalloc, the CFL step without a context or any allocation
(static per-GPU scratch), against hb_cfl_dt on the same inputs: bit for bit,
over consecutive calls whose second input is smaller than the first."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1803_00417_amd import inputs
from tests.helpers import dev, hip_objs, spec

hb = pytest.importorskip("paper_1803_00417_amd.hb")


def test_rejects_bad_arguments_before_device_work():
    L = hb.load()
    big = hb.lid_cavity(3, 512)              # 3 x 512^3 values: above the scratch's limit
    fake = C.c_void_p(1)                     # never dereferenced: every check fails first
    assert L.hb_cfl_dt_noalloc(C.byref(big), 0.5, fake, fake, None) == hb.ERR_ARG
    assert "scratch" in L.hb_last_error(None).decode()
    ok = hb.lid_cavity(2, 32)
    assert L.hb_cfl_dt_noalloc(C.byref(ok), 0.0, fake, fake, None) == hb.ERR_ARG
    assert L.hb_cfl_dt_noalloc(C.byref(ok), 0.5, None, fake, None) == hb.ERR_ARG
    assert L.hb_cfl_dt_noalloc(C.byref(ok), 0.5, fake, None, None) == hb.ERR_ARG
    bad = hb.lid_cavity(2, 32)
    bad.n[0] = 5
    assert L.hb_cfl_dt_noalloc(C.byref(bad), 0.5, fake, fake, None) == hb.ERR_ARG


def _both(s, u, cfl, stream=None):
    g, fl = hip_objs(s)
    ctx = hb.Context(g, fl, hb.make_step_opts(cfl=cfl))
    ud = dev(u)
    want = ctx.cfl_dt(ud)
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    if stream is None:
        hb.cfl_dt_noalloc(g, cfl, ud, out)
    else:
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            hb.cfl_dt_noalloc(g, cfl, ud, out, stream=stream)
        torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    got = out.item()
    ctx.close()
    return got, want


@pytest.mark.gpu
def test_noalloc_cfl_equals_context_cfl_on_consecutive_calls():
    print("noalloc cfl: 3D 64^3 then 2D 32^2 channel then 2D 16^2 at rest", flush=True)
    # first call: a large 3D field whose velocity exceeds the lid speed
    s1 = spec(3, 64, wall_u={(2, 1): (1.0, 0.0, 0.0)})
    u1 = inputs.random_cells((3, 64, 64, 64), seed=3, scale=0.9)
    got, want = _both(s1, u1, 0.5)
    assert got == want and want > 0.0
    # second, smaller call on another stream: periodic x axis whose wall
    # velocity must be ignored, so the slow field's own maximum decides
    s2 = spec(2, 32, bc=((1, 1), (0, 0)), wall_u={(0, 0): (5.0, 0.0, 0.0), (0, 1): (5.0, 0.0, 0.0)})
    u2 = inputs.random_cells((2, 1, 32, 32), seed=4, scale=0.01)
    got2, want2 = _both(s2, u2, 0.3, stream=torch.cuda.Stream())
    assert got2 == want2 and want2 > 0.0
    assert got2 != got
    # third: the fluid at rest under a lid, so the lid speed decides
    s3 = spec(2, 16, wall_u={(1, 1): (2.0, 0.0, 0.0)})
    got3, want3 = _both(s3, np.zeros((2, 1, 16, 16)), 0.5)
    assert got3 == want3 == 0.5 * (1.0 / 16) / 2.0


@pytest.mark.gpu
def test_noalloc_cfl_non_finite_velocity_gives_nan():
    g, _ = hip_objs(spec(2, 16))
    u = torch.zeros((2, 1, 16, 16), dtype=torch.float64, device="cuda")
    u[1, 0, 3, 4] = float("inf")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    hb.cfl_dt_noalloc(g, 0.5, u, out)
    torch.cuda.synchronize()
    assert np.isnan(out.item())
