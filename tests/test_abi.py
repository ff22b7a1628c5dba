"""The C-ABI library loads on any host, exports every symbol include/hb.h
declares, agrees with the binding on struct layouts, and rejects invalid
descriptors before any device work (these calls never reach the GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hb.h")
LIB = os.path.join(ROOT, "paper_1803_00417_amd", "libhb.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_[a-z_]+)\s*\(", txt)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libhb.so not built")


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    names = _declared()
    assert "hb_step" in names and "hb_mg_solve" in names and "hb_viscosity" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_1803_00417_amd import hb
    assert sorted(hb.EXPORTS) == names


def test_struct_layouts_match_header(tmp_path):
    from paper_1803_00417_amd import hb
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hb.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(hb_grid),sizeof(hb_fluid),sizeof(hb_mg_opts),sizeof(hb_mg_report),'
                   'sizeof(hb_step_opts),sizeof(hb_step_report),offsetof(hb_grid,wall_u),'
                   'offsetof(hb_step_opts,proj),sizeof(hb_steady_report),offsetof(hb_steady_report,change),'
                   'sizeof(hb_yield_report),sizeof(hb_cessation_report),offsetof(hb_step_opts,theta));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(hb.Grid), C.sizeof(hb.Fluid), C.sizeof(hb.MGOpts), C.sizeof(hb.MGReport),
            C.sizeof(hb.StepOpts), C.sizeof(hb.StepReport), hb.Grid.wall_u.offset, hb.StepOpts.proj.offset,
            C.sizeof(hb.SteadyReport), hb.SteadyReport.change.offset, C.sizeof(hb.YieldReport),
            C.sizeof(hb.CessationReport), hb.StepOpts.theta.offset]
    assert got == want


@needs_lib
def test_create_rejects_invalid_descriptors_without_device_work():
    from paper_1803_00417_amd import hb
    L = hb.load()
    opts = hb.make_step_opts()
    fl = hb.make_fluid(Re=1.0, HB=1.0, Pa=100.0)
    bad_grids = [hb.make_grid(2, [5, 8]), hb.make_grid(4, [8, 8]), hb.make_grid(2, [2, 8]),
                 hb.make_grid(2, [8, 8], bc=((1, 0), (0, 0))), hb.make_grid(2, [20, 8])]
    for g in bad_grids:
        h = C.c_void_p()
        rc = L.hb_create(C.byref(g), C.byref(fl), C.byref(opts), None, C.byref(h))
        assert rc == hb.ERR_ARG and not h.value
        assert len(L.hb_last_error(None)) > 0
    g = hb.make_grid(2, [8, 8])
    for f in (hb.make_fluid(Re=0.0), hb.make_fluid(Pa=-1.0), hb.make_fluid(n=0.5, reg=hb.REG_YIELD_ONLY),
              hb.make_fluid(HB=-1.0)):
        h = C.c_void_p()
        assert L.hb_create(C.byref(g), C.byref(f), C.byref(opts), None, C.byref(h)) == hb.ERR_ARG
    bad = hb.make_step_opts(nu=0)
    h = C.c_void_p()
    assert L.hb_create(C.byref(g), C.byref(fl), C.byref(bad), None, C.byref(h)) == hb.ERR_ARG
    # null context is rejected by every entry point
    assert L.hb_step(None, None, None, 0.0, None) == hb.ERR_ARG
    assert L.hb_run_steady(None, None, None, 1e-5, 10, 0.0, None) == hb.ERR_ARG
    assert L.hb_refine_state(None, None, None, None, None) == hb.ERR_ARG
    assert L.hb_checkpoint_write(None, b"x", None, None, 0, 0.0) == hb.ERR_ARG
    assert L.hb_checkpoint_read(None, b"x", None, None, None, None) == hb.ERR_ARG
    assert L.hb_yield(None, None, None, None) == hb.ERR_ARG
    assert L.hb_run_cessation(None, None, None, 10, 0.0, None) == hb.ERR_ARG
    # the sequenced driver checks its arguments before it creates anything
    reps = (hb.SteadyReport * 2)()
    one = C.c_void_p(1)
    assert L.hb_run_sequenced(None, C.byref(fl), C.byref(opts), 1, 1e-5, 10, None, one, one, reps) == hb.ERR_ARG
    assert L.hb_run_sequenced(C.byref(g), C.byref(fl), C.byref(opts), 9, 1e-5, 10, None, one, one, reps) == hb.ERR_ARG
    assert L.hb_run_sequenced(C.byref(g), C.byref(fl), C.byref(opts), 1, 0.0, 10, None, one, one, reps) == hb.ERR_ARG
    assert L.hb_run_sequenced(C.byref(bad_grids[0]), C.byref(fl), C.byref(opts), 1, 1e-5, 10, None, one, one,
                              reps) == hb.ERR_ARG
    assert len(L.hb_last_error(None)) > 0
    assert L.hb_viscosity(None, None, None) == hb.ERR_ARG
