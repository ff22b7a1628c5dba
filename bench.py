"""Throughput of the Herschel-Bulkley cavity step on one MI355X.

A step is one full pass of the hot path: viscosity, Godunov advection with
the MAC projection, the tensor viscous multigrid solve and the nodal
projection, all solves to a relative residual of 1e-10.  The workload is the
2D 512^2 lid-driven cavity (Herschel-Bulkley n = 0.5, Bi = 10, Re = 1000,
Pa = 1e4, CFL 0.5) started from rest: W untimed warm-up steps, then K timed
steps.  value = cells x K / T (cell-steps/s), with the inputs resident in
HBM.  The 3D 128^3 Bingham cavity is timed the same way and reported beside
it.  The roofline object describes the tensor smoother (the red-black half
sweep), timed with HIP events on the library's stream inside the timed
region; cpu_baseline times the FP64 CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cavity2d_512_n0.5")
    ap.add_argument("--also", default="cavity3d_128", help="second workload ('' for none)")
    ap.add_argument("--also-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    return ap.parse_args()


def run_gpu(name, steps, warmup, timing=True):
    import torch
    from paper_1803_00417_amd import hb, inputs
    w = inputs.WORKLOADS[name]
    g = hb.lid_cavity(w["dim"], w["n"])
    fl = hb.make_fluid(Re=w["Re"], HB=w["HB"], n=w["nidx"], Pa=w["Pa"])
    ctx = hb.Context(g, fl, hb.make_step_opts(cfl=w["cfl"]))
    u = torch.zeros(hb.cell_shape(g, w["dim"]), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    for k in range(warmup):
        ctx.step(u, p, report=False)
    torch.cuda.synchronize()
    if timing:
        ctx.kernel_timing(True)
    cycles = [0, 0, 0]
    t0 = time.perf_counter()
    for k in range(steps):
        rep = ctx.step(u, p, report=True)
        cycles[0] += rep.mac.cycles
        cycles[1] += rep.visc.cycles
        cycles[2] += rep.proj.cycles
        if (k + 1) % 10 == 0:
            print("[bench] %s step %d/%d dt %.3e max|u| %.4f cycles mac/visc/proj %d/%d/%d"
                  % (name, k + 1, steps, rep.dt, rep.max_u, rep.mac.cycles, rep.visc.cycles, rep.proj.cycles),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    kt = ctx.kernel_timing_read() if timing else (0, 0.0, 0.0)
    ctx.kernel_timing(False)
    ncell = g.n[0] * g.n[1] * g.n[2]
    ctx.close()
    return dict(T=T, ncell=ncell, steps=steps, cycles=[c / steps for c in cycles], kt=kt)


def cpu_baseline(name, nsteps):
    from oracle import orc
    import numpy as np
    from paper_1803_00417_amd import inputs
    w = inputs.WORKLOADS[name]
    g = orc.lid_cavity(w["dim"], w["n"])
    fl = orc.make_fluid(Re=w["Re"], HB=w["HB"], n=w["nidx"], Pa=w["Pa"])
    o = orc.make_step_opts(cfl=w["cfl"])
    u = np.zeros(orc.cell_shape(g, w["dim"]))
    p = np.zeros(orc.node_shape(g))
    t0 = time.perf_counter()
    for _ in range(nsteps):
        rep, rc = orc.step(g, fl, o, u, p)
    T = time.perf_counter() - t0
    ncell = g.n[0] * g.n[1] * g.n[2]
    return dict(value=ncell * nsteps / T, unit="cell-steps/s", cores=1, kind="oracle",
                sample="first %d step(s) of the %s workload from rest, single-threaded FP64 C "
                       "oracle (%.1f s)" % (nsteps, name, T))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1803_00417_amd import hb, inputs  # noqa: F401
    assert torch.cuda.is_available(), "no GPU"
    print("[bench] workload %s: %d warm-up + %d timed steps" % (a.workload, a.warmup, a.steps),
          file=sys.stderr, flush=True)
    r = run_gpu(a.workload, a.steps, a.warmup)
    value = r["ncell"] * r["steps"] / r["T"]
    launches, kms, kbytes = r["kt"]
    achieved = (kbytes / 1e9) / (kms / 1e3) if kms > 0 else 0.0
    w = inputs.WORKLOADS[a.workload]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": ("k_tsmooth (2D: fused red-black sweep of one velocity component, finest level)" if w["dim"] == 2 else "k_trb3 (3D: one colour of one velocity component, finest level)"),
                "launches": launches, "avg_launch_us": 1e3 * kms / max(launches, 1),
                "alg_bytes_per_launch": kbytes / max(launches, 1)}
    out = {"metric": "cell-steps/s", "value": value, "unit": "cell-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * r["T"] / r["steps"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w["desc"] + ", from rest, tol 1e-10", "cells": r["ncell"],
                      "cycles_per_step_mac_visc_proj": r["cycles"]},
           "roofline": roofline}
    if a.also:
        print("[bench] workload %s: 2 warm-up + %d timed steps" % (a.also, a.also_steps), file=sys.stderr, flush=True)
        r2 = run_gpu(a.also, a.also_steps, 2)
        l2, ms2, b2 = r2["kt"]
        ach2 = (b2 / 1e9) / (ms2 / 1e3) if ms2 > 0 else 0.0
        out["also"] = {a.also: {"value": r2["ncell"] * r2["steps"] / r2["T"], "unit": "cell-steps/s",
                                "ms_per_step": 1e3 * r2["T"] / r2["steps"], "steps": r2["steps"], "warmup": 2,
                                "cycles_per_step_mac_visc_proj": r2["cycles"],
                                "smoother_GBs": ach2, "smoother_frac": ach2 / HBM_PEAK_GBS,
                                "desc": inputs.WORKLOADS[a.also]["desc"]}}
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.workload, a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
