"""Throughput of the Herschel-Bulkley cavity step on one MI355X.

A step is one full pass of the hot path: viscosity, Godunov advection with
the MAC projection, the tensor viscous multigrid solve and the nodal
projection, all solves to a relative residual of 1e-10.  The workload is the
2D 512^2 lid-driven cavity (Herschel-Bulkley n = 0.5, Bi = 10, Re = 1000,
Pa = 1e4, CFL 0.5) started from rest: W untimed warm-up steps, then K timed
steps.  value = cells x K / T (cell-steps/s), with the inputs resident in
HBM, all multigrid cycles in FP64.  Beside it: the same workload with
mixed-precision cycles (FP32 V-cycles inside FP64 defect correction, same
1e-10 residual), the n = 1.5 fluid, and the 3D 128^3 Bingham cavity in both
modes.  The roofline object describes the finest-level tensor smoother,
timed with HIP events on the library's stream inside the timed region;
cpu_baseline times the FP64 CPU oracle on the first steps of the workload,
and the GPU runs of those same steps are compared with it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
# kernel timer: every KT_PERIOD-th finest-level smoother launch.  Odd: those
# launches alternate between one that folds in the prolongation and one that
# folds in the restriction, and an even period would time only one kind.
KT_PERIOD = 7
TILE_SOURCE = os.path.join(ROOT, "paper_1803_00417_amd", "csrc", "hb_tile.hip")


def measured_traffic(kernel, workload):
    """HBM bytes per dispatch of the roofline kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by the copy-probe
    factors), or None when the kernel source has changed since then"""
    import hashlib
    if not os.path.exists(TRAFFIC_TABLE):
        return None
    sha = hashlib.sha256(open(TILE_SOURCE, "rb").read()).hexdigest()[:16]
    for line in open(TRAFFIC_TABLE):
        if line.startswith("#") or not line.strip():
            continue
        k, w, fk, wk, fs, ws, src = line.split("\t")
        if k == kernel and w == workload and src.strip() == sha:
            return 1024.0 * (float(fk) * float(fs) + float(wk) * float(ws))
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cavity2d_512_n0.5")
    ap.add_argument("--also", default="cavity2d_512_n1.5,cavity3d_128",
                    help="comma-separated further workloads ('' for none)")
    ap.add_argument("--also-steps", type=int, default=10)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision runs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start runs")
    ap.add_argument("--batch", type=int, default=64, help="cavities of the batched sweep (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--steady", type=int, default=256, metavar="N",
                    help="time to steady state on an N^2 cavity, from rest and by grid sequencing from "
                         "(N/4)^2, then the cessation of the steady flow (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


def _context(name, precision):
    from paper_1803_00417_amd import hb, inputs
    w = inputs.WORKLOADS[name]
    g = hb.lid_cavity(w["dim"], w["n"])
    fl = hb.make_fluid(Re=w["Re"], HB=w["HB"], n=w["nidx"], Pa=w["Pa"])
    return hb.Context(g, fl, hb.make_step_opts(cfl=w["cfl"], precision=precision)), g, w


def run_gpu(name, steps, warmup, precision=0, timing=True, learned=False):
    import torch
    from paper_1803_00417_amd import hb
    ctx, g, w = _context(name, precision)
    net = None
    if learned:
        from paper_1803_00417_amd import warm_start
        net = warm_start.load_net()
        if net is None:
            raise RuntimeError("no trained warm-start weights (run python -m paper_1803_00417_amd.warm_start)")
        ctx.set_warm_start(net)
    u = torch.zeros(hb.cell_shape(g, w["dim"]), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    for k in range(warmup):
        ctx.step(u, p, report=False)
    torch.cuda.synchronize()
    if timing:
        # every KT_PERIOD-th finest-level smoother launch is timed: a timed
        # launch costs the host more, and timing them all would slow the run
        ctx.kernel_timing(KT_PERIOD)
    cycles = [0, 0, 0]
    nrep = 0
    t0 = time.perf_counter()
    for k in range(steps):
        # the step report (diagnostic norms, one more host read) only on the
        # steps that print progress and on the last one
        want = (k + 1) % 10 == 0 or k + 1 == steps
        rep = ctx.step(u, p, report=want)
        if not want:
            continue
        nrep += 1
        cycles[0] += rep.mac.cycles
        cycles[1] += rep.visc.cycles
        cycles[2] += rep.proj.cycles
        if (k + 1) % 10 == 0:
            print("[bench] %s %s step %d/%d dt %.3e max|u| %.4f cycles mac/visc/proj %d/%d/%d"
                  % (name, "mixed" if precision else "fp64", k + 1, steps, rep.dt, rep.max_u, rep.mac.cycles,
                     rep.visc.cycles, rep.proj.cycles),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    kt = ctx.kernel_timing_read() if timing else (0, 0.0, 0.0)
    ctx.kernel_timing(False)
    ncell = g.n[0] * g.n[1] * g.n[2]
    uses = ctx.warm_start_uses() if learned else 0
    # tiles the autotuner chose for the fused sweeps, per level
    tiles = {"tensor": [ctx.tile_config(hb.OP_VISC, l) for l in range(12)],
             "nodal": [ctx.tile_config(hb.OP_NODAL, l) for l in range(12)]}
    tiles = {k: [list(t) if t else None for t in v] for k, v in tiles.items()}
    for k in tiles:
        while tiles[k] and tiles[k][-1] is None:
            tiles[k].pop()
    ctx.close()
    return dict(T=T, ncell=ncell, steps=steps, warmup=warmup, cycles=[c / max(nrep, 1) for c in cycles], kt=kt,
                ws_uses=uses, tiles=tiles)


def run_steady(n, levels=2, tol=1e-5, max_steps=12000):
    """Time to steady state (Sec. III.A test, tolerance 1e-5) on an n^2 lid
    cavity: from rest on n^2, and by grid sequencing (Sec. III.C) from rest
    on (n / 2^levels)^2, refined `levels` times.  Both runs are single
    library calls (hb_run_steady, hb_run_sequenced)."""
    import torch
    from paper_1803_00417_amd import hb
    # Pa = 100: with the sharper regularisation (Pa = 1e3) the scheme keeps a
    # relative change of about 1e-4 per step at 64^2 and above and never
    # meets the 1e-5 test (the oracle does the same)
    fl = hb.make_fluid(Re=100.0, HB=1.0, n=1.0, Pa=100.0)
    opts = hb.make_step_opts()
    g = hb.lid_cavity(2, n)
    ctx = hb.Context(g, fl, opts)
    u = torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep, rc = ctx.run_steady(u, p, tol=tol, max_steps=max_steps)
    torch.cuda.synchronize()
    t_direct = time.perf_counter() - t0
    ctx.close()
    gc = hb.lid_cavity(2, n >> levels)
    us = torch.zeros_like(u)
    ps = torch.zeros_like(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps, rc2 = hb.run_sequenced(gc, fl, opts, levels, us, ps, tol=tol, max_steps=max_steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    diff = float((us - u).abs().max() / u.abs().max())
    # cessation (Sec. IV): the lid of the sequenced steady state stops; a
    # constant step h/2 (the CFL step at lid speed), since the CFL step would
    # grow without bound as the flow comes to rest
    gr = hb.make_grid(2, [n, n], 1.0 / n)
    ctx = hb.Context(gr, fl, opts)
    y0 = ctx.yield_test(us)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    crep, crc = ctx.run_cessation(us, ps, max_steps=max_steps, dt=0.5 / n)
    torch.cuda.synchronize()
    t_cess = time.perf_counter() - t0
    ctx.close()
    return {
        "workload": "2D lid-driven cavity %d^2, Bingham HB=1, Re=100, Pa=100, from rest to steady state "
                    "(largest relative change of u over a step below %g)" % (n, tol),
        "direct": {"grid": n, "steps": rep.steps, "steady": bool(rep.steady), "t": rep.t, "s": t_direct},
        "sequenced": {"grids": [n >> (levels - l) for l in range(levels + 1)], "steps": [r.steps for r in reps],
                      "steady": [bool(r.steady) for r in reps], "s": t_seq},
        "speedup": t_direct / t_seq,
        "max_rel_diff_of_final_u": diff,
        "cessation": {"yielded_fraction_at_steady_state": y0.yielded / y0.cells, "dt": 0.5 / n,
                      "steps": crep.steps, "stopped": bool(crep.stopped), "t_c": crep.t, "s": t_cess},
    }


def run_batch(steps, warmup, precision=0, count=64, seed=0):
    """The batched sweep: count 2D cavities with SplitMix64-drawn sizes and
    parameters, all stepped together (one launch per multigrid kernel)."""
    import torch
    from paper_1803_00417_amd import hb, inputs
    cav = inputs.batch_cavities(count=count, seed=seed)
    grids = [hb.lid_cavity(2, d["n"]) for d in cav]
    fluids = [hb.make_fluid(Re=d["Re"], HB=d["HB"], n=d["nidx"], Pa=d["Pa"]) for d in cav]
    bctx = hb.BatchContext(grids, fluids, hb.make_step_opts(cfl=cav[0]["cfl"], precision=precision))
    us = [torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda") for g in grids]
    ps = [torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda") for g in grids]
    for _ in range(warmup):
        bctx.step(us, ps, report=False)
    torch.cuda.synchronize()
    cyc = [0, 0, 0]
    t0 = time.perf_counter()
    for k in range(steps):
        reps = bctx.step(us, ps, report=True)
        cyc[0] += max(r.mac.cycles for r in reps)
        cyc[1] += max(r.visc.cycles for r in reps)
        cyc[2] += max(r.proj.cycles for r in reps)
        print("[bench] batch%d %s step %d/%d" % (count, "mixed" if precision else "fp64", k + 1, steps),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    bctx.close()
    cells = sum(d["n"] ** 2 for d in cav)
    return {"value": cells * steps / T, "unit": "cell-steps/s", "ms_per_step": 1e3 * T / steps, "steps": steps,
            "warmup": warmup, "cells": cells, "max_cycles_per_step_mac_visc_proj": [x / steps for x in cyc],
            "desc": "%d 2D lid-driven cavities, N from {64,96,128,192,256}, Bi log-uniform [0.1,100], "
                    "n uniform [0.3,1.5], Re log-uniform [1,1000], m=1e3 (SplitMix64 seed %d), one batched "
                    "step" % (count, seed)}


def cpu_baseline(name, nsteps):
    """The FP64 oracle on the first nsteps steps of the workload from rest
    (single thread); returns the record and the oracle's u, p after them."""
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
    rec = dict(value=ncell * nsteps / T, unit="cell-steps/s", cores=1, kind="oracle",
               sample="first %d step(s) of the %s workload from rest, single-threaded FP64 C "
                      "oracle (%.1f s)" % (nsteps, name, T))
    return rec, u, p


def error_vs_oracle(name, nsteps, precision, u_o, p_o):
    """max-norm relative difference of u and p after the first nsteps GPU
    steps from rest against the oracle's"""
    import numpy as np
    import torch
    from paper_1803_00417_amd import hb
    ctx, g, w = _context(name, precision)
    u = torch.zeros(hb.cell_shape(g, w["dim"]), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    for _ in range(nsteps):
        ctx.step(u, p, report=False)
    torch.cuda.synchronize()
    ctx.close()
    uh = u.cpu().numpy().reshape(u_o.shape)
    ph = p.cpu().numpy().reshape(p_o.shape)
    eu = float(np.abs(uh - u_o).max() / max(np.abs(u_o).max(), 1e-300))
    ep = float(np.abs(ph - p_o).max() / max(np.abs(p_o).max(), np.abs(u_o).max() ** 2))
    return max(eu, ep)


def _summary(r, w):
    launches, kms, kbytes = r["kt"]
    ach = (kbytes / 1e9) / (kms / 1e3) if kms > 0 else 0.0
    return {"value": r["ncell"] * r["steps"] / r["T"], "unit": "cell-steps/s",
            "ms_per_step": 1e3 * r["T"] / r["steps"], "steps": r["steps"], "warmup": r["warmup"],
            "cycles_per_step_mac_visc_proj": r["cycles"], "cycles_from": "the reported steps (every 10th and the last)", "smoother_GBs": ach, "smoother_frac": ach / HBM_PEAK_GBS,
            "desc": w["desc"]}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1803_00417_amd import hb, inputs  # noqa: F401
    assert torch.cuda.is_available(), "no GPU"
    if a.copy_probe:
        n = a.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_copy": 8 * n, "copies": 5}), flush=True)
        return
    print("[bench] workload %s: %d warm-up + %d timed steps" % (a.workload, a.warmup, a.steps),
          file=sys.stderr, flush=True)
    r = run_gpu(a.workload, a.steps, a.warmup)
    value = r["ncell"] * r["steps"] / r["T"]
    launches, kms, kbytes = r["kt"]
    achieved = (kbytes / 1e9) / (kms / 1e3) if kms > 0 else 0.0
    w = inputs.WORKLOADS[a.workload]
    # the 2D kernel (and its traffic) depends on the candidate the context
    # kept for the finest level: its rows are keyed by tile and sweeps per
    # launch (the thread count does not change what a launch reads)
    t0 = r["tiles"]["tensor"][0] if r["tiles"]["tensor"] else None
    if w["dim"] == 2:
        tx, ty, th, sw = t0 or (0, 0, 0, 0)
        kname = "fine2d@%dx%ds%d" % (tx, ty, sw)
        klabel = ("%s (2D: %s of both velocity components in one launch, finest level, tile %dx%d, %d threads)"
                  % ("k_tsweep2" if th == 256 else "k_tsweepN", "one red-black sweep" if sw == 1
                     else "%d red-black sweeps" % sw, tx, ty, th))
    else:
        kname = "hb::k_trb3<true,double>"
        klabel = "k_trb3 (3D: one colour of one velocity component, finest level)"
    wname = "cavity2d_512" if w["dim"] == 2 else "cavity3d_128"
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, wname),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-probe scaled)",
                "kernel": klabel,
                "launches": launches, "timed_every": KT_PERIOD, "avg_launch_us": 1e3 * kms / max(launches, 1),
                "alg_bytes_per_launch": kbytes / max(launches, 1)}
    out = {"metric": "cell-steps/s", "value": value, "unit": "cell-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * r["T"] / r["steps"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w["desc"] + ", from rest, tol 1e-10", "cells": r["ncell"],
                      "cycles_per_step_mac_visc_proj": r["cycles"], "cycles_from": "the reported steps (every 10th and the last)", "autotuned_tiles_per_level": r["tiles"]},
           "roofline": roofline}
    also = {}
    runs = [(a.workload, 1)] if not a.no_mixed else []
    for nm in [x for x in a.also.split(",") if x]:
        runs.append((nm, 0))
        if not a.no_mixed:
            runs.append((nm, 1))
    for nm, prec in runs:
        st = a.steps if nm == a.workload else a.also_steps
        wu = a.warmup if nm == a.workload else 2
        print("[bench] workload %s (%s): %d warm-up + %d timed steps" % (nm, "mixed" if prec else "fp64", wu, st),
              file=sys.stderr, flush=True)
        r2 = run_gpu(nm, st, wu, precision=prec)
        also["%s_%s" % (nm, "mixed" if prec else "fp64")] = _summary(r2, inputs.WORKLOADS[nm])
    if not a.no_learned and inputs.WORKLOADS[a.workload]["dim"] == 2:
        # the learned warm start of the projection solve (weights trained by
        # paper_1803_00417_amd.warm_start on 128^2 cavities)
        for prec in ((0, 1) if not a.no_mixed else (0,)):
            tag = "%s_%s_learned" % (a.workload, "mixed" if prec else "fp64")
            print("[bench] workload %s: %d warm-up + %d timed steps" % (tag, a.warmup, a.steps), file=sys.stderr, flush=True)
            r2 = run_gpu(a.workload, a.steps, a.warmup, precision=prec, learned=True)
            rec = _summary(r2, inputs.WORKLOADS[a.workload])
            rec["warm_start_used_in_solves"] = r2["ws_uses"]
            also[tag] = rec
    if a.batch > 0:
        for prec in ((0, 1) if not a.no_mixed else (0,)):
            print("[bench] batched sweep of %d cavities (%s)" % (a.batch, "mixed" if prec else "fp64"),
                  file=sys.stderr, flush=True)
            also["batch%d_%s" % (a.batch, "mixed" if prec else "fp64")] = run_batch(a.batch_steps, 2, prec, a.batch)
    if a.steady > 0:
        print("[bench] time to steady state at %d^2: from rest, and sequenced from %d^2" % (a.steady, a.steady // 4),
              file=sys.stderr, flush=True)
        also["steady_%d" % a.steady] = run_steady(a.steady)
    if also:
        out["also"] = also
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, %d steps)" % a.cpu_steps, file=sys.stderr, flush=True)
        rec, u_o, p_o = cpu_baseline(a.workload, a.cpu_steps)
        out["cpu_baseline"] = rec
        # error of the GPU paths against the oracle on those same first steps
        err = {"steps": a.cpu_steps, "fp64": error_vs_oracle(a.workload, a.cpu_steps, 0, u_o, p_o)}
        if not a.no_mixed:
            err["mixed"] = error_vs_oracle(a.workload, a.cpu_steps, 1, u_o, p_o)
        out["error_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
