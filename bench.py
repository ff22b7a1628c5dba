"""Throughput of the Herschel-Bulkley cavity step on one MI355X.

A step is one full pass of the hot path: viscosity, Godunov advection with
the MAC projection, the tensor viscous multigrid solve and the nodal
projection, all solves to a relative residual of 1e-10.  The headline
workload is the 2D 512^2 lid-driven cavity (Herschel-Bulkley n = 0.5,
Bi = 10, Re = 1000, Pa = 1e4, CFL 0.5): W untimed warm-up steps on the
context, then R repeats of K timed steps, each repeat starting from rest
(K = 200 is the workload's whole run); value = cells x K / T for the median
repeat, with the inputs resident in HBM and every cycle in FP64.  Cycle
counts are summed over every step of one more pass of the same K steps with
step reports on (the path is deterministic, so they are the timed runs'
counts).

Beside it: the paper's timing protocol (Sec. V: constant dt, 100 steps,
then the mean of the next 10), mixed-precision cycles, the n = 1.5 fluid,
the 3D 128^3 Bingham cube, the batched sweep, the learned warm start, time
to steady state with grid sequencing, and the cessation time of the paper's
Re = 1, Bi = 10 cavity.  The roofline object describes the finest-level
tensor smoother, timed with HIP events on the library's stream inside the
timed region, its algorithmic bytes counted per red-black sweep (7 words
per cell in 2D); step_alg_GBs applies the per-cycle byte model of the whole
step to the measured cycle counts.  cpu_baseline times the FP64 oracle (an
OpenMP build on the host's cores, and one thread) on the first steps of the
workload, whose results the GPU runs are also compared with.
"""
import argparse
import json
import os
import statistics
import subprocess
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
# algorithmic bytes per cell of the multigrid passes and of the rest of a
# step (FP64; V(2,2), one read of each input and one write of each output
# per pass, summed over the hierarchy): MAC or nodal V-cycle, tensor
# V-cycle, everything outside the solves
STEP_BYTES = {2: (200.0, 453.0, 300.0), 3: (168.0, 550.0, 480.0)}


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
    ap.add_argument("--steps", type=int, default=200, help="timed steps per repeat, from rest")
    ap.add_argument("--warmup", type=int, default=10, help="untimed steps before the repeats")
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--workload", default="cavity2d_512_n0.5")
    ap.add_argument("--also", default="cavity2d_512_n1.5,cavity3d_128",
                    help="comma-separated further workloads ('' for none)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision runs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start runs")
    ap.add_argument("--no-paper-protocol", action="store_true")
    ap.add_argument("--batch", type=int, default=64, help="cavities of the batched sweep (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200, help="batched steps from rest (as the headline's run)")
    ap.add_argument("--steady", type=int, default=256, metavar="N",
                    help="time to steady state on an N^2 cavity, from rest and by grid sequencing from "
                         "(N/4)^2, then the cessation of the steady flow (0: skip)")
    ap.add_argument("--cessation", type=int, default=256, metavar="N",
                    help="cessation time of the paper's Re=1, Bi=10, Pa=400 cavity on N^2 (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates the HBM byte counters) and exit")
    return ap.parse_args()


def _say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _context(name, precision, opts_kw=None):
    from paper_1803_00417_amd import hb, inputs
    w = inputs.WORKLOADS[name]
    g = hb.lid_cavity(w["dim"], w["n"])
    fl = hb.make_fluid(Re=w["Re"], HB=w["HB"], n=w["nidx"], Pa=w["Pa"])
    return hb.Context(g, fl, hb.make_step_opts(cfl=w["cfl"], precision=precision, **(opts_kw or {}))), g, w


def _state(g, dim):
    import torch
    from paper_1803_00417_amd import hb
    u = torch.zeros(hb.cell_shape(g, dim), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    return u, p


def run_gpu(name, steps, warmup, repeats, precision=0, timing=True, learned=False):
    """W warm-up steps, then `repeats` timed runs of `steps` steps from rest,
    then one more run from rest with reports on every step (cycle counts)."""
    import torch
    from paper_1803_00417_amd import hb
    ctx, g, w = _context(name, precision)
    if learned:
        from paper_1803_00417_amd import warm_start
        net = warm_start.load_net()
        if net is None:
            raise RuntimeError("no trained warm-start weights (run python -m paper_1803_00417_amd.warm_start)")
        ctx.set_warm_start(net)
    u, p = _state(g, w["dim"])
    for _ in range(warmup):
        ctx.step(u, p, report=False)
    torch.cuda.synchronize()
    if timing:
        # every KT_PERIOD-th finest-level smoother launch is timed: a timed
        # launch costs the host more, and timing them all would slow the run
        ctx.kernel_timing(KT_PERIOD)
    Ts = []
    for r in range(repeats):
        u.zero_()
        p.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.step(u, p, report=False)
        torch.cuda.synchronize()
        Ts.append(time.perf_counter() - t0)
        _say("%s %s repeat %d/%d: %.3f ms/step" % (name, "mixed" if precision else "fp64", r + 1, repeats,
                                                    1e3 * Ts[-1] / steps))
    kt = ctx.kernel_timing_read() if timing else (0, 0.0, 0.0)
    ctx.kernel_timing(False)
    # the cycle counts of those runs: the same steps again with reports
    u.zero_()
    p.zero_()
    cyc = [0, 0, 0]
    last = None
    for _ in range(steps):
        last = ctx.step(u, p, report=True)
        cyc[0] += last.mac.cycles
        cyc[1] += last.visc.cycles
        cyc[2] += last.proj.cycles
    ncell = g.n[0] * g.n[1] * g.n[2]
    uses = ctx.warm_start_uses() if learned else 0
    tiles = {"tensor": [ctx.tile_config(hb.OP_VISC, lv) for lv in range(12)],
             "nodal": [ctx.tile_config(hb.OP_NODAL, lv) for lv in range(12)]}
    tiles = {k: [list(t) if t else None for t in v] for k, v in tiles.items()}
    for k in tiles:
        while tiles[k] and tiles[k][-1] is None:
            tiles[k].pop()
    ctx.close()
    T = statistics.median(Ts)
    return dict(T=T, Ts=Ts, ncell=ncell, dim=w["dim"], steps=steps, warmup=warmup, repeats=repeats,
                cycles=[c / steps for c in cyc], kt=kt, ws_uses=uses, tiles=tiles,
                final_max_u=last.max_u if last else None)


def run_paper_protocol(name, precision, repeats, settle=100, window=10):
    """Sec. V: constant dt (the CFL step at lid speed), `settle` untimed
    steps from rest, then the mean time of the next `window` steps; the
    median over repeats"""
    import torch
    ctx, g, w = _context(name, precision)
    u, p = _state(g, w["dim"])
    dt = w["cfl"] * g.h / 1.0
    means = []
    for _ in range(repeats):
        u.zero_()
        p.zero_()
        for _ in range(settle):
            ctx.step(u, p, dt=dt, report=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(window):
            ctx.step(u, p, dt=dt, report=False)
        torch.cuda.synchronize()
        means.append((time.perf_counter() - t0) / window)
    rep = ctx.step(u, p, dt=dt, report=True)
    ctx.close()
    ncell = g.n[0] * g.n[1] * g.n[2]
    m = statistics.median(means)
    return {"value": ncell / m, "unit": "cell-steps/s", "ms_per_step": 1e3 * m, "dt": dt,
            "settle_steps": settle, "window_steps": window, "repeats": repeats,
            "ms_per_step_each": [1e3 * x for x in means],
            "cycles_mac_visc_proj_after": [rep.mac.cycles, rep.visc.cycles, rep.proj.cycles],
            "desc": "constant dt = CFL h / U_lid, %d steps from rest, then the mean of the next %d (Sec. V)"
                    % (settle, window)}


def step_bytes_per_cell(dim, cycles):
    bm, bv, bo = STEP_BYTES[dim]
    return bm * cycles[0] + bv * cycles[1] + bm * cycles[2] + bo


def run_steady(n, levels=2, tol=1e-5, max_steps=12000):
    """Time to steady state (Sec. III.A test, tolerance 1e-5) on an n^2 lid
    cavity: from rest on n^2, and by grid sequencing (Sec. III.C) from rest
    on (n / 2^levels)^2, refined `levels` times.  Both runs are single
    library calls (hb_run_steady, hb_run_sequenced).  Then the cessation of
    the sequenced steady flow at a constant step h/2."""
    import torch
    from paper_1803_00417_amd import hb
    fl = hb.make_fluid(Re=100.0, HB=1.0, n=1.0, Pa=100.0)
    opts = hb.make_step_opts()
    g = hb.lid_cavity(2, n)
    ctx = hb.Context(g, fl, opts)
    u, p = _state(g, 2)
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
        "sequenced": {"grids": [n >> (levels - lv) for lv in range(levels + 1)], "steps": [r.steps for r in reps],
                      "steady": [bool(r.steady) for r in reps], "s": t_seq},
        "speedup": t_direct / t_seq,
        "max_rel_diff_of_final_u": diff,
        "cessation": {"yielded_fraction_at_steady_state": y0.yielded / y0.cells, "dt": 0.5 / n,
                      "steps": crep.steps, "stopped": bool(crep.stopped), "t_c": crep.t, "s": t_cess},
    }


def run_paper_cessation(n, dt=2.5e-6, t_stop=0.0205552):
    """The cessation experiment of Sec. IV (fig:rest-steady-cessation-2d):
    Re = 1, Bi = 10, Pa = 400 from rest; the lid stops at t = 0.0205552,
    the time the paper gives for its steady state; t_c is the time from
    then until no cell is yielded (paper: 1.2844e-3 at 256^2).  Constant
    dt, backward-Euler viscous update."""
    import torch
    from paper_1803_00417_amd import hb
    fl = hb.make_fluid(Re=1.0, HB=10.0, n=1.0, Pa=400.0)
    opts = hb.make_step_opts(theta=1.0)
    g = hb.lid_cavity(2, n)
    ctx = hb.Context(g, fl, opts)
    u, p = _state(g, 2)
    nsteps = int(round(t_stop / dt))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep, rc = ctx.run_steady(u, p, tol=1e-300, max_steps=nsteps, dt=dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.close()
    ctx = hb.Context(hb.make_grid(2, [n, n], 1.0 / n), fl, opts)
    y0 = ctx.yield_test(u)
    crep, crc = ctx.run_cessation(u, p, max_steps=100000, dt=dt)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.close()
    return {"workload": "2D lid-driven cavity %d^2, Bingham Re=1, Bi=10, Pa=400 (Sec. IV); lid stopped at "
                        "t=%g" % (n, t_stop),
            "dt": dt, "theta": 1.0, "steps_to_stop": rep.steps, "change_per_step_at_stop": rep.change,
            "yielded_fraction_at_stop": y0.yielded / y0.cells, "cessation_steps": crep.steps,
            "stopped": bool(crep.stopped), "t_c": crep.t, "t_c_paper": 1.2844e-3,
            "rel_diff": crep.t / 1.2844e-3 - 1.0, "s": t2 - t0}


def run_batch(steps, warmup, precision=0, count=64, seed=0):
    """The batched sweep: count 2D cavities with SplitMix64-drawn sizes and
    parameters, all stepped together (one launch per multigrid kernel).  The
    headline's protocol: W warm-up steps, then `steps` timed steps from
    rest without reports, then the same steps from rest again with reports
    (cycle counts)."""
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

    def rest():
        for t in us + ps:
            t.zero_()

    rest()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        bctx.step(us, ps, report=False)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    rest()
    cyc = [0, 0, 0]
    for k in range(steps):
        reps = bctx.step(us, ps, report=True)
        cyc[0] += max(r.mac.cycles for r in reps)
        cyc[1] += max(r.visc.cycles for r in reps)
        cyc[2] += max(r.proj.cycles for r in reps)
    bctx.close()
    cells = sum(d["n"] ** 2 for d in cav)
    return {"value": cells * steps / T, "unit": "cell-steps/s", "ms_per_step": 1e3 * T / steps, "steps": steps,
            "warmup": warmup, "cells": cells, "max_cycles_per_step_mac_visc_proj": [x / steps for x in cyc],
            "desc": "%d 2D lid-driven cavities, N from {64,96,128,192,256}, Bi log-uniform [0.1,100], "
                    "n uniform [0.3,1.5], Re log-uniform [1,1000], m=1e3 (SplitMix64 seed %d), %d batched "
                    "steps from rest" % (count, seed, steps)}


def _host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or avail
    return model, avail, min(threads, avail)


_ORACLE_RUN = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import orc
from paper_1803_00417_amd import inputs
name, nsteps, out = sys.argv[2], int(sys.argv[3]), sys.argv[4]
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
if out != "-":
    np.savez(out, u=u, p=p)
print(json.dumps({"T": T, "lib": orc.LIB}))
"""


def oracle_run(name, nsteps, threads, save=None):
    """The oracle on the first nsteps steps of the workload from rest, in a
    child process (threads > 1: the OpenMP timing build); returns (seconds,
    u, p) with u, p loaded when save is a path."""
    import numpy as np
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = str(threads)
    if threads > 1:
        env["ORC_OMP"] = "1"
    else:
        env.pop("ORC_OMP", None)
    r = subprocess.run([sys.executable, "-c", _ORACLE_RUN, ROOT, name, str(nsteps), save or "-"],
                       capture_output=True, text=True, env=env, check=True)
    T = json.loads(r.stdout.strip().splitlines()[-1])["T"]
    if save:
        d = np.load(save if save.endswith(".npz") else save + ".npz")
        return T, d["u"], d["p"]
    return T, None, None


def cpu_baseline(name, nsteps, tmpdir):
    """The FP64 oracle on the first nsteps steps of the workload from rest:
    the OpenMP build on every host core this process may use, and one
    thread (whose u, p the GPU runs are compared with)."""
    from paper_1803_00417_amd import inputs
    w = inputs.WORKLOADS[name]
    ncell = w["n"] ** w["dim"]
    model, avail, threads = _host_cpu()
    save = os.path.join(tmpdir, "oracle_%s_%d.npz" % (name, nsteps))
    T1, u, p = oracle_run(name, nsteps, 1, save=save)
    Tn, _, _ = oracle_run(name, nsteps, threads) if threads > 1 else (T1, None, None)
    rec = dict(value=ncell * nsteps / Tn, unit="cell-steps/s", cores=threads, kind="oracle",
               sample="first %d step(s) of the %s workload from rest, FP64 C oracle, OpenMP build on %d "
                      "threads (%.1f s; CPU: %s, %d usable cores)" % (nsteps, name, threads, Tn, model, avail),
               one_thread={"value": ncell * nsteps / T1, "cores": 1, "s": T1})
    return rec, u, p


def error_vs_oracle(name, nsteps, precision, u_o, p_o):
    """max-norm relative difference of u and p after the first nsteps GPU
    steps from rest against the oracle's"""
    import numpy as np
    import torch
    ctx, g, w = _context(name, precision)
    u, p = _state(g, w["dim"])
    for _ in range(nsteps):
        ctx.step(u, p, report=False)
    torch.cuda.synchronize()
    ctx.close()
    uh = u.cpu().numpy().reshape(u_o.shape)
    ph = p.cpu().numpy().reshape(p_o.shape)
    eu = float(np.abs(uh - u_o).max() / max(np.abs(u_o).max(), 1e-300))
    ep = float(np.abs(ph - p_o).max() / max(np.abs(p_o).max(), np.abs(u_o).max() ** 2))
    return max(eu, ep)


def _smoother(r):
    launches, kms, kbytes = r["kt"]
    ach = (kbytes / 1e9) / (kms / 1e3) if kms > 0 else 0.0
    return ach, launches, kms, kbytes


def _summary(r, w):
    ach, _, _, _ = _smoother(r)
    ms = 1e3 * r["T"] / r["steps"]
    sb = step_bytes_per_cell(r["dim"], r["cycles"]) * r["ncell"]
    return {"value": r["ncell"] * r["steps"] / r["T"], "unit": "cell-steps/s", "ms_per_step": ms,
            "ms_per_step_each": [1e3 * t / r["steps"] for t in r["Ts"]], "steps": r["steps"],
            "warmup": r["warmup"], "repeats": r["repeats"],
            "cycles_per_step_mac_visc_proj": r["cycles"], "cycles_from": "every step of the run",
            "step_alg_GBs": sb / 1e9 / (ms / 1e3), "step_alg_frac": sb / 1e9 / (ms / 1e3) / HBM_PEAK_GBS,
            "smoother_GBs": ach, "smoother_frac": ach / HBM_PEAK_GBS, "desc": w["desc"]}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import tempfile
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
    _say("workload %s: %d warm-up steps, then %d x %d timed steps from rest" % (a.workload, a.warmup, a.repeats,
                                                                               a.steps))
    r = run_gpu(a.workload, a.steps, a.warmup, a.repeats)
    value = r["ncell"] * r["steps"] / r["T"]
    achieved, launches, kms, kbytes = _smoother(r)
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
    ms = 1e3 * r["T"] / r["steps"]
    sb = step_bytes_per_cell(w["dim"], r["cycles"]) * r["ncell"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, wname),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-probe scaled)",
                "kernel": klabel,
                "alg_bytes_unit": "per red-black sweep of both components: 2 x, eta/Re and 2 b read, 2 x written "
                                  "(56 B/cell) times the sweeps of the launch, plus the folded transfer's coarse words",
                "launches": launches, "timed_every": KT_PERIOD, "avg_launch_us": 1e3 * kms / max(launches, 1),
                "alg_bytes_per_launch": kbytes / max(launches, 1),
                "step_alg_GBs": sb / 1e9 / (ms / 1e3), "step_alg_frac": sb / 1e9 / (ms / 1e3) / HBM_PEAK_GBS,
                "step_alg_bytes": sb}
    out = {"metric": "cell-steps/s", "value": value, "unit": "cell-steps/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": w["desc"] + ", %d steps from rest, tol 1e-10; median of %d repeats"
                                              % (a.steps, a.repeats),
                      "cells": r["ncell"], "repeats": a.repeats,
                      "ms_per_step_each": [1e3 * t / r["steps"] for t in r["Ts"]],
                      "cycles_per_step_mac_visc_proj": r["cycles"], "cycles_from": "every step of the run",
                      "autotuned_tiles_per_level": r["tiles"]},
           "roofline": roofline}
    also = {}
    if not a.no_paper_protocol:
        _say("paper protocol (constant dt, 100 + 10 steps) on %s" % a.workload)
        also["%s_paper_protocol_fp64" % a.workload] = run_paper_protocol(a.workload, 0, a.repeats)
    runs = [(a.workload, 1)] if not a.no_mixed else []
    for nm in [x for x in a.also.split(",") if x]:
        runs.append((nm, 0))
        if not a.no_mixed:
            runs.append((nm, 1))
    for nm, prec in runs:
        wn = inputs.WORKLOADS[nm]
        st = a.steps if nm == a.workload else wn["steps"]
        _say("workload %s (%s): %d warm-up, %d x %d timed steps" % (nm, "mixed" if prec else "fp64", 5, a.repeats, st))
        r2 = run_gpu(nm, st, 5, a.repeats, precision=prec)
        also["%s_%s" % (nm, "mixed" if prec else "fp64")] = _summary(r2, wn)
    if not a.no_learned and inputs.WORKLOADS[a.workload]["dim"] == 2:
        # the learned warm start of the projection solve (weights trained by
        # paper_1803_00417_amd.warm_start on 128^2 cavities)
        for prec in ((0, 1) if not a.no_mixed else (0,)):
            tag = "%s_%s_learned" % (a.workload, "mixed" if prec else "fp64")
            _say("workload %s" % tag)
            r2 = run_gpu(a.workload, a.steps, a.warmup, 1, precision=prec, learned=True)
            rec = _summary(r2, inputs.WORKLOADS[a.workload])
            rec["warm_start_used_in_solves"] = r2["ws_uses"]
            also[tag] = rec
    if a.batch > 0:
        for prec in ((0, 1) if not a.no_mixed else (0,)):
            _say("batched sweep of %d cavities (%s)" % (a.batch, "mixed" if prec else "fp64"))
            also["batch%d_%s" % (a.batch, "mixed" if prec else "fp64")] = run_batch(a.batch_steps, 2, prec, a.batch)
    if a.steady > 0:
        _say("time to steady state at %d^2: from rest, and sequenced from %d^2" % (a.steady, a.steady // 4))
        also["steady_%d" % a.steady] = run_steady(a.steady)
    if a.cessation > 0:
        _say("cessation of the paper's Re=1, Bi=10 cavity at %d^2" % a.cessation)
        also["cessation_paper_%d" % a.cessation] = run_paper_cessation(a.cessation)
    if also:
        out["also"] = also
    if not a.no_cpu_baseline:
        with tempfile.TemporaryDirectory() as td:
            _say("cpu baseline (oracle, %d steps, OpenMP and one thread)" % a.cpu_steps)
            rec, u_o, p_o = cpu_baseline(a.workload, a.cpu_steps, td)
            out["cpu_baseline"] = rec
            # every mode of the GPU path against the oracle on those steps
            err = {"steps": a.cpu_steps, a.workload + "_fp64": error_vs_oracle(a.workload, a.cpu_steps, 0, u_o, p_o)}
            if not a.no_mixed:
                err[a.workload + "_mixed"] = error_vs_oracle(a.workload, a.cpu_steps, 1, u_o, p_o)
            for nm in [x for x in a.also.split(",") if x]:
                nst = 1 if inputs.WORKLOADS[nm]["dim"] == 3 else a.cpu_steps
                _say("oracle reference for %s (%d step(s))" % (nm, nst))
                _, _, threads = _host_cpu()
                save = os.path.join(td, "ref_%s.npz" % nm)
                _, uo2, po2 = oracle_run(nm, nst, threads, save=save)
                err[nm + "_fp64"] = error_vs_oracle(nm, nst, 0, uo2, po2)
                if not a.no_mixed:
                    err[nm + "_mixed"] = error_vs_oracle(nm, nst, 1, uo2, po2)
                err[nm + "_steps"] = nst
            out["error_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
