"""Training data and training loop of the learned warm start.

The network (paper_1803_00417_amd.hb.Net, BF16 U-Net, library kernels)
maps the initial residual of a nodal projection solve, r0 = b - K p_prev
scaled by 1/|r0|_inf and averaged to cells, to the shape of the correction
e = phi - p_prev (scaled by 1/|e|_inf, cells).  The library rescales the
prediction by least squares and keeps it only when it lowers the residual,
so the multigrid solve and its 1e-10 tolerance decide the answer.

Data come from the solver itself: seeded 2D lid-driven cavities with
Herschel-Bulkley parameters drawn like the batched sweep (SplitMix64), every
projection solve captured through hb_capture.
"""
import os

import numpy as np
import torch

from . import hb, inputs

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "ws_unet_nodal.npy")


def node_to_cell(v):
    """mean of the four corner nodes of every cell (2D, wall axes)"""
    return 0.25 * (v[:-1, :-1] + v[1:, :-1] + v[:-1, 1:] + v[1:, 1:])


def cavity_samples(n, count, steps, seed, every=1, Pa=None):
    """(inputs, targets) float32 GPU tensors [N][n][n][1] from `count`
    cavities of n^2 cells run `steps` steps from rest, one sample per
    `every` steps after the first two"""
    xs, ts = [], []
    for d in inputs.batch_cavities(count=count, seed=seed, sizes=(n,)):
        g = hb.lid_cavity(2, n)
        fl = hb.make_fluid(Re=d["Re"], HB=d["HB"], n=d["nidx"], Pa=Pa if Pa is not None else d["Pa"])
        ctx = hb.Context(g, fl, hb.make_step_opts(cfl=d["cfl"]))
        ctx.capture(True)
        u = torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda")
        p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
        r0 = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
        e = torch.zeros_like(r0)
        for k in range(steps):
            ctx.step(u, p, report=False)
            if k < 2 or (k - 2) % every:
                continue
            ctx.capture_read(r0, e)
            rn, en = r0[0].abs().max(), e[0].abs().max()
            if rn == 0 or en == 0:
                continue
            xs.append(node_to_cell(r0[0] / rn).float())
            ts.append(node_to_cell(e[0] / en).float())
        ctx.close()
    X = torch.stack(xs)[..., None].contiguous()
    T = torch.stack(ts)[..., None].contiguous()
    return X, T


def train(net, X, T, iters, batch=8, lr=1e-3, seed=0, log_every=0):
    """Adam on random minibatches; returns the loss history"""
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    N = X.shape[0]
    for it in range(iters):
        idx = torch.randint(0, N, (min(batch, N),), generator=g).to(X.device)
        loss = net.train_step(X[idx].contiguous(), T[idx].contiguous(), lr)
        hist.append(loss)
        if log_every and (it + 1) % log_every == 0:
            print("[warm start] iteration %d loss %.4e" % (it + 1, loss), flush=True)
    return hist


def save(net, path=WEIGHTS):
    np.save(path, net.get_params())


def load_net(path=WEIGHTS):
    """the trained network, or None when no weights are present"""
    if not os.path.exists(path):
        return None
    w = np.load(path, allow_pickle=False)
    net = hb.Net(1, 1)
    net.set_params(w)
    return net


def _event_ms(fn, reps=10):
    """mean device time of fn() over reps calls (after one untimed call)"""
    fn()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def solve_ceiling(n=512, HB=10.0, nidx=0.5, Re=1000.0, Pa=1e4, warmup=20, samples=4,
                  eps=(1.0, 0.3, 0.1, 0.03, 0.01, 1e-3, 1e-4)):
    """What any warm start of the two solves of a step could gain at most.

    For `samples` steps of a 2D lid-driven cavity (after `warmup` steps from
    rest) the viscous and the projection solves are captured (initial
    residual r0 of the previous-step guess x0, correction e = x - x0).  A
    predictor whose error is a fraction eps of the previous-step guess's
    starts from x0 + (1 - eps) e; by linearity its solve is the solve of
    A d = r0 from d = (1 - eps) e to the step's own tolerance, which is run
    here (same operator, walls at rest, same cycle).  Returned per solve:
    the mean V-cycles for every eps (eps = 1 is the previous-step guess),
    the measured time per V-cycle, and the time of one inference of the
    U-Net at this size.  A predictor pays only where the cycles it saves
    cost more than its inference."""
    g = hb.lid_cavity(2, n)
    fl = hb.make_fluid(Re=Re, HB=HB, n=nidx, Pa=Pa)
    opts = hb.make_step_opts()
    ctx = hb.Context(g, fl, opts)
    gh = hb.make_grid(2, [n, n], 1.0 / n)
    ctxh = hb.Context(gh, fl, opts)
    u = torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.step(u, p, report=False)
    ctx.capture(True, hb.OP_VISC)
    ctx.capture(True, hb.OP_NODAL)
    rv = torch.zeros_like(u)
    ev = torch.zeros_like(u)
    rp = torch.zeros_like(p)
    ep = torch.zeros_like(p)
    eta = torch.zeros(hb.cell_shape(g)[1:], dtype=torch.float64, device="cuda")
    cyc = {"visc": {e: [] for e in eps}, "proj": {e: [] for e in eps}}
    actual = {"visc": [], "proj": []}
    ms = {"visc": [], "proj": []}
    for _ in range(samples):
        u0 = u.clone()
        rep = ctx.step(u, p, report=True)
        ctx.capture_read(rv, ev, hb.OP_VISC)
        ctx.capture_read(rp, ep, hb.OP_NODAL)
        ctx.viscosity(u0, eta)
        actual["visc"].append(rep.visc.cycles)
        actual["proj"].append(rep.proj.cycles)
        dt_op = 2.0 * opts.theta * rep.dt
        for name, op, r0, e, bn, kry in (("visc", hb.OP_VISC, rv, ev, rep.visc.bnorm, 1),
                                         ("proj", hb.OP_NODAL, rp, ep, rep.proj.bnorm, 0)):
            rn = float(r0.abs().max())
            if rn == 0.0:
                continue
            o = hb.mg_opts(tol=1e-10 * bn / rn, max_cycles=200, krylov=kry)
            for e_ in eps:
                d = ((1.0 - e_) * e).contiguous()
                mrep, _ = ctxh.mg_solve(op, eta if op == hb.OP_VISC else None, dt_op, r0, d, opts=o,
                                        allow=(hb.ERR_NOCONV,))
                cyc[name][e_].append(mrep.cycles)
            # time per V-cycle: the solve from the previous-step guess
            def full(op=op, r0=r0, o=o):
                d = torch.zeros_like(r0)
                ctxh.mg_solve(op, eta if op == hb.OP_VISC else None, dt_op, r0, d, opts=o, allow=(hb.ERR_NOCONV,))
            t = _event_ms(full, reps=3)
            ms[name].append(t / max(cyc[name][1.0][-1], 1))
    ctx.close()
    ctxh.close()
    net = hb.Net(1, 1, seed=1)
    x = torch.zeros((1, n, n, 1), dtype=torch.float32, device="cuda")
    t_inf = _event_ms(lambda: net.forward(x))
    out = {"n": n, "samples": samples, "inference_ms": t_inf, "solves": {}}
    for name in ("visc", "proj"):
        mean = {e: float(np.mean(v)) for e, v in cyc[name].items() if v}
        mpc = float(np.mean(ms[name])) if ms[name] else 0.0
        base = mean.get(1.0, 0.0)
        out["solves"][name] = {
            "step_cycles": float(np.mean(actual[name])),
            "cycles_by_eps": mean,
            "ms_per_cycle": mpc,
            "best_saving_ms": {e: (base - c) * mpc for e, c in mean.items()},
            "net_gain_ms": {e: (base - c) * mpc - t_inf for e, c in mean.items()},
        }
    return out


def main():
    """train on 128^2 cavities (seeds 1..), save the weights"""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--cavities", type=int, default=12)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args()
    X, T = cavity_samples(a.n, a.cavities, a.steps, seed=1, Pa=1e4)
    print("[warm start] %d samples of %d^2" % (X.shape[0], a.n), flush=True)
    net = hb.Net(1, 1, seed=7)
    train(net, X, T, a.iters, lr=a.lr, log_every=100)
    save(net, a.out)
    print("[warm start] weights written to %s" % a.out, flush=True)


if __name__ == "__main__":
    main()
