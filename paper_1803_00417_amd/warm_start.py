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
