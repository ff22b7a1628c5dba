"""The BF16 U-Net kernels (MFMA forward, input and weight gradients, Adam)
against the CPU reference in oracle/unet.py, and the learned warm start of
the nodal projection solve.

Two references.  (1) The reference with BF16 emulation rounds where the GPU
stores BF16 (weights, input, activations, the masked output gradient) and
accumulates in FP64; the GPU accumulates in FP32, so the two differ by FP32
rounding (~1e-7) unless a value lands within that distance of a BF16
rounding boundary and rounds the other way, which on a 2 x 16 x 16 batch
does not happen (checked), while on larger images a few such flips give
differences of 1e-3.  The bar on 2 x 16 x 16 is 1e-5 for the output and the
whole gradient, 1e-4 per layer: any mistake in taps, channels, transposes or
reductions is of order one.  (2) The exact FP64 reference: BF16 storage
through 15 layers costs about 1e-2 relative, so the output is held to 3e-2
and the gradient to 5e-2.
"""
import numpy as np
import pytest

from oracle import orc, unet
from paper_1803_00417_amd import inputs

pytestmark = pytest.mark.gpu

hb = pytest.importorskip("paper_1803_00417_amd.hb")


def _say(*a):
    print(*a, flush=True)


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _batch(seed, n=2, H=16, W=24):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, H, W, 1)).astype(np.float32), rng.standard_normal((n, H, W, 1)).astype(np.float32)


def test_param_count_matches_reference():
    net = hb.Net(1, 1, seed=0)
    assert net.nparams == unet.param_count()


def test_forward_matches_reference():
    _say("nn forward")
    net = hb.Net(1, 1, seed=3)
    p = net.get_params().astype(np.float64)
    x, _ = _batch(1, n=2, H=16, W=16)
    y = net.forward(_t(x)).cpu().numpy()
    x64 = x.astype(np.float64)
    e_emu = _rel(y, unet.forward(p, x64, bf16=True)[0][..., :1])
    e_ref = _rel(y, unet.forward(p, x64)[0][..., :1])
    _say("  forward relative error: vs BF16 emulation %.3e, vs FP64 %.3e" % (e_emu, e_ref))
    assert e_emu < 1e-5 and e_ref < 3e-2


def test_gradients_match_reference():
    _say("nn gradient")
    net = hb.Net(1, 1, seed=4)
    p = net.get_params().astype(np.float64)
    x, t = _batch(2, n=2, H=16, W=16)
    loss, g = net.grad(_t(x), _t(t))
    x64, t64 = x.astype(np.float64), t.astype(np.float64)
    le, ge = unet.loss_and_grad(p, x64, t64, bf16=True)
    lr, gr = unet.loss_and_grad(p, x64, t64)
    _say("  loss %.8e emulated %.8e FP64 %.8e" % (loss, le, lr))
    assert abs(loss - le) <= 1e-6 * le and abs(loss - lr) <= 3e-2 * lr
    e_emu = _rel(g, ge)
    e_ref = _rel(g, gr)
    cos = float(np.dot(g, gr) / (np.linalg.norm(g) * np.linalg.norm(gr)))
    _say("  gradient relative error: vs BF16 emulation %.3e, vs FP64 %.3e (cosine %.6f)" % (e_emu, e_ref, cos))
    # cos >= 1 - eps^2 / 2 for an L2-relative error eps; 0.995 is eps ~ 0.1
    assert e_emu < 1e-5 and e_ref < 5e-2 and cos > 0.995
    o = 0
    for i, (ci, co, _) in enumerate(unet.LAYERS):
        nw = co * 9 * ci
        gw, gew = g[o:o + nw], ge[o:o + nw]
        if i == 0:   # only the first input channel is live
            gw, gew = gw.reshape(co, 9, ci)[..., :1], gew.reshape(co, 9, ci)[..., :1]
        assert _rel(gw, gew) < 1e-4, i
        assert _rel(g[o + nw:o + nw + co], ge[o + nw:o + nw + co]) < 1e-4, i
        o += nw + co


def test_training_reduces_loss():
    _say("nn training")
    net = hb.Net(1, 1, seed=5)
    x, _ = _batch(3, n=4, H=32, W=32)
    # a smooth target the network can represent: a blurred copy of the input
    t = 0.25 * (np.roll(x, 1, axis=1) + np.roll(x, -1, axis=1) + np.roll(x, 1, axis=2) + np.roll(x, -1, axis=2))
    X, T = _t(x), _t(t)
    losses = [net.train_step(X, T, 2e-3) for _ in range(80)]
    _say("  loss %.4e -> %.4e" % (losses[0], losses[-1]))
    assert losses[-1] < 0.3 * losses[0]


def test_nn_rejects_bad_shapes():
    net = hb.Net(1, 1)
    x = _t(np.zeros((1, 12, 16, 1)))
    with pytest.raises(hb.HBError):
        net.forward(x)


def _cavity(n, seed=11):
    d = inputs.batch_cavities(count=1, seed=seed, sizes=(n,))[0]
    g = hb.lid_cavity(2, n)
    fl = hb.make_fluid(Re=d["Re"], HB=d["HB"], n=d["nidx"], Pa=d["Pa"])
    return g, fl, d


def _run(g, fl, steps, net=None):
    import torch
    ctx = hb.Context(g, fl, hb.make_step_opts())
    if net is not None:
        ctx.set_warm_start(net)
    u = torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    cyc = []
    for _ in range(steps):
        rep = ctx.step(u, p)
        assert rep.proj.rel_resid <= 1e-10
        cyc.append(rep.proj.cycles)
    uses = ctx.warm_start_uses()
    ctx.close()
    return u, p, cyc, uses


def test_capture_records_residual_and_correction():
    # K e = r0 - r_final with |r_final| <= 1e-10 |b|: checked with the
    # oracle's stiffness operator
    _say("capture")
    import torch
    g, fl, _ = _cavity(32)
    go = orc.lid_cavity(2, 32)
    ctx = hb.Context(g, fl, hb.make_step_opts())
    ctx.capture(True)
    u = torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    r0 = torch.zeros_like(p)
    e = torch.zeros_like(p)
    for _ in range(3):
        rep = ctx.step(u, p)
    ctx.capture_read(r0, e)
    r0h, eh = r0.cpu().numpy(), e.cpu().numpy()
    Ke = orc.apply_K(go, eh)
    assert np.abs(Ke - r0h).max() <= 1e-9 * max(np.abs(r0h).max(), rep.proj.bnorm) + 1e-12 * np.abs(Ke).max()


def test_untrained_warm_start_is_harmless():
    # whatever the network predicts, the residual check keeps or improves
    # the initial guess, and every solve still meets its tolerance
    _say("warm start fallback")
    g, fl, _ = _cavity(32)
    u0, p0, c0, _ = _run(g, fl, 6)
    net = hb.Net(1, 1, seed=9)
    u1, p1, c1, uses = _run(g, fl, 6, net)
    _say("  cycles plain %s warm %s uses %d" % (c0, c1, uses))
    assert _rel(u1.cpu().numpy(), u0.cpu().numpy()) < 1e-7
    assert sum(c1) <= sum(c0) + len(c0)


def test_trained_warm_start_gain():
    # train on captured solves of seeded 64^2 cavities, evaluate on a
    # held-out cavity: report the projection cycles with and without it
    _say("warm start gain")
    from paper_1803_00417_amd import warm_start
    X, T = warm_start.cavity_samples(64, 4, 24, seed=21)
    net = hb.Net(1, 1, seed=7)
    hist = warm_start.train(net, X, T, 300, batch=8, lr=1e-3)
    _say("  %d samples, loss %.4e -> %.4e" % (X.shape[0], np.mean(hist[:10]), np.mean(hist[-10:])))
    assert np.mean(hist[-10:]) < np.mean(hist[:10])
    g, fl, _ = _cavity(64, seed=99)
    _, _, c0, _ = _run(g, fl, 12)
    _, _, c1, uses = _run(g, fl, 12, net)
    _say("  projection cycles over 12 steps: previous-step guess %d, learned %d (used %d times)"
         % (sum(c0), sum(c1), uses))
    assert sum(c1) <= sum(c0) + 12


@pytest.mark.xfail(strict=True, reason="measured ceiling (warm_start.solve_ceiling at 512^2): the cycles a "
                   "predictor can save cost less than one inference unless its guess is ~100x better than the "
                   "previous step's; if this passes, the learned warm start has started to pay")
def test_learned_warm_start_beats_previous_step_guess():
    # the learned path must take fewer projection cycles and less time than
    # the previous-step guess on a held-out cavity
    import time
    _say("learned vs previous-step guess, time and cycles")
    from paper_1803_00417_amd import warm_start
    net = warm_start.load_net()
    if net is None:
        pytest.skip("no trained weights shipped")
    g, fl, _ = _cavity(128, seed=99)
    t0 = time.perf_counter()
    _, _, c0, _ = _run(g, fl, 16)
    t1 = time.perf_counter()
    _, _, c1, uses = _run(g, fl, 16, net)
    t2 = time.perf_counter()
    _say("  cycles %d -> %d, %.3f s -> %.3f s" % (sum(c0), sum(c1), t1 - t0, t2 - t1))
    assert sum(c1) < sum(c0) and (t2 - t1) < (t1 - t0)


def test_solve_ceiling_machinery():
    # the ceiling analysis replays each captured solve from x0 + (1 - eps) e:
    # eps = 1 reproduces the step's own cycle count, fewer cycles for a
    # better guess, none for the exact correction
    _say("solve ceiling at 64^2")
    from paper_1803_00417_amd import warm_start
    r = warm_start.solve_ceiling(n=64, HB=1.0, nidx=1.0, Re=100.0, Pa=1e3, warmup=4, samples=2,
                                 eps=(1.0, 0.1, 1e-3, 0.0))
    for name in ("visc", "proj"):
        s = r["solves"][name]
        c = s["cycles_by_eps"]
        _say("  %s: step %.1f, by eps %s, %.3f ms/cycle" % (name, s["step_cycles"], c, s["ms_per_cycle"]))
        assert abs(c[1.0] - s["step_cycles"]) <= 1.0
        assert c[1.0] >= c[0.1] >= c[1e-3] >= c[0.0]
        assert c[0.0] == 0.0
    assert r["inference_ms"] > 0.0


def test_viscous_capture_is_consistent():
    # r0 and e of the captured viscous solve satisfy A e = r0 to the solve's
    # tolerance (A the homogeneous operator: walls at rest)
    import torch
    _say("viscous capture")
    g, fl, _ = _cavity(32)
    ctx = hb.Context(g, fl, hb.make_step_opts())
    ctx.capture(True, hb.OP_VISC)
    u = torch.zeros(hb.cell_shape(g, 2), dtype=torch.float64, device="cuda")
    p = torch.zeros(hb.node_shape(g), dtype=torch.float64, device="cuda")
    for _ in range(3):
        u0 = u.clone()
        rep = ctx.step(u, p)
    r0 = torch.zeros_like(u)
    e = torch.zeros_like(u)
    ctx.capture_read(r0, e, hb.OP_VISC)
    eta = torch.zeros(hb.cell_shape(g)[1:], dtype=torch.float64, device="cuda")
    ctx.viscosity(u0, eta)
    go = orc.make_grid(2, [32, 32], 1.0 / 32)
    flo = orc.make_fluid(Re=fl.Re, HB=fl.HB, n=fl.n, Pa=fl.Pa)
    eh = e.cpu().numpy()
    Ae = eh - rep.dt * orc.visc_div(go, eta.cpu().numpy() / fl.Re, eh, hom=1)
    r0h = r0.cpu().numpy()
    assert np.abs(Ae - r0h).max() <= 1e-9 * max(np.abs(r0h).max(), rep.visc.bnorm)


def test_shipped_warm_start_on_held_out_cavity():
    # the weights trained by paper_1803_00417_amd.warm_start (128^2 cavities,
    # seeds 1..12, Pa = 1e4) on a held-out 128^2 cavity
    _say("shipped warm start")
    from paper_1803_00417_amd import warm_start
    net = warm_start.load_net()
    if net is None:
        pytest.skip("no trained weights shipped")
    g, fl, _ = _cavity(128, seed=99)
    _, _, c0, _ = _run(g, fl, 16)
    _, _, c1, uses = _run(g, fl, 16, net)
    _say("  projection cycles over 16 steps: previous-step guess %d, learned %d (used %d times)"
         % (sum(c0), sum(c1), uses))
    assert sum(c1) <= sum(c0) + 16
