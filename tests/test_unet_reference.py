"""Pins of the FP64 U-Net reference (the checker of the GPU network):
its convolution against scipy's correlation, and its parameter gradient
against central finite differences of its own loss."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet


def test_conv3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 8, 12, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = unet.conv3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = np.full((8, 12), b[o])
            for c in range(3):
                ref += ndimage.correlate(x[n, :, :, c], w[o, :, :, c], mode="constant", cval=0.0)
            assert np.abs(y[n, :, :, o] - ref).max() < 1e-12


def test_pool_and_upsample_are_adjoint_up_to_scale():
    # <pool(x), y> = <x, pool_bwd(y)> and <up(x), y> = <x, up_bwd(y)>
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 8, 8, 2))
    y = rng.standard_normal((1, 4, 4, 2))
    assert abs(np.sum(unet.pool2(x) * y) - np.sum(x * unet.pool2_bwd(y))) < 1e-12
    assert abs(np.sum(unet.up2(y) * x) - np.sum(y * unet.up2_bwd(x))) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    npar = unet.param_count()
    p = np.zeros(npar)
    o = 0
    for ci, co, _ in unet.LAYERS:
        p[o:o + co * 9 * ci] = rng.standard_normal(co * 9 * ci) * np.sqrt(2.0 / (9 * ci))
        o += co * 9 * ci
        p[o:o + co] = 0.05 * rng.standard_normal(co)
        o += co
    x = rng.standard_normal((1, 8, 8, 1))
    t = rng.standard_normal((1, 8, 8, 1))
    L, g = unet.loss_and_grad(p, x, t)
    idx = rng.choice(npar, 40, replace=False)
    # also the largest entries
    idx = np.concatenate([idx, np.argsort(-np.abs(g))[:10]])
    h = 1e-6
    gmax = np.abs(g).max()
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (unet.loss(unet.forward(pp, x)[0], t) - unet.loss(unet.forward(pm, x)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * gmax + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    # rbf is round-to-nearest-even to BF16; torch's float32 -> bfloat16
    # conversion is the independent reference (CPU)
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
        # exact ties between two BF16 neighbours (both parities of the kept bit)
        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -130 * (1 + 2.0 ** -8)]),
        np.array([0.0, -0.0, 1.0, -3.0, 3.0e38, 1e-40, 65504.0]),
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = unet.rbf(x)
    same = (got == ref) | (np.isnan(got) & np.isnan(ref))
    assert same.all(), x[~same][:5]

