"""FP64 CPU reference of the warm-start U-Net (numpy).

TEST INFRASTRUCTURE ONLY: the GPU network's forward pass and parameter
gradients are checked against this module; the product path never imports
it.  It shares no code with the HIP library.

The network follows the layout of the library: tensors [n][H][W][C]
(channels last); the input is zero-padded to 16 channels; 15 3x3
convolutions (zero padding) with ReLU except the head; 2x2 average pooling
on the way down, nearest-neighbour upsampling and concatenation [upsampled,
skip] on the way up; parameters flat, layer by layer, weights [Cout][3][3][Cin]
then biases [Cout].  The loss is the mean of (y - t)^2 over pixels and the
first out_ch output channels.
"""
import numpy as np

LAYERS = [(16, 16, 1), (16, 16, 1), (16, 32, 1), (32, 32, 1), (32, 64, 1), (64, 64, 1), (64, 64, 1), (64, 64, 1),
          (128, 64, 1), (64, 64, 1), (96, 32, 1), (32, 32, 1), (48, 16, 1), (16, 16, 1), (16, 16, 0)]


def rbf(x):
    """round to the nearest BF16 value (ties to even), returned as float64;
    with bf16=True the functions below round where the GPU network stores
    BF16: weights, the input, every stored activation, and the ReLU-masked
    output gradient that enters the products"""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def param_count():
    return sum(co * 9 * ci + co for ci, co, _ in LAYERS)


def unpack(p):
    """flat parameters -> list of (W [co,3,3,ci], b [co])"""
    out, o = [], 0
    for ci, co, _ in LAYERS:
        w = np.asarray(p[o:o + co * 9 * ci], dtype=np.float64).reshape(co, 3, 3, ci)
        o += co * 9 * ci
        b = np.asarray(p[o:o + co], dtype=np.float64)
        o += co
        out.append((w, b))
    return out


def pack(grads):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in grads])


def conv3(x, w, b):
    """y[n,h,x,o] = b[o] + sum_{dy,dx,c} w[o,dy,dx,c] x[n,h+dy-1,x+dx-1,c] (zero outside)"""
    n, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (n, H, W, w.shape[0])).copy()
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("nhwc,oc->nhwo", xp[:, dy:dy + H, dx:dx + W, :], w[:, dy, dx, :])
    return y


def conv3_bwd(x, w, dz):
    """gradients of conv3 with respect to w, b and x, given dL/dy = dz"""
    n, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            dw[:, dy, dx, :] = np.einsum("nhwo,nhwc->oc", dz, xp[:, dy:dy + H, dx:dx + W, :])
            dxp[:, dy:dy + H, dx:dx + W, :] += np.einsum("nhwo,oc->nhwc", dz, w[:, dy, dx, :])
    return dw, dz.sum(axis=(0, 1, 2)), dxp[:, 1:-1, 1:-1, :]


def pool2(x):
    return 0.25 * (x[:, 0::2, 0::2] + x[:, 1::2, 0::2] + x[:, 0::2, 1::2] + x[:, 1::2, 1::2])


def pool2_bwd(dy):
    return 0.25 * np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2)


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_bwd(dy):
    n, H, W, C = dy.shape
    return dy.reshape(n, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def pad_input(x):
    n, H, W, c = x.shape
    out = np.zeros((n, H, W, 16))
    out[..., :c] = x
    return out


def forward(p, x, bf16=False):
    """network output [n,H,W,16] and the cache for backward"""
    P = unpack(p)
    if bf16:
        P = [(rbf(w), b) for w, b in P]
    r = rbf if bf16 else (lambda v: v)
    a = {"P": P, "bf16": bf16}

    def conv(i, inp):
        z = conv3(inp, *P[i])
        return r(np.maximum(z, 0.0)) if LAYERS[i][2] else z

    def pool(v):
        return r(pool2(v))

    a["in"] = r(pad_input(x))
    a["e0a"] = conv(0, a["in"])
    a["e0"] = conv(1, a["e0a"])
    a["p0"] = pool(a["e0"])
    a["e1a"] = conv(2, a["p0"])
    a["e1"] = conv(3, a["e1a"])
    a["p1"] = pool(a["e1"])
    a["e2a"] = conv(4, a["p1"])
    a["e2"] = conv(5, a["e2a"])
    a["p2"] = pool(a["e2"])
    a["e3a"] = conv(6, a["p2"])
    a["e3"] = conv(7, a["e3a"])
    a["c2"] = np.concatenate([up2(a["e3"]), a["e2"]], axis=3)
    a["d2a"] = conv(8, a["c2"])
    a["d2"] = conv(9, a["d2a"])
    a["c1"] = np.concatenate([up2(a["d2"]), a["e1"]], axis=3)
    a["d1a"] = conv(10, a["c1"])
    a["d1"] = conv(11, a["d1a"])
    a["c0"] = np.concatenate([up2(a["d1"]), a["e0"]], axis=3)
    a["d0a"] = conv(12, a["c0"])
    a["d0"] = conv(13, a["d0a"])
    a["y"] = conv(14, a["d0"])
    return a["y"], a


def loss(y, t):
    oc = t.shape[3]
    d = y[..., :oc] - t
    return float(np.mean(d * d))


def backward(p, cache, t):
    """flat gradient of the loss with respect to the parameters"""
    a = cache
    P = a["P"]
    r = rbf if a["bf16"] else (lambda v: v)
    y = a["y"]
    oc = t.shape[3]
    dy = np.zeros_like(y)
    dy[..., :oc] = 2.0 * (y[..., :oc] - t) / (y[..., :oc].size)
    grads = [None] * len(LAYERS)

    def conv_b(i, inp, out, g):
        dz = g * (out > 0.0) if LAYERS[i][2] else g
        dw, _, dx = conv3_bwd(inp, P[i][0], r(dz))
        grads[i] = (dw, dz.sum(axis=(0, 1, 2)))
        return dx

    g = conv_b(14, a["d0"], a["y"], dy)
    g = conv_b(13, a["d0a"], a["d0"], g)
    g = conv_b(12, a["c0"], a["d0a"], g)
    c1 = a["d1"].shape[3]
    g_d1, g_e0 = up2_bwd(g[..., :c1]), g[..., c1:]
    g = conv_b(11, a["d1a"], a["d1"], g_d1)
    g = conv_b(10, a["c1"], a["d1a"], g)
    c2 = a["d2"].shape[3]
    g_d2, g_e1 = up2_bwd(g[..., :c2]), g[..., c2:]
    g = conv_b(9, a["d2a"], a["d2"], g_d2)
    g = conv_b(8, a["c2"], a["d2a"], g)
    c3 = a["e3"].shape[3]
    g_e3, g_e2 = up2_bwd(g[..., :c3]), g[..., c3:]
    g = conv_b(7, a["e3a"], a["e3"], g_e3)
    g = conv_b(6, a["p2"], a["e3a"], g)
    g = conv_b(5, a["e2a"], a["e2"], g_e2 + pool2_bwd(g))
    g = conv_b(4, a["p1"], a["e2a"], g)
    g = conv_b(3, a["e1a"], a["e1"], g_e1 + pool2_bwd(g))
    g = conv_b(2, a["p0"], a["e1a"], g)
    g = conv_b(1, a["e0a"], a["e0"], g_e0 + pool2_bwd(g))
    conv_b(0, a["in"], a["e0a"], g)
    return pack(grads)


def loss_and_grad(p, x, t, bf16=False):
    y, cache = forward(p, x, bf16)
    return loss(y, t), backward(p, cache, t)
