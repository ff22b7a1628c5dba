"""Seeded synthetic inputs and workload descriptions.

This module holds no arithmetic of the method: it only describes workloads
(grid sizes, dimensionless groups, step counts) and draws seeded random
fields, so the same inputs can be handed to the HIP path and to the checker.
Lid-driven-cavity workloads start from rest, as in the paper's validation
runs (Sec. IV); the random fields below only serve operator-level checks.
"""
import numpy as np

# Workloads.  "Bi" of the Bingham cases is the Herschel-Bulkley number HB
# (identical for n = 1); "m" is the Papanastasiou number Pa (U = L = 1).
WORKLOADS = {
    "cavity2d_64": dict(dim=2, n=64, Re=100.0, HB=1.0, nidx=1.0, Pa=1e3, steps=50, cfl=0.5,
                        desc="2D lid-driven cavity 64^2, Bingham Bi=1, Re=100, m=1e3, 50 steps"),
    "cavity2d_512_n0.5": dict(dim=2, n=512, Re=1000.0, HB=10.0, nidx=0.5, Pa=1e4, steps=200, cfl=0.5,
                              desc="2D lid-driven cavity 512^2, HB n=0.5, Bi=10, Re=1000, m=1e4"),
    "cavity2d_512_n1.5": dict(dim=2, n=512, Re=1000.0, HB=10.0, nidx=1.5, Pa=1e4, steps=200, cfl=0.5,
                              desc="2D lid-driven cavity 512^2, HB n=1.5, Bi=10, Re=1000, m=1e4"),
    "cavity3d_128": dict(dim=3, n=128, Re=1000.0, HB=2.0, nidx=1.0, Pa=1e3, steps=100, cfl=0.5,
                         desc="3D lid-driven cube 128^3, Bingham Bi=2, Re=1000, m=1e3"),
}


def splitmix64(seed):
    """SplitMix64 (Steele, Lea & Flood 2014) as an infinite generator of
    64-bit integers."""
    mask = (1 << 64) - 1
    s = seed & mask
    while True:
        s = (s + 0x9E3779B97F4A7C15) & mask
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        yield z ^ (z >> 31)


def batch_cavities(count=64, seed=0, sizes=(64, 96, 128, 192, 256)):
    """Parameters of a batched sweep: per cavity N (uniform over sizes),
    Bi log-uniform in [0.1, 100], n uniform in [0.3, 1.5], Re log-uniform
    in [1, 1000]; uniforms U = (next >> 11) * 2^-53."""
    g = splitmix64(seed)
    u = lambda: (next(g) >> 11) * (1.0 / 9007199254740992.0)
    out = []
    for _ in range(count):
        N = sizes[min(int(u() * len(sizes)), len(sizes) - 1)]
        HB = 10.0 ** (-1.0 + 3.0 * u())
        n = 0.3 + 1.2 * u()
        Re = 10.0 ** (3.0 * u())
        out.append(dict(dim=2, n=N, HB=HB, nidx=n, Re=Re, Pa=1e3, steps=100, cfl=0.5))
    return out


def random_cells(shape, seed, scale=1.0):
    """Random normal cell field (float64), e.g. shape (C, nz, ny, nx)."""
    return np.random.default_rng(seed).standard_normal(shape) * scale


def smooth_cells(shape, seed, modes=4, scale=1.0):
    """Smooth random cell field: a few random Fourier modes per component,
    sampled at cell centres of the unit box."""
    rng = np.random.default_rng(seed)
    C, nz, ny, nx = shape
    z = (np.arange(nz) + 0.5) / nz
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    out = np.zeros(shape)
    for c in range(C):
        for _ in range(modes):
            kx, ky, kz = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * np.pi, size=3)
            amp = rng.standard_normal()
            out[c] += amp * np.sin(np.pi * kx * X + ph[0]) * np.sin(np.pi * ky * Y + ph[1]) * \
                (np.sin(np.pi * kz * Z + ph[2]) if nz > 1 else 1.0)
    return out * scale


def positive_cells(shape, seed, lo=-1.0, hi=3.0):
    """Log-uniform positive cell field exp(U(lo, hi)) (e.g. a viscosity)."""
    return np.exp(np.random.default_rng(seed).uniform(lo, hi, shape))
