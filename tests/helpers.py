"""Shared test helpers: build matching descriptors for the HIP library and
the CPU oracle from one plain specification, and move arrays between them."""
import numpy as np

from oracle import orc


def spec(dim, n, bc=None, wall_u=None, h=None, Re=1.0, HB=0.0, nidx=1.0, Pa=1e3, reg=0, f=(0.0, 0.0, 0.0)):
    nn = list(n) if isinstance(n, (list, tuple)) else [n] * dim
    return dict(dim=dim, n=nn, bc=bc, wall_u=wall_u or {}, h=h if h is not None else 1.0 / nn[0],
                Re=Re, HB=HB, nidx=nidx, Pa=Pa, reg=reg, f=f)


def lid_spec(dim, n, **kw):
    return spec(dim, n, wall_u={(dim - 1, 1): (1.0, 0.0, 0.0)}, **kw)


def oracle_objs(s):
    g = orc.make_grid(s["dim"], s["n"], s["h"], bc=s["bc"], wall_u=s["wall_u"])
    fl = orc.make_fluid(Re=s["Re"], HB=s["HB"], n=s["nidx"], Pa=s["Pa"], reg=s["reg"], f=s["f"])
    return g, fl


def hip_objs(s):
    from paper_1803_00417_amd import hb
    g = hb.make_grid(s["dim"], s["n"], s["h"], bc=s["bc"], wall_u=s["wall_u"])
    fl = hb.make_fluid(Re=s["Re"], HB=s["HB"], n=s["nidx"], Pa=s["Pa"], reg=s["reg"], f=s["f"])
    return g, fl


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_err(a, b):
    """max |a - b| / max |b| (max-norm relative error)"""
    d = np.abs(np.asarray(a) - np.asarray(b)).max()
    s = np.abs(np.asarray(b)).max()
    return d / s if s > 0 else d
