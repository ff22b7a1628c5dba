"""ctypes view of the plain FP64 CPU oracle (``liborc.so``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module to check the HIP library.  The product
path never imports it, and it imports nothing from the product package.

Array conventions: cell fields are ``(C, nz, ny, nx)`` float64 (``nz = 1`` in
2D); nodal fields ``(nnz, nny, nnx)``; face fields are the per-axis face arrays
concatenated into one flat vector.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the parity build (single-threaded, every loop in order) and, for timing
# only, the same sources built with OpenMP (ORC_OMP=1 in the environment)
LIB_SERIAL = os.path.join(HERE, "liborc.so")
LIB_OMP = os.path.join(HERE, "liborc_omp.so")
LIB = LIB_OMP if os.environ.get("ORC_OMP") == "1" else LIB_SERIAL
SOURCES = ["orc_core.c", "orc_mg.c", "orc_step.c"]

WALL, PERIODIC = 0, 1
REG_PAPER, REG_YIELD_ONLY = 0, 1
OP_VISC, OP_NODAL, OP_MAC = 0, 1, 2
OK, ERR_ARG, ERR_NOCONV, ERR_NONFINITE = 0, -1, -3, -4


def build(force=False):
    """Compile liborc.so with gcc (no FMA contraction, so rounding is the
    plain IEEE sequence written in the source), and liborc_omp.so, the same
    sources with OpenMP over the planes and rows of the heavy loops (CPU
    timing only)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    hdrs = [os.path.join(HERE, s) for s in ("orc.h", "orc_internal.h")]
    for lib_path, extra in ((LIB_SERIAL, []), (LIB_OMP, ["-fopenmp"])):
        if not force and os.path.exists(lib_path):
            t = os.path.getmtime(lib_path)
            if all(os.path.getmtime(s) <= t for s in srcs + hdrs):
                continue
        tmp = lib_path + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off"] + extra + \
              ["-o", tmp] + srcs + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, lib_path)
    return LIB


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double),
                ("bc", (C.c_int * 2) * 3), ("wall_u", ((C.c_double * 3) * 2) * 3)]


class Fluid(C.Structure):
    _fields_ = [("Re", C.c_double), ("HB", C.c_double), ("n", C.c_double),
                ("Pa", C.c_double), ("reg", C.c_int), ("f", C.c_double * 3)]


class MGOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_cycles", C.c_int), ("fixed", C.c_int),
                ("nu1", C.c_int), ("nu2", C.c_int), ("krylov", C.c_int)]


class MGReport(C.Structure):
    _fields_ = [("cycles", C.c_int), ("rel_resid", C.c_double), ("bnorm", C.c_double)]


class StepOpts(C.Structure):
    _fields_ = [("cfl", C.c_double), ("mac_project", C.c_int),
                ("mac", MGOpts), ("visc", MGOpts), ("proj", MGOpts),
                ("pred_visc", C.c_int), ("theta", C.c_double)]


class StepReport(C.Structure):
    _fields_ = [("dt", C.c_double), ("max_u", C.c_double), ("div_mac_rel", C.c_double),
                ("div_node", C.c_double), ("mac", MGReport), ("visc", MGReport),
                ("proj", MGReport)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.POINTER
        dp = P(C.c_double)
        L.orc_eta_of_g.restype = C.c_double
        L.orc_eta_of_g.argtypes = [P(Fluid), C.c_double]
        L.orc_viscosity.argtypes = [P(Grid), P(Fluid), dp, dp]
        L.orc_visc_div.argtypes = [P(Grid), dp, dp, C.c_int, dp]
        L.orc_grad_node.argtypes = [P(Grid), dp, dp]
        L.orc_weak_div.argtypes = [P(Grid), dp, dp]
        L.orc_apply_K.argtypes = [P(Grid), dp, dp]
        L.orc_mac_div.argtypes = [P(Grid), dp, dp]
        L.orc_face_count.restype = C.c_long
        L.orc_face_count.argtypes = [P(Grid), C.c_int]
        L.orc_node_count.restype = C.c_long
        L.orc_node_count.argtypes = [P(Grid)]
        L.orc_mg_solve.argtypes = [P(Grid), P(Fluid), C.c_int, dp, C.c_double, dp, dp,
                                   P(MGOpts), P(MGReport)]
        L.orc_dense_matrix.argtypes = [P(Grid), P(Fluid), C.c_int, dp, C.c_double, dp]
        L.orc_dense_solve.argtypes = [C.c_int, dp, dp]
        L.orc_tensor_diagonal.argtypes = [P(Grid), P(Fluid), dp, C.c_double, dp]
        L.orc_prolong_cells.argtypes = [P(Grid), P(Grid), C.c_int, C.c_double, dp, dp]
        L.orc_prolong_cells.restype = None
        L.orc_restrict_faces.argtypes = [P(Grid), P(Grid), dp, dp]
        L.orc_restrict_faces.restype = None
        L.orc_cfl_dt.restype = C.c_double
        L.orc_cfl_dt.argtypes = [P(Grid), C.c_double, dp]
        L.orc_advect.argtypes = [P(Grid), P(Fluid), P(StepOpts), dp, dp, dp, C.c_double,
                                 dp, dp, dp, dp, P(MGReport), dp]
        L.orc_project.argtypes = [P(Grid), P(StepOpts), dp, dp, C.c_double, dp, P(MGReport)]
        L.orc_step.argtypes = [P(Grid), P(Fluid), P(StepOpts), dp, dp, C.c_double,
                               P(StepReport)]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------- descriptors

def make_grid(dim, n, h=None, bc=None, wall_u=None):
    """Grid descriptor; ``bc`` is ((lo, hi), ...) per axis, default all walls."""
    g = Grid()
    g.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    for a in range(3):
        g.n[a] = nn[a] if a < dim else 1
    g.h = (1.0 / nn[0]) if h is None else h
    for a in range(3):
        for s in range(2):
            g.bc[a][s] = (bc[a][s] if (bc is not None and a < dim) else WALL)
            for c in range(3):
                g.wall_u[a][s][c] = 0.0
    if wall_u:
        for (a, s), vel in wall_u.items():
            for c in range(len(vel)):
                g.wall_u[a][s][c] = vel[c]
    return g


def lid_cavity(dim, n, U=1.0):
    """Unit lid-driven cavity: y-hi lid moving +x in 2D, z-hi lid moving +x in 3D."""
    return make_grid(dim, [n] * dim, 1.0 / n, wall_u={(dim - 1, 1): (U, 0.0, 0.0)})


def make_fluid(Re=1.0, HB=0.0, n=1.0, Pa=1e3, reg=REG_PAPER, f=(0.0, 0.0, 0.0)):
    fl = Fluid()
    fl.Re, fl.HB, fl.n, fl.Pa, fl.reg = Re, HB, n, Pa, reg
    for c in range(3):
        fl.f[c] = f[c] if c < len(f) else 0.0
    return fl


def make_step_opts(cfl=0.5, tol=1e-10, max_cycles=100, nu=2, mac_project=1, fixed=0,
                   visc_krylov=1, pred_visc=0, theta=0.5):
    o = StepOpts()
    o.cfl = cfl
    o.mac_project = mac_project
    o.pred_visc = pred_visc
    o.theta = theta
    for m in (o.mac, o.visc, o.proj):
        m.tol, m.max_cycles, m.fixed, m.nu1, m.nu2, m.krylov = tol, max_cycles, fixed, nu, nu, 0
    o.visc.krylov = visc_krylov
    return o


def mg_opts(tol=1e-10, max_cycles=100, fixed=0, nu1=2, nu2=2, krylov=0):
    o = MGOpts()
    o.tol, o.max_cycles, o.fixed, o.nu1, o.nu2, o.krylov = tol, max_cycles, fixed, nu1, nu2, krylov
    return o


# ----------------------------------------------------------------- shapes

def cell_shape(g, comps=1):
    return (comps, g.n[2], g.n[1], g.n[0])


def node_shape(g):
    nn = []
    for a in range(3):
        if a >= g.dim:
            nn.append(1)
        else:
            nn.append(g.n[a] if g.bc[a][0] == PERIODIC else g.n[a] + 1)
    return (nn[2], nn[1], nn[0])


def face_total(g):
    return sum(lib().orc_face_count(C.byref(g), a) for a in range(g.dim))


# ----------------------------------------------------------------- calls

def eta_of_g(fl, gval):
    return lib().orc_eta_of_g(C.byref(fl), float(gval))


def viscosity(g, fl, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    eta = np.zeros(cell_shape(g)[1:], dtype=np.float64)
    rc = lib().orc_viscosity(C.byref(g), C.byref(fl), _p(u), _p(eta))
    return eta, rc


def visc_div(g, eta_e, u, hom=0):
    u = np.ascontiguousarray(u, dtype=np.float64)
    eta_e = np.ascontiguousarray(eta_e, dtype=np.float64)
    out = np.zeros_like(u)
    lib().orc_visc_div(C.byref(g), _p(eta_e), _p(u), hom, _p(out))
    return out


def grad_node(g, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(cell_shape(g, g.dim), dtype=np.float64)
    lib().orc_grad_node(C.byref(g), _p(phi), _p(out))
    return out


def weak_div(g, V):
    V = np.ascontiguousarray(V, dtype=np.float64)
    r = np.zeros(node_shape(g), dtype=np.float64)
    lib().orc_weak_div(C.byref(g), _p(V), _p(r))
    return r


def apply_K(g, phi):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.zeros(node_shape(g), dtype=np.float64)
    lib().orc_apply_K(C.byref(g), _p(phi), _p(out))
    return out


def mac_div(g, faces):
    faces = np.ascontiguousarray(faces, dtype=np.float64)
    out = np.zeros(cell_shape(g)[1:], dtype=np.float64)
    lib().orc_mac_div(C.byref(g), _p(faces), _p(out))
    return out


def mg_solve(g, fl, op, eta, dt, rhs, x0=None, **kw):
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    o = mg_opts(**kw)
    rep = MGReport()
    e = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
    rc = lib().orc_mg_solve(C.byref(g), C.byref(fl) if fl is not None else None, op, _p(e),
                            float(dt), _p(rhs), _p(x), C.byref(o), C.byref(rep))
    return x, rc, rep


def dense_matrix(g, fl, op, eta, dt):
    if op == OP_VISC:
        N = g.dim * g.n[0] * g.n[1] * g.n[2]
    elif op == OP_MAC:
        N = g.n[0] * g.n[1] * g.n[2]
    else:
        N = int(np.prod(node_shape(g)))
    A = np.zeros((N, N), dtype=np.float64)
    e = None if eta is None else np.ascontiguousarray(eta, dtype=np.float64)
    lib().orc_dense_matrix(C.byref(g), C.byref(fl) if fl is not None else None, op, _p(e),
                           float(dt), _p(A))
    return A


def tensor_diagonal(g, fl, eta, dt):
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    out = np.zeros(cell_shape(g, g.dim), dtype=np.float64)
    lib().orc_tensor_diagonal(C.byref(g), C.byref(fl), _p(eta), float(dt), _p(out))
    return out


def coarse_grid(g):
    """the next multigrid level of g: every used cell count halved, spacing
    doubled, same boundaries, walls at rest"""
    c = Grid()
    C.pointer(c)[0] = g
    for a in range(g.dim):
        c.n[a] = g.n[a] // 2
    c.h = 2.0 * g.h
    for a in range(3):
        for s in range(2):
            for q in range(3):
                c.wall_u[a][s][q] = 0.0
    return c


def prolong_cells(gf, gc, e, wall_sign, x=None):
    """x + P e for a cell field e on gc ([C][cells]); returns the new x"""
    e = np.ascontiguousarray(e, dtype=np.float64)
    ncomp = e.shape[0]
    out = np.zeros(cell_shape(gf, ncomp)) if x is None else np.array(x, dtype=np.float64, copy=True)
    lib().orc_prolong_cells(C.byref(gf), C.byref(gc), ncomp, float(wall_sign), _p(e), _p(out))
    return out


def restrict_faces(gf, gc, bf):
    bf = np.ascontiguousarray(bf, dtype=np.float64)
    out = np.zeros(face_total(gc), dtype=np.float64)
    lib().orc_restrict_faces(C.byref(gf), C.byref(gc), _p(bf), _p(out))
    return out


def cfl_dt(g, cfl, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_cfl_dt(C.byref(g), float(cfl), _p(u))


def advect(g, fl, o, u, p, eta, dt):
    """Returns (b, E, umac, A, mac_report, div_mac_rel, rc)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    b = np.zeros_like(u)
    E = np.zeros_like(u)
    A = np.zeros_like(u)
    umac = np.zeros(face_total(g), dtype=np.float64)
    rep = MGReport()
    dm = C.c_double(0.0)
    rc = lib().orc_advect(C.byref(g), C.byref(fl), C.byref(o), _p(u), _p(p), _p(eta),
                          float(dt), _p(b), _p(E), _p(umac), _p(A), C.byref(rep), C.byref(dm))
    return b, E, umac, A, rep, dm.value, rc


def project(g, o, ustar, p, dt):
    """Returns (u_new, p_new, report, rc); p is not modified."""
    ustar = np.ascontiguousarray(ustar, dtype=np.float64)
    p2 = np.array(p, dtype=np.float64, copy=True)
    u = np.zeros_like(ustar)
    rep = MGReport()
    rc = lib().orc_project(C.byref(g), C.byref(o), _p(ustar), _p(p2), float(dt), _p(u),
                           C.byref(rep))
    return u, p2, rep, rc


def step(g, fl, o, u, p, dt=0.0):
    """One time step in place on (u, p); returns (report, rc)."""
    assert u.dtype == np.float64 and u.flags["C_CONTIGUOUS"]
    assert p.dtype == np.float64 and p.flags["C_CONTIGUOUS"]
    rep = StepReport()
    rc = lib().orc_step(C.byref(g), C.byref(fl), C.byref(o), _p(u), _p(p), float(dt),
                        C.byref(rep))
    return rep, rc
