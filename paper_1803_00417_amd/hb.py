"""Python binding of the HIP library ``libhb.so`` (C ABI in include/hb.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  Arrays are torch tensors on the GPU (float64,
contiguous); torch provides device memory and the stream.  The library is
loaded after torch so both use the same HIP runtime.  If the library is
missing this module raises: there is no CPU fallback.
"""
import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhb.so")

OK, ERR_ARG, ERR_DEVICE, ERR_NOCONV, ERR_NONFINITE, ERR_OOM, ERR_IO = 0, -1, -2, -3, -4, -5, -6
BC_WALL, BC_PERIODIC = 0, 1
REG_PAPER, REG_YIELD_ONLY = 0, 1
OP_VISC, OP_NODAL, OP_MAC = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1

ERR_NAMES = {OK: "HB_OK", ERR_ARG: "HB_ERR_ARG", ERR_DEVICE: "HB_ERR_DEVICE",
             ERR_NOCONV: "HB_ERR_NOCONV", ERR_NONFINITE: "HB_ERR_NONFINITE", ERR_OOM: "HB_ERR_OOM",
             ERR_IO: "HB_ERR_IO"}

# symbols declared in include/hb.h
EXPORTS = ["hb_create", "hb_destroy", "hb_last_error", "hb_viscosity", "hb_mg_solve",
           "hb_advect", "hb_project", "hb_cfl_dt", "hb_step", "hb_create_batch", "hb_batch_size",
           "hb_step_batch", "hb_nn_create", "hb_nn_destroy", "hb_nn_param_count", "hb_nn_get_params",
           "hb_nn_set_params", "hb_nn_forward", "hb_nn_grad", "hb_nn_train_step", "hb_set_warm_start",
           "hb_warm_start_uses", "hb_capture", "hb_capture_read", "hb_kernel_timing", "hb_kernel_timing_read",
           "hb_tile_config", "hb_run_steady", "hb_refine_state", "hb_run_sequenced", "hb_checkpoint_write",
           "hb_checkpoint_read", "hb_yield", "hb_run_cessation", "hb_cfl_dt_noalloc"]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double),
                ("bc", (C.c_int32 * 2) * 3), ("wall_u", ((C.c_double * 3) * 2) * 3)]


class Fluid(C.Structure):
    _fields_ = [("Re", C.c_double), ("HB", C.c_double), ("n", C.c_double), ("Pa", C.c_double),
                ("reg", C.c_int32), ("f", C.c_double * 3)]


class MGOpts(C.Structure):
    _fields_ = [("tol_rel", C.c_double), ("max_cycles", C.c_int32), ("fixed_cycles", C.c_int32),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("krylov", C.c_int32), ("precision", C.c_int32)]


class MGReport(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("rel_resid", C.c_double), ("bnorm", C.c_double)]


class StepOpts(C.Structure):
    _fields_ = [("cfl", C.c_double), ("mac_project", C.c_int32),
                ("mac", MGOpts), ("visc", MGOpts), ("proj", MGOpts),
                ("pred_visc", C.c_int32), ("theta", C.c_double)]


class StepReport(C.Structure):
    _fields_ = [("dt", C.c_double), ("max_u", C.c_double), ("div_mac_rel", C.c_double),
                ("div_node", C.c_double), ("mac", MGReport), ("visc", MGReport), ("proj", MGReport)]


class SteadyReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("steady", C.c_int32), ("t", C.c_double), ("change", C.c_double)]


class YieldReport(C.Structure):
    _fields_ = [("yielded", C.c_int64), ("cells", C.c_int64), ("max_stress", C.c_double)]


class CessationReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("stopped", C.c_int32), ("t", C.c_double)]


_lib = None


def load():
    """Load libhb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhb.so is not built (run __graft_entry__.build() or "
                           "python paper_1803_00417_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    L.hb_create.argtypes = [P(Grid), P(Fluid), P(StepOpts), vp, P(vp)]
    L.hb_destroy.argtypes = [vp]
    L.hb_destroy.restype = None
    L.hb_last_error.argtypes = [vp]
    L.hb_last_error.restype = C.c_char_p
    L.hb_viscosity.argtypes = [vp, vp, vp]
    L.hb_mg_solve.argtypes = [vp, C.c_int, vp, C.c_double, vp, vp, P(MGOpts), P(MGReport)]
    L.hb_advect.argtypes = [vp, vp, vp, vp, C.c_double, vp, vp, vp, P(MGReport)]
    L.hb_project.argtypes = [vp, vp, vp, C.c_double, vp, P(MGReport)]
    L.hb_cfl_dt.argtypes = [vp, vp, P(C.c_double)]
    L.hb_step.argtypes = [vp, vp, vp, C.c_double, P(StepReport)]
    L.hb_create_batch.argtypes = [P(Grid), P(Fluid), C.c_int, P(StepOpts), vp, P(vp)]
    L.hb_batch_size.argtypes = [vp]
    L.hb_step_batch.argtypes = [vp, P(vp), P(vp), P(C.c_double), P(StepReport)]
    L.hb_nn_create.argtypes = [C.c_int, C.c_int, C.c_uint64, P(vp)]
    L.hb_nn_destroy.argtypes = [vp]
    L.hb_nn_destroy.restype = None
    L.hb_nn_param_count.argtypes = [vp]
    L.hb_nn_param_count.restype = C.c_int64
    L.hb_nn_get_params.argtypes = [vp, vp]
    L.hb_nn_set_params.argtypes = [vp, vp]
    L.hb_nn_forward.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, vp]
    L.hb_nn_grad.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, P(C.c_double), vp]
    L.hb_nn_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_float, P(C.c_double)]
    L.hb_set_warm_start.argtypes = [vp, C.c_int, vp]
    L.hb_warm_start_uses.argtypes = [vp]
    L.hb_tile_config.argtypes = [vp, C.c_int, C.c_int, P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int)]
    L.hb_capture.argtypes = [vp, C.c_int, C.c_int]
    L.hb_capture_read.argtypes = [vp, C.c_int, vp, vp]
    L.hb_kernel_timing.argtypes = [vp, C.c_int]
    L.hb_kernel_timing_read.argtypes = [vp, P(C.c_int64), P(C.c_double), P(C.c_double)]
    L.hb_run_steady.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.c_double, P(SteadyReport)]
    L.hb_refine_state.argtypes = [vp, vp, vp, vp, vp]
    L.hb_run_sequenced.argtypes = [P(Grid), P(Fluid), P(StepOpts), C.c_int, C.c_double, C.c_int, vp, vp, vp,
                                   P(SteadyReport)]
    L.hb_checkpoint_write.argtypes = [vp, C.c_char_p, vp, vp, C.c_int64, C.c_double]
    L.hb_checkpoint_read.argtypes = [vp, C.c_char_p, vp, vp, P(C.c_int64), P(C.c_double)]
    L.hb_yield.argtypes = [vp, vp, vp, P(YieldReport)]
    L.hb_run_cessation.argtypes = [vp, vp, vp, C.c_int, C.c_double, P(CessationReport)]
    L.hb_cfl_dt_noalloc.argtypes = [P(Grid), C.c_double, vp, vp, vp]
    _lib = L
    return L


class HBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERR_NAMES.get(code, str(code)), msg))
        self.code = code


# ------------------------------------------------------------------ descriptors

def make_grid(dim, n, h=None, bc=None, wall_u=None):
    g = Grid()
    g.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    for a in range(3):
        g.n[a] = nn[a] if a < dim else 1
    g.h = (1.0 / nn[0]) if h is None else h
    for a in range(3):
        for s in range(2):
            g.bc[a][s] = bc[a][s] if (bc is not None and a < dim) else BC_WALL
            for c in range(3):
                g.wall_u[a][s][c] = 0.0
    for (a, s), vel in (wall_u or {}).items():
        for c in range(len(vel)):
            g.wall_u[a][s][c] = vel[c]
    return g


def lid_cavity(dim, n, U=1.0):
    """Unit lid-driven cavity: y-hi lid moving +x (2D), z-hi lid moving +x (3D)."""
    return make_grid(dim, [n] * dim, 1.0 / n, wall_u={(dim - 1, 1): (U, 0.0, 0.0)})


def refined_grid(g):
    """The grid refined by two along every used axis (half the spacing, the
    same boundaries): the next grid of a sequenced run."""
    r = Grid()
    C.memmove(C.byref(r), C.byref(g), C.sizeof(Grid))
    for a in range(g.dim):
        r.n[a] = 2 * g.n[a]
    r.h = g.h / 2.0
    return r


def make_fluid(Re=1.0, HB=0.0, n=1.0, Pa=1e3, reg=REG_PAPER, f=(0.0, 0.0, 0.0)):
    fl = Fluid()
    fl.Re, fl.HB, fl.n, fl.Pa, fl.reg = Re, HB, n, Pa, reg
    for c in range(3):
        fl.f[c] = f[c] if c < len(f) else 0.0
    return fl


def mg_opts(tol=1e-10, max_cycles=100, fixed=0, nu1=2, nu2=2, krylov=0, precision=PREC_FP64):
    o = MGOpts()
    o.tol_rel, o.max_cycles, o.fixed_cycles = tol, max_cycles, fixed
    o.nu1, o.nu2, o.krylov, o.precision = nu1, nu2, krylov, precision
    return o


def make_step_opts(cfl=0.5, tol=1e-10, max_cycles=100, nu=2, mac_project=1, fixed=0,
                   visc_krylov=1, precision=PREC_FP64, pred_visc=0, theta=0.5):
    o = StepOpts()
    o.cfl = cfl
    o.mac_project = mac_project
    o.pred_visc = pred_visc
    o.theta = theta
    for m in (o.mac, o.visc, o.proj):
        m.tol_rel, m.max_cycles, m.fixed_cycles = tol, max_cycles, fixed
        m.nu1, m.nu2, m.krylov, m.precision = nu, nu, 0, precision
    o.visc.krylov = visc_krylov
    return o


def cell_shape(g, comps=1):
    return (comps, g.n[2], g.n[1], g.n[0])


def node_shape(g):
    nn = []
    for a in range(3):
        if a >= g.dim:
            nn.append(1)
        else:
            nn.append(g.n[a] if g.bc[a][0] == BC_PERIODIC else g.n[a] + 1)
    return (nn[2], nn[1], nn[0])


def face_total(g):
    tot = 0
    for a in range(g.dim):
        c = 1
        for b in range(3):
            if b == a:
                c *= g.n[b] if g.bc[b][0] == BC_PERIODIC else g.n[b] + 1
            else:
                c *= g.n[b]
        tot += c
    return tot


# ------------------------------------------------------------------ context

def _ptr(t, numel, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU torch tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("%s must be contiguous float64" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return C.c_void_p(t.data_ptr())


def cfl_dt_noalloc(grid, cfl, u, dt_out, stream=None):
    """hb_cfl_dt_noalloc: the CFL step of u on grid into the one-element
    float64 GPU tensor dt_out, asynchronously, without a context or any
    allocation (stream: a torch stream, default the current one)."""
    L = load()
    n = grid.dim * grid.n[0] * grid.n[1] * grid.n[2]
    if stream is None:
        stream = torch.cuda.current_stream()
    rc = L.hb_cfl_dt_noalloc(C.byref(grid), float(cfl), _ptr(u, n, "u"), _ptr(dt_out, 1, "dt_out"),
                             C.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise HBError(rc, L.hb_last_error(None).decode())


class Context:
    """One grid / fluid / option set on the current GPU and torch stream."""

    def __init__(self, grid, fluid, opts=None, stream=None):
        L = load()
        self.grid, self.fluid = grid, fluid
        self.opts = opts if opts is not None else make_step_opts()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = L.hb_create(C.byref(grid), C.byref(fluid), C.byref(self.opts),
                         C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise HBError(rc, L.hb_last_error(None).decode())
        self._h = h
        g = grid
        self.ncell = g.n[0] * g.n[1] * g.n[2]
        self.nvel = g.dim * self.ncell
        self.nnode = 1
        for s in node_shape(g):
            self.nnode *= s
        self.nface = face_total(g)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise HBError(rc, load().hb_last_error(self._h).decode())
        return rc

    def error(self):
        return load().hb_last_error(self._h).decode()

    # -- calls ------------------------------------------------------------
    def viscosity(self, u, eta):
        return self._check(load().hb_viscosity(self._h, _ptr(u, self.nvel, "u"), _ptr(eta, self.ncell, "eta")))

    def mg_solve(self, op, eta, dt, rhs, x, opts=None, allow=()):
        n = {OP_VISC: self.nvel, OP_MAC: self.ncell, OP_NODAL: self.nnode}[op]
        rep = MGReport()
        rc = load().hb_mg_solve(self._h, op, _ptr(eta, self.ncell, "eta"), float(dt),
                                _ptr(rhs, n, "rhs"), _ptr(x, n, "x"),
                                C.byref(opts) if opts is not None else None, C.byref(rep))
        self._check(rc, allow)
        return rep, rc

    def advect(self, u, p, eta, dt, b, umac=None, conv=None):
        rep = MGReport()
        rc = load().hb_advect(self._h, _ptr(u, self.nvel, "u"), _ptr(p, self.nnode, "p"),
                              _ptr(eta, self.ncell, "eta"), float(dt), _ptr(b, self.nvel, "b"),
                              _ptr(umac, self.nface, "umac"), _ptr(conv, self.nvel, "conv"), C.byref(rep))
        self._check(rc)
        return rep

    def project(self, ustar, p, dt, u):
        rep = MGReport()
        rc = load().hb_project(self._h, _ptr(ustar, self.nvel, "ustar"), _ptr(p, self.nnode, "p"),
                               float(dt), _ptr(u, self.nvel, "u"), C.byref(rep))
        self._check(rc)
        return rep

    def cfl_dt(self, u):
        d = C.c_double()
        self._check(load().hb_cfl_dt(self._h, _ptr(u, self.nvel, "u"), C.byref(d)))
        return d.value

    def kernel_timing(self, enable):
        """enable: 0 (or False) off; k > 0 (True = 1) times every k-th
        finest-level smoother launch"""
        self._check(load().hb_kernel_timing(self._h, int(enable)))

    def kernel_timing_read(self):
        """(launches, total_ms, algorithmic_bytes) of the timed smoother launches"""
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        self._check(load().hb_kernel_timing_read(self._h, C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def set_warm_start(self, net):
        """learned warm start of the nodal solve (net: Net with 1 -> 1
        channels, or None to switch it off)"""
        self._check(load().hb_set_warm_start(self._h, OP_NODAL, net._h if net is not None else None))

    def warm_start_uses(self):
        return load().hb_warm_start_uses(self._h)

    def tile_config(self, op, level):
        """(tx, ty, threads, sweeps_per_launch) of the candidate the
        autotuner chose for the fused sweep of problem op on `level`, or None
        where no fused sweep runs"""
        tx, ty, th, sw = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        rc = load().hb_tile_config(self._h, op, level, C.byref(tx), C.byref(ty), C.byref(th), C.byref(sw))
        return (tx.value, ty.value, th.value, sw.value) if rc == OK else None

    def capture(self, enable, op=OP_NODAL):
        self._check(load().hb_capture(self._h, op, int(enable)))

    def capture_read(self, r0, e, op=OP_NODAL):
        n = self.nvel if op == OP_VISC else self.nnode
        self._check(load().hb_capture_read(self._h, op, _ptr(r0, n, "r0"), _ptr(e, n, "e")))

    def step(self, u, p, dt=0.0, report=True, allow=()):
        rep = StepReport() if report else None
        rc = load().hb_step(self._h, _ptr(u, self.nvel, "u"), _ptr(p, self.nnode, "p"), float(dt),
                            C.byref(rep) if report else None)
        self._check(rc, allow)
        return rep

    def run_steady(self, u, p, tol=1e-5, max_steps=10000, dt=0.0, allow=(ERR_NOCONV,)):
        """hb_run_steady: step until steady; returns (SteadyReport, rc)"""
        rep = SteadyReport()
        rc = load().hb_run_steady(self._h, _ptr(u, self.nvel, "u"), _ptr(p, self.nnode, "p"), float(tol),
                                  int(max_steps), float(dt), C.byref(rep))
        self._check(rc, allow)
        return rep, rc

    def refine_state(self, u_coarse, p_coarse, u, p):
        """hb_refine_state: the coarser grid's state onto this context's grid"""
        cg = Grid()
        C.memmove(C.byref(cg), C.byref(self.grid), C.sizeof(Grid))
        for a in range(cg.dim):
            cg.n[a] //= 2
        ncn = 1
        for s in node_shape(cg):
            ncn *= s
        nc = cg.dim * cg.n[0] * cg.n[1] * cg.n[2]
        self._check(load().hb_refine_state(self._h, _ptr(u_coarse, nc, "u_coarse"), _ptr(p_coarse, ncn, "p_coarse"),
                                           _ptr(u, self.nvel, "u"), _ptr(p, self.nnode, "p")))

    def yield_test(self, u, mask=None):
        """hb_yield: YieldReport of the state u; mask (optional uint8 GPU
        tensor of ncell elements) receives 1 for yielded cells"""
        if mask is not None:
            if not isinstance(mask, torch.Tensor) or not mask.is_cuda or mask.dtype != torch.uint8 \
                    or not mask.is_contiguous() or mask.numel() != self.ncell:
                raise TypeError("mask must be a contiguous uint8 GPU tensor of %d elements" % self.ncell)
        rep = YieldReport()
        self._check(load().hb_yield(self._h, _ptr(u, self.nvel, "u"),
                                    C.c_void_p(mask.data_ptr()) if mask is not None else None, C.byref(rep)))
        return rep

    def run_cessation(self, u, p, max_steps=10000, dt=0.0, allow=(ERR_NOCONV,)):
        """hb_run_cessation: step until no cell is yielded; (CessationReport, rc)"""
        rep = CessationReport()
        rc = load().hb_run_cessation(self._h, _ptr(u, self.nvel, "u"), _ptr(p, self.nnode, "p"), int(max_steps),
                                     float(dt), C.byref(rep))
        self._check(rc, allow)
        return rep, rc

    def checkpoint_write(self, path, u, p, step=0, t=0.0):
        self._check(load().hb_checkpoint_write(self._h, os.fsencode(path), _ptr(u, self.nvel, "u"),
                                               _ptr(p, self.nnode, "p"), int(step), float(t)))

    def checkpoint_read(self, path, u, p):
        """reads (u, p) in place; returns (step, t)"""
        st, t = C.c_int64(), C.c_double()
        self._check(load().hb_checkpoint_read(self._h, os.fsencode(path), _ptr(u, self.nvel, "u"),
                                              _ptr(p, self.nnode, "p"), C.byref(st), C.byref(t)))
        return st.value, t.value


def run_sequenced(coarse, fluid, opts, levels, u, p, tol=1e-5, max_steps=10000, stream=None, allow=(ERR_NOCONV,)):
    """hb_run_sequenced: from rest on `coarse` to steady state, refined
    `levels` times; u, p on the finest grid.  Returns (reports, rc)."""
    L = load()
    g = coarse
    for _ in range(levels):
        g = refined_grid(g)
    nn = 1
    for s in node_shape(g):
        nn *= s
    if stream is None:
        stream = torch.cuda.current_stream()
    reps = (SteadyReport * (levels + 1))()
    rc = L.hb_run_sequenced(C.byref(coarse), C.byref(fluid), C.byref(opts), int(levels), float(tol), int(max_steps),
                            C.c_void_p(stream.cuda_stream), _ptr(u, g.dim * g.n[0] * g.n[1] * g.n[2], "u"),
                            _ptr(p, nn, "p"), reps)
    if rc != OK and rc not in allow:
        raise HBError(rc, L.hb_last_error(None).decode())
    return list(reps), rc


class BatchContext:
    """A batch of independent cavities (same dimension) stepped together:
    every multigrid launch covers all cavities, each stops at its own
    tolerance."""

    def __init__(self, grids, fluids, opts=None, stream=None):
        L = load()
        n = len(grids)
        if n != len(fluids) or n < 1:
            raise ValueError("need one fluid per grid and at least one cavity")
        self.grids, self.fluids = list(grids), list(fluids)
        self.opts = opts if opts is not None else make_step_opts()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        garr = (Grid * n)(*grids)
        farr = (Fluid * n)(*fluids)
        h = C.c_void_p()
        rc = L.hb_create_batch(garr, farr, n, C.byref(self.opts), C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise HBError(rc, L.hb_last_error(None).decode())
        self._h = h
        self.n = n
        self.nvel = [g.dim * g.n[0] * g.n[1] * g.n[2] for g in grids]
        self.nnode = []
        for g in grids:
            k = 1
            for sdim in node_shape(g):
                k *= sdim
            self.nnode.append(k)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def size(self):
        return load().hb_batch_size(self._h)

    def tile_config(self, op, level):
        """(tx, ty, threads, sweeps_per_launch) of the candidate the
        autotuner chose for the fused sweep of problem op on `level`, or None
        where no fused sweep runs"""
        tx, ty, th, sw = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        rc = load().hb_tile_config(self._h, op, level, C.byref(tx), C.byref(ty), C.byref(th), C.byref(sw))
        return (tx.value, ty.value, th.value, sw.value) if rc == OK else None

    def step(self, us, ps, dts=None, report=True, allow=()):
        """One step of every cavity; us[b], ps[b] GPU float64 tensors (in
        place).  Returns the list of per-cavity reports (or None)."""
        if len(us) != self.n or len(ps) != self.n:
            raise ValueError("need one u and one p per cavity")
        up = (C.c_void_p * self.n)(*[_ptr(u, self.nvel[b], "u[%d]" % b) for b, u in enumerate(us)])
        pp = (C.c_void_p * self.n)(*[_ptr(p, self.nnode[b], "p[%d]" % b) for b, p in enumerate(ps)])
        dt = (C.c_double * self.n)(*dts) if dts is not None else None
        reps = (StepReport * self.n)() if report else None
        rc = load().hb_step_batch(self._h, up, pp, dt, reps)
        if rc != OK and rc not in allow:
            raise HBError(rc, load().hb_last_error(self._h).decode())
        return list(reps) if report else None

    def kernel_timing(self, enable):
        rc = load().hb_kernel_timing(self._h, int(enable))
        if rc != OK:
            raise HBError(rc, load().hb_last_error(self._h).decode())

    def kernel_timing_read(self):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        load().hb_kernel_timing_read(self._h, C.byref(n), C.byref(ms), C.byref(by))
        return n.value, ms.value, by.value


def _fptr(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float32 GPU tensor" % name)
    return C.c_void_p(t.data_ptr())


class Net:
    """The BF16 U-Net of the learned warm start (library kernels for the
    forward pass, the backward pass and Adam).  Tensors: float32 GPU,
    [n][H][W][C]."""

    def __init__(self, in_ch=1, out_ch=1, seed=0):
        L = load()
        h = C.c_void_p()
        rc = L.hb_nn_create(in_ch, out_ch, seed, C.byref(h))
        if rc != OK:
            raise HBError(rc, "hb_nn_create failed")
        self._h = h
        self.in_ch, self.out_ch = in_ch, out_ch
        self.nparams = L.hb_nn_param_count(h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hb_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        rc = load().hb_nn_get_params(self._h, out.ctypes.data_as(C.c_void_p))
        if rc != OK:
            raise HBError(rc, "hb_nn_get_params failed")
        return out

    def set_params(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != self.nparams:
            raise ValueError("expected %d parameters" % self.nparams)
        rc = load().hb_nn_set_params(self._h, w.ctypes.data_as(C.c_void_p))
        if rc != OK:
            raise HBError(rc, "hb_nn_set_params failed")

    def forward(self, x):
        n, H, W, _ = x.shape
        y = torch.empty((n, H, W, self.out_ch), dtype=torch.float32, device=x.device)
        rc = load().hb_nn_forward(self._h, _fptr(x, "x"), n, H, W, _fptr(y, "y"))
        if rc != OK:
            raise HBError(rc, "hb_nn_forward failed")
        return y

    def grad(self, x, t):
        import numpy as np
        n, H, W, _ = x.shape
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = C.c_double()
        rc = load().hb_nn_grad(self._h, _fptr(x, "x"), _fptr(t, "target"), n, H, W, C.byref(loss),
                               g.ctypes.data_as(C.c_void_p))
        if rc != OK:
            raise HBError(rc, "hb_nn_grad failed")
        return loss.value, g

    def train_step(self, x, t, lr):
        n, H, W, _ = x.shape
        loss = C.c_double()
        rc = load().hb_nn_train_step(self._h, _fptr(x, "x"), _fptr(t, "target"), n, H, W, float(lr), C.byref(loss))
        if rc != OK:
            raise HBError(rc, "hb_nn_train_step failed")
        return loss.value
