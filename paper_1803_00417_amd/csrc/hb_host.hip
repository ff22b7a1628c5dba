// hb_host.hip -- context set-up, multigrid drivers (V-cycle and BiCGStab
// acceleration), the time step and the C ABI of include/hb.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "hb_internal.h"

namespace hb {

static thread_local std::string g_create_err;

#define HB_TRY(expr)                                                         \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess) {                                              \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);      \
            return HB_ERR_DEVICE;                                            \
        }                                                                    \
    } while (0)

static int fail(Ctx* c, int code, const std::string& msg)
{
    c->err = msg;
    return code;
}

static bool valid_extent(int n)
{
    if (n < 4) return false;
    while (n % 2 == 0) n /= 2;
    return n == 1 || n == 3;
}

static GridD make_gridd(const hb_grid& g)
{
    GridD d;
    memset(&d, 0, sizeof(d));
    d.dim = g.dim;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = a < g.dim ? g.n[a] : 1;
        d.per[a] = a < g.dim ? (g.bc[a][0] == HB_BC_PERIODIC) : 0;
        for (int s = 0; s < 2; ++s)
            for (int q = 0; q < 3; ++q) d.wall_u[a][s][q] = (a < g.dim && !d.per[a]) ? g.wall_u[a][s][q] : 0.0;
    }
    d.h = g.h;
    return d;
}

static long unknowns(const GridD& g, int op)
{
    if (op == HB_OP_VISC) return ncells(g) * g.dim;
    if (op == HB_OP_MAC) return ncells(g);
    return nnodes(g);
}

static long nface_total(const GridD& g)
{
    long n = 0;
    for (int a = 0; a < g.dim; ++a) n += fcount(g, a);
    return n;
}

template <typename T>
static hipError_t dalloc(T** p, long n)
{
    return hipMalloc((void**)p, sizeof(T) * (size_t)(n > 0 ? n : 1));
}

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------

static int build_mg(Ctx* c, MG& m, int op)
{
    m.op = op;
    GridD cur = c->g;
    int l = 0;
    for (;;) {
        if (l >= kMaxLev) return fail(c, HB_ERR_ARG, "too many multigrid levels");
        Level& L = m.L[l];
        L.g = cur;
        L.nu = unknowns(cur, op);
        HB_TRY(dalloc(&L.xb[0], L.nu));
        HB_TRY(dalloc(&L.xb[1], L.nu));
        if (l > 0) HB_TRY(dalloc(&L.b, L.nu));
        HB_TRY(dalloc(&L.r, L.nu));
        if (op == HB_OP_VISC) HB_TRY(dalloc(&L.beta, nface_total(cur)));
        HB_TRY(dalloc(&L.fx[0], L.nu));
        HB_TRY(dalloc(&L.fx[1], L.nu));
        HB_TRY(dalloc(&L.fb, L.nu));
        if (op == HB_OP_NODAL) HB_TRY(dalloc(&L.fr, L.nu));
        if (op == HB_OP_VISC && l > 0) HB_TRY(dalloc(&L.fbeta, nface_total(cur)));
        ++l;
        bool can = true;
        for (int a = 0; a < cur.dim; ++a)
            if ((cur.n[a] & 1) || cur.n[a] / 2 < 2) can = false;
        if (!can) break;
        GridD nx = cur;
        for (int a = 0; a < cur.dim; ++a) nx.n[a] = cur.n[a] / 2;
        nx.h = cur.h * 2.0;
        memset(nx.wall_u, 0, sizeof(nx.wall_u));
        cur = nx;
    }
    m.nlev = l;
    m.ncoarse = (int)m.L[l - 1].nu;
    HB_TRY(dalloc(&m.A, (long)m.ncoarse * m.ncoarse));
    HB_TRY(dalloc(&m.Ainv, (long)m.ncoarse * m.ncoarse));
    HB_TRY(dalloc(&m.piv, m.ncoarse));
    HB_TRY(dalloc(&m.lvl0_b, m.L[0].nu));
    m.L[0].b = m.lvl0_b;
    if (op == HB_OP_VISC) {
        HB_TRY(dalloc(&m.etae, ncells(c->g)));
        HB_TRY(dalloc(&m.etae32, ncells(c->g)));
    }
    return HB_OK;
}

static void free_mg(MG& m)
{
    for (int l = 0; l < m.nlev; ++l) {
        Level& L = m.L[l];
        (void)hipFree(L.xb[0]);
        (void)hipFree(L.xb[1]);
        if (l > 0) (void)hipFree(L.b);
        (void)hipFree(L.r);
        (void)hipFree(L.beta);
        (void)hipFree(L.fx[0]);
        (void)hipFree(L.fx[1]);
        (void)hipFree(L.fb);
        (void)hipFree(L.fr);
        (void)hipFree(L.fbeta);
    }
    (void)hipFree(m.A);
    (void)hipFree(m.Ainv);
    (void)hipFree(m.piv);
    (void)hipFree(m.lvl0_b);
    (void)hipFree(m.etae);
    (void)hipFree(m.etae32);
    for (int p = 0; p < 2; ++p)
        if (m.gexec[p]) (void)hipGraphExecDestroy(m.gexec[p]);
}

__global__ void k_identity(int N, double* E)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)N * N) return;
    E[t] = (t / N == t % N) ? 1.0 : 0.0;
}

// dense coarsest matrix of the current coefficients, then LU
static void factor_coarsest(Ctx* c, MG& m)
{
    const int N = m.ncoarse;
    const Level& C = m.L[m.nlev - 1];
    const long nn = (long)N * N;
    k_identity<<<(unsigned)((nn + 255) / 256), 256, 0, c->s>>>(N, c->dense_E);
    if (m.op == HB_OP_VISC) launch_visc_dense(c, C, m.dt, N, c->dense_E, m.A);
    else if (m.op == HB_OP_MAC) launch_mac_dense(c, C, N, c->dense_E, m.A);
    else launch_nodal_dense(c, C, N, c->dense_E, m.A);
    if (m.op != HB_OP_VISC) launch_add_ones(c, N, m.A);
    launch_lu_factor(c, N, m.A, m.piv);
    launch_lu_inverse(c, N, m.A, m.piv, m.Ainv);
}

// face viscosities of every level from the cell viscosity eta (not /Re)
static void visc_setup(Ctx* c, const double* eta, double dt)
{
    MG& m = c->visc;
    set_slot(c, S_DT, dt);
    launch_eta_over_re(c, m.L[0].g, eta, m.etae);
    launch_eta_faces(c, m.L[0].g, eta, m.L[0].beta);
    for (int l = 1; l < m.nlev; ++l) launch_restrict_faces(c, m.L[l - 1].g, m.L[l].g, m.L[l - 1].beta, m.L[l].beta);
    m.dt = dt;
    m.f32_ready = false;
    factor_coarsest(c, m);
}

// FP32 copies of the tensor coefficients for mixed-precision cycles (the
// coarsest matrix stays the FP64 one)
static void ensure_f32(Ctx* c, MG& m)
{
    if (m.op != HB_OP_VISC || m.f32_ready) return;
    to_f32(c, m.etae, m.etae32, nullptr, ncells(m.L[0].g));
    for (int l = 1; l < m.nlev; ++l) to_f32(c, m.L[l].beta, m.L[l].fbeta, nullptr, nface_total(m.L[l].g));
    m.f32_ready = true;
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------

// tensor coefficients of level l for the tiled kernels: eta/Re cells on the
// finest level, face arrays below
template <typename R> static const R* tcoef(const MG& m, int l);
template <> const double* tcoef<double>(const MG& m, int l) { return l == 0 ? m.etae : m.L[l].beta; }
template <> const float* tcoef<float>(const MG& m, int l) { return l == 0 ? m.etae32 : m.L[l].fbeta; }

template <typename R> constexpr int prec_index() { return sizeof(R) == sizeof(double) ? 0 : 1; }

template <typename R>
static void smooth(Ctx* c, MG& m, int l, int sweeps)
{
    using B = LB<R>;
    Level& L = m.L[l];
    for (int s = 0; s < sweeps; ++s) {
        if (m.op == HB_OP_VISC && (L.g.dim == 2 || l > 0)) {
            // fused red-black sweep per component into the other buffer (2D,
            // and the small 3D levels, where it halves the launches)
            for (int q = 0; q < L.g.dim; ++q)
                launch_tsmooth<R>(c, L.g, tcoef<R>(m, l), l == 0, c->sc + S_DT, q, B::x(L), B::xo(L), B::b(L));
            L.cur ^= 1;
        } else if (m.op == HB_OP_VISC) {
            // finest 3D level: one colour of one component per launch, in
            // place (a 2-cell halo is costly on a 3D tile)
            for (int q = 0; q < L.g.dim; ++q)
                for (int colour = 0; colour < 2; ++colour)
                    launch_trb3<R>(c, L.g, tcoef<R>(m, l), l == 0, c->sc + S_DT, q, colour, B::x(L), B::b(L));
        } else if (m.op == HB_OP_MAC) {
            for (int colour = 0; colour < 2; ++colour) launch_mac_rb<R>(c, L.g, colour, B::x(L), B::b(L));
        } else {
            for (int colour = 0; colour < (1 << L.g.dim); ++colour) launch_nodal_gs<R>(c, L.g, colour, B::x(L), B::b(L));
        }
    }
}

template <typename R> static void vcycle(Ctx* c, MG& m, int l, int nu1, int nu2);

// Levels 1.. of the V-cycle as one HIP graph per precision: the coarse
// levels are many short launches, so replaying a captured graph removes most
// of their host launch cost.  All their kernel arguments are fixed (buffers,
// and dt read from device memory); with an even number of sweeps per cycle
// every double-buffered level ends the cycle in the buffer it started in.
template <typename R>
static void coarse_graph(Ctx* c, MG& m, int nu1, int nu2)
{
    const int pi = prec_index<R>();
    if (!m.gexec[pi] || m.gnu1[pi] != nu1 || m.gnu2[pi] != nu2) {
        if (m.gexec[pi]) {
            (void)hipGraphExecDestroy(m.gexec[pi]);
            m.gexec[pi] = nullptr;
        }
        if (hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            m.gfail[pi] = true;
            vcycle<R>(c, m, 1, nu1, nu2);
            return;
        }
        m.capturing = true;
        vcycle<R>(c, m, 1, nu1, nu2);
        m.capturing = false;
        hipGraph_t graph = nullptr;
        bool ok = hipStreamEndCapture(c->s, &graph) == hipSuccess && graph;
        ok = ok && hipGraphInstantiate(&m.gexec[pi], graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            m.gfail[pi] = true;
            m.gexec[pi] = nullptr;
            vcycle<R>(c, m, 1, nu1, nu2);
            return;
        }
        m.gnu1[pi] = nu1;
        m.gnu2[pi] = nu2;
    }
    (void)hipGraphLaunch(m.gexec[pi], c->s);
}

// one V-cycle from level l in precision R; the coarsest level is solved with
// the FP64 inverse of its dense matrix
template <typename R>
static void vcycle(Ctx* c, MG& m, int l, int nu1, int nu2)
{
    using B = LB<R>;
    Level& L = m.L[l];
    if (l == m.nlev - 1) {
        launch_coarse_solve<R>(c, m.ncoarse, m.Ainv, B::b(L), B::x(L));
        return;
    }
    if (l == 1 && !m.capturing && !m.gfail[prec_index<R>()] && m.nlev > 2 && (nu1 + nu2) % 2 == 0) {
        coarse_graph<R>(c, m, nu1, nu2);
        return;
    }
    Level& C = m.L[l + 1];
    smooth<R>(c, m, l, nu1);
    if (m.op == HB_OP_VISC) {
        launch_tresid_restr<R>(c, L.g, C.g, tcoef<R>(m, l), l == 0, c->sc + S_DT, B::x(L), B::b(L), B::b(C), B::x(C));
    } else if (m.op == HB_OP_MAC) {
        launch_mac_resid_restrict<R>(c, L.g, C.g, B::x(L), B::b(L), B::b(C), B::x(C));
    } else {
        launch_nodal_resid<R>(c, L.g, B::x(L), B::b(L), B::r(L), -1);
        launch_nodal_restrict<R>(c, L.g, C.g, B::r(L), B::b(C), B::x(C));
    }
    vcycle<R>(c, m, l + 1, nu1, nu2);
    if (m.op == HB_OP_NODAL) launch_nodal_prolong<R>(c, L.g, C.g, B::x(C), B::x(L));
    else launch_prolong_cells<R>(c, L.g, C.g, m.op == HB_OP_VISC ? L.g.dim : 1, m.op == HB_OP_VISC ? -1.0 : 1.0, B::x(C), B::x(L));
    smooth<R>(c, m, l, nu2);
}

// r = b - A x on level 0 (FP64) and its max-norm into slot S_MAX
static void resid0(Ctx* c, MG& m, const double* x, const double* b, double* r)
{
    set_slot_zero(c, S_MAX);
    const Level& L = m.L[0];
    if (m.op == HB_OP_VISC) launch_tresid(c, L.g, m.etae, true, c->sc + S_DT, x, b, r, S_MAX);
    else if (m.op == HB_OP_MAC) launch_mac_resid(c, L.g, x, b, r, S_MAX);
    else launch_nodal_resid<double>(c, L.g, x, b, r, S_MAX);
}

static void apply0(Ctx* c, MG& m, const double* x, double* y)
{
    const Level& L = m.L[0];
    if (m.op == HB_OP_VISC) launch_tresid(c, L.g, m.etae, true, c->sc + S_DT, x, nullptr, y, -1);
    else if (m.op == HB_OP_MAC) launch_mac_apply(c, L.g, x, y);
    else launch_nodal_resid<double>(c, L.g, x, nullptr, y, -1);
}

// z = M^{-1} r: one V-cycle from zero on level 0, in FP64 or (lo) in FP32
static void precond(Ctx* c, MG& m, const double* r, double* z, int nu1, int nu2, bool lo)
{
    Level& L = m.L[0];
    L.cur = 0;
    if (lo) {
        to_f32(c, r, L.fb, L.fx[0], L.nu);
        vcycle<float>(c, m, 0, nu1, nu2);
        from_f32(c, LB<float>::x(L), z, L.nu);
        return;
    }
    double* sb = L.b;
    L.b = const_cast<double*>(r);
    fill(c, L.X(), 0.0, L.nu);
    vcycle<double>(c, m, 0, nu1, nu2);
    copy(c, z, L.X(), L.nu);
    L.b = sb;
}

static double fetch_max(Ctx* c)
{
    fetch_slots(c);
    return c->hsc[S_MAX];
}

// Multigrid (optionally BiCGStab-accelerated) solve of A x = b on the
// prepared level-0 system; x in/out.  bn = |b|_inf.  With mixed precision
// every V-cycle runs in FP32 on the FP64 residual (defect correction, or the
// BiCGStab preconditioner); residuals, norms and the iterate stay FP64.
static int solve_core(Ctx* c, MG& m, double* x, double* b, double bn, const hb_mg_opts& o, hb_mg_report* rep)
{
    Level& L = m.L[0];
    const long n = L.nu;
    L.b = b;
    int cycles = 0, rc = HB_OK;
    double rel = 0.0;
    const bool lo = o.precision == HB_PREC_MIXED;
    if (bn == 0.0) {
        fill(c, x, 0.0, n);
    } else if (!o.krylov && !lo) {
        // the cycles work on the level's double buffer, seeded with x
        L.cur = 0;
        copy(c, L.X(), x, n);
        resid0(c, m, L.X(), b, L.r);
        rel = fetch_max(c) / bn;
        for (;;) {
            if (o.fixed_cycles) {
                if (cycles >= o.max_cycles) break;
            } else {
                if (rel <= o.tol_rel) break;
                if (cycles >= o.max_cycles) { rc = HB_ERR_NOCONV; break; }
            }
            vcycle<double>(c, m, 0, o.nu1, o.nu2);
            ++cycles;
            resid0(c, m, L.X(), b, L.r);
            rel = fetch_max(c) / bn;
            if (!std::isfinite(rel)) { rc = HB_ERR_NONFINITE; break; }
        }
        copy(c, x, L.X(), n);
    } else if (!o.krylov) {
        // defect correction: FP64 residual r = b - A x, one FP32 V-cycle
        // from zero on A e = r, x += e
        double* xw = L.xb[0];
        copy(c, xw, x, n);
        resid0(c, m, xw, b, L.r);
        rel = fetch_max(c) / bn;
        for (;;) {
            if (o.fixed_cycles) {
                if (cycles >= o.max_cycles) break;
            } else {
                if (rel <= o.tol_rel) break;
                if (cycles >= o.max_cycles) { rc = HB_ERR_NOCONV; break; }
            }
            L.cur = 0;
            to_f32(c, L.r, L.fb, L.fx[0], n);
            vcycle<float>(c, m, 0, o.nu1, o.nu2);
            ++cycles;
            add_f32(c, xw, LB<float>::x(L), n);
            resid0(c, m, xw, b, L.r);
            rel = fetch_max(c) / bn;
            if (!std::isfinite(rel)) { rc = HB_ERR_NONFINITE; break; }
        }
        copy(c, x, xw, n);
    } else {
        // BiCGStab with its scalars kept on the device: two host reads per
        // iteration (the residual norms that decide convergence)
        double *r = c->kr, *rh = c->krh, *p = c->kp, *v = c->kv, *ph = c->kph, *s = c->ks, *sh = c->ksh, *t = c->kt;
        resid0(c, m, x, b, r);
        copy(c, rh, r, n);
        fill(c, p, 0.0, n);
        fill(c, v, 0.0, n);
        bicg_init_scalars(c);
        rel = fetch_max(c) / bn;
        for (;;) {
            if (o.fixed_cycles) {
                if (cycles >= o.max_cycles) break;
            } else {
                if (rel <= o.tol_rel) break;
                if (cycles >= o.max_cycles) { rc = HB_ERR_NOCONV; break; }
            }
            red_dot(c, rh, r, n, S_DOT0);
            bicg_beta(c);
            bicg_p_dev(c, p, r, v, n);
            precond(c, m, p, ph, o.nu1, o.nu2, lo);
            ++cycles;
            apply0(c, m, ph, v);
            red_dot(c, rh, v, n, S_DOT1);
            bicg_alpha(c);
            sub_scaled_max_dev(c, s, r, S_ALPHA, v, n, S_MAX);
            fetch_slots(c);
            if (c->hsc[S_RHO] == 0.0) { rc = HB_ERR_NOCONV; break; }
            const double srel = c->hsc[S_MAX] / bn;
            if ((!o.fixed_cycles && srel <= o.tol_rel) || (o.fixed_cycles && cycles >= o.max_cycles)) {
                bicg_x_dev(c, x, ph, nullptr, false, n);
                copy(c, r, s, n);
                rel = srel;
                break;
            }
            precond(c, m, s, sh, o.nu1, o.nu2, lo);
            ++cycles;
            apply0(c, m, sh, t);
            red_dot(c, t, t, n, S_DOT0);
            red_dot(c, t, s, n, S_DOT1);
            bicg_omega(c);
            bicg_x_dev(c, x, ph, sh, true, n);
            sub_scaled_max_dev(c, r, s, S_OMEGA, t, n, S_MAX);
            fetch_slots(c);
            rel = c->hsc[S_MAX] / bn;
            if (!std::isfinite(rel)) { rc = HB_ERR_NONFINITE; break; }
            if (c->hsc[S_OMEGA] == 0.0) { rc = HB_ERR_NOCONV; break; }
        }
        resid0(c, m, x, b, L.r);
        rel = fetch_max(c) / bn;
        if (!std::isfinite(rel)) rc = HB_ERR_NONFINITE;
    }
    if (rep) {
        rep->cycles = cycles;
        rep->rel_resid = rel;
        rep->bnorm = bn;
    }
    return rc;
}

// solve with the right-hand side already in m.lvl0_b (VISC: wall part added,
// NODAL/MAC: mean removed by this function)
static int solve_prepared(Ctx* c, MG& m, double* x, const hb_mg_opts& o, hb_mg_report* rep)
{
    const long n = m.L[0].nu;
    if (m.op != HB_OP_VISC) sub_mean(c, m.lvl0_b, n);
    red_maxabs(c, m.lvl0_b, n, S_MAX);
    red_maxabs(c, x, n, S_MAX2);
    fetch_slots(c);
    const double bn = c->hsc[S_MAX];
    if (!std::isfinite(bn) || !std::isfinite(c->hsc[S_MAX2])) return fail(c, HB_ERR_NONFINITE, "non-finite right-hand side or guess");
    if (o.precision == HB_PREC_MIXED) ensure_f32(c, m);
    int rc = solve_core(c, m, x, m.lvl0_b, bn, o, rep);
    if (m.op != HB_OP_VISC) sub_mean(c, x, n);
    if (rc == HB_ERR_NOCONV) c->err = "multigrid did not reach the tolerance within max_cycles";
    if (rc == HB_ERR_NONFINITE) c->err = "multigrid produced a non-finite residual";
    return rc;
}

static bool valid_opts(const hb_mg_opts& o)
{
    return o.max_cycles >= 0 && o.max_cycles <= 100000 && o.nu1 >= 0 && o.nu2 >= 0 && o.nu1 + o.nu2 > 0 &&
           o.tol_rel >= 0.0 && (o.precision == HB_PREC_FP64 || o.precision == HB_PREC_MIXED);
}

// ---------------------------------------------------------------------------
// stages of the step
// ---------------------------------------------------------------------------

// advection stage; requires visc_setup(eta, dt) and S_MAXU = max|u|
static int advect_stage(Ctx* c, const double* u, const double* p, double dt, double* b, double* conv,
                        hb_mg_report* mac_rep, double* div_mac_rel)
{
    const MG& vm = c->visc;
    launch_visc_div(c, c->g, vm.L[0].beta, u, c->E);
    launch_grad_node(c, p, c->Gp);
    launch_forcing(c);
    launch_slopes(c, u);
    launch_trace_normal(c, u, dt);
    launch_transverse(c);
    launch_trace_full(c, u, dt);
    int rc = HB_OK;
    if (c->opts.mac_project) {
        launch_mac_div(c, c->uadv, c->mac.lvl0_b);
        double d0 = 0.0;
        if (div_mac_rel) {
            red_maxabs(c, c->mac.lvl0_b, c->nc, S_MAX);
            fetch_slots(c);
            d0 = c->hsc[S_MAX];
        }
        fill(c, c->macphi, 0.0, c->nc);
        rc = solve_prepared(c, c->mac, c->macphi, c->opts.mac, mac_rep);
        launch_mac_update(c);
        if (div_mac_rel) {
            launch_mac_div(c, c->umac, c->macrhs);
            red_maxabs(c, c->macrhs, c->nc, S_MAX);
            fetch_slots(c);
            *div_mac_rel = d0 > 0.0 ? c->hsc[S_MAX] / d0 : 0.0;
        }
    } else {
        copy(c, c->umac, c->uadv, c->nf);
        if (mac_rep) memset(mac_rep, 0, sizeof(*mac_rep));
        if (div_mac_rel) *div_mac_rel = 0.0;
    }
    launch_advect_rhs(c, u, dt, b, conv);
    return rc;
}

static int project_stage(Ctx* c, const double* ustar, double* p, double dt, double* u, hb_mg_report* rep)
{
    launch_grad_node(c, p, c->Gp);
    launch_proj_rhs(c, ustar, dt, c->nodal.lvl0_b);
    copy(c, c->phi, p, c->nn);
    int rc = solve_prepared(c, c->nodal, c->phi, c->opts.proj, rep);
    launch_proj_update(c, ustar, c->phi, dt, u);
    copy(c, p, c->phi, c->nn);
    return rc;
}

static bool worse(int rc, int cur) { return cur == HB_OK || (cur == HB_ERR_NOCONV && rc != HB_OK); }

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

void kt_begin(Ctx* c)
{
    KTimer& k = c->ktm;
    if (k.n == k.cap) kt_harvest(c);
    (void)hipEventRecord(k.ev[2 * k.n], c->s);
}

void kt_end(Ctx* c, double bytes)
{
    KTimer& k = c->ktm;
    (void)hipEventRecord(k.ev[2 * k.n + 1], c->s);
    ++k.n;
    ++k.launches;
    k.bytes += bytes;
}

void kt_harvest(Ctx* c)
{
    KTimer& k = c->ktm;
    if (k.n == 0) return;
    (void)hipEventSynchronize(k.ev[2 * k.n - 1]);
    for (int i = 0; i < k.n; ++i) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, k.ev[2 * i], k.ev[2 * i + 1]) == hipSuccess) k.ms += t;
    }
    k.n = 0;
}

static void kt_free(Ctx* c)
{
    KTimer& k = c->ktm;
    if (!k.ev) return;
    for (int i = 0; i < 2 * k.cap; ++i) (void)hipEventDestroy(k.ev[i]);
    delete[] k.ev;
    k.ev = nullptr;
    k.cap = 0;
    k.on = false;
}

}  // namespace hb

using namespace hb;

struct hb_ctx : public Ctx {};

// Work of an ABI call runs on the library's stream, after everything queued
// on the caller's stream before the call, and the caller's stream waits for
// it afterwards.
struct StreamGuard {
    Ctx* c;
    explicit StreamGuard(Ctx* cc) : c(cc)
    {
        (void)hipEventRecord(c->ev_in, c->user);
        (void)hipStreamWaitEvent(c->s, c->ev_in, 0);
    }
    ~StreamGuard()
    {
        (void)hipEventRecord(c->ev_out, c->s);
        (void)hipStreamWaitEvent(c->user, c->ev_out, 0);
    }
};

extern "C" {

const char* hb_last_error(const hb_ctx* ctx)
{
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

void hb_destroy(hb_ctx* ctx)
{
    if (!ctx) return;
    Ctx* c = ctx;
    kt_free(c);
    free_mg(c->visc);
    free_mg(c->mac);
    free_mg(c->nodal);
    if (c->s) (void)hipStreamSynchronize(c->s);
    double* bufs[] = {c->eta, c->E, c->Gp, c->F, c->S, c->trans, c->uhat, c->qhat, c->qLf, c->qRf, c->uadv,
                      c->umac, c->macphi, c->macrhs, c->b, c->ustar, c->rnode, c->phi, c->conv, c->kr, c->krh,
                      c->kp, c->kv, c->kph, c->ks, c->ksh, c->kt, c->dense_E, c->sc, c->partial};
    for (double* p : bufs) (void)hipFree(p);
    if (c->hsc) (void)hipHostFree(c->hsc);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->s) (void)hipStreamDestroy(c->s);
    delete ctx;
}

int hb_create(const hb_grid* grid, const hb_fluid* fluid, const hb_step_opts* opts, void* hip_stream, hb_ctx** out)
{
    if (out) *out = nullptr;
    auto bad = [](const char* m) { g_create_err = m; return HB_ERR_ARG; };
    if (!grid || !fluid || !opts || !out) return bad("null argument");
    if (grid->dim != 2 && grid->dim != 3) return bad("dim must be 2 or 3");
    for (int a = 0; a < grid->dim; ++a) {
        if (!valid_extent(grid->n[a])) return bad("each n[a] must be c*2^k, c in {1,2,3}, n >= 4");
        if (grid->bc[a][0] != grid->bc[a][1] && (grid->bc[a][0] == HB_BC_PERIODIC || grid->bc[a][1] == HB_BC_PERIODIC))
            return bad("periodic faces must come in pairs");
        for (int s = 0; s < 2; ++s)
            if (grid->bc[a][s] != HB_BC_WALL && grid->bc[a][s] != HB_BC_PERIODIC) return bad("unknown boundary type");
    }
    if (!(grid->h > 0.0) || !std::isfinite(grid->h)) return bad("h must be positive");
    if (!(fluid->Re > 0.0) || !(fluid->Pa > 0.0) || !(fluid->n > 0.0) || !(fluid->HB >= 0.0))
        return bad("need Re > 0, Pa > 0, n > 0, HB >= 0");
    if (fluid->reg != HB_REG_PAPER && fluid->reg != HB_REG_YIELD_ONLY) return bad("unknown regularisation");
    if (fluid->reg == HB_REG_YIELD_ONLY && fluid->n < 1.0) return bad("yield-only regularisation needs n >= 1");
    if (!valid_opts(opts->mac) || !valid_opts(opts->visc) || !valid_opts(opts->proj)) return bad("invalid multigrid options");
    if (!(opts->cfl > 0.0)) return bad("cfl must be positive");

    hb_ctx* ctx = new (std::nothrow) hb_ctx();
    if (!ctx) return bad("out of host memory");
    Ctx* c = ctx;
    c->grid = *grid;
    c->fluid = *fluid;
    c->opts = *opts;
    c->user = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
        g_create_err = "stream or event creation failed";
        hb_destroy(ctx);
        return HB_ERR_DEVICE;
    }
    c->g = make_gridd(*grid);
    c->fl.Re = fluid->Re;
    c->fl.HB = fluid->HB;
    c->fl.n = fluid->n;
    c->fl.Pa = fluid->Pa;
    c->fl.reg = fluid->reg;
    for (int q = 0; q < 3; ++q) c->fl.f[q] = q < grid->dim ? fluid->f[q] : 0.0;
    c->dim = grid->dim;
    c->nc = ncells(c->g);
    c->nn = nnodes(c->g);
    c->nf = nface_total(c->g);
    c->ulid = 0.0;
    for (int a = 0; a < c->dim; ++a)
        for (int s = 0; s < 2; ++s)
            for (int q = 0; q < 3; ++q) c->ulid = std::fmax(c->ulid, std::fabs(c->g.wall_u[a][s][q]));

    auto oom = [&](const std::string& m) {
        g_create_err = m.empty() ? "device allocation failed" : m;
        hb_destroy(ctx);
        return HB_ERR_OOM;
    };
    int rc;
    if ((rc = build_mg(c, c->visc, HB_OP_VISC)) != HB_OK) { g_create_err = c->err; hb_destroy(ctx); return rc; }
    if ((rc = build_mg(c, c->mac, HB_OP_MAC)) != HB_OK) { g_create_err = c->err; hb_destroy(ctx); return rc; }
    if ((rc = build_mg(c, c->nodal, HB_OP_NODAL)) != HB_OK) { g_create_err = c->err; hb_destroy(ctx); return rc; }
    const long d = c->dim, nc = c->nc, nf = c->nf, nn = c->nn;
    const long nv = d * nc;
    bool ok = true;
    ok = ok && dalloc(&c->eta, nc) == hipSuccess && dalloc(&c->E, nv) == hipSuccess && dalloc(&c->Gp, nv) == hipSuccess;
    ok = ok && dalloc(&c->F, nv) == hipSuccess && dalloc(&c->S, d * d * nc) == hipSuccess &&
         dalloc(&c->trans, d * d * nc) == hipSuccess;
    ok = ok && dalloc(&c->uhat, nf) == hipSuccess && dalloc(&c->qhat, d * nf) == hipSuccess &&
         dalloc(&c->qLf, d * nf) == hipSuccess && dalloc(&c->qRf, d * nf) == hipSuccess;
    ok = ok && dalloc(&c->uadv, nf) == hipSuccess && dalloc(&c->umac, nf) == hipSuccess &&
         dalloc(&c->macphi, nc) == hipSuccess && dalloc(&c->macrhs, nc) == hipSuccess;
    ok = ok && dalloc(&c->b, nv) == hipSuccess && dalloc(&c->ustar, nv) == hipSuccess &&
         dalloc(&c->rnode, nn) == hipSuccess && dalloc(&c->phi, nn) == hipSuccess && dalloc(&c->conv, nv) == hipSuccess;
    ok = ok && dalloc(&c->kr, nv) == hipSuccess && dalloc(&c->krh, nv) == hipSuccess && dalloc(&c->kp, nv) == hipSuccess &&
         dalloc(&c->kv, nv) == hipSuccess && dalloc(&c->kph, nv) == hipSuccess && dalloc(&c->ks, nv) == hipSuccess &&
         dalloc(&c->ksh, nv) == hipSuccess && dalloc(&c->kt, nv) == hipSuccess;
    int nmax = c->visc.ncoarse;
    if (c->mac.ncoarse > nmax) nmax = c->mac.ncoarse;
    if (c->nodal.ncoarse > nmax) nmax = c->nodal.ncoarse;
    ok = ok && dalloc(&c->dense_E, (long)nmax * nmax) == hipSuccess;
    ok = ok && dalloc(&c->sc, S_NSLOT) == hipSuccess && dalloc(&c->partial, kRedBlocks) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&c->hsc, sizeof(double) * S_NSLOT) == hipSuccess;
    if (!ok) return oom("");
    fill(c, c->sc, 0.0, S_NSLOT);
    // constant coarsest matrices of the MAC and nodal problems
    factor_coarsest(c, c->mac);
    factor_coarsest(c, c->nodal);
    if (hipStreamSynchronize(c->s) != hipSuccess) return oom("stream synchronisation failed during set-up");
    *out = ctx;
    return HB_OK;
}

int hb_viscosity(hb_ctx* ctx, const double* u, double* eta)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    if (!u || !eta) return fail(c, HB_ERR_ARG, "null array");
    StreamGuard guard(c);
    launch_viscosity(c, u, eta);
    return hipGetLastError() == hipSuccess ? HB_OK : fail(c, HB_ERR_DEVICE, "kernel launch failed");
}

int hb_mg_solve(hb_ctx* ctx, int op, const double* eta, double dt, const double* rhs, double* x,
                const hb_mg_opts* opts, hb_mg_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    if (!rhs || !x) return fail(c, HB_ERR_ARG, "null array");
    if (op != HB_OP_VISC && op != HB_OP_NODAL && op != HB_OP_MAC) return fail(c, HB_ERR_ARG, "unknown operator");
    if (op == HB_OP_VISC && (!eta || !(dt > 0.0))) return fail(c, HB_ERR_ARG, "viscous solve needs eta and dt > 0");
    const hb_mg_opts& o = opts ? *opts : (op == HB_OP_VISC ? c->opts.visc : (op == HB_OP_MAC ? c->opts.mac : c->opts.proj));
    if (!valid_opts(o)) return fail(c, HB_ERR_ARG, "invalid multigrid options");
    MG& m = op == HB_OP_VISC ? c->visc : (op == HB_OP_MAC ? c->mac : c->nodal);
    StreamGuard guard(c);
    if (op == HB_OP_VISC) {
        visc_setup(c, eta, dt);
        launch_visc_wall_rhs(c, c->g, m.L[0].beta, dt, rhs, m.lvl0_b);
    } else {
        copy(c, m.lvl0_b, rhs, m.L[0].nu);
    }
    return solve_prepared(c, m, x, o, report);
}

int hb_advect(hb_ctx* ctx, const double* u, const double* p, const double* eta, double dt, double* b, double* umac,
              double* conv, hb_mg_report* mac_report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    if (!u || !p || !eta || !b) return fail(c, HB_ERR_ARG, "null array");
    if (!(dt > 0.0)) return fail(c, HB_ERR_ARG, "dt must be positive");
    StreamGuard guard(c);
    red_maxabs(c, u, c->dim * c->nc, S_MAXU);
    visc_setup(c, eta, dt);
    int rc = advect_stage(c, u, p, dt, b, conv, mac_report, nullptr);
    if (umac) copy(c, umac, c->umac, c->nf);
    if (hipStreamSynchronize(c->s) != hipSuccess) return fail(c, HB_ERR_DEVICE, "stream synchronisation failed");
    return rc;
}

int hb_project(hb_ctx* ctx, const double* ustar, double* p, double dt, double* u, hb_mg_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    if (!ustar || !p || !u) return fail(c, HB_ERR_ARG, "null array");
    if (!(dt > 0.0)) return fail(c, HB_ERR_ARG, "dt must be positive");
    StreamGuard guard(c);
    return project_stage(c, ustar, p, dt, u, report);
}

int hb_cfl_dt(hb_ctx* ctx, const double* u, double* dt_out)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    if (!u || !dt_out) return fail(c, HB_ERR_ARG, "null argument");
    StreamGuard guard(c);
    red_maxabs(c, u, c->dim * c->nc, S_MAXU);
    fetch_slots(c);
    const double m = std::fmax(c->ulid, c->hsc[S_MAXU]);
    if (!std::isfinite(m)) return fail(c, HB_ERR_NONFINITE, "non-finite velocity");
    *dt_out = m > 0.0 ? c->opts.cfl * c->g.h / m : 0.0;
    return HB_OK;
}

int hb_step(hb_ctx* ctx, double* u, double* p, double dt, hb_step_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    if (!u || !p) return fail(c, HB_ERR_ARG, "null array");
    StreamGuard guard(c);
    const long nv = c->dim * c->nc;
    red_maxabs(c, u, nv, S_MAXU);
    red_maxabs(c, p, c->nn, S_MAX2);
    fetch_slots(c);
    if (!std::isfinite(c->hsc[S_MAXU]) || !std::isfinite(c->hsc[S_MAX2])) return fail(c, HB_ERR_NONFINITE, "non-finite u or p");
    if (!(dt > 0.0)) {
        const double m = std::fmax(c->ulid, c->hsc[S_MAXU]);
        if (!(m > 0.0)) return fail(c, HB_ERR_ARG, "dt <= 0 with zero velocity everywhere");
        dt = c->opts.cfl * c->g.h / m;
    }
    hb_step_report R;
    memset(&R, 0, sizeof(R));
    R.dt = dt;
    launch_viscosity(c, u, c->eta);
    visc_setup(c, c->eta, dt);
    int rc = advect_stage(c, u, p, dt, c->b, nullptr, &R.mac, report ? &R.div_mac_rel : nullptr);
    if (rc != HB_OK && rc != HB_ERR_NOCONV) return rc;
    int rc2 = HB_OK;
    launch_visc_wall_rhs(c, c->g, c->visc.L[0].beta, dt, c->b, c->visc.lvl0_b);
    copy(c, c->ustar, u, nv);
    rc2 = solve_prepared(c, c->visc, c->ustar, c->opts.visc, &R.visc);
    if (worse(rc2, rc)) rc = rc2;
    if (rc != HB_OK && rc != HB_ERR_NOCONV) return rc;
    rc2 = project_stage(c, c->ustar, p, dt, u, &R.proj);
    if (worse(rc2, rc)) rc = rc2;
    if (report) {
        red_maxabs(c, u, nv, S_MAX);
        launch_weak_div(c, u, c->rnode);
        red_maxabs(c, c->rnode, c->nn, S_MAX2);
        fetch_slots(c);
        R.max_u = c->hsc[S_MAX];
        R.div_node = c->hsc[S_MAX2] / std::pow(c->g.h, c->dim);
        *report = R;
    }
    if (hipGetLastError() != hipSuccess) return fail(c, HB_ERR_DEVICE, "kernel launch failed");
    return rc;
}

int hb_kernel_timing(hb_ctx* ctx, int enable)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = ctx;
    KTimer& k = c->ktm;
    if (enable && !k.ev) {
        const int cap = 2048;
        k.ev = new (std::nothrow) hipEvent_t[2 * cap];
        if (!k.ev) return fail(c, HB_ERR_OOM, "out of host memory");
        for (int i = 0; i < 2 * cap; ++i)
            if (hipEventCreate(&k.ev[i]) != hipSuccess) {
                k.cap = i / 2;
                kt_free(c);
                return fail(c, HB_ERR_DEVICE, "hipEventCreate failed");
            }
        k.cap = cap;
    }
    if (!enable) kt_harvest(c);
    k.on = enable != 0;
    k.n = 0;
    k.launches = 0;
    k.ms = 0.0;
    k.bytes = 0.0;
    return HB_OK;
}

int hb_kernel_timing_read(hb_ctx* ctx, int64_t* launches, double* total_ms, double* alg_bytes)
{
    if (!ctx || !launches || !total_ms || !alg_bytes) return HB_ERR_ARG;
    Ctx* c = ctx;
    kt_harvest(c);
    *launches = c->ktm.launches;
    *total_ms = c->ktm.ms;
    *alg_bytes = c->ktm.bytes;
    return HB_OK;
}

}  // extern "C"
