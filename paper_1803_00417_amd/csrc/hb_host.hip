// hb_host.hip -- context set-up, batched multigrid drivers (V-cycle and
// BiCGStab acceleration, FP64 or mixed precision), the time step and the C
// ABI of include/hb.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "hb_internal.h"

// the opaque handle of the C ABI is the context itself
struct hb_ctx : public hb::Ctx {};

namespace hb {

static thread_local std::string g_create_err;

void set_global_error(const char* msg) { g_create_err = msg; }

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

static GridD absent_grid()
{
    GridD d;
    memset(&d, 0, sizeof(d));
    return d;
}

static long comp_count(const GridD& g, int op) { return op == HB_OP_NODAL ? nnodes(g) : ncells(g); }

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

// allocate n device buffers, all or none (on failure every one is freed
// and nulled)
static bool alloc_all(void** b, const size_t* sz, int n)
{
    for (int i = 0; i < n; ++i) {
        if (hipMalloc(&b[i], sz[i]) != hipSuccess) {
            for (int k = 0; k < n; ++k) {
                if (b[k]) (void)hipFree(b[k]);
                b[k] = nullptr;
            }
            return false;
        }
    }
    return true;
}

template <typename T>
static hipError_t upload(T* dst, const std::vector<T>& src)
{
    return hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------

// unknowns of problem op on grid g
static long op_unknowns(const GridD& g, int op)
{
    if (op == HB_OP_VISC) return (long)g.dim * ncells(g);
    return op == HB_OP_MAC ? ncells(g) : nnodes(g);
}

// The levels of one cavity's hierarchy for problem op: halve every extent
// while all are even and at least 4, and stop at the first level with at
// most kDenseMax unknowns (MAC 8^2 / 4^3 cells, nodal 9^2 / 5^3 nodes,
// tensor 2 x 8^2 in 2D, 3 x 2^3 in 3D), which is solved by its dense inverse
static std::vector<GridD> level_grids(const GridD& g0, int op)
{
    std::vector<GridD> out;
    GridD cur = g0;
    for (;;) {
        out.push_back(cur);
        bool can = (int)out.size() < kMaxLev;
        for (int a = 0; a < cur.dim; ++a)
            if ((cur.n[a] & 1) || cur.n[a] / 2 < 2) can = false;
        if (op_unknowns(cur, op) <= kDenseMax) can = false;
        if (!can) break;
        GridD nx = cur;
        for (int a = 0; a < cur.dim; ++a) nx.n[a] = cur.n[a] / 2;
        nx.h = cur.h * 2.0;
        memset(nx.wall_u, 0, sizeof(nx.wall_u));
        cur = nx;
    }
    return out;
}

static int build_mg(Ctx* c, MG& m, int op)
{
    m.op = op;
    m.rec = op == HB_OP_VISC ? S_REC_VISC : (op == HB_OP_MAC ? S_REC_MAC : S_REC_NODAL);
    m.ncomp = op == HB_OP_VISC ? c->dim : 1;
    const int nb = c->nb;
    std::vector<std::vector<GridD>> lg(nb);
    m.nlev = 0;
    m.nlevc.resize(nb);
    for (int b = 0; b < nb; ++b) {
        lg[b] = level_grids(c->cv[b].g, op);
        m.nlevc[b] = (int)lg[b].size();
        m.nlev = std::max(m.nlev, m.nlevc[b]);
    }
    for (int l = 0; l < m.nlev; ++l) {
        Level& L = m.L[l];
        L.hg.assign(nb, absent_grid());
        L.ho.assign(nb, 0);
        L.hof.assign(nb, 0);
        L.hou.assign(nb, 0);
        L.hnu.assign(nb, 0);
        std::vector<GridD> gsm(nb, absent_grid());
        L.gmax = absent_grid();
        L.gmax.dim = c->dim;
        L.gmax.n[0] = L.gmax.n[1] = L.gmax.n[2] = 1;
        long oc = 0, of = 0;
        for (int b = 0; b < nb; ++b) {
            L.ho[b] = oc;
            L.hof[b] = of;
            L.hou[b] = m.ncomp * oc;
            if (l >= m.nlevc[b]) continue;
            const GridD& g = lg[b][l];
            L.hg[b] = g;
            if (l < m.nlevc[b] - 1) {
                gsm[b] = g;
                L.any_sm = true;
            } else {
                L.any_cs = true;
            }
            for (int a = 0; a < 3; ++a) L.gmax.n[a] = std::max(L.gmax.n[a], g.n[a]);
            const long cnt = comp_count(g, op);
            L.hnu[b] = m.ncomp * cnt;
            oc += cnt;
            if (op == HB_OP_VISC) of += nface_total(g);
        }
        L.nu = m.ncomp * oc;
        HB_TRY(dalloc(&L.xb[0], L.nu));
        HB_TRY(dalloc(&L.xb[1], L.nu));
        if (l > 0) HB_TRY(dalloc(&L.b, L.nu));
        HB_TRY(dalloc(&L.r, L.nu));
        if (op == HB_OP_VISC) HB_TRY(dalloc(&L.beta, of));
        HB_TRY(dalloc(&L.fx[0], L.nu));
        HB_TRY(dalloc(&L.fx[1], L.nu));
        HB_TRY(dalloc(&L.fb, L.nu));
        if (op == HB_OP_NODAL) HB_TRY(dalloc(&L.fr, L.nu));
        if (op == HB_OP_VISC && l > 0) HB_TRY(dalloc(&L.fbeta, of));
        HB_TRY(dalloc(&L.gall, nb));
        HB_TRY(dalloc(&L.gsm, nb));
        HB_TRY(dalloc(&L.o, nb));
        HB_TRY(dalloc(&L.of, nb));
        HB_TRY(dalloc(&L.ou, nb));
        HB_TRY(dalloc(&L.nuc, nb));
        HB_TRY(upload(L.gall, L.hg));
        HB_TRY(upload(L.gsm, gsm));
        HB_TRY(upload(L.o, L.ho));
        HB_TRY(upload(L.of, L.hof));
        HB_TRY(upload(L.ou, L.hou));
        HB_TRY(upload(L.nuc, L.hnu));
    }
    // single-workgroup coarse tail: the first level from which every
    // cavity's remaining levels fit the LDS budget
    m.tail_lt = -1;
    if (c->tail && c->lds_budget > 0) {
        for (int l = 1; l < m.nlev && m.tail_lt < 0; ++l) {
            if (m.nlev - l > kMaxTail) continue;
            size_t need[2] = {0, 0};
            std::vector<TailPlan> plans(nb);
            for (int b = 0; b < nb; ++b) {
                if (m.nlevc[b] - 1 < l) continue;
                const std::vector<GridD> gl(lg[b].begin() + l, lg[b].end());
                std::vector<long> gofs;
                for (int k = l; k < m.nlevc[b]; ++k) gofs.push_back(m.L[k].hof[b]);
                const long o0 = m.L[l].ho[b];
                need[0] = std::max(need[0], tail_plan(op, gl, gofs, o0, sizeof(double), &plans[b]));
                need[1] = std::max(need[1], tail_plan(op, gl, gofs, o0, sizeof(float), nullptr));
            }
            if (need[0] > 0 && need[0] <= c->lds_budget) {
                m.tail_lt = l;
                m.tail_lds[0] = need[0];
                m.tail_lds[1] = need[1];
                HB_TRY(dalloc(&m.tplan, nb));
                HB_TRY(upload(m.tplan, plans));
            }
        }
    }
    // coarsest systems
    m.hcs.resize(nb);
    long aoff = 0, poff = 0;
    m.ncmax = 0;
    for (int b = 0; b < nb; ++b) {
        CoarseD& d = m.hcs[b];
        d.lev = m.nlevc[b] - 1;
        d.N = (int)m.L[d.lev].hnu[b];
        d.aoff = aoff;
        d.poff = poff;
        d.xoff = m.L[d.lev].hou[b];
        aoff += (long)d.N * d.N;
        poff += d.N;
        m.ncmax = std::max(m.ncmax, d.N);
    }
    HB_TRY(dalloc(&m.cs, nb));
    HB_TRY(upload(m.cs, m.hcs));
    HB_TRY(dalloc(&m.A, aoff));
    HB_TRY(dalloc(&m.Ainv, aoff));
    HB_TRY(dalloc(&m.piv, poff));
    HB_TRY(dalloc(&m.lvl0_b, m.L[0].nu));
    m.L[0].b = m.lvl0_b;
    if (op == HB_OP_VISC) {
        HB_TRY(dalloc(&m.etae, m.L[0].nu / m.ncomp));
        HB_TRY(dalloc(&m.etae32, m.L[0].nu / m.ncomp));
    }
    m.seg0.off = m.L[0].ou;
    m.seg0.n = m.L[0].nuc;
    m.seg0.act = nullptr;
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
        (void)hipFree(L.gall);
        (void)hipFree(L.gsm);
        (void)hipFree(L.o);
        (void)hipFree(L.of);
        (void)hipFree(L.ou);
        (void)hipFree(L.nuc);
    }
    (void)hipFree(m.cs);
    (void)hipFree(m.dd);
    (void)hipFree(m.tplan);
    (void)hipFree(m.A);
    (void)hipFree(m.Ainv);
    (void)hipFree(m.piv);
    (void)hipFree(m.lvl0_b);
    (void)hipFree(m.etae);
    (void)hipFree(m.etae32);
    for (int p = 0; p < 2; ++p)
        if (m.gexec[p]) (void)hipGraphExecDestroy(m.gexec[p]);
}

// dense coarsest matrix of cavity b of the MAC or nodal problem (constant),
// A + 1 1^T / N, LU and inverse; at context creation
static void factor_coarsest(Ctx* c, MG& m, int b)
{
    const CoarseD& d = m.hcs[b];
    const int N = d.N;
    const Level& C = m.L[d.lev];
    const GridD& g = C.hg[b];
    double* A = m.A + d.aoff;
    launch_identity(c, N, c->cv[b].dense_E);
    if (m.op == HB_OP_MAC) launch_mac_dense(c, g, N, c->cv[b].dense_E, A);
    else launch_nodal_dense(c, g, N, c->cv[b].dense_E, A);
    launch_add_ones(c, N, A);
    launch_dense_inverse(c, N, A, m.piv + d.poff, m.Ainv + d.aoff);
}

// The tensor problem's coarsest matrices of every cavity (new with every
// viscosity), assembled and inverted on the second stream: the work needs
// the coefficients just written on s, and only the viscous solve reads its
// result (join_visc_factor), so it overlaps whatever s runs in between.
static void factor_visc_async(Ctx* c)
{
    (void)hipEventRecord(c->ev_f0, c->s);
    (void)hipStreamWaitEvent(c->s2, c->ev_f0, 0);
    hipStream_t keep = c->s;
    c->s = c->s2;   // the launch helpers enqueue on c->s
    launch_visc_dense_batch(c, c->visc);
    launch_gj_inverse_batch(c, c->visc);
    c->s = keep;
    (void)hipEventRecord(c->ev_f1, c->s2);
    c->visc_factor_pending = true;
}

// order s after the factorisation factor_visc_async enqueued
static void join_visc_factor(Ctx* c)
{
    if (!c->visc_factor_pending) return;
    (void)hipStreamWaitEvent(c->s, c->ev_f1, 0);
    c->visc_factor_pending = false;
}

// Upload the per-call table.  The two halves of the pinned staging buffer
// are used in turn; every call that uploads ends by waiting for its stream
// (fetch_slots), so a half is never rewritten while its copy is pending.
static void set_io(Ctx* c, const std::vector<CavIO>& io)
{
    c->io_half ^= 1;
    CavIO* h = c->hio + (long)c->io_half * c->nb;
    memcpy(h, io.data(), sizeof(CavIO) * c->nb);
    (void)hipMemcpyAsync(c->cio, h, sizeof(CavIO) * c->nb, hipMemcpyHostToDevice, c->s);
}

static CavIO io_zero()
{
    CavIO z;
    memset(&z, 0, sizeof(z));
    return z;
}

// face viscosities of every level of every cavity from its cell viscosity
// (CavIO::eta, not /Re) and its operator coefficient (CavIO::vdt) into the
// slot S_DT; the coarsest matrices follow (factor_visc_async)
static void visc_setup(Ctx* c)
{
    MG& m = c->visc;
    stage_visc_coef(c);
    for (int l = 1; l < m.nlev; ++l) stage_restrict_faces(c, l);
    m.f32_ready = false;
}

// FP32 copies of the tensor coefficients for mixed-precision cycles (the
// coarsest matrices stay the FP64 ones)
static void ensure_f32(Ctx* c, MG& m)
{
    if (m.op != HB_OP_VISC || m.f32_ready) return;
    flat_to_f32(c, m.etae, m.etae32, m.L[0].nu / m.ncomp);
    for (int l = 1; l < m.nlev; ++l) {
        long nf = 0;
        for (const GridD& g : m.L[l].hg)
            if (g.dim) nf += nface_total(g);
        flat_to_f32(c, m.L[l].beta, m.L[l].fbeta, nf);
    }
    m.f32_ready = true;
}

// ---------------------------------------------------------------------------
// V-cycle over the batch (cavities masked by c->act)
// ---------------------------------------------------------------------------

// tensor coefficients of level l for the tiled kernels: eta/Re cells on the
// finest level, face arrays below
template <typename R> static const R* tcoef(const MG& m, int l);
template <> const double* tcoef<double>(const MG& m, int l) { return l == 0 ? m.etae : m.L[l].beta; }
template <> const float* tcoef<float>(const MG& m, int l) { return l == 0 ? m.etae32 : m.L[l].fbeta; }

template <typename R> constexpr int prec_index() { return sizeof(R) == sizeof(double) ? 0 : 1; }

// Batched views of a level: the cavities that smooth on it, or all that have
// it.  A single-cavity context passes its grids by value (BV::one).
static BV smooth_view(const Ctx* c, const Level& L)
{
    BV v{L.gsm, L.o, L.of, c->act, 1};
    if (c->nb == 1) {
        v.one = 1;
        v.g1 = L.any_sm ? L.hg[0] : absent_grid();
    }
    return v;
}

static BV all_view(const Ctx* c, const Level& L, const int* act)
{
    BV v{L.gall, L.o, L.of, act, 1};
    if (c->nb == 1) {
        v.one = 1;
        v.g1 = L.hg[0];
    }
    return v;
}

// the view with the grid of the paired level of a transfer kernel
static BV paired(BV v, const Level& P)
{
    if (v.one) v.g2 = P.hg[0];
    return v;
}

// True when the last pre-smoothing launch of level L may also restrict the
// residual: its tile halo (tensor problem 4 sweeps per launch + 1, MAC 2
// sweeps + 1, nodal 4 sweeps + 2; sweeps at most 2) wraps a periodic axis
// once, so every periodic extent must be at least that halo.
static bool periodic_at_least(const Level& L, int n)
{
    for (const GridD& g : L.hg)
        for (int a = 0; a < g.dim; ++a)
            if (g.per[a] && g.n[a] < n) return false;
    return true;
}

static bool res_fold_ok(const Level& L, int op)
{
    return periodic_at_least(L, op == HB_OP_MAC ? 2 * 2 + 1 : 4 * L.sweeps + (op == HB_OP_NODAL ? 2 : 1));
}

// Smoothing sweeps on level l.  C (optional): the coarse level whose
// correction the first sweep adds to the iterate first (2D, fused sweeps:
// MAC and nodal problems, tensor problem with a staged candidate).
// RC (optional, 2D: MAC and nodal problems, tensor problem with a staged
// candidate): the coarse level into which the last launch restricts the
// residual of its result (see res_fold_ok).
template <typename R>
static void smooth(Ctx* c, MG& m, int l, int sweeps, bool pair, const Level* C = nullptr, Level* RC = nullptr)
{
    using B = LB<R>;
    Level& L = m.L[l];
    const BV v = smooth_view(c, L);
    for (int s = 0; s < sweeps; ++s) {
        if (m.op == HB_OP_VISC && c->dim == 2 && c->fuse) {
            // both components of the sweep in one launch; with `pair`, two
            // sweeps per launch where the level's candidate runs them so
            const int n = (pair && L.sweeps == 2 && sweeps - s >= 2) ? 2 : 1;
            // a zero level-0 iterate is not read (nullptr: the sweep takes zeros)
            const R* xc = (l == 0 && s == 0 && m.zero0) ? nullptr : B::x(L);
            if (s == 0 && C)
                launch_tsweep2<R>(c, L, paired(v, *C), tcoef<R>(m, l), l == 0, B::x(L), B::xo(L), B::b(L), L.tile, n,
                                  B::x(*C), C->gall, C->o);
            else if (s + n == sweeps && RC)
                launch_tsweep2<R>(c, L, paired(v, *RC), tcoef<R>(m, l), l == 0, xc, B::xo(L), B::b(L), L.tile, n,
                                  nullptr, RC->gall, RC->o, B::b(*RC), B::x(*RC));
            else
                launch_tsweep2<R>(c, L, v, tcoef<R>(m, l), l == 0, xc, B::xo(L), B::b(L), L.tile, n);
            if (l == 0) m.zero0 = false;
            L.cur ^= 1;
            s += n - 1;
        } else if (m.op == HB_OP_VISC && (c->dim == 2 || l > 0 || c->fine3 == 1)) {
            // fused red-black sweep per component into the other buffer (2D,
            // and the small 3D levels, where it halves the launches)
            for (int q = 0; q < c->dim; ++q)
                launch_tsmooth<R>(c, L, v, tcoef<R>(m, l), l == 0, q, B::x(L), B::xo(L), B::b(L));
            L.cur ^= 1;
        } else if (m.op == HB_OP_VISC) {
            // finest 3D level: one colour of one component per launch, in
            // place (a 2-cell halo is costly on a 3D tile)
            for (int q = 0; q < c->dim; ++q)
                for (int colour = 0; colour < 2; ++colour)
                    launch_trb3<R>(c, L, v, tcoef<R>(m, l), l == 0, q, colour, B::x(L), B::b(L));
        } else if (m.op == HB_OP_MAC && c->fuse) {
            // both colours in one launch, into the other buffer (2D: two
            // sweeps per launch with `pair`)
            const int n = (c->dim == 2 && pair && sweeps - s >= 2) ? 2 : 1;
            if (s == 0 && C)
                launch_mac_sweep<R>(c, L, paired(v, *C), B::x(L), B::xo(L), B::b(L), n, B::x(*C), C->gall, C->o);
            else if (s + n == sweeps && RC)
                launch_mac_sweep<R>(c, L, paired(v, *RC), B::x(L), B::xo(L), B::b(L), n, nullptr, RC->gall, RC->o,
                                    B::b(*RC), B::x(*RC));
            else
                launch_mac_sweep<R>(c, L, v, B::x(L), B::xo(L), B::b(L), n);
            L.cur ^= 1;
            s += n - 1;
        } else if (m.op == HB_OP_MAC) {
            for (int colour = 0; colour < 2; ++colour) launch_mac_rb<R>(c, L, v, colour, B::x(L), B::b(L));
        } else if (c->fuse) {
            // all colours of a sweep in one launch (two in 3D) into the other
            // buffer; 2D: two sweeps per launch with `pair` where the level allows
            const int n = (pair && L.sweeps == 2 && sweeps - s >= 2) ? 2 : 1;
            if (s == 0 && C)
                launch_nodal_sweep<R>(c, L, paired(v, *C), B::x(L), B::xo(L), B::b(L), L.tile, n, B::x(*C), C->gall,
                                      C->o);
            else if (s + n == sweeps && RC)
                launch_nodal_sweep<R>(c, L, paired(v, *RC), B::x(L), B::xo(L), B::b(L), L.tile, n, nullptr, RC->gall,
                                      RC->o, B::b(*RC), B::x(*RC));
            else
                launch_nodal_sweep<R>(c, L, v, B::x(L), B::xo(L), B::b(L), L.tile, n);
            L.cur ^= 1;
            s += n - 1;
        } else {
            for (int colour = 0; colour < (1 << c->dim); ++colour) launch_nodal_gs<R>(c, L, v, colour, B::x(L), B::b(L));
        }
    }
}

template <typename R> static void vcycle(Ctx* c, MG& m, int l, int nu1, int nu2);

// Levels 1.. of the V-cycle as one HIP graph per precision: the coarse
// levels are many short launches, so replaying a captured graph removes most
// of their host launch cost.  All their kernel arguments are fixed (arenas,
// tables, and the active flags and dt read from device memory); with an even
// number of sweeps per cycle every double-buffered level ends the cycle in
// the buffer it started in.
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

// One V-cycle from level l in precision R for the active cavities.  A
// cavity whose coarsest level is l is solved there with the FP64 inverse of
// its dense matrix, after the level's smoothing for the other cavities (so
// its result sits in the buffer that is current when the level returns).
template <typename R>
static void vcycle(Ctx* c, MG& m, int l, int nu1, int nu2)
{
    using B = LB<R>;
    Level& L = m.L[l];
    if (l == 1 && c->graph && !m.capturing && !m.gfail[prec_index<R>()] && m.nlev > 2 && (nu1 + nu2) % 2 == 0) {
        coarse_graph<R>(c, m, nu1, nu2);
        return;
    }
    if (l == m.tail_lt) {
        if (m.op == HB_OP_VISC) launch_visc_tail<R>(c, m, l, nu1, nu2, m.tail_lds[prec_index<R>()], c->act);
        else if (m.op == HB_OP_MAC) launch_mac_tail<R>(c, m, l, nu1, nu2, m.tail_lds[prec_index<R>()], c->act);
        else launch_nodal_tail<R>(c, m, l, nu1, nu2, m.tail_lds[prec_index<R>()], c->act);
        return;
    }
    if (L.any_sm) {
        Level& C = m.L[l + 1];
        const BV v = smooth_view(c, L);
        // sweeps are paired into one launch only where each level then
        // swaps its buffers an even number of times per cycle, as the
        // captured graph of the coarse levels requires
        const bool pair = nu1 % 2 == 0 && nu2 % 2 == 0 && ((nu1 + nu2) / 2) % 2 == 0;
        const BV vpc = paired(v, C);                     // fine level, paired with the coarse one
        const BV vc = paired(all_view(c, C, c->act), L);  // coarse level, paired with the fine one
        // 2D (MAC and nodal problems; tensor problem with a staged smoother):
        // the residual restriction ends the last pre-smoothing launch
        const bool rfold = c->dim == 2 && c->fuse && nu1 > 0 && res_fold_ok(L, m.op) &&
                           (m.op != HB_OP_VISC || sweep2_shape(L.tile).staged);
        smooth<R>(c, m, l, nu1, pair, nullptr, rfold ? &C : nullptr);
        if (m.op == HB_OP_VISC) {
            if (!rfold)
                launch_tresid_restr<R>(c, L, vpc, C.gall, C.o, tcoef<R>(m, l), l == 0, B::x(L), B::b(L), B::b(C),
                                       B::x(C));
        } else if (m.op == HB_OP_MAC) {
            if (!rfold) launch_mac_resid_restrict<R>(c, C, vc, L.gall, L.o, B::x(L), B::b(L), B::b(C), B::x(C));
        } else if (!rfold) {
            launch_nodal_resid<R>(c, L, v, B::x(L), B::b(L), B::r(L), -1);
            launch_nodal_restrict<R>(c, C, vc, L.gall, L.o, B::r(L), B::b(C), B::x(C));
        }
        vcycle<R>(c, m, l + 1, nu1, nu2);
        // 2D (MAC and nodal problems; tensor problem with a staged smoother):
        // the prolongation is folded into the first post-smoothing launch
        const bool fold = c->dim == 2 && c->fuse && nu2 > 0 && (m.op != HB_OP_VISC || sweep2_shape(L.tile).staged);
        if (m.op == HB_OP_NODAL && !fold) launch_nodal_prolong<R>(c, L, vpc, C.gall, C.o, B::x(C), B::x(L));
        else if (m.op != HB_OP_NODAL && !fold)
            launch_prolong_cells<R>(c, L, vpc, C.gall, C.o, m.ncomp, m.op == HB_OP_VISC ? -1.0 : 1.0, B::x(C), B::x(L));
        smooth<R>(c, m, l, nu2, pair, fold ? &C : nullptr);
    }
    if (L.any_cs) launch_coarse_solve<R>(c, m, l, c->act, B::b(L), B::x(L));
}

// r = b - A x on level 0 (FP64) and its max-norm into each cavity's S_MAX
static void resid0(Ctx* c, MG& m, const double* x, const double* b, double* r, const int* act)
{
    // the residual kernels' final max pass writes S_MAX of every active
    // cavity (the only ones whose norm is read)
    const Level& L = m.L[0];
    const BV v = all_view(c, L, act);
    if (m.op == HB_OP_VISC) launch_tresid(c, L, v, m.etae, x, b, r, S_MAX);
    else if (m.op == HB_OP_MAC) launch_mac_resid(c, L, v, x, b, r, S_MAX);
    else launch_nodal_resid<double>(c, L, v, x, b, r, S_MAX);
}

static void apply0(Ctx* c, MG& m, const double* x, double* y)
{
    const Level& L = m.L[0];
    const BV v = all_view(c, L, c->act);
    if (m.op == HB_OP_VISC) launch_tresid(c, L, v, m.etae, x, nullptr, y, -1);
    else if (m.op == HB_OP_MAC) launch_mac_resid(c, L, v, x, nullptr, y, -1);
    else launch_nodal_resid<double>(c, L, v, x, nullptr, y, -1);
}

static SegV seg_of(const MG& m, const int* act) { return SegV{m.seg0.off, m.seg0.n, act}; }

// z = M^{-1} r: one V-cycle from zero on level 0, in FP64 or (lo) in FP32
static void precond(Ctx* c, MG& m, const double* r, double* z, int nu1, int nu2, bool lo)
{
    Level& L = m.L[0];
    const SegV sv = seg_of(m, c->act);
    L.cur = 0;
    if (lo) {
        seg_to_f32(c, sv, r, L.fb, L.fx[0]);
        vcycle<float>(c, m, 0, nu1, nu2);
        seg_from_f32(c, sv, LB<float>::x(L), z);
        return;
    }
    // the cycle runs on z as the first buffer of level 0 (zeroed), so it
    // ends there when the level swaps its buffers an even number of times
    double* sb = L.b;
    double* sx = L.xb[0];
    L.b = const_cast<double*>(r);
    L.xb[0] = z;
    // The 2D fused tensor sweep starts from zeros without reading z; every
    // other first launch reads it, so z is cleared for them.
    if (m.op == HB_OP_VISC && c->dim == 2 && c->fuse && nu1 > 0) m.zero0 = true;
    else seg_fill(c, sv, z, 0.0);
    vcycle<double>(c, m, 0, nu1, nu2);
    m.zero0 = false;
    if (L.cur != 0) seg_copy(c, sv, z, L.X());
    L.xb[0] = sx;
    L.b = sb;
}

// ---- the solve loop ----------------------------------------------------------
//
// Every convergence decision is taken on the device (k_conv, one small kernel
// per check point: after the first residual, after each V-cycle, after each
// BiCGStab half step), in the order a host-driven loop would take it, and the
// cycle kernels skip the cavities it has stopped.  The host only has to know
// when to stop launching: after queueing the work up to check point j + 1 it
// waits for the active count of check point j, so the GPU always has the
// next block of work queued while the host waits, and the block queued after
// the last active check point finds every cavity stopped.  The per-cavity
// outcome (|b|, cycles, relative residual, return code) stays in the
// operator's record slots until the host reads all slots once per step.

static double slot(const Ctx* c, int b, int s) { return c->hsc[(long)b * S_NSLOT + s]; }

struct ConvLoop {
    Ctx* c;
    ConvArgs a{};
    unsigned long long prev = 0, last = 0;
    ConvLoop(Ctx* cc, const MG& m, const hb_mg_opts& o) : c(cc)
    {
        a.nb = cc->nb;
        a.rec = m.rec;
        a.tol = o.tol_rel;
        a.max_cycles = o.max_cycles;
        a.fixed = o.fixed_cycles;
    }
    // a check point whose active count is published
    void check(int mode, int cur_sel = 0)
    {
        a.mode = mode;
        a.cur_sel = cur_sel;
        a.seq = ++c->cseq;
        launch_conv(c, a);
        prev = last;
        last = a.seq;
    }
    // the max-norm of the next residual is finished by the next check
    void defer() { c->defer_mf = true; }
    // a rule applied without publication
    void apply(int mode)
    {
        a.mode = mode;
        a.cur_sel = 0;
        a.seq = 0;
        launch_conv(c, a);
    }
    // true while the check point before the last one had active cavities
    bool lagged_active() const { return prev == 0 || wait_active(c, prev) != 0; }
};

// Multigrid (optionally BiCGStab-accelerated) solves A x = b of every cavity
// on the prepared level-0 systems; x, b are level-0 arenas.  Cavities stop
// independently.  With mixed precision every V-cycle runs in FP32 on the
// FP64 residual (defect correction, or the BiCGStab preconditioner);
// residuals, norms and the iterate stay FP64.  Requires CV_BEGIN.
static void solve_core(Ctx* c, MG& m, double* x, double* b, const hb_mg_opts& o)
{
    Level& L = m.L[0];
    const bool lo = o.precision == HB_PREC_MIXED;
    const SegV sv = seg_of(m, c->act);
    ConvLoop cl(c, m, o);
    if (!o.krylov) {
        // Plain V-cycles.  FP64: on the level's double buffer seeded with x.
        // Mixed: x in the first FP64 buffer; each cycle corrects it by one
        // FP32 V-cycle on A e = r.
        L.cur = 0;
        double* xw = L.xb[0];
        seg_copy(c, sv, xw, x);
        cl.defer();
        resid0(c, m, xw, b, L.r, c->act);
        cl.check(CV_INIT, 0);
        for (int k = 0; k < o.max_cycles; ++k) {
            if (lo) {
                L.cur = 0;
                seg_to_f32(c, sv, L.r, L.fb, L.fx[0]);
                vcycle<float>(c, m, 0, o.nu1, o.nu2);
                seg_add_f32(c, sv, xw, LB<float>::x(L));
                cl.defer();
                resid0(c, m, xw, b, L.r, c->act);
            } else {
                vcycle<double>(c, m, 0, o.nu1, o.nu2);
                cl.defer();
                resid0(c, m, L.X(), b, L.r, c->act);
            }
            cl.check(CV_CYCLE, lo ? 0 : L.cur);
            if (!cl.lagged_active()) break;
        }
        // copy out each cavity's iterate from the buffer it ended in
        cl.apply(CV_END_PLAIN);
        seg_copy_sel(c, seg_of(m, c->act2), x, L.xb[0], L.xb[1], c->sel);
        return;
    }

    // BiCGStab with its scalars kept on the device, per cavity
    double *r = c->kr, *rh = c->krh, *p = c->kp, *v = c->kv, *ph = c->kph, *s = c->ks, *sh = c->ksh, *t = c->kt;
    resid0(c, m, x, b, r, c->act);
    seg_copy(c, sv, rh, r);
    seg_fill(c, sv, p, 0.0);
    seg_fill(c, sv, v, 0.0);
    bicg_init_scalars(c, c->act);
    cl.check(CV_INIT, 0);
    // Each dot product is a partial pass whose total the kernel that needs
    // the scalar takes itself; rho's partials after the first come from the
    // update of r.
    double* rp = rho_partials(c);
    seg_dot_part(c, sv, rh, r, nullptr, rp, -1);
    // a cavity may take one V-cycle past max_cycles (its last half step)
    for (int k = 0; k < o.max_cycles + 1; k += 2) {
        bicg_p_rho(c, sv, p, r, v, rp);   // rho, beta; p = r + beta (p - omega v)
        precond(c, m, p, ph, o.nu1, o.nu2, lo);
        apply0(c, m, ph, v);
        seg_dot_part(c, sv, rh, v, nullptr, c->partial, S_MAX);   // r^.v; S_MAX cleared for the max of s
        bicg_s_alpha(c, sv, s, r, v, c->partial, S_MAX);           // alpha; s = r - alpha v
        cl.check(CV_HALF);
        // cavities that finish at the half step: x += alpha ph, r = s
        bicg_half_finish(c, seg_of(m, c->act2), x, ph, r, s);
        if (!cl.lagged_active()) break;
        precond(c, m, s, sh, o.nu1, o.nu2, lo);
        apply0(c, m, sh, t);
        seg_dot_part(c, sv, t, t, s, c->partial, S_MAX);   // t.t, t.s; S_MAX cleared for the max of r
        // omega; x += alpha ph + omega sh, r = s - omega t, the next rho's partials
        bicg_full_update(c, sv, x, ph, sh, r, s, t, S_MAX, c->partial, rh, rp);
        cl.check(CV_FULL);
        if (!cl.lagged_active()) break;
    }
    // the true residual of every solved cavity
    cl.apply(CV_END_KRYLOV);
    cl.defer();
    resid0(c, m, x, b, L.r, c->act);
    cl.apply(CV_FINAL);
}

// Start of a nodal solve of a single-cavity context: record the initial
// residual and guess for training data, and replace the guess x0 by the
// network's x0 + s y when that lowers the residual (learned warm start).
static void nodal_prestart(Ctx* c, MG& m, double* x)
{
    Level& L = m.L[0];
    const long n = L.nu;
    const GridD& g = c->cv[0].g;
    resid0(c, m, x, m.lvl0_b, L.r, nullptr);
    fetch_slots(c);
    const double s0 = slot(c, 0, S_MAX);
    if (c->cap) {
        copy(c, c->cap_r0, L.r, n);
        copy(c, c->cap_x0, x, n);
    }
    if (!c->ws || !(s0 > 0.0) || !std::isfinite(s0)) return;
    launch_node_to_cell(c, g, L.r, 1.0 / s0, c->ws_in);
    if (hipStreamSynchronize(c->s) != hipSuccess) return;
    if (nn_infer(c->ws, c->ws_in, 1, g.n[1], g.n[0], c->ws_out) != HB_OK) return;
    launch_cell_to_node(c, g, c->ws_out, c->ws_y);
    // least-squares scale of the network's shape: min_s |r0 - s K y|_2
    launch_nodal_resid<double>(c, L, all_view(c, L, nullptr), c->ws_y, nullptr, c->ws_z, -1);
    const SegV sv = seg_of(m, nullptr);
    seg_dot(c, sv, L.r, c->ws_z, S_DOT0);
    seg_dot(c, sv, c->ws_z, c->ws_z, S_DOT1);
    fetch_slots(c);
    const double zz = slot(c, 0, S_DOT1);
    if (!(zz > 0.0) || !std::isfinite(zz)) return;
    const double sc = slot(c, 0, S_DOT0) / zz;
    launch_axpy(c, c->ws_x1, x, c->ws_y, sc, n);
    resid0(c, m, c->ws_x1, m.lvl0_b, L.r, nullptr);
    fetch_slots(c);
    const double s1 = slot(c, 0, S_MAX);
    if (s1 < s0) {   // the residual check decides; otherwise keep x0
        copy(c, x, c->ws_x1, n);
        ++c->ws_report_used;
    }
}

// Solve with the right-hand sides already in m.lvl0_b (VISC: wall part
// added; NODAL/MAC: mean removed by this function).  x: level-0 arena.  The
// outcome stays on the device (solve_outcome reads it).
static void solve_prepared(Ctx* c, MG& m, double* x, const hb_mg_opts& o)
{
    if (m.op == HB_OP_VISC) join_visc_factor(c);
    const SegV all = seg_of(m, nullptr);
    if (m.op != HB_OP_VISC) seg_sub_mean(c, all, m.lvl0_b);
    if (m.op == HB_OP_NODAL && (c->ws || c->cap)) nodal_prestart(c, m, x);
    if (m.op == HB_OP_VISC && c->capv) {
        // training data / analysis: initial residual and guess of the solve
        resid0(c, m, x, m.lvl0_b, m.L[0].r, nullptr);
        copy(c, c->capv_r0, m.L[0].r, m.L[0].nu);
        copy(c, c->capv_x0, x, m.L[0].nu);
    }
    seg_maxabs2(c, all, m.lvl0_b, S_MAX, x, S_MAX2);
    if (o.precision == HB_PREC_MIXED) ensure_f32(c, m);
    ConvLoop(c, m, o).apply(CV_BEGIN);
    // cavities with b = 0 have x = 0
    seg_fill(c, seg_of(m, c->act2), x, 0.0);
    solve_core(c, m, x, m.lvl0_b, o);
    if (m.op != HB_OP_VISC) seg_sub_mean(c, all, x);
    if (m.op == HB_OP_NODAL && c->cap) launch_axpy(c, c->cap_e, x, c->cap_x0, -1.0, m.L[0].nu);
    if (m.op == HB_OP_VISC && c->capv) launch_axpy(c, c->capv_e, x, c->capv_x0, -1.0, m.L[0].nu);
}

// The outcome of the last solve of m per cavity, from the slots a
// fetch_slots has brought to the host, and the worst return code.
static int solve_outcome(Ctx* c, const MG& m, std::vector<hb_mg_report>* rep)
{
    int rc = HB_OK;
    for (int b = 0; b < c->nb; ++b) {
        const double* R = c->hsc + (long)b * S_NSLOT + m.rec;
        const int src = (int)R[R_RC];
        if (rep) {
            (*rep)[b].cycles = (int)R[R_CYC];
            (*rep)[b].rel_resid = R[R_REL];
            (*rep)[b].bnorm = R[R_BN];
        }
        if (src == HB_ERR_NONFINITE) rc = HB_ERR_NONFINITE;
        else if (src == HB_ERR_NOCONV && rc == HB_OK) rc = HB_ERR_NOCONV;
    }
    if (rc == HB_ERR_NOCONV) c->err = "multigrid did not reach the tolerance within max_cycles";
    if (rc == HB_ERR_NONFINITE) c->err = "non-finite right-hand side, guess or residual in a multigrid solve";
    return rc;
}

static bool valid_opts(const hb_mg_opts& o)
{
    return o.max_cycles >= 0 && o.max_cycles <= 100000 && o.nu1 >= 0 && o.nu2 >= 0 && o.nu1 + o.nu2 > 0 &&
           o.tol_rel >= 0.0 && (o.precision == HB_PREC_FP64 || o.precision == HB_PREC_MIXED);
}

static int worse(int rc, int cur)
{
    if (cur == HB_OK) return rc;
    if (cur == HB_ERR_NOCONV && rc != HB_OK) return rc;
    return cur;
}

// ---------------------------------------------------------------------------
// stages of the step (per cavity around the batched solves)
// ---------------------------------------------------------------------------

// the Godunov prediction of every cavity up to the MAC divergence (into
// the MAC right-hand sides); requires visc_setup, the per-call table and
// S_MAXU = max|u|
static void advect_predict(Ctx* c)
{
    stage_visc_div(c);
    stage_grad_node(c);
    stage_forcing(c);
    stage_slopes(c);
    stage_trace_normal(c);
    stage_transverse(c);
    stage_trace_full(c);
    if (c->opts.mac_project) stage_mac_div(c, 0);
}

// MAC projection of every cavity's face velocity, then each cavity's
// viscous right-hand side into CavIO::b (and CavIO::conv when set); with
// div_rel, the MAC divergence after the projection relative to before it
// (host reads)
static void advect_finish(Ctx* c, std::vector<double>* div_rel)
{
    const int nb = c->nb;
    std::vector<double> d0(nb, 0.0);
    if (c->opts.mac_project) {
        if (div_rel) {
            seg_maxabs(c, seg_of(c->mac, nullptr), c->mac.lvl0_b, S_MAX);
            fetch_slots(c);
            for (int b = 0; b < nb; ++b) d0[b] = slot(c, b, S_MAX);
        }
        fill(c, c->macphi, 0.0, c->mac.L[0].nu);
        solve_prepared(c, c->mac, c->macphi, c->opts.mac);
        stage_mac_update(c);
        if (div_rel) {
            stage_mac_div(c, 1);
            stage_maxabs(c, SF_MACRHS, S_MAX);
            fetch_slots(c);
            for (int b = 0; b < nb; ++b) (*div_rel)[b] = d0[b] > 0.0 ? slot(c, b, S_MAX) / d0[b] : 0.0;
        }
    } else {
        for (int b = 0; b < nb; ++b) {
            copy(c, c->cv[b].umac, c->cv[b].uadv, c->cv[b].nf);
            if (div_rel) (*div_rel)[b] = 0.0;
        }
    }
    stage_advect_rhs(c);
}

// outcome of the step's MAC solve (zero reports when it does not run)
static int mac_outcome(Ctx* c, std::vector<hb_mg_report>* rep)
{
    if (c->opts.mac_project) return solve_outcome(c, c->mac, rep);
    if (rep)
        for (auto& r : *rep) memset(&r, 0, sizeof(r));
    return HB_OK;
}

// projection of every cavity (per-call table: ustar, p, uout, dt):
// V = ustar/dt + G p, K phi = weak div V, uout = ustar + dt (G p - G phi),
// p = phi
static void project_all(Ctx* c)
{
    stage_grad_node(c);
    stage_proj_rhs(c);
    stage_copy(c, SF_PHI, SF_P);
    solve_prepared(c, c->nodal, c->phi, c->opts.proj);
    stage_proj_update(c);
    stage_copy(c, SF_P, SF_PHI);
}

// One full step of every cavity in place.  dt[b] <= 0 selects the CFL time
// step of cavity b.
static int step_all(Ctx* c, double* const* u, double* const* p, const double* dt_in, hb_step_report* reports)
{
    const int nb = c->nb;
    std::vector<CavIO> io(nb, io_zero());
    for (int b = 0; b < nb; ++b) {
        io[b].u = u[b];
        io[b].p = p[b];
    }
    set_io(c, io);
    stage_maxabs(c, SF_U, S_MAXU);
    stage_maxabs(c, SF_P, S_MAX2);
    fetch_slots(c);
    std::vector<double> dt(nb);
    for (int b = 0; b < nb; ++b) {
        const Cav& v = c->cv[b];
        if (!std::isfinite(slot(c, b, S_MAXU)) || !std::isfinite(slot(c, b, S_MAX2)))
            return fail(c, HB_ERR_NONFINITE, "non-finite u or p");
        dt[b] = dt_in ? dt_in[b] : 0.0;
        if (!(dt[b] > 0.0)) {
            const double mu = std::fmax(v.ulid, slot(c, b, S_MAXU));
            if (!(mu > 0.0)) return fail(c, HB_ERR_ARG, "dt <= 0 with zero velocity everywhere");
            dt[b] = c->opts.cfl * v.g.h / mu;
        }
    }
    std::vector<hb_mg_report> mrep(nb), vrep(nb), prep(nb);
    std::vector<double> divr(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
        Cav& v = c->cv[b];
        io[b].eta = v.eta;
        io[b].b = v.rhs;
        io[b].conv = nullptr;
        io[b].ustar = v.ustar;
        io[b].uout = u[b];
        io[b].dt = dt[b];
        // the solve's operator is I - 2 theta dt div(eta/Re gamma_dot(.))
        io[b].vdt = 2.0 * c->opts.theta * dt[b];
        v.step_dt = dt[b];
    }
    set_io(c, io);
    stage_viscosity(c);
    visc_setup(c);
    factor_visc_async(c);
    advect_predict(c);
    advect_finish(c, reports ? &divr : nullptr);
    stage_visc_wall_rhs(c);
    stage_copy(c, SF_USTAR, SF_U);
    solve_prepared(c, c->visc, c->ustar, c->opts.visc);
    project_all(c);
    if (reports) {
        stage_maxabs(c, SF_UOUT, S_MAX);
        stage_weak_div_u(c);
        stage_maxabs(c, SF_RNODE, S_MAX2);
    }
    // the one read of the step's outcome: the solves' records (and the
    // diagnostics of a report)
    fetch_slots(c);
    int rc = mac_outcome(c, &mrep);
    rc = worse(solve_outcome(c, c->visc, &vrep), rc);
    rc = worse(solve_outcome(c, c->nodal, &prep), rc);
    if (reports) {
        for (int b = 0; b < nb; ++b) {
            hb_step_report& R = reports[b];
            memset(&R, 0, sizeof(R));
            R.dt = dt[b];
            R.max_u = slot(c, b, S_MAX);
            R.div_node = slot(c, b, S_MAX2) / std::pow(c->cv[b].g.h, c->dim);
            R.div_mac_rel = divr[b];
            R.mac = mrep[b];
            R.visc = vrep[b];
            R.proj = prep[b];
        }
    }
    if (hipGetLastError() != hipSuccess) return fail(c, HB_ERR_DEVICE, "kernel launch failed");
    return rc;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

void kt_pair(Ctx* c, hipEvent_t* start, hipEvent_t* stop, double bytes)
{
    KTimer& k = c->ktm;
    if (k.n == k.cap) kt_harvest(c);
    *start = k.ev[2 * k.n];
    *stop = k.ev[2 * k.n + 1];
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

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------

const char* check_grid(const hb_grid* grid)
{
    if (grid->dim != 2 && grid->dim != 3) return "dim must be 2 or 3";
    for (int a = 0; a < grid->dim; ++a) {
        if (!valid_extent(grid->n[a])) return "each n[a] must be c*2^k, c in {1,2,3}, n >= 4";
        if (grid->bc[a][0] != grid->bc[a][1] && (grid->bc[a][0] == HB_BC_PERIODIC || grid->bc[a][1] == HB_BC_PERIODIC))
            return "periodic faces must come in pairs";
        for (int s = 0; s < 2; ++s)
            if (grid->bc[a][s] != HB_BC_WALL && grid->bc[a][s] != HB_BC_PERIODIC) return "unknown boundary type";
    }
    if (!(grid->h > 0.0) || !std::isfinite(grid->h)) return "h must be positive";
    return nullptr;
}

static const char* check_fluid(const hb_fluid* fluid)
{
    if (!(fluid->Re > 0.0) || !(fluid->Pa > 0.0) || !(fluid->n > 0.0) || !(fluid->HB >= 0.0))
        return "need Re > 0, Pa > 0, n > 0, HB >= 0";
    if (fluid->reg != HB_REG_PAPER && fluid->reg != HB_REG_YIELD_ONLY) return "unknown regularisation";
    if (fluid->reg == HB_REG_YIELD_ONLY && fluid->n < 1.0) return "yield-only regularisation needs n >= 1";
    return nullptr;
}

static void destroy_ctx(Ctx* c);

// True when every periodic extent of the level's grids is at least the halo
// of a launch that runs two tensor sweeps.
static bool level_pairs(const Level& L)
{
    for (const GridD& g : L.hg)
        for (int a = 0; a < g.dim; ++a)
            if (g.per[a] && g.n[a] < 8) return false;
    return true;
}

// Tile autotuning.  For every level of the nodal problem (and, in 2D, of
// the tensor problem) on which a fused sweep runs, each candidate is timed
// on the level's own arenas and the fastest is kept.  The unit timed is two
// sweeps: two launches of one sweep, or one launch where the candidate runs
// two sweeps in one and the level allows it.  After a warm-up unit per
// candidate, kRounds rounds time one unit of every candidate in turn (an
// event pair per unit), and a candidate's time is its minimum, so one slow
// sample does not decide; a candidate replaces an earlier one only when more
// than 2% faster.  The candidates compute the same values bit for
// bit, so the choice changes only the speed.  HB_TILE=k in the environment
// forces candidate k instead (modulo the problem's candidate count).
static void autotune(Ctx* c)
{
    if (!c->fuse) return;
    const char* e = std::getenv("HB_TILE");
    const int forced = (e && e[0] >= '0' && e[0] <= '9') ? std::atoi(e) : -1;
    constexpr int kRounds = 6;
    constexpr int kMaxCands = kSweep2Cands > kNodalCands ? kSweep2Cands : kNodalCands;
    hipEvent_t ev[2 * kRounds * kMaxCands] = {};
    if (forced < 0)
        for (hipEvent_t& x : ev)
            if (hipEventCreate(&x) != hipSuccess) return;
    MG* ms[2] = {&c->visc, &c->nodal};
    for (MG* m : ms) {
        const bool visc = m->op == HB_OP_VISC;
        if (visc && c->dim != 2) continue;
        const int nc = visc ? kSweep2Cands : kNodalCands;
        for (int l = 0; l < m->nlev; ++l) {
            Level& L = m->L[l];
            if (!L.any_sm || (m->tail_lt >= 0 && l >= m->tail_lt)) continue;
            // sweeps per launch of each candidate on this level, and whether
            // it fits the LDS at all
            int nsw[kMaxCands];
            bool usable[kMaxCands];
            for (int k = 0; k < nc; ++k) {
                nsw[k] = 1;
                usable[k] = true;
                if (!visc) {
                    if (c->dim == 2 && level_pairs(L)) nsw[k] = 2;
                    continue;
                }
                if (sweep2_shape(k).nsw >= 2 && level_pairs(L) && sweep2_lds(k, 2) <= c->lds_budget) nsw[k] = 2;
                usable[k] = sweep2_lds(k, 1) <= c->lds_budget;
            }
            if (forced >= 0) {
                L.tile = usable[forced % nc] ? forced % nc : 0;
                L.sweeps = nsw[L.tile];
                continue;
            }
            BV v{L.gsm, L.o, L.of, nullptr, 1};
            if (c->nb == 1) {
                v.one = 1;
                v.g1 = L.hg[0];
            }
            auto unit = [&](int k) {
                if (visc && nsw[k] == 2) {
                    launch_tsweep2<double>(c, L, v, tcoef<double>(*m, l), l == 0, L.xb[0], L.xb[1], L.b, k, 2);
                } else if (visc) {
                    launch_tsweep2<double>(c, L, v, tcoef<double>(*m, l), l == 0, L.xb[0], L.xb[1], L.b, k, 1);
                    launch_tsweep2<double>(c, L, v, tcoef<double>(*m, l), l == 0, L.xb[1], L.xb[0], L.b, k, 1);
                } else if (nsw[k] == 2) {
                    launch_nodal_sweep<double>(c, L, v, L.xb[0], L.xb[1], L.b, k, 2);
                } else {
                    launch_nodal_sweep<double>(c, L, v, L.xb[0], L.xb[1], L.b, k);
                    launch_nodal_sweep<double>(c, L, v, L.xb[1], L.xb[0], L.b, k);
                }
            };
            for (int k = 0; k < nc; ++k)
                if (usable[k]) unit(k);
            for (int r = 0; r < kRounds; ++r)
                for (int k = 0; k < nc; ++k) {
                    hipEvent_t* p = ev + 2 * (r * nc + k);
                    (void)hipEventRecord(p[0], c->s);
                    if (usable[k]) unit(k);
                    (void)hipEventRecord(p[1], c->s);
                }
            if (hipEventSynchronize(ev[2 * kRounds * nc - 1]) != hipSuccess) continue;
            float best = 0.0f;
            bool have = false;
            for (int k = 0; k < nc; ++k) {
                if (!usable[k]) continue;
                float tk = 0.0f;
                for (int r = 0; r < kRounds; ++r) {
                    const hipEvent_t* p = ev + 2 * (r * nc + k);
                    float t = 0.0f;
                    if (hipEventElapsedTime(&t, p[0], p[1]) != hipSuccess) t = 1e30f;
                    tk = r == 0 ? t : (t < tk ? t : tk);
                }
                // a later candidate must be more than 2% faster to replace the
                // best so far, so near-ties resolve the same way run to run
                if (!have || tk < 0.98f * best) {
                    best = tk;
                    have = true;
                    L.tile = k;
                    L.sweeps = nsw[k];
                }
            }
        }
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
}

// The stage kernels' tables: per cavity its grid, fluid and buffers, the
// face-viscosity restrictions per level, and the largest extents over the
// cavities (launch grids), checked against the device's grid limit.
static int build_stage_tables(Ctx* c)
{
    const int nb = c->nb;
    std::vector<CavK> ck(nb);
    int cx[3] = {1, 1, 1}, fx[3] = {1, 1, 1}, nx[3] = {1, 1, 1};
    for (int b = 0; b < nb; ++b) {
        const Cav& v = c->cv[b];
        CavK& K = ck[b];
        memset(&K, 0, sizeof(K));
        K.g = v.g;
        K.fl = v.fl;
        K.ulid = v.ulid;
        K.nc = v.nc;
        K.nf = v.nf;
        K.nn = v.nn;
        K.sc = v.sc;
        K.eta = v.eta;
        K.E = v.E;
        K.Gp = v.Gp;
        K.F = v.F;
        K.S = v.S;
        K.trans = v.trans;
        K.uhat = v.uhat;
        K.qhat = v.qhat;
        K.qLf = v.qLf;
        K.qRf = v.qRf;
        K.uadv = v.uadv;
        K.umac = v.umac;
        K.macrhs = v.macrhs;
        K.rnode = v.rnode;
        K.rhs = v.rhs;
        K.ustar = v.ustar;
        K.phi = v.phi;
        K.macphi = v.macphi;
        K.beta0 = c->visc.L[0].beta + c->visc.L[0].hof[b];
        K.etae = c->visc.etae + c->visc.L[0].ho[b];
        K.macb = c->mac.lvl0_b + c->mac.L[0].ho[b];
        K.nodb = c->nodal.lvl0_b + c->nodal.L[0].ho[b];
        K.viscb = c->visc.lvl0_b + c->visc.L[0].hou[b];
        for (int e = 0; e < 3; ++e) {
            cx[e] = std::max(cx[e], v.g.n[e]);
            nx[e] = std::max(nx[e], nnode(v.g, e));
            for (int a = 0; a < v.g.dim; ++a) fx[e] = std::max(fx[e], fext(v.g, a, e));
        }
    }
    const MG& m = c->visc;
    std::vector<RFace> rf((size_t)std::max(m.nlev - 1, 1) * nb);
    c->rfx.assign(m.nlev, {1, 1, 1});
    for (int l = 1; l < m.nlev; ++l)
        for (int b = 0; b < nb; ++b) {
            RFace& R = rf[(size_t)(l - 1) * nb + b];
            memset(&R, 0, sizeof(R));
            if (m.nlevc[b] <= l) continue;
            R.gf = m.L[l - 1].hg[b];
            R.gc = m.L[l].hg[b];
            R.bf = m.L[l - 1].beta + m.L[l - 1].hof[b];
            R.bc = m.L[l].beta + m.L[l].hof[b];
            for (int e = 0; e < 3; ++e)
                for (int a = 0; a < R.gc.dim; ++a) c->rfx[l][e] = std::max(c->rfx[l][e], fext(R.gc, a, e));
        }
    int dev = 0, zmax = 65535;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&zmax, hipDeviceAttributeMaxGridDimZ, dev);
    const long zneed = (long)nb * std::max({(long)cx[2], (long)nx[2], 3L * fx[2], 2L * c->dim});
    if (zneed > zmax) return HB_ERR_ARG;
    memcpy(c->cx, cx, sizeof(cx));
    memcpy(c->fx, fx, sizeof(fx));
    memcpy(c->nx, nx, sizeof(nx));
    if (dalloc(&c->ck, nb) != hipSuccess || upload(c->ck, ck) != hipSuccess) return HB_ERR_OOM;
    if (dalloc(&c->rface, (long)rf.size()) != hipSuccess || upload(c->rface, rf) != hipSuccess) return HB_ERR_OOM;
    if (dalloc(&c->cio, nb) != hipSuccess) return HB_ERR_OOM;
    if (hipHostMalloc((void**)&c->hio, sizeof(CavIO) * 2 * nb, 0) != hipSuccess) {
        c->hio = nullptr;
        return HB_ERR_OOM;
    }
    memset(c->hio, 0, sizeof(CavIO) * 2 * nb);
    return HB_OK;
}

static int create_ctx(const hb_grid* grids, const hb_fluid* fluids, int count, const hb_step_opts* opts,
                      void* hip_stream, Ctx** out)
{
    if (out) *out = nullptr;
    auto bad = [](const char* m) { g_create_err = m; return HB_ERR_ARG; };
    if (!grids || !fluids || !opts || !out) return bad("null argument");
    if (count < 1 || count > 4096) return bad("batch size must be 1 .. 4096");
    for (int b = 0; b < count; ++b) {
        if (const char* e = check_grid(&grids[b])) return bad(e);
        if (const char* e = check_fluid(&fluids[b])) return bad(e);
        if (grids[b].dim != grids[0].dim) return bad("all cavities of a batch need the same dim");
    }
    if (!valid_opts(opts->mac) || !valid_opts(opts->visc) || !valid_opts(opts->proj)) return bad("invalid multigrid options");
    if (!(opts->cfl > 0.0)) return bad("cfl must be positive");
    if (!(opts->theta == 0.0 || (opts->theta >= 0.5 && opts->theta <= 1.0))) return bad("theta must be 0 or in [0.5, 1]");
    if (opts->pred_visc != 0 && opts->pred_visc != 1) return bad("pred_visc must be 0 or 1");

    Ctx* c = new (std::nothrow) ::hb_ctx();
    if (!c) return bad("out of host memory");
    c->opts = *opts;
    if (c->opts.theta == 0.0) c->opts.theta = 0.5;
    c->user = (hipStream_t)hip_stream;
    c->nb = count;
    c->dim = grids[0].dim;
    auto give_up = [&](int code, const std::string& m) {
        g_create_err = m;
        destroy_ctx(c);
        return code;
    };
    if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_f0, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_f1, hipEventDisableTiming) != hipSuccess)
        return give_up(HB_ERR_DEVICE, "stream or event creation failed");
    // the slot mirror and its publication word are coherent pinned memory
    // the device writes directly (fetch_slots)
    const unsigned pin = hipHostMallocMapped | hipHostMallocCoherent;
    bool ok = dalloc(&c->sc, (long)S_NSLOT * count) == hipSuccess &&
              hipHostMalloc((void**)&c->hsc, sizeof(double) * S_NSLOT * count, pin) == hipSuccess &&
              hipHostMalloc((void**)&c->hseq, sizeof(unsigned long long), pin) == hipSuccess &&
              hipHostMalloc((void**)&c->hring, sizeof(unsigned long long) * kRing, pin) == hipSuccess &&
              hipHostGetDevicePointer((void**)&c->dring, c->hring, 0) == hipSuccess &&
              hipHostGetDevicePointer((void**)&c->dhsc, c->hsc, 0) == hipSuccess &&
              hipHostGetDevicePointer((void**)&c->dhseq, c->hseq, 0) == hipSuccess &&
              dalloc(&c->partial, 3L * kRedBlocks * count) == hipSuccess && dalloc(&c->act, count) == hipSuccess &&
              dalloc(&c->mpart, (long)kSubMax * count) == hipSuccess &&
              hipMemsetAsync(c->mpart, 0, sizeof(unsigned long long) * kSubMax * count, c->s) == hipSuccess &&
              dalloc(&c->act2, count) == hipSuccess && dalloc(&c->sel, count) == hipSuccess &&
              hipHostMalloc((void**)&c->hact, sizeof(int) * count) == hipSuccess &&
              hipHostMalloc((void**)&c->hact2, sizeof(int) * count) == hipSuccess &&
              hipHostMalloc((void**)&c->hsel, sizeof(int) * count) == hipSuccess;
    if (!ok) return give_up(HB_ERR_OOM, "device allocation failed");
    memset(c->hsc, 0, sizeof(double) * S_NSLOT * count);
    *c->hseq = 0;
    for (int i = 0; i < kRing; ++i) c->hring[i] = ~0ull;
    c->cv.resize(count);
    for (int b = 0; b < count; ++b) {
        Cav& v = c->cv[b];
        v.grid = grids[b];
        v.fluid = fluids[b];
        v.g = make_gridd(grids[b]);
        v.fl.Re = fluids[b].Re;
        v.fl.HB = fluids[b].HB;
        v.fl.n = fluids[b].n;
        v.fl.Pa = fluids[b].Pa;
        v.fl.reg = fluids[b].reg;
        for (int q = 0; q < 3; ++q) v.fl.f[q] = q < grids[b].dim ? fluids[b].f[q] : 0.0;
        v.dim = grids[b].dim;
        v.nc = ncells(v.g);
        v.nn = nnodes(v.g);
        v.nf = nface_total(v.g);
        v.ulid = 0.0;
        for (int a = 0; a < v.dim; ++a)
            for (int s = 0; s < 2; ++s)
                for (int q = 0; q < 3; ++q) v.ulid = std::fmax(v.ulid, std::fabs(v.g.wall_u[a][s][q]));
        v.sc = c->sc + (long)b * S_NSLOT;
        v.hsc = c->hsc + (long)b * S_NSLOT;
    }
    // dynamic LDS a workgroup may take (coarse tail, staged sweeps): the
    // device's per-workgroup limit less the kernels' static arrays; HB_TAIL=0
    // in the environment turns the tail off (every level then runs its own
    // launches)
    {
        int dev = 0, lim = 0;
        const char* e = std::getenv("HB_TAIL");
        c->tail = !(e && e[0] == '0');
        // HB_FUSE=0: one launch per colour in the nodal and MAC smoothers
        // and per component in the 2D tensor smoother
        const char* f = std::getenv("HB_FUSE");
        c->fuse = !(f && f[0] == '0');
        // HB_FINE3=k selects the finest 3D tensor smoother (experiment switch)
        const char* f3 = std::getenv("HB_FINE3");
        c->fine3 = f3 ? std::atoi(f3) : 0;
        // HB_GRAPH=1: the coarse levels of a V-cycle are replayed as one
        // captured graph instead of launched one by one.  Off by default: the
        // host issues a step's launches without waiting on the device, so it
        // stays ahead of the queue, and a graph replay costs the device more
        // time than the same kernels launched directly.
        const char* gr = std::getenv("HB_GRAPH");
        c->graph = gr && gr[0] == '1';
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lim > 8192) {
            c->lds_budget = (size_t)lim - 4096;
            tail_allow_lds(c->lds_budget);
            sweep2_allow_lds(c->lds_budget);
            tsmooth_allow_lds(c->lds_budget);
        }
    }
    int rc;
    if ((rc = build_mg(c, c->visc, HB_OP_VISC)) != HB_OK) return give_up(rc, c->err);
    if ((rc = build_mg(c, c->mac, HB_OP_MAC)) != HB_OK) return give_up(rc, c->err);
    if ((rc = build_mg(c, c->nodal, HB_OP_NODAL)) != HB_OK) return give_up(rc, c->err);
    const long nvt = c->visc.L[0].nu;
    ok = dalloc(&c->macphi, c->mac.L[0].nu) == hipSuccess && dalloc(&c->ustar, nvt) == hipSuccess &&
         dalloc(&c->phi, c->nodal.L[0].nu) == hipSuccess;
    ok = ok && dalloc(&c->kr, nvt) == hipSuccess && dalloc(&c->krh, nvt) == hipSuccess && dalloc(&c->kp, nvt) == hipSuccess &&
         dalloc(&c->kv, nvt) == hipSuccess && dalloc(&c->kph, nvt) == hipSuccess && dalloc(&c->ks, nvt) == hipSuccess &&
         dalloc(&c->ksh, nvt) == hipSuccess && dalloc(&c->kt, nvt) == hipSuccess;
    for (int b = 0; ok && b < count; ++b) {
        Cav& v = c->cv[b];
        const long d = v.dim, nc = v.nc, nf = v.nf, nn = v.nn, nv = d * nc;
        ok = ok && dalloc(&v.eta, nc) == hipSuccess && dalloc(&v.E, nv) == hipSuccess && dalloc(&v.Gp, nv) == hipSuccess;
        ok = ok && dalloc(&v.F, nv) == hipSuccess && dalloc(&v.S, d * d * nc) == hipSuccess &&
             dalloc(&v.trans, d * d * nc) == hipSuccess;
        ok = ok && dalloc(&v.uhat, nf) == hipSuccess && dalloc(&v.qhat, d * nf) == hipSuccess &&
             dalloc(&v.qLf, d * nf) == hipSuccess && dalloc(&v.qRf, d * nf) == hipSuccess;
        ok = ok && dalloc(&v.uadv, nf) == hipSuccess && dalloc(&v.umac, nf) == hipSuccess &&
             dalloc(&v.macrhs, nc) == hipSuccess && dalloc(&v.rnode, nn) == hipSuccess &&
             dalloc(&v.conv, nv) == hipSuccess && dalloc(&v.rhs, nv) == hipSuccess;
        const int nmax = std::max(c->visc.hcs[b].N, std::max(c->mac.hcs[b].N, c->nodal.hcs[b].N));
        ok = ok && dalloc(&v.dense_E, (long)nmax * nmax) == hipSuccess;
        v.macphi = c->macphi + c->mac.L[0].ho[b];
        v.ustar = c->ustar + c->visc.L[0].hou[b];
        v.phi = c->phi + c->nodal.L[0].ho[b];
    }
    if (!ok) return give_up(HB_ERR_OOM, "device allocation failed");
    fill(c, c->sc, 0.0, (long)S_NSLOT * count);
    // constant coarsest matrices of the MAC and nodal problems
    for (int b = 0; b < count; ++b) {
        factor_coarsest(c, c->mac, b);
        factor_coarsest(c, c->nodal, b);
    }
    // the tensor problem's per-step assembly: per-cavity table and unit
    // vectors (the MAC and nodal assemblies above used them first)
    {
        MG& m = c->visc;
        std::vector<DenseD> dd(count);
        for (int b = 0; b < count; ++b) {
            const CoarseD& d = m.hcs[b];
            const Level& C = m.L[d.lev];
            dd[b].g = C.hg[b];
            dd[b].beta = C.beta + C.hof[b];
            dd[b].aoff = d.aoff;
            dd[b].N = d.N;
            dd[b].E = c->cv[b].dense_E;
            launch_identity(c, d.N, c->cv[b].dense_E);
        }
        if (dalloc(&m.dd, count) != hipSuccess || upload(m.dd, dd) != hipSuccess)
            return give_up(HB_ERR_OOM, "device allocation failed");
    }
    {
        const int rc2 = build_stage_tables(c);
        if (rc2 != HB_OK) return give_up(rc2, rc2 == HB_ERR_OOM ? "device allocation failed"
                                                               : "batch too large for the stage launch grid");
    }
    autotune(c);
    if (hipStreamSynchronize(c->s) != hipSuccess) return give_up(HB_ERR_DEVICE, "stream synchronisation failed during set-up");
    *out = c;
    return HB_OK;
}

static void destroy_ctx(Ctx* c)
{
    if (!c) return;
    if (const char* st = std::getenv("HB_STATS"))
        if (st[0] == '1') fprintf(stderr, "[hb] host waits: %ld, %.3f s\n", c->waits, c->wait_s);
    if (c->s2) (void)hipStreamSynchronize(c->s2);
    if (c->s) (void)hipStreamSynchronize(c->s);
    kt_free(c);
    (void)hipFree(c->ck);
    (void)hipFree(c->cio);
    (void)hipFree(c->rface);
    if (c->hio) (void)hipHostFree(c->hio);
    free_mg(c->visc);
    free_mg(c->mac);
    free_mg(c->nodal);
    for (Cav& v : c->cv) {
        double* bufs[] = {v.eta, v.E, v.Gp, v.F, v.S, v.trans, v.uhat, v.qhat, v.qLf, v.qRf, v.uadv, v.umac,
                          v.macrhs, v.rnode, v.conv, v.rhs, v.dense_E};
        for (double* p : bufs) (void)hipFree(p);
    }
    double* bufs[] = {c->macphi, c->ustar, c->phi, c->kr, c->krh, c->kp, c->kv, c->kph, c->ks, c->ksh, c->kt,
                      c->sc, c->partial, c->uold};
    for (double* p : bufs) (void)hipFree(p);
    (void)hipFree(c->mpart);
    (void)hipFree(c->act);
    (void)hipFree(c->act2);
    (void)hipFree(c->sel);
    (void)hipFree(c->ws_in);
    (void)hipFree(c->ws_out);
    (void)hipFree(c->ws_y);
    (void)hipFree(c->ws_z);
    (void)hipFree(c->ws_x1);
    (void)hipFree(c->cap_r0);
    (void)hipFree(c->cap_e);
    (void)hipFree(c->cap_x0);
    (void)hipFree(c->capv_r0);
    (void)hipFree(c->capv_e);
    (void)hipFree(c->capv_x0);
    if (c->hsc) (void)hipHostFree(c->hsc);
    if (c->hseq) (void)hipHostFree(c->hseq);
    if (c->hring) (void)hipHostFree(c->hring);
    if (c->hact) (void)hipHostFree(c->hact);
    if (c->hact2) (void)hipHostFree(c->hact2);
    if (c->hsel) (void)hipHostFree(c->hsel);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->ev_f0) (void)hipEventDestroy(c->ev_f0);
    if (c->ev_f1) (void)hipEventDestroy(c->ev_f1);
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->s) (void)hipStreamDestroy(c->s);
    delete static_cast<::hb_ctx*>(c);
}

}  // namespace hb

using namespace hb;

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

static int single_only(Ctx* c)
{
    return c->nb == 1 ? HB_OK : fail(c, HB_ERR_ARG, "this call takes a single-cavity context (use hb_step_batch)");
}

static Ctx* C_(hb_ctx* h) { return static_cast<Ctx*>(h); }
static const Ctx* C_(const hb_ctx* h) { return static_cast<const Ctx*>(h); }

extern "C" {

const char* hb_last_error(const hb_ctx* ctx)
{
    if (!ctx) return g_create_err.c_str();
    return C_(ctx)->err.c_str();
}

void hb_destroy(hb_ctx* ctx)
{
    if (ctx) destroy_ctx(C_(ctx));
}

int hb_create(const hb_grid* grid, const hb_fluid* fluid, const hb_step_opts* opts, void* hip_stream, hb_ctx** out)
{
    Ctx* c = nullptr;
    const int rc = create_ctx(grid, fluid, 1, opts, hip_stream, &c);
    if (out) *out = static_cast<hb_ctx*>(c);
    return rc;
}

int hb_create_batch(const hb_grid* grids, const hb_fluid* fluids, int count, const hb_step_opts* opts,
                    void* hip_stream, hb_ctx** out)
{
    Ctx* c = nullptr;
    const int rc = create_ctx(grids, fluids, count, opts, hip_stream, &c);
    if (out) *out = static_cast<hb_ctx*>(c);
    return rc;
}

int hb_batch_size(const hb_ctx* ctx) { return ctx ? C_(ctx)->nb : 0; }

int hb_viscosity(hb_ctx* ctx, const double* u, double* eta)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u || !eta) return fail(c, HB_ERR_ARG, "null array");
    StreamGuard guard(c);
    launch_viscosity(c, c->cv[0], u, eta);
    return hipGetLastError() == hipSuccess ? HB_OK : fail(c, HB_ERR_DEVICE, "kernel launch failed");
}

int hb_mg_solve(hb_ctx* ctx, int op, const double* eta, double dt, const double* rhs, double* x,
                const hb_mg_opts* opts, hb_mg_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!rhs || !x) return fail(c, HB_ERR_ARG, "null array");
    if (op != HB_OP_VISC && op != HB_OP_NODAL && op != HB_OP_MAC) return fail(c, HB_ERR_ARG, "unknown operator");
    if (op == HB_OP_VISC && (!eta || !(dt > 0.0))) return fail(c, HB_ERR_ARG, "viscous solve needs eta and dt > 0");
    const hb_mg_opts& o = opts ? *opts : (op == HB_OP_VISC ? c->opts.visc : (op == HB_OP_MAC ? c->opts.mac : c->opts.proj));
    if (!valid_opts(o)) return fail(c, HB_ERR_ARG, "invalid multigrid options");
    MG& m = op == HB_OP_VISC ? c->visc : (op == HB_OP_MAC ? c->mac : c->nodal);
    StreamGuard guard(c);
    if (op == HB_OP_VISC) {
        std::vector<CavIO> io(1, io_zero());
        io[0].eta = eta;
        io[0].vdt = dt;
        io[0].b = const_cast<double*>(rhs);   // read only (the wall terms' base)
        set_io(c, io);
        visc_setup(c);
        factor_visc_async(c);
        stage_visc_wall_rhs(c);
    } else {
        copy(c, m.lvl0_b, rhs, m.L[0].nu);
    }
    solve_prepared(c, m, x, o);
    fetch_slots(c);
    std::vector<hb_mg_report> rep(1);
    const int rc = solve_outcome(c, m, &rep);
    if (report) *report = rep[0];
    return rc;
}

int hb_advect(hb_ctx* ctx, const double* u, const double* p, const double* eta, double dt, double* b, double* umac,
              double* conv, hb_mg_report* mac_report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u || !p || !eta || !b) return fail(c, HB_ERR_ARG, "null array");
    if (!(dt > 0.0)) return fail(c, HB_ERR_ARG, "dt must be positive");
    StreamGuard guard(c);
    Cav& v = c->cv[0];
    std::vector<CavIO> io(1, io_zero());
    io[0].u = u;
    io[0].p = const_cast<double*>(p);   // read only here
    io[0].eta = eta;
    io[0].b = b;
    io[0].conv = conv;
    io[0].dt = dt;
    io[0].vdt = dt;
    set_io(c, io);
    stage_maxabs(c, SF_U, S_MAXU);
    visc_setup(c);
    advect_predict(c);
    advect_finish(c, nullptr);
    if (umac) copy(c, umac, v.umac, v.nf);
    fetch_slots(c);
    std::vector<hb_mg_report> mrep(1);
    const int rc = mac_outcome(c, &mrep);
    if (mac_report) *mac_report = mrep[0];
    if (hipStreamSynchronize(c->s) != hipSuccess) return fail(c, HB_ERR_DEVICE, "stream synchronisation failed");
    return rc;
}

int hb_project(hb_ctx* ctx, const double* ustar, double* p, double dt, double* u, hb_mg_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!ustar || !p || !u) return fail(c, HB_ERR_ARG, "null array");
    if (!(dt > 0.0)) return fail(c, HB_ERR_ARG, "dt must be positive");
    StreamGuard guard(c);
    std::vector<CavIO> io(1, io_zero());
    io[0].ustar = ustar;
    io[0].p = p;
    io[0].uout = u;
    io[0].dt = dt;
    set_io(c, io);
    project_all(c);
    fetch_slots(c);
    std::vector<hb_mg_report> rep(1);
    const int rc = solve_outcome(c, c->nodal, &rep);
    if (report) *report = rep[0];
    return rc;
}

int hb_cfl_dt(hb_ctx* ctx, const double* u, double* dt_out)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u || !dt_out) return fail(c, HB_ERR_ARG, "null argument");
    StreamGuard guard(c);
    const Cav& v = c->cv[0];
    red_maxabs(c, 0, u, v.dim * v.nc, S_MAXU);
    fetch_slots(c);
    const double m = std::fmax(v.ulid, slot(c, 0, S_MAXU));
    if (!std::isfinite(m)) return fail(c, HB_ERR_NONFINITE, "non-finite velocity");
    *dt_out = m > 0.0 ? c->opts.cfl * v.g.h / m : 0.0;
    return HB_OK;
}

int hb_step(hb_ctx* ctx, double* u, double* p, double dt, hb_step_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u || !p) return fail(c, HB_ERR_ARG, "null array");
    StreamGuard guard(c);
    return step_all(c, &u, &p, &dt, report);
}

int hb_step_batch(hb_ctx* ctx, double* const* u, double* const* p, const double* dt, hb_step_report* reports)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (!u || !p) return fail(c, HB_ERR_ARG, "null array");
    for (int b = 0; b < c->nb; ++b)
        if (!u[b] || !p[b]) return fail(c, HB_ERR_ARG, "null array");
    StreamGuard guard(c);
    return step_all(c, u, p, dt, reports);
}

int hb_set_warm_start(hb_ctx* ctx, int op, hb_nn* nn)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (op != HB_OP_NODAL) return fail(c, HB_ERR_ARG, "the warm start serves the nodal projection solve only");
    if (!nn) {
        c->ws = nullptr;
        return HB_OK;
    }
    if (single_only(c)) return HB_ERR_ARG;
    const GridD& g = c->cv[0].g;
    if (c->dim != 2 || g.n[0] % 8 || g.n[1] % 8) return fail(c, HB_ERR_ARG, "the warm start needs a 2D grid with cell counts multiple of 8");
    NNet* t = nn_of(nn);
    if (nn_channels_in(t) != 1 || nn_channels_out(t) != 1) return fail(c, HB_ERR_ARG, "the warm-start network maps 1 channel to 1");
    if (!c->ws_in) {
        // all five buffers or none: a failed allocation frees the others
        const long nc = c->cv[0].nc, nn_ = c->nodal.L[0].nu;
        void* b[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
        const size_t sz[5] = {(size_t)4 * nc, (size_t)4 * nc, (size_t)8 * nn_, (size_t)8 * nn_, (size_t)8 * nn_};
        if (!alloc_all(b, sz, 5)) return fail(c, HB_ERR_OOM, "device allocation failed");
        c->ws_in = (float*)b[0];
        c->ws_out = (float*)b[1];
        c->ws_y = (double*)b[2];
        c->ws_z = (double*)b[3];
        c->ws_x1 = (double*)b[4];
    }
    c->ws = t;
    return HB_OK;
}

int hb_capture(hb_ctx* ctx, int op, int enable)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (op != HB_OP_NODAL && op != HB_OP_VISC) return fail(c, HB_ERR_ARG, "capture serves the nodal and viscous solves");
    if (single_only(c)) return HB_ERR_ARG;
    const bool visc = op == HB_OP_VISC;
    double** r0 = visc ? &c->capv_r0 : &c->cap_r0;
    double** e = visc ? &c->capv_e : &c->cap_e;
    double** x0 = visc ? &c->capv_x0 : &c->cap_x0;
    if (enable && !*r0) {
        // all three buffers or none
        const long n = (visc ? c->visc : c->nodal).L[0].nu;
        void* b[3] = {nullptr, nullptr, nullptr};
        const size_t sz[3] = {(size_t)8 * n, (size_t)8 * n, (size_t)8 * n};
        if (!alloc_all(b, sz, 3)) return fail(c, HB_ERR_OOM, "device allocation failed");
        *r0 = (double*)b[0];
        *e = (double*)b[1];
        *x0 = (double*)b[2];
        StreamGuard guard(c);
        fill(c, *r0, 0.0, n);
        fill(c, *e, 0.0, n);
        if (hipStreamSynchronize(c->s) != hipSuccess) return fail(c, HB_ERR_DEVICE, "stream synchronisation failed");
    }
    (visc ? c->capv : c->cap) = enable != 0;
    return HB_OK;
}

int hb_capture_read(hb_ctx* ctx, int op, double* r0, double* e)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    const bool visc = op == HB_OP_VISC;
    const double* cr = visc ? c->capv_r0 : c->cap_r0;
    const double* ce = visc ? c->capv_e : c->cap_e;
    if ((op != HB_OP_NODAL && !visc) || !r0 || !e || !cr) return fail(c, HB_ERR_ARG, "nothing captured");
    StreamGuard guard(c);
    const long n = (visc ? c->visc : c->nodal).L[0].nu;
    copy(c, r0, cr, n);
    copy(c, e, ce, n);
    return hipStreamSynchronize(c->s) == hipSuccess ? HB_OK : fail(c, HB_ERR_DEVICE, "stream synchronisation failed");
}

int hb_warm_start_uses(const hb_ctx* ctx) { return ctx ? (int)C_(ctx)->ws_report_used : 0; }

int hb_tile_config(const hb_ctx* ctx, int op, int level, int* tx, int* ty, int* threads, int* sweeps)
{
    if (!ctx || !tx || !ty) return HB_ERR_ARG;
    const Ctx* c = C_(ctx);
    const MG* m = op == HB_OP_VISC ? &c->visc : (op == HB_OP_NODAL ? &c->nodal : nullptr);
    if (!m || !c->fuse || (op == HB_OP_VISC && c->dim != 2) || level < 0 || level >= m->nlev) return HB_ERR_ARG;
    const Level& L = m->L[level];
    if (!L.any_sm || (m->tail_lt >= 0 && level >= m->tail_lt)) return HB_ERR_ARG;
    int th = 256, sw = 1;
    if (op == HB_OP_VISC) {
        const SweepShape sh = sweep2_shape(L.tile);
        *tx = sh.tx;
        *ty = sh.ty;
        th = sh.threads;
        sw = L.sweeps;
    } else {
        nodal_sweep_tile(c->dim, L.tile, tx, ty, &th);
        sw = L.sweeps;
    }
    if (threads) *threads = th;
    if (sweeps) *sweeps = sw;
    return HB_OK;
}

int hb_kernel_timing(hb_ctx* ctx, int enable)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
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
    k.on = enable > 0;
    k.period = enable > 0 ? enable : 1;
    k.seen = 0;
    k.n = 0;
    k.launches = 0;
    k.ms = 0.0;
    k.bytes = 0.0;
    return HB_OK;
}

int hb_kernel_timing_read(hb_ctx* ctx, int64_t* launches, double* total_ms, double* alg_bytes)
{
    if (!ctx || !launches || !total_ms || !alg_bytes) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    kt_harvest(c);
    *launches = c->ktm.launches;
    *total_ms = c->ktm.ms;
    *alg_bytes = c->ktm.bytes;
    return HB_OK;
}

// ---- steady state, grid sequencing, checkpoints (Sec. III.A, Sec. III.C) ---

// the grid one refinement below g (every used axis halved, spacing doubled);
// false when a used axis has an odd cell count
static bool coarser_grid(const GridD& g, GridD* out)
{
    GridD c = g;
    for (int a = 0; a < g.dim; ++a) {
        if (g.n[a] % 2 || g.n[a] < 2) return false;
        c.n[a] = g.n[a] / 2;
    }
    c.h = 2.0 * g.h;
    *out = c;
    return true;
}

// steps (u, p) until the largest change of u over a step, relative to the
// largest |u| before it, is below tol (Sec. III.A), or max_steps have run
static int run_steady(Ctx* c, double* u, double* p, double tol, int max_steps, double dt, hb_steady_report* rep)
{
    const Cav& v = c->cv[0];
    const long n = (long)v.dim * v.nc;
    if (!c->uold && dalloc(&c->uold, n) != hipSuccess) return fail(c, HB_ERR_OOM, "device allocation failed");
    hb_steady_report R;
    memset(&R, 0, sizeof(R));
    R.change = HUGE_VAL;
    int rc = HB_ERR_NOCONV;
    for (int m = 0; m < max_steps; ++m) {
        copy(c, c->uold, u, n);
        const int src = step_all(c, &u, &p, &dt, nullptr);
        R.steps = m + 1;
        if (src != HB_OK && src != HB_ERR_NOCONV) {
            rc = src;
            break;
        }
        red_maxdiff(c, 0, u, c->uold, n, S_CHG);
        red_maxabs(c, 0, c->uold, n, S_CHGREF);
        fetch_slots(c);
        R.t += c->cv[0].step_dt;
        const double ref = slot(c, 0, S_CHGREF);
        R.change = ref > 0.0 ? slot(c, 0, S_CHG) / ref : HUGE_VAL;
        if (src == HB_ERR_NOCONV) {
            rc = src;
            break;
        }
        if (R.change < tol) {
            R.steady = 1;
            rc = HB_OK;
            break;
        }
    }
    if (rep) *rep = R;
    if (hipGetLastError() != hipSuccess) return fail(c, HB_ERR_DEVICE, "kernel launch failed");
    return rc;
}

int hb_run_steady(hb_ctx* ctx, double* u, double* p, double tol, int max_steps, double dt, hb_steady_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u || !p) return fail(c, HB_ERR_ARG, "null array");
    if (!(tol > 0.0) || max_steps < 1) return fail(c, HB_ERR_ARG, "tol must be > 0 and max_steps >= 1");
    StreamGuard guard(c);
    return run_steady(c, u, p, tol, max_steps, dt, report);
}

int hb_refine_state(hb_ctx* ctx, const double* u_coarse, const double* p_coarse, double* u, double* p)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u_coarse || !p_coarse || !u || !p) return fail(c, HB_ERR_ARG, "null array");
    GridD gc;
    if (!coarser_grid(c->cv[0].g, &gc)) return fail(c, HB_ERR_ARG, "every cell count must be even");
    StreamGuard guard(c);
    launch_refine_state(c, gc, c->cv[0].g, u_coarse, p_coarse, u, p);
    return hipGetLastError() == hipSuccess ? HB_OK : fail(c, HB_ERR_DEVICE, "kernel launch failed");
}

int hb_run_sequenced(const hb_grid* coarse, const hb_fluid* fluid, const hb_step_opts* opts, int levels, double tol,
                     int max_steps, void* hip_stream, double* u, double* p, hb_steady_report* reports)
{
    auto bad = [](int code, const std::string& m) { g_create_err = m; return code; };
    if (!coarse || !fluid || !opts || !u || !p || !reports) return bad(HB_ERR_ARG, "null argument");
    if (levels < 0 || levels > 8) return bad(HB_ERR_ARG, "levels must be 0 .. 8");
    if (!(tol > 0.0) || max_steps < 1) return bad(HB_ERR_ARG, "tol must be > 0 and max_steps >= 1");
    hb_grid g = *coarse;
    Ctx* prev = nullptr;
    double *uprev = nullptr, *pprev = nullptr;
    int rc = HB_OK;
    memset(reports, 0, sizeof(hb_steady_report) * (levels + 1));
    for (int l = 0; l <= levels; ++l) {
        if (l > 0) {
            for (int a = 0; a < g.dim; ++a) g.n[a] *= 2;
            g.h *= 0.5;
        }
        Ctx* c = nullptr;
        const int crc = create_ctx(&g, fluid, 1, opts, hip_stream, &c);
        if (crc != HB_OK) {
            rc = crc;
            break;
        }
        const Cav& v = c->cv[0];
        double *ul = u, *pl = p;
        if (l < levels) {
            ul = pl = nullptr;
            if (dalloc(&ul, (long)v.dim * v.nc) != hipSuccess || dalloc(&pl, v.nn) != hipSuccess) {
                (void)hipFree(ul);
                (void)hipFree(pl);
                destroy_ctx(c);
                rc = bad(HB_ERR_OOM, "device allocation failed");
                break;
            }
        }
        int lrc;
        {
            StreamGuard guard(c);
            if (l == 0) {
                fill(c, ul, 0.0, (long)v.dim * v.nc);
                fill(c, pl, 0.0, v.nn);
            } else {
                GridD gc;
                coarser_grid(v.g, &gc);
                launch_refine_state(c, gc, v.g, uprev, pprev, ul, pl);
            }
            lrc = run_steady(c, ul, pl, tol, max_steps, 0.0, &reports[l]);
        }
        if (prev) {
            (void)hipStreamSynchronize(c->s);
            (void)hipFree(uprev);
            (void)hipFree(pprev);
            destroy_ctx(prev);
        }
        prev = c;
        uprev = ul;
        pprev = pl;
        // a level that did not become steady within max_steps is refined
        // all the same; any other failure ends the run
        if (lrc != HB_OK) {
            g_create_err = c->err;
            rc = lrc;
            if (lrc != HB_ERR_NOCONV) break;
        }
    }
    if (prev) {
        (void)hipStreamSynchronize(prev->s);
        if (uprev != u) (void)hipFree(uprev);
        if (pprev != p) (void)hipFree(pprev);
        destroy_ctx(prev);
    }
    return rc;
}

// yield test of the state u: count of yielded cells and largest stress
// magnitude in the slots S_SUM and S_MAX (read after fetch_slots)
static void yield_slots(Ctx* c, const double* u, unsigned char* mask)
{
    set_slot(c, 0, S_SUM, 0.0);
    set_slot(c, 0, S_MAX, 0.0);
    double* sc = c->sc;
    launch_yield(c, c->cv[0], u, mask, sc + S_SUM, sc + S_MAX);
}

int hb_yield(hb_ctx* ctx, const double* u, uint8_t* mask, hb_yield_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u) return fail(c, HB_ERR_ARG, "null array");
    StreamGuard guard(c);
    yield_slots(c, u, mask);
    if (report) {
        fetch_slots(c);
        report->yielded = (int64_t)slot(c, 0, S_SUM);
        report->cells = c->cv[0].nc;
        report->max_stress = slot(c, 0, S_MAX);
    }
    return hipGetLastError() == hipSuccess ? HB_OK : fail(c, HB_ERR_DEVICE, "kernel launch failed");
}

int hb_run_cessation(hb_ctx* ctx, double* u, double* p, int max_steps, double dt, hb_cessation_report* report)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!u || !p) return fail(c, HB_ERR_ARG, "null array");
    if (max_steps < 1) return fail(c, HB_ERR_ARG, "max_steps must be >= 1");
    if (!(c->cv[0].fluid.HB > 0.0)) return fail(c, HB_ERR_ARG, "cessation needs a yield stress (HB > 0)");
    StreamGuard guard(c);
    hb_cessation_report R;
    memset(&R, 0, sizeof(R));
    yield_slots(c, u, nullptr);
    fetch_slots(c);
    int rc = HB_OK;
    if (slot(c, 0, S_SUM) == 0.0) {
        R.stopped = 1;
    } else {
        rc = HB_ERR_NOCONV;
        for (int m = 0; m < max_steps; ++m) {
            const int src = step_all(c, &u, &p, &dt, nullptr);
            R.steps = m + 1;
            if (src != HB_OK && src != HB_ERR_NOCONV) {
                rc = src;
                break;
            }
            yield_slots(c, u, nullptr);
            fetch_slots(c);
            R.t += c->cv[0].step_dt;
            if (src == HB_ERR_NOCONV) {
                rc = src;
                break;
            }
            if (slot(c, 0, S_SUM) == 0.0) {
                R.stopped = 1;
                rc = HB_OK;
                break;
            }
        }
    }
    if (report) *report = R;
    if (hipGetLastError() != hipSuccess) return fail(c, HB_ERR_DEVICE, "kernel launch failed");
    return rc;
}

// checkpoint file: this header, then u ([dim][cells]) and p (nodes) as raw
// doubles in host byte order
struct CkptHeader {
    char magic[8];
    int32_t version, dim, n[3], per[3];
    int64_t nu, np, step;
    double t, h;
};
static_assert(sizeof(CkptHeader) == 80, "checkpoint header layout");
static const char kCkptMagic[8] = {'H', 'B', 'C', 'K', 'P', 'T', '\0', '\0'};

static void ckpt_header_of(const Cav& v, CkptHeader* H)
{
    memset(H, 0, sizeof(*H));
    memcpy(H->magic, kCkptMagic, 8);
    H->version = 1;
    H->dim = v.dim;
    for (int a = 0; a < 3; ++a) {
        H->n[a] = v.g.n[a];
        H->per[a] = v.g.per[a];
    }
    H->nu = (int64_t)v.dim * v.nc;
    H->np = v.nn;
    H->h = v.g.h;
}

int hb_checkpoint_write(hb_ctx* ctx, const char* path, const double* u, const double* p, int64_t step, double t)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!path || !u || !p) return fail(c, HB_ERR_ARG, "null argument");
    const Cav& v = c->cv[0];
    CkptHeader H;
    ckpt_header_of(v, &H);
    H.step = step;
    H.t = t;
    std::vector<double> hu(H.nu), hp(H.np);
    {
        StreamGuard guard(c);
        if (hipMemcpyAsync(hu.data(), u, sizeof(double) * H.nu, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
            hipMemcpyAsync(hp.data(), p, sizeof(double) * H.np, hipMemcpyDeviceToHost, c->s) != hipSuccess ||
            hipStreamSynchronize(c->s) != hipSuccess)
            return fail(c, HB_ERR_DEVICE, "device to host copy failed");
    }
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, HB_ERR_IO, std::string("cannot open for writing: ") + path);
    const bool ok = fwrite(&H, sizeof(H), 1, f) == 1 && fwrite(hu.data(), sizeof(double), H.nu, f) == (size_t)H.nu &&
                    fwrite(hp.data(), sizeof(double), H.np, f) == (size_t)H.np;
    const bool closed = fclose(f) == 0;
    return ok && closed ? HB_OK : fail(c, HB_ERR_IO, std::string("write failed: ") + path);
}

int hb_checkpoint_read(hb_ctx* ctx, const char* path, double* u, double* p, int64_t* step, double* t)
{
    if (!ctx) return HB_ERR_ARG;
    Ctx* c = C_(ctx);
    if (single_only(c)) return HB_ERR_ARG;
    if (!path || !u || !p) return fail(c, HB_ERR_ARG, "null argument");
    const Cav& v = c->cv[0];
    CkptHeader want, H;
    ckpt_header_of(v, &want);
    FILE* f = fopen(path, "rb");
    if (!f) return fail(c, HB_ERR_IO, std::string("cannot open for reading: ") + path);
    std::vector<double> hu, hp;
    bool ok = fread(&H, sizeof(H), 1, f) == 1;
    if (ok && (memcmp(H.magic, kCkptMagic, 8) != 0 || H.version != 1)) {
        fclose(f);
        return fail(c, HB_ERR_IO, std::string("not a checkpoint of this format: ") + path);
    }
    if (ok) {
        bool same = H.dim == want.dim && H.nu == want.nu && H.np == want.np && H.h == want.h;
        for (int a = 0; a < 3; ++a) same = same && H.n[a] == want.n[a] && H.per[a] == want.per[a];
        if (!same) {
            fclose(f);
            return fail(c, HB_ERR_ARG, "the checkpoint's grid differs from the context's");
        }
        hu.resize(H.nu);
        hp.resize(H.np);
        ok = fread(hu.data(), sizeof(double), H.nu, f) == (size_t)H.nu &&
             fread(hp.data(), sizeof(double), H.np, f) == (size_t)H.np;
    }
    fclose(f);
    if (!ok) return fail(c, HB_ERR_IO, std::string("truncated checkpoint: ") + path);
    {
        StreamGuard guard(c);
        if (hipMemcpyAsync(u, hu.data(), sizeof(double) * H.nu, hipMemcpyHostToDevice, c->s) != hipSuccess ||
            hipMemcpyAsync(p, hp.data(), sizeof(double) * H.np, hipMemcpyHostToDevice, c->s) != hipSuccess ||
            hipStreamSynchronize(c->s) != hipSuccess)
            return fail(c, HB_ERR_DEVICE, "host to device copy failed");
    }
    if (step) *step = H.step;
    if (t) *t = H.t;
    return HB_OK;
}

}  // extern "C"
