// hb_internal.h -- host-side context, multigrid hierarchy and kernel
// launchers of the HIP library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <string>

#include "../../include/hb.h"
#include "hb_dev.h"

namespace hb {

struct FluidD {
    double Re, HB, n, Pa;
    int reg;
    double f[3];
};

struct Level {
    GridD g;
    long nu = 0;             // unknowns of this level
    int cur = 0;             // buffer holding the current iterate
    // FP64 arrays
    double* xb[2] = {nullptr, nullptr};  // double-buffered iterate
    double* b = nullptr;     // right-hand side
    double* r = nullptr;     // residual scratch
    double* beta = nullptr;  // face viscosity (tensor problem only)
    // FP32 arrays of the mixed-precision correction cycles
    float* fx[2] = {nullptr, nullptr};
    float* fb = nullptr;
    float* fr = nullptr;
    float* fbeta = nullptr;
    double* X() const { return xb[cur]; }
};

// the arrays of a level in storage precision R
template <typename R> struct LB;
template <> struct LB<double> {
    static double* x(const Level& L) { return L.xb[L.cur]; }
    static double* xo(const Level& L) { return L.xb[1 - L.cur]; }
    static double* b(const Level& L) { return L.b; }
    static double* r(const Level& L) { return L.r; }
    static const double* beta(const Level& L) { return L.beta; }
};
template <> struct LB<float> {
    static float* x(const Level& L) { return L.fx[L.cur]; }
    static float* xo(const Level& L) { return L.fx[1 - L.cur]; }
    static float* b(const Level& L) { return L.fb; }
    static float* r(const Level& L) { return L.fr; }
    static const float* beta(const Level& L) { return L.fbeta; }
};

struct MG {
    int op = 0;
    int nlev = 0;
    Level L[kMaxLev];
    int ncoarse = 0;         // unknowns on the coarsest level
    double* A = nullptr;     // coarsest dense matrix -> LU factors
    int* piv = nullptr;
    double* Ainv = nullptr;  // inverse of the coarsest matrix (from the LU factors)
    double dt = 0.0;         // tensor problem: dt of the factorised matrix
    double* lvl0_b = nullptr;  // level-0 right-hand side storage
    double* etae = nullptr;    // tensor problem: eta/Re per fine cell
    float* etae32 = nullptr;   // its FP32 copy
    bool f32_ready = false;    // FP32 coefficient copies match the FP64 ones
    // levels 1.. of a V-cycle captured once per precision as a HIP graph and
    // replayed (index 0: FP64, 1: FP32)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gnu1[2] = {-1, -1}, gnu2[2] = {-1, -1};
    bool gfail[2] = {false, false};
    bool capturing = false;
};

// HIP-event timing of every launch of one kernel (measurement support)
struct KTimer {
    bool on = false;
    int cap = 0, n = 0;
    hipEvent_t* ev = nullptr;   // 2 * cap events: start/stop pairs
    long launches = 0;
    double ms = 0.0, bytes = 0.0;
};

// scalar slots in ctx->sc (device doubles)
enum Slot {
    S_MAX = 0, S_SUM = 1, S_DOT0 = 2, S_DOT1 = 3, S_MAXU = 4, S_MAX2 = 5, S_DT = 6,
    // BiCGStab scalars, computed and used on the device
    S_RHO = 8, S_RHOP = 9, S_ALPHA = 10, S_OMEGA = 11, S_BETA = 12,
    S_NSLOT = 16
};

struct Ctx {
    hb_grid grid;
    hb_fluid fluid;
    hb_step_opts opts;
    hipStream_t s = nullptr;      // the library's own stream (all work runs here)
    hipStream_t user = nullptr;   // the caller's stream, ordered with s by events
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    GridD g;                 // finest grid
    FluidD fl;
    int dim = 2;
    long nc = 0, nn = 0, nf = 0;
    double ulid = 0.0;
    MG visc, mac, nodal;
    // step scratch
    double *eta = nullptr, *E = nullptr, *Gp = nullptr, *F = nullptr, *S = nullptr, *trans = nullptr;
    double *uhat = nullptr, *qhat = nullptr, *qLf = nullptr, *qRf = nullptr, *uadv = nullptr, *umac = nullptr;
    double *macphi = nullptr, *macrhs = nullptr, *b = nullptr, *ustar = nullptr, *rnode = nullptr;
    double *phi = nullptr, *conv = nullptr;
    // Krylov vectors (tensor problem size)
    double *kr = nullptr, *krh = nullptr, *kp = nullptr, *kv = nullptr, *kph = nullptr, *ks = nullptr,
           *ksh = nullptr, *kt = nullptr;
    double* dense_E = nullptr;   // unit-vector scratch for dense assembly
    double* sc = nullptr;        // device scalar slots
    double* partial = nullptr;   // reduction partials
    double* hsc = nullptr;       // pinned host mirror of the slots
    KTimer ktm;                  // timing of the tensor smoother launches
    std::string err;
};

void kt_begin(Ctx* c);
void kt_end(Ctx* c, double bytes);
void kt_harvest(Ctx* c);

// ---- launch helpers --------------------------------------------------------
inline dim3 grid3(int ex, int ey, int ez, dim3 blk) { return dim3((ex + blk.x - 1) / blk.x, (ey + blk.y - 1) / blk.y, ez); }
constexpr int kRedBlocks = 512;   // fixed block count: deterministic sums

// reductions (hb_reduce.hip)
void red_maxabs(Ctx* c, const double* v, long n, int slot, bool accumulate = false);
void red_sum(Ctx* c, const double* v, long n, int slot);
void red_dot(Ctx* c, const double* a, const double* b, long n, int slot);
void fetch_slots(Ctx* c);  // copies all slots to c->hsc and synchronises
void set_slot_zero(Ctx* c, int slot);
void set_slot(Ctx* c, int slot, double v);
void sub_mean(Ctx* c, double* v, long n);   // v -= sum(v)/n (device-side)
// device-scalar BiCGStab steps (scalars in the slots S_RHO .. S_BETA)
void bicg_init_scalars(Ctx* c);
void bicg_beta(Ctx* c);             // rho = DOT0, beta = (rho/rho_prev)(alpha/omega)
void bicg_alpha(Ctx* c);            // alpha = rho / DOT1
void bicg_omega(Ctx* c);            // omega = DOT0 > 0 ? DOT1 / DOT0 : 0; rho_prev = rho
void bicg_p_dev(Ctx* c, double* p, const double* r, const double* v, long n);
void sub_scaled_max_dev(Ctx* c, double* out, const double* a, int sslot, const double* b, long n, int mslot);
void bicg_x_dev(Ctx* c, double* x, const double* ph, const double* sh, bool with_omega, long n);
void copy(Ctx* c, double* dst, const double* src, long n);
void fill(Ctx* c, double* dst, double v, long n);

// viscosity and tensor operator (hb_visc.hip)
void launch_viscosity(Ctx* c, const double* u, double* eta);
void launch_eta_faces(Ctx* c, const GridD& g, const double* eta, double* beta);
void launch_restrict_faces(Ctx* c, const GridD& gf, const GridD& gc, const double* bf, double* bc);
void launch_visc_div(Ctx* c, const GridD& g, const double* beta, const double* u, double* out);
void launch_visc_wall_rhs(Ctx* c, const GridD& g, const double* beta, double dt, const double* rhs, double* out);
void launch_visc_dense(Ctx* c, const Level& l, double dt, int N, double* E, double* A);
void launch_eta_over_re(Ctx* c, const GridD& g, const double* eta, double* etae);

// LDS-tiled tensor kernels (hb_tile.hip), R = storage and arithmetic
// precision of the multigrid cycle; fine = coef is eta/Re per cell (else the
// level's face viscosities).  dt is read from device memory, so a captured
// graph stays valid across steps.
template <typename R>
void launch_tsmooth(Ctx* c, const GridD& g, const R* coef, bool fine, const double* dtp, int comp, const R* xcur,
                    R* xnext, const R* b);
template <typename R>
void launch_trb3(Ctx* c, const GridD& g, const R* coef, bool fine, const double* dtp, int comp, int colour, R* x,
                 const R* b);
template <typename R>
void launch_tresid_restr(Ctx* c, const GridD& g, const GridD& gc, const R* coef, bool fine, const double* dtp,
                         const R* x, const R* b, R* bc, R* xc);
// FP64 finest-level residual r = b - A x (max-norm into slot) or y = A x (b null)
void launch_tresid(Ctx* c, const GridD& g, const double* coef, bool fine, const double* dtp, const double* x,
                   const double* b, double* out, int slot);

// scalar cell problem (MAC) and nodal problem, transfers, coarsest solve
// (hb_mg.hip, hb_nodal.hip)
template <typename R> void launch_mac_rb(Ctx* c, const GridD& g, int colour, R* x, const R* b);
template <typename R>
void launch_mac_resid_restrict(Ctx* c, const GridD& gf, const GridD& gc, const R* xf, const R* bf, R* bc, R* xc);
void launch_mac_resid(Ctx* c, const GridD& g, const double* x, const double* b, double* r, int slot);
void launch_mac_apply(Ctx* c, const GridD& g, const double* x, double* y);
void launch_mac_dense(Ctx* c, const Level& l, int N, double* E, double* A);
template <typename R>
void launch_prolong_cells(Ctx* c, const GridD& gf, const GridD& gc, int ncomp, double wall_sign, const R* e, R* x);
template <typename R> void launch_nodal_gs(Ctx* c, const GridD& g, int colour, R* x, const R* b);
// r = b - K x (slot >= 0: FP64 only, max-norm into the slot) or y = K x (b null)
template <typename R> void launch_nodal_resid(Ctx* c, const GridD& g, const R* x, const R* b, R* r, int slot);
template <typename R> void launch_nodal_restrict(Ctx* c, const GridD& gf, const GridD& gc, const R* rf, R* bc, R* xc);
template <typename R> void launch_nodal_prolong(Ctx* c, const GridD& gf, const GridD& gc, const R* e, R* x);
void launch_nodal_dense(Ctx* c, const Level& l, int N, double* E, double* A);
void launch_add_ones(Ctx* c, int N, double* A);
void launch_lu_factor(Ctx* c, int N, double* A, int* piv);
void launch_lu_inverse(Ctx* c, int N, const double* LU, const int* piv, double* Ainv);
// x = A^{-1} b on the coarsest level, accumulated in FP64
template <typename R> void launch_coarse_solve(Ctx* c, int N, const double* Ainv, const R* b, R* x);

// precision conversions of the mixed-precision cycles (hb_reduce.hip)
void to_f32(Ctx* c, const double* src, float* dst, float* zero, long n);   // dst = src, zero = 0 (nullable)
void add_f32(Ctx* c, double* x, const float* e, long n);                   // x += e
void from_f32(Ctx* c, const float* e, double* x, long n);                  // x = e

// step stages (hb_step.hip)
void launch_grad_node(Ctx* c, const double* p, double* Gp);
void launch_forcing(Ctx* c);
void launch_slopes(Ctx* c, const double* u);
void launch_trace_normal(Ctx* c, const double* u, double dt);
void launch_transverse(Ctx* c);
void launch_trace_full(Ctx* c, const double* u, double dt);
void launch_mac_div(Ctx* c, const double* faces, double* out);
void launch_mac_update(Ctx* c);
void launch_advect_rhs(Ctx* c, const double* u, double dt, double* b, double* conv);
void launch_proj_rhs(Ctx* c, const double* ustar, double dt, double* r);
void launch_weak_div(Ctx* c, const double* V, double* r);
void launch_proj_update(Ctx* c, const double* ustar, const double* phi, double dt, double* u);

}  // namespace hb
