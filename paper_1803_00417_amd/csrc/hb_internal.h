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
    double* x = nullptr;     // iterate (level 0: points at the solve's x)
    double* b = nullptr;     // right-hand side
    double* r = nullptr;     // residual scratch
    double* beta = nullptr;  // face viscosity (tensor problem only)
    float* xs = nullptr;     // FP32 shadows for mixed-precision cycles
    float* bs = nullptr;
    float* betas = nullptr;
};

struct MG {
    int op = 0;
    int nlev = 0;
    Level L[kMaxLev];
    int ncoarse = 0;         // unknowns on the coarsest level
    double* A = nullptr;     // coarsest dense matrix -> LU factors
    int* piv = nullptr;
    double dt = 0.0;         // tensor problem: dt of the factorised matrix
    double* lvl0_b = nullptr;  // level-0 right-hand side storage
    double* lvl0_x = nullptr;  // level-0 iterate storage (preconditioner use)
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
enum Slot { S_MAX = 0, S_SUM = 1, S_DOT0 = 2, S_DOT1 = 3, S_MAXU = 4, S_MAX2 = 5, S_NSLOT = 8 };

struct Ctx {
    hb_grid grid;
    hb_fluid fluid;
    hb_step_opts opts;
    hipStream_t s = nullptr;
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
void sub_mean(Ctx* c, double* v, long n);   // v -= sum(v)/n (device-side)
void axpby(Ctx* c, double* y, double a, const double* x, double b, long n);   // y = a x + b y
void bicg_p(Ctx* c, double* p, const double* r, const double* v, double beta, double omega, long n);
void sub_scaled_max(Ctx* c, double* out, const double* a, double s, const double* b, long n, int slot);
void bicg_x(Ctx* c, double* x, const double* ph, const double* sh, double alpha, double omega, long n);
void copy(Ctx* c, double* dst, const double* src, long n);
void fill(Ctx* c, double* dst, double v, long n);

// viscosity and tensor operator (hb_visc.hip)
void launch_viscosity(Ctx* c, const double* u, double* eta);
void launch_eta_faces(Ctx* c, const GridD& g, const double* eta, double* beta);
void launch_restrict_faces(Ctx* c, const GridD& gf, const GridD& gc, const double* bf, double* bc);
void launch_visc_div(Ctx* c, const GridD& g, const double* beta, const double* u, double* out);
void launch_visc_wall_rhs(Ctx* c, const GridD& g, const double* beta, double dt, const double* rhs, double* out);
void launch_visc_rb(Ctx* c, const Level& l, double dt, int comp, int colour);
void launch_visc_resid(Ctx* c, const Level& l, double dt, const double* x, const double* b, double* r, int slot);
void launch_visc_apply(Ctx* c, const Level& l, double dt, const double* x, double* y);
void launch_visc_resid_restrict(Ctx* c, const Level& f, const Level& cl, double dt);
void launch_visc_dense(Ctx* c, const Level& l, double dt, int N, double* E, double* A);

// scalar cell problem (MAC) and nodal problem, transfers, dense (hb_mg.hip)
void launch_mac_rb(Ctx* c, const Level& l, int colour);
void launch_mac_resid(Ctx* c, const Level& l, const double* x, const double* b, double* r, int slot);
void launch_mac_apply(Ctx* c, const Level& l, const double* x, double* y);
void launch_mac_resid_restrict(Ctx* c, const Level& f, const Level& cl);
void launch_mac_dense(Ctx* c, const Level& l, int N, double* E, double* A);
void launch_prolong_cells(Ctx* c, const Level& f, const Level& cl, int ncomp, double wall_sign);
void launch_nodal_gs(Ctx* c, const Level& l, int colour);
void launch_nodal_resid(Ctx* c, const Level& l, const double* x, const double* b, double* r, int slot);
void launch_nodal_apply(Ctx* c, const Level& l, const double* x, double* y);
void launch_nodal_restrict(Ctx* c, const Level& f, const Level& cl);
void launch_nodal_prolong(Ctx* c, const Level& f, const Level& cl);
void launch_nodal_dense(Ctx* c, const Level& l, int N, double* E, double* A);
void launch_add_ones(Ctx* c, int N, double* A);
void launch_lu_factor(Ctx* c, int N, double* A, int* piv);
void launch_lu_solve(Ctx* c, int N, const double* A, const int* piv, const double* b, double* x);

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
