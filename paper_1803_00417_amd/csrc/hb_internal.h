// hb_internal.h -- host-side context, batched multigrid hierarchy and kernel
// launchers of the HIP library (not part of the public ABI).
//
// A context holds a batch of nb independent cavities (nb = 1 for hb_create).
// The per-step work outside the solves runs per cavity.  The three linear
// solves run batched: every array of a multigrid level is one arena holding
// all cavities back to back, and every multigrid kernel covers all cavities
// in one launch, each block finding its cavity (grid, array offsets, active
// flag) in small device tables.  Cavities converge independently: a cavity
// that has reached its tolerance is masked out of the following launches.
#pragma once
#include <hip/hip_runtime.h>
#include <string>
#include <array>
#include <vector>

#include "../../include/hb.h"
#include "hb_dev.h"

namespace hb {

struct FluidD {
    double Re, HB, n, Pa;
    int reg;
    double f[3];
};

// scalar slots of each cavity (device doubles, S_NSLOT per cavity)
enum Slot {
    S_MAX = 0, S_SUM = 1, S_DOT0 = 2, S_DOT1 = 3, S_MAXU = 4, S_MAX2 = 5, S_DT = 6,
    // steady-state driver: largest change of u over a step, largest |u| before it
    S_CHG = 13, S_CHGREF = 14,
    // BiCGStab scalars, computed and used on the device
    S_RHO = 8, S_RHOP = 9, S_ALPHA = 10, S_OMEGA = 11, S_BETA = 12,
    // per-solve records, kept on the device while the solve runs (decided
    // there, read by the host once per step): |b|_inf, relative residual,
    // V-cycles, return code; one record per operator
    S_REC_MAC = 16, S_REC_VISC = 20, S_REC_NODAL = 24,
    S_NSLOT = 32
};
enum RecField { R_BN = 0, R_REL = 1, R_CYC = 2, R_RC = 3 };

// Convergence decisions of a multigrid solve, taken on the device by one
// small kernel per check point (the host only learns, one check point late,
// whether any cavity is still active).
enum ConvMode {
    CV_BEGIN = 0,      // record |b| (slot S_MAX) and the finiteness of b, x; set the active flags
    CV_INIT = 1,       // after the first residual: relative residual, stop test
    CV_CYCLE = 2,      // after a V-cycle (plain iteration): count it, residual, stop test
    CV_HALF = 3,       // BiCGStab half step: count, finish on |s| (flags act2)
    CV_FULL = 4,       // BiCGStab full step: count, residual, breakdown, stop test
    CV_END_PLAIN = 5,  // act2 = the cavities whose iterate is copied out
    CV_END_KRYLOV = 6, // act = the cavities whose true residual is taken
    CV_FINAL = 7       // relative true residual of those
};
struct ConvArgs {
    int nb, rec, mode, cur_sel;
    double tol;
    int max_cycles, fixed;
    unsigned long long seq;   // publication number of the active count (0: none)
    // single-cavity contexts: the final pass of the max-norm just before the
    // check (slot, or -1), done by the check kernel itself
    int mf_slot, mf_act;
};
constexpr int kRing = 8;      // entries of the pinned ring of active counts

// Batched view of one multigrid level, passed by value to the cycle kernels.
// Block z index = cavity * zb + z-block within the cavity.
struct BV {
    const GridD* g;     // per cavity; dim == 0: the cavity takes no part
    const long* o;      // per cavity offset of a one-component array (cells, or nodes)
    const long* of;     // per cavity offset of the face arrays (tensor problem)
    const int* act;     // per cavity active flag (nullptr: all active)
    int zb;             // z-blocks per cavity in the launch grid
    // Single-cavity contexts: the grids travel in the kernel arguments and
    // the offsets are 0, so a block's first data loads wait only for its
    // active flag (the device stops a converged solve; the host does not
    // know when).
    int one = 0;
    GridD g1{};         // the cavity's grid on this level (dim 0: takes no part)
    GridD g2{};         // its grid on the paired level of a transfer kernel
};

__device__ inline long bv_o(const BV& v, int cav) { return v.one ? 0 : v.o[cav]; }
__device__ inline long bv_of(const BV& v, int cav) { return v.one ? 0 : v.of[cav]; }
// grid and offset of the paired level (table t, offsets to)
__device__ inline GridD bv_g2(const BV& v, const GridD* __restrict__ t, int cav) { return v.one ? v.g2 : t[cav]; }
__device__ inline long bv_o2(const BV& v, const long* __restrict__ to, int cav) { return v.one ? 0 : to[cav]; }

// Segmented view of a batch vector (vector kernels and reductions)
struct SegV {
    const long* off;    // per cavity first element
    const long* n;      // per cavity length
    const int* act;     // per cavity active flag (nullptr: all)
};

// XCD-aware tile order.  Workgroups are dispatched to the 8 XCDs (each with
// its own L2) round-robin by linear block id; this map gives XCD k the k-th
// contiguous eighth of the tiles (x fastest, then y, then z), so the halo a
// tile shares with its neighbours is mostly fetched into the same L2.  It is
// a bijection for any block count.
__device__ inline void xcd_tile(int& bx, int& by, int& bz)
{
    const unsigned T = gridDim.x * gridDim.y * gridDim.z;
    const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned q = T / 8, r = T % 8, x = b % 8;
    const unsigned lin = x * q + (x < r ? x : r) + b / 8;
    bx = (int)(lin % gridDim.x);
    by = (int)((lin / gridDim.x) % gridDim.y);
    bz = (int)(lin / (gridDim.x * gridDim.y));
}

// cavity of the block at z index bzg and its z index within the cavity;
// false when the cavity takes no part in the launch
__device__ inline bool bv_enter_at(const BV& v, int bzg, int& cav, int& bz, GridD& g)
{
    if (v.one) {
        cav = 0;
        bz = bzg;
        g = v.g1;
        return g.dim != 0 && (!v.act || v.act[0]);
    }
    cav = bzg / v.zb;
    bz = bzg - cav * v.zb;
    // both table reads are issued before either is tested, so a block pays
    // one memory latency for them
    g = v.g[cav];
    const bool on = !v.act || v.act[cav];
    return on && g.dim != 0;
}

// cavity of this block and the block's z index within it; false when the
// cavity takes no part in the launch
__device__ inline bool bv_enter(const BV& v, int& cav, int& bz, GridD& g)
{
    if (v.one) {
        cav = 0;
        bz = blockIdx.z;
        g = v.g1;
        return g.dim != 0 && (!v.act || v.act[0]);
    }
    cav = blockIdx.z / v.zb;
    bz = blockIdx.z - cav * v.zb;
    // both table reads are issued before either is tested, so a block pays
    // one memory latency for them
    g = v.g[cav];
    const bool on = !v.act || v.act[cav];
    return on && g.dim != 0;
}

struct Level {
    GridD gmax;              // largest extents over the batch (launch grids)
    long nu = 0;             // unknowns over the batch (arena length)
    int cur = 0;             // buffer holding the current iterate
    // FP64 arenas
    double* xb[2] = {nullptr, nullptr};  // double-buffered iterate
    double* b = nullptr;     // right-hand side
    double* r = nullptr;     // residual scratch
    double* beta = nullptr;  // face viscosity (tensor problem only)
    // FP32 arenas of the mixed-precision correction cycles
    float* fx[2] = {nullptr, nullptr};
    float* fb = nullptr;
    float* fr = nullptr;
    float* fbeta = nullptr;
    // device tables (nb entries)
    GridD* gall = nullptr;   // cavities that have this level
    GridD* gsm = nullptr;    // cavities that smooth here (not their coarsest level)
    long* o = nullptr;       // component-array offsets (cells or nodes)
    long* of = nullptr;      // face-array offsets
    long* ou = nullptr;      // unknown offsets (ncomp * o)
    long* nuc = nullptr;     // unknowns per cavity
    // host copies
    std::vector<GridD> hg;   // per cavity grid (dim == 0: absent)
    std::vector<long> ho, hof, hou, hnu;
    bool any_sm = false, any_cs = false;   // some cavity smooths here / is at its coarsest
    int tile = 0;            // smoother tile candidate chosen by the autotuner
    int sweeps = 1;          // 2D tensor problem: sweeps per launch of that candidate
    double* X() const { return xb[cur]; }
};

// the arenas of a level in storage precision R
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

// coarsest-level description of one cavity (device table)
struct CoarseD {
    int lev;        // its coarsest level
    int N;          // unknowns there
    long aoff;      // offset of its N x N matrix in the A / Ainv arenas
    long poff;      // offset of its pivots
    long xoff;      // offset of its unknowns in that level's arenas
};

// what the batched assembly of a cavity's dense coarsest tensor matrix
// needs: the coarsest grid, the offset of its face viscosities in that
// level's arena, the matrix offset and size, and the cavity's unit vectors
struct DenseD {
    GridD g;
    const double* beta;
    long aoff;
    int N;
    const double* E;
};

// one level of a cavity's coarse tail (hb_tail.hip): its grid, LDS layout
// (offsets in storage elements) and the offset of its face arrays
struct TailLevel {
    int n[3], per[3];
    int nc, ns, nf;           // cells, halo positions per component, faces
    int xoff, boff, foff;     // LDS offsets of iterate, right-hand side, faces
    long gofs;                // face offset of the cavity in the level arena
    double h;
};
struct TailPlan {
    int nl = 0;               // levels in the tail (0: the cavity ends above it)
    int roff = 0;             // LDS offset of the residual scratch
    long o0 = 0;              // component-array offset of the cavity at the first level
    TailLevel lv[kMaxTail];
};

struct MG {
    int op = 0;
    int nlev = 0;            // levels of the deepest cavity
    int ncomp = 1;           // components per cell (tensor problem: dim)
    Level L[kMaxLev];
    std::vector<int> nlevc;  // levels per cavity
    std::vector<CoarseD> hcs;
    CoarseD* cs = nullptr;   // device copy
    DenseD* dd = nullptr;    // tensor problem: per-cavity dense assembly table
    int ncmax = 0;           // largest coarsest system
    double* A = nullptr;     // coarsest dense matrices -> LU factors (arena)
    int* piv = nullptr;
    double* Ainv = nullptr;  // their inverses
    double* lvl0_b = nullptr;  // level-0 right-hand side arena
    double* etae = nullptr;    // tensor problem: eta/Re per fine cell (arena)
    float* etae32 = nullptr;   // its FP32 copy
    bool f32_ready = false;    // FP32 coefficient copies match the FP64 ones
    SegV seg0;                 // level-0 unknowns as a segmented vector
    // levels 1.. of a V-cycle captured once per precision as a HIP graph and
    // replayed (index 0: FP64, 1: FP32)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gnu1[2] = {-1, -1}, gnu2[2] = {-1, -1};
    bool gfail[2] = {false, false};
    bool capturing = false;
    // level 0's iterate is zero (a preconditioner cycle): the first sweep
    // takes zeros instead of reading it, so the buffer need not be cleared
    bool zero0 = false;
    // levels tail_lt.. of a V-cycle run by one workgroup per cavity in LDS
    // (-1: none); its dynamic LDS bytes per precision
    int tail_lt = -1;
    size_t tail_lds[2] = {0, 0};
    TailPlan* tplan = nullptr;    // per cavity (device)
    int rec = S_REC_MAC;          // first slot of this operator's solve record
};

// one cavity of a context: its descriptors and the step's scratch
struct Cav {
    hb_grid grid;
    hb_fluid fluid;
    GridD g;
    FluidD fl;
    int dim = 2;
    long nc = 0, nn = 0, nf = 0;
    double ulid = 0.0;
    double step_dt = 0.0;   // dt of the last step (host copy)
    double* sc = nullptr;    // its scalar slots (device)
    double* hsc = nullptr;   // their pinned host mirror
    double *eta = nullptr, *E = nullptr, *Gp = nullptr, *F = nullptr, *S = nullptr, *trans = nullptr;
    double *uhat = nullptr, *qhat = nullptr, *qLf = nullptr, *qRf = nullptr, *uadv = nullptr, *umac = nullptr;
    double *macrhs = nullptr, *rnode = nullptr, *conv = nullptr, *rhs = nullptr;
    double* dense_E = nullptr;   // unit vectors for the dense coarsest assembly
    // views into the solve arenas
    double *macphi = nullptr, *ustar = nullptr, *phi = nullptr;
};

// Per-cavity arguments of the step's stage kernels (viscosity, face
// coefficients, Godunov prediction, MAC correction, projection right-hand
// side and update), one entry per cavity in a device table built at context
// creation: each stage kernel runs over all cavities in one launch, block z
// = (cavity, axis for face loops, z plane).
struct CavK {
    GridD g;
    FluidD fl;
    double ulid;
    long nc, nf, nn;
    double* sc;   // the cavity's scalar slots
    double *eta, *E, *Gp, *F, *S, *trans, *uhat, *qhat, *qLf, *qRf, *uadv, *umac, *macrhs, *rnode, *rhs, *ustar, *phi;
    double* macphi;             // MAC potential (view into the MAC arena)
    double *beta0, *etae;       // level-0 face viscosities and eta/Re (viscous arenas)
    double *macb, *nodb, *viscb;   // level-0 right-hand sides of the MAC, nodal and viscous problems
};

// Per-call arrays and scalars of each cavity, uploaded once per call
struct CavIO {
    const double* u;       // velocity: viscosity and advection input
    double* p;             // pressure (the projection overwrites it)
    const double* eta;     // viscosity the face coefficients come from
    double* b;             // advection output; the viscous solve's right-hand side
    double* conv;          // optional convective term
    const double* ustar;   // projection input
    double* uout;          // projection output
    double dt;             // time step
    double vdt;            // the viscous operator's coefficient (2 theta dt)
};

// one cavity's face-viscosity restriction from level l - 1 to level l
// (gc.dim == 0: the cavity has no level l)
struct RFace {
    GridD gf, gc;
    const double* bf;
    double* bc;
};

// HIP-event timing of every launch of one kernel (measurement support)
struct KTimer {
    bool on = false;
    int period = 1;             // time every period-th candidate launch
    long seen = 0;              // candidate launches since enabling
    int cap = 0, n = 0;
    hipEvent_t* ev = nullptr;   // 2 * cap events: start/stop pairs
    long launches = 0;
    double ms = 0.0, bytes = 0.0;
};

struct Ctx {
    hb_step_opts opts;
    hipStream_t s = nullptr;      // the library's own stream (all work runs here
                                  // but the factorisation below)
    hipStream_t user = nullptr;   // the caller's stream, ordered with s by events
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // the per-step dense coarsest factorisation of the tensor problem runs on
    // s2, overlapping the advection stage on s: ev_f0 (on s) orders it after
    // the coefficients, ev_f1 (on s2) orders the viscous solve after it
    hipStream_t s2 = nullptr;
    hipEvent_t ev_f0 = nullptr, ev_f1 = nullptr;
    bool visc_factor_pending = false;
    // stage-kernel tables: per cavity (constant), per call (uploaded from the
    // pinned staging buffer hio, two halves used in turn), the face-viscosity
    // restrictions per level, and the largest cell, face and node extents over
    // the cavities (the launch grids)
    CavK* ck = nullptr;
    CavIO* cio = nullptr;
    CavIO* hio = nullptr;
    int io_half = 0;
    RFace* rface = nullptr;   // [level - 1][cavity]
    std::vector<std::array<int, 3>> rfx;   // per level: largest coarse face extents
    int cx[3] = {1, 1, 1}, fx[3] = {1, 1, 1}, nx[3] = {1, 1, 1};
    int nb = 1;                   // cavities
    int dim = 2;                  // common dimension
    std::vector<Cav> cv;
    MG visc, mac, nodal;
    // solve arenas over the batch (offsets from the level-0 tables)
    double *macphi = nullptr, *ustar = nullptr, *phi = nullptr;
    double* uold = nullptr;   // steady-state driver: u before the step (allocated on first use)
    // Krylov vectors (tensor problem, arena layout)
    double *kr = nullptr, *krh = nullptr, *kp = nullptr, *kv = nullptr, *kph = nullptr, *ks = nullptr,
           *ksh = nullptr, *kt = nullptr;
    double* sc = nullptr;        // device scalar slots, S_NSLOT per cavity
    double* hsc = nullptr;       // pinned host mirror (coherent, device-mapped)
    unsigned long long* hseq = nullptr;   // pinned word the device sets after publishing the slots
    double* dhsc = nullptr;               // device addresses of hsc and hseq
    unsigned long long* dhseq = nullptr;
    unsigned long long pub = 0;           // last publication number
    // active counts published by the convergence kernels: entry seq % kRing
    // holds (count << 32) | (seq & 0xffffffff) (pinned, device-mapped)
    unsigned long long* hring = nullptr;
    unsigned long long* dring = nullptr;
    unsigned long long cseq = 0;          // last check point number
    // a max-norm final pass deferred to the next convergence check
    // (single-cavity contexts): requested by defer_mf, held in mf_slot
    bool defer_mf = false;
    int mf_slot = -1;
    const int* mf_act = nullptr;
    double wait_s = 0.0;                  // host time spent waiting for the device (HB_STATS=1)
    long waits = 0;
    double* partial = nullptr;   // reduction partials (3 x kRedBlocks per cavity)
    unsigned long long* mpart = nullptr;   // max-norm partials (kSubMax per cavity, kept zero between uses)
    int* act = nullptr;          // device active flags (nb)
    int* hact = nullptr;         // pinned host staging of the flags
    int* act2 = nullptr;         // second flag set (cavities finishing at a half step)
    int* hact2 = nullptr;
    int* sel = nullptr;          // per cavity buffer choice (device) and staging
    int* hsel = nullptr;
    // what each device flag array holds (uploads are skipped when unchanged)
    std::vector<int> dact, dact2, dsel;
    KTimer ktm;                  // timing of the finest tensor smoother launches
    // learned warm start of the nodal solve and training-data capture
    struct NNet* ws = nullptr;
    float *ws_in = nullptr, *ws_out = nullptr;   // cell fields of the network
    double *ws_y = nullptr, *ws_z = nullptr, *ws_x1 = nullptr;   // node fields
    bool cap = false;
    double *cap_r0 = nullptr, *cap_e = nullptr, *cap_x0 = nullptr;
    // the same for the viscous solve ([dim][cells] layout)
    bool capv = false;
    double *capv_r0 = nullptr, *capv_e = nullptr, *capv_x0 = nullptr;
    long ws_report_used = 0;      // solves that started from the network's guess
    size_t lds_budget = 0;        // dynamic LDS bytes one workgroup may use
    bool tail = false;            // coarse levels in one single-workgroup launch
    bool fuse = true;             // fused-colour nodal sweeps
    int fine3 = 0;                // finest 3D tensor smoother variant
    bool graph = false;           // coarse levels replayed as a captured graph
    std::string err;
};

// next start/stop event pair of the kernel timer, counting one launch of
// `bytes` algorithmic bytes
void kt_pair(Ctx* c, hipEvent_t* start, hipEvent_t* stop, double bytes);
// grid descriptor check of hb_create (message, or nullptr when valid), and
// the thread's message for calls without a context (hb_last_error(NULL))
const char* check_grid(const hb_grid* grid);
void set_global_error(const char* msg);
void kt_harvest(Ctx* c);

// ---- launch helpers --------------------------------------------------------
inline dim3 grid3(int ex, int ey, int ez, dim3 blk) { return dim3((ex + blk.x - 1) / blk.x, (ey + blk.y - 1) / blk.y, ez); }
constexpr int kRedBlocks = 512;   // fixed block count per cavity: deterministic sums
constexpr int kSubMax = 1024;     // max-norm partial words per cavity

// Max-norm partial of one block of cavity cav (bit pattern of |v|, as
// abits): the blocks of a cavity spread their atomics over kSubMax words, so
// thousands of blocks do not queue on one address; launch_max_final then
// combines the words into the cavity's slot and clears them.
__device__ inline void max_partial(unsigned long long* mp, int cav, long blk, unsigned long long m)
{
    if (m) atomicMax(mp + (long)cav * kSubMax + (blk & (kSubMax - 1)), m);
}
void launch_max_final(Ctx* c, const int* act, int slot);

// ---- reductions and vector kernels (hb_reduce.hip) -------------------------
// single-array forms, result into slot of cavity cav
void red_maxabs(Ctx* c, int cav, const double* v, long n, int slot);
void red_maxdiff(Ctx* c, int cav, const double* a, const double* b, long n, int slot);
// yield test per cell (hb_visc.hip): mask (nullable), count of yielded cells
// added to *count, largest stress magnitude max-reduced into *maxtau
void launch_yield(Ctx* c, const Cav& v, const double* u, unsigned char* mask, double* count, double* maxtau);
// grid sequencing (hb_seq.hip): velocity and pressure of grid gc carried to
// gf, the grid refined by two along every used axis
void launch_refine_state(Ctx* c, const GridD& gc, const GridD& gf, const double* uc, const double* pc, double* uf,
                         double* pf);
void set_slot(Ctx* c, int cav, int slot, double v);
// true when this finest-level smoother launch is to be timed (the timer is
// on and the launch is the period-th since the last timed one)
inline bool kt_take(Ctx* c)
{
    KTimer& k = c->ktm;
    return k.on && (k.seen++ % k.period) == 0;
}
// per-cavity int flags host -> device (in kernel arguments up to kFlagArgs
// cavities, else a copy from the pinned host array)
constexpr int kFlagArgs = 64;
struct FlagArgs {
    int n;
    int v[kFlagArgs];
};
void set_flags(Ctx* c, int* dev, const int* host);
void fetch_slots(Ctx* c);  // all slots to c->hsc once the stream's work so far has completed
// launch the convergence kernel of a check point; publish (a.seq != 0) the
// number of cavities still active
void launch_conv(Ctx* c, ConvArgs a);
// launch a deferred max-norm final pass that no check consumed
void flush_max_final(Ctx* c);
// BiCGStab: x += alpha ph, r = s (cavities finishing at the half step); and
// x += alpha ph + omega sh, r = s - omega t with max|r| into slot mslot
void bicg_half_finish(Ctx* c, const SegV& s, double* x, const double* ph, double* r, const double* sv);
// omega from the partials of t.t and t.s, x += alpha ph + omega sh, r = s -
// omega t with its max-norm into mslot, and the partials of the next rho
void bicg_full_update(Ctx* c, const SegV& s, double* x, const double* ph, const double* sh, double* r,
                      const double* sv, const double* t, int mslot, const double* part, const double* rh,
                      double* rpart);
// wait until check point seq has published; returns its active count (-1
// if it never did, even after a stream synchronisation)
int wait_active(Ctx* c, unsigned long long seq);
void copy(Ctx* c, double* dst, const double* src, long n);
void fill(Ctx* c, double* dst, double v, long n);
// segmented forms over the batch (per cavity slot, inactive cavities skipped)
void seg_maxabs(Ctx* c, const SegV& s, const double* v, int slot);
void seg_maxabs2(Ctx* c, const SegV& s, const double* a, int slot0, const double* b, int slot1);
void seg_set_zero(Ctx* c, int slot);                       // every cavity
void seg_dot(Ctx* c, const SegV& s, const double* a, const double* b, int slot);
// partial pass only: a.b0 (and a.b1) per block into part, clearing slot
// `zero` (-1: none); the kernel that uses the product totals the partials
void seg_dot_part(Ctx* c, const SegV& s, const double* a, const double* b0, const double* b1, double* part, int zero);
double* rho_partials(Ctx* c);   // partials of BiCGStab's rho (the third row block of c->partial)
void seg_sub_mean(Ctx* c, const SegV& s, double* v);
void seg_copy(Ctx* c, const SegV& s, double* dst, const double* src);
void seg_fill(Ctx* c, const SegV& s, double* dst, double v);
void seg_copy_sel(Ctx* c, const SegV& s, double* dst, const double* src0, const double* src1, const int* sel);
void seg_to_f32(Ctx* c, const SegV& s, const double* src, float* dst, float* zero);
void seg_add_f32(Ctx* c, const SegV& s, double* x, const float* e);
void seg_from_f32(Ctx* c, const SegV& s, const float* e, double* x);
void flat_to_f32(Ctx* c, const double* src, float* dst, long n);
// device-scalar BiCGStab steps (scalars in each cavity's slots S_RHO .. S_BETA)
void bicg_init_scalars(Ctx* c, const int* act);
// rho and beta from rho's partials, p = r + beta (p - omega v)
void bicg_p_rho(Ctx* c, const SegV& s, double* p, const double* r, const double* v, const double* part);
// alpha from the partials of r^.v, s = r - alpha v with its max-norm into mslot
void bicg_s_alpha(Ctx* c, const SegV& s, double* out, const double* r, const double* v, const double* part, int mslot);

// ---- viscosity and tensor operator, per cavity (hb_visc.hip) ----------------
void launch_viscosity(Ctx* c, const Cav& v, const double* u, double* eta);
void launch_visc_dense(Ctx* c, const GridD& g, const double* beta, double dt, int N, const double* E, double* A);
void launch_visc_dense_batch(Ctx* c, const MG& m);

// ---- LDS-tiled tensor kernels, batched (hb_tile.hip) ------------------------
// R = storage and arithmetic precision of the cycle; fine = coef is eta/Re
// per cell (else the level's face viscosities).  dt is read from each
// cavity's slot S_DT, so a captured graph stays valid across steps.
template <typename R>
void launch_tsmooth(Ctx* c, const Level& L, const BV& v, const R* coef, bool fine, int comp, const R* xcur, R* xnext,
                    const R* b);
// 2D: nsw (1 or 2) red-black sweeps of both components from xcur into
// xnext in one launch, with candidate `tile` (0 .. kSweep2Cands - 1); two
// sweeps need a candidate whose sweeps may be paired and every periodic
// extent of the level at least 8.  sweep2_shape gives a candidate's tile,
// threads and most sweeps per launch, sweep2_lds its dynamic LDS bytes.
// pe (optional): the coarse iterate of a V-cycle, whose prolongation the
// launch adds to xcur first (v then also carries the coarse level: gct/oct
// its grid and offset tables); staged candidates fold it into their fill,
// the others launch the prolongation kernel before the sweep.
struct SweepShape {
    int tx, ty, threads, nsw;
    bool staged;
};
constexpr int kSweep2Cands = 8;
// bc/xc (optional): the launch ends a pre-smoothing and also restricts the
// residual of its result to the coarse level (coarse b, coarse x = 0; v
// then also carries the coarse level), as launch_tresid_restr would after it.
template <typename R>
void launch_tsweep2(Ctx* c, const Level& L, const BV& v, const R* coef, bool fine, const R* xcur, R* xnext, const R* b,
                    int tile, int nsw, const R* pe = nullptr, const GridD* gct = nullptr, const long* oct = nullptr,
                    R* bc = nullptr, R* xc = nullptr);
SweepShape sweep2_shape(int tile);
size_t sweep2_lds(int tile, int nsw);
void sweep2_allow_lds(size_t bytes);
void tsmooth_allow_lds(size_t bytes);
template <typename R>
void launch_trb3(Ctx* c, const Level& L, const BV& v, const R* coef, bool fine, int comp, int colour, R* x, const R* b);
template <typename R>
void launch_tresid_restr(Ctx* c, const Level& L, const BV& v, const GridD* gc, const long* oc, const R* coef, bool fine,
                         const R* x, const R* b, R* bc, R* xc);
// FP64 finest-level residual r = b - A x (max-norm into each cavity's slot)
// or y = A x (b null)
void launch_tresid(Ctx* c, const Level& L, const BV& v, const double* coef, const double* x, const double* b, double* out,
                   int slot);

// ---- scalar cell problem (MAC), nodal problem, transfers, coarsest ----------
// (hb_mg.hip, hb_nodal.hip), batched
template <typename R> void launch_mac_rb(Ctx* c, const Level& L, const BV& v, int colour, R* x, const R* b);
// both colours of a red-black sweep from cur into next (hb_tile.hip)
// (2D: nsw (1 or 2) sweeps per launch, every periodic extent at least 2 nsw;
// pe: coarse iterate whose prolongation is added to cur first, v then also
// carrying the coarse level, gct/oct its tables; bc/xc: the launch ends a
// pre-smoothing and restricts the residual to the coarse level, every
// periodic extent then at least 2 nsw + 1)
template <typename R>
void launch_mac_sweep(Ctx* c, const Level& L, const BV& v, const R* cur, R* next, const R* b, int nsw = 1,
                      const R* pe = nullptr, const GridD* gct = nullptr, const long* oct = nullptr,
                      R* bc = nullptr, R* xc = nullptr);
// one thread per coarse cell: vc covers the coarse level, gf / of_ give the
// fine grid and offsets of the same cavities
template <typename R>
void launch_mac_resid_restrict(Ctx* c, const Level& C, const BV& vc, const GridD* gf, const long* of_, const R* xf,
                               const R* bf, R* bc, R* xc);
// FP64 r = b - L x (max-norm into each cavity's slot) or y = L x (b null)
void launch_mac_resid(Ctx* c, const Level& L, const BV& v, const double* x, const double* b, double* r, int slot);
void launch_mac_dense(Ctx* c, const GridD& g, int N, const double* E, double* A);
template <typename R>
void launch_prolong_cells(Ctx* c, const Level& L, const BV& v, const GridD* gc, const long* oc, int ncomp,
                          double wall_sign, const R* e, R* x);
template <typename R> void launch_nodal_gs(Ctx* c, const Level& L, const BV& v, int colour, R* x, const R* b);
// nsw (1, or 2 in 2D with every periodic extent at least 8) whole
// Gauss-Seidel sweeps from cur into next (one launch; 3D: one sweep, two launches),
// with candidate tile `tile` (0 .. kNodalCands - 1); nodal_sweep_tile gives
// its extents and thread count
// (2D: pe folds the prolongation of the coarse iterate in, bc/xc the
// residual restriction to the coarse level, v then also carrying the coarse
// level, gct/oct its tables; every periodic extent at least the halo:
// 4 nsw, or 4 nsw + 2 with the restriction)
template <typename R>
void launch_nodal_sweep(Ctx* c, const Level& L, const BV& v, const R* cur, R* next, const R* b, int tile,
                        int nsw = 1, const R* pe = nullptr, const GridD* gct = nullptr, const long* oct = nullptr,
                        R* bc = nullptr, R* xc = nullptr);
void nodal_sweep_tile(int dim, int tile, int* tx, int* ty, int* threads);
constexpr int kNodalCands = 4;
// r = b - K x (slot >= 0: FP64 only, max-norm into each cavity's slot) or y = K x (b null)
template <typename R>
void launch_nodal_resid(Ctx* c, const Level& L, const BV& v, const R* x, const R* b, R* r, int slot);
template <typename R>
void launch_nodal_restrict(Ctx* c, const Level& C, const BV& vc, const GridD* gf, const long* of_, const R* rf, R* bc,
                           R* xc);
template <typename R>
void launch_nodal_prolong(Ctx* c, const Level& L, const BV& v, const GridD* gc, const long* oc, const R* e, R* x);
void launch_nodal_dense(Ctx* c, const GridD& g, int N, const double* E, double* A);
void launch_add_ones(Ctx* c, int N, double* A);
void launch_lu_factor(Ctx* c, int N, double* A, int* piv);
void launch_lu_inverse(Ctx* c, int N, const double* LU, const int* piv, double* Ainv);
void launch_dense_inverse(Ctx* c, int N, double* A, int* piv, double* Ainv);
void launch_gj_inverse_batch(Ctx* c, const MG& m);
// x = A^{-1} b for the cavities whose coarsest level is lev (FP64 accumulation)
template <typename R>
void launch_coarse_solve(Ctx* c, const MG& m, int lev, const int* act, const R* b, R* x);
void launch_identity(Ctx* c, int N, double* E);
// the coarse end of a V-cycle from level lt in one launch (hb_tail.hip)
size_t tail_plan(int op, const std::vector<GridD>& levels, const std::vector<long>& gofs, long o0, size_t elem,
                 TailPlan* out);
template <typename R>
void launch_visc_tail(Ctx* c, const MG& m, int lt, int nu1, int nu2, size_t lds, const int* act);
template <typename R>
void launch_mac_tail(Ctx* c, const MG& m, int lt, int nu1, int nu2, size_t lds, const int* act);
template <typename R>
void launch_nodal_tail(Ctx* c, const MG& m, int lt, int nu1, int nu2, size_t lds, const int* act);
void tail_allow_lds(size_t bytes);

// ---- learned warm start (hb_nn.hip, hb_ws.hip) --------------------------------
struct NNet;
int nn_infer(NNet* t, const float* x, int n, int H, int W, float* y);   // device fp32 in/out, synchronous
NNet* nn_of(hb_nn* nn);
int nn_channels_in(const NNet* t);
int nn_channels_out(const NNet* t);
// cell value = scale * mean of its 2^d corner nodes (2D), fp32 [ny][nx]
void launch_node_to_cell(Ctx* c, const GridD& g, const double* v, double scale, float* out);
// node value = mean of the cells around it (2D)
void launch_cell_to_node(Ctx* c, const GridD& g, const float* v, double* out);
void launch_axpy(Ctx* c, double* y, const double* x, const double* a, double s, long n);   // y = x + s a

// ---- step stages, per cavity (hb_step.hip) ----------------------------------
// stage kernels over every cavity (tables c->ck and c->cio)
void stage_grad_node(Ctx* c);                 // Gp = G p
void stage_forcing(Ctx* c);
void stage_slopes(Ctx* c);
void stage_trace_normal(Ctx* c);
void stage_transverse(Ctx* c);
void stage_trace_full(Ctx* c);
void stage_mac_div(Ctx* c, int after);        // after: div of u^MAC into macrhs, else of u^adv into the MAC rhs
void stage_mac_update(Ctx* c);
void stage_advect_rhs(Ctx* c);
void stage_proj_rhs(Ctx* c);
void stage_weak_div_u(Ctx* c);                // rnode = weak div of uout
void stage_proj_update(Ctx* c);
void stage_viscosity(Ctx* c);                 // eta = eta(u)
void stage_visc_coef(Ctx* c);                 // eta/Re, level-0 faces, coefficient slot
void stage_restrict_faces(Ctx* c, int level);
void stage_visc_div(Ctx* c);                  // E = div(eta_e gamma_dot(u)) with the cavity's faces
void stage_visc_wall_rhs(Ctx* c);             // viscous level-0 rhs = b + wall terms
// field selectors of the stage copies and max-norms
enum StageField { SF_U, SF_P, SF_UOUT, SF_RNODE, SF_MACRHS, SF_USTAR, SF_PHI };
void stage_copy(Ctx* c, int dst, int src);    // SF_USTAR <- SF_U, SF_PHI <- SF_P, SF_P <- SF_PHI
void stage_maxabs(Ctx* c, int field, int slot);

}  // namespace hb
