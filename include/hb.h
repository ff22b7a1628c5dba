/*
 * hb.h -- C ABI of the MI355X (gfx950) library for one semi-implicit time
 * step of the Papanastasiou-regularised Herschel-Bulkley incompressible flow
 * solver of Sverdrup, Nikiforakis & Almgren, arXiv 1803.00417.
 *
 * The step (Sec. III.A) on one uniform level of a structured grid:
 *   1. strain rate and regularised apparent viscosity
 *      (eq:rheology:papanastasiou in the dimensionless form
 *       eq:dimensionless:herschel-bulkley, Sec. IV);
 *   2. second-order Godunov prediction of face states at t^{m+1/2}
 *      (Taylor extrapolation with Colella's limited slopes, transverse terms,
 *       eq:iamr:extrap) and upwinding by a projected face velocity;
 *   3. the coupled tensor viscous (Helmholtz) solve with the lagged viscosity
 *      eta^m (Crank-Nicolson);
 *   4. the approximate nodal projection and pressure update.
 * Both solves use geometric multigrid V-cycles run by HIP kernels.
 *
 * Memory.  Every array argument is caller-owned DEVICE memory (e.g. a torch
 * CUDA/HIP tensor), contiguous FP64, x fastest, without ghost cells:
 *   cell field with C components : [C][nz][ny][nx]      (nz = 1 in 2D)
 *   nodal field                  : [nnz][nny][nnx], nn_a = n_a + 1 on wall
 *                                  axes, n_a on periodic axes, 1 on unused axes
 *   face fields (umac)           : one array per axis, concatenated; the
 *                                  array of axis a has n_a + 1 (wall) or n_a
 *                                  (periodic) faces along a and n_b cells
 *                                  along the other axes.
 * The library owns only the scratch it allocates: in hb_create (multigrid
 * hierarchies, face arrays, reduction buffers: everything hb_step and the
 * per-stage calls use) and, on their first use on a context, in the calls
 * that need more: hb_run_steady and hb_run_cessation (one velocity-sized
 * buffer), hb_set_warm_start (the network's input, output and node fields),
 * hb_capture (three fields of the captured solve); a network allocates its
 * activations in hb_nn_forward/grad/train_step for each new (n, H, W).  Such
 * an allocation is all or nothing (a failure frees what it had allocated
 * and returns HB_ERR_OOM).  The library never frees caller memory.
 * hb_cfl_dt_noalloc allocates nothing at all.
 *
 * Streams.  Work runs asynchronously on the hipStream_t given to hb_create
 * (NULL = the default stream): each call orders the library's internal
 * streams after the work already on it and orders that stream after the
 * call's results.  One internal stream carries the step; a second one runs
 * the per-step dense factorisation of the viscous coarsest level beside the
 * advection stage, joined before the viscous solve.  Multigrid convergence is decided on the
 * device: after each V-cycle (or BiCGStab half step) a small kernel tests
 * the residual and stops the cavity, and the cycle kernels skip stopped
 * cavities; the host only waits for the active count one check point late,
 * so the GPU always has the next cycle queued.  A call reads its outcome
 * (return code, report) once at its end, and a step whose dt comes from the
 * CFL condition reads max |u| once at its start; both synchronise.  A solve
 * that meets a non-finite value leaves the outputs of that call undefined
 * (the call returns HB_ERR_NONFINITE).
 *
 * Errors.  Functions return HB_OK or a negative code; nothing throws or
 * aborts across the ABI.  Arguments are checked before any device work.
 * hb_last_error gives a message for the last failing call on a context (or,
 * with ctx == NULL, for the last failing hb_create on this thread).
 */
#ifndef HB_H
#define HB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HB_OK = 0,
    HB_ERR_ARG = -1,        /* invalid argument; nothing was launched */
    HB_ERR_DEVICE = -2,     /* a HIP call failed */
    HB_ERR_NOCONV = -3,     /* a solve hit max_cycles; outputs hold the last iterate */
    HB_ERR_NONFINITE = -4,  /* NaN/Inf in an input or produced by a solve */
    HB_ERR_OOM = -5,        /* a device allocation failed (hb_create, or a call's first use) */
    HB_ERR_IO = -6          /* a checkpoint file could not be opened, read or written */
};

enum { HB_BC_WALL = 0, HB_BC_PERIODIC = 1 };

/* Regularisation: PAPER multiplies the whole apparent viscosity by
 * (1 - exp(-Pa |gamma_dot|)) as printed (eq:rheology:papanastasiou);
 * YIELD_ONLY applies the factor to the yield-stress term only (needs n >= 1),
 * which gives exactly eta = 1 for HB = 0, n = 1 (the Newtonian limit). */
enum { HB_REG_PAPER = 0, HB_REG_YIELD_ONLY = 1 };

enum { HB_OP_VISC = 0, HB_OP_NODAL = 1, HB_OP_MAC = 2 };

enum { HB_PREC_FP64 = 0, HB_PREC_MIXED = 1 };

/* Grid: n[a] cells per axis (n[2] = 1 when dim = 2), uniform spacing h.
 * Each n[a] (a < dim) must be c * 2^k with c in {1, 2, 3} and n[a] >= 4.
 * bc[a][side]: HB_BC_WALL or HB_BC_PERIODIC; periodic faces come in pairs.
 * wall_u[a][side][c]: velocity of a wall face (lid), component c. */
typedef struct {
    int32_t dim;
    int32_t n[3];
    double h;
    int32_t bc[3][2];
    double wall_u[3][2][3];
} hb_grid;

/* Fluid: dimensionless groups Re, HB (Herschel-Bulkley number), n (flow
 * index), Pa (Papanastasiou number) of Sec. IV; constant body force f. */
typedef struct {
    double Re, HB, n, Pa;
    int32_t reg;
    double f[3];
} hb_fluid;

/* Multigrid options.  A solve stops when |b - A x|_inf <= tol_rel |b|_inf
 * (checked before the first cycle and after each); fixed_cycles = 1 runs
 * exactly max_cycles V-cycles.  krylov = 1 wraps the V-cycle in BiCGStab
 * (one V-cycle per preconditioner application).  precision: HB_PREC_FP64
 * runs every cycle in FP64; HB_PREC_MIXED runs each V-cycle in FP32 (FP32
 * copies of the coefficients, smoothing, transfers) on the FP64 residual and
 * adds the correction to the FP64 iterate (defect correction); the residual,
 * the convergence test, the viscosity and the coarsest dense solve stay FP64,
 * so the tolerance means the same in both modes. */
typedef struct {
    double tol_rel;
    int32_t max_cycles, fixed_cycles, nu1, nu2, krylov, precision;
} hb_mg_opts;

typedef struct {
    int32_t cycles;      /* V-cycles run */
    double rel_resid;    /* |b - A x|_inf / |b|_inf at exit */
    double bnorm;        /* |b|_inf of the system solved */
} hb_mg_report;

/* Step options.  pred_visc and theta choose between readings of Sec. III.A:
 *   pred_visc = 1 puts the explicit stress divergence 2E into the forcing of
 *     the Taylor prediction of the face states, as eq:iamr:extrap prints it;
 *     0 (default) predicts with -G p + f only.  With 2E the face states take
 *     (dt/2) div tau^m, which is unstable once the diffusion number
 *     dt eta/(Re h^2) is large (a Newtonian Re = 1 cavity at dt = h/2 from
 *     16^2, and the Bingham Re = 1 cavity of Sec. IV), so it is off by default.
 *   theta is the implicit weight of the viscous update: 0.5 (or 0) is the
 *     Crank-Nicolson update printed in Sec. III.A, 1 backward Euler;
 *     0.5 <= theta <= 1.  The solve is (I - 2 theta dt div(eta/Re
 *     gamma_dot(.))) u* = b with 2 (1 - theta) dt E in b.  Crank-Nicolson is
 *     not L-stable: with the lagged, strongly varying viscosity of a yield-
 *     stress fluid its stiff modes keep the velocity changing by about 1e-2
 *     per step at Re = 1, so runs to a steady state there use theta = 1. */
typedef struct {
    double cfl;          /* dt = cfl h / max(U_wall, max |u|) when dt <= 0 */
    int32_t mac_project; /* 1: project the face advection velocity (default) */
    hb_mg_opts mac, visc, proj;
    int32_t pred_visc;   /* 1: explicit stress divergence in the predictor forcing */
    double theta;        /* implicit weight of the viscous update (0: 0.5) */
} hb_step_opts;

typedef struct {
    double dt, max_u;
    double div_mac_rel;  /* |D_mac u^MAC|_inf / |D_mac u^adv|_inf */
    double div_node;     /* max_k |weak div(u^{m+1})_k| / h^d */
    hb_mg_report mac, visc, proj;
} hb_step_report;

typedef struct hb_ctx hb_ctx;

/* Create a context for one grid, fluid and option set; allocates every
 * device buffer the step needs on the current device.  hip_stream: a
 * hipStream_t (NULL: default stream).  Returns HB_ERR_ARG for an invalid
 * descriptor, HB_ERR_OOM / HB_ERR_DEVICE on HIP failures. */
int hb_create(const hb_grid* grid, const hb_fluid* fluid, const hb_step_opts* opts,
              void* hip_stream, hb_ctx** out);
void hb_destroy(hb_ctx* ctx);
const char* hb_last_error(const hb_ctx* ctx);

/* Regularised apparent viscosity per cell (Sec. III.B, Sec. IV):
 *   g = |gamma_dot|, gamma_dot = (grad u + grad u^T)/2 by centred differences
 *   with wall ghosts (odd reflection about the wall velocity);
 *   PAPER:      eta = (g^n + HB/2) (1 - exp(-Pa g)) / g   (bounded: HB Pa/2 at g = 0)
 *   YIELD_ONLY: eta = g^(n-1) + (HB/2) (1 - exp(-Pa g)) / g.
 * u: [dim][cells] in, eta: [cells] out (dimensionless, not divided by Re). */
int hb_viscosity(hb_ctx* ctx, const double* u, double* eta);

/* One multigrid solve on the context's grid (Sec. III.A):
 *   HB_OP_VISC : (I - dt div(eta/Re gamma_dot(.))) x = rhs with the grid's
 *                wall velocities; eta [cells] is the dimensionless viscosity;
 *                x, rhs: [dim][cells];
 *   HB_OP_NODAL: K x = rhs, K the Q1 stiffness (Neumann); rhs [nodes] has its
 *                mean removed, x is returned with zero mean;
 *   HB_OP_MAC  : L_mac x = rhs (cell-centred, zero wall flux), same mean rules.
 * x: in initial guess, out solution (last iterate on HB_ERR_NOCONV).
 * opts NULL: the context's option set for that operator.  report nullable. */
int hb_mg_solve(hb_ctx* ctx, int op, const double* eta, double dt,
                const double* rhs, double* x, const hb_mg_opts* opts,
                hb_mg_report* report);

/* The advection stage (Sec. III.A, eq:iamr:extrap and the provisional
 * velocity): viscosity-weighted explicit term E = div(eta/Re gamma_dot(u)),
 * the Godunov prediction with forcing -G p + f (-G p + 2E + f with
 * pred_visc), the MAC projection of the face velocity, and the viscous-solve
 * right-hand side
 *   b = u - dt [u^MAC . grad u~] + dt (-G p + 2 (1 - theta) E + f).
 * u: [dim][cells], p: nodes, eta: [cells] (from hb_viscosity), b: [dim][cells]
 * out.  umac (faces), conv ([dim][cells], the convective term) nullable. */
int hb_advect(hb_ctx* ctx, const double* u, const double* p, const double* eta,
              double dt, double* b, double* umac, double* conv,
              hb_mg_report* mac_report);

/* Approximate projection (Sec. III.A, the projection step and pressure
 * update that close the algorithm): V = ustar/dt + G p; K phi = weak div V;
 * u = ustar + dt (G p - G phi); p = phi (mean zero).  The printed velocity
 * update has no + dt G p term, which would leave D u = -dt D G p; with it, u
 * is dt times the projection of V.
 * ustar [dim][cells] in, p nodes in/out, u [dim][cells] out (may alias
 * ustar). */
int hb_project(hb_ctx* ctx, const double* ustar, double* p, double dt, double* u,
               hb_mg_report* report);

/* dt from the CFL condition: cfl h / max(max wall speed, max |u|).  The
 * paper fixes no time-step rule (it notes only that the step shrinks with
 * the grid spacing, Sec. III.C, and times runs at constant dt, Sec. V);
 * this advective CFL bound is the library's rule for dt <= 0. */
int hb_cfl_dt(hb_ctx* ctx, const double* u, double* dt_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the value
 * of hb_cfl_dt without a context and without any allocation, bit for bit.
 * grid: as for hb_create (wall speeds of non-periodic faces enter U_wall);
 * u: [dim][cells] device FP64 in; dt_out: ONE device double out (caller-
 * owned), cfl h / max(U_wall, max |u|), 0 when both vanish, NaN when u holds
 * a non-finite value.  Asynchronous on hip_stream (NULL: default stream);
 * nothing is read back, so it may be captured in a graph.  Its scratch is a
 * static device array of 16384 words per GPU, shared by every call on that
 * GPU: calls that overlap on one GPU race.  HB_ERR_ARG (message in
 * hb_last_error(NULL)) for a null pointer, an invalid grid, cfl <= 0, or more
 * than 67,108,864 velocity values (dim x cells); HB_ERR_DEVICE if the
 * scratch address cannot be taken or a launch fails. */
int hb_cfl_dt_noalloc(const hb_grid* grid, double cfl, const double* u, double* dt_out, void* hip_stream);

/* One full time step of Sec. III.A in place: u^m -> u^{m+1},
 * p^{m-1/2} -> p^{m+1/2} (viscosity, advection stage, coupled viscous
 * solve, projection; the calls above in that order, on the library's own
 * buffers).  dt <= 0 selects the CFL time step.  report nullable. */
int hb_step(hb_ctx* ctx, double* u, double* p, double dt, hb_step_report* report);

/* Batched sweeps: one context holding `count` independent cavities of the
 * same dimension (each with its own grid, fluid and wall velocities; one
 * option set).  hb_step_batch advances every cavity by one step, as hb_step
 * would (u[b], p[b]: cavity b's caller-owned device arrays in the hb_step
 * layout; dt[b] <= 0 or dt NULL: cavity b's CFL step; reports: NULL or
 * `count` entries).  The three solves of all cavities run as one batched
 * multigrid: every launch covers all cavities, and each cavity stops at its
 * own tolerance.  A cavity's result does not depend on the rest of the batch.
 * The single-cavity calls above reject a context with count > 1 (HB_ERR_ARG);
 * hb_step_batch also accepts a single-cavity context.  count: 1 .. 4096. */
int hb_create_batch(const hb_grid* grids, const hb_fluid* fluids, int count, const hb_step_opts* opts,
                    void* hip_stream, hb_ctx** out);
int hb_batch_size(const hb_ctx* ctx);
int hb_step_batch(hb_ctx* ctx, double* const* u, double* const* p, const double* dt, hb_step_report* reports);

/* ---- steady state, grid sequencing, checkpoints ---------------------------
 * Steadiness (Sec. III.A, the test that closes the description of the
 * projection; Sec. IV): a run is steady once the velocity's largest relative
 * change over one step is below a tolerance (1e-5 in the paper).  The
 * printed quotient divides by u^m cell by cell, undefined where u^m = 0; the
 * change used here is max|u^(m+1) - u^m| / max|u^m| (infinite while u^m is
 * zero everywhere).
 *
 * hb_run_steady: hb_step on (u, p) in place (dt <= 0: the CFL step of each
 * step, else that constant step) until the change is below tol or max_steps
 * steps have run.  Single-cavity contexts.  Returns HB_OK when steady,
 * HB_ERR_NOCONV when max_steps ran out or a solve of the last step did not
 * converge (u, p hold the last state), other codes as hb_step (the run
 * stops at the failing step).  report (nullable): steps run, steady flag,
 * simulated time of the steps that ran, last change.  The first call
 * allocates one velocity-sized device buffer, kept by the context.
 *
 * hb_refine_state (grid sequencing, Sec. III.C): the state of a run on the
 * grid one refinement below the context's (every used cell count halved,
 * spacing doubled, same boundaries) carried to the context's grid.  The
 * paper does not name the interpolation; velocity: conservative linear
 * interpolation with central slopes, child = u(C) + sum over axes (x, y, z)
 * of (+-1/4) (u(C+1) - u(C-1))/2, + on the parent's high half, a neighbour
 * beyond a wall being the wall ghost 2 u_wall - u(C) and beyond a periodic
 * face the wrapped cell; pressure: multilinear interpolation between the
 * coarse nodes.  u_coarse [dim][coarse cells], p_coarse [coarse nodes] in;
 * u, p on the context's grid out (device, caller-owned, not aliased).
 * HB_ERR_ARG if a cell count of the context's grid is odd.
 *
 * hb_run_sequenced (Sec. III.C): from rest on `coarse` to steady state, then
 * `levels` times: refine the state by two and continue to steady state
 * (tol, max_steps as hb_run_steady, CFL steps).  u, p (device, caller-owned)
 * receive the state on the finest grid; the intermediate grids' contexts and
 * arrays are created and freed inside (every level's grid must be valid for
 * hb_create).  reports: levels + 1 entries, one per grid.  A level that is
 * not steady within max_steps is refined all the same and the call returns
 * HB_ERR_NOCONV at the end; any other failure stops the run and returns its
 * code, with the message in hb_last_error(NULL).  levels: 0 .. 8.
 *
 * hb_checkpoint_write / hb_checkpoint_read: raw checkpoint of a run (the
 * restart of Sec. III.C): an 80-byte header (magic "HBCKPT", version 1,
 * dim, n[3], periodic flags[3], value counts of u and p, step, t, h) then u
 * ([dim][cells]) and p (nodes) as raw doubles in host byte order.  The
 * step carries no state beyond (u, p), so a run restarted from a checkpoint
 * continues bit for bit as the uninterrupted run.  Reading checks the header
 * against the context's grid (HB_ERR_ARG if it differs); HB_ERR_IO for a
 * file that cannot be opened, is not a checkpoint or is truncated. */
typedef struct {
    int32_t steps;   /* steps run */
    int32_t steady;  /* 1 when the last step's change was below tol */
    double t;        /* simulated time of those steps */
    double change;   /* max|u^(m+1) - u^m| / max|u^m| of the last step */
} hb_steady_report;

int hb_run_steady(hb_ctx* ctx, double* u, double* p, double tol, int max_steps, double dt, hb_steady_report* report);
int hb_refine_state(hb_ctx* ctx, const double* u_coarse, const double* p_coarse, double* u, double* p);
int hb_run_sequenced(const hb_grid* coarse, const hb_fluid* fluid, const hb_step_opts* opts, int levels, double tol,
                     int max_steps, void* hip_stream, double* u, double* p, hb_steady_report* reports);
int hb_checkpoint_write(hb_ctx* ctx, const char* path, const double* u, const double* p, int64_t step, double t);
int hb_checkpoint_read(hb_ctx* ctx, const char* path, double* u, double* p, int64_t* step, double* t);

/* ---- yield surfaces and cessation ------------------------------------------
 * Yield test (Sec. II, Sec. IV): in the dimensionless variables the stress
 * is 2 eta gamma_dot, its magnitude 2 eta g (g = |gamma_dot| as in
 * hb_viscosity, eta the regularised apparent viscosity) and the yield
 * stress HB.  A cell is yielded where 2 eta g > HB; the unyielded cells form
 * the plugs and dead zones whose boundaries are the yield surfaces.
 *
 * hb_yield: u [dim][cells] in; mask (nullable, device, caller-owned,
 * [cells] bytes) receives 1 for a yielded cell, 0 otherwise; report
 * (nullable; non-null waits for the result): the number of yielded cells,
 * the cell count and the largest stress magnitude.  Single-cavity contexts.
 *
 * hb_run_cessation (the cessation experiment of Sec. IV): from a state,
 * typically steady, of a run whose lid is then stopped, step (u, p) in
 * place on the context (create it with the walls at rest; dt <= 0: CFL
 * steps, else that constant step) until no cell is yielded, tested before
 * the first step and after each, or max_steps steps have run.  Returns
 * HB_OK once the flow has stopped, HB_ERR_NOCONV when max_steps ran out or a
 * solve of the last step did not converge, HB_ERR_ARG for HB <= 0 (no yield
 * stress, so no finite stopping), other codes as hb_step.  report
 * (nullable): steps run, stopped flag, simulated time (the cessation time
 * when stopped). */
typedef struct {
    int64_t yielded;    /* cells with 2 eta g > HB */
    int64_t cells;      /* all cells */
    double max_stress;  /* largest 2 eta g */
} hb_yield_report;

typedef struct {
    int32_t steps;    /* steps run */
    int32_t stopped;  /* 1 when no cell is yielded */
    double t;         /* simulated time of those steps */
} hb_cessation_report;

int hb_yield(hb_ctx* ctx, const double* u, uint8_t* mask, hb_yield_report* report);
int hb_run_cessation(hb_ctx* ctx, double* u, double* p, int max_steps, double dt, hb_cessation_report* report);

/* ---- learned warm start (BF16 U-Net on the matrix cores) -----------------
 * A small convolutional U-Net (4 levels, 16/32/64/64 channels, two 3x3
 * convolutions with ReLU per level, average pooling down, nearest upsampling
 * and skip concatenation up, 3x3 head) with BF16 weights and activations and
 * FP32 accumulation, trained on the GPU by the library's own forward and
 * backward kernels (MSE loss, Adam).  Tensors are device FP32, [n][H][W][C]
 * (channels fastest), H and W multiples of 8; in_ch, out_ch in 1..16.  The
 * network allocates its activation buffers for the last (n, H, W) it saw.
 * Parameters: a flat FP32 vector, layer by layer: weights [Cout][3][3][Cin]
 * then biases [Cout]; the first layer has 16 input channels (the input is
 * zero-padded) and the head 16 outputs, of which the first out_ch count. */
typedef struct hb_nn hb_nn;
int hb_nn_create(int in_ch, int out_ch, uint64_t seed, hb_nn** out);
void hb_nn_destroy(hb_nn* nn);
int64_t hb_nn_param_count(const hb_nn* nn);
int hb_nn_get_params(hb_nn* nn, float* host_out);
int hb_nn_set_params(hb_nn* nn, const float* host_in);
int hb_nn_forward(hb_nn* nn, const float* x, int n, int H, int W, float* y);
/* loss = mean over pixels and the first out_ch channels of (y - target)^2;
 * grad_host (nullable): dloss/dparams, param_count floats */
int hb_nn_grad(hb_nn* nn, const float* x, const float* target, int n, int H, int W, double* loss, float* grad_host);
int hb_nn_train_step(hb_nn* nn, const float* x, const float* target, int n, int H, int W, float lr, double* loss);

/* Warm start of the nodal projection solve (2D, cell counts multiples of 8):
 * with a network set (in_ch = out_ch = 1), each solve starts from the
 * previous pressure x0, forms r0 = b - K x0, feeds r0 / |r0|_inf averaged to
 * cells to the network, averages its output y back to nodes, scales it by the
 * least-squares factor s = (r0 . K y) / (K y . K y), and starts from
 * x0 + s y only when that lowers |b - K x|_inf (otherwise from x0).  The
 * multigrid solve and its tolerance are unchanged.  nn NULL: off.  The
 * network must outlive its use by the context.  op: HB_OP_NODAL only. */
int hb_set_warm_start(hb_ctx* ctx, int op, hb_nn* nn);
/* number of solves so far that started from the network's guess */
int hb_warm_start_uses(const hb_ctx* ctx);

/* Training and analysis data: while enabled for op (HB_OP_NODAL or
 * HB_OP_VISC), each solve of that operator on a single-cavity context
 * records its initial residual r0 = b - A x0 and its correction e = x - x0
 * (FP64; node layout, or [dim][cells] for the viscous solve, whose b holds
 * the wall terms); hb_capture_read copies the last pair to caller device
 * arrays. */
int hb_capture(hb_ctx* ctx, int op, int enable);
int hb_capture_read(hb_ctx* ctx, int op, double* r0, double* e);

/* Measurement support.  While enabled (enable = k > 0), every k-th launch
 * of the tensor viscous smoother on the finest multigrid level (k = 1: every
 * launch) is timed with events that the dispatch itself records; such a
 * launch costs the host more than a plain one, so sampling keeps the timer
 * from slowing the run it measures (2D: one red-black sweep of both velocity
 * components, or two where the level's autotuned candidate runs two sweeps
 * per launch; 3D: one colour of one component); hb_kernel_timing_read
 * synchronises, and returns the number of timed launches, their summed
 * device time and their summed algorithmic bytes, counted per red-black
 * sweep of all components (every x component, eta/Re and every b component
 * read once, every x component written once: 7 words per cell in 2D, 10 in
 * 3D) times the part of a sweep the launch runs (2D: one or two sweeps; 3D:
 * one colour of one component, a sixth), plus in 2D both components of the
 * coarse iterate where the launch adds the prolongation of a V-cycle's
 * coarse correction, and of the coarse right-hand side and iterate where it
 * ends with the restriction; words of the storage type).  Enabling resets the
 * counters. */
int hb_kernel_timing(hb_ctx* ctx, int enable);
int hb_kernel_timing_read(hb_ctx* ctx, int64_t* launches, double* total_ms, double* alg_bytes);

/* Tile autotuning (batched sweeps; Sec. III.D's tiling, chosen for the GPU
 * by measurement).  At context creation every multigrid level on which a
 * fused smoother sweep runs (nodal problem; tensor problem in 2D) times its
 * candidates over two sweeps on its own arenas and keeps the fastest; all
 * candidates compute the same values.  A candidate is a tile (tx x ty cells
 * or nodes per plane) with a workgroup size and, for the 2D tensor problem,
 * the number of sweeps one launch runs (1, or 2 with the tile's halo doubled
 * and everything staged in LDS; two need every periodic extent of the level
 * to be at least 8, and are used when the cycle's pre- and post-smoothing
 * sweep counts are even with an even sum of halves, as for V(2,2)).
 * hb_tile_config reports, for level `level` of problem op (HB_OP_VISC, 2D
 * only, or HB_OP_NODAL), the tile, the threads per workgroup and the
 * sweeps per launch; threads and sweeps may be NULL.  Returns HB_ERR_ARG
 * for other problems, for levels without sweep launches (the coarsest, and
 * those run by the single-workgroup coarse cycle) and when HB_FUSE=0 turned
 * the fused sweeps off.  HB_TILE=k in the environment at creation forces
 * candidate k (modulo the problem's candidate count: 6 for the 2D tensor
 * problem, 3 for the nodal one). */
int hb_tile_config(const hb_ctx* ctx, int op, int level, int* tx, int* ty, int* threads, int* sweeps);

#ifdef __cplusplus
}
#endif
#endif
