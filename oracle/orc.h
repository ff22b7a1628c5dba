/*
 * orc.h -- plain FP64 CPU oracle for one semi-implicit time step of the
 * Papanastasiou-regularised Herschel-Bulkley incompressible solver
 * (Sverdrup, Nikiforakis & Almgren, arXiv 1803.00417).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it.  It shares no code, header, table or helper with the HIP library; the
 * product path never calls it.
 *
 * What it follows (paper sections / equations):
 *   - scaled Frobenius norm and gradient conventions: Sec. II (start);
 *   - Herschel-Bulkley apparent viscosity, Papanastasiou regularisation:
 *     eq:viscosity:hb, eq:regularisation, eq:rheology:papanastasiou, and the
 *     dimensionless form eq:dimensionless:herschel-bulkley (Sec. IV);
 *   - the step: Sec. III.A (Taylor extrapolation, eq:iamr:extrap, upwinding,
 *     Crank-Nicolson provisional velocity with lagged viscosity, tensor solve,
 *     approximate projection);
 *   - multigrid: Sec. III.D names AMReX cell and nodal multigrid but gives no
 *     detail; the V-cycle here is a textbook geometric multigrid (coarsening
 *     by two while every extent is even and at least 4, stopping at the first
 *     level with at most 128 unknowns; dense LU on the coarsest level).
 *
 * Conventions.  All arrays are FP64, x fastest: a cell field with C components
 * is [C][nz][ny][nx]; nodal fields are [nnz][nny][nnx] with nn_a = n_a + 1 on
 * wall axes and n_a on periodic axes.  2D grids use n[2] = 1.  No ghost cells
 * are stored; boundary values are produced on the fly.
 */
#ifndef ORC_H
#define ORC_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_WALL = 0, ORC_PERIODIC = 1 };
enum { ORC_REG_PAPER = 0, ORC_REG_YIELD_ONLY = 1 };
enum { ORC_OP_VISC = 0, ORC_OP_NODAL = 1, ORC_OP_MAC = 2 };
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NOCONV = -3, ORC_ERR_NONFINITE = -4 };

typedef struct {
    int dim;                  /* 2 or 3 */
    int n[3];                 /* cells per axis; n[2] = 1 in 2D */
    double h;                 /* uniform spacing */
    int bc[3][2];             /* ORC_WALL / ORC_PERIODIC per face (axis, lo/hi) */
    double wall_u[3][2][3];   /* wall velocity per face (axis, side, component) */
} orc_grid;

typedef struct {
    double Re, HB, n, Pa;     /* dimensionless groups of Sec. IV */
    int reg;                  /* ORC_REG_PAPER (product form) or ORC_REG_YIELD_ONLY */
    double f[3];              /* constant body force */
} orc_fluid;

typedef struct {
    double tol;               /* stop when |b - Ax|_inf <= tol |b|_inf */
    int max_cycles;
    int fixed;                /* 1: run exactly max_cycles V-cycles */
    int nu1, nu2;
    int krylov;               /* 1: BiCGStab preconditioned by one V-cycle */
} orc_mg_opts;

typedef struct {
    int cycles;
    double rel_resid;         /* |b - Ax|_inf / |b|_inf at exit */
    double bnorm;             /* |b|_inf of the system actually solved */
} orc_mg_report;

typedef struct {
    double cfl;
    int mac_project;          /* 1: project the face velocity (default) */
    orc_mg_opts mac, visc, proj;
    int pred_visc;            /* 1: the explicit stress divergence enters the
                                 forcing of the Taylor prediction (as printed in
                                 eq:iamr:extrap); 0 (default): -G p + f only */
    double theta;             /* implicit weight of the viscous update: 0.5 (or
                                 0) Crank-Nicolson as printed in Sec. III.A,
                                 1 backward Euler */
} orc_step_opts;

typedef struct {
    double dt, max_u;
    double div_mac_rel;       /* |D_mac u^MAC|_inf / |D_mac u^adv|_inf */
    double div_node;          /* max_k |weak div(u^{m+1})_k| / h^d */
    orc_mg_report mac, visc, proj;
} orc_step_report;

/* ---- pointwise viscosity law -------------------------------------------- */
/* eta_hat(g) for the scaled strain-rate norm g (eq:dimensionless:herschel-bulkley) */
double orc_eta_of_g(const orc_fluid* fl, double g);
/* eta_hat(u) per cell; eta has n cells */
int orc_viscosity(const orc_grid* g, const orc_fluid* fl, const double* u, double* eta);

/* ---- operators (exposed for pins and parity of single kernels) ---------- */
/* out[c] = div(eta_e * gamma_dot(u))_c ; hom=1: homogeneous wall values */
void orc_visc_div(const orc_grid* g, const double* eta_e, const double* u, int hom, double* out);
/* cell-average gradient of a nodal field: out [dim][cells] */
void orc_grad_node(const orc_grid* g, const double* phi, double* out);
/* weak divergence of a cell vector field onto nodes */
void orc_weak_div(const orc_grid* g, const double* V, double* r);
/* Q1 stiffness applied to a nodal field, by element assembly */
void orc_apply_K(const orc_grid* g, const double* phi, double* out);
/* MAC divergence of face fields (face arrays per axis, concatenated) */
void orc_mac_div(const orc_grid* g, const double* faces, double* out);
long orc_face_count(const orc_grid* g, int axis);
long orc_node_count(const orc_grid* g);

/* ---- multigrid solve ----------------------------------------------------- */
/* VISC: (I - dt div(eta_hat/Re gamma_dot(.))) x = rhs, with the grid's wall
 * velocities;  NODAL: K x = rhs (rhs mean removed, x mean zero);  MAC:
 * L_mac x = rhs (same).  x: in guess, out solution. */
int orc_mg_solve(const orc_grid* g, const orc_fluid* fl, int op, const double* eta,
                 double dt, const double* rhs, double* x, const orc_mg_opts* o,
                 orc_mg_report* rep);
/* Dense operator matrix of a level (row-major, N x N) -- for the dense pins. */
int orc_dense_matrix(const orc_grid* g, const orc_fluid* fl, int op, const double* eta,
                     double dt, double* A);
int orc_dense_solve(int N, double* A, double* b);  /* LU, partial pivoting, in place */
/* Multigrid transfers of the cell problems (for the pins): x += P e, the
 * (bi/tri)linear prolongation from the coarse grid gc (every cell count of gf
 * halved) with the homogeneous ghost e(wall) = wall_sign e(inner) beyond a wall
 * (-1: the Dirichlet viscous problem, +1: the Neumann MAC problem); and the
 * coarse face viscosity as the mean of the fine faces tiling each coarse face
 * (face arrays per axis, concatenated). */
void orc_prolong_cells(const orc_grid* gf, const orc_grid* gc, int ncomp, double wall_sign, const double* e,
                       double* x);
void orc_restrict_faces(const orc_grid* gf, const orc_grid* gc, const double* bf, double* bc);
/* Diagonal used by the tensor Gauss-Seidel smoother ([dim][cells]). */
int orc_tensor_diagonal(const orc_grid* g, const orc_fluid* fl, const double* eta, double dt, double* out);

/* ---- the step ------------------------------------------------------------ */
double orc_cfl_dt(const orc_grid* g, double cfl, const double* u);
double orc_theta(const orc_step_opts* o);
/* Godunov stage: from u^m, p^{m-1/2}, eta_hat and dt produce the viscous-solve
 * right-hand side b (before wall terms), and optionally the explicit term E,
 * the MAC velocity (per axis, concatenated face arrays) and the convective
 * term A.  Any optional pointer may be NULL. */
int orc_advect(const orc_grid* g, const orc_fluid* fl, const orc_step_opts* o,
               const double* u, const double* p, const double* eta, double dt,
               double* b, double* E_out, double* umac_out, double* A_out,
               orc_mg_report* mac_rep, double* div_mac_rel);
int orc_project(const orc_grid* g, const orc_step_opts* o, const double* ustar,
                double* p, double dt, double* u_out, orc_mg_report* rep);
int orc_step(const orc_grid* g, const orc_fluid* fl, const orc_step_opts* o,
             double* u, double* p, double dt, orc_step_report* rep);

#ifdef __cplusplus
}
#endif
#endif
