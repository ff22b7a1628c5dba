/* orc_mg.c -- textbook geometric multigrid V-cycles of the oracle for the
 * three linear systems of the step (Sec. III.A: the tensor viscous solve and
 * the nodal projection; the MAC projection of the face velocity).  The paper
 * uses AMReX's cell and nodal multigrid (Sec. III.D) without detail; the
 * cycle here is the plain one: V(nu1, nu2), Gauss-Seidel smoothing, dense LU
 * on the coarsest level.  Test infrastructure only (see orc.h). */
#include "orc_internal.h"

#define MAXLEV 32

typedef struct {
    orc_grid g;
    long nu;          /* unknowns */
    double* x;
    double* b;
    double* r;
    double* beta;     /* face viscosity per axis (VISC only) */
} level_t;

typedef struct {
    int op;
    int nlev;
    double dt;
    level_t L[MAXLEV];
    double* Ac;       /* coarsest dense matrix, LU factors */
    int* piv;
} mg_t;

/* largest dense coarsest system the hierarchy stops at */
#define ORC_MG_DENSE_MAX 128

static long unknowns(const orc_grid* g, int op)
{
    if (op == ORC_OP_VISC) return ncells(g) * g->dim;
    if (op == ORC_OP_MAC) return ncells(g);
    return orc_node_count(g);
}

/* y = A x on a level */
static void apply_op(const mg_t* m, const level_t* l, const double* x, double* y)
{
    if (m->op == ORC_OP_VISC) orc_tensor_apply_h(&l->g, l->beta, m->dt, x, y);
    else if (m->op == ORC_OP_MAC) orc_mac_lap(&l->g, x, y);
    else orc_apply_K(&l->g, x, y);
}

static void residual(const mg_t* m, level_t* l)
{
    apply_op(m, l, l->x, l->r);
    for (long i = 0; i < l->nu; ++i) l->r[i] = l->b[i] - l->r[i];
}

/* ---- dense coarsest solve -------------------------------------------------- */

/* LU with partial pivoting: factors A in place (row-major), piv[k] = pivot row */
static int lu_factor(int N, double* A, int* piv)
{
    for (int k = 0; k < N; ++k) {
        int p = k;
        double best = fabs(A[(long)k * N + k]);
        for (int i = k + 1; i < N; ++i) {
            double v = fabs(A[(long)i * N + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < N; ++j) {
                double t = A[(long)k * N + j];
                A[(long)k * N + j] = A[(long)p * N + j];
                A[(long)p * N + j] = t;
            }
        for (int i = k + 1; i < N; ++i) {
            double f = A[(long)i * N + k] / A[(long)k * N + k];
            A[(long)i * N + k] = f;
            for (int j = k + 1; j < N; ++j) A[(long)i * N + j] -= f * A[(long)k * N + j];
        }
    }
    return 0;
}

static void lu_solve(int N, const double* A, const int* piv, double* b)
{
    for (int k = 0; k < N; ++k) {
        int p = piv[k];
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < i; ++j) b[i] -= A[(long)i * N + j] * b[j];
    for (int i = N - 1; i >= 0; --i) {
        for (int j = i + 1; j < N; ++j) b[i] -= A[(long)i * N + j] * b[j];
        b[i] /= A[(long)i * N + i];
    }
}

int orc_dense_solve(int N, double* A, double* b)
{
    int* piv = (int*)xcalloc(N, sizeof(int));
    int rc = lu_factor(N, A, piv);
    if (rc == 0) lu_solve(N, A, piv, b);
    free(piv);
    return rc == 0 ? ORC_OK : ORC_ERR_ARG;
}

/* Column j of the dense matrix = operator applied to the j-th unit vector.
 * Singular problems (MAC, nodal) get 1 1^T / N added, which makes the matrix
 * regular and selects the mean-zero solution for a compatible right side. */
static void dense_of_level(const mg_t* m, const level_t* l, double* A, int regularise)
{
    const long N = l->nu;
    double* e = (double*)xcalloc(N, sizeof(double));
    double* y = (double*)xcalloc(N, sizeof(double));
    for (long j = 0; j < N; ++j) {
        e[j] = 1.0;
        apply_op(m, l, e, y);
        e[j] = 0.0;
        for (long i = 0; i < N; ++i) A[i * N + j] = y[i];
    }
    if (regularise && m->op != ORC_OP_VISC)
        for (long i = 0; i < N * N; ++i) A[i] += 1.0 / (double)N;
    free(e);
    free(y);
}

/* ---- smoothers ------------------------------------------------------------- */

/* Tensor: component-sequential red-black Gauss-Seidel; colour = (i+j+k) mod 2,
 * red (0) first; cross terms read the current arrays. */
static void smooth_visc(const mg_t* m, level_t* l, int sweeps)
{
    const orc_grid* g = &l->g;
    const long N = ncells(g);
    for (int s = 0; s < sweeps; ++s)
        for (int c = 0; c < g->dim; ++c)
            for (int colour = 0; colour < 2; ++colour)
                ORC_PAR_KJ
                for (int k = 0; k < g->n[2]; ++k)
                    for (int j = 0; j < g->n[1]; ++j)
                        for (int i = 0; i < g->n[0]; ++i) {
                            if (((i + j + k) & 1) != colour) continue;
                            long q = (long)c * N + cid(g, i, j, k);
                            double Au = l->x[q] - m->dt * orc_visc_div_at(g, l->beta, l->x, 1, c, i, j, k);
                            double dg = orc_tensor_diag(g, l->beta, m->dt, c, i, j, k);
                            l->x[q] += (l->b[q] - Au) / dg;
                        }
}

/* MAC Poisson: red-black Gauss-Seidel on L_mac (5/7-point, zero wall flux) */
static void smooth_mac(level_t* l, int sweeps)
{
    const orc_grid* g = &l->g;
    const double ih2 = 1.0 / (g->h * g->h);
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour)
            ORC_PAR_KJ
            for (int k = 0; k < g->n[2]; ++k)
                for (int j = 0; j < g->n[1]; ++j)
                    for (int i = 0; i < g->n[0]; ++i) {
                        if (((i + j + k) & 1) != colour) continue;
                        long q = cid(g, i, j, k);
                        double Lx = 0.0;
                        int cnt = 0;
                        for (int a = 0; a < g->dim; ++a)
                            for (int side = 0; side < 2; ++side) {
                                int p[3] = {i, j, k};
                                p[a] += side ? 1 : -1;
                                if (!wrap_cell(g, p)) continue;
                                Lx += (l->x[cid(g, p[0], p[1], p[2])] - l->x[q]) * ih2;
                                cnt += 1;
                            }
                        double dg = -(double)cnt * ih2;
                        l->x[q] += (l->b[q] - Lx) / dg;
                    }
}

/* Nodal: 2^d-colour Gauss-Seidel, colour = (i&1) + 2(j&1) + 4(k&1) */
static void smooth_nodal(level_t* l, int sweeps)
{
    const orc_grid* g = &l->g;
    const int ncol = 1 << g->dim;
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < ncol; ++colour)
            ORC_PAR_KJ
            for (int k = 0; k < nnodes(g, 2); ++k)
                for (int j = 0; j < nnodes(g, 1); ++j)
                    for (int i = 0; i < nnodes(g, 0); ++i) {
                        if (((i & 1) + 2 * (j & 1) + 4 * (k & 1)) != colour) continue;
                        double dg;
                        double Kx = orc_K_at(g, l->x, i, j, k, &dg);
                        long q = nid(g, i, j, k);
                        l->x[q] += (l->b[q] - Kx) / dg;
                    }
}

static void smooth(const mg_t* m, level_t* l, int sweeps)
{
    if (m->op == ORC_OP_VISC) smooth_visc(m, l, sweeps);
    else if (m->op == ORC_OP_MAC) smooth_mac(l, sweeps);
    else smooth_nodal(l, sweeps);
}

/* ---- transfers --------------------------------------------------------------- */

/* cell problems: coarse value = mean of the 2^d children */
static void restrict_cells(const orc_grid* gf, const orc_grid* gc, int ncomp, const double* f, double* c)
{
    const long Nf = ncells(gf), Nc = ncells(gc);
    const int nch = 1 << gf->dim;
    const orc_grid* g = gc;   /* the grid the loop nest runs over */
    (void)g;
    for (int q = 0; q < ncomp; ++q)
        ORC_PAR_KJ
        for (int k = 0; k < gc->n[2]; ++k)
            for (int j = 0; j < gc->n[1]; ++j)
                for (int i = 0; i < gc->n[0]; ++i) {
                    double s = 0.0;
                    for (int bits = 0; bits < nch; ++bits) {
                        int fi = 2 * i + (bits & 1);
                        int fj = 2 * j + ((bits >> 1) & 1);
                        int fk = gf->dim == 3 ? 2 * k + ((bits >> 2) & 1) : 0;
                        s += f[(long)q * Nf + cid(gf, fi, fj, fk)];
                    }
                    c[(long)q * Nc + cid(gc, i, j, k)] = s / (double)nch;
                }
}

/* cell problems: x_f += P e_c, (bi/tri)linear with 3/4, 1/4 weights per axis;
 * a coarse neighbour outside a wall takes the homogeneous ghost value
 * (sign -1 for the Dirichlet viscous problem, +1 for the Neumann MAC one). */
static void prolong_cells(const orc_grid* gf, const orc_grid* gc, int ncomp, double wall_sign,
                          const double* e, double* x)
{
    const long Nf = ncells(gf), Nc = ncells(gc);
    const int d = gf->dim;
    const int nco = 1 << d;
    const orc_grid* g = gf;   /* the grid the loop nest runs over */
    (void)g;
    for (int q = 0; q < ncomp; ++q)
        ORC_PAR_KJ
        for (int k = 0; k < gf->n[2]; ++k)
            for (int j = 0; j < gf->n[1]; ++j)
                for (int i = 0; i < gf->n[0]; ++i) {
                    int fi[3] = {i, j, k};
                    double s = 0.0;
                    for (int bits = 0; bits < nco; ++bits) {
                        int p[3] = {0, 0, 0};
                        double w = 1.0, sg = 1.0;
                        for (int a = 0; a < d; ++a) {
                            int I = fi[a] / 2;
                            int far = (bits >> a) & 1;
                            if (!far) { p[a] = I; w *= 0.75; continue; }
                            int J = (fi[a] & 1) ? I + 1 : I - 1;
                            w *= 0.25;
                            if (J < 0 || J >= gc->n[a]) {
                                if (is_periodic(gc, a)) J = (J + gc->n[a]) % gc->n[a];
                                else { J = I; sg *= wall_sign; }
                            }
                            p[a] = J;
                        }
                        s += w * sg * e[(long)q * Nc + cid(gc, p[0], p[1], p[2])];
                    }
                    x[(long)q * Nf + cid(gf, i, j, k)] += s;
                }
}

/* nodal: restriction R = P^T (full weighting), fine node 2I+delta has weight
 * prod_a (delta_a == 0 ? 1 : 1/2) */
static void restrict_nodes(const orc_grid* gf, const orc_grid* gc, const double* f, double* c)
{
    const int d = gf->dim;
    int nd = 1;
    for (int a = 0; a < d; ++a) nd *= 3;
    for (int k = 0; k < nnodes(gc, 2); ++k)
        for (int j = 0; j < nnodes(gc, 1); ++j)
            for (int i = 0; i < nnodes(gc, 0); ++i) {
                int I[3] = {i, j, k};
                double s = 0.0;
                for (int t = 0; t < nd; ++t) {
                    int del[3] = {0, 0, 0}, tt = t;
                    for (int a = 0; a < d; ++a) { del[a] = tt % 3 - 1; tt /= 3; }
                    int p[3] = {0, 0, 0};
                    double w = 1.0;
                    int ok = 1;
                    for (int a = 0; a < d; ++a) {
                        int F = 2 * I[a] + del[a];
                        if (del[a] != 0) w *= 0.5;
                        int nf = nnodes(gf, a);
                        if (F < 0 || F >= nf) {
                            if (is_periodic(gf, a)) F = (F + nf) % nf; else ok = 0;
                        }
                        p[a] = F;
                    }
                    if (ok) s += w * f[nid(gf, p[0], p[1], p[2])];
                }
                c[nid(gc, i, j, k)] = s;
            }
}

/* nodal: x_f += P e_c, (bi/tri)linear on nodes */
static void prolong_nodes(const orc_grid* gf, const orc_grid* gc, const double* e, double* x)
{
    const int d = gf->dim;
    for (int k = 0; k < nnodes(gf, 2); ++k)
        for (int j = 0; j < nnodes(gf, 1); ++j)
            for (int i = 0; i < nnodes(gf, 0); ++i) {
                int F[3] = {i, j, k};
                double s = 0.0;
                for (int bits = 0; bits < (1 << d); ++bits) {
                    int p[3] = {0, 0, 0};
                    double w = 1.0;
                    int ok = 1;
                    for (int a = 0; a < d; ++a) {
                        int hi = (bits >> a) & 1;
                        if (!(F[a] & 1)) {       /* coincident coarse node */
                            if (hi) { ok = 0; break; }
                            p[a] = F[a] / 2;
                        } else {
                            w *= 0.5;
                            int C = (F[a] - 1) / 2 + hi;
                            if (is_periodic(gc, a)) C %= nnodes(gc, a);
                            p[a] = C;
                        }
                    }
                    if (ok) s += w * e[nid(gc, p[0], p[1], p[2])];
                }
                x[nid(gf, i, j, k)] += s;
            }
}

/* coarse face viscosity = mean of the 2^(d-1) fine faces that tile the coarse
 * face (the coarse face at index I along a coincides with fine face 2I) */
static void restrict_faces(const orc_grid* gf, const orc_grid* gc, const double* bf, double* bc)
{
    const int d = gf->dim;
    for (int a = 0; a < d; ++a) {
        const double* F = bf + orc_face_offset(gf, a);
        double* Cc = bc + orc_face_offset(gc, a);
        int ext[3] = {gc->n[0], gc->n[1], gc->n[2]};
        ext[a] = nfaces(gc, a);
        for (int k = 0; k < ext[2]; ++k)
            for (int j = 0; j < ext[1]; ++j)
                for (int i = 0; i < ext[0]; ++i) {
                    int I[3] = {i, j, k};
                    double s = 0.0;
                    int cnt = 0;
                    for (int t = 0; t < (1 << d); ++t) {
                        if ((t >> a) & 1) continue;
                        int p[3] = {0, 0, 0};
                        for (int b = 0; b < 3; ++b) {
                            if (b >= d) { p[b] = 0; continue; }
                            p[b] = (b == a) ? 2 * I[b] : 2 * I[b] + ((t >> b) & 1);
                        }
                        s += F[fid(gf, a, p[0], p[1], p[2])];
                        cnt += 1;
                    }
                    Cc[fid(gc, a, i, j, k)] = s / (double)cnt;
                }
    }
}

static long nface_total(const orc_grid* g)
{
    long n = 0;
    for (int a = 0; a < g->dim; ++a) n += face_count(g, a);
    return n;
}

/* ---- hierarchy ---------------------------------------------------------------- */

static void build(mg_t* m, const orc_grid* g, const orc_fluid* fl, int op, const double* eta, double dt)
{
    memset(m, 0, sizeof(*m));
    m->op = op;
    m->dt = dt;
    orc_grid cur = *g;
    int l = 0;
    for (;;) {
        level_t* L = &m->L[l];
        L->g = cur;
        L->nu = unknowns(&cur, op);
        L->x = (double*)xcalloc(L->nu, sizeof(double));
        L->b = (double*)xcalloc(L->nu, sizeof(double));
        L->r = (double*)xcalloc(L->nu, sizeof(double));
        if (op == ORC_OP_VISC) {
            L->beta = (double*)xcalloc(nface_total(&cur), sizeof(double));
            if (l == 0) {
                const long N = ncells(&cur);
                double* eta_e = (double*)xcalloc(N, sizeof(double));
                for (long i = 0; i < N; ++i) eta_e[i] = eta[i] / fl->Re;
                orc_eta_faces(&cur, eta_e, L->beta);
                free(eta_e);
            } else {
                restrict_faces(&m->L[l - 1].g, &cur, m->L[l - 1].beta, L->beta);
            }
        }
        ++l;
        int can = (l < MAXLEV);
        for (int a = 0; a < cur.dim; ++a)
            if ((cur.n[a] & 1) || cur.n[a] / 2 < 2) can = 0;
        /* stop at the first level with at most ORC_MG_DENSE_MAX unknowns
         * (MAC 8^2 / 4^3 cells, nodal 9^2 / 5^3 nodes, tensor 2 x 8^2 in 2D
         * and 3 x 2^3 in 3D); that level is solved densely */
        if (L->nu <= ORC_MG_DENSE_MAX) can = 0;
        if (!can) break;
        orc_grid nx = cur;
        for (int a = 0; a < cur.dim; ++a) nx.n[a] = cur.n[a] / 2;
        nx.h = cur.h * 2.0;
        memset(nx.wall_u, 0, sizeof(nx.wall_u));
        cur = nx;
    }
    m->nlev = l;
    const level_t* C = &m->L[l - 1];
    m->Ac = (double*)xcalloc(C->nu * C->nu, sizeof(double));
    m->piv = (int*)xcalloc(C->nu, sizeof(int));
    dense_of_level(m, C, m->Ac, 1);
    lu_factor((int)C->nu, m->Ac, m->piv);
}

static void destroy(mg_t* m)
{
    for (int l = 0; l < m->nlev; ++l) {
        free(m->L[l].x);
        free(m->L[l].b);
        free(m->L[l].r);
        free(m->L[l].beta);
    }
    free(m->Ac);
    free(m->piv);
}

static void vcycle(mg_t* m, int l, int nu1, int nu2)
{
    level_t* L = &m->L[l];
    if (l == m->nlev - 1) {
        memcpy(L->x, L->b, sizeof(double) * L->nu);
        lu_solve((int)L->nu, m->Ac, m->piv, L->x);
        return;
    }
    level_t* C = &m->L[l + 1];
    smooth(m, L, nu1);
    residual(m, L);
    if (m->op == ORC_OP_NODAL) restrict_nodes(&L->g, &C->g, L->r, C->b);
    else restrict_cells(&L->g, &C->g, m->op == ORC_OP_VISC ? L->g.dim : 1, L->r, C->b);
    memset(C->x, 0, sizeof(double) * C->nu);
    vcycle(m, l + 1, nu1, nu2);
    if (m->op == ORC_OP_NODAL) prolong_nodes(&L->g, &C->g, C->x, L->x);
    else prolong_cells(&L->g, &C->g, m->op == ORC_OP_VISC ? L->g.dim : 1,
                       m->op == ORC_OP_VISC ? -1.0 : 1.0, C->x, L->x);
    smooth(m, L, nu2);
}

static void remove_mean(double* v, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += v[i];
    s /= (double)n;
    for (long i = 0; i < n; ++i) v[i] -= s;
}

static double dot(const double* a, const double* b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* z = M^{-1} r: one V-cycle from a zero guess on the finest level */
static void precond(mg_t* m, const double* r, double* z, int nu1, int nu2)
{
    level_t* F = &m->L[0];
    double* bsave = (double*)xcalloc(F->nu, sizeof(double));
    double* xsave = (double*)xcalloc(F->nu, sizeof(double));
    memcpy(bsave, F->b, sizeof(double) * F->nu);
    memcpy(xsave, F->x, sizeof(double) * F->nu);
    memcpy(F->b, r, sizeof(double) * F->nu);
    memset(F->x, 0, sizeof(double) * F->nu);
    vcycle(m, 0, nu1, nu2);
    memcpy(z, F->x, sizeof(double) * F->nu);
    memcpy(F->b, bsave, sizeof(double) * F->nu);
    memcpy(F->x, xsave, sizeof(double) * F->nu);
    free(bsave);
    free(xsave);
}

/* BiCGStab, right-preconditioned by one V-cycle per application (van der
 * Vorst 1992).  Counts V-cycles in *cycles; returns the recurrence residual
 * norm relative to bn. */
static int bicgstab(mg_t* m, const orc_mg_opts* o, double bn, int* cycles, double* rel_out)
{
    level_t* F = &m->L[0];
    const long n = F->nu;
    double* r = (double*)xcalloc(n, sizeof(double));
    double* rh = (double*)xcalloc(n, sizeof(double));
    double* p = (double*)xcalloc(n, sizeof(double));
    double* v = (double*)xcalloc(n, sizeof(double));
    double* ph = (double*)xcalloc(n, sizeof(double));
    double* s = (double*)xcalloc(n, sizeof(double));
    double* sh = (double*)xcalloc(n, sizeof(double));
    double* t = (double*)xcalloc(n, sizeof(double));
    residual(m, F);
    memcpy(r, F->r, sizeof(double) * n);
    memcpy(rh, r, sizeof(double) * n);
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    double rel = vmax_abs(r, n) / bn;
    int rc = ORC_OK;
    for (;;) {
        if (o->fixed) { if (*cycles >= o->max_cycles) break; }
        else {
            if (rel <= o->tol) break;
            if (*cycles >= o->max_cycles) { rc = ORC_ERR_NOCONV; break; }
        }
        double rho = dot(rh, r, n);
        if (rho == 0.0) { rc = ORC_ERR_NOCONV; break; }
        double beta = (rho / rho_prev) * (alpha / omega);
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        precond(m, p, ph, o->nu1, o->nu2);
        *cycles += 1;
        apply_op(m, F, ph, v);
        alpha = rho / dot(rh, v, n);
        for (long i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double srel = vmax_abs(s, n) / bn;
        if ((!o->fixed && srel <= o->tol) || (o->fixed && *cycles >= o->max_cycles)) {
            for (long i = 0; i < n; ++i) F->x[i] += alpha * ph[i];
            memcpy(r, s, sizeof(double) * n);
            rel = srel;
            break;
        }
        precond(m, s, sh, o->nu1, o->nu2);
        *cycles += 1;
        apply_op(m, F, sh, t);
        double tt = dot(t, t, n);
        omega = tt > 0.0 ? dot(t, s, n) / tt : 0.0;
        for (long i = 0; i < n; ++i) F->x[i] += alpha * ph[i] + omega * sh[i];
        for (long i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rel = vmax_abs(r, n) / bn;
        if (!isfinite(rel)) { rc = ORC_ERR_NONFINITE; break; }
        if (omega == 0.0) { rc = ORC_ERR_NOCONV; break; }
        rho_prev = rho;
    }
    *rel_out = rel;
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    return rc;
}

int orc_mg_solve(const orc_grid* g, const orc_fluid* fl, int op, const double* eta,
                 double dt, const double* rhs, double* x, const orc_mg_opts* o,
                 orc_mg_report* rep)
{
    if (op < 0 || op > 2 || !o || o->max_cycles < 0 || o->nu1 < 0 || o->nu2 < 0) return ORC_ERR_ARG;
    if (op == ORC_OP_VISC && (!eta || !fl)) return ORC_ERR_ARG;
    mg_t m;
    build(&m, g, fl, op, eta, dt);
    level_t* F = &m.L[0];
    const long nu = F->nu;
    if (!all_finite(rhs, nu) || !all_finite(x, nu)) { destroy(&m); return ORC_ERR_NONFINITE; }
    memcpy(F->b, rhs, sizeof(double) * nu);
    memcpy(F->x, x, sizeof(double) * nu);
    if (op == ORC_OP_VISC) {
        /* move the inhomogeneous wall values to the right side:
         * A(u) = A_h(u) - dt * div(eta_e gamma_dot(0; wall values)) */
        double* zero = (double*)xcalloc(nu, sizeof(double));
        double* w = (double*)xcalloc(nu, sizeof(double));
        orc_visc_div_faces(g, F->beta, zero, 0, w);
        for (long i = 0; i < nu; ++i) F->b[i] += dt * w[i];
        free(zero);
        free(w);
    } else {
        remove_mean(F->b, nu);
    }
    double bn = vmax_abs(F->b, nu);
    int cycles = 0, rc = ORC_OK;
    double rel = 0.0;
    if (bn == 0.0) {
        memset(F->x, 0, sizeof(double) * nu);
    } else if (o->krylov) {
        rc = bicgstab(&m, o, bn, &cycles, &rel);
        residual(&m, F);
        rel = vmax_abs(F->r, nu) / bn;
    } else {
        residual(&m, F);
        rel = vmax_abs(F->r, nu) / bn;
        for (;;) {
            if (o->fixed) {
                if (cycles >= o->max_cycles) break;
            } else {
                if (rel <= o->tol) break;
                if (cycles >= o->max_cycles) { rc = ORC_ERR_NOCONV; break; }
            }
            vcycle(&m, 0, o->nu1, o->nu2);
            ++cycles;
            residual(&m, F);
            rel = vmax_abs(F->r, nu) / bn;
            if (!isfinite(rel)) { rc = ORC_ERR_NONFINITE; break; }
        }
    }
    if (op != ORC_OP_VISC) remove_mean(F->x, nu);
    memcpy(x, F->x, sizeof(double) * nu);
    if (rep) { rep->cycles = cycles; rep->rel_resid = rel; rep->bnorm = bn; }
    destroy(&m);
    return rc;
}

int orc_dense_matrix(const orc_grid* g, const orc_fluid* fl, int op, const double* eta,
                     double dt, double* A)
{
    mg_t m;
    memset(&m, 0, sizeof(m));
    m.op = op;
    m.dt = dt;
    m.nlev = 1;
    level_t* L = &m.L[0];
    L->g = *g;
    L->nu = unknowns(g, op);
    if (op == ORC_OP_VISC) {
        const long N = ncells(g);
        double* eta_e = (double*)xcalloc(N, sizeof(double));
        for (long i = 0; i < N; ++i) eta_e[i] = eta[i] / fl->Re;
        L->beta = (double*)xcalloc(nface_total(g), sizeof(double));
        orc_eta_faces(g, eta_e, L->beta);
        free(eta_e);
    }
    dense_of_level(&m, L, A, 0);   /* plain operator, without the 1 1^T / N term */
    free(L->beta);
    return ORC_OK;
}

/* Diagonal the tensor smoother divides by, for every component and cell. */
int orc_tensor_diagonal(const orc_grid* g, const orc_fluid* fl, const double* eta, double dt, double* out)
{
    const long N = ncells(g);
    double* eta_e = (double*)xcalloc(N, sizeof(double));
    double* beta = (double*)xcalloc(nface_total(g), sizeof(double));
    for (long i = 0; i < N; ++i) eta_e[i] = eta[i] / fl->Re;
    orc_eta_faces(g, eta_e, beta);
    for (int c = 0; c < g->dim; ++c)
        for (int k = 0; k < g->n[2]; ++k)
            for (int j = 0; j < g->n[1]; ++j)
                for (int i = 0; i < g->n[0]; ++i)
                    out[(long)c * N + cid(g, i, j, k)] = orc_tensor_diag(g, beta, dt, c, i, j, k);
    free(eta_e);
    free(beta);
    return ORC_OK;
}

/* ---- transfers exposed for the pins ------------------------------------------ */

void orc_prolong_cells(const orc_grid* gf, const orc_grid* gc, int ncomp, double wall_sign, const double* e,
                       double* x)
{
    prolong_cells(gf, gc, ncomp, wall_sign, e, x);
}

void orc_restrict_faces(const orc_grid* gf, const orc_grid* gc, const double* bf, double* bc)
{
    restrict_faces(gf, gc, bf, bc);
}
