/* orc_core.c -- viscosity law and discrete operators of the oracle.
 * Test infrastructure only (see orc.h). */
#include "orc_internal.h"

/* ------------------------------------------------------------------------ */
/* Viscosity (Sec. II norm; Sec. III.B regularisation; Sec. IV dimensionless) */
/* ------------------------------------------------------------------------ */

/* (1 - exp(-x)) / x, the Papanastasiou factor divided by its argument;
 * equals 1 at x = 0 (eq:regularisation:limit). */
static double papa_phi(double x)
{
    if (x == 0.0) return 1.0;
    return -expm1(-x) / x;
}

/* Dimensionless apparent viscosity as a function of g = |gamma_dot|:
 *   PAPER      eta = (g^n + HB/2) (1 - exp(-Pa g)) / g
 *                  = (g^n + HB/2) Pa phi(Pa g)      (eq:dimensionless:herschel-bulkley)
 *   YIELD_ONLY eta = g^(n-1) + (HB/2) Pa phi(Pa g)   (regularise the yield term only) */
double orc_eta_of_g(const orc_fluid* fl, double g)
{
    double x = fl->Pa * g;
    if (fl->reg == ORC_REG_YIELD_ONLY)
        return pow(g, fl->n - 1.0) + 0.5 * fl->HB * fl->Pa * papa_phi(x);
    return (pow(g, fl->n) + 0.5 * fl->HB) * fl->Pa * papa_phi(x);
}

/* Velocity gradient (grad u)_{ij} = d u_j / d x_i by centred differences with
 * wall ghosts; strain rate = symmetric part; g = sqrt(tr(A A^T)/2). */
int orc_viscosity(const orc_grid* g, const orc_fluid* fl, const double* u, double* eta)
{
    const int d = g->dim;
    const long N = ncells(g);
    const double h = g->h;
    ORC_PAR_KJ
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                double G[3][3] = {{0}};
                for (int a = 0; a < d; ++a)        /* derivative direction */
                    for (int c = 0; c < d; ++c) {  /* velocity component */
                        int pp[3] = {i, j, k}, pm[3] = {i, j, k};
                        pp[a] += 1;
                        pm[a] -= 1;
                        const double* q = u + (long)c * N;
                        G[a][c] = (cell_val(g, q, c, pp, 0) - cell_val(g, q, c, pm, 0)) / (2.0 * h);
                    }
                double s = 0.0;
                for (int a = 0; a < d; ++a)
                    for (int c = 0; c < d; ++c) {
                        double gd = 0.5 * (G[a][c] + G[c][a]);
                        s += gd * gd;
                    }
                double gn = sqrt(0.5 * s);
                eta[cid(g, i, j, k)] = orc_eta_of_g(fl, gn);
            }
    return all_finite(eta, N) ? ORC_OK : ORC_ERR_NONFINITE;
}

/* ------------------------------------------------------------------------ */
/* Tensor viscous operator: out_c = div(eta_e gamma_dot(u))_c                */
/* ------------------------------------------------------------------------ */

/* Face viscosity of the fine grid: the mean of the two adjacent cells on
 * interior (and periodic) faces, the interior cell's value on wall faces.
 * beta holds one face array per axis, concatenated. */
void orc_eta_faces(const orc_grid* g, const double* eta_e, double* beta)
{
    long off = 0;
    for (int a = 0; a < g->dim; ++a) {
        int ext[3] = {g->n[0], g->n[1], g->n[2]};
        ext[a] = nfaces(g, a);
        ORC_PAR_KJ
        for (int k = 0; k < ext[2]; ++k)
            for (int j = 0; j < ext[1]; ++j)
                for (int i = 0; i < ext[0]; ++i) {
                    int R[3] = {i, j, k}, L[3] = {i, j, k};
                    L[a] -= 1;
                    int okL = wrap_cell(g, L), okR = wrap_cell(g, R);
                    double v;
                    if (okL && okR)
                        v = 0.5 * (eta_e[cid(g, L[0], L[1], L[2])] + eta_e[cid(g, R[0], R[1], R[2])]);
                    else if (okL)
                        v = eta_e[cid(g, L[0], L[1], L[2])];
                    else
                        v = eta_e[cid(g, R[0], R[1], R[2])];
                    beta[off + fid(g, a, i, j, k)] = v;
                }
        off += face_count(g, a);
    }
}

long orc_face_offset(const orc_grid* g, int a)
{
    long off = 0;
    for (int b = 0; b < a; ++b) off += face_count(g, b);
    return off;
}

/* Flux of component c through the face normal to axis a whose hi-side cell
 * is p (so the lo-side cell is p - e_a).  gamma_dot = (grad u + grad u^T)/2,
 * so the flux is beta_f * ( du_c/dx_a + du_a/dx_c ) / 2:
 *   a == c : beta_f (u_c(R) - u_c(L)) / h
 *   a != c : beta_f * 1/2 [ (u_c(R) - u_c(L))/h + (du_a/dx_c)_f ],
 * (du_a/dx_c)_f = mean of the centred differences in the two cells; on a
 * wall face it is the tangential derivative of the wall velocity, which is
 * zero for rigid walls and a uniformly moving lid. */
static double visc_flux(const orc_grid* g, const double* beta, const double* u, int hom,
                        int c, int a, const int p[3])
{
    const long N = ncells(g);
    const double h = g->h;
    int R[3] = {p[0], p[1], p[2]};
    int L[3] = {p[0], p[1], p[2]};
    L[a] -= 1;
    int wall = 0;
    if (!is_periodic(g, a) && (p[a] == 0 || p[a] == g->n[a])) wall = 1;
    int fp[3] = {p[0], p[1], p[2]};
    if (is_periodic(g, a)) fp[a] %= g->n[a];
    const double bf = beta[orc_face_offset(g, a) + fid(g, a, fp[0], fp[1], fp[2])];
    const double* uc = u + (long)c * N;
    double uR = cell_val(g, uc, c, R, hom);
    double uL = cell_val(g, uc, c, L, hom);
    double dn = (uR - uL) / h;
    if (a == c) return bf * dn;
    if (wall) return bf * 0.5 * dn;
    int Rw[3] = {R[0], R[1], R[2]}, Lw[3] = {L[0], L[1], L[2]};
    wrap_cell(g, Rw);
    wrap_cell(g, Lw);
    const double* ua = u + (long)a * N;
    int Lp[3] = {Lw[0], Lw[1], Lw[2]}, Lm[3] = {Lw[0], Lw[1], Lw[2]};
    int Rp[3] = {Rw[0], Rw[1], Rw[2]}, Rm[3] = {Rw[0], Rw[1], Rw[2]};
    Lp[c] += 1; Lm[c] -= 1; Rp[c] += 1; Rm[c] -= 1;
    double dL = (cell_val(g, ua, a, Lp, hom) - cell_val(g, ua, a, Lm, hom)) / (2.0 * h);
    double dR = (cell_val(g, ua, a, Rp, hom) - cell_val(g, ua, a, Rm, hom)) / (2.0 * h);
    double cross = 0.5 * (dL + dR);
    return bf * 0.5 * (dn + cross);
}

/* div(beta gamma_dot(u))_c at one cell (for the smoother) */
double orc_visc_div_at(const orc_grid* g, const double* beta, const double* u, int hom,
                       int c, int i, int j, int k)
{
    double s = 0.0;
    for (int a = 0; a < g->dim; ++a) {
        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
        hi[a] += 1;
        s += (visc_flux(g, beta, u, hom, c, a, hi) - visc_flux(g, beta, u, hom, c, a, lo)) / g->h;
    }
    return s;
}

void orc_visc_div_faces(const orc_grid* g, const double* beta, const double* u, int hom, double* out)
{
    const long N = ncells(g);
    for (int c = 0; c < g->dim; ++c)
        ORC_PAR_KJ
        for (int k = 0; k < g->n[2]; ++k)
            for (int j = 0; j < g->n[1]; ++j)
                for (int i = 0; i < g->n[0]; ++i)
                    out[(long)c * N + cid(g, i, j, k)] = orc_visc_div_at(g, beta, u, hom, c, i, j, k);
}

void orc_visc_div(const orc_grid* g, const double* eta_e, const double* u, int hom, double* out)
{
    long nf = 0;
    for (int a = 0; a < g->dim; ++a) nf += face_count(g, a);
    double* beta = (double*)xcalloc(nf, sizeof(double));
    orc_eta_faces(g, eta_e, beta);
    orc_visc_div_faces(g, beta, u, hom, out);
    free(beta);
}

/* A_h(u) = u - dt * div(beta gamma_dot(u)) with homogeneous wall values */
void orc_tensor_apply_h(const orc_grid* g, const double* beta, double dt, const double* u, double* out)
{
    const long n = ncells(g) * g->dim;
    orc_visc_div_faces(g, beta, u, 1, out);
    for (long i = 0; i < n; ++i) out[i] = u[i] - dt * out[i];
}

/* Diagonal of A_h for component c at a cell: 1 + dt/h^2 * sum over the
 * cell's faces of w * s * beta_f, with s = 1 on faces normal to c and 1/2
 * otherwise, and w = 2 on wall faces (odd ghost) else 1. */
double orc_tensor_diag(const orc_grid* g, const double* beta, double dt, int c, int i, int j, int k)
{
    double coef = 0.0;
    for (int a = 0; a < g->dim; ++a)
        for (int side = 0; side < 2; ++side) {
            int q[3] = {i, j, k};
            q[a] += side;
            int wall = (!is_periodic(g, a) && (q[a] == 0 || q[a] == g->n[a]));
            if (is_periodic(g, a)) q[a] %= g->n[a];
            double bf = beta[orc_face_offset(g, a) + fid(g, a, q[0], q[1], q[2])];
            double s = (a == c) ? 1.0 : 0.5;
            coef += (wall ? 2.0 : 1.0) * s * bf;
        }
    return 1.0 + dt * coef / (g->h * g->h);
}

/* ------------------------------------------------------------------------ */
/* Nodal operators of the approximate projection (Sec. III.A)                */
/* ------------------------------------------------------------------------ */

long orc_node_count(const orc_grid* g) { return (long)nnodes(g, 0) * nnodes(g, 1) * nnodes(g, 2); }

/* node index of corner `bits` of cell (i,j,k) */
static long corner_node(const orc_grid* g, int i, int j, int k, int bits)
{
    int p[3] = {i, j, k};
    for (int a = 0; a < g->dim; ++a) {
        p[a] += (bits >> a) & 1;
        if (is_periodic(g, a)) p[a] %= g->n[a];
    }
    return nid(g, p[0], p[1], p[2]);
}


#ifdef _OPENMP
/* Timing build: the cells touching node (i,j,k) and the node's corner index
 * in each, in the order of the cells' linear index (the order in which the
 * serial loops over cells add their contributions to the node, so a gather
 * in this order forms the same sums).  Returns the count. */
static int node_cells(const orc_grid* g, int i, int j, int k, long* cell, int* corner)
{
    const int d = g->dim;
    const int node[3] = {i, j, k};
    int cnt = 0;
    for (int m = 0; m < (1 << d); ++m) {
        int c[3] = {0, 0, 0};
        int ok = 1;
        for (int a = 0; a < d; ++a) {
            int v = node[a] - ((m >> a) & 1);   /* the node is corner bit (m>>a)&1 of cell v */
            if (v < 0) { if (is_periodic(g, a)) v += g->n[a]; else ok = 0; }
            if (v >= g->n[a]) ok = 0;
            c[a] = v;
        }
        if (!ok) continue;
        long id = cid(g, c[0], c[1], c[2]);
        int t = cnt++;
        while (t > 0 && cell[t - 1] > id) { cell[t] = cell[t - 1]; corner[t] = corner[t - 1]; --t; }
        cell[t] = id;
        corner[t] = m;
    }
    return cnt;
}
#endif

/* (G phi)_a = mean over the cell's 2^(d-1) edges along a of (phi_hi - phi_lo)/h */
void orc_grad_node(const orc_grid* g, const double* phi, double* out)
{
    const int d = g->dim;
    const long N = ncells(g);
    const int nc = 1 << d;
    ORC_PAR_KJ
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i)
                for (int a = 0; a < d; ++a) {
                    double s = 0.0;
                    for (int bits = 0; bits < nc; ++bits) {
                        if (!((bits >> a) & 1)) continue;
                        s += (phi[corner_node(g, i, j, k, bits)] - phi[corner_node(g, i, j, k, bits & ~(1 << a))]) / g->h;
                    }
                    out[(long)a * N + cid(g, i, j, k)] = s / (double)(nc / 2);
                }
}

/* r_k = sum over cells c touching node k of sum_a s_a (h/2)^(d-1) V_a(c):
 * the integral of grad(N_k) . V for the Q1 hat N_k and cellwise constant V. */
void orc_weak_div(const orc_grid* g, const double* V, double* r)
{
    const int d = g->dim;
    const long N = ncells(g);
    const int nc = 1 << d;
    const double w = pow(0.5 * g->h, d - 1);
#ifdef _OPENMP
    ORC_PAR_KJ
    for (int k = 0; k < nnodes(g, 2); ++k)
        for (int j = 0; j < nnodes(g, 1); ++j)
            for (int i = 0; i < nnodes(g, 0); ++i) {
                long cell[8];
                int corner[8];
                const int cnt = node_cells(g, i, j, k, cell, corner);
                double acc = 0.0;
                for (int t = 0; t < cnt; ++t) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) {
                        double sg = ((corner[t] >> a) & 1) ? 1.0 : -1.0;
                        s += sg * w * V[(long)a * N + cell[t]];
                    }
                    acc += s;
                }
                r[nid(g, i, j, k)] = acc;
            }
    (void)nc;
    return;
#endif
    memset(r, 0, sizeof(double) * orc_node_count(g));
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i)
                for (int bits = 0; bits < nc; ++bits) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) {
                        double sg = ((bits >> a) & 1) ? 1.0 : -1.0;
                        s += sg * w * V[(long)a * N + cid(g, i, j, k)];
                    }
                    r[corner_node(g, i, j, k, bits)] += s;
                }
}

/* Q1 element stiffness K_e[p][q] = int grad N_p . grad N_q over a cube of side
 * h, as the sum over axes of (1D stiffness) x (1D mass) products:
 * S = [[1,-1],[-1,1]]/h, M = h [[1/3,1/6],[1/6,1/3]]. */
static void q1_element(int d, double h, double Ke[8][8])
{
    const double S[2][2] = {{1.0 / h, -1.0 / h}, {-1.0 / h, 1.0 / h}};
    const double M[2][2] = {{h / 3.0, h / 6.0}, {h / 6.0, h / 3.0}};
    const int nc = 1 << d;
    for (int p = 0; p < nc; ++p)
        for (int q = 0; q < nc; ++q) {
            double s = 0.0;
            for (int a = 0; a < d; ++a) {
                double t = S[(p >> a) & 1][(q >> a) & 1];
                for (int b = 0; b < d; ++b)
                    if (b != a) t *= M[(p >> b) & 1][(q >> b) & 1];
                s += t;
            }
            Ke[p][q] = s;
        }
}

void orc_apply_K(const orc_grid* g, const double* phi, double* out)
{
    const int d = g->dim;
    const int nc = 1 << d;
    double Ke[8][8];
    q1_element(d, g->h, Ke);
#ifdef _OPENMP
    ORC_PAR_KJ
    for (int k = 0; k < nnodes(g, 2); ++k)
        for (int j = 0; j < nnodes(g, 1); ++j)
            for (int i = 0; i < nnodes(g, 0); ++i) {
                long cell[8];
                int corner[8];
                const int cnt = node_cells(g, i, j, k, cell, corner);
                double acc = 0.0;
                for (int t = 0; t < cnt; ++t) {
                    const long c = cell[t];
                    const int ci = (int)(c % g->n[0]), cj = (int)((c / g->n[0]) % g->n[1]),
                              ck = (int)(c / ((long)g->n[0] * g->n[1]));
                    long ids[8];
                    for (int b = 0; b < nc; ++b) ids[b] = corner_node(g, ci, cj, ck, b);
                    double s = 0.0;
                    for (int q = 0; q < nc; ++q) s += Ke[corner[t]][q] * phi[ids[q]];
                    acc += s;
                }
                out[nid(g, i, j, k)] = acc;
            }
    return;
#endif
    memset(out, 0, sizeof(double) * orc_node_count(g));
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long ids[8];
                for (int b = 0; b < nc; ++b) ids[b] = corner_node(g, i, j, k, b);
                for (int p = 0; p < nc; ++p) {
                    double s = 0.0;
                    for (int q = 0; q < nc; ++q) s += Ke[p][q] * phi[ids[q]];
                    out[ids[p]] += s;
                }
            }
}

/* (K phi) at one node and the diagonal K_kk, assembled from the elements
 * that touch the node */
double orc_K_at(const orc_grid* g, const double* phi, int i, int j, int k, double* diag)
{
    const int d = g->dim;
    const int nc = 1 << d;
    double Ke[8][8];
    q1_element(d, g->h, Ke);
    double s = 0.0, dg = 0.0;
    for (int bits = 0; bits < nc; ++bits) {
        /* the element whose corner `bits` is this node */
        int c[3] = {i, j, k};
        int ok = 1;
        for (int a = 0; a < d; ++a) {
            c[a] -= (bits >> a) & 1;
            if (c[a] < 0) {
                if (is_periodic(g, a)) c[a] += g->n[a]; else ok = 0;
            }
            if (c[a] >= g->n[a]) ok = 0;
        }
        if (!ok) continue;
        for (int q = 0; q < nc; ++q) s += Ke[bits][q] * phi[corner_node(g, c[0], c[1], c[2], q)];
        dg += Ke[bits][bits];
    }
    if (diag) *diag = dg;
    return s;
}

/* ------------------------------------------------------------------------ */
/* MAC (face-centred) operators                                              */
/* ------------------------------------------------------------------------ */

long orc_face_count(const orc_grid* g, int axis) { return face_count(g, axis); }

static long face_offset(const orc_grid* g, int a)
{
    long off = 0;
    for (int b = 0; b < a; ++b) off += face_count(g, b);
    return off;
}

/* D_mac: sum over axes of (F(hi face) - F(lo face)) / h */
void orc_mac_div(const orc_grid* g, const double* faces, double* out)
{
    ORC_PAR_KJ
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                double s = 0.0;
                for (int a = 0; a < g->dim; ++a) {
                    const double* F = faces + face_offset(g, a);
                    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                    hi[a] += 1;
                    if (is_periodic(g, a)) hi[a] %= g->n[a];
                    s += (F[fid(g, a, hi[0], hi[1], hi[2])] - F[fid(g, a, lo[0], lo[1], lo[2])]) / g->h;
                }
                out[cid(g, i, j, k)] = s;
            }
}

/* G_mac on faces: (phi(R) - phi(L)) / h on interior faces, 0 on wall faces */
void orc_mac_grad(const orc_grid* g, const double* phi, double* faces)
{
    for (int a = 0; a < g->dim; ++a) {
        double* F = faces + face_offset(g, a);
        int ext[3] = {g->n[0], g->n[1], g->n[2]};
        ext[a] = nfaces(g, a);
        ORC_PAR_KJ
        for (int k = 0; k < ext[2]; ++k)
            for (int j = 0; j < ext[1]; ++j)
                for (int i = 0; i < ext[0]; ++i) {
                    int R[3] = {i, j, k}, L[3] = {i, j, k};
                    L[a] -= 1;
                    long f = fid(g, a, i, j, k);
                    if (!wrap_cell(g, L) || !wrap_cell(g, R)) { F[f] = 0.0; continue; }
                    F[f] = (phi[cid(g, R[0], R[1], R[2])] - phi[cid(g, L[0], L[1], L[2])]) / g->h;
                }
    }
}

/* L_mac = D_mac G_mac (zero flux through walls) */
void orc_mac_lap(const orc_grid* g, const double* phi, double* out)
{
    long nf = 0;
    for (int a = 0; a < g->dim; ++a) nf += face_count(g, a);
    double* F = (double*)xcalloc(nf, sizeof(double));
    orc_mac_grad(g, phi, F);
    orc_mac_div(g, F, out);
    free(F);
}

double orc_lid_speed(const orc_grid* g)
{
    double m = 0.0;
    for (int a = 0; a < g->dim; ++a)
        for (int s = 0; s < 2; ++s) {
            if (g->bc[a][s] != ORC_WALL) continue;
            for (int c = 0; c < 3; ++c) {
                double v = fabs(g->wall_u[a][s][c]);
                if (v > m) m = v;
            }
        }
    return m;
}
