/* orc_step.c -- the oracle's time step: second-order Godunov advection,
 * MAC projection of the advection velocity, Crank-Nicolson viscous solve with
 * lagged viscosity, approximate nodal projection (Sec. III.A).
 * Test infrastructure only (see orc.h). */
#include "orc_internal.h"

static double sgn(double x) { return (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0); }
static double dmin(double a, double b) { return a < b ? a : b; }

/* Monotonicity-limited fourth-order slope of Colella (1985), in units of q per
 * cell, from five consecutive values q[0..4] centred on q[2] (Sec. III.A). */
static double slope4(const double q[5])
{
    double dc[3], dlim[3], df[3];
    for (int t = 0; t < 3; ++t) {
        double qm = q[t], q0 = q[t + 1], qp = q[t + 2];
        dc[t] = 0.5 * (qp - qm);
        double dp = qp - q0, dm = q0 - qm;
        dlim[t] = (dp * dm > 0.0) ? 2.0 * dmin(fabs(dp), fabs(dm)) : 0.0;
        df[t] = sgn(dc[t]) * dmin(fabs(dc[t]), dlim[t]);
    }
    double d4 = (4.0 / 3.0) * dc[1] - (1.0 / 6.0) * (df[2] + df[0]);
    return sgn(dc[1]) * dmin(fabs(d4), dlim[1]);
}

/* Burgers Riemann solution for the normal velocity (Sec. III.A, the
 * Godunov predictor): uL for a right-moving wave (0 for a rarefaction with
 * uL <= 0), uR for a left-moving one; a stationary shock, |uL + uR| within
 * the dead band, takes the mean of the two */
static double riemann(double uL, double uR, double delta)
{
    const double s = uL + uR;
    const double l = uL > 0.0 ? uL : 0.0, r = uR < 0.0 ? uR : 0.0;
    if (s > delta) return l;
    if (s < -delta) return r;
    return 0.5 * (l + r);
}

/* upwind choice between two face states with a dead band of width delta */
static double upwind(double vel, double qL, double qR, double delta)
{
    if (vel > delta) return qL;
    if (vel < -delta) return qR;
    return 0.5 * (qL + qR);
}

double orc_cfl_dt(const orc_grid* g, double cfl, const double* u)
{
    double U = orc_lid_speed(g);
    double um = vmax_abs(u, ncells(g) * g->dim);
    double m = U > um ? U : um;
    if (m == 0.0) return 0.0;
    return cfl * g->h / m;
}

static long face_off(const orc_grid* g, int a)
{
    long off = 0;
    for (int b = 0; b < a; ++b) off += face_count(g, b);
    return off;
}

/* implicit weight of the viscous update; 0 selects Crank-Nicolson */
double orc_theta(const orc_step_opts* o)
{
    return o->theta > 0.0 ? o->theta : 0.5;
}

/* Godunov predictor, MAC projection and the right-hand side of the viscous
 * solve:  b = u - dt A + dt(-G p + 2(1 - theta) E + f),  with
 *   E = div(eta_e gamma_dot(u^m)) (half the explicit stress divergence),
 *   F = -G p + f, or -G p + 2E + f with pred_visc (the forcing of the Taylor
 *       prediction, eq:iamr:extrap),
 *   A = [u^MAC . grad u~]         (convective term, non-conservative form).
 * Crank-Nicolson (theta = 1/2) is the update printed in Sec. III.A. */
int orc_advect(const orc_grid* g, const orc_fluid* fl, const orc_step_opts* o,
               const double* u, const double* p, const double* eta, double dt,
               double* b, double* E_out, double* umac_out, double* A_out,
               orc_mg_report* mac_rep, double* div_mac_rel)
{
    const int d = g->dim;
    const long N = ncells(g);
    const double h = g->h;
    long nf_tot = 0;
    for (int a = 0; a < d; ++a) nf_tot += face_count(g, a);

    double* eta_e = (double*)xcalloc(N, sizeof(double));
    for (long i = 0; i < N; ++i) eta_e[i] = eta[i] / fl->Re;
    double* E = (double*)xcalloc(N * d, sizeof(double));
    double* Gp = (double*)xcalloc(N * d, sizeof(double));
    double* F = (double*)xcalloc(N * d, sizeof(double));
    orc_visc_div(g, eta_e, u, 0, E);
    orc_grad_node(g, p, Gp);
    /* weight of E in the predictor forcing: 2 (the whole stress divergence,
     * as printed) or 0; and in b: 2 (1 - theta), 1 for Crank-Nicolson */
    const double wF = o->pred_visc ? 2.0 : 0.0;
    const double wb = 2.0 * (1.0 - orc_theta(o));
    for (int c = 0; c < d; ++c)
        for (long i = 0; i < N; ++i)
            F[(long)c * N + i] = -Gp[(long)c * N + i] + wF * E[(long)c * N + i] + fl->f[c];

    const double delta = 1e-12 * fmax(orc_lid_speed(g), vmax_abs(u, N * d));

    /* T1: slopes S[a][q][cell] */
    double* S = (double*)xcalloc(N * d * d, sizeof(double));
    for (int a = 0; a < d; ++a)
        for (int q = 0; q < d; ++q)
            ORC_PAR_KJ
            for (int k = 0; k < g->n[2]; ++k)
                for (int j = 0; j < g->n[1]; ++j)
                    for (int i = 0; i < g->n[0]; ++i) {
                        double st[5];
                        for (int t = 0; t < 5; ++t) {
                            int pp[3] = {i, j, k};
                            pp[a] += t - 2;
                            st[t] = cell_val(g, u + (long)q * N, q, pp, 0);
                        }
                        S[((long)a * d + q) * N + cid(g, i, j, k)] = slope4(st);
                    }
#define SL(a, q, cell) S[((long)(a) * d + (q)) * N + (cell)]
#define U(q, cell) u[(long)(q) * N + (cell)]

    /* T2/T3: normal-only traced states, upwinded: uhat[a][face], qhat[a][q][face] */
    double* uhat = (double*)xcalloc(nf_tot, sizeof(double));
    double* qhat = (double*)xcalloc(nf_tot * d, sizeof(double));
    for (int a = 0; a < d; ++a) {
        int ext[3] = {g->n[0], g->n[1], g->n[2]};
        ext[a] = nfaces(g, a);
        const long off = face_off(g, a);
        ORC_PAR_KJ
        for (int k = 0; k < ext[2]; ++k)
            for (int j = 0; j < ext[1]; ++j)
                for (int i = 0; i < ext[0]; ++i) {
                    long f = off + fid(g, a, i, j, k);
                    int R[3] = {i, j, k}, L[3] = {i, j, k};
                    L[a] -= 1;
                    int okL = wrap_cell(g, L), okR = wrap_cell(g, R);
                    if (!okL || !okR) {    /* wall face: wall values */
                        int side = okL ? 1 : 0;
                        uhat[f] = 0.0;
                        for (int q = 0; q < d; ++q) qhat[(long)q * nf_tot + f] = g->wall_u[a][side][q];
                        continue;
                    }
                    long cL = cid(g, L[0], L[1], L[2]), cR = cid(g, R[0], R[1], R[2]);
                    double qL[3], qR[3];
                    for (int q = 0; q < d; ++q) {
                        qL[q] = U(q, cL) + (0.5 - dt * U(a, cL) / (2.0 * h)) * SL(a, q, cL);
                        qR[q] = U(q, cR) - (0.5 + dt * U(a, cR) / (2.0 * h)) * SL(a, q, cR);
                    }
                    double uh = riemann(qL[a], qR[a], delta);
                    uhat[f] = uh;
                    for (int q = 0; q < d; ++q)
                        qhat[(long)q * nf_tot + f] = (q == a) ? uh : upwind(uh, qL[q], qR[q], delta);
                }
    }

    /* T4: transverse terms trans[b][q][cell] = (u_b dq/dx_b)^ */
    double* trans = (double*)xcalloc(N * d * d, sizeof(double));
    for (int bb = 0; bb < d; ++bb) {
        const long off = face_off(g, bb);
        for (int q = 0; q < d; ++q)
            ORC_PAR_KJ
            for (int k = 0; k < g->n[2]; ++k)
                for (int j = 0; j < g->n[1]; ++j)
                    for (int i = 0; i < g->n[0]; ++i) {
                        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                        hi[bb] += 1;
                        if (is_periodic(g, bb)) hi[bb] %= g->n[bb];
                        long flo = off + fid(g, bb, lo[0], lo[1], lo[2]);
                        long fhi = off + fid(g, bb, hi[0], hi[1], hi[2]);
                        double ubar = 0.5 * (uhat[flo] + uhat[fhi]);
                        double dq = (qhat[(long)q * nf_tot + fhi] - qhat[(long)q * nf_tot + flo]) / h;
                        trans[((long)bb * d + q) * N + cid(g, i, j, k)] = ubar * dq;
                    }
    }
#define TR(b, q, cell) trans[((long)(b) * d + (q)) * N + (cell)]

    /* T5/T6: full states qLf, qRf [q][face] and the advection velocity */
    double* qLf = (double*)xcalloc(nf_tot * d, sizeof(double));
    double* qRf = (double*)xcalloc(nf_tot * d, sizeof(double));
    double* uadv = (double*)xcalloc(nf_tot, sizeof(double));
    for (int a = 0; a < d; ++a) {
        int ext[3] = {g->n[0], g->n[1], g->n[2]};
        ext[a] = nfaces(g, a);
        const long off = face_off(g, a);
        ORC_PAR_KJ
        for (int k = 0; k < ext[2]; ++k)
            for (int j = 0; j < ext[1]; ++j)
                for (int i = 0; i < ext[0]; ++i) {
                    long f = off + fid(g, a, i, j, k);
                    int R[3] = {i, j, k}, L[3] = {i, j, k};
                    L[a] -= 1;
                    int okL = wrap_cell(g, L), okR = wrap_cell(g, R);
                    if (!okL || !okR) {
                        int side = okL ? 1 : 0;
                        uadv[f] = 0.0;
                        for (int q = 0; q < d; ++q) {
                            qLf[(long)q * nf_tot + f] = g->wall_u[a][side][q];
                            qRf[(long)q * nf_tot + f] = g->wall_u[a][side][q];
                        }
                        continue;
                    }
                    long cL = cid(g, L[0], L[1], L[2]), cR = cid(g, R[0], R[1], R[2]);
                    for (int q = 0; q < d; ++q) {
                        double tl = 0.0, tr = 0.0;
                        for (int bb = 0; bb < d; ++bb) {
                            if (bb == a) continue;
                            tl += TR(bb, q, cL);
                            tr += TR(bb, q, cR);
                        }
                        double vl = U(q, cL) + (0.5 - dt * U(a, cL) / (2.0 * h)) * SL(a, q, cL)
                                    - 0.5 * dt * tl + 0.5 * dt * F[(long)q * N + cL];
                        double vr = U(q, cR) - (0.5 + dt * U(a, cR) / (2.0 * h)) * SL(a, q, cR)
                                    - 0.5 * dt * tr + 0.5 * dt * F[(long)q * N + cR];
                        qLf[(long)q * nf_tot + f] = vl;
                        qRf[(long)q * nf_tot + f] = vr;
                    }
                    uadv[f] = riemann(qLf[(long)a * nf_tot + f], qRf[(long)a * nf_tot + f], delta);
                }
    }

    /* T7: MAC projection  L_mac phi = D_mac u^adv,  u^MAC = u^adv - G_mac phi */
    double* umac = (double*)xcalloc(nf_tot, sizeof(double));
    memcpy(umac, uadv, sizeof(double) * nf_tot);
    int rc = ORC_OK;
    if (o->mac_project) {
        double* div = (double*)xcalloc(N, sizeof(double));
        double* phi = (double*)xcalloc(N, sizeof(double));
        double* gphi = (double*)xcalloc(nf_tot, sizeof(double));
        orc_mac_div(g, uadv, div);
        double d0 = vmax_abs(div, N);
        rc = orc_mg_solve(g, fl, ORC_OP_MAC, NULL, 0.0, div, phi, &o->mac, mac_rep);
        orc_mac_grad(g, phi, gphi);
        for (long f = 0; f < nf_tot; ++f) umac[f] = uadv[f] - gphi[f];
        orc_mac_div(g, umac, div);
        if (div_mac_rel) *div_mac_rel = d0 > 0.0 ? vmax_abs(div, N) / d0 : 0.0;
        free(div);
        free(phi);
        free(gphi);
    } else {
        if (mac_rep) memset(mac_rep, 0, sizeof(*mac_rep));
        if (div_mac_rel) *div_mac_rel = 0.0;
    }

    /* T8/T9: upwind full states by u^MAC, convective term A */
    double* A = (double*)xcalloc(N * d, sizeof(double));
    for (int a = 0; a < d; ++a) {
        const long off = face_off(g, a);
        for (int q = 0; q < d; ++q)
            ORC_PAR_KJ
            for (int k = 0; k < g->n[2]; ++k)
                for (int j = 0; j < g->n[1]; ++j)
                    for (int i = 0; i < g->n[0]; ++i) {
                        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                        hi[a] += 1;
                        if (is_periodic(g, a)) hi[a] %= g->n[a];
                        long flo = off + fid(g, a, lo[0], lo[1], lo[2]);
                        long fhi = off + fid(g, a, hi[0], hi[1], hi[2]);
                        double tlo = upwind(umac[flo], qLf[(long)q * nf_tot + flo], qRf[(long)q * nf_tot + flo], delta);
                        double thi = upwind(umac[fhi], qLf[(long)q * nf_tot + fhi], qRf[(long)q * nf_tot + fhi], delta);
                        A[(long)q * N + cid(g, i, j, k)] += 0.5 * (umac[flo] + umac[fhi]) * (thi - tlo) / h;
                    }
    }

    for (int c = 0; c < d; ++c)
        for (long i = 0; i < N; ++i) {
            long q = (long)c * N + i;
            b[q] = u[q] - dt * A[q] + dt * (-Gp[q] + wb * E[q] + fl->f[c]);
        }
    if (E_out) memcpy(E_out, E, sizeof(double) * N * d);
    if (umac_out) memcpy(umac_out, umac, sizeof(double) * nf_tot);
    if (A_out) memcpy(A_out, A, sizeof(double) * N * d);
#undef SL
#undef U
#undef TR
    free(eta_e); free(E); free(Gp); free(F); free(S); free(uhat); free(qhat);
    free(trans); free(qLf); free(qRf); free(uadv); free(umac); free(A);
    return rc;
}

/* Approximate projection: V = ustar / dt + G p;  K phi = r(V);
 * u^{m+1} = ustar + dt (G p - G phi);  p^{m+1/2} = phi (mean zero). */
int orc_project(const orc_grid* g, const orc_step_opts* o, const double* ustar,
                double* p, double dt, double* u_out, orc_mg_report* rep)
{
    const int d = g->dim;
    const long N = ncells(g);
    const long nn = orc_node_count(g);
    double* Gp = (double*)xcalloc(N * d, sizeof(double));
    double* V = (double*)xcalloc(N * d, sizeof(double));
    double* r = (double*)xcalloc(nn, sizeof(double));
    double* phi = (double*)xcalloc(nn, sizeof(double));
    double* Gphi = (double*)xcalloc(N * d, sizeof(double));
    orc_grad_node(g, p, Gp);
    for (long q = 0; q < N * d; ++q) V[q] = ustar[q] / dt + Gp[q];
    orc_weak_div(g, V, r);
    memcpy(phi, p, sizeof(double) * nn);
    int rc = orc_mg_solve(g, NULL, ORC_OP_NODAL, NULL, 0.0, r, phi, &o->proj, rep);
    orc_grad_node(g, phi, Gphi);
    for (long q = 0; q < N * d; ++q) u_out[q] = ustar[q] + dt * (Gp[q] - Gphi[q]);
    memcpy(p, phi, sizeof(double) * nn);
    free(Gp); free(V); free(r); free(phi); free(Gphi);
    return rc;
}

int orc_step(const orc_grid* g, const orc_fluid* fl, const orc_step_opts* o,
             double* u, double* p, double dt, orc_step_report* rep)
{
    const int d = g->dim;
    const long N = ncells(g);
    const long nn = orc_node_count(g);
    if (!all_finite(u, N * d) || !all_finite(p, nn)) return ORC_ERR_NONFINITE;
    if (dt <= 0.0) dt = orc_cfl_dt(g, o->cfl, u);
    if (!(dt > 0.0)) return ORC_ERR_ARG;
    orc_step_report R;
    memset(&R, 0, sizeof(R));
    R.dt = dt;
    double* eta = (double*)xcalloc(N, sizeof(double));
    double* b = (double*)xcalloc(N * d, sizeof(double));
    double* us = (double*)xcalloc(N * d, sizeof(double));
    int rc = orc_viscosity(g, fl, u, eta);
    int rc2 = ORC_OK;
    if (rc == ORC_OK) rc = orc_advect(g, fl, o, u, p, eta, dt, b, NULL, NULL, NULL, &R.mac, &R.div_mac_rel);
    if (rc == ORC_OK || rc == ORC_ERR_NOCONV) {
        rc2 = rc;
        memcpy(us, u, sizeof(double) * N * d);
        /* (I - 2 theta dt div(eta_e gamma_dot(.))) u* = b */
        rc = orc_mg_solve(g, fl, ORC_OP_VISC, eta, 2.0 * orc_theta(o) * dt, b, us, &o->visc, &R.visc);
        if (rc == ORC_OK) rc = rc2;
    }
    if (rc == ORC_OK || rc == ORC_ERR_NOCONV) {
        rc2 = rc;
        rc = orc_project(g, o, us, p, dt, u, &R.proj);
        if (rc == ORC_OK) rc = rc2;
        R.max_u = vmax_abs(u, N * d);
        double* r = (double*)xcalloc(nn, sizeof(double));
        orc_weak_div(g, u, r);
        R.div_node = vmax_abs(r, nn) / pow(g->h, d);
        free(r);
    }
    if (rep) *rep = R;
    free(eta); free(b); free(us);
    return rc;
}
