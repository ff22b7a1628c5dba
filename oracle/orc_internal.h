/* orc_internal.h -- index and boundary helpers private to the oracle.
 * Test infrastructure only (see orc.h). */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H
#include "orc.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static inline long ncells(const orc_grid* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static inline long cid(const orc_grid* g, int i, int j, int k)
{
    return ((long)k * g->n[1] + j) * g->n[0] + i;
}

static inline int is_periodic(const orc_grid* g, int a) { return g->bc[a][0] == ORC_PERIODIC; }

/* nodes along axis a: n+1 on wall axes, n on periodic axes, 1 on unused axes */
static inline int nnodes(const orc_grid* g, int a)
{
    if (a >= g->dim) return 1;
    return is_periodic(g, a) ? g->n[a] : g->n[a] + 1;
}

static inline long nid(const orc_grid* g, int i, int j, int k)
{
    return ((long)k * nnodes(g, 1) + j) * nnodes(g, 0) + i;
}

/* faces normal to axis a: n+1 on wall axes, n on periodic axes */
static inline int nfaces(const orc_grid* g, int a)
{
    return is_periodic(g, a) ? g->n[a] : g->n[a] + 1;
}

/* face array of axis a: the extent along a is nfaces, other axes n */
static inline long fid(const orc_grid* g, int a, int i, int j, int k)
{
    int ex = (a == 0) ? nfaces(g, 0) : g->n[0];
    int ey = (a == 1) ? nfaces(g, 1) : g->n[1];
    return ((long)k * ey + j) * ex + i;
}

static inline long face_count(const orc_grid* g, int a)
{
    long c = 1;
    for (int b = 0; b < 3; ++b) c *= (b == a) ? nfaces(g, b) : g->n[b];
    return c;
}

/* Value of component c of a cell field (pointer to that component's data) at
 * cell index p, which may lie up to two cells outside the domain along one
 * wall axis.  Wall ghosts are the odd reflection about the wall value:
 * q(-k) = 2 u_b - q(k-1); periodic axes wrap.  hom = 1 uses u_b = 0. */
static inline double cell_val(const orc_grid* g, const double* q, int c, const int p_in[3], int hom)
{
    int p[3] = {p_in[0], p_in[1], p_in[2]};
    int out_axis = -1, side = 0;
    for (int a = 0; a < g->dim; ++a) {
        int n = g->n[a];
        if (p[a] >= 0 && p[a] < n) continue;
        if (is_periodic(g, a)) {
            p[a] = ((p[a] % n) + n) % n;
            continue;
        }
        if (out_axis >= 0) {
            fprintf(stderr, "oracle: corner ghost requested\n");
            abort();
        }
        out_axis = a;
        side = p[a] < 0 ? 0 : 1;
        p[a] = p[a] < 0 ? -1 - p[a] : 2 * n - 1 - p[a];
        if (p[a] < 0 || p[a] >= n) {
            fprintf(stderr, "oracle: ghost beyond two layers\n");
            abort();
        }
    }
    double v = q[cid(g, p[0], p[1], p[2])];
    if (out_axis < 0) return v;
    double ub = hom ? 0.0 : g->wall_u[out_axis][side][c];
    return 2.0 * ub - v;
}

/* wrap a cell index on periodic axes; returns 0 if it lies outside a wall */
static inline int wrap_cell(const orc_grid* g, int p[3])
{
    for (int a = 0; a < g->dim; ++a) {
        int n = g->n[a];
        if (p[a] >= 0 && p[a] < n) continue;
        if (!is_periodic(g, a)) return 0;
        p[a] = ((p[a] % n) + n) % n;
    }
    return 1;
}

static inline void* xcalloc(long n, long sz)
{
    void* p = calloc((size_t)(n > 0 ? n : 1), (size_t)sz);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

/* Timing build only (compiled with -fopenmp): the planes and rows of a loop
 * nest, or of one colour of a smoother, split over threads.  The parity
 * build has no OpenMP and runs every loop in order. */
#ifdef _OPENMP
#define ORC_PAR_KJ _Pragma("omp parallel for collapse(2) schedule(static) if (orc_par_ok(g))")
#else
#define ORC_PAR_KJ
#endif

/* a loop nest over a grid is worth splitting only on the larger levels */
static inline int orc_par_ok(const orc_grid* g) { return (long)g->n[0] * g->n[1] * g->n[2] >= 4096; }

static inline double vmax_abs(const double* v, long n)
{
    double m = 0.0;
    for (long i = 0; i < n; ++i) { double a = fabs(v[i]); if (a > m) m = a; }
    return m;
}

static inline int all_finite(const double* v, long n)
{
    for (long i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
    return 1;
}

/* internal entry points shared between oracle files */
void orc_tensor_apply_h(const orc_grid* g, const double* beta, double dt, const double* u, double* out);
double orc_tensor_diag(const orc_grid* g, const double* beta, double dt, int c, int i, int j, int k);
void orc_eta_faces(const orc_grid* g, const double* eta_e, double* beta);
void orc_visc_div_faces(const orc_grid* g, const double* beta, const double* u, int hom, double* out);
long orc_face_offset(const orc_grid* g, int a);
void orc_mac_lap(const orc_grid* g, const double* phi, double* out);
void orc_mac_grad(const orc_grid* g, const double* phi, double* faces);
double orc_lid_speed(const orc_grid* g);
double orc_visc_div_at(const orc_grid* g, const double* beta, const double* u, int hom,
                       int c, int i, int j, int k);
double orc_K_at(const orc_grid* g, const double* phi, int i, int j, int k, double* diag);

#endif
