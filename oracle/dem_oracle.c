/*
 * dem_oracle.c -- plain, slow FP64 reference for one soft-sphere DEM timestep.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library: it is written from the paper
 * (Washizawa & Nakahara, "Parallel Computing of Discrete Element Method on
 * GPU", arXiv:1301.1714) and nothing else.
 *
 * What it computes, in the paper's order (Sec. 4.2, Steps 1-8):
 *   Step 1  update of all particle properties: kick-drift-kick velocity Verlet
 *   Step 2  correspondence map CM: cell id of every particle (Sec. 4.1)
 *   Step 3  sort of CM by (cell, id): SCM[j] = CM[SCCM[j]] (Eq. 11)
 *   Step 5-6  for every particle, the 27 neighbour cells (Eq. 12)
 *   Step 7  pair contact force of the practical model (Eqs. 2-10) or of the
 *           simple model (Eq. 1)
 *   Step 8  particle-wall contact, the wall being a particle of infinite
 *           radius
 * Step 4 (physical reorder) only changes memory layout, so the oracle keeps
 * every array in input (id) order and walks the sorted order SCCM instead.
 *
 * Everything is FP64.  Radii are rounded to FP32 on input (the GPU stores
 * them in FP32); sums of two such radii are exact in FP64.  Build with
 * -ffp-contract=off: the contact test d^2 < (r_i + r_j)^2 and the cell hash
 * must be evaluated as written, with no fused multiply-add.
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *  - n is the unit vector from particle i to its partner j, the relative
 *    velocity is v = v_i - v_j and every force is the force on i; with this
 *    convention Eq. 6's (r_i w_i + r_j w_j) x n is the slip of the contact
 *    point and Eq. 4 is repulsive and dissipative.
 *  - Eq. 1 is applied as F_i = -k_sp d n - k_da v - k_sh v_t; gravity is
 *    added once per particle in the kick, not per pair.  The simple model
 *    produces no torque and keeps no history, and its v_t is the tangential
 *    component v - (v.n) n of the relative velocity (the suffix t as Sec. 3
 *    defines it), without Eq. 6's spin term, which belongs to the practical
 *    model.
 *  - Eq. 4's tangential damping is eta_t = eta_t_ratio * eta (ratio 1 is the
 *    literal reading of Eq. 4).
 *  - Eq. 5 (sliding): the stored tangential displacement is rescaled to the
 *    Coulomb limit, delta_t = -(F_t + eta_t v_t) / k_t when k_t > 0.
 *  - Eq. 10: alpha = -2 ln e / sqrt(pi^2 + ln^2 e), which gives restitution
 *    exactly e for the linear law.
 *  - Eqs. 8-9: |delta_n| / (1/r_i + 1/r_j) = delta * R with R = r_i r_j / S.
 *  - Walls (Step 8): R = r_i, M = m_i, partner velocity and spin are zero.
 *  - Contact iff d^2 < S^2 strictly; a pair's history starts at zero when it
 *    first touches and is dropped as soon as it separates.
 *  - m = rho 4/3 pi r^3, I = 2/5 m r^2 (solid spheres).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum {
    ORC_OK = 0,
    ORC_E_INVALID = -1,
    ORC_E_OUT_OF_DOMAIN = -4,
    ORC_E_NONFINITE = -5,
    ORC_E_NOMEM = -8,
    ORC_E_CAPACITY = -9
};
enum { ORC_LINEAR = 0, ORC_HERTZ = 1, ORC_SIMPLE = 2 };
/* Optional contact terms, each added to the law's result on its own (the
 * paper's C++ code is built so that a force term can be added or removed
 * without touching the rest, Sec. 4; the terms themselves are not in the
 * paper).  Practical law only. */
enum {
    ORC_TERM_COHESION = 1, /* constant attraction f_c along n while in contact */
    ORC_TERM_ROLLING = 2   /* rolling resistance: couple -mu_r R |F_n| w_rel / |w_rel| */
};

/* A finite wall: the rectangle of the plane x[axis] = at spanning lo[0]..hi[0]
 * along axis (axis + 1) % 3 and lo[1]..hi[1] along axis (axis + 2) % 3, of no
 * thickness.  Like the walls of Step 8 it is a body of infinite radius and
 * mass at rest; a sphere touches it where the nearest point of the rectangle
 * is closer than its radius, and n points from the centre to that point.  Two
 * such plates side by side leave a slit between them (Sec. 5's box with a
 * slit at its bottom). */
typedef struct {
    int32_t axis, pad_;
    double at;
    double lo[2], hi[2];
} orc_plate;
enum { ORC_MAX_PLATES = 4 };

typedef struct {
    double lo[3], hi[3];
    int32_t wall_mask; /* bit 2a: wall at lo[a]; bit 2a+1: wall at hi[a] */
    int32_t law;
    double g[3];
    double dt, rho;
    double kn, kt;     /* linear: springs; Hertz: C_kn, C_kt of Eqs. 8-9 */
    double e;          /* restitution parameter, fixes alpha of Eq. 10 */
    double eta_t_ratio;
    double mu;
    double k_sp, k_da, k_sh; /* Eq. 1 */
    double cell;       /* requested cell width, >= 2 r_max */
    int32_t terms;     /* ORC_TERM_* bits */
    int32_t pad_;
    double cohesion;   /* f_c (N) of ORC_TERM_COHESION */
    double rolling_mu; /* mu_r of ORC_TERM_ROLLING */
    int32_t nplates;   /* finite walls, numbered 6, 7, ... after the six box walls */
    int32_t pad2_;
    orc_plate plates[ORC_MAX_PLATES];
} orc_params;

/* One history entry: the pair (a, b) with a < b seen from a, or the wall
 * contact (a, -1-w).  d is the tangential displacement delta_t of Eq. 7. */
typedef struct {
    int64_t a, b;
    double d[3];
} orc_hentry;

typedef struct {
    int64_t a, b; /* a < b, or b = -1-w for wall w */
} orc_contact;

/* Contact constants of one pair of materials (Sec. 3: the C_kn, C_kt and
 * alpha of Eqs. 8-10 carry the indices of the two particles' materials, and
 * so does the friction coefficient of Eq. 5 here): the springs (linear law)
 * or the Hertz constants, alpha from the pair's restitution, mu. */
typedef struct {
    double kn, kt, alpha, mu;
} orc_pairk;

enum { ORC_MAX_TYPES = 16 };

typedef struct {
    orc_params p;
    int64_t n;
    double *x, *v, *w, *F, *T; /* 3n, [i*3 + axis], id order */
    double *r, *m, *I;
    int32_t nc[3];
    double sc[3];
    int64_t ncell;
    double alpha;
    orc_hentry *H;
    int64_t nH;
    int64_t steps;
    /* material-pair table: ntypes = 0 means one material (the orc_params
     * constants); otherwise type[i] is particle i's material, walls are of
     * material wall_type, and mat[t * ntypes + u] holds the pair (t, u) */
    int32_t ntypes, wall_type;
    int32_t *type;
    orc_pairk *mat;
} orc_sys;

/* Eq. 10's alpha for restitution e: -2 ln e / sqrt(pi^2 + ln^2 e), which
 * makes a linear contact's restitution exactly e (no damping at e = 1) */
static double alpha_of(double e)
{
    return e >= 1.0 ? 0.0 : -2.0 * log(e) / sqrt(M_PI * M_PI + log(e) * log(e));
}

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------ */
/* Step 2: the correspondence map CM (Sec. 4.1).  Cell counts n_a are
 * floor(L_a / cell) so that every cell is at least the requested width, and
 * the coordinate is scaled by s_a = n_a / L_a.  A particle further than one
 * cell outside the box is an error; one closer is clamped into the edge cell. */

static int cell_of(const orc_sys *s, const double *x, int32_t *ijk)
{
    for (int a = 0; a < 3; a++) {
        double u = (x[a] - s->p.lo[a]) * s->sc[a];
        if (!(u >= -1.0 && u < (double)s->nc[a] + 1.0)) return ORC_E_OUT_OF_DOMAIN;
        double f = floor(u);
        int32_t i = f < 0.0 ? 0 : (int32_t)f;
        if (i > s->nc[a] - 1) i = s->nc[a] - 1;
        ijk[a] = i;
    }
    return ORC_OK;
}

static int64_t linear_cell(const orc_sys *s, const int32_t *ijk)
{
    return (int64_t)ijk[0] + (int64_t)s->nc[0] * ((int64_t)ijk[1] + (int64_t)s->nc[1] * (int64_t)ijk[2]);
}

typedef struct {
    int32_t *cm;     /* CM[id] */
    int32_t *sccm;   /* SCCM[slot] = id */
    int32_t *start;  /* ncell + 1 */
} orc_grid;

static const int32_t *g_sort_cm; /* comparator context (single-threaded oracle) */

static int cmp_cell_id(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_sort_cm[a] != g_sort_cm[b]) return g_sort_cm[a] < g_sort_cm[b] ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static void grid_free(orc_grid *g)
{
    free(g->cm);
    free(g->sccm);
    free(g->start);
    memset(g, 0, sizeof(*g));
}

/* Steps 2-3: CM, then SCCM = order of ids sorted by (CM, id), which makes
 * SCM[j] = CM[SCCM[j]] (Eq. 11) non-decreasing; start[c] is the first slot
 * of cell c (an exclusive scan of the cell counts, start[ncell] = n). */
static int grid_build(const orc_sys *s, orc_grid *g)
{
    int64_t n = s->n;
    memset(g, 0, sizeof(*g));
    g->cm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    g->sccm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    g->start = (int32_t *)calloc((size_t)s->ncell + 1, sizeof(int32_t));
    if (!g->cm || !g->sccm || !g->start) {
        grid_free(g);
        return ORC_E_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) {
        int32_t ijk[3];
        if (cell_of(s, s->x + 3 * i, ijk) != ORC_OK) {
            grid_free(g);
            return ORC_E_OUT_OF_DOMAIN;
        }
        g->cm[i] = (int32_t)linear_cell(s, ijk);
        g->sccm[i] = (int32_t)i;
    }
    g_sort_cm = g->cm;
    qsort(g->sccm, (size_t)n, sizeof(int32_t), cmp_cell_id);
    g_sort_cm = NULL;
    for (int64_t i = 0; i < n; i++) g->start[g->cm[i] + 1]++;
    for (int64_t c = 0; c < s->ncell; c++) g->start[c + 1] += g->start[c];
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Steps 5-8, detection: every pair (a, b), a < b, with d^2 < S^2 among the
 * particles of the 27 cells around a's cell (Eq. 12), then a's walls.     */

static int pair_touch(const orc_sys *s, int64_t a, int64_t b)
{
    const double *xa = s->x + 3 * a, *xb = s->x + 3 * b;
    double dx = xb[0] - xa[0], dy = xb[1] - xa[1], dz = xb[2] - xa[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double S = s->r[a] + s->r[b];
    return d2 < S * S;
}

/* nearest point q of plate k to the centre c, and c - q */
static void plate_nearest(const orc_plate *P, const double *c, double q[3], double d[3])
{
    int u = (P->axis + 1) % 3, v = (P->axis + 2) % 3;
    q[P->axis] = P->at;
    q[u] = c[u] < P->lo[0] ? P->lo[0] : (c[u] > P->hi[0] ? P->hi[0] : c[u]);
    q[v] = c[v] < P->lo[1] ? P->lo[1] : (c[v] > P->hi[1] ? P->hi[1] : c[v]);
    for (int k = 0; k < 3; k++) d[k] = c[k] - q[k];
}

/* wall w: 0..5 the box walls (Step 8), 6.. the plates */
static int wall_touch(const orc_sys *s, int64_t a, int w)
{
    if (w >= 6) {
        double q[3], d[3];
        plate_nearest(&s->p.plates[w - 6], s->x + 3 * a, q, d);
        return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2] < s->r[a] * s->r[a];
    }
    int axis = w >> 1;
    double gap = (w & 1) ? (s->p.hi[axis] - s->x[3 * a + axis]) : (s->x[3 * a + axis] - s->p.lo[axis]);
    return gap < s->r[a];
}

typedef struct {
    orc_contact *c;
    int64_t n, cap;
} orc_clist;

static int clist_push(orc_clist *L, int64_t a, int64_t b)
{
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 1024;
        orc_contact *p = (orc_contact *)realloc(L->c, sizeof(orc_contact) * (size_t)nc);
        if (!p) return ORC_E_NOMEM;
        L->c = p;
        L->cap = nc;
    }
    L->c[L->n].a = a;
    L->c[L->n].b = b;
    L->n++;
    return ORC_OK;
}

static int detect(const orc_sys *s, const orc_grid *g, orc_clist *L)
{
    L->c = NULL;
    L->n = L->cap = 0;
    for (int64_t slot = 0; slot < s->n; slot++) {
        int64_t a = g->sccm[slot];
        int32_t ijk[3] = {0, 0, 0};
        cell_of(s, s->x + 3 * a, ijk); /* in domain: grid_build succeeded */
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int32_t q[3] = {ijk[0] + dx, ijk[1] + dy, ijk[2] + dz};
                    if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= s->nc[0] || q[1] >= s->nc[1] ||
                        q[2] >= s->nc[2])
                        continue;
                    int64_t c = linear_cell(s, q);
                    for (int32_t t = g->start[c]; t < g->start[c + 1]; t++) {
                        int64_t b = g->sccm[t];
                        if (b <= a) continue;
                        if (pair_touch(s, a, b) && clist_push(L, a, b) != ORC_OK) return ORC_E_NOMEM;
                    }
                }
        for (int w = 0; w < 6 + s->p.nplates; w++)
            if ((w >= 6 || ((s->p.wall_mask >> w) & 1)) && wall_touch(s, a, w))
                if (clist_push(L, a, -1 - (int64_t)w) != ORC_OK) return ORC_E_NOMEM;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 7: contact law.  Geometry of one contact seen from particle i.     */

typedef struct {
    double n[3];     /* unit vector from i towards the partner */
    double delta;    /* overlap S - d (pair) or r_i - gap (wall) */
    double R;        /* r_i r_j / (r_i + r_j), or r_i for a wall */
    double M;        /* m_i m_j / (m_i + m_j), or m_i for a wall */
    double v[3];     /* v_i - v_j */
    double spin[3];  /* r_i w_i + r_j w_j */
    double wrel[3];  /* w_i - w_j (rolling resistance) */
} orc_geom;

static int pair_geom(const orc_sys *s, int64_t a, int64_t b, orc_geom *G)
{
    const double *xa = s->x + 3 * a, *xb = s->x + 3 * b;
    double dx[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
    double d = sqrt((dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]);
    double S = s->r[a] + s->r[b];
    if (!(d > 0.0)) return ORC_E_NONFINITE; /* coincident centres: n undefined */
    for (int k = 0; k < 3; k++) {
        G->n[k] = dx[k] / d;
        G->v[k] = s->v[3 * a + k] - s->v[3 * b + k];
        G->spin[k] = s->r[a] * s->w[3 * a + k] + s->r[b] * s->w[3 * b + k];
        G->wrel[k] = s->w[3 * a + k] - s->w[3 * b + k];
    }
    G->delta = S - d;
    G->R = s->r[a] * s->r[b] / S;
    G->M = s->m[a] * s->m[b] / (s->m[a] + s->m[b]);
    return ORC_OK;
}

static int wall_geom(const orc_sys *s, int64_t a, int w, orc_geom *G)
{
    if (w >= 6) {
        double q[3], d[3];
        plate_nearest(&s->p.plates[w - 6], s->x + 3 * a, q, d);
        double dist = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        if (!(dist > 0.0)) return ORC_E_NONFINITE; /* centre on the plate: n undefined */
        for (int k = 0; k < 3; k++) {
            G->n[k] = -d[k] / dist;
            G->v[k] = s->v[3 * a + k];
            G->spin[k] = s->r[a] * s->w[3 * a + k];
            G->wrel[k] = s->w[3 * a + k];
        }
        G->delta = s->r[a] - dist;
        G->R = s->r[a];
        G->M = s->m[a];
        return ORC_OK;
    }
    int axis = w >> 1;
    double gap = (w & 1) ? (s->p.hi[axis] - s->x[3 * a + axis]) : (s->x[3 * a + axis] - s->p.lo[axis]);
    for (int k = 0; k < 3; k++) {
        G->n[k] = 0.0;
        G->v[k] = s->v[3 * a + k];
        G->spin[k] = s->r[a] * s->w[3 * a + k];
        G->wrel[k] = s->w[3 * a + k];
    }
    G->n[axis] = (w & 1) ? 1.0 : -1.0;
    G->delta = s->r[a] - gap;
    G->R = s->r[a];
    G->M = s->m[a];
    return ORC_OK;
}

/* The contact constants of particle a with partner b (b = -1-w: wall w):
 * the system's one material, or the entry of the two materials in the
 * material-pair table. */
static orc_pairk pair_consts(const orc_sys *s, int64_t a, int64_t b)
{
    orc_pairk k;
    if (s->ntypes == 0) {
        k.kn = s->p.kn;
        k.kt = s->p.kt;
        k.alpha = s->alpha;
        k.mu = s->p.mu;
        return k;
    }
    int32_t ta = s->type[a], tb = b >= 0 ? s->type[b] : s->wall_type;
    return s->mat[(int64_t)ta * s->ntypes + tb];
}

/* Eqs. 2, 4-10 for one contact with constants K.  h is the previous
 * tangential displacement delta_t,old (zero for a new contact).  Returns the
 * total force on i (F), its tangential part (Ft, which sets the torque of
 * Eq. 3) and the new tangential displacement (dt_new).  Also the normal and
 * tangential stiffness actually used, for the elastic-energy diagnostic, and
 * |F_n| of Eq. 4 (the magnitude Eq. 5 compares with). */
static void contact_law(const orc_sys *s, const orc_pairk *K, const orc_geom *G, const double h[3], double F[3],
                        double Ft[3], double dt_new[3], double *kn_out, double *kt_out, double *fn_out)
{
    const orc_params *p = &s->p;
    double vn_s = dot3(G->v, G->n);
    double vn[3], sxn[3], vt[3];
    cross3(G->spin, G->n, sxn);
    for (int k = 0; k < 3; k++) {
        vn[k] = vn_s * G->n[k];
        vt[k] = G->v[k] - vn[k] + sxn[k]; /* Eq. 6 */
    }
    if (p->law == ORC_SIMPLE) { /* Eq. 1, gravity excluded */
        /* Sec. 3 defines the suffix t of Eq. 1 as the tangential component of
         * the relative velocity v; the simple model carries no rotation, so
         * Eq. 6's spin term does not enter it */
        double vts[3];
        for (int k = 0; k < 3; k++) vts[k] = G->v[k] - vn[k];
        for (int k = 0; k < 3; k++) {
            F[k] = -p->k_sp * G->delta * G->n[k] - p->k_da * G->v[k] - p->k_sh * vts[k];
            Ft[k] = 0.0;
            dt_new[k] = 0.0;
        }
        *kn_out = p->k_sp;
        *kt_out = 0.0;
        *fn_out = 0.0;
        return;
    }
    double kn, kt;
    if (p->law == ORC_HERTZ) { /* Eqs. 8-9 */
        double q = sqrt(G->delta * G->R);
        kn = K->kn * q;
        kt = K->kt * q;
    } else {
        kn = K->kn;
        kt = K->kt;
    }
    double eta = K->alpha * sqrt(kn * G->M); /* Eq. 10 */
    double eta_t = p->eta_t_ratio * eta;
    double hn = dot3(h, G->n);
    double Fn[3];
    for (int k = 0; k < 3; k++) {
        dt_new[k] = h[k] - hn * G->n[k] + vt[k] * p->dt;     /* Eq. 7 */
        Fn[k] = -kn * G->delta * G->n[k] - eta * vn[k];       /* Eq. 4, normal */
        Ft[k] = -kt * dt_new[k] - eta_t * vt[k];              /* Eq. 4, tangential */
    }
    double ftn = norm3(Ft), fnn = norm3(Fn);
    if (ftn > K->mu * fnn) { /* Eq. 5 */
        double scale = K->mu * fnn / ftn;
        for (int k = 0; k < 3; k++) Ft[k] *= scale;
        if (kt > 0.0)
            for (int k = 0; k < 3; k++) dt_new[k] = -(Ft[k] + eta_t * vt[k]) / kt;
    }
    for (int k = 0; k < 3; k++) F[k] = Fn[k] + Ft[k]; /* Eq. 2 */
    *kn_out = kn;
    *kt_out = kt;
    *fn_out = fnn;
}

/* The optional terms of the contact, each added on its own after the law:
 *  cohesion  F_i += f_c n: a constant pull towards the partner (or the wall)
 *            while the bodies overlap; it does not enter Eq. 5's limit.
 *  rolling   a couple C = -mu_r R |F_n| w_rel / |w_rel| on i and -C on the
 *            partner (nothing on a wall), with R of Eqs. 8-9 (r_i for a
 *            wall), |F_n| of Eq. 4 and w_rel = w_i - w_j; zero when
 *            w_rel = 0.  This is the constant directional torque model of
 *            rolling resistance, which also opposes spin about n.
 * Neither is in the paper; they exercise the composition of force terms. */
static void extra_terms(const orc_sys *s, const orc_geom *G, double fn, double F[3], double C[3])
{
    const orc_params *p = &s->p;
    C[0] = C[1] = C[2] = 0.0;
    if (p->terms & ORC_TERM_COHESION)
        for (int k = 0; k < 3; k++) F[k] += p->cohesion * G->n[k];
    if (p->terms & ORC_TERM_ROLLING) {
        double wn = norm3(G->wrel);
        if (wn > 0.0)
            for (int k = 0; k < 3; k++) C[k] = -p->rolling_mu * G->R * fn * G->wrel[k] / wn;
    }
}

/* ------------------------------------------------------------------ */
/* history lookup                                                          */

static int cmp_hentry(const void *pa, const void *pb)
{
    const orc_hentry *x = (const orc_hentry *)pa, *y = (const orc_hentry *)pb;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

static const orc_hentry *hist_find(const orc_sys *s, int64_t a, int64_t b)
{
    orc_hentry key;
    key.a = a;
    key.b = b;
    if (s->nH == 0) return NULL;
    return (const orc_hentry *)bsearch(&key, s->H, (size_t)s->nH, sizeof(orc_hentry), cmp_hentry);
}

/* ------------------------------------------------------------------ */
/* Steps 2-8: forces on the current state.  Each pair is visited once and
 * its force applied with opposite signs to the two particles; the torque
 * r (n x F_t) of Eq. 3 has the same sign on both (n and F_t both flip).
 * When commit is set the new history replaces the old one.              */

static int evaluate(orc_sys *s, double *F, double *T, int commit, double *e_el, int64_t *npair,
                    int64_t *nwall, double *dmax, double *Fabs, double *Tabs)
{
    orc_grid g;
    orc_clist L;
    int st = grid_build(s, &g);
    if (st != ORC_OK) return st;
    st = detect(s, &g, &L);
    grid_free(&g);
    if (st != ORC_OK) {
        free(L.c);
        return st;
    }
    orc_hentry *Hn = NULL;
    if (s->p.law != ORC_SIMPLE && L.n > 0) {
        Hn = (orc_hentry *)malloc(sizeof(orc_hentry) * (size_t)L.n);
        if (!Hn) {
            free(L.c);
            return ORC_E_NOMEM;
        }
    }
    memset(F, 0, sizeof(double) * 3 * (size_t)s->n);
    memset(T, 0, sizeof(double) * 3 * (size_t)s->n);
    if (Fabs) memset(Fabs, 0, sizeof(double) * (size_t)s->n);
    if (Tabs) memset(Tabs, 0, sizeof(double) * (size_t)s->n);
    double E = 0.0, Ec = 0.0, dm = 0.0;
    int64_t np = 0, nw = 0;
    for (int64_t k = 0; k < L.n; k++) {
        int64_t a = L.c[k].a, b = L.c[k].b;
        orc_geom G;
        if (b >= 0) {
            st = pair_geom(s, a, b, &G);
            if (st != ORC_OK) {
                free(L.c);
                free(Hn);
                return st;
            }
            np++;
        } else {
            st = wall_geom(s, a, (int)(-1 - b), &G);
            if (st != ORC_OK) {
                free(L.c);
                free(Hn);
                return st;
            }
            nw++;
        }
        const orc_hentry *he = hist_find(s, a, b);
        double zero[3] = {0.0, 0.0, 0.0};
        const double *h = he ? he->d : zero;
        double Fc[3], Ft[3], dtn[3], kn, kt, fn, Cr[3];
        const orc_pairk K = pair_consts(s, a, b);
        contact_law(s, &K, &G, h, Fc, Ft, dtn, &kn, &kt, &fn);
        extra_terms(s, &G, fn, Fc, Cr);
        double nxft[3];
        cross3(G.n, Ft, nxft);
        for (int q = 0; q < 3; q++) {
            F[3 * a + q] += Fc[q];
            T[3 * a + q] += s->r[a] * nxft[q] + Cr[q]; /* Eq. 3, and the rolling couple */
            if (b >= 0) {
                F[3 * b + q] -= Fc[q];
                T[3 * b + q] += s->r[b] * nxft[q] - Cr[q];
            }
        }
        if (Fabs) {
            double fm = norm3(Fc);
            Fabs[a] += fm;
            if (b >= 0) Fabs[b] += fm;
        }
        if (Tabs) {
            Tabs[a] += s->r[a] * norm3(nxft) + norm3(Cr);
            if (b >= 0) Tabs[b] += s->r[b] * norm3(nxft) + norm3(Cr);
        }
        if (Hn) {
            Hn[k].a = a;
            Hn[k].b = b;
            memcpy(Hn[k].d, dtn, sizeof(dtn));
        }
        if (e_el) {
            /* elastic energy of the contact, with the committed history */
            double en;
            if (s->p.law == ORC_HERTZ)
                en = 0.4 * K.kn * sqrt(G.R) * pow(G.delta, 2.5) + 0.5 * kt * dot3(h, h);
            else if (s->p.law == ORC_SIMPLE)
                en = 0.5 * s->p.k_sp * G.delta * G.delta;
            else
                en = 0.5 * kn * G.delta * G.delta + 0.5 * kt * dot3(h, h);
            double y = en - Ec, t = E + y; /* Kahan */
            Ec = (t - E) - y;
            E = t;
            if (G.delta > dm) dm = G.delta;
        }
    }
    for (int64_t i = 0; i < 3 * s->n; i++)
        if (!isfinite(F[i]) || !isfinite(T[i])) {
            free(L.c);
            free(Hn);
            return ORC_E_NONFINITE;
        }
    if (commit) {
        free(s->H);
        s->H = Hn;
        s->nH = Hn ? L.n : 0;
        if (Hn) qsort(s->H, (size_t)s->nH, sizeof(orc_hentry), cmp_hentry);
    } else {
        free(Hn);
    }
    if (e_el) *e_el = E;
    if (npair) *npair = np;
    if (nwall) *nwall = nw;
    if (dmax) *dmax = dm;
    free(L.c);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 1: half kick v += dt/2 (F/m + g), w += dt/2 T/I.               */

static void half_kick(orc_sys *s)
{
    double h = 0.5 * s->p.dt;
    for (int64_t i = 0; i < s->n; i++)
        for (int k = 0; k < 3; k++) {
            s->v[3 * i + k] += h * (s->F[3 * i + k] / s->m[i] + s->p.g[k]);
            s->w[3 * i + k] += h * (s->T[3 * i + k] / s->I[i]);
        }
}

static int all_finite(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* public interface                                                        */

void orc_destroy(orc_sys *s)
{
    if (!s) return;
    free(s->x);
    free(s->v);
    free(s->w);
    free(s->F);
    free(s->T);
    free(s->r);
    free(s->m);
    free(s->I);
    free(s->H);
    free(s->type);
    free(s->mat);
    free(s);
}

/* Create a system.  x, v, w are n x 3 (row per particle), r is n.  F0, T0
 * (n x 3) may be NULL: then the forces are evaluated on the given state with
 * the given history, and that evaluation's history is not kept (history
 * changes once per step).  hist_pairs is nh x 2 ((a, b) with a < b, or
 * (a, -1-w)), hist_dt is nh x 3. */
int orc_create(const orc_params *p, int64_t n, const double *x, const double *v, const double *w,
               const double *r, const double *F0, const double *T0, int64_t nh, const int64_t *hist_pairs,
               const double *hist_dt, orc_sys **out)
{
    *out = NULL;
    if (!p || n < 0 || (n > 0 && (!x || !v || !w || !r))) return ORC_E_INVALID;
    if (!(p->dt > 0.0) || !(p->rho > 0.0) || !(p->cell > 0.0)) return ORC_E_INVALID;
    if (p->law < ORC_LINEAR || p->law > ORC_SIMPLE) return ORC_E_INVALID;
    if (!(p->e > 0.0 && p->e <= 1.0) || !(p->mu >= 0.0)) return ORC_E_INVALID;
    if ((p->terms & ~(ORC_TERM_COHESION | ORC_TERM_ROLLING)) != 0) return ORC_E_INVALID;
    if (p->nplates < 0 || p->nplates > ORC_MAX_PLATES) return ORC_E_INVALID;
    for (int k = 0; k < p->nplates; k++) {
        const orc_plate *P = &p->plates[k];
        if (P->axis < 0 || P->axis > 2 || !isfinite(P->at) || !(P->lo[0] <= P->hi[0]) || !(P->lo[1] <= P->hi[1]) ||
            !isfinite(P->lo[0]) || !isfinite(P->hi[0]) || !isfinite(P->lo[1]) || !isfinite(P->hi[1]))
            return ORC_E_INVALID;
    }
    if (p->terms && (p->law == ORC_SIMPLE || !isfinite(p->cohesion) || !(p->rolling_mu >= 0.0) ||
                     !isfinite(p->rolling_mu)))
        return ORC_E_INVALID;
    if (n > 2000000000) return ORC_E_INVALID;
    orc_sys *s = (orc_sys *)calloc(1, sizeof(orc_sys));
    if (!s) return ORC_E_NOMEM;
    s->p = *p;
    s->n = n;
    size_t n3 = (size_t)(n > 0 ? n : 1) * 3, n1 = (size_t)(n > 0 ? n : 1);
    s->x = (double *)malloc(n3 * sizeof(double));
    s->v = (double *)malloc(n3 * sizeof(double));
    s->w = (double *)malloc(n3 * sizeof(double));
    s->F = (double *)calloc(n3, sizeof(double));
    s->T = (double *)calloc(n3, sizeof(double));
    s->r = (double *)malloc(n1 * sizeof(double));
    s->m = (double *)malloc(n1 * sizeof(double));
    s->I = (double *)malloc(n1 * sizeof(double));
    if (!s->x || !s->v || !s->w || !s->F || !s->T || !s->r || !s->m || !s->I) {
        orc_destroy(s);
        return ORC_E_NOMEM;
    }
    double rmax = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double ri = (double)(float)r[i];
        if (!(ri > 0.0) || !isfinite(ri)) {
            orc_destroy(s);
            return ORC_E_INVALID;
        }
        s->r[i] = ri;
        s->m[i] = p->rho * (4.0 / 3.0) * M_PI * ri * ri * ri;
        s->I[i] = 0.4 * s->m[i] * ri * ri;
        if (ri > rmax) rmax = ri;
    }
    if (n > 0) {
        memcpy(s->x, x, n3 * sizeof(double));
        memcpy(s->v, v, n3 * sizeof(double));
        memcpy(s->w, w, n3 * sizeof(double));
    }
    if (!all_finite(s->x, 3 * n) || !all_finite(s->v, 3 * n) || !all_finite(s->w, 3 * n)) {
        orc_destroy(s);
        return ORC_E_NONFINITE;
    }
    /* the 27-cell search (Eq. 12) finds every contact only if cells are at
     * least one contact distance wide */
    if (p->cell < 2.0 * rmax) {
        orc_destroy(s);
        return ORC_E_INVALID;
    }
    s->ncell = 1;
    for (int a = 0; a < 3; a++) {
        double L = p->hi[a] - p->lo[a];
        if (!(L > 0.0)) {
            orc_destroy(s);
            return ORC_E_INVALID;
        }
        double nf = floor(L / p->cell);
        if (nf < 1.0 || nf > 1.0e6) {
            orc_destroy(s);
            return ORC_E_INVALID;
        }
        s->nc[a] = (int32_t)nf;
        s->sc[a] = (double)s->nc[a] / L;
        s->ncell *= s->nc[a];
    }
    if (s->ncell > 2000000000) {
        orc_destroy(s);
        return ORC_E_INVALID;
    }
    s->alpha = alpha_of(p->e);
    if (nh > 0 && p->law != ORC_SIMPLE) {
        if (!hist_pairs || !hist_dt) {
            orc_destroy(s);
            return ORC_E_INVALID;
        }
        s->H = (orc_hentry *)malloc(sizeof(orc_hentry) * (size_t)nh);
        if (!s->H) {
            orc_destroy(s);
            return ORC_E_NOMEM;
        }
        for (int64_t k = 0; k < nh; k++) {
            int64_t a = hist_pairs[2 * k], b = hist_pairs[2 * k + 1];
            int ok = a >= 0 && a < n && ((b > a && b < n) || (b < 0 && b >= -6 - p->nplates));
            if (!ok) {
                orc_destroy(s);
                return ORC_E_INVALID;
            }
            s->H[k].a = a;
            s->H[k].b = b;
            memcpy(s->H[k].d, hist_dt + 3 * k, 3 * sizeof(double));
        }
        s->nH = nh;
        qsort(s->H, (size_t)nh, sizeof(orc_hentry), cmp_hentry);
        for (int64_t k = 1; k < nh; k++)
            if (cmp_hentry(&s->H[k - 1], &s->H[k]) == 0) {
                orc_destroy(s);
                return ORC_E_INVALID;
            }
    }
    int st;
    if (F0 && T0) {
        memcpy(s->F, F0, n3 * sizeof(double));
        memcpy(s->T, T0, n3 * sizeof(double));
        st = ORC_OK;
        orc_grid g;
        st = grid_build(s, &g); /* domain check */
        if (st == ORC_OK) grid_free(&g);
    } else {
        st = evaluate(s, s->F, s->T, 0, NULL, NULL, NULL, NULL, NULL, NULL);
    }
    if (st != ORC_OK) {
        orc_destroy(s);
        return st;
    }
    *out = s;
    return ORC_OK;
}

/* nsteps of kick-drift-kick velocity Verlet with Steps 2-8 between the
 * kicks; the forces of one step's second kick are the next step's first. */
int orc_step(orc_sys *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return ORC_E_INVALID;
    for (int64_t k = 0; k < nsteps; k++) {
        half_kick(s);
        for (int64_t i = 0; i < 3 * s->n; i++) s->x[i] += s->p.dt * s->v[i];
        int st = evaluate(s, s->F, s->T, 1, NULL, NULL, NULL, NULL, NULL, NULL);
        if (st != ORC_OK) return st;
        half_kick(s);
        s->steps++;
    }
    return ORC_OK;
}

/* Contact force and torque on every particle of the current state with the
 * committed history; nothing is committed.  Gravity is not included. */
int orc_forces(orc_sys *s, double *F, double *T)
{
    if (!s || !F || !T) return ORC_E_INVALID;
    return evaluate(s, F, T, 0, NULL, NULL, NULL, NULL, NULL, NULL);
}

/* The same, plus the error scale of every particle's force and torque:
 * the sums of the magnitudes of the contact forces (and torques) acting on
 * it.  A particle without contacts has scale 0. */
int orc_forces_scale(orc_sys *s, double *F, double *T, double *Fabs, double *Tabs)
{
    if (!s || !F || !T) return ORC_E_INVALID;
    return evaluate(s, F, T, 0, NULL, NULL, NULL, NULL, Fabs, Tabs);
}

int orc_read_state(const orc_sys *s, double *x, double *v, double *w, double *F, double *T)
{
    if (!s) return ORC_E_INVALID;
    size_t b = sizeof(double) * 3 * (size_t)s->n;
    if (x) memcpy(x, s->x, b);
    if (v) memcpy(v, s->v, b);
    if (w) memcpy(w, s->w, b);
    if (F) memcpy(F, s->F, b);
    if (T) memcpy(T, s->T, b);
    return ORC_OK;
}

/* Committed history, sorted by (a, b). */
int orc_read_contacts(const orc_sys *s, int64_t cap, int64_t *n_out, int64_t *pairs, double *dt)
{
    if (!s || !n_out) return ORC_E_INVALID;
    *n_out = s->nH;
    if (s->nH > cap) return ORC_E_CAPACITY;
    for (int64_t k = 0; k < s->nH; k++) {
        if (pairs) {
            pairs[2 * k] = s->H[k].a;
            pairs[2 * k + 1] = s->H[k].b;
        }
        if (dt) memcpy(dt + 3 * k, s->H[k].d, 3 * sizeof(double));
    }
    return ORC_OK;
}

static int cmp_contact(const void *pa, const void *pb)
{
    const orc_contact *x = (const orc_contact *)pa, *y = (const orc_contact *)pb;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

/* Contacts of the current positions (Steps 5-8 detection), sorted by (a, b). */
int orc_contacts(const orc_sys *s, int64_t cap, int64_t *n_out, int64_t *pairs)
{
    if (!s || !n_out) return ORC_E_INVALID;
    orc_grid g;
    orc_clist L;
    int st = grid_build(s, &g);
    if (st != ORC_OK) return st;
    st = detect(s, &g, &L);
    grid_free(&g);
    if (st != ORC_OK) {
        free(L.c);
        return st;
    }
    if (L.n > 0) qsort(L.c, (size_t)L.n, sizeof(orc_contact), cmp_contact);
    *n_out = L.n;
    if (L.n > cap) {
        free(L.c);
        return ORC_E_CAPACITY;
    }
    for (int64_t k = 0; k < L.n && pairs; k++) {
        pairs[2 * k] = L.c[k].a;
        pairs[2 * k + 1] = L.c[k].b;
    }
    free(L.c);
    return ORC_OK;
}

/* Grid of the current positions: CM (cell of every id), SCCM (id at every
 * sorted slot) and the cell starts (ncell + 1 entries). */
int orc_read_grid(const orc_sys *s, int32_t *cell_of_id, int32_t *id_at_slot, int32_t *cell_start)
{
    if (!s) return ORC_E_INVALID;
    orc_grid g;
    int st = grid_build(s, &g);
    if (st != ORC_OK) return st;
    if (cell_of_id) memcpy(cell_of_id, g.cm, sizeof(int32_t) * (size_t)s->n);
    if (id_at_slot) memcpy(id_at_slot, g.sccm, sizeof(int32_t) * (size_t)s->n);
    if (cell_start) memcpy(cell_start, g.start, sizeof(int32_t) * (size_t)(s->ncell + 1));
    grid_free(&g);
    return ORC_OK;
}

int orc_grid_dims(const orc_sys *s, int32_t dims[3])
{
    if (!s) return ORC_E_INVALID;
    memcpy(dims, s->nc, sizeof(s->nc));
    return ORC_OK;
}

/* FP64 diagnostics with compensated sums:
 *  out[0..2] momentum sum m v      out[3] translational kinetic energy
 *  out[4] rotational kinetic energy  out[5] potential energy -sum m g.(x-lo)
 *  out[6] elastic energy of the contacts of the current positions (normal
 *         spring energy plus 1/2 k_t |delta_t|^2 with the committed history)
 *  out[7] pair contacts  out[8] wall contacts  out[9] largest overlap */
int orc_diagnostics(orc_sys *s, double out[10])
{
    if (!s || !out) return ORC_E_INVALID;
    double sum[6] = {0}, comp[6] = {0};
    for (int64_t i = 0; i < s->n; i++) {
        const double *v = s->v + 3 * i, *w = s->w + 3 * i, *x = s->x + 3 * i;
        double term[6];
        for (int k = 0; k < 3; k++) term[k] = s->m[i] * v[k];
        term[3] = 0.5 * s->m[i] * dot3(v, v);
        term[4] = 0.5 * s->I[i] * dot3(w, w);
        term[5] = 0.0;
        for (int k = 0; k < 3; k++) term[5] -= s->m[i] * s->p.g[k] * (x[k] - s->p.lo[k]);
        for (int k = 0; k < 6; k++) {
            double y = term[k] - comp[k], t = sum[k] + y;
            comp[k] = (t - sum[k]) - y;
            sum[k] = t;
        }
    }
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)(s->n > 0 ? s->n : 1));
    double *T = (double *)malloc(sizeof(double) * 3 * (size_t)(s->n > 0 ? s->n : 1));
    if (!F || !T) {
        free(F);
        free(T);
        return ORC_E_NOMEM;
    }
    double E, dm;
    int64_t np, nw;
    int st = evaluate(s, F, T, 0, &E, &np, &nw, &dm, NULL, NULL);
    free(F);
    free(T);
    if (st != ORC_OK) return st;
    for (int k = 0; k < 6; k++) out[k] = sum[k];
    out[6] = E;
    out[7] = (double)np;
    out[8] = (double)nw;
    out[9] = dm;
    return ORC_OK;
}

int64_t orc_num_cells(const orc_sys *s) { return s ? s->ncell : -1; }

/* Largest speed |v_i| of the current state.  Sec. 5 runs its sample problem
 * until the displacements of all particles are below a set value; here a
 * particle's displacement is read as dt |v_i|, the step it would make at its
 * current velocity, checked between steps. */
int orc_max_speed(const orc_sys *s, double *vmax)
{
    if (!s || !vmax) return ORC_E_INVALID;
    double m = 0.0;
    for (int64_t i = 0; i < s->n; i++) {
        double q = norm3(s->v + 3 * i);
        if (q > m) m = q;
    }
    *vmax = m;
    return ORC_OK;
}

/* Material-pair table (Sec. 3, the (i, j) indices of Eqs. 8-10).  ntypes
 * materials, 1 <= ntypes <= ORC_MAX_TYPES; table holds ntypes x ntypes rows
 * (kn, kt, restitution, mu), row t * ntypes + u for a particle of material t
 * touching one of material u, and must be symmetric (the pair's constants
 * do not depend on which side is looked from); type[i] is particle i's
 * material (input order); walls are of material wall_type.  The law
 * switches to the table, and the forces of the current state are evaluated
 * again with it (with the committed history, which is kept), as if the
 * system had been created with these materials.  ntypes = 0 goes back to the
 * parameters' single material. */
int orc_set_materials(orc_sys *s, int32_t ntypes, const double *table, const int32_t *type, int32_t wall_type)
{
    if (!s || ntypes < 0 || ntypes > ORC_MAX_TYPES) return ORC_E_INVALID;
    int32_t *ty = NULL;
    orc_pairk *mat = NULL;
    if (ntypes > 0) {
        if (!table || (s->n > 0 && !type) || wall_type < 0 || wall_type >= ntypes) return ORC_E_INVALID;
        for (int32_t t = 0; t < ntypes; t++)
            for (int32_t u = 0; u < ntypes; u++) {
                const double *q = table + 4 * ((int64_t)t * ntypes + u), *qt = table + 4 * ((int64_t)u * ntypes + t);
                if (!(q[0] > 0.0) || !(q[1] >= 0.0) || !(q[2] > 0.0 && q[2] <= 1.0) || !(q[3] >= 0.0) ||
                    !isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[3]))
                    return ORC_E_INVALID;
                for (int c = 0; c < 4; c++)
                    if (q[c] != qt[c]) return ORC_E_INVALID;
            }
        for (int64_t i = 0; i < s->n; i++)
            if (type[i] < 0 || type[i] >= ntypes) return ORC_E_INVALID;
        ty = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s->n > 0 ? s->n : 1));
        mat = (orc_pairk *)malloc(sizeof(orc_pairk) * (size_t)ntypes * (size_t)ntypes);
        if (!ty || !mat) {
            free(ty);
            free(mat);
            return ORC_E_NOMEM;
        }
        if (s->n > 0) memcpy(ty, type, sizeof(int32_t) * (size_t)s->n);
        for (int64_t q = 0; q < (int64_t)ntypes * ntypes; q++) {
            mat[q].kn = table[4 * q];
            mat[q].kt = table[4 * q + 1];
            mat[q].alpha = alpha_of(table[4 * q + 2]);
            mat[q].mu = table[4 * q + 3];
        }
    }
    free(s->type);
    free(s->mat);
    s->type = ty;
    s->mat = mat;
    s->ntypes = ntypes;
    s->wall_type = ntypes > 0 ? wall_type : 0;
    return evaluate(s, s->F, s->T, 0, NULL, NULL, NULL, NULL, NULL, NULL);
}
