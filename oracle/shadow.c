/*
 * Oracle shadow predicate and accumulation -- TEST INFRASTRUCTURE ONLY.
 *
 * Definitions followed:
 *   gross shadow = time a point spends in shadow over the interval
 *   (Sec. 3.1); with discrete instants it is the count of shadowed instants
 *   scaled by the step (Sec. 4 step 2, Sec. 5), here reported both as the
 *   integer count and as minutes with each instant weighted by its share of
 *   the interval.
 *   The sun is a directional light (Sec. 3.2).  Between two knot instants
 *   the path model is the great circle at constant angular rate, the motion
 *   under which Theorem 1 (Sec. 4) holds.
 *   Several occluders along one ray: every one of them is a shadow source
 *   (Sec. 5, "source levels"); here all of them are taken, no level cap.
 *
 * Brute force: every building is tested for every ray.  FP64 throughout.
 * Nothing here is shared with, or derived from, the HIP library.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct {
    int n_b;
    const int32_t *off;
    double *xy;    /* [2V] */
    double *H;     /* [n_b] */
    double *box;   /* [4 n_b]: xmin, ymin, xmax, ymax */
} scene64;

static void scene64_init(scene64 *S, const orc_scene *s)
{
    S->n_b = s->n_b;
    S->off = s->vert_off;
    int V = s->n_b ? s->vert_off[s->n_b] : 0;
    S->xy = (double *)malloc(sizeof(double) * (2 * (size_t)V + 1));
    S->H = (double *)malloc(sizeof(double) * ((size_t)s->n_b + 1));
    S->box = (double *)malloc(sizeof(double) * (4 * (size_t)s->n_b + 1));
    for (int i = 0; i < 2 * V; ++i) S->xy[i] = s->xy[i];
    for (int b = 0; b < s->n_b; ++b) {
        S->H[b] = s->height[b];
        double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
        for (int v = s->vert_off[b]; v < s->vert_off[b + 1]; ++v) {
            x0 = fmin(x0, S->xy[2 * v]);
            x1 = fmax(x1, S->xy[2 * v]);
            y0 = fmin(y0, S->xy[2 * v + 1]);
            y1 = fmax(y1, S->xy[2 * v + 1]);
        }
        S->box[4 * b] = x0; S->box[4 * b + 1] = y0;
        S->box[4 * b + 2] = x1; S->box[4 * b + 3] = y1;
    }
}

static void scene64_free(scene64 *S)
{
    free(S->xy);
    free(S->H);
    free(S->box);
}

/* Does the ray p + s d, s > 0, meet the closed axis-aligned box
 * [x0,x1] x [y0,y1] x [0,H]?  A necessary condition for meeting the prism
 * inside it. */
static int ray_meets_box(const double *p, const double *d, const double *bx, double H)
{
    double lo = 0.0, hi = INFINITY;
    double blo[3] = {bx[0], bx[1], 0.0}, bhi[3] = {bx[2], bx[3], H};
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (p[a] < blo[a] || p[a] > bhi[a]) return 0;
        } else {
            double t0 = (blo[a] - p[a]) / d[a], t1 = (bhi[a] - p[a]) / d[a];
            if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
            if (t0 > lo) lo = t0;
            if (t1 < hi) hi = t1;
            if (lo > hi) return 0;
        }
    }
    return 1;
}

/* Ray against the closed convex prism b: clip the ray's horizontal
 * projection by every edge half-plane of the footprint (Cyrus-Beck) to get
 * the parameter range [s_in, s_out] over the footprint; the ray rises, so
 * it is lowest where it enters (or at its origin): it meets the prism iff
 * that range is non-empty for s >= 0 and the height there is <= H. */
static int hit_prism(const scene64 *S, int b, const double *p, const double *d)
{
    if (!ray_meets_box(p, d, S->box + 4 * b, S->H[b])) return 0;
    double s_in = -INFINITY, s_out = INFINITY;
    int o = S->off[b], m = S->off[b + 1] - o;
    for (int i = 0; i < m; ++i) {
        const double *a = S->xy + 2 * (o + i), *c = S->xy + 2 * (o + (i + 1) % m);
        double nx = c[1] - a[1], ny = -(c[0] - a[0]);     /* outward normal (CCW) */
        double num = nx * (a[0] - p[0]) + ny * (a[1] - p[1]);
        double den = nx * d[0] + ny * d[1];
        if (den > 0.0) {
            double s = num / den;
            if (s < s_out) s_out = s;
        } else if (den < 0.0) {
            double s = num / den;
            if (s > s_in) s_in = s;
        } else if (num < 0.0) {
            return 0;                                      /* parallel, outside */
        }
    }
    double s0 = s_in > 0.0 ? s_in : 0.0;
    if (s_out < s0) return 0;
    return p[2] + s0 * d[2] <= S->H[b];
}

static int shadow64(const scene64 *S, const double *p, const double *nrm, int owner,
                    const double *d)
{
    if (owner >= 0 && nrm[0] * d[0] + nrm[1] * d[1] <= 0.0) return 1;  /* back-facing wall */
    for (int b = 0; b < S->n_b; ++b)
        if (b != owner && hit_prism(S, b, p, d)) return 1;
    return 0;
}

int orc_shadow(const orc_scene *s, double px, double py, double pz,
               double nx, double ny, int owner, const double *d)
{
    scene64 S;
    scene64_init(&S, s);
    double p[3] = {px, py, pz}, n[2] = {nx, ny};
    int r = shadow64(&S, p, n, owner, d);
    scene64_free(&S);
    return r;
}

/* ---- independent check: Moller-Trumbore against the triangulated prism ---- */
static int ray_tri(const double *o, const double *d, const double *v0, const double *v1,
                   const double *v2)
{
    double e1[3], e2[3], pv[3], tv[3], qv[3];
    for (int i = 0; i < 3; ++i) { e1[i] = v1[i] - v0[i]; e2[i] = v2[i] - v0[i]; }
    pv[0] = d[1] * e2[2] - d[2] * e2[1];
    pv[1] = d[2] * e2[0] - d[0] * e2[2];
    pv[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (fabs(det) < 1e-300) return 0;
    double inv = 1.0 / det;
    for (int i = 0; i < 3; ++i) tv[i] = o[i] - v0[i];
    double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    qv[0] = tv[1] * e1[2] - tv[2] * e1[1];
    qv[1] = tv[2] * e1[0] - tv[0] * e1[2];
    qv[2] = tv[0] * e1[1] - tv[1] * e1[0];
    double v = (d[0] * qv[0] + d[1] * qv[1] + d[2] * qv[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    return t > 0.0;
}

int orc_shadow_mt(const orc_scene *s, double px, double py, double pz,
                  double nx, double ny, int owner, const double *d)
{
    double p[3] = {px, py, pz};
    if (owner >= 0 && nx * d[0] + ny * d[1] <= 0.0) return 1;
    for (int b = 0; b < s->n_b; ++b) {
        if (b == owner) continue;
        int o = s->vert_off[b], m = s->vert_off[b + 1] - o;
        double H = s->height[b];
        for (int i = 0; i < m; ++i) {
            int j = (i + 1) % m;
            double a0[3] = {s->xy[2 * (o + i)], s->xy[2 * (o + i) + 1], 0.0};
            double b0[3] = {s->xy[2 * (o + j)], s->xy[2 * (o + j) + 1], 0.0};
            double a1[3] = {a0[0], a0[1], H}, b1[3] = {b0[0], b0[1], H};
            if (ray_tri(p, d, a0, b0, b1) || ray_tri(p, d, a0, b1, a1)) return 1;   /* wall */
            if (i >= 1 && i + 1 < m) {
                double r0[3] = {s->xy[2 * o], s->xy[2 * o + 1], H};
                double g0[3] = {r0[0], r0[1], 0.0};
                if (ray_tri(p, d, r0, a1, b1) || ray_tri(p, d, g0, a0, b0)) return 1; /* roof, base */
            }
        }
    }
    return 0;
}

/* ---- thread pool over points ---- */
typedef struct {
    void (*fn)(void *ctx, int64_t i);
    void *ctx;
    int64_t n;
    int64_t next;
    pthread_mutex_t mu;
} pool_t;

static void *pool_worker(void *arg)
{
    pool_t *P = (pool_t *)arg;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int64_t i = P->next++;
        pthread_mutex_unlock(&P->mu);
        if (i >= P->n) break;
        P->fn(P->ctx, i);
    }
    return NULL;
}

static void parallel_for(int64_t n, int threads, void (*fn)(void *, int64_t), void *ctx)
{
    pool_t P = {fn, ctx, n, 0, PTHREAD_MUTEX_INITIALIZER};
    if (threads <= 1) {
        for (int64_t i = 0; i < n; ++i) fn(ctx, i);
        return;
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    for (int t = 0; t < threads; ++t) pthread_create(&th[t], NULL, pool_worker, &P);
    for (int t = 0; t < threads; ++t) pthread_join(th[t], NULL);
    free(th);
}

/* ---- sampled form ---- */
typedef struct {
    const scene64 *S;
    const orc_points *P;
    int K;
    const double *dirs, *w;
    const int32_t *bin;
    int n_bins;
    int32_t *counts;
    double *minutes;
    uint32_t *bits;
    uint8_t *amb;
} sampled_ctx;

/* Directions 1.1e-5 rad from d, displaced toward 8 evenly spaced azimuths
 * about d: a ray whose predicate differs from any of them passes within
 * 1e-5 rad of a silhouette (or of the wall's own plane). */
static int ambiguous(const scene64 *S, const double *p, const double *nrm, int owner,
                     const double *d, int s0)
{
    const double eps = 1.1e-5;
    double a[3], b[3];
    /* orthonormal a, b perpendicular to d */
    if (fabs(d[2]) < 0.9) { a[0] = -d[1]; a[1] = d[0]; a[2] = 0.0; }
    else { a[0] = 0.0; a[1] = -d[2]; a[2] = d[1]; }
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int i = 0; i < 3; ++i) a[i] /= na;
    b[0] = d[1] * a[2] - d[2] * a[1];
    b[1] = d[2] * a[0] - d[0] * a[2];
    b[2] = d[0] * a[1] - d[1] * a[0];
    for (int j = 0; j < 8; ++j) {
        double c = cos(j * M_PI / 4.0), s = sin(j * M_PI / 4.0), q[3];
        for (int i = 0; i < 3; ++i) q[i] = d[i] * cos(eps) + (c * a[i] + s * b[i]) * sin(eps);
        if (shadow64(S, p, nrm, owner, q) != s0) return 1;
    }
    return 0;
}

static void sampled_point(void *vctx, int64_t i)
{
    sampled_ctx *C = (sampled_ctx *)vctx;
    const orc_points *P = C->P;
    int64_t n = P->n;
    double p[3] = {P->x[i], P->y[i], P->z[i]};
    double nrm[2] = {P->nx ? P->nx[i] : 0.0, P->ny ? P->ny[i] : 0.0};
    int owner = P->owner ? P->owner[i] : -1;
    int words = (C->K + 31) / 32;
    for (int k = 0; k < C->K; ++k) {
        const double *d = C->dirs + 3 * k;
        int s = shadow64(C->S, p, nrm, owner, d);
        int bin = C->bin ? C->bin[k] : 0;
        if (C->counts) C->counts[(int64_t)bin * n + i] += s;
        if (C->minutes) C->minutes[(int64_t)bin * n + i] += s * C->w[k];
        if (C->bits && s) C->bits[i * words + k / 32] |= 1u << (k % 32);
        if (C->amb) C->amb[i * C->K + k] = (uint8_t)ambiguous(C->S, p, nrm, owner, d, s);
    }
}

void orc_sampled(const orc_scene *s, const orc_points *p, int K, const double *dirs,
                 const double *w, const int32_t *sample_bin, int n_bins,
                 int32_t *counts, double *minutes, uint32_t *bits, uint8_t *amb,
                 int threads)
{
    scene64 S;
    scene64_init(&S, s);
    if (counts) memset(counts, 0, sizeof(int32_t) * (size_t)n_bins * p->n);
    if (minutes) memset(minutes, 0, sizeof(double) * (size_t)n_bins * p->n);
    if (bits) memset(bits, 0, sizeof(uint32_t) * (size_t)p->n * ((K + 31) / 32));
    sampled_ctx C = {&S, p, K, dirs, w, sample_bin, n_bins, counts, minutes, bits, amb};
    parallel_for(p->n, threads, sampled_point, &C);
    scene64_free(&S);
}

/* ---- continuous duration along the piecewise great-circle path ---- */
void orc_slerp(const double *a, const double *b, double f, double *out)
{
    double c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double s = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double th = atan2(s, c);
    if (th < 1e-15) {
        for (int i = 0; i < 3; ++i) out[i] = a[i];
        return;
    }
    double wa = sin((1.0 - f) * th) / sin(th), wb = sin(f * th) / sin(th);
    for (int i = 0; i < 3; ++i) out[i] = wa * a[i] + wb * b[i];
}

typedef struct { double lo, hi; } ival;
typedef struct { ival *v; int n, cap; } ivec;

static void ivec_push(ivec *a, double lo, double hi)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 64;
        a->v = (ival *)realloc(a->v, sizeof(ival) * a->cap);
    }
    a->v[a->n].lo = lo;
    a->v[a->n].hi = hi;
    a->n++;
}

static int ival_cmp(const void *x, const void *y)
{
    double a = ((const ival *)x)->lo, b = ((const ival *)y)->lo;
    return (a > b) - (a < b);
}

/* sort + merge in place; returns the number of disjoint intervals */
static int ivec_union(ivec *a)
{
    qsort(a->v, a->n, sizeof(ival), ival_cmp);
    int m = 0;
    for (int i = 0; i < a->n;) {
        double lo = a->v[i].lo, hi = a->v[i].hi;
        int j = i + 1;
        while (j < a->n && a->v[j].lo <= hi) {
            if (a->v[j].hi > hi) hi = a->v[j].hi;
            ++j;
        }
        a->v[m].lo = lo;
        a->v[m].hi = hi;
        ++m;
        i = j;
    }
    a->n = m;
    return m;
}

typedef struct {
    const scene64 *S;
    const orc_points *P;
    int n_seg;
    const double *seg_t, *seg_dir;
    const int32_t *seg_day;
    int n_days;
    const int32_t *day_bin;
    double grid;
    const double *sample_t;
    const int32_t *sample_day;
    int n_samples;
    double *minutes;
    int32_t *counts;
    double *longest;
    /* gradient mode */
    const double *dl;
    double *grad;
    pthread_mutex_t *grad_mu;
} cont_ctx;

/* one occluder's predicate: b >= 0 a prism, b == -1 the point's own wall
 * facing away from the sun */
static int occl(const scene64 *S, int b, const double *p, const double *nrm, const double *d)
{
    if (b < 0) return nrm[0] * d[0] + nrm[1] * d[1] <= 0.0;
    return hit_prism(S, b, p, d);
}

/* Every ray of the segment lies in the plane through p spanned by the two
 * knot directions: a prism whose bounding box lies strictly on one side of
 * that plane cannot be met during the segment. */
static int box_off_plane(const scene64 *S, int b, const double *p, const double *N)
{
    const double *bx = S->box + 4 * b;
    int pos = 0, neg = 0;
    for (int c = 0; c < 8; ++c) {
        double q[3] = {(c & 1) ? bx[2] : bx[0], (c & 2) ? bx[3] : bx[1], (c & 4) ? S->H[b] : 0.0};
        double f = N[0] * (q[0] - p[0]) + N[1] * (q[1] - p[1]) + N[2] * (q[2] - p[2]);
        if (f > 0) pos = 1;
        else if (f < 0) neg = 1;
        else return 0;
    }
    return !(pos && neg);
}

static void seg_dir_at(const double *da, const double *db, double ta, double tb, double t,
                       double *d)
{
    orc_slerp(da, db, (t - ta) / (tb - ta), d);
}

/* A stretch of the sun's path as a function of time: either the great
 * circle between two knot directions at a constant angular rate (the path
 * model of the accrual form), or the sun's actual direction from the solar
 * position equations (the definition of Sec. 3.1 / 3.2).  For the actual
 * path a table of directions at T0 + i * tab_step saves recomputing the
 * solar position on the scan grid; any other time is computed. */
typedef struct {
    int kind;                    /* 0: great circle between knots; 1: actual path */
    const double *da, *db;       /* kind 0 */
    double ta, tb;               /* kind 0 */
    int year, month, day;        /* kind 1 */
    double tz_h, lat, lon;       /* kind 1 */
    const double *tab;           /* kind 1: [3 * n_tab] directions, or NULL */
    double tab_t0, tab_step;
    int64_t n_tab;
} sunarc;

static void arc_dir(const sunarc *A, double t, double *d)
{
    if (A->kind == 0) {
        seg_dir_at(A->da, A->db, A->ta, A->tb, t, d);
        return;
    }
    if (A->tab) {
        double f = (t - A->tab_t0) / A->tab_step;
        double r = floor(f + 0.5);
        if (fabs(f - r) < 1e-7 && r >= 0 && r < (double)A->n_tab) {
            const double *q = A->tab + 3 * (int64_t)r;
            d[0] = q[0]; d[1] = q[1]; d[2] = q[2];
            return;
        }
    }
    double sol[9];
    orc_solar(A->year, A->month, A->day, t, A->tz_h, A->lat, A->lon, sol);
    d[0] = sol[0]; d[1] = sol[1]; d[2] = sol[2];
}

/* Does the ray from p along d meet the box of prism b grown by delta on
 * every side? */
static int ray_meets_grown_box(const scene64 *S, int b, const double *p, const double *d, double delta)
{
    const double *bx = S->box + 4 * b;
    double g[4] = {bx[0] - delta, bx[1] - delta, bx[2] + delta, bx[3] + delta};
    double lo = 0.0, hi = INFINITY;
    double blo[3] = {g[0], g[1], -delta}, bhi[3] = {g[2], g[3], S->H[b] + delta};
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (p[a] < blo[a] || p[a] > bhi[a]) return 0;
        } else {
            double t0 = (blo[a] - p[a]) / d[a], t1 = (bhi[a] - p[a]) / d[a];
            if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
            if (t0 > lo) lo = t0;
            if (t1 < hi) hi = t1;
            if (lo > hi) return 0;
        }
    }
    return 1;
}

/* Scan [t0, t1] on G+1 evenly spaced instants for switches of one
 * occluder's predicate along the path A, locating each by bisection to
 * 1e-9 minutes.  `state` carries the predicate value and the start of an
 * open shadowed run across calls; closed runs are appended to out. */
static void scan_cell(const scene64 *S, int b, const double *p, const double *nrm, const sunarc *A,
                      double t0, double t1, int G, int *state, double *open_t, ivec *out)
{
    double d[3], t_prev = t0;
    for (int g = 1; g <= G; ++g) {
        double t = (g == G) ? t1 : t0 + (t1 - t0) * g / G;
        arc_dir(A, t, d);
        int v = occl(S, b, p, nrm, d);
        if (v != *state) {
            double lo = t_prev, hi = t;
            for (int it = 0; it < 80 && hi - lo > 1e-9; ++it) {
                double mid = 0.5 * (lo + hi);
                arc_dir(A, mid, d);
                if (occl(S, b, p, nrm, d) == *state) lo = mid;
                else hi = mid;
            }
            double sw = 0.5 * (lo + hi);
            if (v) *open_t = sw;
            else ivec_push(out, *open_t, sw);
            *state = v;
        }
        t_prev = t;
    }
}

/* Times in [ta, tb] at which one occluder shadows p along the path A: its
 * predicate sampled on a grid of spacing <= grid, each change located by
 * bisection.  A short shadowed run can hide between two unshadowed grid
 * instants; it can only do so if the rays at those instants pass within
 * (distance x the angle turned over the cell) of the prism, so such cells
 * are rescanned 64 times finer.  (Within one great-circle segment a convex
 * prism shadows p over a single run, so no unshadowed gap can hide between
 * two shadowed instants; along the actual path, cut into minutes-long
 * pieces, a gap could only hide where the path runs within its tiny
 * curvature of a silhouette for less than one grid cell.)  Appends the
 * shadowed intervals to out. */
static void occluder_intervals_arc(const scene64 *S, int b, const double *p, const double *nrm,
                                   const sunarc *A, double ta, double tb, double grid, ivec *out)
{
    int G = (int)ceil((tb - ta) / grid - 1e-12);
    if (G < 1) G = 1;
    double d[3], e[3], open_t = ta;
    arc_dir(A, ta, d);
    arc_dir(A, tb, e);
    double c = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
    double dphi = acos(c > 1.0 ? 1.0 : c) / G;         /* angle turned per cell */
    if (A->kind == 1) dphi = 1.01 * dphi + 1e-9;       /* the actual path turns at a near-constant rate */
    double R = 0.0;                                     /* farthest box corner from p */
    if (b >= 0) {
        const double *bx = S->box + 4 * b;
        for (int k = 0; k < 8; ++k) {
            double q[3] = {(k & 1) ? bx[2] : bx[0], (k & 2) ? bx[3] : bx[1], (k & 4) ? S->H[b] : 0.0};
            double r = sqrt((q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]) +
                            (q[2] - p[2]) * (q[2] - p[2]));
            if (r > R) R = r;
        }
    }
    double delta = 2.0 * R * dphi + 1e-6;
    int state = occl(S, b, p, nrm, d);
    int near_prev = b >= 0 && ray_meets_grown_box(S, b, p, d, delta);
    double t_prev = ta;
    for (int g = 1; g <= G; ++g) {
        double t = (g == G) ? tb : ta + (tb - ta) * g / G;
        arc_dir(A, t, d);
        int v = occl(S, b, p, nrm, d);
        int near = b >= 0 && ray_meets_grown_box(S, b, p, d, delta);
        if (state == 0 && v == 0 && (near || near_prev))
            scan_cell(S, b, p, nrm, A, t_prev, t, 64, &state, &open_t, out);
        else
            scan_cell(S, b, p, nrm, A, t_prev, t, 1, &state, &open_t, out);
        near_prev = near;
        t_prev = t;
    }
    if (state) ivec_push(out, open_t, tb);
}

/* The same along the great-circle segment from da (at ta) to db (at tb). */
static void occluder_intervals(const scene64 *S, int b, const double *p, const double *nrm,
                               double ta, double tb, const double *da, const double *db,
                               double grid, ivec *out)
{
    sunarc A;
    memset(&A, 0, sizeof(A));
    A.kind = 0; A.da = da; A.db = db; A.ta = ta; A.tb = tb;
    occluder_intervals_arc(S, b, p, nrm, &A, ta, tb, grid, out);
}

static void seg_plane(const double *da, const double *db, double *N)
{
    N[0] = da[1] * db[2] - da[2] * db[1];
    N[1] = da[2] * db[0] - da[0] * db[2];
    N[2] = da[0] * db[1] - da[1] * db[0];
    double s = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    if (s > 0) for (int i = 0; i < 3; ++i) N[i] /= s;
}

/* Does prism b's box lie wholly behind the segment: every direction of a
 * great-circle arc shorter than a half circle makes an acute angle with
 * the arc's mean direction m, so a point the rays meet has (q - p).m > 0;
 * a box with every corner at (q - p).m <= 0 cannot be met. */
static int box_behind(const scene64 *S, int b, const double *p, const double *m)
{
    const double *bx = S->box + 4 * b;
    for (int k = 0; k < 8; ++k) {
        double q[3] = {((k & 1) ? bx[2] : bx[0]) - p[0], ((k & 2) ? bx[3] : bx[1]) - p[1],
                       ((k & 4) ? S->H[b] : 0.0) - p[2]};
        if (m[0] * q[0] + m[1] * q[1] + m[2] * q[2] > 0.0) return 0;
    }
    return 1;
}

/* Does prism b's box lie wholly below the segment's rays: a ray that rises
 * at least tan_min metres per horizontal metre is, at the box's nearest
 * horizontal distance d from p, already above p_z + d tan_min; a box whose
 * top is lower cannot be met.  (Along a great-circle arc above the horizon
 * and shorter than a half circle the elevation is smallest at an end.) */
static int box_below(const scene64 *S, int b, const double *p, double tan_min)
{
    const double *bx = S->box + 4 * b;
    const double dx = p[0] < bx[0] ? bx[0] - p[0] : (p[0] > bx[2] ? p[0] - bx[2] : 0.0);
    const double dy = p[1] < bx[1] ? bx[1] - p[1] : (p[1] > bx[3] ? p[1] - bx[3] : 0.0);
    return S->H[b] - p[2] < sqrt(dx * dx + dy * dy) * tan_min;
}

/* Shadowed intervals of one point over one segment, all occluders, not
 * merged.  Once one occluder shadows the whole segment the union over it is
 * the segment whatever the others add, so they are skipped. */
static void segment_intervals(const scene64 *S, const double *p, const double *nrm, int owner,
                              double ta, double tb, const double *da, const double *db,
                              double grid, ivec *out)
{
    if (!(tb > ta)) return;
    double N[3], m[3];
    seg_plane(da, db, N);
    for (int i = 0; i < 3; ++i) m[i] = da[i] + db[i];
    const int arc_ok = da[0] * db[0] + da[1] * db[1] + da[2] * db[2] > -0.5;   /* shorter than 120 degrees */
    const double ta_ = da[2] / sqrt(da[0] * da[0] + da[1] * da[1] + 1e-300);
    const double tb_ = db[2] / sqrt(db[0] * db[0] + db[1] * db[1] + 1e-300);
    const double tan_min = arc_ok && da[2] > 0.0 && db[2] > 0.0 ? (ta_ < tb_ ? ta_ : tb_) : 0.0;
    int first = out->n;
    for (int b = (owner >= 0 ? -1 : 0); b < S->n_b; ++b) {
        if (b >= 0 && (b == owner || box_off_plane(S, b, p, N) ||
                       (arc_ok && (box_behind(S, b, p, m) || box_below(S, b, p, tan_min)))))
            continue;
        occluder_intervals(S, b, p, nrm, ta, tb, da, db, grid, out);
        for (; first < out->n; ++first)
            if (out->v[first].lo <= ta && out->v[first].hi >= tb) return;
    }
}

static void continuous_point(void *vctx, int64_t i)
{
    cont_ctx *C = (cont_ctx *)vctx;
    const orc_points *P = C->P;
    int64_t n = P->n;
    double p[3] = {P->x[i], P->y[i], P->z[i]};
    double nrm[2] = {P->nx ? P->nx[i] : 0.0, P->ny ? P->ny[i] : 0.0};
    int owner = P->owner ? P->owner[i] : -1;
    ivec day = {0, 0, 0};
    int j = 0, k = 0;
    for (int dd = 0; dd < C->n_days; ++dd) {
        day.n = 0;
        for (; j < C->n_seg && C->seg_day[j] == dd; ++j)
            segment_intervals(C->S, p, nrm, owner, C->seg_t[2 * j], C->seg_t[2 * j + 1],
                              C->seg_dir + 6 * j, C->seg_dir + 6 * j + 3, C->grid, &day);
        int m = ivec_union(&day);
        double meas = 0.0, run = 0.0;
        for (int a = 0; a < m; ++a) {
            meas += day.v[a].hi - day.v[a].lo;
            /* continuous shadow (Sec. 3.1): the longest member of the day's
             * union; runs that meet at a knot were merged by ivec_union */
            if (day.v[a].hi - day.v[a].lo > run) run = day.v[a].hi - day.v[a].lo;
        }
        int cnt = 0;
        for (; k < C->n_samples && C->sample_day[k] == dd; ++k) {
            double t = C->sample_t[k];
            for (int a = 0; a < m; ++a)
                if (t >= day.v[a].lo && t <= day.v[a].hi) { ++cnt; break; }
        }
        int bin = C->day_bin ? C->day_bin[dd] : dd;
        if (C->minutes) C->minutes[(int64_t)bin * n + i] += meas;
        if (C->counts) C->counts[(int64_t)bin * n + i] += cnt;
        /* over several days: the maximum over the bin's days (Sec. 3.1) */
        if (C->longest && run > C->longest[(int64_t)bin * n + i]) C->longest[(int64_t)bin * n + i] = run;
    }
    free(day.v);
}

void orc_continuous(const orc_scene *s, const orc_points *p, int n_seg,
                    const double *seg_t, const double *seg_dir, const int32_t *seg_day,
                    int n_days, const int32_t *day_bin, int n_bins, double grid_min,
                    const double *sample_t, const int32_t *sample_day, int n_samples,
                    double *minutes, int32_t *counts, double *longest, int threads)
{
    scene64 S;
    scene64_init(&S, s);
    if (minutes) memset(minutes, 0, sizeof(double) * (size_t)n_bins * p->n);
    if (counts) memset(counts, 0, sizeof(int32_t) * (size_t)n_bins * p->n);
    if (longest) memset(longest, 0, sizeof(double) * (size_t)n_bins * p->n);
    cont_ctx C;
    memset(&C, 0, sizeof(C));
    C.S = &S; C.P = p; C.n_seg = n_seg; C.seg_t = seg_t; C.seg_dir = seg_dir;
    C.seg_day = seg_day; C.n_days = n_days; C.day_bin = day_bin; C.grid = grid_min;
    C.sample_t = sample_t; C.sample_day = sample_day; C.n_samples = n_samples;
    C.minutes = minutes; C.counts = counts; C.longest = longest;
    parallel_for(p->n, threads, continuous_point, &C);
    scene64_free(&S);
}

/* ---- continuous duration along the actual sun path (Sec. 3.1, 3.2) ----
 *
 * D(p) = measure of { t in [T0, T1] : p is in shadow for the sun's actual
 * direction at t }, per day, summed into the day's bin.  The same
 * per-occluder scan and bisection as above, with every direction taken
 * from the solar position equations instead of an interpolated path.  To
 * keep the brute force affordable the day is cut into hour-long and then
 * `piece`-long stretches; a prism is skipped for a stretch only when no
 * ray within the stretch's angular reach of its chord plane can meet the
 * prism's box (box_off_slab). */

/* Can a ray from p, whose direction lies within an angle eps of the plane
 * through p with unit normal N, meet prism b's box?  A point q such a ray
 * meets satisfies |N.(q-p)| <= |q-p| sin(eps).  The function
 * +-N.(q-p) - |q-p| sin(eps) is concave in q, so if it is positive at every
 * corner of the box it is positive on the whole box: no such ray meets it.
 * Returns 1 when the box is out of reach (the prism can be skipped). */
static int box_off_slab(const scene64 *S, int b, const double *p, const double *N, double sin_eps,
                        const double *m)
{
    const double *bx = S->box + 4 * b;
    /* behind the stretch: every direction of the stretch makes an acute
     * angle with m, so a point the rays meet has (q - p).m > 0; a box with
     * every corner at (q - p).m <= 0 is out of reach */
    int behind = 1;
    for (int k = 0; k < 8 && behind; ++k) {
        double q[3] = {((k & 1) ? bx[2] : bx[0]) - p[0], ((k & 2) ? bx[3] : bx[1]) - p[1],
                       ((k & 4) ? S->H[b] : 0.0) - p[2]};
        if (m[0] * q[0] + m[1] * q[1] + m[2] * q[2] > 0.0) behind = 0;
    }
    if (behind) return 1;
    /* bounding sphere first (cheap, weaker) */
    double c[3] = {0.5 * (bx[0] + bx[2]) - p[0], 0.5 * (bx[1] + bx[3]) - p[1], 0.5 * S->H[b] - p[2]};
    double r = 0.5 * sqrt((bx[2] - bx[0]) * (bx[2] - bx[0]) + (bx[3] - bx[1]) * (bx[3] - bx[1]) +
                          S->H[b] * S->H[b]);
    double dc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double f = N[0] * c[0] + N[1] * c[1] + N[2] * c[2];
    if (fabs(f) - r - (dc + r) * sin_eps > 0.0) return 1;
    int pos = 1, neg = 1;
    for (int k = 0; k < 8 && (pos || neg); ++k) {
        double q[3] = {((k & 1) ? bx[2] : bx[0]) - p[0], ((k & 2) ? bx[3] : bx[1]) - p[1],
                       ((k & 4) ? S->H[b] : 0.0) - p[2]};
        double g = N[0] * q[0] + N[1] * q[1] + N[2] * q[2];
        double m = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) * sin_eps;
        if (!(g > m)) pos = 0;
        if (!(-g > m)) neg = 0;
    }
    return pos || neg;
}

/* Chord plane of the path over [ta, tb] (unit normal N) and a bound on how
 * far (radians) the path strays from it: the sun's daily circle deviates
 * from the great circle through two of its points by at most about
 * beta^2 sin(2 rho) / 16 (beta the hour angle between them, rho the
 * circle's angular radius), so beta^2 / 8 bounds it twice over; the largest
 * deviation seen at 15 interior instants, doubled, guards the rest.  m:
 * the unit mean of the two end directions; an arc of the daily circle
 * shorter than a half circle stays within the angle between its ends of
 * that mean, so every direction of a stretch of less than 120 degrees
 * makes an acute angle with m.  Returns 0 when the chord is too short to
 * define a plane or too long for m. */
static int chord_plane(const sunarc *A, double ta, double tb, double *N, double *sin_eps, double *m)
{
    double da[3], db[3], d[3];
    arc_dir(A, ta, da);
    arc_dir(A, tb, db);
    seg_plane(da, db, N);
    if (!(N[0] * N[0] + N[1] * N[1] + N[2] * N[2] > 0.5)) return 0;
    if (!(da[0] * db[0] + da[1] * db[1] + da[2] * db[2] > -0.5)) return 0;
    for (int i = 0; i < 3; ++i) m[i] = da[i] + db[i];
    double mm = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    for (int i = 0; i < 3; ++i) m[i] /= mm;
    double dev = 0.0;
    for (int k = 1; k < 16; ++k) {
        arc_dir(A, ta + (tb - ta) * k / 16.0, d);
        double v = fabs(N[0] * d[0] + N[1] * d[1] + N[2] * d[2]);
        if (v > dev) dev = v;
    }
    double beta = (tb - ta) * (2.0 * M_PI / 1440.0) * 1.01;
    double eps = fmax(2.0 * dev, beta * beta / 8.0) + 1e-9;
    *sin_eps = sin(eps);
    return 1;
}

typedef struct {
    const scene64 *S;
    const orc_points *P;
    int n_days;
    const int32_t *ymd;
    const double *tz_h, *span;
    const int32_t *day_bin;
    double lat, lon, piece, grid, tab_step;
    double *const *tab;
    const int64_t *n_tab;
    double *minutes, *longest;
} true_ctx;

typedef struct {
    const int32_t *ymd;
    const double *tz_h, *span;
    double lat, lon, step;
    double *const *tab;
    const int64_t *n_tab;
    int n_days;
} day_table_ctx;

/* one 64th of one day's direction table */
static void day_table_part(void *vctx, int64_t i)
{
    const day_table_ctx *T = (const day_table_ctx *)vctx;
    int dd = (int)(i / 64), part = (int)(i % 64);
    int64_t m = T->n_tab[dd], k0 = m * part / 64, k1 = m * (part + 1) / 64;
    for (int64_t k = k0; k < k1; ++k) {
        double sol[9];
        orc_solar(T->ymd[3 * dd], T->ymd[3 * dd + 1], T->ymd[3 * dd + 2], T->span[2 * dd] + k * T->step,
                  T->tz_h[dd], T->lat, T->lon, sol);
        T->tab[dd][3 * k] = sol[0]; T->tab[dd][3 * k + 1] = sol[1]; T->tab[dd][3 * k + 2] = sol[2];
    }
}

static void true_point(void *vctx, int64_t i)
{
    const true_ctx *C = (const true_ctx *)vctx;
    const scene64 *S = C->S;
    const orc_points *P = C->P;
    int64_t n = P->n;
    double p[3] = {P->x[i], P->y[i], P->z[i]};
    double nrm[2] = {P->nx ? P->nx[i] : 0.0, P->ny ? P->ny[i] : 0.0};
    int owner = P->owner ? P->owner[i] : -1;
    int *cand = (int *)malloc(sizeof(int) * ((size_t)S->n_b + 1));
    ivec day = {0, 0, 0};
    for (int dd = 0; dd < C->n_days; ++dd) {
        double T0 = C->span[2 * dd], T1 = C->span[2 * dd + 1];
        day.n = 0;
        sunarc A;
        memset(&A, 0, sizeof(A));
        A.kind = 1;
        A.year = C->ymd[3 * dd]; A.month = C->ymd[3 * dd + 1]; A.day = C->ymd[3 * dd + 2];
        A.tz_h = C->tz_h[dd]; A.lat = C->lat; A.lon = C->lon;
        A.tab = C->tab[dd]; A.tab_t0 = T0; A.tab_step = C->tab_step; A.n_tab = C->n_tab[dd];
        for (double ha = T0; ha < T1; ha += 60.0) {
            double hb = fmin(ha + 60.0, T1), N[3], se, mid[3];
            int nc = 0;
            int plane = chord_plane(&A, ha, hb, N, &se, mid);
            for (int b = 0; b < S->n_b; ++b)
                if (b != owner && !(plane && box_off_slab(S, b, p, N, se, mid))) cand[nc++] = b;
            for (double ta = ha; ta < hb; ta += C->piece) {
                double tb = fmin(ta + C->piece, hb), M[3], sm, mid2[3];
                int plane2 = chord_plane(&A, ta, tb, M, &sm, mid2);
                /* once one occluder shadows the whole stretch the union over it is
                 * the stretch, whatever the others add: they are skipped */
                int first = day.n, covered = 0;
                if (owner >= 0) occluder_intervals_arc(S, -1, p, nrm, &A, ta, tb, C->grid, &day);
                for (int k = 0; k < nc; ++k) {
                    for (; first < day.n && !covered; ++first)
                        covered = day.v[first].lo <= ta && day.v[first].hi >= tb;
                    if (covered) break;
                    if (plane2 && box_off_slab(S, cand[k], p, M, sm, mid2)) continue;
                    occluder_intervals_arc(S, cand[k], p, nrm, &A, ta, tb, C->grid, &day);
                }
            }
        }
        int m = ivec_union(&day);
        double meas = 0.0, run = 0.0;
        for (int a = 0; a < m; ++a) {
            meas += day.v[a].hi - day.v[a].lo;
            if (day.v[a].hi - day.v[a].lo > run) run = day.v[a].hi - day.v[a].lo;
        }
        int bin = C->day_bin ? C->day_bin[dd] : dd;
        if (C->minutes) C->minutes[(int64_t)bin * n + i] += meas;
        if (C->longest && run > C->longest[(int64_t)bin * n + i]) C->longest[(int64_t)bin * n + i] = run;
    }
    free(day.v);
    free(cand);
}

void orc_continuous_true(const orc_scene *s, const orc_points *p, int n_days, const int32_t *ymd,
                         const double *tz_h, const double *span, const int32_t *day_bin, int n_bins,
                         double lat_deg, double lon_deg, double piece_min, double grid_min,
                         double *minutes, double *longest, int threads)
{
    scene64 S;
    scene64_init(&S, s);
    if (minutes) memset(minutes, 0, sizeof(double) * (size_t)n_bins * p->n);
    if (longest) memset(longest, 0, sizeof(double) * (size_t)n_bins * p->n);
    /* the directions at the scan grid's instants and at the 64 sub-instants
     * of its finer rescans, once per day for all points */
    const double tab_step = grid_min / 64.0;
    double **tab = (double **)calloc(n_days + 1, sizeof(double *));
    int64_t *n_tab = (int64_t *)calloc(n_days + 1, sizeof(int64_t));
    for (int dd = 0; dd < n_days; ++dd) {
        double T0 = span[2 * dd], T1 = span[2 * dd + 1];
        int64_t m = T1 > T0 ? (int64_t)ceil((T1 - T0) / tab_step) + 1 : 0;
        n_tab[dd] = m;
        tab[dd] = (double *)malloc(sizeof(double) * (3 * (size_t)m + 1));
    }
    day_table_ctx T = {ymd, tz_h, span, lat_deg, lon_deg, tab_step, tab, n_tab, n_days};
    parallel_for((int64_t)n_days * 64, threads, day_table_part, &T);
    true_ctx C = {&S, p, n_days, ymd, tz_h, span, day_bin, lat_deg, lon_deg, piece_min, grid_min,
                  tab_step, tab, n_tab, minutes, longest};
    parallel_for(p->n, threads, true_point, &C);
    for (int dd = 0; dd < n_days; ++dd) free(tab[dd]);
    free(tab);
    free(n_tab);
    scene64_free(&S);
}

/* ---- gradient of sum_p w(p, day) D_L(p, day) with respect to heights ----
 *
 * D_L is the measure of the union of the occluders' shadowed intervals.
 * A boundary of the union at time t* is an end of one occluder's interval.
 * If that end is where the ray grazes the occluder's roof edge, t* solves
 *     g(t, H) = H - z_in(t) = 0,
 * with z_in(t) the height of the ray where it enters the footprint, so
 * d(t*) / dH = 1 / z_in'(t*) (implicit function theorem; z_in' by a central
 * difference in t).  An end made by a vertical edge (the ray leaving the
 * footprint's angular range) does not move with H.  A union boundary that
 * closes contributes +d(t*) / dH, one that opens -d(t*) / dH; ties go to the lower
 * building id. */

/* Height of the ray p + s d where it enters footprint b (s_in >= 0), or -1
 * if it does not cross the footprint ahead of p. */
static double entry_height(const scene64 *S, int b, const double *p, const double *d)
{
    double s_in = -INFINITY, s_out = INFINITY;
    int o = S->off[b], m = S->off[b + 1] - o;
    for (int i = 0; i < m; ++i) {
        const double *a = S->xy + 2 * (o + i), *c = S->xy + 2 * (o + (i + 1) % m);
        double nx = c[1] - a[1], ny = -(c[0] - a[0]);
        double num = nx * (a[0] - p[0]) + ny * (a[1] - p[1]);
        double den = nx * d[0] + ny * d[1];
        if (den > 0.0) { double t = num / den; if (t < s_out) s_out = t; }
        else if (den < 0.0) { double t = num / den; if (t > s_in) s_in = t; }
        else if (num < 0.0) return -1.0;
    }
    if (s_in < 0.0 || s_out < s_in) return -1.0;
    return p[2] + s_in * d[2];
}

typedef struct { double t; int b; int close; } endpoint;

typedef struct {
    const scene64 *S;
    const orc_points *P;
    int n_seg;
    const double *seg_t, *seg_dir;
    const int32_t *seg_day;
    const int32_t *day_bin;
    double grid;
    const double *dl;   /* [n_bins][n] or NULL */
    double *grad;       /* [n_b] per thread slice */
    int threads;
} grad_ctx;

/* d(t*) / dH of one interval end of prism b at time t (0 if a wall edge). */
static double end_rate(const scene64 *S, int b, const double *p, const double *da, const double *db,
                       double ta, double tb, double t)
{
    if (b < 0) return 0.0;
    double d[3];
    seg_dir_at(da, db, ta, tb, t, d);
    double z = entry_height(S, b, p, d);
    if (z < 0.0 || fabs(z - S->H[b]) > 1e-4) return 0.0;
    const double h = 1e-4;       /* minutes */
    double d0[3], d1[3];
    seg_dir_at(da, db, ta, tb, t - h, d0);
    seg_dir_at(da, db, ta, tb, t + h, d1);
    double z0 = entry_height(S, b, p, d0), z1 = entry_height(S, b, p, d1);
    if (z0 < 0.0 || z1 < 0.0) return 0.0;
    double dz = (z1 - z0) / (2 * h);
    return dz != 0.0 ? 1.0 / dz : 0.0;
}

static pthread_mutex_t grad_mu = PTHREAD_MUTEX_INITIALIZER;

static void grad_point(void *vctx, int64_t i)
{
    grad_ctx *C = (grad_ctx *)vctx;
    const scene64 *S = C->S;
    const orc_points *P = C->P;
    double p[3] = {P->x[i], P->y[i], P->z[i]};
    double nrm[2] = {P->nx ? P->nx[i] : 0.0, P->ny ? P->ny[i] : 0.0};
    int owner = P->owner ? P->owner[i] : -1;
    double *g = (double *)calloc(S->n_b ? S->n_b : 1, sizeof(double));
    for (int j = 0; j < C->n_seg; ++j) {
        double ta = C->seg_t[2 * j], tb = C->seg_t[2 * j + 1];
        const double *da = C->seg_dir + 6 * j, *db = da + 3;
        int day = C->seg_day ? C->seg_day[j] : 0;
        int bin = C->day_bin ? C->day_bin[day] : day;
        double w = C->dl ? C->dl[(int64_t)bin * P->n + i] : 1.0;
        if (w == 0.0 || !(tb > ta)) continue;
        /* intervals of every occluder, tagged with the occluder */
        double N[3];
        seg_plane(da, db, N);
        int ne = 0, cap = 64;
        endpoint *ev = (endpoint *)malloc(sizeof(endpoint) * cap);
        for (int b = (owner >= 0 ? -1 : 0); b < S->n_b; ++b) {
            if (b >= 0 && (b == owner || box_off_plane(S, b, p, N))) continue;
            ivec iv = {0, 0, 0};
            occluder_intervals(S, b, p, nrm, ta, tb, da, db, C->grid, &iv);
            for (int k = 0; k < iv.n; ++k) {
                if (ne + 2 > cap) { cap *= 2; ev = (endpoint *)realloc(ev, sizeof(endpoint) * cap); }
                ev[ne].t = iv.v[k].lo; ev[ne].b = b; ev[ne].close = 0; ++ne;
                ev[ne].t = iv.v[k].hi; ev[ne].b = b; ev[ne].close = 1; ++ne;
            }
            free(iv.v);
        }
        /* sweep: a union boundary is where the number of covering intervals
         * goes 0 -> 1 (opening) or 1 -> 0 (closing); equal times: opens
         * first (closed intervals touching merge), then lower id */
        for (int a = 1; a < ne; ++a) {           /* insertion sort: few events */
            endpoint e = ev[a];
            int c = a - 1;
            while (c >= 0 && (ev[c].t > e.t || (ev[c].t == e.t && (ev[c].close > e.close ||
                   (ev[c].close == e.close && ev[c].b > e.b))))) {
                ev[c + 1] = ev[c];
                --c;
            }
            ev[c + 1] = e;
        }
        int depth = 0;
        for (int a = 0; a < ne; ++a) {
            if (!ev[a].close) {
                if (depth == 0 && ev[a].t > ta && ev[a].b >= 0)
                    g[ev[a].b] -= w * end_rate(S, ev[a].b, p, da, db, ta, tb, ev[a].t);
                ++depth;
            } else {
                --depth;
                if (depth == 0 && ev[a].t < tb && ev[a].b >= 0)
                    g[ev[a].b] += w * end_rate(S, ev[a].b, p, da, db, ta, tb, ev[a].t);
            }
        }
        free(ev);
    }
    pthread_mutex_lock(&grad_mu);
    for (int b = 0; b < S->n_b; ++b) C->grad[b] += g[b];
    pthread_mutex_unlock(&grad_mu);
    free(g);
}

void orc_grad_implicit(const orc_scene *s, const orc_points *p, int n_seg,
                       const double *seg_t, const double *seg_dir, const int32_t *seg_day,
                       const int32_t *day_bin, double grid_min, const double *dl_dmin,
                       double *grad, int threads)
{
    scene64 S;
    scene64_init(&S, s);
    memset(grad, 0, sizeof(double) * (s->n_b ? s->n_b : 1));
    grad_ctx C;
    memset(&C, 0, sizeof(C));
    C.S = &S; C.P = p; C.n_seg = n_seg; C.seg_t = seg_t; C.seg_dir = seg_dir; C.seg_day = seg_day;
    C.day_bin = day_bin; C.grid = grid_min; C.dl = dl_dmin; C.grad = grad;
    parallel_for(p->n, threads, grad_point, &C);
    scene64_free(&S);
}

/* ---- building contribution (Sec. 7.2): per building, the weighted time
 * the points spend in that building's own shadow ----
 *
 * Each building's shadowed intervals over a point's path are found exactly
 * as for the continuous duration, but never merged with other buildings':
 * a moment shadowed by two buildings counts for both.  The shadow of a
 * facade point's own wall facing away from the sun belongs to its own
 * building.  contrib[bin][b] += weight(p) x minutes. */
typedef struct {
    const scene64 *S;
    const orc_points *P;
    int n_seg;
    const double *seg_t, *seg_dir;
    const int32_t *seg_day, *day_bin;
    double grid;
    const double *weight;
    int n_b;
    double *contrib;
} contrib_ctx;

static pthread_mutex_t contrib_mu = PTHREAD_MUTEX_INITIALIZER;

typedef struct { int64_t k; double v; } kv;

static void contrib_point(void *vctx, int64_t i)
{
    contrib_ctx *C = (contrib_ctx *)vctx;
    const scene64 *S = C->S;
    const orc_points *P = C->P;
    double p[3] = {P->x[i], P->y[i], P->z[i]};
    double nrm[2] = {P->nx ? P->nx[i] : 0.0, P->ny ? P->ny[i] : 0.0};
    int owner = P->owner ? P->owner[i] : -1;
    double w = C->weight ? C->weight[i] : 1.0;
    int n = 0, cap = 64;
    kv *acc = (kv *)malloc(sizeof(kv) * cap);
    for (int j = 0; j < C->n_seg; ++j) {
        double ta = C->seg_t[2 * j], tb = C->seg_t[2 * j + 1];
        if (!(tb > ta) || w == 0.0) continue;
        const double *da = C->seg_dir + 6 * j, *db = da + 3;
        int day = C->seg_day ? C->seg_day[j] : 0;
        int bin = C->day_bin ? C->day_bin[day] : day;
        double N[3];
        seg_plane(da, db, N);
        for (int b = (owner >= 0 ? -1 : 0); b < S->n_b; ++b) {
            if (b >= 0 && (b == owner || box_off_plane(S, b, p, N))) continue;
            ivec iv = {0, 0, 0};
            occluder_intervals(S, b, p, nrm, ta, tb, da, db, C->grid, &iv);
            double m = 0.0;
            for (int k = 0; k < iv.n; ++k) m += iv.v[k].hi - iv.v[k].lo;
            free(iv.v);
            if (m == 0.0) continue;
            if (n == cap) { cap *= 2; acc = (kv *)realloc(acc, sizeof(kv) * cap); }
            acc[n].k = (int64_t)bin * C->n_b + (b >= 0 ? b : owner);
            acc[n].v = w * m;
            ++n;
        }
    }
    pthread_mutex_lock(&contrib_mu);
    for (int a = 0; a < n; ++a) C->contrib[acc[a].k] += acc[a].v;
    pthread_mutex_unlock(&contrib_mu);
    free(acc);
}

void orc_contribution(const orc_scene *s, const orc_points *p, int n_seg,
                      const double *seg_t, const double *seg_dir, const int32_t *seg_day,
                      const int32_t *day_bin, int n_bins, double grid_min, const double *weight,
                      double *contrib, int threads)
{
    scene64 S;
    scene64_init(&S, s);
    memset(contrib, 0, sizeof(double) * (size_t)n_bins * (s->n_b ? s->n_b : 1));
    contrib_ctx C;
    memset(&C, 0, sizeof(C));
    C.S = &S; C.P = p; C.n_seg = n_seg; C.seg_t = seg_t; C.seg_dir = seg_dir; C.seg_day = seg_day;
    C.day_bin = day_bin; C.grid = grid_min; C.weight = weight; C.n_b = s->n_b; C.contrib = contrib;
    parallel_for(p->n, threads, contrib_point, &C);
    scene64_free(&S);
}

/* ---- raster shadow accrual map depth (Sec. 4) ----
 * For each ray X[r] + lam d (lam >= 0): the largest lam at which it leaves
 * a prism, each prism a convex solid clipped by its height slab and the
 * inner half-plane of every footprint edge, all moved outward by `grow`
 * metres (negative: inward); -INFINITY where it meets none. */
typedef struct {
    const orc_scene *s;
    const double *X, *d;
    double grow;
    double *out;
} exit_ctx;

static void exit_one(void *arg, int64_t r)
{
    const exit_ctx *E = (const exit_ctx *)arg;
    const orc_scene *s = E->s;
    const double *x = E->X + 3 * r, *d = E->d;
    const double grow = E->grow;
    double best = -INFINITY;
    for (int b = 0; b < s->n_b; ++b) {
        const int v0 = s->vert_off[b], v1 = s->vert_off[b + 1];
        const double H = s->height[b];
        double lo = fmax(0.0, (-grow - x[2]) / d[2]);
        double hi = (H + grow - x[2]) / d[2];
        int ok = 1;
        for (int v = v0; v < v1 && ok; ++v) {
            const int w = v + 1 < v1 ? v + 1 : v0;
            const double p0x = s->xy[2 * v], p0y = s->xy[2 * v + 1];
            const double ex = s->xy[2 * w] - p0x, ey = s->xy[2 * w + 1] - p0y;
            /* inside: cross(e, x - p0) >= -grow |e|; along the ray f0 + lam g */
            const double f0 = ex * (x[1] - p0y) - ey * (x[0] - p0x) + grow * sqrt(ex * ex + ey * ey);
            const double g = ex * d[1] - ey * d[0];
            if (g > 0.0) lo = fmax(lo, -f0 / g);
            else if (g < 0.0) hi = fmin(hi, -f0 / g);
            else if (f0 < 0.0) ok = 0;
        }
        if (ok && lo <= hi && hi > best) best = hi;
    }
    E->out[r] = best;
}

void orc_exit_depths(const orc_scene *s, int64_t m, const double *X, const double *d, double grow, double *out,
                     int threads)
{
    exit_ctx E = {s, X, d, grow, out};
    parallel_for(m, threads, exit_one, &E);
}
