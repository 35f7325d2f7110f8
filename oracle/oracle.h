/*
 * CPU oracle for city-scale shadow accumulation -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 C.  It computes the quantities the paper defines
 * (gross shadow: the time a point spends in shadow over an interval,
 * Sec. 3.1) by their definitions, brute force against every building.
 * It shares no code, header or table with the HIP library; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Frame: local east-north-up, metres; ground z = 0; the sun is a
 * directional light (Sec. 3.2).  Prisms are convex CCW footprints extruded
 * from z = 0 to z = H, closed.
 */
#ifndef SHADOW_ORACLE_H
#define SHADOW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_b;
    const int32_t *vert_off; /* [n_b+1] */
    const float *xy;         /* [2*V]   */
    const float *height;     /* [n_b]   */
} orc_scene;

typedef struct {
    int64_t n;
    const float *x, *y, *z;
    const float *nx, *ny;  /* outward wall normal, 0 for ground points */
    const int32_t *owner;  /* building the point sits on, -1 for ground */
} orc_points;

/* ---- solar position (NOAA solar calculator = Meeus low-precision) ---- */
double orc_julian_day(int year, int month, double day);
/* out: [0..2] unit direction toward the sun (E,N,U), [3] elevation deg,
 * [4] azimuth deg clockwise from north, [5] declination deg,
 * [6] equation of time (minutes), [7] apparent longitude deg,
 * [8] true obliquity deg.  t_loc_min: minutes after local midnight,
 * local = UTC + tz_h hours. */
void orc_solar(int year, int month, int day, double t_loc_min, double tz_h,
               double lat_deg, double lon_deg, double *out);
/* Same quantities at a Julian day given directly (UT). */
void orc_solar_jd(double jd, double lat_deg, double lon_deg, double *out);

/* Sample instants of one day.  t0 < 0: whole local minutes with positive
 * geometric elevation (sunrise..sunset); otherwise t0, t0+step, ... <= t1.
 * Writes t (local minutes) and weights (minutes: each instant's share of
 * [T0, T1], nearest-instant cells) and the span T0, T1.  Returns K, or -1
 * if cap is too small / the daylight minutes are not contiguous. */
int orc_day_samples(int year, int month, int day, double tz_h, double lat, double lon,
                    double t0, double t1, double step, double *t, double *w,
                    int cap, double *span);

/* ---- predicate ---- */
int orc_shadow(const orc_scene *s, double px, double py, double pz,
               double nx, double ny, int owner, const double *d);
int orc_shadow_mt(const orc_scene *s, double px, double py, double pz,
                  double nx, double ny, int owner, const double *d);

/* ---- sampled form ---- */
void orc_sampled(const orc_scene *s, const orc_points *p, int K, const double *dirs,
                 const double *w, const int32_t *sample_bin, int n_bins,
                 int32_t *counts, double *minutes, uint32_t *bits, uint8_t *amb,
                 int threads);

/* ---- continuous duration along a piecewise great-circle path ---- */
/* seg_t [n_seg][2] knot times (minutes), seg_dir [n_seg][2][3] knot
 * directions, seg_day [n_seg] non-decreasing day index; day_bin [n_days]
 * output bin of each day (NULL: bin = day); sample_t / sample_day: the
 * sample instants counted when inside the day's shadowed set.
 * minutes / counts: [n_bins][n].  longest [n_bins][n] (NULL: not wanted):
 * the continuous shadow of Sec. 3.1, the longest member of a day's shadowed
 * set, maximum over the bin's days. */
void orc_continuous(const orc_scene *s, const orc_points *p, int n_seg,
                    const double *seg_t, const double *seg_dir, const int32_t *seg_day,
                    int n_days, const int32_t *day_bin, int n_bins, double grid_min,
                    const double *sample_t, const int32_t *sample_day, int n_samples,
                    double *minutes, int32_t *counts, double *longest, int threads);

/* ---- continuous duration along the actual sun path (Sec. 3.1, 3.2) ----
 * Per point and day: the measure of the times in [T0, T1] at which the
 * point is in shadow for the sun's actual direction (solar position
 * equations above, FP64), found per occluder on a `grid_min` scan with
 * every switch bisected, then unioned.  The day is walked in stretches of
 * `piece_min` minutes (a prism is skipped for a stretch only when provably
 * out of reach).  ymd [3 n_days] (year, month, day), tz_h [n_days],
 * span [2 n_days] (T0, T1 local minutes), day_bin [n_days] (NULL: bin =
 * day); minutes / longest [n_bins][n] (NULL: not wanted; longest = the
 * longest member of a day's shadowed set, maximum over the bin's days). */
void orc_continuous_true(const orc_scene *s, const orc_points *p, int n_days, const int32_t *ymd,
                         const double *tz_h, const double *span, const int32_t *day_bin, int n_bins,
                         double lat_deg, double lon_deg, double piece_min, double grid_min,
                         double *minutes, double *longest, int threads);

/* ---- building contribution (Sec. 7.2) ---- */
/* contrib [n_bins][n_b]: per building the weighted minutes the points spend
 * in that building's own shadow along the path (a moment shadowed by several
 * buildings counts for each; a facade point's back-facing wall counts for
 * its own building).  weight [n] (NULL: 1). */
void orc_contribution(const orc_scene *s, const orc_points *p, int n_seg,
                      const double *seg_t, const double *seg_dir, const int32_t *seg_day,
                      const int32_t *day_bin, int n_bins, double grid_min, const double *weight,
                      double *contrib, int threads);

/* ---- gradient of sum_p D_L(p) w.r.t. building heights ---- */
/* grad [n_b]: d/dH_b of sum over points and days of dl_dmin[bin][p] *
 * (continuous shadowed minutes), dl_dmin NULL = all ones. */
void orc_grad_implicit(const orc_scene *s, const orc_points *p, int n_seg,
                       const double *seg_t, const double *seg_dir, const int32_t *seg_day,
                       const int32_t *day_bin, double grid_min, const double *dl_dmin,
                       double *grad, int threads);

/* slerp on the great circle through a and b at constant angular rate */
void orc_slerp(const double *a, const double *b, double f, double *out);

/* ---- raster shadow accrual map (Sec. 4) ----
 * Per ray X[3r..3r+2] + lam d, lam >= 0: the largest lam at which it leaves
 * a prism (height slab and inner edge half-planes moved outward by grow m),
 * -INFINITY where it meets none. */
void orc_exit_depths(const orc_scene *s, int64_t m, const double *X, const double *d, double grow, double *out,
                     int threads);

#ifdef __cplusplus
}
#endif
#endif
