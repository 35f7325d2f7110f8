/*
 * Oracle solar position -- TEST INFRASTRUCTURE ONLY.
 *
 * The paper treats the sun as a directional light whose direction it takes
 * as given ("actual sun direction", Sec. 3.2, Table 1) without naming an
 * ephemeris.  This file follows the NOAA solar-calculator equations, which
 * are Meeus' low-precision solar coordinates (Astronomical Algorithms, 2nd
 * ed., ch. 7 Julian day, ch. 22 obliquity, ch. 25 solar coordinates) with
 * the equation of time in the Smart form NOAA uses.  Geometric elevation,
 * no refraction, Delta-T ignored.  FP64 throughout.
 */
#include <math.h>
#include "oracle.h"

#define DEG (M_PI / 180.0)

double orc_julian_day(int year, int month, double day)
{
    /* Meeus ch. 7, Gregorian calendar */
    if (month <= 2) {
        year -= 1;
        month += 12;
    }
    double a = floor(year / 100.0);
    double b = 2.0 - a + floor(a / 4.0);
    return floor(365.25 * (year + 4716)) + floor(30.6001 * (month + 1)) + day + b - 1524.5;
}

void orc_solar_jd(double jd, double lat_deg, double lon_deg, double *out)
{
    double T = (jd - 2451545.0) / 36525.0;          /* Julian centuries from J2000 */
    double L0 = fmod(280.46646 + T * (36000.76983 + T * 0.0003032), 360.0);
    if (L0 < 0) L0 += 360.0;
    double M = 357.52911 + T * (35999.05029 - 0.0001537 * T);
    double ecc = 0.016708634 - T * (0.000042037 + 0.0000001267 * T);
    double C = sin(M * DEG) * (1.914602 - T * (0.004817 + 0.000014 * T))
             + sin(2 * M * DEG) * (0.019993 - 0.000101 * T)
             + sin(3 * M * DEG) * 0.000289;
    double true_long = L0 + C;
    double omega = 125.04 - 1934.136 * T;
    double lambda = true_long - 0.00569 - 0.00478 * sin(omega * DEG);
    double eps0 = 23.0 + (26.0 + (21.448 - T * (46.815 + T * (0.00059 - T * 0.001813))) / 60.0) / 60.0;
    double eps = eps0 + 0.00256 * cos(omega * DEG);
    double decl = asin(sin(eps * DEG) * sin(lambda * DEG));

    double y = tan(eps * DEG / 2.0);
    y *= y;
    double eot_rad = y * sin(2 * L0 * DEG) - 2 * ecc * sin(M * DEG)
                   + 4 * ecc * y * sin(M * DEG) * cos(2 * L0 * DEG)
                   - 0.5 * y * y * sin(4 * L0 * DEG) - 1.25 * ecc * ecc * sin(2 * M * DEG);
    double eot_min = 4.0 * eot_rad / DEG;

    /* true solar time from UT: minutes of the UT day + EoT + 4 min/deg east */
    double ut_min = (jd + 0.5 - floor(jd + 0.5)) * 1440.0;
    double tst = ut_min + eot_min + 4.0 * lon_deg;
    double H = (tst / 4.0 - 180.0) * DEG;            /* hour angle, west positive */

    /* equatorial (H, decl) -> horizontal east-north-up unit vector */
    double phi = lat_deg * DEG;
    double e = -cos(decl) * sin(H);
    double n = cos(phi) * sin(decl) - sin(phi) * cos(decl) * cos(H);
    double u = sin(phi) * sin(decl) + cos(phi) * cos(decl) * cos(H);
    double r = sqrt(e * e + n * n + u * u);
    out[0] = e / r;
    out[1] = n / r;
    out[2] = u / r;
    out[3] = asin(out[2]) / DEG;
    double az = atan2(out[0], out[1]) / DEG;
    out[4] = az < 0 ? az + 360.0 : az;
    out[5] = decl / DEG;
    out[6] = eot_min;
    out[7] = lambda;
    out[8] = eps;
}

void orc_solar(int year, int month, int day, double t_loc_min, double tz_h,
               double lat_deg, double lon_deg, double *out)
{
    double jd = orc_julian_day(year, month, (double)day) + (t_loc_min / 60.0 - tz_h) / 24.0;
    orc_solar_jd(jd, lat_deg, lon_deg, out);
}

int orc_day_samples(int year, int month, int day, double tz_h, double lat, double lon,
                    double t0, double t1, double step, double *t, double *w,
                    int cap, double *span)
{
    double sol[9];
    int K = 0;
    if (t0 < 0) {
        /* whole local minutes with the sun above the geometric horizon */
        int first = -1, last = -1;
        for (int m = 0; m < 1440; ++m) {
            orc_solar(year, month, day, (double)m, tz_h, lat, lon, sol);
            if (sol[2] > 0.0) {
                if (first < 0) first = m;
                else if (m != last + 1) return -1;   /* not one daylight run */
                last = m;
            }
        }
        if (first < 0) { span[0] = span[1] = 0; return 0; }
        K = last - first + 1;
        if (K > cap) return -1;
        for (int k = 0; k < K; ++k) t[k] = first + k;
        span[0] = first;
        span[1] = last;
        step = 1.0;
    } else {
        K = (int)floor((t1 - t0) / step + 1e-9) + 1;
        if (K > cap) return -1;
        for (int k = 0; k < K; ++k) {
            t[k] = t0 + k * step;
            orc_solar(year, month, day, t[k], tz_h, lat, lon, sol);
            if (!(sol[2] > 0.0)) return -1;          /* fixed windows lie in daylight */
        }
        span[0] = t0;
        span[1] = t[K - 1];
    }
    /* each instant's cell: the part of [T0, T1] nearer to it than to any other */
    for (int k = 0; k < K; ++k) {
        double lo = (k == 0) ? span[0] : 0.5 * (t[k - 1] + t[k]);
        double hi = (k == K - 1) ? span[1] : 0.5 * (t[k] + t[k + 1]);
        w[k] = hi - lo;
    }
    return K;
}
