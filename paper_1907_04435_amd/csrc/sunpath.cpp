// Sun path of the library: sample instants and great-circle knots of a time
// selection (start date, number of days, daily window -- Sec. 7.1), with
// solar position from the NOAA solar-calculator equations (Meeus'
// low-precision solar coordinates; the same published equations any
// implementation of that calculator follows).  Host code, FP64.
#include <cmath>
#include <cstring>

#include "sa_internal.h"

namespace sa {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kRad = kPi / 180.0;

// Days from the Julian-day epoch of 0h UT on a Gregorian calendar date.
double julian_day_0h(int y, int m, int d)
{
    if (m < 3) {
        y -= 1;
        m += 12;
    }
    const double century = std::floor(y / 100.0);
    const double greg = 2.0 - century + std::floor(century / 4.0);
    return std::floor(365.25 * (y + 4716)) + std::floor(30.6001 * (m + 1)) + d + greg - 1524.5;
}

struct SunCoords {
    double decl;     // radians
    double eot_min;  // apparent minus mean solar time, minutes
};

// Declination and equation of time at Julian day `jd` (UT).
SunCoords sun_coords(double jd)
{
    const double t = (jd - 2451545.0) / 36525.0;
    double mean_long = 280.46646 + t * (36000.76983 + 0.0003032 * t);
    mean_long = std::fmod(mean_long, 360.0);
    if (mean_long < 0.0) mean_long += 360.0;
    const double anomaly = 357.52911 + t * (35999.05029 - 0.0001537 * t);
    const double ecc = 0.016708634 - t * (0.000042037 + 0.0000001267 * t);
    const double m_r = anomaly * kRad;
    const double centre = std::sin(m_r) * (1.914602 - t * (0.004817 + 0.000014 * t)) +
                          std::sin(2.0 * m_r) * (0.019993 - 0.000101 * t) +
                          std::sin(3.0 * m_r) * 0.000289;
    const double node = (125.04 - 1934.136 * t) * kRad;
    const double app_long = (mean_long + centre - 0.00569 - 0.00478 * std::sin(node)) * kRad;
    const double obl_arcsec = 21.448 - t * (46.815 + t * (0.00059 - t * 0.001813));
    const double obliq = (23.0 + (26.0 + obl_arcsec / 60.0) / 60.0 + 0.00256 * std::cos(node)) * kRad;

    SunCoords c;
    c.decl = std::asin(std::sin(obliq) * std::sin(app_long));
    const double yv = std::tan(obliq * 0.5) * std::tan(obliq * 0.5);
    const double l2 = 2.0 * mean_long * kRad;
    const double eot = yv * std::sin(l2) - 2.0 * ecc * std::sin(m_r) +
                       4.0 * ecc * yv * std::sin(m_r) * std::cos(l2) -
                       0.5 * yv * yv * std::sin(2.0 * l2) - 1.25 * ecc * ecc * std::sin(2.0 * m_r);
    c.eot_min = eot * 4.0 / kRad;
    return c;
}

// Unit vector toward the sun (east, north, up) at local minute `t_loc` of the
// given date; local = UTC + tz hours.
void sun_direction(const sa_site &site, int y, int m, int d, double t_loc, double out[3])
{
    const double ut_min = t_loc - 60.0 * site.tz_offset_h;
    const double jd = julian_day_0h(y, m, d) + ut_min / 1440.0;
    const SunCoords c = sun_coords(jd);
    double frac = jd + 0.5;
    frac -= std::floor(frac);
    const double solar_min = frac * 1440.0 + c.eot_min + 4.0 * site.lon_deg;
    const double hour_angle = (solar_min * 0.25 - 180.0) * kRad;
    const double lat = site.lat_deg * kRad;
    const double cd = std::cos(c.decl), sd = std::sin(c.decl);
    const double ch = std::cos(hour_angle), sh = std::sin(hour_angle);
    double v[3] = {-cd * sh, std::cos(lat) * sd - std::sin(lat) * cd * ch,
                   std::sin(lat) * sd + std::cos(lat) * cd * ch};
    const double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) out[i] = v[i] / len;
}

void civil_add_days(int &y, int &m, int &d, int add)
{
    static const int mdays[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    while (add-- > 0) {
        const bool leap = (y % 4 == 0 && y % 100 != 0) || y % 400 == 0;
        const int dim = (m == 2 && leap) ? 29 : mdays[m - 1];
        if (++d > dim) {
            d = 1;
            if (++m > 12) {
                m = 1;
                ++y;
            }
        }
    }
}

}  // namespace

sa_status sunpath_fill(const sa_site &site, const sa_timespan &span, sa_sunpath_buf &out,
                       std::string &err)
{
    if (span.n_days < 1 || !(span.step_min > 0.0) || !(span.seg_min > 0.0) || span.month < 1 ||
        span.month > 12 || span.day < 1 || span.day > 31 || std::fabs(site.lat_deg) > 90.0) {
        err = "sa_sunpath: invalid time span or site";
        return SA_ERR_INVALID_ARG;
    }
    const bool sizing = out.cap_days == 0 && out.cap_samples == 0 && out.cap_knots == 0;
    int y = span.year, m = span.month, d = span.day;
    int n_samples = 0, n_knots = 0;
    if (!sizing && out.cap_days < span.n_days) {
        err = "sa_sunpath: cap_days too small";
        return SA_ERR_CAPACITY;
    }
    for (int day = 0; day < span.n_days; ++day) {
        if (day) civil_add_days(y, m, d, 1);
        // instants of the day
        double t0, t1, step;
        double dir[3];
        if (span.t_start_min < 0.0) {
            int first = -1, last = -1;
            for (int minute = 0; minute < 1440; ++minute) {
                sun_direction(site, y, m, d, minute, dir);
                if (dir[2] > 0.0) {
                    if (first >= 0 && minute != last + 1) {
                        err = "sa_sunpath: more than one daylight run in a day";
                        return SA_ERR_INVALID_ARG;
                    }
                    if (first < 0) first = minute;
                    last = minute;
                }
            }
            if (first < 0) {
                t0 = 0.0;
                t1 = -1.0;
            } else {
                t0 = first;
                t1 = last;
            }
            step = 1.0;
        } else {
            t0 = span.t_start_min;
            step = span.step_min;
            const int k = (int)std::floor((span.t_end_min - t0) / step + 1e-9);
            t1 = t0 + k * step;
        }
        const int K = t1 >= t0 ? (int)std::floor((t1 - t0) / step + 1e-9) + 1 : 0;
        if (!sizing) {
            out.day_sample_off[day] = n_samples;
            out.day_knot_off[day] = n_knots;
            if (n_samples + K > out.cap_samples) {
                err = "sa_sunpath: cap_samples too small";
                return SA_ERR_CAPACITY;
            }
            for (int k = 0; k < K; ++k) {
                const double t = t0 + k * step;
                double *dd = out.dir + 3 * (n_samples + k);
                sun_direction(site, y, m, d, t, dd);
                if (!(dd[2] > 0.0)) {
                    err = "sa_sunpath: window reaches below the horizon";
                    return SA_ERR_INVALID_ARG;
                }
                out.t_min[n_samples + k] = t;
                // the share of [t0, t1] closer to this instant than to any other
                const double lo = k == 0 ? t0 : t - 0.5 * step;
                const double hi = k == K - 1 ? t1 : t + 0.5 * step;
                out.weight[n_samples + k] = hi - lo;
            }
        }
        n_samples += K;
        // knots: t0, then t0 + L, t0 + 2L, ... (or the multiples of L in
        // local time after t0), below t1, and t1
        if (K > 0) {
            const double L = span.seg_min, first_clock = (std::floor(t0 / L) + 1.0) * L;
            auto knot = [&](int j) { return span.knot_clock ? first_clock + (j - 1) * L : t0 + j * L; };
            int J = 0;
            for (double tk = t0; tk < t1; tk = knot(++J)) {
                if (!sizing) {
                    if (n_knots + J >= out.cap_knots) {
                        err = "sa_sunpath: cap_knots too small";
                        return SA_ERR_CAPACITY;
                    }
                    out.knot_t[n_knots + J] = tk;
                    sun_direction(site, y, m, d, tk, out.knot_dir + 3 * (n_knots + J));
                }
            }
            if (!sizing) {
                if (n_knots + J >= out.cap_knots) {
                    err = "sa_sunpath: cap_knots too small";
                    return SA_ERR_CAPACITY;
                }
                out.knot_t[n_knots + J] = t1;
                sun_direction(site, y, m, d, t1, out.knot_dir + 3 * (n_knots + J));
            }
            n_knots += J + 1;
        }
        if (!sizing && out.day_bin) out.day_bin[day] = day;
    }
    if (!sizing) {
        out.day_sample_off[span.n_days] = n_samples;
        out.day_knot_off[span.n_days] = n_knots;
    }
    out.n_days = span.n_days;
    out.n_samples = n_samples;
    out.n_knots = n_knots;
    return SA_OK;
}

}  // namespace sa
