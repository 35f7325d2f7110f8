/* A plain C program that uses the shadow accrual library through its C ABI
 * only (no Python, no C++): three box buildings, four ground points and
 * two facade points, 21 June 2019 at 40.7 N 74.0 W from sunrise to sunset
 * at 5-minute instants with knots every 30 minutes.  Prints, for the
 * sampled and the accrual form, one line per point: form, index, shadowed
 * instants, shadow minutes.  Device memory comes from the HIP runtime; the
 * library enqueues on the default stream.  Exit status 1 on any error. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "shadow_accrual.h"

#define N_PTS 6

static sa_ctx *ctx = NULL;

static int check(sa_status s, const char *what)
{
    if (s == SA_OK) return 0;
    fprintf(stderr, "%s failed (%d): %s\n", what, (int)s, ctx ? sa_last_error(ctx) : "");
    return 1;
}

static int hcheck(hipError_t e, const char *what)
{
    if (e == hipSuccess) return 0;
    fprintf(stderr, "%s failed: %s\n", what, hipGetErrorString(e));
    return 1;
}

static int upload(const void *src, size_t bytes, void **dst)
{
    if (hcheck(hipMalloc(dst, bytes), "hipMalloc")) return 1;
    return hcheck(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
}

int main(void)
{
    if (check(sa_create(0, NULL, &ctx), "sa_create")) return 1;

    /* three counter-clockwise boxes */
    const int32_t vert_off[4] = {0, 4, 8, 12};
    const float xy[24] = {0, 0, 20, 0, 20, 20, 0, 20,      /* 30 m */
                          40, 0, 60, 0, 60, 30, 40, 30,    /* 60 m */
                          0, 50, 25, 50, 25, 70, 0, 70};   /* 15 m */
    const float height[3] = {30.f, 60.f, 15.f};
    sa_scene *scene = NULL;
    if (check(sa_scene_upload(ctx, 3, vert_off, xy, height, &scene), "sa_scene_upload")) return 1;

    const sa_site site = {40.7, -74.0, -4.0};
    const sa_timespan span = {2019, 6, 21, 1, -1.0, -1.0, 5.0, 30.0, 0};
    sa_sunpath_buf buf = {0};
    if (check(sa_sunpath(&site, &span, &buf), "sa_sunpath (sizes)")) return 1;
    buf.cap_days = buf.n_days;
    buf.cap_samples = buf.n_samples;
    buf.cap_knots = buf.n_knots;
    buf.day_sample_off = malloc(sizeof(int32_t) * (buf.n_days + 1));
    buf.t_min = malloc(sizeof(double) * buf.n_samples);
    buf.dir = malloc(sizeof(double) * 3 * buf.n_samples);
    buf.weight = malloc(sizeof(double) * buf.n_samples);
    buf.day_knot_off = malloc(sizeof(int32_t) * (buf.n_days + 1));
    buf.knot_t = malloc(sizeof(double) * buf.n_knots);
    buf.knot_dir = malloc(sizeof(double) * 3 * buf.n_knots);
    buf.day_bin = NULL;
    if (check(sa_sunpath(&site, &span, &buf), "sa_sunpath")) return 1;
    sa_path *path = NULL;
    if (check(sa_path_upload(ctx, &buf, &path), "sa_path_upload")) return 1;

    /* four ground points, then facade points on the east wall of building
     * 0 and the north wall of building 1 */
    const float x[N_PTS] = {30, 10, 50, 70, 20, 50};
    const float y[N_PTS] = {10, 35, 40, 10, 10, 30};
    const float z[N_PTS] = {0, 0, 0, 0, 10, 20};
    const float nx[N_PTS] = {0, 0, 0, 0, 1, 0};
    const float ny[N_PTS] = {0, 0, 0, 0, 0, 1};
    const int32_t owner[N_PTS] = {-1, -1, -1, -1, 0, 1};
    void *dx, *dy, *dz, *dnx, *dny, *down, *dcounts, *dminutes;
    if (upload(x, sizeof x, &dx) || upload(y, sizeof y, &dy) || upload(z, sizeof z, &dz) ||
        upload(nx, sizeof nx, &dnx) || upload(ny, sizeof ny, &dny) || upload(owner, sizeof owner, &down))
        return 1;
    if (hcheck(hipMalloc(&dcounts, sizeof(int32_t) * N_PTS), "hipMalloc") ||
        hcheck(hipMalloc(&dminutes, sizeof(float) * N_PTS), "hipMalloc"))
        return 1;
    const sa_points pts = {N_PTS, dx, dy, dz, dnx, dny, down};

    const int32_t modes[2] = {SA_SAMPLED, SA_ACCRUAL};
    const char *names[2] = {"sampled", "accrual"};
    for (int f = 0; f < 2; ++f) {
        sa_accum_opts o = {0};
        o.mode = modes[f];
        if (check(sa_accumulate(ctx, scene, &pts, path, &o, dcounts, dminutes, NULL), "sa_accumulate")) return 1;
        if (check(sa_sync(ctx), "sa_sync")) return 1;
        int32_t counts[N_PTS];
        float minutes[N_PTS];
        if (hcheck(hipMemcpy(counts, dcounts, sizeof counts, hipMemcpyDeviceToHost), "hipMemcpy") ||
            hcheck(hipMemcpy(minutes, dminutes, sizeof minutes, hipMemcpyDeviceToHost), "hipMemcpy"))
            return 1;
        for (int i = 0; i < N_PTS; ++i) printf("%s %d %d %.6f\n", names[f], i, counts[i], minutes[i]);
    }

    (void)hipFree(dx); (void)hipFree(dy); (void)hipFree(dz); (void)hipFree(dnx); (void)hipFree(dny);
    (void)hipFree(down); (void)hipFree(dcounts); (void)hipFree(dminutes);
    sa_path_destroy(path);
    sa_scene_destroy(scene);
    sa_destroy(ctx);
    free(buf.day_sample_off); free(buf.t_min); free(buf.dir); free(buf.weight);
    free(buf.day_knot_off); free(buf.knot_t); free(buf.knot_dir);
    return 0;
}
