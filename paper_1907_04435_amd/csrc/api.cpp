// C entry points of libsa: argument checking, object lifetimes, path
// preparation, and dispatch to the device code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "sa_internal.h"

struct sa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    sa::SpillQueue spill;
    sa::Scratch scratch;          // region sums
    sa::Scratch scratch_batched;  // per-variant hierarchy copies
    sa::Scratch scratch_seg;      // per-segment node views of the accrual form
    sa::Scratch scratch_sam;      // one segment's raster shadow accrual map
    sa::Scratch scratch_grad;     // FP64 height-gradient accumulator
    sa::Scratch scratch_w;        // per-bin weights of a region score
    sa::Scratch scratch_piece;    // per-piece sums of accrual launches on few tiles
    uint32_t sam_stamp = 0;       // the last segment stamp written into it
    sa_launch launch = {0, 0, 1, 0, 0, 0, {0, 0}};  // tuning choices (sa_set_launch)
    int32_t n_cu = 256;           // compute units of the device
    void *noalloc = nullptr;      // this device's fixed scratch (device address), or null
    std::string noalloc_err;      // why it is null
};

struct sa_scene {
    sa_ctx *ctx = nullptr;
    int device = 0;  // kept here: the scene may outlive its context object
    sa::DeviceScene d;
    std::vector<int32_t> rank_h;  // original id -> hierarchy position
    bool max_h_stale = false;     // heights changed on the device since d.max_h was known
};

namespace {

// The tallest height the scene has had, reading the device heights when a
// device-side edit made the host copy stale (host-synchronous).
float scene_max_height(const sa_scene *scene)
{
    if (scene->max_h_stale && scene->d.n_b > 0) {
        std::vector<float> h(scene->d.n_b);
        if (hipMemcpy(h.data(), scene->d.height, sizeof(float) * h.size(), hipMemcpyDeviceToHost) == hipSuccess) {
            sa_scene *s = const_cast<sa_scene *>(scene);
            for (float v : h) s->d.max_h = std::max(s->d.max_h, v);
            s->max_h_stale = false;
        }
    }
    return scene->d.max_h;
}

}  // namespace

struct sa_path {
    sa_ctx *ctx = nullptr;
    int device = 0;
    sa::DevicePath d;
};

namespace {

constexpr int32_t kSpillCapacity = 1 << 20;

sa_status fail(sa_ctx *ctx, sa_status rc, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return rc;
}

sa_status hip_fail(sa_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? SA_ERR_OOM : SA_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

// Select the context's device and drop any error left pending by
// unrelated HIP calls, so that the launch checks below see only ours.
bool set_device(sa_ctx *ctx)
{
    (void)hipGetLastError();
    return hipSetDevice(ctx->device) == hipSuccess;
}

}  // namespace

// Fixed device scratch of sa_accumulate_noalloc, for callers that cannot
// allocate: the accrual form's per-segment hierarchy views.  Every device
// the library runs on holds its own copy from first use until the process
// ends.  Host code never uses this name as an address: the device address
// comes from hipGetSymbolAddress, once per device, in sa_create.
static __device__ __align__(256) unsigned char scratch[SA_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_noalloc_mu;
std::map<int, void *> g_noalloc_ptr;  // device -> address of `scratch` on it

// With ctx->device current: the device address of this device's fixed
// scratch (looked up on the device's first context, then reused).
void attach_noalloc_scratch(sa_ctx *ctx)
{
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(ctx->device);
    if (it != g_noalloc_ptr.end()) {
        ctx->noalloc = it->second;
        return;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        ctx->noalloc = nullptr;
        ctx->noalloc_err = std::string("fixed scratch unavailable: hipGetSymbolAddress: ") + hipGetErrorString(e);
        return;
    }
    g_noalloc_ptr[ctx->device] = ptr;
    ctx->noalloc = ptr;
}

}  // namespace

namespace {

// Is p device memory (as opposed to host memory the CPU can read)?
static bool on_device(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // plain host memory on some runtimes
        return false;
    }
    return a.type == hipMemoryTypeDevice && !a.isManaged;
}

// A host-readable copy of n elements at p: p itself for host memory, else
// the elements copied into `stash`.
template <class T>
static const T *host_view(const T *p, size_t n, std::vector<T> &stash, hipError_t &e)
{
    e = hipSuccess;
    if (n == 0 || !on_device(p)) return p;
    stash.resize(n);
    e = hipMemcpy(stash.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost);
    return stash.data();
}

}  // namespace

extern "C" {

const char *sa_version(void) { return "libsa 0.1 (gfx950)"; }

// Device words of a context's counters: the spill queue's (lengths,
// overflow flag), then the accrual launch's eight work counters.
constexpr int kCounterWords = 64 + 8 * 32;

sa_status sa_create(int32_t device, void *hip_stream, sa_ctx **out)
{
    if (!out) return SA_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SA_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return SA_ERR_DEVICE;
    sa_ctx *c = new (std::nothrow) sa_ctx();
    if (!c) return SA_ERR_OOM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->spill.capacity = kSpillCapacity;
    if (hipMalloc((void **)&c->spill.entries[0], sizeof(int4) * kSpillCapacity) != hipSuccess ||
        hipMalloc((void **)&c->spill.entries[1], sizeof(int4) * kSpillCapacity) != hipSuccess ||
        hipMalloc((void **)&c->spill.counters, sizeof(uint32_t) * kCounterWords) != hipSuccess ||
        hipMemset(c->spill.counters, 0, sizeof(uint32_t) * kCounterWords) != hipSuccess) {
        sa_destroy(c);
        return SA_ERR_OOM;
    }
    c->spill.grab = c->spill.counters + 64;  // 256 B in, eight 128 B lines
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && n_cu > 0)
        c->n_cu = n_cu;
    attach_noalloc_scratch(c);
    *out = c;
    return SA_OK;
}

void sa_destroy(sa_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->spill.entries[0]);
    (void)hipFree(ctx->spill.entries[1]);
    (void)hipFree(ctx->spill.counters);
    (void)hipFree(ctx->scratch.ptr);
    (void)hipFree(ctx->scratch_batched.ptr);
    (void)hipFree(ctx->scratch_seg.ptr);
    (void)hipFree(ctx->scratch_sam.ptr);
    (void)hipFree(ctx->scratch_grad.ptr);
    (void)hipFree(ctx->scratch_w.ptr);
    (void)hipFree(ctx->scratch_piece.ptr);
    delete ctx;
}

sa_status sa_set_launch(sa_ctx *ctx, const sa_launch *l)
{
    if (!ctx || !l) return SA_ERR_INVALID_ARG;
    if (l->accrual_segments_per_launch < 0 || l->batched_grid_blocks < 0 || l->batched_grid_blocks > (1 << 20) ||
        l->batched_tiles_per_grab < 0 || l->batched_tiles_per_grab > 1024 || l->tile_grid_blocks < 0 ||
        l->tile_grid_blocks > (1 << 20) ||
        (l->accrual_waves_per_simd != 0 && (l->accrual_waves_per_simd < 6 || l->accrual_waves_per_simd > 8)) ||
        (l->sampled_instants_per_packet < 0 || l->sampled_instants_per_packet > 16 ||
         (l->sampled_instants_per_packet & (l->sampled_instants_per_packet - 1)) != 0) ||
        l->reserved[0] != 0 || l->reserved[1] != 0)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_set_launch: value out of range");
    ctx->launch = *l;
    if (ctx->launch.batched_tiles_per_grab == 0) ctx->launch.batched_tiles_per_grab = 1;
    return SA_OK;
}

sa_status sa_get_launch(const sa_ctx *ctx, sa_launch *l)
{
    if (!ctx || !l) return SA_ERR_INVALID_ARG;
    *l = ctx->launch;
    return SA_OK;
}

sa_status sa_set_stream(sa_ctx *ctx, void *hip_stream)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return SA_OK;
}

const char *sa_last_error(const sa_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

sa_status sa_measure_valu_peak(sa_ctx *ctx, double *lane_ops_per_s)
{
    if (!ctx || !lane_ops_per_s) return SA_ERR_INVALID_ARG;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    std::string err;
    const sa_status rc = sa::measure_valu_peak(ctx->n_cu, (float *)ctx->spill.entries[0],
                                               (int64_t)ctx->spill.capacity * 4, ctx->stream, *lane_ops_per_s, err);
    return rc == SA_OK ? SA_OK : fail(ctx, rc, err);
}

sa_status sa_sync(sa_ctx *ctx)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
    uint32_t flag = 0;
    e = hipMemcpy(&flag, ctx->spill.counters + 2, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "read spill flag");
    if (flag) {
        (void)hipMemset(ctx->spill.counters + 2, 0, sizeof(uint32_t));
        // bit 0: spill queue full; bit 1: a window could not be split finely
        // enough; bit 2: a variant named a bad building id or height
        if (flag & 4u)
            return fail(ctx, SA_ERR_INVALID_ARG,
                        "a building id or height was invalid (batched variants or a device height edit)");
        return fail(ctx, SA_ERR_CAPACITY,
                    (flag & 1u) ? "accrual spill queue overflowed: results incomplete"
                                : "occluded set too fragmented to split: results incomplete");
    }
    return SA_OK;
}

// ------------------------------------------------------------------ scene
sa_status sa_scene_upload(sa_ctx *ctx, int32_t n_b, const int32_t *vert_off_in, const float *xy_in,
                          const float *height_in, sa_scene **out)
{
    if (!ctx || !out) return SA_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_b < 0 || (n_b > 0 && (!vert_off_in || !xy_in || !height_in)))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_scene_upload: bad arguments");
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    // host or device arrays: device ones are read through host copies
    std::vector<int32_t> off_h;
    std::vector<float> xy_h, h_h;
    hipError_t he = hipSuccess;
    const int32_t *vert_off = n_b > 0 ? host_view(vert_off_in, (size_t)n_b + 1, off_h, he) : vert_off_in;
    if (he != hipSuccess) return hip_fail(ctx, he, "sa_scene_upload: reading vert_off");
    if (n_b > 0 && vert_off[0] != 0) return fail(ctx, SA_ERR_INVALID_ARG, "sa_scene_upload: vert_off[0] != 0");
    if (n_b > 0 && vert_off[n_b] < 3 * (int64_t)n_b)
        return fail(ctx, SA_ERR_GEOMETRY, "sa_scene_upload: fewer than 3 vertices per prism");
    const float *xy = n_b > 0 ? host_view(xy_in, 2 * (size_t)vert_off[n_b], xy_h, he) : xy_in;
    if (he != hipSuccess) return hip_fail(ctx, he, "sa_scene_upload: reading xy");
    const float *height = n_b > 0 ? host_view(height_in, (size_t)n_b, h_h, he) : height_in;
    if (he != hipSuccess) return hip_fail(ctx, he, "sa_scene_upload: reading height");
    // the accrual traversal addresses per-segment node views (64 bytes
    // each) with 32-bit byte offsets
    if (n_b > (1 << 25)) return fail(ctx, SA_ERR_CAPACITY, "sa_scene_upload: more than 2^25 prisms");
    for (int32_t b = 0; b < n_b; ++b) {
        const int32_t o = vert_off[b], m = vert_off[b + 1] - o;
        if (m < 3) return fail(ctx, SA_ERR_GEOMETRY, "prism " + std::to_string(b) + ": fewer than 3 vertices");
        if (!(height[b] > 0.f) || !std::isfinite(height[b]))
            return fail(ctx, SA_ERR_GEOMETRY, "prism " + std::to_string(b) + ": height must be > 0");
        for (int32_t i = 0; i < m; ++i) {
            const double ax = xy[2 * (o + i)], ay = xy[2 * (o + i) + 1];
            const int32_t i1 = (i + 1) % m, i2 = (i + 2) % m;
            const double bx = xy[2 * (o + i1)], by = xy[2 * (o + i1) + 1];
            const double cx = xy[2 * (o + i2)], cy = xy[2 * (o + i2) + 1];
            if (!std::isfinite(ax) || !std::isfinite(ay))
                return fail(ctx, SA_ERR_GEOMETRY, "prism " + std::to_string(b) + ": non-finite vertex");
            if ((bx - ax) * (cy - by) - (by - ay) * (cx - bx) <= 0.0)
                return fail(ctx, SA_ERR_GEOMETRY,
                            "prism " + std::to_string(b) + ": footprint not strictly convex and counter-clockwise");
        }
    }
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    sa_scene *s = new (std::nothrow) sa_scene();
    if (!s) return fail(ctx, SA_ERR_OOM, "host allocation failed");
    s->ctx = ctx;
    s->device = ctx->device;
    std::string err;
    sa_status rc = sa::scene_build(s->d, ctx->stream, n_b, vert_off, xy, height, err);
    if (rc != SA_OK) {
        delete s;
        return fail(ctx, rc, "sa_scene_upload: " + err);
    }
    s->rank_h.resize(n_b);
    if (n_b > 0) {
        hipError_t e = hipMemcpy(s->rank_h.data(), s->d.rank, sizeof(int32_t) * n_b, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            sa::scene_free(s->d);
            delete s;
            return hip_fail(ctx, e, "sa_scene_upload: rank copy");
        }
    }
    *out = s;
    return SA_OK;
}

sa_status sa_scene_set_heights(sa_ctx *ctx, sa_scene *scene, int32_t n, const int32_t *ids, const float *h)
{
    if (!ctx || !scene || n < 0 || (n > 0 && (!ids || !h)))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_scene_set_heights: bad arguments");
    if (n == 0) return SA_OK;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    const bool dev_ids = on_device(ids), dev_h = on_device(h);
    if (dev_ids != dev_h)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_scene_set_heights: ids and heights must both be host or device");
    if (dev_ids) {
        // stream-ordered: scatter on the device (bad entries are skipped and
        // flagged for sa_sync), then refit; nothing returns to the host
        std::string err;
        sa_status rc = sa::scene_set_heights_device(scene->d, n, ids, h, ctx->spill.counters + 2, ctx->stream, err);
        if (rc == SA_OK) rc = sa::scene_refit(scene->d, ctx->stream, err);
        if (rc != SA_OK) return fail(ctx, rc, "sa_scene_set_heights: " + err);
        scene->max_h_stale = true;
        return SA_OK;
    }
    std::vector<int32_t> pos(n);
    for (int32_t k = 0; k < n; ++k) {
        if (ids[k] < 0 || ids[k] >= scene->d.n_b)
            return fail(ctx, SA_ERR_INVALID_ARG, "sa_scene_set_heights: building id out of range");
        if (!(h[k] > 0.f) || !std::isfinite(h[k])) return fail(ctx, SA_ERR_GEOMETRY, "height must be > 0");
        pos[k] = scene->rank_h[ids[k]];
    }
    // heights are few: scatter them with small copies, then refit on device
    for (int32_t k = 0; k < n; ++k) {
        hipError_t e = hipMemcpyAsync(scene->d.height + pos[k], h + k, sizeof(float), hipMemcpyHostToDevice,
                                      ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "sa_scene_set_heights: copy");
    }
    std::string err;
    sa_status rc = sa::scene_refit(scene->d, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_scene_set_heights: " + err);
    float mh = 0.f;
    for (int32_t k = 0; k < n; ++k) mh = std::max(mh, h[k]);
    scene->d.max_h = std::max(scene->d.max_h, mh);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "sa_scene_set_heights");
    return SA_OK;
}

sa_status sa_scene_get_info(const sa_scene *scene, sa_scene_info *out)
{
    if (!scene || !out) return SA_ERR_INVALID_ARG;
    out->n_b = scene->d.n_b;
    out->n_vert = scene->d.n_vert;
    out->n_nodes = scene->d.n_nodes;
    out->depth = scene->d.depth;
    for (int i = 0; i < 4; ++i) out->bounds[i] = scene->d.bounds[i];
    out->max_height = scene_max_height(scene);
    return SA_OK;
}

sa_status sa_scene_read_bvh(sa_ctx *ctx, const sa_scene *scene, void *nodes, int32_t *prim_order)
{
    if (!ctx || !scene) return SA_ERR_INVALID_ARG;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess && nodes && scene->d.n_nodes > 0)
        e = hipMemcpy(nodes, scene->d.nodes, sizeof(sa::Node) * scene->d.n_nodes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && prim_order && scene->d.n_b > 0)
        e = hipMemcpy(prim_order, scene->d.order, sizeof(int32_t) * scene->d.n_b, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "sa_scene_read_bvh");
    return SA_OK;
}

void sa_scene_destroy(sa_scene *scene)
{
    if (!scene) return;
    (void)hipSetDevice(scene->device);
    sa::scene_free(scene->d);
    delete scene;
}

// ------------------------------------------------------------------ paths
sa_status sa_sunpath(const sa_site *site, const sa_timespan *span, sa_sunpath_buf *out)
{
    if (!site || !span || !out) return SA_ERR_INVALID_ARG;
    const bool sizing = out->cap_days == 0 && out->cap_samples == 0 && out->cap_knots == 0;
    if (!sizing && (!out->day_sample_off || !out->t_min || !out->dir || !out->weight || !out->day_knot_off ||
                    !out->knot_t || !out->knot_dir))
        return SA_ERR_INVALID_ARG;
    std::string err;
    return sa::sunpath_fill(*site, *span, *out, err);
}

}  // extern "C"

namespace {

// The great-circle geometry of a segment from knot direction a (at ta) to
// b (at tb), both unit vectors above the horizon: plane basis, angle, the
// lift of horizontal offsets into the plane (times |nz|), the fan's offsets
// per metre of rise, the visit-order direction and the time map.  False if
// the directions coincide.
bool seg_geometry(const double *a, const double *b, double ta, double tb, sa::SegConst &g)
{
    const double c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double sn = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(sn > 1e-12)) return false;
    const double theta = std::atan2(sn, c);
    double e2[3] = {b[0] - c * a[0], b[1] - c * a[1], b[2] - c * a[2]};
    const double l2 = std::sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    for (double &v : e2) v /= l2;
    const double N[3] = {a[1] * e2[2] - a[2] * e2[1], a[2] * e2[0] - a[0] * e2[2], a[0] * e2[1] - a[1] * e2[0]};
    // the lift of horizontal offsets into the plane, times |nz|:
    // |nz| (a - a_z N_xy / nz) = |nz| a - sgn(nz) a_z N_xy
    const double anz = std::fabs(N[2]), sg = N[2] < 0.0 ? -1.0 : 1.0;
    g.m00 = (float)(anz * a[0] - sg * a[2] * N[0]);
    g.m01 = (float)(anz * a[1] - sg * a[2] * N[1]);
    g.m10 = (float)(anz * e2[0] - sg * e2[2] * N[0]);
    g.m11 = (float)(anz * e2[1] - sg * e2[2] * N[1]);
    g.steep = anz < std::sin(5.0 * M_PI / 180.0) ? 1 : 0;
    g.e1z = (float)a[2];
    g.e2z = (float)e2[2];
    g.theta = (float)theta;
    g.cth = (float)std::cos(theta);
    g.sth = (float)std::sin(theta);
    g.nz = (float)N[2];
    g.e1x = (float)a[0];
    g.e1y = (float)a[1];
    g.e2x = (float)e2[0];
    g.e2y = (float)e2[1];
    g.ua_x = (float)(a[0] / a[2]);
    g.ua_y = (float)(a[1] / a[2]);
    g.ub_x = (float)(b[0] / b[2]);
    g.ub_y = (float)(b[1] / b[2]);
    g.rate = (float)((tb - ta) / theta);
    g.wrate = g.rate;
    g.mdx = (float)(a[0] + e2[0] * 0.5 * theta);
    g.mdy = (float)(a[1] + e2[1] * 0.5 * theta);
    return true;
}

// Direction-graph reuse (Sec. 6): the hemisphere is cut into cells of at
// most `bound` radians (rings of that height in elevation, each cut into
// the fewest azimuth sectors no wider than `bound` at the ring's lower
// edge); segments of one output bin whose start and end knots fall in the
// same pair of cells are one edge, computed once and weighted by how many
// segments it stands for (Eq. (1) sums the edges' maps by multiplicity).  The
// edge's arc runs from the members' mean start direction to their mean end
// direction (the cluster's representative) over the first member's times;
// the minutes per radian its measure is weighted by become the members'
// total duration over that arc's angle, so each member counts with its own
// duration; sample counts are scaled by the multiplicity.
void merge_segments(std::vector<sa::SegConst> &segs, const std::vector<std::array<double, 6>> &knots,
                    double bound)
{
    auto cell = [bound](const double *d) {
        const double el = std::asin(std::max(-1.0, std::min(1.0, d[2])));
        const double az = std::atan2(d[0], d[1]);
        const int64_t ring = (int64_t)std::floor(el / bound);
        const int64_t naz =
            std::max<int64_t>(1, (int64_t)std::ceil(2.0 * M_PI * std::cos((double)ring * bound) / bound));
        const int64_t c = (int64_t)std::floor((az + M_PI) / (2.0 * M_PI) * (double)naz);
        // a ring has fewer than 2^32 sectors for bounds >= 1e-6 degrees
        return ring * ((int64_t)1 << 32) + std::min(c, naz - 1);
    };
    std::map<std::tuple<int32_t, int64_t, int64_t>, size_t> edge;
    std::vector<sa::SegConst> out;
    std::vector<double> dt_sum;
    std::vector<std::array<double, 6>> dir_sum;  // summed start and end directions of the members
    for (size_t s = 0; s < segs.size(); ++s) {
        const auto key = std::make_tuple(segs[s].bin, cell(knots[s].data()), cell(knots[s].data() + 3));
        auto it = edge.find(key);
        if (it == edge.end()) {
            edge.emplace(key, out.size());
            out.push_back(segs[s]);
            dt_sum.push_back(segs[s].dt);
            dir_sum.push_back(knots[s]);
            continue;
        }
        const size_t e = it->second;
        sa::SegConst &g = out[e];
        dt_sum[e] += segs[s].dt;
        for (int i = 0; i < 6; ++i) dir_sum[e][i] += knots[s][i];
        g.mult += 1;
        g.ns_all += segs[s].ns;
    }
    for (size_t e = 0; e < out.size(); ++e) {
        sa::SegConst &g = out[e];
        if (g.mult == 1) continue;  // a lone segment keeps its own arc and weights
        // the members' mean start and end directions, each normalised; the
        // first member's arc stays if they were ever to coincide
        double a[3], b[3];
        const double *s = dir_sum[e].data();
        const double la = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        const double lb = std::sqrt(s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
        for (int i = 0; i < 3; ++i) {
            a[i] = s[i] / la;
            b[i] = s[3 + i] / lb;
        }
        sa::SegConst rep = g;
        if (a[2] > 0.0 && b[2] > 0.0 && seg_geometry(a, b, (double)g.ta, (double)g.ta + (double)g.dt, rep)) g = rep;
        g.dt = (float)dt_sum[e];
        g.wrate = (float)(dt_sum[e] / g.theta);
    }
    segs = std::move(out);
}

sa_status path_upload(sa_ctx *ctx, const sa_sunpath_buf *in, double bound_deg, sa_path **out)
{
    if (!ctx || !in || !out) return SA_ERR_INVALID_ARG;
    *out = nullptr;
    const int D = in->n_days;
    if (D < 1 || in->n_samples < 0 || in->n_knots < 0 || !in->day_sample_off || !in->day_knot_off ||
        (in->n_samples > 0 && (!in->t_min || !in->dir || !in->weight)) ||
        (in->n_knots > 0 && (!in->knot_t || !in->knot_dir)))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: bad arguments");
    std::vector<sa::SampleConst> samples(in->n_samples);
    std::vector<sa::SegConst> segs;
    std::vector<std::array<double, 6>> seg_knots;  // knot directions of each segment
    std::vector<sa::SamSegHost> seg_host;          // the raster form's per-segment record
    std::vector<sa::SamSlice> sam(in->n_samples);  // and its slice per instant
    std::vector<int32_t> day_seg_off;
    std::vector<double> bin_span;  // daylight minutes per bin: the instants' weights add up to each day's span
    int n_bins = 0;
    for (int d = 0; d < D; ++d) {
        day_seg_off.push_back((int32_t)segs.size());
        const int bin = in->day_bin ? in->day_bin[d] : d;
        if (bin < 0 || bin > sa::kBinMask) return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: bad bin");
        n_bins = std::max(n_bins, bin + 1);
        const int s0 = in->day_sample_off[d], s1 = in->day_sample_off[d + 1];
        const int k0 = in->day_knot_off[d], k1 = in->day_knot_off[d + 1];
        if (s0 < 0 || s1 < s0 || s1 > in->n_samples || k0 < 0 || k1 < k0 || k1 > in->n_knots)
            return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: bad day offsets");
        for (int k = s0; k < s1; ++k) {
            const double *dd = in->dir + 3 * k;
            if (!(dd[2] > 0.0)) return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: sun below the horizon");
            sa::SampleConst &c = samples[k];
            c.dx = (float)dd[0];
            c.dy = (float)dd[1];
            c.dz = (float)dd[2];
            c.w = (float)in->weight[k];
            auto inv = [](float v) { return 1.0f / (std::fabs(v) < 1e-20f ? std::copysign(1e-20f, v) : v); };
            c.ix = inv(c.dx);
            c.iy = inv(c.dy);
            c.iz = inv(c.dz);
            c.tag = bin | (k == s0 ? sa::kDayStart : 0);
            if ((int)bin_span.size() <= bin) bin_span.resize(bin + 1, 0.0);
            bin_span[bin] += in->weight[k];
        }
        const double step = s1 - s0 >= 2 ? in->t_min[s0 + 1] - in->t_min[s0] : 1.0;
        for (int k = k0; k + 1 < k1; ++k) {
            const double ta = in->knot_t[k], tb = in->knot_t[k + 1];
            if (!(tb > ta)) return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: knots not increasing");
            const double *a = in->knot_dir + 3 * k, *b = in->knot_dir + 3 * (k + 1);
            if (!(a[2] > 0.0) || !(b[2] > 0.0))
                return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: knot below the horizon");
            sa::SegConst g;
            std::memset(&g, 0, sizeof(g));
            if (!seg_geometry(a, b, ta, tb, g))
                return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload: coincident knot directions");
            // FP64 angle of the arc, for the raster slices' directions below
            const double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
            const double sn = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            const double theta = std::atan2(sn, a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
            g.dt = (float)(tb - ta);
            g.ta = (float)ta;
            g.mult = 1;
            g.bin = bin;
            g.day = d;
            // sample instants attributed to this segment: [ta, tb), the day's
            // last segment also takes tb
            const bool last = k + 2 == k1;
            int first = -1, ns = 0;
            for (int s = s0; s < s1; ++s) {
                const double t = in->t_min[s];
                if (t >= ta && (t < tb || (last && t <= tb))) {
                    if (first < 0) first = s;
                    ++ns;
                }
            }
            g.s0 = first >= 0 ? (float)(in->t_min[first] - ta) : 0.f;
            g.ns = ns;
            g.ns_all = ns;
            g.inv_step = (float)(1.0 / step);
            segs.push_back(g);
            seg_knots.push_back({a[0], a[1], a[2], b[0], b[1], b[2]});
            // raster slices (Sec. 4): each instant's direction on the great
            // circle from a to b at its share of the segment's time
            sa::SamSegHost sh;
            for (int i = 0; i < 3; ++i) {
                sh.a[i] = a[i];
                sh.b[i] = b[i];
            }
            sh.ta = ta;
            sh.tb = tb;
            sh.first = first >= 0 ? first : 0;
            sh.ns = ns;
            sh.bin = bin;
            seg_host.push_back(sh);
            for (int s = sh.first; s < sh.first + ns; ++s) {
                const double f = (in->t_min[s] - ta) / (tb - ta);
                // sin(theta) = sn: a and b are unit vectors
                const double wa = std::sin((1.0 - f) * theta) / sn, wb = std::sin(f * theta) / sn;
                const double dd[3] = {wa * a[0] + wb * b[0], wa * a[1] + wb * b[1], wa * a[2] + wb * b[2]};
                sa::SamSlice &q = sam[s];
                std::memset(&q, 0, sizeof(q));
                q.dx = (float)dd[0];
                q.dy = (float)dd[1];
                q.dz = (float)dd[2];
                q.inv_da = (float)(1.0 / (dd[0] * a[0] + dd[1] * a[1] + dd[2] * a[2]));
                q.w = (float)in->weight[s];
            }
        }
    }
    bool merged = false;
    if (bound_deg > 0.0) {
        merge_segments(segs, seg_knots, bound_deg * M_PI / 180.0);
        merged = true;
    }
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    sa_path *p = new (std::nothrow) sa_path();
    if (!p) return fail(ctx, SA_ERR_OOM, "host allocation failed");
    p->ctx = ctx;
    p->device = ctx->device;
    p->d.n_days = D;
    p->d.n_samples = in->n_samples;
    p->d.n_segs = (int32_t)segs.size();
    p->d.n_bins = n_bins;
    if (merged) {
        // edges mix days: no per-day segment ranges
        day_seg_off.assign(1, 0);
    }
    day_seg_off.push_back((int32_t)segs.size());
    p->d.day_seg_off = std::move(day_seg_off);
    p->d.merged = merged;
    // each bin's segments one contiguous run, every bin with segments: the
    // accrual outputs can then be stored once per bin without clearing
    p->d.seg_bin.resize(segs.size());
    std::vector<char> seen(n_bins, 0);
    bool contiguous = true;
    for (size_t j = 0; j < segs.size(); ++j) {
        const int b = segs[j].bin;
        p->d.seg_bin[j] = b;
        if (j == 0 || segs[j - 1].bin != b) {
            if (seen[b]) contiguous = false;
            seen[b] = 1;
        }
    }
    for (int b = 0; b < n_bins; ++b) contiguous = contiguous && seen[b];
    p->d.bins_contiguous = contiguous;
    for (size_t j = 0; j < segs.size(); ++j)
        if (j == 0 || segs[j - 1].bin != segs[j].bin) {
            p->d.seg_runs.start.push_back((int32_t)j);
            p->d.seg_runs.bin.push_back(segs[j].bin);
        }
    p->d.seg_runs.start.push_back((int32_t)segs.size());
    for (size_t k = 0; k < samples.size(); ++k) {
        const int b = (int)(samples[k].tag & sa::kBinMask);
        if (k == 0 || (int)(samples[k - 1].tag & sa::kBinMask) != b) {
            p->d.sample_runs.start.push_back((int32_t)k);
            p->d.sample_runs.bin.push_back(b);
        }
    }
    p->d.sample_runs.start.push_back((int32_t)samples.size());
    if (!merged) {
        p->d.seg_host = std::move(seg_host);
        p->d.sample_t.assign(in->t_min, in->t_min + in->n_samples);
        p->d.sample_w.assign(in->weight, in->weight + in->n_samples);
    }
    bin_span.resize(n_bins, 0.0);
    p->d.bin_span = std::move(bin_span);
    p->d.words = (in->n_samples + 31) / 32;
    hipError_t e = hipSuccess;
    if (!samples.empty()) {
        e = hipMalloc((void **)&p->d.samples, sizeof(sa::SampleConst) * samples.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d.samples, samples.data(), sizeof(sa::SampleConst) * samples.size(),
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !merged && !sam.empty()) {
        e = hipMalloc((void **)&p->d.sam_slices, sizeof(sa::SamSlice) * sam.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d.sam_slices, sam.data(), sizeof(sa::SamSlice) * sam.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && !segs.empty()) {
        e = hipMalloc((void **)&p->d.segs, sizeof(sa::SegConst) * segs.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d.segs, segs.data(), sizeof(sa::SegConst) * segs.size(), hipMemcpyHostToDevice);
    }
    for (sa::BinRuns *R : {&p->d.seg_runs, &p->d.sample_runs}) {
        if (e != hipSuccess || R->start.size() < 2) continue;
        e = hipMalloc((void **)&R->dev, sizeof(int32_t) * R->start.size());
        if (e == hipSuccess)
            e = hipMemcpy(R->dev, R->start.data(), sizeof(int32_t) * R->start.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        sa_path_destroy(p);
        return hip_fail(ctx, e, "sa_path_upload");
    }
    *out = p;
    return SA_OK;
}

}  // namespace

extern "C" {

sa_status sa_path_upload(sa_ctx *ctx, const sa_sunpath_buf *in, sa_path **out)
{
    return path_upload(ctx, in, 0.0, out);
}

sa_status sa_path_upload_graph(sa_ctx *ctx, const sa_sunpath_buf *in, double bound_deg, sa_path **out)
{
    if (!(bound_deg >= 1e-6 && bound_deg <= 90.0))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_path_upload_graph: bound must be in [1e-6, 90] degrees");
    return path_upload(ctx, in, bound_deg, out);
}

sa_status sa_path_info(const sa_path *path, int32_t *n_bins, int32_t *n_samples, int32_t *n_segments)
{
    if (!path) return SA_ERR_INVALID_ARG;
    if (n_bins) *n_bins = path->d.n_bins;
    if (n_samples) *n_samples = path->d.n_samples;
    if (n_segments) *n_segments = path->d.n_segs;
    return SA_OK;
}

void sa_path_destroy(sa_path *path)
{
    if (!path) return;
    (void)hipSetDevice(path->device);
    (void)hipFree(path->d.samples);
    (void)hipFree(path->d.sam_slices);
    (void)hipFree(path->d.segs);
    (void)hipFree(path->d.seg_runs.dev);
    (void)hipFree(path->d.sample_runs.dev);
    delete path;
}

// ------------------------------------------------------------------ accumulate
static sa_status check_points(sa_ctx *ctx, const sa_points *pts)
{
    if (!pts || pts->n < 0 || (pts->n > 0 && (!pts->x || !pts->y || !pts->z)))
        return fail(ctx, SA_ERR_INVALID_ARG, "bad points");
    if (pts->n > (int64_t)INT32_MAX) return fail(ctx, SA_ERR_INVALID_ARG, "more than 2^31-1 points");
    return SA_OK;
}

static sa::PointsView view(const sa_points *p)
{
    return sa::PointsView{p->n, p->x, p->y, p->z, p->nx, p->ny, p->owner};
}

// Outputs are cleared with a fill kernel (not a memset node), so a call can
// be captured into a HIP graph and replayed.
static sa_status clear_outputs(sa_ctx *ctx, uint32_t flags, int64_t count, int32_t *counts, float *minutes,
                               float *longest = nullptr, double *minutes64 = nullptr)
{
    if (flags & SA_FLAG_ADD) return SA_OK;
    std::string err;
    sa_status rc = SA_OK;
    if (counts) rc = sa::fill_u32(counts, count, 0u, ctx->stream, err);
    if (rc == SA_OK && minutes) rc = sa::fill_u32(minutes, count, 0u, ctx->stream, err);
    if (rc == SA_OK && longest) rc = sa::fill_u32(longest, count, 0u, ctx->stream, err);
    if (rc == SA_OK && minutes64) rc = sa::fill_u32(minutes64, 2 * count, 0u, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "clear outputs: " + err);
    return SA_OK;
}

// The per-tile launch choices of a context.
static sa::TileLaunch tile_launch(const sa_ctx *ctx)
{
    return sa::TileLaunch{ctx->launch.accrual_segments_per_launch, ctx->launch.tile_grid_blocks, ctx->n_cu,
                          ctx->launch.accrual_waves_per_simd, ctx->launch.sampled_instants_per_packet};
}

// The accrual form stores each bin once (no clearing) unless asked to add
// or the path's bins interleave.
static bool accrual_stores(const sa_accum_opts *opts, const sa_path *path)
{
    return opts->mode == SA_ACCRUAL && !(opts->flags & SA_FLAG_ADD) && path->d.bins_contiguous;
}

sa_status sa_accumulate(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts, const sa_path *path,
                        const sa_accum_opts *opts, int32_t *counts, float *minutes, uint32_t *bits)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!scene || !path || !opts) return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate: null argument");
    sa_status rc = check_points(ctx, pts);
    if (rc != SA_OK) return rc;
    if (opts->mode != SA_SAMPLED && opts->mode != SA_ACCRUAL)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate: unknown mode");
    if (bits && opts->mode != SA_SAMPLED)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate: bit vectors exist for the sampled form only");
    if (opts->longest && opts->mode == SA_ACCRUAL && path->d.merged)
        return fail(ctx, SA_ERR_INVALID_ARG,
                    "sa_accumulate: a direction-graph path has no time order: no continuous shadow");
    if (opts->minutes64 && opts->mode != SA_ACCRUAL)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate: FP64 minutes exist for the accrual form only");
    if (!counts && !minutes && !bits && !opts->longest && !opts->minutes64) return SA_OK;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    const float scale = opts->out_scale == 0.f ? 1.f : opts->out_scale;
    const bool store = accrual_stores(opts, path);
    if (!store) {
        rc = clear_outputs(ctx, opts->flags, (int64_t)path->d.n_bins * pts->n, counts, minutes, opts->longest,
                           opts->minutes64);
        if (rc != SA_OK) return rc;
    }
    std::string err;
    if (opts->mode == SA_SAMPLED)
        rc = sa::launch_sampled(scene->d, path->d, view(pts), scale, counts, minutes, bits, opts->longest,
                                opts->work, tile_launch(ctx), ctx->spill.grab, ctx->stream, err);
    else
        rc = sa::launch_accrual(scene->d, path->d, view(pts), scale, counts, minutes, opts->minutes64,
                                opts->longest, opts->work, store, tile_launch(ctx), ctx->spill,
                                ctx->scratch_seg, ctx->scratch_piece, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_accumulate: " + err);
    return SA_OK;
}

sa_status sa_accumulate_noalloc(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts, const sa_path *path,
                                const sa_accum_opts *opts, int32_t *counts, float *minutes, uint32_t *bits)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!scene || !path || !opts) return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate_noalloc: null argument");
    sa_status rc = check_points(ctx, pts);
    if (rc != SA_OK) return rc;
    if (opts->mode != SA_SAMPLED && opts->mode != SA_ACCRUAL)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate_noalloc: unknown mode");
    if (bits && opts->mode != SA_SAMPLED)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate_noalloc: bit vectors exist for the sampled form only");
    if (opts->longest && opts->mode == SA_ACCRUAL && path->d.merged)
        return fail(ctx, SA_ERR_INVALID_ARG,
                    "sa_accumulate_noalloc: a direction-graph path has no time order: no continuous shadow");
    if (opts->minutes64 && opts->mode != SA_ACCRUAL)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate_noalloc: FP64 minutes exist for the accrual form only");
    if (!ctx->noalloc) return fail(ctx, SA_ERR_DEVICE, "sa_accumulate_noalloc: " + ctx->noalloc_err);
    if (!counts && !minutes && !bits && !opts->longest && !opts->minutes64) return SA_OK;
    if (opts->mode == SA_ACCRUAL && scene->d.n_b > 0 && path->d.n_segs > 0 && pts->n > 0) {
        // refuse before any work: a launch must hold one segment's views, and
        // with the continuous shadow a whole day's
        const int64_t per_seg = (int64_t)std::max(scene->d.n_nodes, 1) * (int64_t)sizeof(sa::SegNode);
        const int64_t cap = (int64_t)SA_NOALLOC_SCRATCH_BYTES / per_seg;
        int64_t need = 1;
        if (opts->longest)
            for (size_t d = 0; d + 1 < path->d.day_seg_off.size(); ++d)
                need = std::max<int64_t>(need, path->d.day_seg_off[d + 1] - path->d.day_seg_off[d]);
        if (need > cap)
            return fail(ctx, SA_ERR_CAPACITY,
                        "sa_accumulate_noalloc: " + std::to_string(need) + " segments of node views (" +
                            std::to_string(per_seg) + " bytes each) must fit the fixed scratch of " +
                            std::to_string((int64_t)SA_NOALLOC_SCRATCH_BYTES) + " bytes");
    }
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    const float scale = opts->out_scale == 0.f ? 1.f : opts->out_scale;
    const bool store = accrual_stores(opts, path);
    if (!store) {
        rc = clear_outputs(ctx, opts->flags, (int64_t)path->d.n_bins * pts->n, counts, minutes, opts->longest,
                           opts->minutes64);
        if (rc != SA_OK) return rc;
    }
    std::string err;
    if (opts->mode == SA_SAMPLED) {
        rc = sa::launch_sampled(scene->d, path->d, view(pts), scale, counts, minutes, bits, opts->longest,
                                opts->work, tile_launch(ctx), ctx->spill.grab, ctx->stream, err);
    } else {
        sa::Scratch fixed;
        fixed.ptr = ctx->noalloc;
        fixed.bytes = (size_t)SA_NOALLOC_SCRATCH_BYTES;
        fixed.fixed = true;
        sa::Scratch no_pieces;  // whole runs: nothing to allocate
        no_pieces.fixed = true;
        rc = sa::launch_accrual(scene->d, path->d, view(pts), scale, counts, minutes, opts->minutes64,
                                opts->longest, opts->work, store, tile_launch(ctx), ctx->spill,
                                fixed, no_pieces, ctx->stream, err);
    }
    if (rc != SA_OK) return fail(ctx, rc, "sa_accumulate_noalloc: " + err);
    return SA_OK;
}

sa_status sa_accumulate_batched(sa_ctx *ctx, const sa_scene *scene, int32_t n_var, int32_t ids_per_var,
                                const int32_t *var_ids, const float *var_h, const sa_points *pts,
                                const int64_t *var_off, const sa_path *path, const sa_accum_opts *opts,
                                int32_t *counts, float *minutes)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!scene || !path || !opts || n_var < 0 || ids_per_var < 0 || !var_off ||
        (n_var > 0 && ids_per_var > 0 && (!var_ids || !var_h)))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate_batched: bad arguments");
    if (opts->mode != SA_ACCRUAL) return fail(ctx, SA_ERR_INVALID_ARG, "sa_accumulate_batched: accrual form only");
    if (opts->longest || opts->minutes64)
        return fail(ctx, SA_ERR_INVALID_ARG,
                    "sa_accumulate_batched: continuous shadow and FP64 minutes are not offered here");
    sa_status rc = check_points(ctx, pts);
    if (rc != SA_OK) return rc;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    const float scale = opts->out_scale == 0.f ? 1.f : opts->out_scale;
    rc = clear_outputs(ctx, opts->flags, (int64_t)path->d.n_bins * pts->n, counts, minutes);
    if (rc != SA_OK) return rc;
    std::string err;
    const int32_t grid = opts->grid_blocks > 0 ? opts->grid_blocks : ctx->launch.batched_grid_blocks;
    rc = sa::launch_batched(scene->d, path->d, n_var, ids_per_var, var_ids, var_h, view(pts), var_off, scale,
                            counts, minutes, grid, ctx->launch.batched_tiles_per_grab, ctx->spill.counters + 2,
                            ctx->scratch_batched, ctx->scratch_seg, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_accumulate_batched: " + err);
    return SA_OK;
}

sa_status sa_grad_heights(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts, const sa_path *path,
                          const sa_accum_opts *opts, const float *dl_dmin, float *grad)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!scene || !path || !grad) return fail(ctx, SA_ERR_INVALID_ARG, "sa_grad_heights: null argument");
    if (opts && opts->mode != SA_ACCRUAL)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_grad_heights: the accrual form only (sampled counts are piecewise "
                                             "constant in the heights)");
    sa_status rc = check_points(ctx, pts);
    if (rc != SA_OK) return rc;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    const float scale = (!opts || opts->out_scale == 0.f) ? 1.f : opts->out_scale;
    const bool add = opts && (opts->flags & SA_FLAG_ADD);
    std::string err;
    rc = sa::launch_grad(scene->d, path->d, view(pts), dl_dmin, scale, add, grad, tile_launch(ctx), ctx->spill,
                         ctx->scratch_seg, ctx->scratch_grad, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_grad_heights: " + err);
    return SA_OK;
}

sa_status sa_region_sum(sa_ctx *ctx, const float *values, int64_t n, const int64_t *region_off, int32_t n_reg,
                        const float *area, double *out)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (n < 0 || n_reg < 0 || (n_reg > 0 && (!region_off || !out)) || (n > 0 && !values))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_region_sum: bad arguments");
    if (n_reg == 0) return SA_OK;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    std::string err;
    sa_status rc = sa::launch_region_sum(values, 1, n, nullptr, region_off, n_reg, area, out, ctx->scratch,
                                         ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_region_sum: " + err);
    return SA_OK;
}

sa_status sa_region_score(sa_ctx *ctx, const sa_path *path, const float *values, int64_t n,
                          const double *interval_weight, const int64_t *region_off, int32_t n_reg, const float *area,
                          double *out)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!path || n < 0 || n_reg < 0 || !interval_weight || (n_reg > 0 && (!region_off || !out)) ||
        (n > 0 && !values))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_region_score: bad arguments");
    if (n_reg == 0) return SA_OK;
    const int32_t n_bins = path->d.n_bins;
    if (n_bins < 1) return fail(ctx, SA_ERR_INVALID_ARG, "sa_region_score: the path has no bins");
    // each interval's weight per minute of its daylight: the score takes the
    // fraction of the interval's daylight spent in shadow (Sec. 7.2)
    std::vector<double> w(n_bins);
    for (int32_t b = 0; b < n_bins; ++b) {
        const double span = path->d.bin_span[b];
        if (!std::isfinite(interval_weight[b]) || !(span > 0.0))
            return fail(ctx, SA_ERR_INVALID_ARG, "sa_region_score: bad weight or a bin without daylight");
        w[b] = interval_weight[b] / span;
    }
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    const size_t need = sizeof(double) * (size_t)n_bins;
    if (ctx->scratch_w.bytes < need) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->scratch_w.ptr);
        ctx->scratch_w.ptr = nullptr;
        ctx->scratch_w.bytes = 0;
        hipError_t e = hipMalloc(&ctx->scratch_w.ptr, need);
        if (e != hipSuccess) {
            ctx->scratch_w.ptr = nullptr;
            return hip_fail(ctx, e, "sa_region_score: weights");
        }
        ctx->scratch_w.bytes = need;
    }
    // the weights go with the work on the stream (the host vector is gone
    // by the time the copy runs, so copy synchronously first)
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = hipMemcpy(ctx->scratch_w.ptr, w.data(), need, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "sa_region_score: weights");
    std::string err;
    sa_status rc = sa::launch_region_sum(values, n_bins, n, (const double *)ctx->scratch_w.ptr, region_off, n_reg,
                                         area, out, ctx->scratch, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_region_score: " + err);
    return SA_OK;
}

sa_status sa_path_bin_span(const sa_path *path, double *span)
{
    if (!path || !span) return SA_ERR_INVALID_ARG;
    for (int b = 0; b < path->d.n_bins; ++b) span[b] = path->d.bin_span[b];
    return SA_OK;
}

sa_status sa_building_contribution(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts, const sa_path *path,
                                   const float *weight, double *contrib)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!scene || !path || !contrib) return fail(ctx, SA_ERR_INVALID_ARG, "sa_building_contribution: null argument");
    sa_status rc = check_points(ctx, pts);
    if (rc != SA_OK) return rc;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    std::string err;
    rc = sa::fill_u32(contrib, 2 * (int64_t)path->d.n_bins * scene->d.n_b, 0u, ctx->stream, err);
    if (rc == SA_OK)
        rc = sa::launch_contribution(scene->d, path->d, view(pts), weight, contrib, tile_launch(ctx), ctx->spill.grab,
                                     ctx->scratch_seg, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, "sa_building_contribution: " + err);
    return SA_OK;
}

sa_status sa_sam_accumulate(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts, const sa_path *path,
                            const sa_sam_opts *opts, int32_t *counts, float *minutes)
{
    if (!ctx) return SA_ERR_INVALID_ARG;
    if (!scene || !path || !opts) return fail(ctx, SA_ERR_INVALID_ARG, "sa_sam_accumulate: null argument");
    sa_status rc = check_points(ctx, pts);
    if (rc != SA_OK) return rc;
    if (pts->owner || pts->nx || pts->ny)
        return fail(ctx, SA_ERR_INVALID_ARG,
                    "sa_sam_accumulate: ground-type points only (no owner or facade normal arrays)");
    if (!(opts->texel_m > 0.f) || !(opts->bias_m >= 0.f) || !std::isfinite(opts->texel_m) ||
        !std::isfinite(opts->bias_m))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_sam_accumulate: texel must be > 0 and bias >= 0");
    if (path->d.merged)
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_sam_accumulate: a direction-graph path has no instants per segment");
    double box[6];
    bool given = false;
    for (int i = 0; i < 6; ++i) {
        box[i] = opts->box[i];
        given = given || opts->box[i] != 0.f;
    }
    if (!given) {
        box[0] = scene->d.bounds[0];
        box[1] = scene->d.bounds[1];
        box[2] = 0.0;
        box[3] = scene->d.bounds[2];
        box[4] = scene->d.bounds[3];
        box[5] = scene_max_height(scene);
    }
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(box[i])) return fail(ctx, SA_ERR_INVALID_ARG, "sa_sam_accumulate: box not finite");
    if (!(box[3] >= box[0] && box[4] >= box[1] && box[5] >= box[2]))
        return fail(ctx, SA_ERR_INVALID_ARG, "sa_sam_accumulate: empty box");
    if (!counts && !minutes) return SA_OK;
    if (!set_device(ctx)) return fail(ctx, SA_ERR_DEVICE, "hipSetDevice failed");
    rc = clear_outputs(ctx, opts->flags, (int64_t)path->d.n_bins * pts->n, counts, minutes);
    if (rc != SA_OK) return rc;
    const float scale = opts->out_scale == 0.f ? 1.f : opts->out_scale;
    const int64_t cap = opts->max_texels > 0 ? opts->max_texels : (int64_t)1 << 31;
    std::string err;
    rc = sa::launch_sam(scene->d, path->d, view(pts), opts->texel_m, opts->bias_m, box, cap, scale, counts, minutes,
                        ctx->scratch_sam, ctx->sam_stamp, ctx->stream, err);
    if (rc != SA_OK) return fail(ctx, rc, err);
    return SA_OK;
}

}  // extern "C"
