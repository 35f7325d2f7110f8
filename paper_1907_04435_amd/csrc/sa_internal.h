// Internal types shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "shadow_accrual.h"

namespace sa {

// The work-item index within its work-group and the work-group index, read
// straight from the registers the hardware fills at dispatch.  The
// runtime's own accessors (threadIdx, blockIdx) are calls into its device
// library in this build: that library keeps IEEE mode on and the kernels
// turn it off, so the calls are not inlined, and a call site makes the
// register allocator keep to the calling convention (the accrual kernel
// spilled two vector registers to scratch memory for it).
__device__ __forceinline__ unsigned tid() { return __builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ unsigned wg_id() { return __builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ unsigned wg_id_y() { return __builtin_amdgcn_workgroup_id_y(); }
// Work-items per work-group and work-groups in the grid (x), from the
// dispatch packet.
__device__ __forceinline__ unsigned wg_size() { return __builtin_amdgcn_workgroup_size_x(); }
__device__ __forceinline__ unsigned n_wg() { return __builtin_amdgcn_grid_size_x() / __builtin_amdgcn_workgroup_size_x(); }

// One interior node of the binary hierarchy: the boxes of both children
// (footprint-plane box x0,y0,x1,y1 and the top z1; every box starts at
// z = 0 because every prism stands on the ground) and the child
// references: >= 0 an interior node, < 0 the leaf ~prim (prism index in
// hierarchy order).  For leaf children the vertex range of the footprint
// is stored beside the reference so a leaf costs no extra indirection.
// 64 bytes: one scalar 16-dword load brings a whole node into SGPRs.
struct alignas(64) Node {
    float lx0, ly0, lx1, ly1;
    float rx0, ry0, rx1, ry1;
    float lz1, rz1;
    int32_t left, right;
    int32_t l_voff, l_m, r_voff, r_m;
};
static_assert(sizeof(Node) == 64, "node is one 64-byte line");

// Per sample instant, read uniformly by every lane of a wave.
struct alignas(32) SampleConst {
    float dx, dy, dz, w;  // unit direction toward the sun, weight (minutes)
    float ix, iy, iz;     // 1 / direction (components kept away from zero)
    int32_t tag;          // output bin | kDayStart on the first instant of a day
};
constexpr int32_t kDayStart = 1 << 30;
constexpr int32_t kBinMask = kDayStart - 1;

// Per great-circle segment of the accrual form.  In the segment's plane
// the direction at angle phi from the first knot is
// cos(phi) e1 + sin(phi) e2, phi in [0, theta], reached at time
// t = ta + dt * phi / theta.  An xy offset w from a point maps to the
// point of the plane above/below it, whose in-plane coordinates times
// |nz| (n = e1 x e2) are (u, v) = M w, and whose height above the point
// times |nz| is u * e1z + v * e2z (the factor keeps M bounded for planes
// through the zenith; directions are unchanged by it).
struct alignas(64) SegConst {
    float m00, m01, m10, m11;    // M (scaled by |nz|)
    float e1z, e2z, theta, dt;   // clip normal (u,v)->z, angle, minutes
    float ta;                    // start, minutes after local midnight
    float cth, sth;              // (cos theta, sin theta): end direction in (u, v)
    float nz;                    // vertical part of the plane normal e1 x e2
    int32_t mult;                // segments this one stands for (direction graph; else 1)
    int32_t ns_all;              // their sample instants
    int32_t bin;
    int32_t day;
    float e1x, e1y, e2x, e2y;    // horizontal parts of e1, e2 (facade back-face term)
    float ua_x, ua_y, ub_x, ub_y;  // horizontal offset per metre of rise, at both knots
    float s0;                    // first sample instant in the segment, minutes after ta
    float wrate;                 // minutes per radian the measure is weighted by: rate, or for a
                                 // direction-graph edge its segments' total duration / theta
    int32_t ns;                  // sample instants attributed to the segment
    int32_t steep;               // plane within 5 degrees of vertical: in-plane extreme search
    float rate;                  // dt / theta: minutes per radian
    float inv_step;              // 1 / step
    float mdx, mdy;              // horizontal part of the direction at theta / 2 (visit order)
};
static_assert(sizeof(SegConst) == 128, "two lines");

// A hierarchy node seen from one accrual segment: for each child, the box
// terms of the fan test against that segment (z1; the box edges shifted by
// the fan's per-metre reach: x1 - z1 umnx, x0 - z1 umxx, y1 - z1 umny,
// y0 - z1 umxy; the two wedge projections), children in the segment's
// visit order.  64 bytes, one scalar load.
struct alignas(64) SegNode {
    float c[2][7];
    int32_t ref[2];  // interior: byte offset of the child's view; leaf: ~prism; or absent
};
static_assert(sizeof(SegNode) == 64, "one line");

struct DeviceScene {
    int32_t n_b = 0;
    int32_t n_vert = 0;
    int32_t n_nodes = 0;
    int32_t depth = 0;
    float bounds[4] = {0, 0, 0, 0};
    float max_h = 0;
    Node *nodes = nullptr;       // [n_nodes]
    float4 *verts = nullptr;     // [n_vert] x, y, edge normal (ey, -ex) in hierarchy order
    int32_t *voff = nullptr;     // [n_b + 1] hierarchy order
    float *height = nullptr;     // [n_b] hierarchy order
    int32_t *order = nullptr;    // [n_b] hierarchy position -> original id
    int32_t *rank = nullptr;     // [n_b] original id -> hierarchy position
    int32_t *parent = nullptr;   // [n_nodes + n_b] parent*2+side of interior nodes then leaves
    int32_t *flags = nullptr;    // [n_nodes] refit arrival counters
    float4 *pbox = nullptr;      // [n_b] prism footprint boxes, hierarchy order
};

// Raster shadow accrual map (Sec. 4) of one segment: the shadow plane
// (normal a, the segment's start direction) and its texel grid, float32,
// every coordinate relative to the box centre o.
struct SamGrid {
    float ax, ay, az;  // plane normal
    float ux, uy, uz;  // in-plane basis, u horizontal
    float vx, vy, vz;
    float c;           // plane: (x - o).a = c
    float u0, v0;      // grid corner in (u, v)
    float h, inv_h;    // texel edge and its inverse
    int32_t nu, nv;    // texels along u and v
    float ox, oy, oz;  // o, world coordinates
    float bias;        // depth margin of the shadow test (m)
    float dq, inv_dq;  // depth quantum of the map words (m) and its inverse
};

// One slice: an instant's direction on the great circle between the
// segment's knots, 1 / (d.a) (distance along the light per distance from
// the plane), and the instant's minutes.
struct SamSlice {
    float dx, dy, dz, inv_da;
    float w;
    int32_t pad[3];
};

struct SamSegHost {
    double a[3], b[3];  // knot directions
    double ta, tb;      // knot times (local minutes)
    int32_t first, ns;  // its sample instants
    int32_t bin;
};

// Maximal runs of consecutive items (segments or instants) with the same
// output bin: where each starts (then the item count) and its bin, on the
// host, and the starts on the device.
struct BinRuns {
    std::vector<int32_t> start, bin;
    int32_t *dev = nullptr;
};

struct DevicePath {
    int32_t n_days = 0, n_samples = 0, n_segs = 0, n_bins = 0;
    SampleConst *samples = nullptr;  // [n_samples]
    SamSlice *sam_slices = nullptr;  // [n_samples] raster slices (unmerged paths)
    SegConst *segs = nullptr;        // [n_segs]
    int32_t words = 0;               // ceil(n_samples / 32)
    std::vector<int32_t> day_seg_off;  // host: first segment of each day, [n_days + 1]
    std::vector<int32_t> seg_bin;      // host: output bin of each segment
    bool bins_contiguous = false;      // host: every bin has segments, all in one run
    BinRuns seg_runs;                  // runs of equal bins over the segments
    BinRuns sample_runs;               // and over the instants
    std::vector<double> bin_span;      // host: daylight minutes of each output bin
    bool merged = false;               // host: segments merged into direction-graph edges
    // host, for the raster form: each segment's knot directions, times, its
    // instants [first, first + ns) and bin; every instant's time and weight
    std::vector<SamSegHost> seg_host;
    std::vector<double> sample_t, sample_w;
};

// Host-side builders implemented in the .hip sources.
sa_status scene_build(DeviceScene &s, hipStream_t st, int32_t n_b, const int32_t *voff,
                      const float *xy, const float *h, std::string &err);
sa_status scene_refit(DeviceScene &s, hipStream_t st, std::string &err);
// Heights from device arrays ids / h (original ids) into the scene, on the
// stream; an id out of range or a height that is not a positive finite
// number is skipped and raises bit 2 of *flag.
sa_status scene_set_heights_device(DeviceScene &s, int32_t n, const int32_t *ids, const float *h, uint32_t *flag,
                                   hipStream_t st, std::string &err);
void scene_free(DeviceScene &s);
sa_status sunpath_fill(const sa_site &site, const sa_timespan &span, sa_sunpath_buf &out,
                       std::string &err);

struct PointsView {
    int64_t n;
    const float *x, *y, *z, *nx, *ny;
    const int32_t *owner;
};

// Scratch owned by a context (grown on demand, freed with it), or a fixed
// buffer the library never grows or frees (fixed = true).
struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;
};

struct SpillQueue {
    int4 *entries[2] = {nullptr, nullptr};  // (point, segment, w0 bits, w1 bits)
    uint32_t *counters = nullptr;           // [0],[1] queue lengths, [2] overflow flag
    uint32_t *grab = nullptr;               // the accrual launch's work counters (eight, 128 B apart)
    int32_t capacity = 0;
};

// Launch choices of the per-tile kernels: the most segments one accrual
// launch covers (0: as many as the view budget allows) and the blocks of
// the persistent launches (0: as many as the device holds at once, from
// the kernel's occupancy and the device's compute units) and the accrual
// kernel's occupancy variant.
struct TileLaunch {
    int32_t segments_per_launch;
    int64_t grid_blocks;
    int32_t n_cu;
    int32_t waves_per_simd;  // the accrual kernel's occupancy variant: 6, 7 or 8 (0: 8)
    int32_t sampled_instants;  // instants per packet of the sampled form: 1, 2, 4, 8 or 16 (0: 8)
};

sa_status launch_sampled(const DeviceScene &s, const DevicePath &p, const PointsView &pts,
                         float scale, int32_t *counts, float *minutes, uint32_t *bits, float *longest,
                         uint64_t *work, const TileLaunch &L, uint32_t *grab, hipStream_t st,
                         std::string &err);
// store: outputs need no clearing (no SA_FLAG_ADD and p.bins_contiguous):
// each bin is stored by the launch holding its first segment.
// L: the launch choices (segments per launch, persistent grid size).
// piece_scr: per-piece sums when the tiles are too few to fill the device
// (grown on demand unless fixed; a fixed one of 0 bytes keeps whole runs).
sa_status launch_accrual(const DeviceScene &s, const DevicePath &p, const PointsView &pts,
                         float scale, int32_t *counts, float *minutes, double *minutes64, float *longest,
                         uint64_t *work, bool store, const TileLaunch &L, SpillQueue &q, Scratch &scr,
                         Scratch &piece_scr, hipStream_t st, std::string &err);
// grad = (add ? grad : 0) + scale * d(sum dl * minutes)/dH, accumulated in
// FP64 in acc (grown to n_b doubles as needed).
sa_status launch_grad(const DeviceScene &s, const DevicePath &p, const PointsView &pts,
                      const float *dl, float scale, bool add, float *grad, const TileLaunch &L, SpillQueue &q,
                      Scratch &scr, Scratch &acc, hipStream_t st, std::string &err);
sa_status launch_region_sum(const float *v, int n_bins, int64_t n, const double *bin_w,
                            const int64_t *off, int32_t n_reg, const float *area, double *out,
                            Scratch &scr, hipStream_t st, std::string &err);
// The FP32 FMA lane-op rate the device sustains (a roofline measurement aid).
sa_status measure_valu_peak(int n_cu, float *sink, int64_t sink_floats, hipStream_t st, double &lane_ops_per_s,
                            std::string &err);
sa_status launch_contribution(const DeviceScene &s, const DevicePath &p, const PointsView &pts,
                              const float *weight, double *contrib, const TileLaunch &L, uint32_t *grab,
                              Scratch &scr, hipStream_t st, std::string &err);
// Per-segment node views (SegNode) of segments [j0, j1) into scr (grown as
// needed, with the stream synchronised first; a fixed scr that is too small
// is a CAPACITY error), segment j's views at (j - j0) * stride; views =
// nullptr for an empty scene.  seg_views_cap: segments whose views fit the
// per-launch budget (a fixed scr: its size; 0 if not even one fits).
sa_status build_seg_views(const DeviceScene &s, const DevicePath &p, int j0, int j1, int64_t stride, Scratch &scr,
                          hipStream_t st, SegNode *&views, std::string &err);
int64_t seg_views_cap(const DeviceScene &s, const Scratch &scr);
// Gross shadow by raster shadow accrual maps (Sec. 4) into counts/minutes
// [n_bins * n] (already cleared): per segment a map of slices x nu x nv
// 64-bit words (stamp, depth) in scr (grown as needed; max_texels caps one
// segment's map); stamp: the last segment stamp written into scr, kept by
// the caller with scr.
sa_status launch_sam(const DeviceScene &s, const DevicePath &p, const PointsView &pts, double texel,
                     double bias, const double box[6], int64_t max_texels, float scale, int32_t *counts,
                     float *minutes, Scratch &scr, uint32_t &stamp, hipStream_t st, std::string &err);
sa_status launch_batched(const DeviceScene &s, const DevicePath &p, int32_t n_var, int32_t k,
                         const int32_t *ids, const float *h, const PointsView &pts,
                         const int64_t *var_off, float scale, int32_t *counts, float *minutes,
                         int32_t grid_blocks, int32_t grab, uint32_t *flag, Scratch &scr, Scratch &views_scr,
                         hipStream_t st, std::string &err);
// Graph-capturable fill of n 32-bit words.
sa_status fill_u32(void *p, int64_t n, uint32_t v, hipStream_t st, std::string &err);

}  // namespace sa
