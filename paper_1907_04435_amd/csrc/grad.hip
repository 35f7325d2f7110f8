// Adjoint of the accrual form with respect to building heights.
//
// The gross shadow of a point over a segment is the measure of the union of
// the occluders' angular intervals, times dt/theta.  Each boundary of that
// union is one end of one occluder's interval; when that end is a crossing
// of the clip line z = H (the ray grazing the roof edge), it moves with the
// height as d(angle)/dH = cross(c, c1 - c0) / (|c|^2 (z1 - z0)) (see
// prism_interval).  So
//     dL/dH_b = sum over points and segments of w * dt/theta *
//               (sum of d(close)/dH - sum of d(open)/dH)
// over the union boundaries owned by b.  The traversal is recomputed here,
// nothing is kept from the forward pass.  Contributions are summed across
// the wave per building and added with one FP64 atomic per building and
// wave into an accumulator (original building ids), which a last kernel
// rounds into the caller's float gradient.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sa_internal.h"
#include "traverse.h"
#include "unit_sched.h"

namespace sa {
namespace {
using namespace dev;

constexpr int kThreads = kSchedThreads;
constexpr int kWaves = kSchedWaves;
// Spill rounds: each refines a window 64-fold (three reach 1/262144 of a
// segment).
constexpr int kSpillRounds = 3;
constexpr int kSpillBlocks = 1024;

struct GradArgs {
    const float *dl;       // [n_bins * n] or null (all ones)
    double *acc;           // [n_b] FP64 accumulator, original ids
    const int32_t *order;  // hierarchy position -> original id
};

__device__ __forceinline__ void grad_segment(cSegNode *snodes, cint *voff, StackEntry *stack, cfloat4 *verts,
                                             cfloat *height, const SegConst &g, const LanePoint &q, bool active,
                                             float w0, float w1, UnionG &U, bool &ov)
{
    union_clear(U);
    ov = false;
    if (!active) return;
    float W0u, W0v, W1u, W1v;
    window_dirs(g, w0, w1, W0u, W0v, W1u, W1v);
    bool live = true;
    if (q.own >= 0) {
        float a, b;
        if (backface_interval(q.nx, q.ny, g, w0, w1, W0u, W0v, W1u, W1v, a, b)) {
            union_insert(U, a, b, -1, -1, 0.f, 0.f);
            live = !(a <= w0 && b >= w1);
        }
    }
    if (snodes == nullptr) return;
    uint64_t ovm = 0;
    auto leaf = [&](int prim, int voff, int m, uint64_t want) -> uint64_t {
        const uint64_t gm = want & ballot(prim != q.own);
        if (!gm) return 0;
        const bool go = lane_in(gm);
        float a = 0.f, b = 0.f, da = 0.f, db = 0.f;
        const int r = go ? prism_interval<true>(verts, voff, m, ld(height + prim), q.px, q.py, q.pz, g, w0, w1,
                                                W0u, W0v, W1u, W1v, a, b, da, db)
                         : 0;
        bool over = false, full = false;
        if (r) {
            over = !union_insert(U, a, b, prim, prim, da, db);
            // the whole window is shadowed: no boundary inside it
            full = !over && U.n == 1 && U.lo[0] <= w0 && U.hi[0] >= w1;
        }
        const uint64_t om = ballot(over);
        ovm |= om;
        return om | ballot(full);
    };
    const SegFan ft(g, q.px, q.py, q.pz);
    Work none{0, 0, 0, 0, 0, 0, 0};
    packet_traverse_seg<false>(snodes, voff, stack, ballot(live), ft, leaf, none);
    ov = lane_in(ovm);
}

// Add v into acc[order[prim]] for every lane with prim >= 0.  Lanes that
// hold the same building are summed across the wave first (a fixed
// butterfly order), then one lane issues a single FP64 atomic: one atomic
// per building and wave instead of one per lane.  Must be reached by every
// lane of the wave (the shuffles read all lanes).
__device__ __forceinline__ void wave_scatter(int prim, double v, const GradArgs &G)
{
    const int lane = tid() & 63;
    uint64_t pend = ballot(prim >= 0);
    while (pend) {
        const int lead = __builtin_ctzll(pend);
        const int key = __shfl(prim, lead, 64);
        const uint64_t m = pend & ballot(prim == key);
        double sum = lane_in(m) ? v : 0.0;
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (lane == lead) atomicAdd(&G.acc[G.order[key]], sum);
        pend &= ~m;
    }
}

// The union boundaries of one lane's window that move with a height:
// closing ends +, opening ends -, each times wscale; ok = false adds
// nothing (every lane of the wave must call this).
__device__ __forceinline__ void scatter_grad(const UnionG &U, bool ok, float wscale, const GradArgs &G)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const bool in = ok && r < U.n;
        wave_scatter(in && U.plo[r] >= 0 && U.dlo[r] != 0.f ? U.plo[r] : -1, -(double)(wscale * U.dlo[r]), G);
        wave_scatter(in && U.phi[r] >= 0 && U.dhi[r] != 0.f ? U.phi[r] : -1, (double)(wscale * U.dhi[r]), G);
    }
}

__device__ __forceinline__ bool roof_covered_g(cNode *nodes, StackEntry *stack, cfloat4 *verts, cfloat *height,
                                               const LanePoint &q, bool valid)
{
    if (nodes == nullptr) return false;
    uint64_t covm = 0;
    auto bt = [&](float x0, float y0, float x1, float y1, float z1) {
        return q.px >= x0 && q.px <= x1 && q.py >= y0 && q.py <= y1 && q.pz <= z1;
    };
    auto leaf = [&](int prim, int voff, int m, uint64_t want) -> uint64_t {
        const bool t = lane_in(want) && prim != q.own && q.pz <= ld(height + prim) &&
                       in_footprint(verts, voff, m, q.px, q.py);
        const uint64_t tm = ballot(t);
        covm |= tm;
        return tm;
    };
    auto key = [&](float, float, float, float, float) { return 0.f; };
    Work none{0, 0, 0, 0, 0, 0, 0};
    packet_traverse<false>(nodes, stack, ballot(valid), bt, leaf, key, none);
    return lane_in(covm);
}

// Seven waves per SIMD (72 VGPRs): 2 % faster than the six of the natural
// allocation.  Persistent: its units are (tile, chunk of segments), enough
// of them to keep every wave busy on small point sets (the gradient sums
// are atomic, so any split adds up the same).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_grad(
    const Node *nodes_g, const SegNode *snodes_g, int n_nodes, const int32_t *voff_g, const float4 *verts_g,
    const float *height_g, const SegConst *segs_g, int j0, int j1, Sched W, PointArgs P, GradArgs G, SpillArgs S)
{
    cNode *nodes = nodes_g ? (cNode *)nodes_g : nullptr;
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSeg *segs = (cSeg *)segs_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    __shared__ int s_W[sizeof(Sched) / 4];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    __shared__ int s_G[sizeof(GradArgs) / 4];
    __shared__ int s_S[sizeof(SpillArgs) / 4];
    if (tid() == 0) {
        lds_park((lds_int *)s_W, W);
        lds_park((lds_int *)s_P, P);
        lds_park((lds_int *)s_G, G);
        lds_park((lds_int *)s_S, S);
    }
    __syncthreads();
    StackEntry *stack = s_stack[tid() >> 6];
    const int lane = tid() & 63;
    int kx = 0;
    Unit un;
    while (next_unit((lds_int *)s_W, j0, j1, kx, un)) {
        const int ja = uniform(un.a), jb = uniform(un.b);
        const PointArgs Pd = lds_uniform<PointArgs>((lds_int *)s_P);
        const int64_t i = (int64_t)un.tile * 64 + lane;
        const bool valid = i < Pd.n;
        const LanePoint q = load_point(Pd, i, valid);
        const bool covered = roof_covered_g(nodes, stack, verts, height, q, valid);
        int bin = -1;
        float w = 0.f;
        for (int j = ja; j < jb; ++j) {
            const SegConst g = ld(segs + j);
            if (g.bin != bin) {
                bin = g.bin;
                const GradArgs Gd = lds_uniform<GradArgs>((lds_int *)s_G);
                w = (valid && Gd.dl) ? Gd.dl[(int64_t)bin * Pd.n + i] : 1.f;
            }
            UnionG U;
            bool ov;
            cSegNode *sn = snodes_g ? (cSegNode *)(snodes_g + (int64_t)(j - j0) * n_nodes) : nullptr;
            grad_segment(sn, (cint *)voff_g, stack, verts, height, g, q, valid && !covered && w != 0.f, 0.f, g.theta,
                         U, ov);
            scatter_grad(U, valid && !covered && !ov && w != 0.f, w * g.wrate, lds_uniform<GradArgs>((lds_int *)s_G));
            if (ballot(valid && ov))
                spill_push(lds_uniform<SpillArgs>((lds_int *)s_S), valid && ov, i, j, 0.f, g.theta);
        }
    }
}

// One spill round of the adjoint: as the accrual spill rounds, one wave per
// queued (point, segment, window), each lane one 64th of the window.  Ends
// clamped to a sub-window do not move with a height, so splitting adds no
// gradient terms.
__global__ __launch_bounds__(kThreads) void k_grad_spill(const SegNode *snodes_g, int n_nodes, int j0,
                                                         const int32_t *voff_g, const float4 *verts_g,
                                                         const float *height_g, const SegConst *segs_g, PointArgs P,
                                                         GradArgs G, const int4 *in, const uint32_t *in_count,
                                                         int32_t cap, SpillArgs S)
{
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSeg *segs = (cSeg *)segs_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    StackEntry *stack = s_stack[tid() >> 6];
    const int lane = tid() & 63;
    const int64_t total = min((int32_t)*in_count, cap);
    const int64_t stride = (int64_t)n_wg() * kWaves;
    for (int64_t e = (int64_t)wg_id() * kWaves + (tid() >> 6); e < total; e += stride) {
        const int4 en = in[e];
        const int64_t i = uniform(en.x);
        const int j = uniform(en.y);
        const float ew0 = __int_as_float(uniform(en.z)), ew1 = __int_as_float(uniform(en.w));
        const float d = (ew1 - ew0) * (1.f / 64.f);
        const float w0 = lane == 0 ? ew0 : fmaf((float)lane, d, ew0);
        const float w1 = lane == 63 ? ew1 : fmaf((float)(lane + 1), d, ew0);
        const LanePoint q = load_point(P, i, true);
        const SegConst g = ld(segs + j);
        const float w = G.dl ? G.dl[(int64_t)g.bin * P.n + i] : 1.f;
        UnionG U;
        bool ov;
        cSegNode *sn = snodes_g ? (cSegNode *)(snodes_g + (int64_t)(j - j0) * n_nodes) : nullptr;
        grad_segment(sn, (cint *)voff_g, stack, verts, height, g, q, true, w0, w1, U, ov);
        scatter_grad(U, !ov, w * g.wrate, G);
        spill_push(S, ov, i, j, w0, w1);
    }
}

__global__ void k_zero1(uint32_t *p) { *p = 0u; }

// grad[b] = (add ? grad[b] : 0) + scale * acc[b], rounded once to float.
__global__ void k_grad_out(const double *acc, int32_t n_b, double scale, int add, float *grad)
{
    const int b = wg_id() * wg_size() + tid();
    if (b < n_b) grad[b] = (float)((add ? (double)grad[b] : 0.0) + scale * acc[b]);
}

__global__ void k_spill_left(const uint32_t *count, uint32_t *overflow)
{
    if (*count) atomicOr(overflow, 2u);
}

}  // namespace

sa_status launch_grad(const DeviceScene &s, const DevicePath &p, const PointsView &pts, const float *dl, float scale,
                      bool add, float *grad, const TileLaunch &L, SpillQueue &q, Scratch &scr, Scratch &acc_scr,
                      hipStream_t st, std::string &err)
{
    if (s.n_b == 0) return SA_OK;
    const size_t need = sizeof(double) * (size_t)s.n_b;
    if (acc_scr.bytes < need) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(acc_scr.ptr);
        acc_scr.ptr = nullptr;
        acc_scr.bytes = 0;
        if (hipMalloc(&acc_scr.ptr, need) != hipSuccess) {
            (void)hipGetLastError();
            acc_scr.ptr = nullptr;
            err = "gradient accumulator allocation failed";
            return SA_ERR_OOM;
        }
        acc_scr.bytes = need;
    }
    double *acc = (double *)acc_scr.ptr;
    sa_status rc = fill_u32(acc, 2 * (int64_t)s.n_b, 0u, st, err);
    if (rc != SA_OK) return rc;
    int64_t tiles;
    if (!tile_count(pts.n, tiles, err)) return SA_ERR_INVALID_ARG;
    const int64_t res = resident_blocks(k_grad, L);
    const PointArgs P{pts.n, pts.x, pts.y, pts.z, pts.nx, pts.ny, pts.owner, s.rank, s.n_b};
    const GradArgs G{dl, acc, s.order};
    // segment ranges whose per-segment node views fit the budget, each
    // followed by its spill rounds
    const int64_t per = seg_views_cap(s, scr);
    for (int64_t j0 = 0; pts.n > 0 && j0 < p.n_segs; j0 += per) {
        const int j1 = (int)std::min<int64_t>(j0 + per, p.n_segs);
        SegNode *views;
        rc = build_seg_views(s, p, (int)j0, j1, s.n_nodes, scr, st, views, err);
        if (rc != SA_OK) return rc;
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, q.counters);
        SpillArgs S{q.entries[0], q.counters, q.counters + 2, q.capacity};
        const Sched W = plan_units(p.seg_runs, (int)j0, j1, tiles, Split::kChunks, res, q.grab);
        rc = fill_u32(q.grab, 8 * kGrabStride, 0u, st, err);
        if (rc != SA_OK) return rc;
        hipLaunchKernelGGL(k_grad, dim3((unsigned)unit_blocks(res, W)), dim3(kThreads), 0, st, s.nodes, views,
                           s.n_nodes, s.voff, s.verts, s.height, p.segs, (int)j0, j1, W, P, G, S);
        int cur = 0;
        for (int r = 0; r < kSpillRounds; ++r) {
            hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, q.counters + (cur ^ 1));
            SpillArgs S2{q.entries[cur ^ 1], q.counters + (cur ^ 1), q.counters + 2, q.capacity};
            hipLaunchKernelGGL(k_grad_spill, dim3(kSpillBlocks), dim3(kThreads), 0, st, views, s.n_nodes, (int)j0,
                               s.voff, s.verts, s.height, p.segs, P, G, (const int4 *)q.entries[cur],
                               (const uint32_t *)(q.counters + cur), q.capacity, S2);
            cur ^= 1;
        }
        hipLaunchKernelGGL(k_spill_left, dim3(1), dim3(1), 0, st, (const uint32_t *)(q.counters + cur),
                           q.counters + 2);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            err = std::string("gradient kernels: ") + hipGetErrorString(e);
            return SA_ERR_DEVICE;
        }
    }
    hipLaunchKernelGGL(k_grad_out, dim3((unsigned)((s.n_b + 255) / 256)), dim3(256), 0, st, (const double *)acc,
                       s.n_b, (double)scale, add ? 1 : 0, grad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("gradient output: ") + hipGetErrorString(e);
        return SA_ERR_DEVICE;
    }
    return SA_OK;
}

}  // namespace sa
