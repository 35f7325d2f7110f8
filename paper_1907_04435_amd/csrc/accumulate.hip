// Gross-shadow kernels: the sampled form (one shadow ray per point per sun
// instant) and the accrual form (one occluded interval per occluder per
// point per great-circle segment, union, measure), plus the accrual spill
// rounds that finish the rare point-segments whose occluded set has more
// than four disjoint pieces by splitting their window 64 ways.
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
// Spill rounds: each refines a window 64-fold, so three rounds reach
// 1/262144 of a segment.
constexpr int kSpillRounds = 3;
constexpr int kSpillBlocks = 1024;
constexpr int64_t kChunkWork = 4000000000ll;  // point-segments per accrual launch
constexpr int64_t kSegNodeBytes = 256ll << 20;  // per-segment node views per accrual launch
constexpr int64_t kPieceBytes = 256ll << 20;    // per-piece sums of an accrual launch on few tiles

// Per-bin outputs of the accrual kernels.  A bin whose first segment lies in
// the launch is stored (no clear beforehand, no read); a bin continued from
// an earlier launch, or any bin under SA_FLAG_ADD, is added to.  Each
// (tile, bin) belongs to one unit, so the sums are deterministic.  With
// pieces (pcnt non-null) a unit holds one piece of a bin's run instead and
// writes its sums to its part's row of pcnt / pmin ([part][n]); a second
// kernel adds a bin's pieces in order into the outputs.
struct BinOut {
    int32_t *counts;
    float *minutes;
    double *minutes64;    // the FP64 lane sums behind minutes (optional)
    int32_t *pcnt;        // per-piece sums, or null
    double *pmin;
    int32_t fresh_first;  // the launch's first bin starts in it
    int32_t fresh_rest;   // the later bins of the launch start in it
    float scale;          // minutes are multiplied by this
    int32_t pad;
};

__device__ __forceinline__ void put_bin(const BinOut &O, int64_t o, bool fresh, int cnt, double mins)
{
    const double v = mins * O.scale;
    if (O.counts) O.counts[o] = (fresh ? 0 : O.counts[o]) + cnt;
    if (O.minutes) O.minutes[o] = (fresh ? 0.f : O.minutes[o]) + (float)v;
    if (O.minutes64) O.minutes64[o] = (fresh ? 0.0 : O.minutes64[o]) + v;
}

// ------------------------------------------------------------------ sampled
// Sum a per-lane counter over the wave and add it to a global total.
__device__ __forceinline__ void flush_work(const Work &w, uint64_t *work)
{
    uint32_t v[8] = {w.box, w.prism, w.edges, w.inserts, w.nodes, w.units, w.spills, w.leaves};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        uint64_t s = v[c];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if ((tid() & 63) == 0 && s) atomicAdd((unsigned long long *)&work[c], (unsigned long long)s);
    }
}

// Outputs of the sampled form (parked in LDS by the kernel).
struct SampOut {
    int32_t *counts;
    float *minutes;
    uint32_t *bits;
    float *longest;
    float scale;
    int32_t pad;
};

// Adds a unit's sums for one bin (outputs cleared beforehand; a bin of a
// tile belongs to one unit).
__device__ __forceinline__ void sampled_put(const SampOut &O, int64_t o, int cnt, float mins, float best)
{
    if (O.counts) O.counts[o] += cnt;
    if (O.minutes) O.minutes[o] += mins * O.scale;
    if (O.longest) O.longest[o] = fmaxf(O.longest[o], best * O.scale);
}

// The sampled form: an any-hit ray per (point, instant), in packets of
// 64 / kInst neighbouring points x kInst consecutive instants of one
// 64-point tile (kInst is a launch choice; 16 x 4 on the block scene).  A
// packet first takes the back-face test and the occluder cache: each wave
// remembers the prism that blocked the most lanes of its previous walk and
// tests it first; a blocked ray is blocked whichever prism is found first,
// so the predicate is unchanged.  The rays left go to a per-wave queue in
// LDS as (instant, point of the group), and a walk of the hierarchy runs
// whenever 64 are queued, and once more for the rest at the end of the
// point group.  A packet enters the queue with about four rays in five
// live (block scene: the rest face away from their facade or are blocked
// by the cached occluder), while every node visit costs the wave the same
// whatever its live lanes; refilled walks are full.  The queue fills in the
// order of the instants, so a walk holds the group's points at neighbouring
// instants.  Eight waves per SIMD (the compiler's own choice gives seven).
//
// k_sampled_q: counts and minutes of units that lie in one bin; a walk's
// hits add their instant's weight to their point's sum in LDS.
template <bool kCount, int kInst>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_sampled_q(
    const Node *nodes_g, const float4 *verts_g, const float *height_g, const SampleConst *samples_g, int K, Sched W,
    PointArgs P, SampOut O, uint64_t *work)
{
    static_assert(kInst >= 1 && kInst <= 16 && (kInst & (kInst - 1)) == 0, "instants per packet");
    constexpr int kPts = 64 / kInst;  // points per packet (a group)
    constexpr int kQueue = 128;       // < 64 waiting plus one packet
    Work wk{0, 0, 0, 0, 0, 0, 0};
    cNode *nodes = (cNode *)nodes_g;
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSample *samples = (cSample *)samples_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    __shared__ uint32_t s_queue[kWaves][kQueue];
    __shared__ int s_cnt[kWaves][kPts];
    __shared__ float s_min[kWaves][kPts];
    __shared__ int s_W[sizeof(Sched) / 4];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    __shared__ int s_O[sizeof(SampOut) / 4];
    if (tid() == 0) {
        lds_park((lds_int *)s_W, W);
        lds_park((lds_int *)s_P, P);
        lds_park((lds_int *)s_O, O);
    }
    __syncthreads();
    const int wave = tid() >> 6;
    StackEntry *stack = s_stack[wave];
    uint32_t *queue = s_queue[wave];
    int *g_cnt = s_cnt[wave];
    float *g_min = s_min[wave];
    const int lane = tid() & 63;
    const int slot = lane & (kInst - 1);  // the lane's instant within the packet
    int kx = 0;
    Unit un;
    while (next_unit((lds_int *)s_W, 0, K, kx, un)) {
        const int ka = uniform(un.a), kb = uniform(un.b);
        if (kb <= ka) continue;
        const int64_t n = lds_uniform<PointArgs>((lds_int *)s_P).n;
        const int bin = ld(samples + ka).tag & kBinMask;
        for (int g = 0; g < kInst; ++g) {
            const int64_t i0 = (int64_t)un.tile * 64 + g * kPts;  // the group's first point
            if (i0 >= n) break;
            if (lane < kPts) {
                g_cnt[lane] = 0;
                g_min[lane] = 0.f;
            }
            int c_prim = -1, c_voff = 0, c_m = 0;  // the occluder cache
            int queued = 0;
            // one walk over the first nq queued rays; lanes past nq idle
            auto walk = [&](int nq) {
                const bool on = lane < nq;
                const uint32_t e = on ? queue[lane] : 0u;
                const int pt = (int)(e & 63u);
                const SampleConst s = samples_g[on ? (int)(e >> 6) : ka];
                // the middle ray's direction orders the children
                const SampleConst sm = ld(samples + uniform((int)(queue[nq >> 1] >> 6)));
                const LanePoint q = load_point(lds_uniform<PointArgs>((lds_int *)s_P), i0 + pt, on);
                uint64_t hitm = 0;
                int b_prim = -1, b_voff = 0, b_m = 0, b_cnt = 0;
                const float ox = -q.px * s.ix, oy = -q.py * s.iy, oz = -q.pz * s.iz;
                auto bt = [&](float x0, float y0, float x1, float y1, float z1) {
                    const float ax = fmaf(x0, s.ix, ox), bx = fmaf(x1, s.ix, ox);
                    const float ay = fmaf(y0, s.iy, oy), by = fmaf(y1, s.iy, oy);
                    const float tfz = fmaf(z1, s.iz, oz);
                    const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), 0.f);
                    const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), tfz);
                    return le_mask(tn, tf);
                };
                auto leaf = [&](int prim, int voff, int m, uint64_t want) -> uint64_t {
                    const bool go = lane_in(want & ballot(prim != q.own));
                    if constexpr (kCount) {
                        wk.prism += go ? 1u : 0u;
                        wk.edges += go ? (uint32_t)m : 0u;
                        wk.leaves += first_active_lane() ? 1u : 0u;
                    }
                    const bool t =
                        go & ray_prism(verts, voff, m, ld(height + prim), q.px, q.py, q.pz, s.dx, s.dy, s.dz);
                    const uint64_t tm = ballot(t);
                    hitm |= tm;
                    const int cn = __builtin_popcountll(tm);
                    if (cn > b_cnt) {
                        b_cnt = cn;
                        b_prim = prim;
                        b_voff = voff;
                        b_m = m;
                    }
                    return tm;  // a blocked ray needs no further test
                };
                auto key = [&](float x0, float y0, float x1, float y1, float z1) {
                    return fmaf(x0 + x1, sm.dx, fmaf(y0 + y1, sm.dy, z1 * sm.dz));
                };
                packet_traverse<kCount>(nodes, stack, ballot(on), bt, leaf, key, wk);
                c_prim = uniform(b_cnt > 0 ? b_prim : -1);
                c_voff = uniform(b_voff);
                c_m = uniform(b_m);
                if (lane_in(hitm)) {
                    atomicAdd(&g_cnt[pt], 1);
                    atomicAdd(&g_min[pt], s.w);
                }
            };
            const int64_t i = i0 + lane / kInst;
            const bool pvalid = i < n;
            const LanePoint q = load_point(lds_uniform<PointArgs>((lds_int *)s_P), pvalid ? i : 0, pvalid);
            int cnt = 0;  // this lane's instants settled before any walk
            float mins = 0.f;
            for (int c0 = ka; c0 < kb; c0 += kInst) {
                const int k = c0 + slot;
                const bool valid = pvalid && k < kb;
                const SampleConst s = samples_g[k < kb ? k : ka];
                const bool back = q.own >= 0 && fmaf(q.nx, s.dx, q.ny * s.dy) <= 0.f;
                uint64_t live = ballot(valid && !back);
                uint64_t cached = 0;
                if (nodes_g != nullptr && c_prim >= 0 && live) {
                    const bool go = lane_in(live & ballot(c_prim != q.own));
                    if constexpr (kCount) {
                        wk.prism += go ? 1u : 0u;
                        wk.edges += go ? (uint32_t)c_m : 0u;
                        wk.leaves += first_active_lane() ? 1u : 0u;
                    }
                    cached = ballot(go & ray_prism(verts, c_voff, c_m, ld(height + c_prim), q.px, q.py, q.pz, s.dx,
                                                   s.dy, s.dz));
                    live &= ~cached;
                }
                if constexpr (kCount) wk.units += valid ? 1u : 0u;
                const bool sh = valid && (back || lane_in(cached));
                cnt += sh ? 1 : 0;
                mins += sh ? s.w : 0.f;
                if (nodes_g != nullptr && live) {
                    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0u));
                    if (lane_in(live)) queue[queued + rank] = ((uint32_t)k << 6) | (uint32_t)(lane / kInst);
                    queued += __builtin_popcountll(live);
                    if (queued >= 64) {
                        walk(64);
                        // the rest (fewer than 64) to the front
                        const bool more = 64 + lane < queued;
                        const uint32_t e = more ? queue[64 + lane] : 0u;
                        if (more) queue[lane] = e;
                        queued -= 64;
                    }
                }
            }
            if (queued > 0) walk(queued);
            // the point's lanes together, then its walks' hits
            for (int o = 1; o < kInst; o <<= 1) {
                cnt += __shfl_xor(cnt, o, 64);
                mins += __shfl_xor(mins, o, 64);
            }
            if (slot == 0 && pvalid) {
                const int pt = lane / kInst;
                sampled_put(lds_uniform<SampOut>((lds_int *)s_O), (int64_t)bin * n + i, cnt + g_cnt[pt],
                            mins + g_min[pt], 0.f);
            }
        }
    }
    if constexpr (kCount) flush_work(wk, work);
}

// k_sampled_qb: the outputs that need every instant's result -- bit
// vectors, the continuous shadow (in time order), and bins that interleave
// (a unit then spans them).  The instants of a unit go in windows of kWin
// (a 2 KB bitmap per wave: 256 instants for 64 points, up to 4096 for 4):
// each window's packets and walks set their shadowed (point, instant)
// pairs in a per-wave LDS bitmap, the queue is drained at the window's
// end, and each point's lane then replays the window's bits in time order:
// counts, minutes and runs per bin, a run reset at each day's first instant
// (runs never cross days) and the longest kept per bin.  A queue entry
// holds the instant's offset in the window, so any path length fits.  With
// bit vectors a unit is a whole tile from the first instant, so windows
// start on 32-instant words and the bitmap words are the output words.
template <bool kCount, int kInst>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_sampled_qb(
    const Node *nodes_g, const float4 *verts_g, const float *height_g, const SampleConst *samples_g, int K, Sched W,
    PointArgs P, SampOut O, uint64_t *work)
{
    static_assert(kInst >= 1 && kInst <= 16 && (kInst & (kInst - 1)) == 0, "instants per packet");
    constexpr int kPts = 64 / kInst;  // points per packet (a group)
    constexpr int kQueue = 128;       // < 64 waiting plus one packet
    constexpr int kWords = 512 / kPts;  // bitmap words per point and window (2 KB a wave)
    constexpr int kWin = 32 * kWords;   // instants per window
    constexpr int kRow = kWords + 1;    // a point's row, padded: lanes reading one word of
                                        // consecutive points hit different banks
    Work wk{0, 0, 0, 0, 0, 0, 0};
    cNode *nodes = (cNode *)nodes_g;
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSample *samples = (cSample *)samples_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    __shared__ uint32_t s_queue[kWaves][kQueue];
    __shared__ uint32_t s_map[kWaves][kPts * kRow];
    __shared__ int s_W[sizeof(Sched) / 4];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    __shared__ int s_O[sizeof(SampOut) / 4];
    if (tid() == 0) {
        lds_park((lds_int *)s_W, W);
        lds_park((lds_int *)s_P, P);
        lds_park((lds_int *)s_O, O);
    }
    __syncthreads();
    const int wave = tid() >> 6;
    StackEntry *stack = s_stack[wave];
    uint32_t *queue = s_queue[wave];
    uint32_t *map = s_map[wave];
    const int lane = tid() & 63;
    const int slot = lane & (kInst - 1);  // the lane's instant within the packet
    int kx = 0;
    Unit un;
    while (next_unit((lds_int *)s_W, 0, K, kx, un)) {
        const int ka = uniform(un.a), kb = uniform(un.b);
        if (kb <= ka) continue;
        const int64_t n = lds_uniform<PointArgs>((lds_int *)s_P).n;
        for (int g = 0; g < kInst; ++g) {
            const int64_t i0 = (int64_t)un.tile * 64 + g * kPts;  // the group's first point
            if (i0 >= n) break;
            const int64_t i = i0 + lane / kInst;
            const bool pvalid = i < n;
            const LanePoint q = load_point(lds_uniform<PointArgs>((lds_int *)s_P), pvalid ? i : 0, pvalid);
            // replay state of point `lane` of the group (lanes < kPts)
            const bool rvalid = lane < kPts && i0 + lane < n;
            int cnt = 0;
            float mins = 0.f, run = 0.f, best = 0.f;
            int bin = ld(samples + ka).tag & kBinMask;
            int c_prim = -1, c_voff = 0, c_m = 0;  // the occluder cache
            for (int w0 = ka; w0 < kb; w0 += kWin) {
                const int w1 = min(w0 + kWin, kb);
                for (int t = lane; t < kPts * kRow; t += 64) map[t] = 0u;
                int queued = 0;
                // one walk over the first nq queued rays; lanes past nq idle
                auto walk = [&](int nq) {
                    const bool on = lane < nq;
                    const uint32_t e = on ? queue[lane] : 0u;
                    const int pt = (int)(e & 63u), j = (int)(e >> 6);
                    const SampleConst s = samples_g[on ? w0 + j : ka];
                    // the middle ray's direction orders the children
                    const SampleConst sm = ld(samples + w0 + uniform((int)(queue[nq >> 1] >> 6)));
                    const LanePoint qw = load_point(lds_uniform<PointArgs>((lds_int *)s_P), i0 + pt, on);
                    uint64_t hitm = 0;
                    int b_prim = -1, b_voff = 0, b_m = 0, b_cnt = 0;
                    const float ox = -qw.px * s.ix, oy = -qw.py * s.iy, oz = -qw.pz * s.iz;
                    auto bt = [&](float x0, float y0, float x1, float y1, float z1) {
                        const float ax = fmaf(x0, s.ix, ox), bx = fmaf(x1, s.ix, ox);
                        const float ay = fmaf(y0, s.iy, oy), by = fmaf(y1, s.iy, oy);
                        const float tfz = fmaf(z1, s.iz, oz);
                        const float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), 0.f);
                        const float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), tfz);
                        return le_mask(tn, tf);
                    };
                    auto leaf = [&](int prim, int voff, int m, uint64_t want) -> uint64_t {
                        const bool go = lane_in(want & ballot(prim != qw.own));
                        if constexpr (kCount) {
                            wk.prism += go ? 1u : 0u;
                            wk.edges += go ? (uint32_t)m : 0u;
                            wk.leaves += first_active_lane() ? 1u : 0u;
                        }
                        const bool t = go & ray_prism(verts, voff, m, ld(height + prim), qw.px, qw.py, qw.pz, s.dx,
                                                      s.dy, s.dz);
                        const uint64_t tm = ballot(t);
                        hitm |= tm;
                        const int cn = __builtin_popcountll(tm);
                        if (cn > b_cnt) {
                            b_cnt = cn;
                            b_prim = prim;
                            b_voff = voff;
                            b_m = m;
                        }
                        return tm;  // a blocked ray needs no further test
                    };
                    auto key = [&](float x0, float y0, float x1, float y1, float z1) {
                        return fmaf(x0 + x1, sm.dx, fmaf(y0 + y1, sm.dy, z1 * sm.dz));
                    };
                    packet_traverse<kCount>(nodes, stack, ballot(on), bt, leaf, key, wk);
                    c_prim = uniform(b_cnt > 0 ? b_prim : -1);
                    c_voff = uniform(b_voff);
                    c_m = uniform(b_m);
                    if (lane_in(hitm)) atomicOr(&map[pt * kRow + (j >> 5)], 1u << (j & 31));
                };
                for (int c0 = w0; c0 < w1; c0 += kInst) {
                    const int k = c0 + slot;
                    const bool valid = pvalid && k < w1;
                    const SampleConst s = samples_g[k < w1 ? k : ka];
                    const bool back = q.own >= 0 && fmaf(q.nx, s.dx, q.ny * s.dy) <= 0.f;
                    uint64_t live = ballot(valid && !back);
                    uint64_t cached = 0;
                    if (nodes_g != nullptr && c_prim >= 0 && live) {
                        const bool go = lane_in(live & ballot(c_prim != q.own));
                        if constexpr (kCount) {
                            wk.prism += go ? 1u : 0u;
                            wk.edges += go ? (uint32_t)c_m : 0u;
                            wk.leaves += first_active_lane() ? 1u : 0u;
                        }
                        cached = ballot(go & ray_prism(verts, c_voff, c_m, ld(height + c_prim), q.px, q.py, q.pz,
                                                       s.dx, s.dy, s.dz));
                        live &= ~cached;
                    }
                    if constexpr (kCount) wk.units += valid ? 1u : 0u;
                    const int pt = lane / kInst, j = k - w0;
                    if (valid && (back || lane_in(cached))) atomicOr(&map[pt * kRow + (j >> 5)], 1u << (j & 31));
                    if (nodes_g != nullptr && live) {
                        const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0u));
                        if (lane_in(live)) queue[queued + rank] = ((uint32_t)j << 6) | (uint32_t)pt;
                        queued += __builtin_popcountll(live);
                        if (queued >= 64) {
                            walk(64);
                            // the rest (fewer than 64) to the front
                            const bool more = 64 + lane < queued;
                            const uint32_t e = more ? queue[64 + lane] : 0u;
                            if (more) queue[lane] = e;
                            queued -= 64;
                        }
                    }
                }
                if (queued > 0) walk(queued);
                // the window's bitmap words are the output words
                uint32_t *bits = lds_uniform<SampOut>((lds_int *)s_O).bits;
                if (bits != nullptr)
                    for (int t = lane; t < kPts * kWords; t += 64) {
                        const int wd = t / kPts, p = t - wd * kPts;  // consecutive lanes: consecutive points
                        if (i0 + p < n && w0 + 32 * wd < w1)
                            bits[(int64_t)((w0 >> 5) + wd) * n + i0 + p] = map[p * kRow + wd];
                    }
                // replay in time order, one point per lane
                for (int wd = 0; wd < kWords && w0 + 32 * wd < w1; ++wd) {
                    const uint32_t word = rvalid ? map[lane * kRow + wd] : 0u;
                    const int jb = min(32, w1 - w0 - 32 * wd);
                    for (int b = 0; b < jb; ++b) {
                        const SampleConst sj = ld(samples + (w0 + 32 * wd + b));
                        const int sbin = sj.tag & kBinMask;
                        if (sbin != bin) {
                            if (rvalid)
                                sampled_put(lds_uniform<SampOut>((lds_int *)s_O), (int64_t)bin * n + i0 + lane, cnt,
                                            mins, best);
                            cnt = 0;
                            mins = 0.f;
                            best = 0.f;
                            bin = sbin;
                        }
                        if (sj.tag & kDayStart) run = 0.f;
                        const bool sh = (word >> b) & 1u;
                        cnt += sh ? 1 : 0;
                        mins += sh ? sj.w : 0.f;
                        run = sh ? run + sj.w : 0.f;
                        best = fmaxf(best, run);
                    }
                }
            }
            if (rvalid) sampled_put(lds_uniform<SampOut>((lds_int *)s_O), (int64_t)bin * n + i0 + lane, cnt, mins, best);
        }
    }
    if constexpr (kCount) flush_work(wk, work);
}

// ------------------------------------------------------------------ accrual
// Segment j's constants read again where they are used after a traversal
// rather than held in registers across it (an opaque copy of the index
// keeps the compiler from reusing the first load): a scalar-cache hit
// costs less than spilling them to lanes of a vector register.
__device__ __forceinline__ SegConst reload(cSeg *segs, int j)
{
    int jr = j;
    asm volatile("" : "+s"(jr));
    return ld(segs + jr);
}

// Measure and sample count of the occluded set of one point over the
// window [w0, w1] of segment g.  `last_window` says whether w1 is the end
// of the segment (instants at the window end belong to the next window
// otherwise).
__device__ __forceinline__ void measure(const Union4 &U, const SegConst &g, float w0, float w1,
                                        bool last_window, double &mins, int &cnt)
{
    const float scale = g.rate;
    float m = 0.f;
    int c = 0;
    const float inv_step = g.inv_step;
    int kmax = g.ns - 1;
    if (!last_window) kmax = min(kmax, (int)ceilf((w1 * scale - g.s0) * inv_step) - 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r < U.n) {
            m += U.hi[r] - U.lo[r];
            const int klo = max((int)ceilf((U.lo[r] * scale - g.s0) * inv_step), 0);
            // a set that reaches the window end holds the window's last
            // instant: taken as is, not through the rounding of w1 * scale
            const int khi = U.hi[r] >= w1 ? kmax : min((int)floorf((U.hi[r] * scale - g.s0) * inv_step), kmax);
            c += max(khi - klo + 1, 0);
        }
    }
    mins += (double)(m * g.wrate);
    cnt += c * g.mult;
}

// The occluded set of every live lane's point over its window of segment g:
// back-face term, then the packet fan traversal.  On return `ov` marks
// lanes whose set needed more than four pieces.
// The hierarchy as seen from the current segment: its per-segment node
// views (SegFan: seven compares per child), the vertex offsets of the
// leaves, and the view the walk starts at.
struct SegSrc {
    cSegNode *nodes;
    cint *voff;
    int root;  // byte offset of the root's view
};

template <bool kCount>
__device__ __forceinline__ void accrue_segment(SegSrc src, StackEntry *stack, cfloat4 *verts, cfloat *height,
                                               const SegConst &g, const LanePoint &q, bool active, float w0,
                                               float w1, Union4 &U, bool &ov, Work &wk)
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
            union_insert(U, a, b);
            live = !(a <= w0 && b >= w1);
        }
    }
    if (src.nodes == nullptr) return;
    // liveness and overflow as wave masks (see packet_traverse)
    uint64_t ovm = 0;
    auto leaf_m = [&](int prim, int voff, int m, uint64_t want) -> uint64_t {
        const uint64_t gm = want & ballot(prim != q.own);
        if (!gm) return 0;
        const bool go = lane_in(gm);
        if constexpr (kCount) {
            wk.prism += go ? 1u : 0u;
            wk.edges += go ? (uint32_t)m : 0u;
            wk.leaves += first_active_lane() ? 1u : 0u;
        }
        float a = 0.f, b = 0.f;
        float da, db;
        const int r = go ? prism_interval<false>(verts, voff, m, ld(height + prim), q.px, q.py, q.pz, g, w0, w1, W0u,
                                                 W0v, W1u, W1v, a, b, da, db)
                         : 0;
        if constexpr (kCount) wk.inserts += r ? 1u : 0u;
        bool over = false, full = false;
        if (r) {
            over = !union_insert(U, a, b);
            full = !over && U.n == 1 && U.lo[0] <= w0 && U.hi[0] >= w1;  // the whole window is in shadow
        }
        const uint64_t om = ballot(over);
        ovm |= om;
        return om | ballot(full);
    };
    const SegFan ft(g, q.px, q.py, q.pz);
    packet_traverse_seg<kCount>(src.nodes, src.voff, stack, ballot(live), ft, leaf_m, wk, src.root);
    ov = lane_in(ovm);
}

// The view of node `nd` for segment g, with child references r0 (left)
// and r1 (right) already in view form (byte offsets, or leaf / absent).
__device__ __forceinline__ SegNode make_view(const Node &nd, int r0, int r1, const SegConst &g)
{
    const FanGeom f = fan_geom(g);
    const bool lfirst = seg_key(nd.lx0, nd.ly0, nd.lx1, nd.ly1, g.mdx, g.mdy) <=
                        seg_key(nd.rx0, nd.ry0, nd.rx1, nd.ry1, g.mdx, g.mdy);
    SegNode v;
    const int a = lfirst ? 0 : 1;
    seg_child(f, nd.lx0, nd.ly0, nd.lx1, nd.ly1, nd.lz1, nd.left != kNone, v.c[a]);
    seg_child(f, nd.rx0, nd.ry0, nd.rx1, nd.ry1, nd.rz1, nd.right != kNone, v.c[1 - a]);
    v.ref[a] = r0;
    v.ref[1 - a] = r1;
    return v;
}

__device__ __forceinline__ int view_ref(int r) { return r >= 0 ? r * (int)sizeof(SegNode) : r; }

// The per-segment node views of segments [j0, j1): one thread per
// (segment, node), written to out[(j - j0) * stride + node].
__global__ void k_seg_nodes(const Node *__restrict__ nodes, int n_nodes, const SegConst *__restrict__ segs, int j0,
                            int j1, int64_t stride, SegNode *__restrict__ out)
{
    const int64_t t = (int64_t)wg_id() * wg_size() + tid();
    if (t >= (int64_t)(j1 - j0) * n_nodes) return;
    const int jj = (int)(t / n_nodes);
    const int node = (int)(t - (int64_t)jj * n_nodes);
    const Node nd = nodes[node];
    out[jj * stride + node] = make_view(nd, view_ref(nd.left), view_ref(nd.right), segs[j0 + jj]);
}

// Roof-covered: inside a footprint (other than the point's own building)
// and not above that roof -- shadowed from every direction.
__device__ __forceinline__ bool roof_covered(cNode *nodes, StackEntry *stack, cfloat4 *verts, cfloat *height,
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

// kOcc waves per SIMD, a launch choice (6, 7 or 8; the tuner measures
// them).  At 8 the kernel fits in 64 VGPRs (the compiler would settle for
// fewer waves otherwise), which hides more of the scalar-load and
// compare-chain latency of the traversal loop.
template <bool kCount, int kOcc>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kOcc))) void k_accrual(
    const Node *nodes_g, const SegNode *snodes_g, int n_nodes, const int32_t *voff_g, const float4 *verts_g,
    const float *height_g, const SegConst *segs_g, int j0, int j1, Sched W, PointArgs P, BinOut O, SpillArgs S,
    uint64_t *work)
{
    Work wk{0, 0, 0, 0, 0, 0, 0};
    cNode *nodes = (cNode *)nodes_g;
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSeg *segs = (cSeg *)segs_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    // the outputs are needed only when a bin ends, the schedule once per
    // unit: parked in LDS so their pointers hold no scalar registers
    // through the traversal loop
    __shared__ int s_O[sizeof(BinOut) / 4];
    __shared__ int s_S[sizeof(SpillArgs) / 4];
    __shared__ int s_W[sizeof(Sched) / 4];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    if (tid() == 0) {
        lds_park((lds_int *)s_O, O);
        lds_park((lds_int *)s_S, S);
        lds_park((lds_int *)s_W, W);
        lds_park((lds_int *)s_P, P);
    }
    __syncthreads();
    StackEntry *stack = s_stack[tid() >> 6];
    const int lane = tid() & 63;
    int kx = 0;
    Unit un;
    while (next_unit((lds_int *)s_W, j0, j1, kx, un)) {
        const int ja = uniform(un.a), jb = uniform(un.b);
        const PointArgs Pd = lds_uniform<PointArgs>((lds_int *)s_P);
        const int64_t n = Pd.n;
        const int64_t i = (int64_t)un.tile * 64 + lane;
        const bool valid = i < n;
        const LanePoint q = load_point(Pd, i, valid);
        const bool covered = roof_covered(nodes_g ? nodes : nullptr, stack, verts, height, q, valid);

        int cnt = 0;
        double mins = 0.0;  // per-lane FP64: long spans sum thousands of segment measures
        int bin = jb > ja ? ld(segs + ja).bin : 0;
        const BinOut O0 = lds_uniform<BinOut>((lds_int *)s_O);
        bool fresh = (ja == j0 ? O0.fresh_first : O0.fresh_rest) != 0;
        for (int j = ja; j < jb; ++j) {
            const SegConst g = ld(segs + j);
            if (g.bin != bin) {
                const BinOut Ob = lds_uniform<BinOut>((lds_int *)s_O);
                if (valid) put_bin(Ob, (int64_t)bin * n + i, fresh, cnt, mins);
                cnt = 0;
                mins = 0.0;
                bin = g.bin;
                fresh = Ob.fresh_rest != 0;
            }
            Union4 U;
            bool ov;
            const SegSrc src{snodes_g ? (cSegNode *)(snodes_g + (int64_t)(j - j0) * n_nodes) : nullptr,
                             (cint *)voff_g, 0};
            accrue_segment<kCount>(src, stack, verts, height, g, q, valid && !covered, 0.f, g.theta, U, ov, wk);
            if constexpr (kCount) {
                wk.units += valid ? 1u : 0u;
                wk.spills += (valid && ov) ? 1u : 0u;
            }
            const SegConst gm = reload(segs, j);
            if (covered && valid) {
                mins += (double)gm.dt;
                cnt += gm.ns_all;
            } else if (!ov) {
                measure(U, gm, 0.f, gm.theta, true, mins, cnt);
            }
            if (ballot(valid && ov))
                spill_push(lds_uniform<SpillArgs>((lds_int *)s_S), valid && ov, i, j, 0.f, gm.theta);
        }
        const BinOut Oe = lds_uniform<BinOut>((lds_int *)s_O);
        if (Oe.pcnt) {
            // a piece of one bin's run: its sums go to the part's row
            if (valid) {
                Oe.pcnt[(int64_t)un.part * n + i] = cnt;
                Oe.pmin[(int64_t)un.part * n + i] = mins;
            }
        } else if (valid && jb > ja) {
            put_bin(Oe, (int64_t)bin * n + i, fresh, cnt, mins);
        }
    }
    if constexpr (kCount) flush_work(wk, work);
}

// Adds the pieces of every run of a launch, in piece order, into the run's
// bin: the launch's first run is stored or added to as O says for the
// launch's first bin, the others as for its later bins.
__global__ void k_add_pieces(Sched W, int j0, int j1, const SegConst *__restrict__ segs, int64_t n, BinOut O)
{
    const int sub = W.sub > 1 ? W.sub : 1;
    const int runs = (int)W.n_parts / sub;
    const int64_t total = (int64_t)runs * n;
    const int64_t stride = (int64_t)n_wg() * wg_size();
    for (int64_t t = (int64_t)wg_id() * wg_size() + tid(); t < total; t += stride) {
        const int r = (int)(t / n);
        const int64_t i = t - (int64_t)r * n;
        int cnt = 0;
        double mins = 0.0;
        for (int p = r * sub; p < (r + 1) * sub; ++p) {
            cnt += O.pcnt[(int64_t)p * n + i];
            mins += O.pmin[(int64_t)p * n + i];
        }
        const int bin = segs[max(W.part_start[r], j0)].bin;
        put_bin(O, (int64_t)bin * n + i, (r == 0 ? O.fresh_first : O.fresh_rest) != 0, cnt, mins);
    }
}

// Continuous shadow (Sec. 3.1) over one window [w0, w1] whose occluded set
// U is sorted and disjoint: a set that starts at w0 extends the current run
// (the run so far reached the window start), any gap ends it; best keeps
// the longest run in minutes.  Applied window after window in time order
// this joins the per-segment prefix, longest and suffix as Sec. 6 stitches
// them across the edges of a day's path.
__device__ __forceinline__ void runs_update(const Union4 &U, float w0, float w1, float rate, float &run, float &best)
{
    if (U.n == 0) run = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r < U.n) {
            const float len = (U.hi[r] - U.lo[r]) * rate;
            run = (r == 0 && U.lo[0] <= w0) ? run + len : len;
            best = fmaxf(best, run);
            if (U.hi[r] < w1) run = 0.f;
        }
    }
}

// The accrual form with the continuous shadow of every point.  Runs must be
// followed in time order, so a segment whose set needs more than four
// pieces is not queued for the spill rounds: the lane walks that segment
// window by window from its start (halving the window on overflow,
// doubling it after a success) while the other lanes wait.  A window would
// have to shrink below theta / 4096 to raise the overflow flag.  Seven
// waves per SIMD (the compiler fits the kernel in 72 VGPRs) measured 4 %
// faster than the six its natural allocation allows.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_accrual_runs(
    const Node *nodes_g, const SegNode *snodes_g, int n_nodes, const int32_t *voff_g, const float4 *verts_g,
    const float *height_g, const SegConst *segs_g, int j0, int j1, Sched W, PointArgs P, BinOut O, float *longest,
    uint32_t *overflow)
{
    cNode *nodes = (cNode *)nodes_g;
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSeg *segs = (cSeg *)segs_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    // outputs (and where to flag overflow), schedule and points parked in
    // LDS: needed once per unit or at a bin's end, they hold no scalar
    // registers through the traversal
    __shared__ int s_O[sizeof(BinOut) / 4];
    __shared__ int s_W[sizeof(Sched) / 4];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    __shared__ float *s_longest;
    __shared__ uint32_t *s_overflow;
    if (tid() == 0) {
        lds_park((lds_int *)s_O, O);
        lds_park((lds_int *)s_W, W);
        lds_park((lds_int *)s_P, P);
        s_longest = longest;
        s_overflow = overflow;
    }
    __syncthreads();
    StackEntry *stack = s_stack[tid() >> 6];
    const int lane = tid() & 63;
    Work none{0, 0, 0, 0, 0, 0, 0};
    int kx = 0;
    Unit un;
    while (next_unit((lds_int *)s_W, j0, j1, kx, un)) {
        const PointArgs Pd = lds_uniform<PointArgs>((lds_int *)s_P);
        const int64_t n = Pd.n;
        const int64_t i = (int64_t)un.tile * 64 + lane;
        const bool valid = i < n;
        const LanePoint q = load_point(Pd, i, valid);
        const bool covered = roof_covered(nodes_g ? nodes : nullptr, stack, verts, height, q, valid);
        const int ja = uniform(un.a), jb = uniform(un.b);

        int cnt = 0;
        double mins = 0.0;
        float run = 0.f, best = 0.f;
        int bin = jb > ja ? ld(segs + ja).bin : 0;
        int day = jb > ja ? ld(segs + ja).day : 0;
        const BinOut O0 = lds_uniform<BinOut>((lds_int *)s_O);
        bool fresh = (ja == j0 ? O0.fresh_first : O0.fresh_rest) != 0;
        auto flush = [&]() {
            if (!valid) return;
            const int64_t o = (int64_t)bin * n + i;
            const BinOut Ob = lds_uniform<BinOut>((lds_int *)s_O);
            put_bin(Ob, o, fresh, cnt, mins);
            float *lg = s_longest;
            if (lg) lg[o] = fresh ? best * Ob.scale : fmaxf(lg[o], best * Ob.scale);
        };
        for (int j = ja; j < jb; ++j) {
            const SegConst g = ld(segs + j);
            if (g.bin != bin) {
                flush();
                cnt = 0;
                mins = 0.0;
                best = 0.f;
                bin = g.bin;
                fresh = lds_uniform<BinOut>((lds_int *)s_O).fresh_rest != 0;
            }
            if (g.day != day) {
                run = 0.f;
                day = g.day;
            }
            if (covered && valid) {
                mins += (double)g.dt;
                cnt += g.ns_all;
                run += g.dt;
                best = fmaxf(best, run);
            }
            bool pending = valid && !covered;
            float w0 = 0.f, s = g.theta;
            while (ballot(pending)) {
                const float w1 = fminf(w0 + s, g.theta);
                Union4 U;
                bool ov;
                const SegSrc src{snodes_g ? (cSegNode *)(snodes_g + (int64_t)(j - j0) * n_nodes) : nullptr,
                                 (cint *)voff_g, 0};
                accrue_segment<false>(src, stack, verts, height, g, q, pending, w0, w1, U, ov, none);
                if (pending) {
                    if (ov) {
                        if (s < g.theta * (1.0f / 4096.0f)) {
                            atomicOr(s_overflow, 2u);
                            pending = false;
                        } else {
                            s *= 0.5f;
                        }
                    } else {
                        const SegConst gm = reload(segs, j);
                        measure(U, gm, w0, w1, w1 >= gm.theta, mins, cnt);
                        runs_update(U, w0, w1, gm.rate, run, best);
                        w0 = w1;
                        pending = w0 < g.theta;
                        s = fminf(2.f * s, g.theta);
                    }
                }
            }
        }
        if (jb > ja) flush();
    }
}

// One spill round: each queued (point, segment, window) is taken by one
// wave whose 64 lanes take one 64th of the window each.  Every lane follows
// the same point along the same segment, so the wave's traversal stays
// coherent (a lane per queued entry would walk 64 unrelated points).  The
// lanes' measures are summed across the wave and added with one atomic per
// output; sub-windows that still need more than four pieces go to the
// next queue.
__global__ __launch_bounds__(kThreads) void k_spill(const SegNode *snodes_g, int n_nodes, int j0, const int32_t *voff_g,
                                                    const float4 *verts_g, const float *height_g,
                                                    const SegConst *segs_g, PointArgs P, float scale, int32_t *counts,
                                                    float *minutes, double *minutes64, const int4 *in,
                                                    const uint32_t *in_count, int32_t cap, SpillArgs S)
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
        // lane l takes [w0 + l d, w0 + (l + 1) d]: neighbours share the same
        // rounded boundary, the last lane ends exactly at ew1
        const float d = (ew1 - ew0) * (1.f / 64.f);
        const float w0 = lane == 0 ? ew0 : fmaf((float)lane, d, ew0);
        const float w1 = lane == 63 ? ew1 : fmaf((float)(lane + 1), d, ew0);
        const LanePoint q = load_point(P, i, true);
        const SegConst g = ld(segs + j);
        Union4 U;
        bool ov;
        Work none{0, 0, 0, 0, 0, 0, 0};
        const SegSrc src{snodes_g ? (cSegNode *)(snodes_g + (int64_t)(j - j0) * n_nodes) : nullptr,
                         (cint *)voff_g, 0};
        accrue_segment<false>(src, stack, verts, height, g, q, true, w0, w1, U, ov, none);
        double mins = 0.0;
        int cnt = 0;
        if (!ov) measure(U, g, w0, w1, w1 >= g.theta, mins, cnt);
        for (int o = 32; o > 0; o >>= 1) {
            mins += __shfl_xor(mins, o, 64);
            cnt += __shfl_xor(cnt, o, 64);
        }
        if (lane == 0) {
            const int64_t o = (int64_t)g.bin * P.n + i;
            if (minutes) atomicAdd(&minutes[o], (float)(mins * scale));
            if (minutes64) atomicAdd(&minutes64[o], mins * scale);
            if (counts) atomicAdd(&counts[o], cnt);
        }
        spill_push(S, ov, i, j, w0, w1);
    }
}

// ------------------------------------------------------------------ contribution
// Building contribution (Sec. 7.2): every building's own occluded interval
// over each segment, never merged with the others' and with no early exit
// (a lane whose window is already shadowed keeps walking: later buildings
// still count).  The lanes' weighted minutes for one leaf are summed across
// the wave and added with one FP64 atomic; a back-facing wall counts for
// the point's own building.  Eight waves per SIMD (56 VGPRs): 17.5 ms on
// the block scene against 19.4 at the compiler's seven.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_contrib(const SegNode *snodes_g, int n_nodes, const int32_t *voff_g,
                                                      const float4 *verts_g, const float *height_g,
                                                      const SegConst *segs_g, int j0, int j1, Sched W, PointArgs P,
                                                      const float *weight, const int32_t *order, int n_b,
                                                      double *contrib)
{
    cfloat4 *verts = (cfloat4 *)verts_g;
    cfloat *height = (cfloat *)height_g;
    cSeg *segs = (cSeg *)segs_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    __shared__ int s_W[sizeof(Sched) / 4];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    if (tid() == 0) {
        lds_park((lds_int *)s_W, W);
        lds_park((lds_int *)s_P, P);
    }
    __syncthreads();
    StackEntry *stack = s_stack[tid() >> 6];
    const int lane = tid() & 63;
    Work none{0, 0, 0, 0, 0, 0, 0};
    int kx = 0;
    Unit un;
    while (next_unit((lds_int *)s_W, j0, j1, kx, un)) {
        const PointArgs Pd = lds_uniform<PointArgs>((lds_int *)s_P);
        const int64_t i = (int64_t)un.tile * 64 + lane;
        const bool valid = i < Pd.n;
        const LanePoint q = load_point(Pd, i, valid);
        const float wt = valid ? (weight ? weight[i] : 1.f) : 0.f;
        const bool active = valid & (wt != 0.f);
        // Back-facing minutes go to the point's own building: kept per lane
        // over the bin's segments and added once per bin, with one atomic
        // for the wave when all its contributing lanes share the building
        // (facade points come wall by wall, so they nearly always do).
        const int ja = uniform(un.a), jb = uniform(un.b);
        double bf = 0.0;
        int bin = jb > ja ? ld(segs + ja).bin : 0;
        auto flush_backface = [&]() {
            const uint64_t has = ballot(bf != 0.0);
            if (!has) return;
            const int lead = (int)__builtin_ctzll(has);
            const int o0 = __shfl(q.own, lead, 64);
            double *row = contrib + (int64_t)bin * n_b;
            if (!ballot(bf != 0.0 && q.own != o0)) {
                double s = bf;
                for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
                if (lane == lead) atomicAdd(&row[order[o0]], s);
            } else if (bf != 0.0) {
                atomicAdd(&row[order[q.own]], bf);
            }
            bf = 0.0;
        };
        for (int j = ja; j < jb; ++j) {
            const SegConst g = ld(segs + j);
            if (g.bin != bin) {
                flush_backface();
                bin = g.bin;
            }
            double *row = contrib + (int64_t)g.bin * n_b;
            if (active && q.own >= 0) {
                float a, b;
                if (backface_interval(q.nx, q.ny, g, 0.f, g.theta, 1.f, 0.f, g.cth, g.sth, a, b))
                    bf += (double)((b - a) * g.wrate * wt);
            }
            if (snodes_g == nullptr) continue;
            const SegFan ft(g, q.px, q.py, q.pz);
            auto leaf = [&](int prim, int voff, int m, uint64_t want) -> uint64_t {
                const uint64_t gm = want & ballot(prim != q.own);
                if (!gm) return 0;
                const bool go = lane_in(gm);
                float a = 0.f, b = 0.f, da, db;
                const int r = go ? prism_interval<false>(verts, voff, m, ld(height + prim), q.px, q.py, q.pz, g, 0.f,
                                                         g.theta, 1.f, 0.f, g.cth, g.sth, a, b, da, db)
                                 : 0;
                // the wave's total for this building (every lane is active
                // here: the traversal runs on the whole wave)
                const float v = wave_sum(r ? (b - a) * g.wrate * wt : 0.f);
                if (first_active_lane() && v != 0.f) atomicAdd(&row[order[prim]], (double)v);
                return 0;  // no lane retires: every building counts
            };
            packet_traverse_seg<false>((cSegNode *)(snodes_g + (int64_t)(j - j0) * n_nodes), (cint *)voff_g, stack,
                                       ballot(active), ft, leaf, none);
        }
        flush_backface();
    }
}

// ------------------------------------------------------------------ batched
// Variant v of the scene differs from the base only in the heights of a few
// buildings.  Each variant gets its own copy of the node array and heights;
// only the ancestors of the changed leaves need new box tops, which one
// thread per variant walks up sequentially (no races between its walks).

__global__ void k_var_copy(const int4 *__restrict__ base_nodes, int64_t node_words, const float *__restrict__ base_h,
                           int n_b, int V, int4 *__restrict__ vnodes, float *__restrict__ vh)
{
    const int64_t stride = (int64_t)n_wg() * wg_size();
    for (int64_t t = (int64_t)wg_id() * wg_size() + tid(); t < (int64_t)V * node_words; t += stride)
        vnodes[t] = base_nodes[t % node_words];
    for (int64_t t = (int64_t)wg_id() * wg_size() + tid(); t < (int64_t)V * n_b; t += stride)
        vh[t] = base_h[t % n_b];
}

__global__ void k_var_heights(int V, int k, const int32_t *__restrict__ ids, const float *__restrict__ h,
                              const int32_t *__restrict__ rank, int n_b, float *__restrict__ vh, uint32_t *flag)
{
    const int t = wg_id() * wg_size() + tid();
    if (t >= V * k) return;
    const int id = ids[t];
    const float hv = h[t];
    if (id < 0 || id >= n_b || !(hv > 0.f)) {
        atomicOr(flag, 4u);
        return;
    }
    vh[(int64_t)(t / k) * n_b + rank[id]] = hv;
}

__global__ void k_var_refit(int V, int k, const int32_t *__restrict__ ids, const int32_t *__restrict__ rank,
                            const int32_t *__restrict__ parent, int n_int, int n_b, int n_nodes,
                            const float *__restrict__ vh, Node *vnodes)
{
    const int v = wg_id() * wg_size() + tid();
    if (v >= V) return;
    Node *nodes = vnodes + (int64_t)v * n_nodes;
    for (int j = 0; j < k; ++j) {
        const int id = ids[v * k + j];
        if (id < 0 || id >= n_b) continue;
        const int prim = rank[id];
        float z = pad_hi(vh[(int64_t)v * n_b + prim]);
        int pp = parent[n_int + prim];
        for (int guard = 0; pp >= 0 && guard < 64; ++guard) {
            Node &nd = nodes[pp >> 1];
            if (pp & 1) nd.rz1 = z;
            else nd.lz1 = z;
            z = fmaxf(nd.lz1, nd.rz1);
            pp = parent[pp >> 1];
        }
    }
}

// Per-segment views of the variants.  A variant differs from the base only
// in the boxes of the ancestors of its changed leaves, so it shares the
// base views everywhere else: each variant gets its own copies of the
// views of those ancestors ("changed nodes"), whose child references point
// to the variant's copy where the child changed too and to the base view
// otherwise.  Every ancestor of a changed node is changed, so a walk
// started at the variant's copy of the root sees exactly the variant's
// hierarchy.  Copies of variant v live at view index n_nodes + v * cmax + c.

// vlist[v][0, vcount[v]): the changed interior nodes of variant v (one
// thread per variant; a chain walk stops at the first node already listed,
// whose ancestors are listed too); vroot[v]: byte offset of the root's view.
__global__ void k_var_list(int V, int k, const int32_t *__restrict__ ids, const int32_t *__restrict__ rank,
                           const int32_t *__restrict__ parent, int n_int, int n_b, int n_nodes, int cmax,
                           int32_t *__restrict__ vlist, int32_t *__restrict__ vcount, int32_t *__restrict__ vroot)
{
    const int v = wg_id() * wg_size() + tid();
    if (v >= V) return;
    int32_t *L = vlist + (int64_t)v * cmax;
    int c = 0;
    for (int j = 0; j < k; ++j) {
        const int id = ids[v * k + j];
        if (id < 0 || id >= n_b) continue;
        int pp = parent[n_int + rank[id]];
        for (int guard = 0; pp >= 0 && guard < 64 && c < cmax; ++guard) {
            const int a = pp >> 1;
            bool seen = false;
            for (int q = 0; q < c; ++q) seen = seen || L[q] == a;
            if (seen) break;
            L[c++] = a;
            pp = parent[a];
        }
    }
    vcount[v] = c;
    int root = 0;
    for (int q = 0; q < c; ++q)
        if (L[q] == 0) root = (n_nodes + v * cmax + q) * (int)sizeof(SegNode);
    vroot[v] = root;
}

// Child references of the copies, in view form: one thread per (variant,
// copy).
__global__ void k_var_refs(int V, int cmax, int n_nodes, const Node *__restrict__ nodes,
                           const int32_t *__restrict__ vlist, const int32_t *__restrict__ vcount, int2 *__restrict__ vref)
{
    const int64_t t = (int64_t)wg_id() * wg_size() + tid();
    if (t >= (int64_t)V * cmax) return;
    const int v = (int)(t / cmax), c = (int)(t - (int64_t)v * cmax);
    const int n = vcount[v];
    if (c >= n) return;
    const int32_t *L = vlist + (int64_t)v * cmax;
    const Node nd = nodes[L[c]];
    int r[2] = {nd.left, nd.right};
    for (int s = 0; s < 2; ++s) {
        if (r[s] < 0) continue;  // a leaf or absent
        int at = -1;
        for (int q = 0; q < n; ++q) at = L[q] == r[s] ? q : at;
        r[s] = (at >= 0 ? n_nodes + v * cmax + at : r[s]) * (int)sizeof(SegNode);
    }
    vref[t] = make_int2(r[0], r[1]);
}

// The copies' views for segments [j0, j1), from the variants' refitted
// boxes: one thread per (segment, variant, copy).
__global__ void k_seg_var(int V, int cmax, int n_nodes, const Node *__restrict__ vnodes,
                          const int32_t *__restrict__ vlist, const int32_t *__restrict__ vcount,
                          const int2 *__restrict__ vref, const SegConst *__restrict__ segs, int j0, int j1,
                          int64_t stride, SegNode *__restrict__ out)
{
    const int64_t t = (int64_t)wg_id() * wg_size() + tid();
    const int64_t per = (int64_t)V * cmax;
    if (t >= (int64_t)(j1 - j0) * per) return;
    const int jj = (int)(t / per);
    const int64_t vc = t - jj * per;
    const int v = (int)(vc / cmax), c = (int)(vc - (int64_t)v * cmax);
    if (c >= vcount[v]) return;
    const Node nd = vnodes[(int64_t)v * n_nodes + vlist[vc]];
    const int2 r = vref[vc];
    out[jj * stride + n_nodes + vc] = make_view(nd, r.x, r.y, segs[j0 + jj]);
}

// tile_off[v] = first tile of variant v, 64 points per tile
__global__ void k_var_tiles(int V, const int64_t *__restrict__ var_off, int64_t *__restrict__ tile_off)
{
    if (wg_id() != 0 || tid() != 0) return;
    int64_t t = 0;
    for (int v = 0; v < V; ++v) {
        tile_off[v] = t;
        t += (var_off[v + 1] - var_off[v] + 63) / 64;
    }
    tile_off[V] = t;
}

// Persistent accrual over the (variant, tile) queue.  A wave takes the next
// tile with one atomic, finds its variant by binary search, and runs every
// segment for its 64 points on that variant's hierarchy.  A point-segment
// whose occluded set needs more than four pieces is finished in place by
// walking its window left to right with halving / doubling sub-windows.
// Seven waves per SIMD: 72 VGPRs with a few spilled to scratch, measured
// faster (64.5 ms on 256 variants) than six waves (77 ms) or eight (75 ms).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(7))) void k_batched(const Node *vnodes_g, int n_nodes, const SegNode *views_g,
                                                      int64_t stride, const int32_t *voff_g,
                                                      const int32_t *__restrict__ vroot, const float4 *verts_g,
                                                      const float *vh_g, int n_b, const SegConst *segs_g, int j0,
                                                      int j1, PointArgs P, const int64_t *__restrict__ var_off,
                                                      const int64_t *__restrict__ tile_off, int V,
                                                      uint32_t *tile_counter, int32_t grab, float scale,
                                                      int32_t *counts, float *minutes, uint32_t *flag)
{
    cfloat4 *verts = (cfloat4 *)verts_g;
    cSeg *segs = (cSeg *)segs_g;
    __shared__ StackEntry s_stack[kWaves][kStackDepth];
    __shared__ int s_P[sizeof(PointArgs) / 4];
    StackEntry *stack = s_stack[tid() >> 6];
    const int lane = tid() & 63;
    const int64_t T = tile_off[V];
    const int64_t n = P.n;
    if (tid() == 0) lds_park((lds_int *)s_P, P);
    __syncthreads();
    // a wave takes `grab` consecutive (variant, tile) items per atomic
    int64_t t = 0, t_end = 0;
    for (;;) {
        if (t >= t_end) {
            int64_t g0 = 0;
            if (lane == 0) g0 = atomicAdd((unsigned long long *)tile_counter, (unsigned long long)grab);
            g0 = __shfl(g0, 0, 64);
            t = g0;
            t_end = min(g0 + (int64_t)grab, T);
        }
        if (t >= T) break;
        int lo = 0, hi = V - 1;               // last v with tile_off[v] <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_off[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int v = uniform(lo);
        cNode *nodes = (cNode *)(vnodes_g + (int64_t)v * n_nodes);
        cfloat *height = (cfloat *)(vh_g + (int64_t)v * n_b);
        const int64_t i = var_off[v] + (t - tile_off[v]) * 64 + lane;
        const bool valid = i < var_off[v + 1];
        const LanePoint q = load_point(lds_uniform<PointArgs>((lds_int *)s_P), i, valid);
        const bool covered = roof_covered(nodes, stack, verts, height, q, valid);
        const int root = vroot ? vroot[v] : 0;
        int cnt = 0;
        double mins = 0.0;
        int bin = j1 > j0 ? ld(segs + j0).bin : 0;
        Work none{0, 0, 0, 0, 0, 0, 0};
        for (int j = j0; j < j1; ++j) {
            const SegConst g = ld(segs + j);
            if (g.bin != bin) {
                if (valid) {
                    if (counts) counts[(int64_t)bin * n + i] += cnt;
                    if (minutes) minutes[(int64_t)bin * n + i] += (float)(mins * scale);
                }
                cnt = 0;
                mins = 0.0;
                bin = g.bin;
            }
            if (covered && valid) {
                mins += (double)g.dt;
                cnt += g.ns_all;
                continue;
            }
            float w0 = 0.f, s = g.theta;
            bool pending = valid;
            while (ballot(pending)) {
                const float w1 = fminf(w0 + s, g.theta);
                Union4 U;
                bool ov;
                const SegSrc src{views_g ? (cSegNode *)(views_g + (int64_t)(j - j0) * stride) : nullptr,
                                 (cint *)voff_g, root};
                accrue_segment<false>(src, stack, verts, height, g, q, pending, w0, w1, U, ov, none);
                if (pending) {
                    if (ov) {
                        if (s < g.theta * (1.0f / 4096.0f)) {
                            atomicOr(flag, 2u);
                            pending = false;
                        } else {
                            s *= 0.5f;
                        }
                    } else {
                        measure(U, reload(segs, j), w0, w1, w1 >= g.theta, mins, cnt);
                        w0 = w1;
                        pending = w0 < g.theta;
                        s = fminf(2.f * s, g.theta);
                    }
                }
            }
        }
        if (valid && j1 > j0) {
            if (counts) counts[(int64_t)bin * n + i] += cnt;
            if (minutes) minutes[(int64_t)bin * n + i] += (float)(mins * scale);
        }
        ++t;
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t stride = (int64_t)n_wg() * wg_size();
    for (int64_t t = (int64_t)wg_id() * wg_size() + tid(); t < n; t += stride) p[t] = v;
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

__global__ void k_spill_check(const uint32_t *count, uint32_t *overflow)
{
    if (*count) atomicOr(overflow, 2u);
}

}  // namespace

#define SA_CHECK_LAUNCH(what)                                                   \
    do {                                                                        \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) {                                                 \
            err = std::string(what) + ": " + hipGetErrorString(e_);             \
            return SA_ERR_DEVICE;                                               \
        }                                                                       \
    } while (0)

static PointArgs point_args(const PointsView &pts, const DeviceScene &s)
{
    return PointArgs{pts.n, pts.x, pts.y, pts.z, pts.nx, pts.ny, pts.owner, s.rank, s.n_b};
}

sa_status launch_sampled(const DeviceScene &s, const DevicePath &p, const PointsView &pts, float scale,
                         int32_t *counts, float *minutes, uint32_t *bits, float *longest, uint64_t *work,
                         const TileLaunch &L, uint32_t *grab, hipStream_t st, std::string &err)
{
    if (pts.n == 0) return SA_OK;
    int64_t tiles;
    if (!tile_count(pts.n, tiles, err)) return SA_ERR_INVALID_ARG;
    const Node *nodes = s.n_b > 0 ? s.nodes : nullptr;
    const int ni = L.sampled_instants;
    // Counts and minutes of units that lie in one bin: the queue with the
    // points' sums in LDS (its entries hold the instant, below 2^26).  Bit
    // vectors, the continuous shadow and bins that interleave: the queue
    // with a bitmap replayed in time order; bit vectors pack 32 instants a
    // word across bin boundaries, so a unit is then a whole tile and each
    // word has one writer.
    auto kern = work ? k_sampled_qb<true, 8> : k_sampled_qb<false, 8>;
    if (ni == 1) kern = work ? k_sampled_qb<true, 1> : k_sampled_qb<false, 1>;
    if (ni == 2) kern = work ? k_sampled_qb<true, 2> : k_sampled_qb<false, 2>;
    if (ni == 4) kern = work ? k_sampled_qb<true, 4> : k_sampled_qb<false, 4>;
    if (ni == 16) kern = work ? k_sampled_qb<true, 16> : k_sampled_qb<false, 16>;
    const Split split = bits ? Split::kNone : Split::kUniqueBins;
    int64_t res = resident_blocks(kern, L);
    Sched W = plan_units(p.sample_runs, 0, p.n_samples, tiles, split, res, grab);
    if (!bits && !longest && p.n_samples < (1 << 26) &&
        (W.part_start != nullptr || p.sample_runs.start.size() == 2)) {
        kern = work ? k_sampled_q<true, 8> : k_sampled_q<false, 8>;
        if (ni == 1) kern = work ? k_sampled_q<true, 1> : k_sampled_q<false, 1>;
        if (ni == 2) kern = work ? k_sampled_q<true, 2> : k_sampled_q<false, 2>;
        if (ni == 4) kern = work ? k_sampled_q<true, 4> : k_sampled_q<false, 4>;
        if (ni == 16) kern = work ? k_sampled_q<true, 16> : k_sampled_q<false, 16>;
    }
    res = resident_blocks(kern, L);
    W = plan_units(p.sample_runs, 0, p.n_samples, tiles, split, res, grab);
    sa_status rc = fill_u32(grab, 8 * kGrabStride, 0u, st, err);
    if (rc != SA_OK) return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)unit_blocks(res, W)), dim3(kThreads), 0, st, nodes, s.verts,
                       s.height, p.samples, p.n_samples, W, point_args(pts, s),
                       SampOut{counts, minutes, bits, longest, scale, 0}, work);
    SA_CHECK_LAUNCH("sampled kernel");
    return SA_OK;
}

sa_status run_spill(const DeviceScene &s, const DevicePath &p, const SegNode *views, int j0, const PointArgs &P,
                    float scale, int32_t *counts, float *minutes, double *minutes64, SpillQueue &q, hipStream_t st,
                    std::string &err)
{
    int cur = 0;
    for (int r = 0; r < kSpillRounds; ++r) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, q.counters + (cur ^ 1));
        SpillArgs S{q.entries[cur ^ 1], q.counters + (cur ^ 1), q.counters + 2, q.capacity};
        hipLaunchKernelGGL(k_spill, dim3(kSpillBlocks), dim3(kThreads), 0, st, views, s.n_nodes, j0, s.voff, s.verts,
                           s.height, p.segs, P, scale, counts, minutes, minutes64, (const int4 *)q.entries[cur],
                           (const uint32_t *)(q.counters + cur), q.capacity, S);
        cur ^= 1;
    }
    // anything still queued after the last round is unfinished work
    hipLaunchKernelGGL(k_spill_check, dim3(1), dim3(1), 0, st, (const uint32_t *)(q.counters + cur), q.counters + 2);
    SA_CHECK_LAUNCH("accrual spill");
    return SA_OK;
}

sa_status fill_u32(void *p, int64_t n, uint32_t v, hipStream_t st, std::string &err)
{
    if (n <= 0) return SA_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, n, v);
    SA_CHECK_LAUNCH("fill");
    return SA_OK;
}

sa_status launch_batched(const DeviceScene &s, const DevicePath &p, int32_t n_var, int32_t k, const int32_t *ids,
                         const float *h, const PointsView &pts, const int64_t *var_off, float scale, int32_t *counts,
                         float *minutes, int32_t grid_blocks, int32_t grab, uint32_t *flag, Scratch &scr,
                         Scratch &views_scr, hipStream_t st, std::string &err)
{
    if (n_var == 0 || pts.n == 0) return SA_OK;
    grab = std::max(grab, 1);
    const int n_nodes = s.n_b > 0 ? s.n_nodes : 0;
    // copies of changed nodes per variant: at most one chain of ancestors
    // per changed building
    const int cmax = std::max(1, k * std::max(s.depth, 1));
    const int64_t stride = (int64_t)n_nodes + (int64_t)n_var * cmax;  // views per segment
    if (stride * (int64_t)sizeof(SegNode) >= (1ll << 31)) {
        err = "too many variants x changed buildings for one call (views are addressed with 32-bit offsets)";
        return SA_ERR_CAPACITY;
    }
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t node_bytes = up(sizeof(Node) * (size_t)n_var * n_nodes);
    const size_t h_bytes = up(sizeof(float) * (size_t)n_var * s.n_b);
    const size_t tile_bytes = up(sizeof(int64_t) * (n_var + 1));
    const size_t list_bytes = up(sizeof(int32_t) * (size_t)n_var * cmax);
    const size_t ref_bytes = up(sizeof(int2) * (size_t)n_var * cmax);
    const size_t cnt_bytes = up(sizeof(int32_t) * (size_t)n_var);
    const size_t off1 = node_bytes, off2 = off1 + h_bytes, off3 = off2 + tile_bytes, off4 = off3 + list_bytes;
    const size_t off5 = off4 + ref_bytes, off6 = off5 + cnt_bytes, off7 = off6 + cnt_bytes;
    const size_t need = off7 + 256;
    if (scr.bytes < need) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(scr.ptr);
        scr.ptr = nullptr;
        scr.bytes = 0;
        if (hipMalloc(&scr.ptr, need) != hipSuccess) {
            (void)hipGetLastError();
            scr.ptr = nullptr;
            err = "variant scratch allocation failed";
            return SA_ERR_OOM;
        }
        scr.bytes = need;
    }
    char *base = (char *)scr.ptr;
    Node *vnodes = (Node *)base;
    float *vh = (float *)(base + off1);
    int64_t *tile_off = (int64_t *)(base + off2);
    int32_t *vlist = (int32_t *)(base + off3);
    int2 *vref = (int2 *)(base + off4);
    int32_t *vcount = (int32_t *)(base + off5);
    int32_t *vroot = (int32_t *)(base + off6);
    uint32_t *counter = (uint32_t *)(base + off7);
    const int n_int = s.n_b == 1 ? 1 : s.n_b - 1;
    if (s.n_b > 0) {
        hipLaunchKernelGGL(k_var_copy, dim3(2048), dim3(256), 0, st, (const int4 *)s.nodes, (int64_t)n_nodes * 4,
                           (const float *)s.height, s.n_b, n_var, (int4 *)vnodes, vh);
        if (k > 0) {
            hipLaunchKernelGGL(k_var_heights, dim3((n_var * k + 255) / 256), dim3(256), 0, st, n_var, k, ids, h,
                               (const int32_t *)s.rank, s.n_b, vh, flag);
            hipLaunchKernelGGL(k_var_refit, dim3((n_var + 63) / 64), dim3(64), 0, st, n_var, k, ids,
                               (const int32_t *)s.rank, (const int32_t *)s.parent, n_int, s.n_b, n_nodes,
                               (const float *)vh, vnodes);
        }
        hipLaunchKernelGGL(k_var_list, dim3((n_var + 63) / 64), dim3(64), 0, st, n_var, k, ids,
                           (const int32_t *)s.rank, (const int32_t *)s.parent, n_int, s.n_b, n_nodes, cmax, vlist,
                           vcount, vroot);
        const int64_t nr = (int64_t)n_var * cmax;
        hipLaunchKernelGGL(k_var_refs, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, n_var, cmax, n_nodes,
                           (const Node *)s.nodes, (const int32_t *)vlist, (const int32_t *)vcount, vref);
    }
    hipLaunchKernelGGL(k_var_tiles, dim3(1), dim3(1), 0, st, n_var, var_off, tile_off);
    SA_CHECK_LAUNCH("variant set-up");
    const PointArgs P = point_args(pts, s);
    const int blocks = grid_blocks > 0 ? grid_blocks : 2048;
    // segment ranges whose views (base and every variant's copies) fit the
    // per-launch budget; outputs accumulate across the launches
    const int64_t per = std::max<int64_t>(1, kSegNodeBytes / (stride * (int64_t)sizeof(SegNode)));
    for (int64_t j0 = 0; j0 < std::max(p.n_segs, 1); j0 += per) {
        const int j1 = (int)std::min<int64_t>(j0 + per, p.n_segs);
        SegNode *views = nullptr;
        if (s.n_b > 0 && j1 > j0) {
            sa_status rc = build_seg_views(s, p, (int)j0, j1, stride, views_scr, st, views, err);
            if (rc != SA_OK) return rc;
            const int64_t nt = (int64_t)(j1 - j0) * n_var * cmax;
            hipLaunchKernelGGL(k_seg_var, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, n_var, cmax, n_nodes,
                               (const Node *)vnodes, (const int32_t *)vlist, (const int32_t *)vcount,
                               (const int2 *)vref, p.segs, (int)j0, j1, stride, views);
            SA_CHECK_LAUNCH("variant segment views");
        }
        sa_status rc = fill_u32(counter, 2, 0u, st, err);
        if (rc != SA_OK) return rc;
        hipLaunchKernelGGL(k_batched, dim3(blocks), dim3(kThreads), 0, st, s.n_b > 0 ? vnodes : nullptr, n_nodes,
                           views, stride, s.voff, s.n_b > 0 ? (const int32_t *)vroot : nullptr, s.verts,
                           (const float *)vh, s.n_b, p.segs, (int)j0, j1, P, var_off, (const int64_t *)tile_off,
                           n_var, counter, grab, scale, counts, minutes, flag);
        SA_CHECK_LAUNCH("batched accrual");
    }
    return SA_OK;
}

int64_t seg_views_cap(const DeviceScene &s, const Scratch &scr)
{
    const int64_t per_seg = (int64_t)std::max(s.n_nodes, 1) * (int64_t)sizeof(SegNode);
    if (scr.fixed) return (int64_t)scr.bytes / per_seg;
    return std::max<int64_t>(1, kSegNodeBytes / per_seg);
}

sa_status build_seg_views(const DeviceScene &s, const DevicePath &p, int j0, int j1, int64_t stride, Scratch &scr,
                          hipStream_t st, SegNode *&views, std::string &err)
{
    views = nullptr;
    if (s.n_b == 0 || j1 <= j0) return SA_OK;
    const int64_t nt = (int64_t)(j1 - j0) * s.n_nodes;
    const size_t need = (size_t)(j1 - j0) * stride * sizeof(SegNode);
    if (scr.bytes < need && scr.fixed) {
        err = "per-segment node views need " + std::to_string(need) + " bytes, more than the fixed " +
              std::to_string(scr.bytes);
        return SA_ERR_CAPACITY;
    }
    if (scr.bytes < need) {
        // the previous contents may still be read by queued kernels
        (void)hipStreamSynchronize(st);
        (void)hipFree(scr.ptr);
        scr.ptr = nullptr;
        scr.bytes = 0;
        if (hipMalloc(&scr.ptr, need) != hipSuccess) {
            (void)hipGetLastError();
            scr.ptr = nullptr;
            err = "segment node view allocation failed";
            return SA_ERR_OOM;
        }
        scr.bytes = need;
    }
    views = (SegNode *)scr.ptr;
    hipLaunchKernelGGL(k_seg_nodes, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, s.nodes, s.n_nodes, p.segs,
                       j0, j1, stride, views);
    SA_CHECK_LAUNCH("segment node views");
    return SA_OK;
}

// Output mode of an accrual launch starting at segment j0: with `store`
// (no SA_FLAG_ADD, and every bin's segments one contiguous run) a bin is
// stored by the launch holding its first segment and added to by later
// ones, so the outputs need no clearing.
static BinOut bin_out(const DevicePath &p, int j0, bool store, int32_t *counts, float *minutes, double *minutes64,
                      float scale)
{
    const bool first = store && (j0 == 0 || p.seg_bin[j0 - 1] != p.seg_bin[j0]);
    return BinOut{counts, minutes, minutes64, nullptr, nullptr, first ? 1 : 0, store ? 1 : 0, scale, 0};
}

sa_status launch_accrual(const DeviceScene &s, const DevicePath &p, const PointsView &pts, float scale,
                         int32_t *counts, float *minutes, double *minutes64, float *longest, uint64_t *work,
                         bool store, const TileLaunch &L, SpillQueue &q, Scratch &scr, Scratch &piece_scr,
                         hipStream_t st, std::string &err)
{
    const int32_t seg_per_launch = L.segments_per_launch;
    if (pts.n == 0) return SA_OK;
    int64_t tiles;
    if (!tile_count(pts.n, tiles, err)) return SA_ERR_INVALID_ARG;
    const Node *nodes = s.n_b > 0 ? s.nodes : nullptr;
    const PointArgs P = point_args(pts, s);
    // Long spans run as several launches over consecutive segment ranges,
    // each about kChunkWork point-segments and covering at most
    // kSegNodeBytes of per-segment node views (built just before it);
    // outputs are accumulated, so the split is invisible in the results.
    const int64_t cap = seg_views_cap(s, scr);
    if (s.n_b > 0 && p.n_segs > 0 && cap < 1) {
        err = "one segment's node views (" + std::to_string((int64_t)s.n_nodes * (int64_t)sizeof(SegNode)) +
              " bytes) exceed the fixed scratch (" + std::to_string(scr.bytes) + " bytes)";
        return SA_ERR_CAPACITY;
    }
    int64_t per = std::min(std::max<int64_t>(1, kChunkWork / std::max<int64_t>(pts.n, 1)), std::max<int64_t>(cap, 1));
    if (seg_per_launch > 0) per = std::min<int64_t>(per, seg_per_launch);
    if (longest) {
        // whole days per launch, so a run never spans two launches (one
        // day per launch at least, whatever its views take)
        const int D = (int)p.day_seg_off.size() - 1;
        if (scr.fixed && s.n_b > 0)
            for (int d = 0; d < D; ++d)
                if (p.day_seg_off[d + 1] - p.day_seg_off[d] > cap) {
                    err = "one day's node views (" + std::to_string(p.day_seg_off[d + 1] - p.day_seg_off[d]) +
                          " segments) exceed the fixed scratch (" + std::to_string(cap) + " segments fit)";
                    return SA_ERR_CAPACITY;
                }
        for (int d0 = 0; d0 < D;) {
            int d1 = d0 + 1;
            while (d1 < D && p.day_seg_off[d1 + 1] - p.day_seg_off[d0] <= per) ++d1;
            const int j0 = p.day_seg_off[d0], j1 = p.day_seg_off[d1];
            SegNode *views;
            sa_status rc = build_seg_views(s, p, j0, j1, s.n_nodes, scr, st, views, err);
            if (rc != SA_OK) return rc;
            const int64_t res = resident_blocks(k_accrual_runs, L);
            const Sched W = plan_units(p.seg_runs, j0, j1, tiles, Split::kUniqueBins, res, q.grab);
            rc = fill_u32(q.grab, 8 * kGrabStride, 0u, st, err);
            if (rc != SA_OK) return rc;
            hipLaunchKernelGGL(k_accrual_runs, dim3((unsigned)unit_blocks(res, W)), dim3(kThreads), 0,
                               st, nodes, views, s.n_nodes, s.voff, s.verts, s.height, p.segs, j0, j1, W, P,
                               bin_out(p, j0, store, counts, minutes, minutes64, scale), longest, q.counters + 2);
            SA_CHECK_LAUNCH("accrual kernel (continuous shadow)");
            d0 = d1;
        }
        return SA_OK;
    }
    auto kern = work ? k_accrual<true, 8> : k_accrual<false, 8>;
    if (L.waves_per_simd == 6) kern = work ? k_accrual<true, 6> : k_accrual<false, 6>;
    if (L.waves_per_simd == 7) kern = work ? k_accrual<true, 7> : k_accrual<false, 7>;
    const int64_t res = resident_blocks(kern, L);
    // Too few tiles to give every resident wave several (tile, bin) units:
    // each bin's run is then cut into pieces, held as per-piece sums in
    // piece_scr ([part][n] counts and FP64 minutes) and added up in order
    // by a second kernel, so the results stay deterministic.  Without room
    // for the sums (a fixed scratch), whole runs.
    const bool pieces = tiles < 2 * res * kWaves;
    int64_t max_parts = 1;
    if (pieces) {
        // counts of every part, then (256-byte aligned) their FP64 minutes
        const int64_t per_part = (int64_t)pts.n * (int64_t)(sizeof(int32_t) + sizeof(double));
        if (piece_scr.fixed) {
            max_parts = std::max<int64_t>(0, (int64_t)piece_scr.bytes - 256) / per_part;
        } else {
            max_parts = std::max<int64_t>(1, kPieceBytes / per_part);
            const size_t need = (size_t)(std::min<int64_t>(max_parts, 8 * res * kWaves) * per_part) + 256;
            if (piece_scr.bytes < need) {
                (void)hipStreamSynchronize(st);  // earlier launches may still read it
                (void)hipFree(piece_scr.ptr);
                piece_scr.ptr = nullptr;
                piece_scr.bytes = 0;
                if (hipMalloc(&piece_scr.ptr, need) != hipSuccess) {
                    (void)hipGetLastError();
                    piece_scr.ptr = nullptr;
                    err = "accrual piece sums allocation failed";
                    return SA_ERR_OOM;
                }
                piece_scr.bytes = need;
            }
            max_parts = ((int64_t)piece_scr.bytes - 256) / per_part;
        }
    }
    for (int64_t j0 = 0; j0 < p.n_segs; j0 += per) {
        const int j1 = (int)std::min<int64_t>(j0 + per, p.n_segs);
        SegNode *views;
        sa_status rc = build_seg_views(s, p, (int)j0, j1, s.n_nodes, scr, st, views, err);
        if (rc != SA_OK) return rc;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, q.counters);
        SpillArgs S{q.entries[0], q.counters, q.counters + 2, q.capacity};
        const Sched W = plan_units(p.seg_runs, (int)j0, j1, tiles, pieces ? Split::kRunPieces : Split::kUniqueBins,
                                   res, q.grab, max_parts);
        BinOut O = bin_out(p, (int)j0, store, counts, minutes, minutes64, scale);
        if (W.sub > 1) {
            const size_t cnt_bytes = (size_t)W.n_parts * (size_t)pts.n * sizeof(int32_t);
            O.pcnt = (int32_t *)piece_scr.ptr;
            O.pmin = (double *)((char *)piece_scr.ptr + ((cnt_bytes + 255) & ~(size_t)255));
        }
        rc = fill_u32(q.grab, 8 * kGrabStride, 0u, st, err);
        if (rc != SA_OK) return rc;
        hipLaunchKernelGGL(kern, dim3((unsigned)unit_blocks(res, W)), dim3(kThreads), 0, st, nodes, views, s.n_nodes,
                           s.voff, s.verts, s.height, p.segs, (int)j0, j1, W, P, O, S, work);
        SA_CHECK_LAUNCH("accrual kernel");
        if (W.sub > 1) {
            const int64_t total = (int64_t)(W.n_parts / W.sub) * pts.n;
            hipLaunchKernelGGL(k_add_pieces, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)), dim3(256),
                               0, st, W, (int)j0, j1, (const SegConst *)p.segs, pts.n, O);
            SA_CHECK_LAUNCH("accrual piece sums");
        }
        rc = run_spill(s, p, views, (int)j0, P, scale, counts, minutes, minutes64, q, st, err);
        if (rc != SA_OK) return rc;
    }
    return SA_OK;
}

sa_status launch_contribution(const DeviceScene &s, const DevicePath &p, const PointsView &pts, const float *weight,
                              double *contrib, const TileLaunch &L, uint32_t *grab, Scratch &scr, hipStream_t st,
                              std::string &err)
{
    if (pts.n == 0 || s.n_b == 0) return SA_OK;
    int64_t tiles;
    if (!tile_count(pts.n, tiles, err)) return SA_ERR_INVALID_ARG;
    const PointArgs P = point_args(pts, s);
    // long spans: several launches over consecutive segment ranges
    const int64_t per =
        std::min(std::max<int64_t>(1, kChunkWork / 2 / std::max<int64_t>(pts.n, 1)), seg_views_cap(s, scr));
    for (int64_t j0 = 0; j0 < p.n_segs; j0 += per) {
        const int j1 = (int)std::min<int64_t>(j0 + per, p.n_segs);
        SegNode *views;
        sa_status rc = build_seg_views(s, p, (int)j0, j1, s.n_nodes, scr, st, views, err);
        if (rc != SA_OK) return rc;
        // the sums are atomic: on few tiles the units are chunks of segments
        const int64_t res = resident_blocks(k_contrib, L);
        const Split split = tiles < 2 * res * kWaves ? Split::kChunks : Split::kBinRuns;
        const Sched W = plan_units(p.seg_runs, (int)j0, j1, tiles, split, res, grab);
        rc = fill_u32(grab, 8 * kGrabStride, 0u, st, err);
        if (rc != SA_OK) return rc;
        hipLaunchKernelGGL(k_contrib, dim3((unsigned)unit_blocks(res, W)), dim3(kThreads), 0, st, views,
                           s.n_nodes, s.voff, s.verts, s.height, p.segs, (int)j0, j1, W, P, weight,
                           (const int32_t *)s.order, s.n_b, contrib);
        SA_CHECK_LAUNCH("contribution kernel");
    }
    return SA_OK;
}

}  // namespace sa
