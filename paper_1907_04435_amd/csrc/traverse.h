// Device-side building blocks shared by the traversal kernels.
//
// Traversal is wave-coherent: a wave of 64 lanes (64 neighbouring points,
// one sun instant or one path segment) walks the hierarchy as one packet.
// The node index is wave-uniform, so a node is fetched once per wave with a
// scalar load into SGPRs; each lane tests the two child boxes against its
// own ray or fan; a child is entered when any still-live lane needs it.
// The traversal stack is wave-uniform too: one 64-entry array per wave in
// LDS (every lane writes the same entry, pops are broadcast reads), so no
// per-lane stack and no scratch memory is needed.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "sa_internal.h"

namespace sa {
namespace dev {

constexpr int32_t kNone = INT_MIN;

typedef __attribute__((address_space(4))) const Node cNode;
typedef __attribute__((address_space(4))) const float4 cfloat4;
typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const SampleConst cSample;
typedef __attribute__((address_space(4))) const SegConst cSeg;

typedef __attribute__((address_space(4))) const int cint;

// Word-wise copy out of the constant address space: with a wave-uniform
// address this becomes one scalar load of the whole object.
template <class T>
__device__ __forceinline__ T ld(const __attribute__((address_space(4))) T *p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized objects");
    T r;
    int *d = (int *)&r;
    cint *s = (cint *)p;
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) d[i] = s[i];
    return r;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lane masks of float comparisons: one compare each, straight into a mask
// (no round trip through a per-lane boolean).
__device__ __forceinline__ uint64_t ge_mask(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, 3); }
__device__ __forceinline__ uint64_t le_mask(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, 5); }
__device__ __forceinline__ uint64_t lt_mask(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, 4); }
__device__ __forceinline__ uint64_t gt_mask(float a, float b) { return __builtin_amdgcn_fcmpf(a, b, 2); }
__device__ __forceinline__ uint64_t to_mask(bool b) { return ballot(b); }
__device__ __forceinline__ uint64_t to_mask(uint64_t m) { return m; }

constexpr int kStackDepth = 64;

// Box padding of the hierarchy: absorbs the rounding of the slab test at
// large coordinates (boxes only decide what is tested, never a result).
__device__ __forceinline__ float pad_lo(float v) { return v - (1e-2f + fabsf(v) * 0x1p-20f); }
__device__ __forceinline__ float pad_hi(float v) { return v + (1e-2f + fabsf(v) * 0x1p-20f); }

// Work a lane's own traversal needed (instrumented instantiations only).
struct Work {
    uint32_t box, prism, edges, inserts, nodes, units, spills, leaves;
};

__device__ __forceinline__ bool first_active_lane()
{
    const int lane = __lane_id();
    return __builtin_amdgcn_readfirstlane(lane) == lane;
}

// One entry of a wave's traversal stack: a deferred node and the mask of
// the lanes that reached it.
struct alignas(16) StackEntry {
    int32_t node;
    uint32_t lo, hi, pad;
};

__device__ __forceinline__ uint64_t uniform64(uint32_t lo, uint32_t hi)
{
    const uint32_t l = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
    const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi);
    return ((uint64_t)h << 32) | l;
}

// Sum of v over all 64 lanes, returned to every lane; call with every lane
// of the wave active.  Quad permutes and row rotations (DPP, no LDS round
// trips) leave each 16-lane row's sum in all its lanes; the four row sums
// are read out and added.
template <int kCtrl>
__device__ __forceinline__ float add_dpp(float x)
{
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v)
{
    v = add_dpp<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v = add_dpp<0x4E>(v);   // quad_perm [2, 3, 0, 1]: quad sums
    v = add_dpp<0x124>(v);  // row_ror 4: two quads
    v = add_dpp<0x128>(v);  // row_ror 8: the row
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Is this lane's bit set in a wave-uniform mask?  (maps to the exec mask)
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Scalar helpers of the traversal loops.  Written as compare-and-selects
// on 64-bit lane masks: the compiler otherwise turns these conditions into
// lane-mask booleans and spends three or four extra scalar instructions
// per node on them.
// defer = h0 != 0 ? h1 : 0 (the second child, when both are wanted)
__device__ __forceinline__ uint64_t defer_mask(uint64_t h0, uint64_t h1)
{
    uint64_t d;
    asm("s_cmp_lg_u64 %[h0], 0\n"
        "s_cselect_b64 %[d], %[h1], 0"
        : [d] "=&s"(d)
        : [h0] "s"(h0), [h1] "s"(h1)
        : "scc");
    return d;
}
// (node, cur) = h0 != 0 ? (r0, h0) : (r1, h1) (the first child wanted)
__device__ __forceinline__ void descend(uint64_t h0, uint64_t h1, int r0, int r1, int &node, uint64_t &cur)
{
    asm("s_cmp_lg_u64 %[h0], 0\n"
        "s_cselect_b32 %[n], %[r0], %[r1]\n"
        "s_cselect_b64 %[c], %[h0], %[h1]"
        : [n] "=&s"(node), [c] "=&s"(cur)
        : [h0] "s"(h0), [h1] "s"(h1), [r0] "s"(r0), [r1] "s"(r1)
        : "scc");
}

// Packet traversal.  `bt(x0, y0, x1, y1, z1)` is the per-lane child-box
// test (a bool, or directly the lane mask of the lanes that pass);
// `leaf(prim, voff, m, want)` processes a leaf for the lanes in the mask
// `want` and returns the mask of lanes it retires.  `key(x0,y0,x1,y1,z1)`
// orders two wanted children (smaller first).  The walk starts with the
// lanes in `alive` and ends when none is left or the stack runs dry.  A
// lane only tests the children of nodes it reached itself: the walk
// carries the wave mask of the lanes that reached the current node, and
// every stack entry keeps the mask of the lanes that wanted it, so leaves
// no lane reached are skipped.  All the bookkeeping is on those
// wave-uniform masks (scalar registers; liveness too, so no per-lane flag
// is carried around the loop); the only per-lane work is the box tests.
// With kCount, `w` accumulates those box tests and the wave's node
// fetches.
template <bool kCount, class BoxTest, class LeafFn, class KeyFn>
__device__ __forceinline__ void packet_traverse(cNode *nodes, StackEntry *stack, uint64_t alive, BoxTest bt,
                                                LeafFn leaf, KeyFn key, Work &w)
{
    typedef __attribute__((address_space(4))) const char cchar;
    uint64_t cur = alive;
    int sp = 0, node = 0;
    while (cur) {
        // 64-byte nodes: a shifted index is the register offset of one
        // scalar load
        const Node nd = ld((cNode *)((cchar *)nodes + ((uint32_t)node << 6)));
        if constexpr (kCount) {
            w.box += lane_in(cur) ? 2u : 0u;
            w.nodes += first_active_lane() ? 1u : 0u;
        }
        uint64_t h0 = to_mask(bt(nd.lx0, nd.ly0, nd.lx1, nd.ly1, nd.lz1)) & cur;
        uint64_t h1 = to_mask(bt(nd.rx0, nd.ry0, nd.rx1, nd.ry1, nd.rz1)) & cur;
        int r0 = nd.left, r1 = nd.right;
        if ((r0 | r1) < 0) {
            // a leaf child, or the absent right child of a one-prism
            // hierarchy
            uint64_t out = 0;
            if (r0 < 0) {
                if (h0 && r0 != kNone) out |= leaf(~r0, nd.l_voff, nd.l_m, h0);
                h0 = 0;
            }
            if (r1 < 0) {
                if (h1 && r1 != kNone) out |= leaf(~r1, nd.r_voff, nd.r_m, h1);
                h1 = 0;
            }
            alive &= ~out;
            h0 &= alive;
            h1 &= alive;
        }
        if (h0 && h1) {
            // the visiting order must be one decision for the whole wave:
            // with per-lane keys (lanes on different segments) lanes could
            // disagree and the shared stack would lose a subtree
            const bool rfirst = uniform(key(nd.lx0, nd.ly0, nd.lx1, nd.ly1, nd.lz1) >
                                        key(nd.rx0, nd.ry0, nd.rx1, nd.ry1, nd.rz1)) != 0;
            if (rfirst) {
                const uint64_t th = h0;
                h0 = h1;
                h1 = th;
                const int tr = r0;
                r0 = r1;
                r1 = tr;
            }
        }
        const uint64_t defer = defer_mask(h0, h1);
        if (defer) {
            stack[sp] = StackEntry{r1, (uint32_t)defer, (uint32_t)(defer >> 32), 0u};
            ++sp;
        }
        descend(h0, h1, r0, r1, node, cur);
        if (!cur) {
            const uint64_t keep = alive;
            while (sp > 0) {
                --sp;
                const StackEntry e = stack[sp];
                node = uniform(e.node);
                cur = uniform64(e.lo, e.hi) & keep;
                if (cur) break;
            }
        }
    }
}

// Closed convex prism vs the ray p + s d (s > 0): clip the ray's footprint
// projection by every edge half-plane (Cyrus-Beck) in coordinates relative
// to p, then compare the height where it enters with the roof.
__device__ __forceinline__ bool ray_prism(cfloat4 *verts, int voff, int m, float H, float px, float py,
                                          float pz, float dx, float dy, float dz)
{
    float s_in = -INFINITY, s_out = INFINITY;
    for (int e = 0; e < m; ++e) {
        const float4 v = ld(verts + voff + e);
        const float wx = v.x - px, wy = v.y - py;
        const float num = fmaf(v.z, wx, v.w * wy);
        const float den = fmaf(v.z, dx, v.w * dy);   // the same for every lane
        const float s = num * __builtin_amdgcn_rcpf(den);
        // selects, not branches (see packet_traverse)
        s_out = den > 0.f ? fminf(s_out, s) : s_out;
        s_in = den < 0.f ? fmaxf(s_in, s) : s_in;
        s_out = ((den == 0.f) & (num < 0.f)) ? -INFINITY : s_out;
    }
    const float s0 = fmaxf(s_in, 0.f);
    return (s_out >= s0) & (fmaf(s0, dz, pz) <= H);
}

// Is (px, py) inside (or on) the convex CCW footprint?
__device__ __forceinline__ bool in_footprint(cfloat4 *verts, int voff, int m, float px, float py)
{
    bool in = true;
    for (int e = 0; e < m; ++e) {
        const float4 v = ld(verts + voff + e);
        // v.z, v.w = outward normal of the edge from this vertex
        in = in && fmaf(v.z, px - v.x, v.w * (py - v.y)) <= 0.f;
    }
    return in;
}

// ---- angles and directions of the segment geometry, written out so that
// the kernels make no library calls (a call imposes the calling convention
// on the whole kernel: registers saved and reloaded around every site) ----

// atan on [0, 1].  Above tan(pi/8) the reflection
// atan(t) = pi/4 + atan((t - 1) / (t + 1)) brings the argument to
// |u| <= tan(pi/8); there the Taylor series u - u^3/3 + ... - u^15/15 +
// u^17/17 is within |u|^19/19 < 3e-9 of atan(u).
__device__ __forceinline__ float atan01(float t)
{
    const bool refl = t > 0.41421356f;
    const float u = refl ? (t - 1.f) * __builtin_amdgcn_rcpf(t + 1.f) : t;
    const float s = u * u;
    float p = 1.f / 17.f;
    p = fmaf(p, s, -1.f / 15.f);
    p = fmaf(p, s, 1.f / 13.f);
    p = fmaf(p, s, -1.f / 11.f);
    p = fmaf(p, s, 1.f / 9.f);
    p = fmaf(p, s, -1.f / 7.f);
    p = fmaf(p, s, 1.f / 5.f);
    p = fmaf(p, s, -1.f / 3.f);
    p = fmaf(p, s, 1.f);
    const float r = u * p;
    return refl ? r + 0.785398163f : r;
}

// Polar angle of (x, y) in [-pi, pi] (atan2(y, x)), by the octant
// symmetries atan(y/x) = pi/2 - atan(x/y) and pi - angle for x < 0.
__device__ __forceinline__ float polar_angle(float x, float y)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.f ? fminf(mn * __builtin_amdgcn_rcpf(mx), 1.f) : 0.f;
    float r = atan01(t);
    r = ay > ax ? 1.57079633f - r : r;
    r = x < 0.f ? 3.14159265f - r : r;
    return y < 0.f ? -r : r;
}

// sin and cos of an angle in [0, 2 pi): w = k pi/2 + r with |r| <= pi/4
// (pi/2 split in two parts, Cody and Waite, so k pi/2 is subtracted
// without cancellation), Taylor series of sin to r^9 and cos to r^10
// (truncation below 2e-9), then the quadrant k.
__device__ __forceinline__ void sincos_small(float w, float &sn, float &cs)
{
    const float k = rintf(w * 0.636619772f);
    float r = fmaf(-k, 1.5703125f, w);
    r = fmaf(-k, 4.83826794897e-4f, r);
    const float z = r * r;
    float ps = -1.f / 362880.f;
    ps = fmaf(ps, z, 1.f / 5040.f);
    ps = fmaf(ps, z, -1.f / 120.f);
    ps = fmaf(ps, z, 1.f / 6.f);
    const float s = fmaf(-r * z, ps, r);
    float pc = -1.f / 3628800.f;
    pc = fmaf(pc, z, 1.f / 40320.f);
    pc = fmaf(pc, z, -1.f / 720.f);
    pc = fmaf(pc, z, 1.f / 24.f);
    pc = fmaf(pc, z, -0.5f);
    const float c = fmaf(pc, z, 1.f);
    const int q = (int)k & 3;
    sn = q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
    cs = q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}

// ---- sorted disjoint interval set of at most 4 members, in registers ----
struct Union4 {
    float lo[4], hi[4];
    int n;
};

__device__ __forceinline__ void union_clear(Union4 &U)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) U.lo[i] = U.hi[i] = 0.f;
    U.n = 0;
}

// Insert the closed interval [a, b]; false if the result would need more
// than four disjoint members (the set is left unchanged).
__device__ __forceinline__ bool union_insert(Union4 &U, float a, float b)
{
    int nb = 0, na = 0;
    float mlo = a, mhi = b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool use = i < U.n;
        const bool before = use && U.hi[i] < a;
        const bool after = use && U.lo[i] > b;
        const bool ov = use && !before && !after;
        nb += before;
        na += after;
        mlo = ov ? fminf(mlo, U.lo[i]) : mlo;
        mhi = ov ? fmaxf(mhi, U.hi[i]) : mhi;
    }
    const int k = U.n - nb - na;
    const int nn = nb + 1 + na;
    if (nn > 4) return false;
    float nlo[4], nhi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int src = j - 1 + k;
        float slo = U.lo[0], shi = U.hi[0];
#pragma unroll
        for (int s = 1; s < 4; ++s) {
            slo = src == s ? U.lo[s] : slo;
            shi = src == s ? U.hi[s] : shi;
        }
        nlo[j] = j < nb ? U.lo[j] : (j == nb ? mlo : slo);
        nhi[j] = j < nb ? U.hi[j] : (j == nb ? mhi : shi);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        U.lo[j] = nlo[j];
        U.hi[j] = nhi[j];
    }
    U.n = nn;
    return true;
}

__device__ __forceinline__ float cross2(float au, float av, float bu, float bv)
{
    return fmaf(au, bv, -av * bu);
}

// Occluded angle interval of one prism over the window [w0, w1] of a
// segment, for a point at p.  In the segment's plane through p the prism
// is a convex polygon: the footprint lifted vertically into the plane and
// clipped to heights <= H.  The directions from p that meet it form one
// angular interval of span < pi (p is outside); its ends are found by
// cross products over the clipped polygon's vertices (the kept footprint
// vertices and the two clip crossings), and intersected with the window.
// Returns 0: no overlap, 1: [a, b] written.
//
// The lift of a horizontal offset w into the plane divides by the plane
// normal's vertical part nz, which vanishes for a plane through the
// zenith.  Only directions from p matter, so the segment's map M (and the
// heights it gives) carries the factor |nz|: vertices stay bounded for
// every plane, and the clip compares scaled heights with |nz| (H - pz).
// A clip crossing lies at height H - pz itself, so its in-plane point is
// formed directly from its world offset c as (e1 . (c, H - pz),
// e2 . (c, H - pz)), which has no cancellation when nz is small.
//
// With kGrad, da / db receive d(a)/dH and d(b)/dH: an end at a clip
// crossing moves with the roof along the lifted edge, dc/dH = (c1 - c0) /
// (z1 - z0) (the scale cancels), so d(angle)/dH = cross(c, c1 - c0) /
// (|c|^2 (z1 - z0)); ends at footprint vertices (vertical edges) or
// clamped to the window do not move.
template <bool kGrad>
__device__ __forceinline__ int prism_interval(cfloat4 *verts, int voff, int m, float H, float px, float py,
                                              float pz, const SegConst &g, float w0, float w1, float W0u,
                                              float W0v, float W1u, float W1v, float &a, float &b, float &da,
                                              float &db)
{
    const float h = H - pz;
    const float hs = h * fabsf(g.nz);  // the clip height in the scaled plane
    float lou = 0.f, lov = 0.f, hiu = 0.f, hiv = 0.f, dlo = 0.f, dhi = 0.f;
    // Lane masks (scalar registers) for the per-lane flags: which lanes have
    // a candidate yet, which see the footprint from inside every edge, which
    // vertices are below the roof line.  Only the selects are vector work.
    uint64_t have = 0, inside = ~0ull;
    if (kGrad || g.steep) {
        // extremes tracked in in-plane coordinates (derivatives, or a plane
        // too close to vertical for the world-offset shortcut below)
        auto cand = [&](float cu, float cv, float dc, uint64_t ok) {
            const uint64_t take_lo = ok & (~have | lt_mask(cross2(lou, lov, cu, cv), 0.f));
            const uint64_t take_hi = ok & (~have | gt_mask(cross2(hiu, hiv, cu, cv), 0.f));
            lou = lane_in(take_lo) ? cu : lou;
            lov = lane_in(take_lo) ? cv : lov;
            hiu = lane_in(take_hi) ? cu : hiu;
            hiv = lane_in(take_hi) ? cv : hiv;
            if constexpr (kGrad) {
                dlo = lane_in(take_lo) ? dc : dlo;
                dhi = lane_in(take_hi) ? dc : dhi;
            }
            have |= ok;
        };
        const float e1h = g.e1z * h, e2h = g.e2z * h;
        // footprint vertex k relative to p: world offset (wx, wy), scaled
        // in-plane (u, v) and scaled height z of the plane above p there
        auto vertex = [&](int k, float &wx, float &wy, float &u, float &v, float &z) {
            const float4 q = ld(verts + voff + k);
            wx = q.x - px;
            wy = q.y - py;
            u = fmaf(g.m00, wx, g.m01 * wy);
            v = fmaf(g.m10, wx, g.m11 * wy);
            z = fmaf(g.e1z, u, g.e2z * v);
        };
        // edge from vertex A to vertex B (world offsets, scaled in-plane
        // coordinates and heights, below-roof masks); returns the lanes for
        // which the edge faces away from p
        auto edge = [&](float awx, float awy, float au, float av, float az, uint64_t ain, float bwx, float bwy,
                        float bu, float bv, float bz, uint64_t bin) -> uint64_t {
            const uint64_t back = ge_mask(cross2(awx, awy, bwx, bwy), 0.f);
            inside &= back;
            const uint64_t crossing = (ain ^ bin) & ballot(true);
            if (crossing) {
                const float rdz = __builtin_amdgcn_rcpf(bz - az);
                const float t = (hs - az) * rdz;
                const float cx = fmaf(t, bwx - awx, awx), cy = fmaf(t, bwy - awy, awy);
                const float cu = fmaf(g.e1x, cx, fmaf(g.e1y, cy, e1h));
                const float cv = fmaf(g.e2x, cx, fmaf(g.e2y, cy, e2h));
                float dc = 0.f;
                if constexpr (kGrad)
                    dc = cross2(cu, cv, bu - au, bv - av) * rdz * __builtin_amdgcn_rcpf(fmaf(cu, cu, cv * cv));
                cand(cu, cv, dc, crossing);
            }
            return back;
        };
        // kept vertices: candidates only at the silhouette (see the
        // world-offset branch below)
        auto vcand = [&](float u, float v, uint64_t in, uint64_t b_in, uint64_t b_out) {
            const uint64_t ok = in & (b_in ^ b_out);
            if (ok) cand(u, v, 0.f, ok);
        };
        // two vertices per trip, as in the world-offset branch below
        float awx, awy, au, av, az, bwx, bwy, bu, bv, bz;
        vertex(0, awx, awy, au, av, az);
        uint64_t ain = le_mask(az, hs);
        vertex(1, bwx, bwy, bu, bv, bz);
        uint64_t bin = le_mask(bz, hs);
        const uint64_t back0 = edge(awx, awy, au, av, az, ain, bwx, bwy, bu, bv, bz, bin);
        uint64_t bprev = back0;
        int e = 2;
        for (; e + 1 < m; e += 2) {
            vertex(e, awx, awy, au, av, az);
            ain = le_mask(az, hs);
            uint64_t back = edge(bwx, bwy, bu, bv, bz, bin, awx, awy, au, av, az, ain);
            vcand(bu, bv, bin, bprev, back);
            bprev = back;
            vertex(e + 1, bwx, bwy, bu, bv, bz);
            bin = le_mask(bz, hs);
            back = edge(awx, awy, au, av, az, ain, bwx, bwy, bu, bv, bz, bin);
            vcand(au, av, ain, bprev, back);
            bprev = back;
        }
        if (e < m) {  // one vertex left before the closing edge
            vertex(e, awx, awy, au, av, az);
            ain = le_mask(az, hs);
            const uint64_t back = edge(bwx, bwy, bu, bv, bz, bin, awx, awy, au, av, az, ain);
            vcand(bu, bv, bin, bprev, back);
            bprev = back;
            bwx = awx;
            bwy = awy;
            bu = au;
            bv = av;
            bz = az;
            bin = ain;
        }
        vertex(0, awx, awy, au, av, az);
        ain = le_mask(az, hs);
        const uint64_t bclose = edge(bwx, bwy, bu, bv, bz, bin, awx, awy, au, av, az, ain);
        vcand(bu, bv, bin, bprev, bclose);
        vcand(au, av, ain, bclose, back0);
    } else {
        // Without derivatives the extremes are found in world offsets from p:
        // the map M into the segment plane is linear, so it keeps the angular
        // order of directions (reverses it when det M < 0), and only the two
        // extremes are mapped at the end.  z, the plane's (scaled) height
        // above p at a footprint point, is linear in the offset too:
        // z = Z1 wx + Z2 wy.
        const float Z1 = fmaf(g.e1z, g.m00, g.e2z * g.m10), Z2 = fmaf(g.e1z, g.m01, g.e2z * g.m11);
        float lox = 0.f, loy = 0.f, hix = 0.f, hiy = 0.f;
        auto cand = [&](float cx, float cy, uint64_t ok) {
            const uint64_t take_lo = ok & (~have | lt_mask(cross2(lox, loy, cx, cy), 0.f));
            const uint64_t take_hi = ok & (~have | gt_mask(cross2(hix, hiy, cx, cy), 0.f));
            lox = lane_in(take_lo) ? cx : lox;
            loy = lane_in(take_lo) ? cy : loy;
            hix = lane_in(take_hi) ? cx : hix;
            hiy = lane_in(take_hi) ? cy : hiy;
            have |= ok;
        };
        auto vertex = [&](int k, float &wx, float &wy, float &z) {
            const float4 q = ld(verts + voff + k);
            wx = q.x - px;
            wy = q.y - py;
            z = fmaf(Z1, wx, Z2 * wy);
        };
        // Edge from vertex (ax, ay) (height az, below the roof line in the
        // lanes of ain) to vertex (bx, by, bz, bin); returns the lanes for
        // which the edge faces away from p (p on its inner side).
        auto edge = [&](float ax, float ay, float az, uint64_t ain, float bx, float by, float bz,
                        uint64_t bin) -> uint64_t {
            const uint64_t back = ge_mask(cross2(ax, ay, bx, by), 0.f);
            inside &= back;
            const uint64_t crossing = (ain ^ bin) & ballot(true);
            if (crossing) {
                const float t = (hs - az) * __builtin_amdgcn_rcpf(bz - az);
                cand(fmaf(t, bx - ax, ax), fmaf(t, by - ay, ay), crossing);
            }
            return back;
        };
        // Seen from p outside it, a convex polygon's extreme directions are
        // at its silhouette vertices, where the edge before and the edge
        // after face p differently.  The clipped polygon's edges at a kept
        // footprint vertex lie on the footprint's own edges, so a kept
        // vertex is a candidate only where the two footprint edges at it
        // disagree (the clip crossings are always candidates).  A vertex is
        // weighed once its outgoing edge is known; a vertex no lane needs
        // is skipped for the whole wave.
        auto vcand = [&](float x, float y, uint64_t in, uint64_t b_in, uint64_t b_out) {
            const uint64_t ok = in & (b_in ^ b_out);
            if (ok) cand(x, y, ok);
        };
        // Two vertices per trip (A, then B, then A again), so the previous
        // vertex never has to be copied between registers; vertex 0 is read
        // again for the closing edge rather than kept in registers.
        float ax, ay, az, bx, by, bz;
        vertex(0, ax, ay, az);
        uint64_t ain = le_mask(az, hs);
        vertex(1, bx, by, bz);
        uint64_t bin = le_mask(bz, hs);
        const uint64_t back0 = edge(ax, ay, az, ain, bx, by, bz, bin);  // edge 0 -> 1
        uint64_t bprev = back0;
        int e = 2;
        for (; e + 1 < m; e += 2) {
            vertex(e, ax, ay, az);
            ain = le_mask(az, hs);
            uint64_t back = edge(bx, by, bz, bin, ax, ay, az, ain);
            vcand(bx, by, bin, bprev, back);
            bprev = back;
            vertex(e + 1, bx, by, bz);
            bin = le_mask(bz, hs);
            back = edge(ax, ay, az, ain, bx, by, bz, bin);
            vcand(ax, ay, ain, bprev, back);
            bprev = back;
        }
        if (e < m) {  // one vertex left before the closing edge
            vertex(e, ax, ay, az);
            ain = le_mask(az, hs);
            const uint64_t back = edge(bx, by, bz, bin, ax, ay, az, ain);
            vcand(bx, by, bin, bprev, back);
            bprev = back;
            bx = ax;
            by = ay;
            bz = az;
            bin = ain;
        }
        vertex(0, ax, ay, az);
        ain = le_mask(az, hs);
        const uint64_t bclose = edge(bx, by, bz, bin, ax, ay, az, ain);  // edge m-1 -> 0
        vcand(bx, by, bin, bprev, bclose);
        vcand(ax, ay, ain, bclose, back0);
        const bool flip = fmaf(g.m00, g.m11, -g.m01 * g.m10) < 0.f;
        const float fx = flip ? hix : lox, fy = flip ? hiy : loy;
        const float gx = flip ? lox : hix, gy = flip ? loy : hiy;
        lou = fmaf(g.m00, fx, g.m01 * fy);
        lov = fmaf(g.m10, fx, g.m11 * fy);
        hiu = fmaf(g.m00, gx, g.m01 * gy);
        hiv = fmaf(g.m10, gx, g.m11 * gy);
    }
    da = db = 0.f;
    if (lane_in(inside)) {
        if (h < 0.f) return 0;
        a = w0;
        b = w1;
        return 1;
    }
    if (!lane_in(have)) return 0;
    const bool in0 = cross2(lou, lov, W0u, W0v) >= 0.f && cross2(W0u, W0v, hiu, hiv) >= 0.f;
    const bool in1 = cross2(lou, lov, W1u, W1v) >= 0.f && cross2(W1u, W1v, hiu, hiv) >= 0.f;
    float plo, phi;
    if (in0 && in1) {
        a = w0;
        b = w1;
        return 1;
    }
    if (in0) {
        a = w0;
        phi = polar_angle(hiu, hiv);
        b = fminf(fmaxf(phi, w0), w1);
        if constexpr (kGrad) db = (b == phi) ? dhi : 0.f;
        return 1;
    }
    if (in1) {
        plo = polar_angle(lou, lov);
        a = fminf(fmaxf(plo, w0), w1);
        if constexpr (kGrad) da = (a == plo) ? dlo : 0.f;
        b = w1;
        return 1;
    }
    const bool lo_in = cross2(W0u, W0v, lou, lov) >= 0.f && cross2(lou, lov, W1u, W1v) >= 0.f;
    if (!lo_in) return 0;
    plo = polar_angle(lou, lov);
    phi = polar_angle(hiu, hiv);
    a = fminf(fmaxf(plo, w0), w1);
    b = fminf(fmaxf(phi, w0), w1);
    if constexpr (kGrad) {
        da = (a == plo) ? dlo : 0.f;
        db = (b == phi) ? dhi : 0.f;
    }
    return 1;
}

// ---- interval set that also remembers, for every boundary, the prism
// whose interval end it is and that end's d(angle)/dH ----
struct UnionG {
    float lo[4], hi[4], dlo[4], dhi[4];
    int plo[4], phi[4];
    int n;
};

__device__ __forceinline__ void union_clear(UnionG &U)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        U.lo[i] = U.hi[i] = U.dlo[i] = U.dhi[i] = 0.f;
        U.plo[i] = U.phi[i] = -1;
    }
    U.n = 0;
}

// As union_insert; a merged boundary keeps the owner of the extreme end
// (equal ends: the lower prism index, -1 for the wall term first).
__device__ __forceinline__ bool union_insert(UnionG &U, float a, float b, int pa, int pb, float da, float db)
{
    int nb = 0, na = 0;
    float mlo = a, mhi = b, mdlo = da, mdhi = db;
    int mplo = pa, mphi = pb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool use = i < U.n;
        const bool before = use && U.hi[i] < a;
        const bool after = use && U.lo[i] > b;
        const bool ov = use && !before && !after;
        nb += before;
        na += after;
        const bool tlo = ov && (U.lo[i] < mlo || (U.lo[i] == mlo && U.plo[i] < mplo));
        const bool thi = ov && (U.hi[i] > mhi || (U.hi[i] == mhi && U.phi[i] < mphi));
        mlo = tlo ? U.lo[i] : mlo;
        mdlo = tlo ? U.dlo[i] : mdlo;
        mplo = tlo ? U.plo[i] : mplo;
        mhi = thi ? U.hi[i] : mhi;
        mdhi = thi ? U.dhi[i] : mdhi;
        mphi = thi ? U.phi[i] : mphi;
    }
    const int k = U.n - nb - na;
    const int nn = nb + 1 + na;
    if (nn > 4) return false;
    UnionG R;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int src = j - 1 + k;
        float slo = U.lo[0], shi = U.hi[0], sdlo = U.dlo[0], sdhi = U.dhi[0];
        int splo = U.plo[0], sphi = U.phi[0];
#pragma unroll
        for (int s = 1; s < 4; ++s) {
            const bool q = src == s;
            slo = q ? U.lo[s] : slo;
            shi = q ? U.hi[s] : shi;
            sdlo = q ? U.dlo[s] : sdlo;
            sdhi = q ? U.dhi[s] : sdhi;
            splo = q ? U.plo[s] : splo;
            sphi = q ? U.phi[s] : sphi;
        }
        const bool keep = j < nb, mid = j == nb;
        R.lo[j] = keep ? U.lo[j] : (mid ? mlo : slo);
        R.hi[j] = keep ? U.hi[j] : (mid ? mhi : shi);
        R.dlo[j] = keep ? U.dlo[j] : (mid ? mdlo : sdlo);
        R.dhi[j] = keep ? U.dhi[j] : (mid ? mdhi : sdhi);
        R.plo[j] = keep ? U.plo[j] : (mid ? mplo : splo);
        R.phi[j] = keep ? U.phi[j] : (mid ? mphi : sphi);
    }
    R.n = nn;
    U = R;
    return true;
}

// Facade point whose wall faces away from the sun: n . d(phi) <= 0 with
// d(phi) = cos(phi) e1 + sin(phi) e2.  Over a window narrower than pi the
// set is one interval.  W0, W1: the window's end directions in (u, v).
// Returns 0 or 1 with [a, b].
__device__ __forceinline__ int backface_interval(float nx, float ny, const SegConst &g, float w0, float w1,
                                                 float W0u, float W0v, float W1u, float W1v, float &a, float &b)
{
    const float A = fmaf(nx, g.e1x, ny * g.e1y), B = fmaf(nx, g.e2x, ny * g.e2y);
    const float f0 = fmaf(A, W0u, B * W0v), f1 = fmaf(A, W1u, B * W1v);
    const bool s0 = f0 <= 0.f, s1 = f1 <= 0.f;
    if (s0 && s1) {
        a = w0;
        b = w1;
        return 1;
    }
    if (!s0 && !s1) return 0;
    // zero of A cos + B sin inside the window (|phi| < pi/2 there, B != 0):
    // atan(-A / B), taken as the polar angle of (|B|, -A sign B)
    const float z = fminf(fmaxf(polar_angle(fabsf(B), B > 0.f ? -A : A), w0), w1);
    if (s0) {
        a = w0;
        b = z;
    } else {
        a = z;
        b = w1;
    }
    return 1;
}

// End directions of the window [w0, w1] of segment g in (u, v): exact
// constants for the whole segment, sincos only for sub-windows.
__device__ __forceinline__ void window_dirs(const SegConst &g, float w0, float w1, float &W0u, float &W0v,
                                            float &W1u, float &W1v)
{
    if (w0 == 0.f) {
        W0u = 1.f;
        W0v = 0.f;
    } else {
        sincos_small(w0, W0v, W0u);
    }
    if (w1 == g.theta) {
        W1u = g.cth;
        W1v = g.sth;
    } else {
        sincos_small(w1, W1v, W1u);
    }
}

struct PointArgs {
    int64_t n;
    const float *x, *y, *z, *nx, *ny;
    const int32_t *owner;
    const int32_t *rank;  // original id -> hierarchy position
    int32_t n_b;
};

struct LanePoint {
    float px, py, pz, nx, ny;
    int own;  // hierarchy position of the owner, -1 for ground points
};

__device__ __forceinline__ LanePoint load_point(const PointArgs &P, int64_t i, bool valid)
{
    LanePoint q{0.f, 0.f, 0.f, 0.f, 0.f, -1};
    if (valid) {
        q.px = P.x[i];
        q.py = P.y[i];
        q.pz = P.z[i];
        if (P.nx) q.nx = P.nx[i];
        if (P.ny) q.ny = P.ny[i];
        if (P.owner) {
            const int o = P.owner[i];
            q.own = (o >= 0 && o < P.n_b) ? P.rank[o] : -1;
        }
    }
    return q;
}

// A kernel argument parked in LDS and read back, wave-uniform, where a
// persistent loop needs it: the register allocator then has no reason to
// hold it in scalar registers across the traversal (where it would spill
// them to vector lanes and restore them on every node visit).  The volatile
// read keeps the compiler from hoisting the reload out of the loop.
typedef __attribute__((address_space(3))) int lds_int;

template <class T>
__device__ __forceinline__ void lds_park(lds_int *w, const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized objects");
    const int *s = (const int *)&v;
#pragma unroll
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) w[k] = s[k];
}

template <class T>
__device__ __forceinline__ T lds_uniform(const lds_int *w)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized objects");
    T r;
    int *d = (int *)&r;
    const volatile lds_int *p = w;
#pragma unroll
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) d[k] = __builtin_amdgcn_readfirstlane(p[k]);
    return r;
}

struct SpillArgs {
    int4 *out;          // queue to push to
    uint32_t *counter;  // its length
    uint32_t *overflow;
    int32_t cap;
};

__device__ __forceinline__ void spill_push(const SpillArgs &S, bool want, int64_t i, int j, float w0, float w1)
{
    if (!want) return;
    const uint32_t slot = atomicAdd(S.counter, 1u);
    if ((int32_t)slot < S.cap)
        S.out[slot] = make_int4((int)i, j, __float_as_int(w0), __float_as_int(w1));
    else
        atomicOr(S.overflow, 1u);
}

// Per-lane fan/box test of one segment: the fan of directions from p below
// height z1 projects on the ground to the triangle p, p + (z1 - pz) ua,
// p + (z1 - pz) ub (central projection maps the great-circle arc to a
// segment), so the box test is a 2D separating-axis test against that
// triangle: its bounding box and the normals of its two edges through p.
// (The third edge, at the far end, is left out: the bounding box already
// bounds the far end, and measured over the block scene the edge removes
// under 1% of the box hits for 23% of the test's arithmetic.)  For an edge
// with normal n the box point farthest along n is the corner picked by
// the signs of n, so max n.x over the box is
//     x1 max(nx,0) + x0 min(nx,0) + y1 max(ny,0) + y0 min(ny,0),
// a wave-uniform value (the box is the wave's node) compared with the
// lane's n.p.
// The fan of a segment seen from the xy plane: over the segment the rays
// from p sweep the wedge between the horizontal offsets ua (first knot) and
// ub (last knot), reaching (z - pz) * u at height z.  Returned: the
// per-metre reach box [umnx, umxx] x [umny, umxy] of the wedge and the two
// inward edge normals na (of p -> ua) and nb (of p -> ub).  Uniform per
// segment.
struct FanGeom {
    float umnx, umxx, umny, umxy;
    float nax, nay, nbx, nby;
};

__device__ __forceinline__ FanGeom fan_geom(const SegConst &g)
{
    FanGeom f;
    f.umnx = fminf(0.f, fminf(g.ua_x, g.ub_x));
    f.umxx = fmaxf(0.f, fmaxf(g.ua_x, g.ub_x));
    f.umny = fminf(0.f, fminf(g.ua_y, g.ub_y));
    f.umxy = fmaxf(0.f, fmaxf(g.ua_y, g.ub_y));
    f.nax = -g.ua_y;
    f.nay = g.ua_x;  // inward normal of p -> A (toward B)
    if (fmaf(f.nax, g.ub_x, f.nay * g.ub_y) < 0.f) {
        f.nax = -f.nax;
        f.nay = -f.nay;
    }
    f.nbx = -g.ub_y;
    f.nby = g.ub_x;  // inward normal of p -> B (toward A)
    if (fmaf(f.nbx, g.ua_x, f.nby * g.ua_y) < 0.f) {
        f.nbx = -f.nbx;
        f.nby = -f.nby;
    }
    return f;
}

// Largest value of n . x over the box [x0, x1] x [y0, y1] (the corner the
// normal points to), for a wedge edge normal n.
__device__ __forceinline__ float box_reach(float x0, float y0, float x1, float y1, float nx, float ny)
{
    return fmaf(y0, fminf(ny, 0.f), fmaf(y1, fmaxf(ny, 0.f), fmaf(x0, fminf(nx, 0.f), x1 * fmaxf(nx, 0.f))));
}

// Visit order of two child boxes in a segment: nearer along the
// horizontal direction of the mid-segment sun first.
__device__ __forceinline__ float seg_key(float x0, float y0, float x1, float y1, float mdx, float mdy)
{
    return fmaf(x0 + x1, mdx, (y0 + y1) * mdy);
}

// ---- the accrual fan test on per-segment node views ----
//
// A direct fan test of a child box (the wedge edges' box_reach against
// each lane's n . p, and the box against the fan's bounding box, whose
// corners move with the box top by the per-metre reach) spends most of its
// arithmetic on values that are the same for every lane.  CDNA has no
// scalar floating point, so those values would cost full vector
// instructions at every node visit.  Moving the lane's
// terms to the other side of each inequality,
//   x1 >= px + (z1 - pz) umnx   <=>   x1 - z1 umnx >= px - pz umnx,
// leaves one side that depends only on (segment, box), computed once per
// segment for the whole hierarchy (SegNode), and one that depends only on
// (segment, point), computed once per lane and segment (SegFan): a child
// test becomes seven compares.  Both sides are rounded outward, so the
// test passes every box that meets the fan exactly (boxes only decide
// what is tested, never a result).

typedef __attribute__((address_space(4))) const SegNode cSegNode;

__device__ __forceinline__ float round_up_rel(float v) { return v + fabsf(v) * 0x1p-22f; }
__device__ __forceinline__ float round_dn_rel(float v) { return v - fabsf(v) * 0x1p-22f; }

struct SegFan {
    float pz, cxl, cxh, cyl, cyh, naP, nbP;

    __device__ __forceinline__ SegFan(const SegConst &g, float px, float py, float pz_)
    {
        const FanGeom f = fan_geom(g);
        pz = pz_;
        cxl = round_dn_rel(fmaf(-pz, f.umnx, px));
        cxh = round_up_rel(fmaf(-pz, f.umxx, px));
        cyl = round_dn_rel(fmaf(-pz, f.umny, py));
        cyh = round_up_rel(fmaf(-pz, f.umxy, py));
        naP = fmaf(f.nax, px, f.nay * py);
        nbP = fmaf(f.nbx, px, f.nby * py);
    }

    __device__ __forceinline__ uint64_t operator()(const float *c) const
    {
        return ge_mask(c[0], pz) & ge_mask(c[1], cxl) & le_mask(c[2], cxh) & ge_mask(c[3], cyl) &
               le_mask(c[4], cyh) & ge_mask(c[5], naP) & ge_mask(c[6], nbP);
    }

    // Both children at once, for the lanes in cur.
    __device__ __forceinline__ void both(const SegNode &nd, uint64_t cur, uint64_t &h0, uint64_t &h1) const
    {
        uint64_t sv;
        asm volatile(
            "s_mov_b64 %[sv], exec\n"
            "s_mov_b64 exec, %[cur]\n"
            "v_cmpx_ge_f32 vcc, %[a0], %[pz]\n"
            "v_cmpx_ge_f32 vcc, %[a1], %[cxl]\n"
            "v_cmpx_le_f32 vcc, %[a2], %[cxh]\n"
            "v_cmpx_ge_f32 vcc, %[a3], %[cyl]\n"
            "v_cmpx_le_f32 vcc, %[a4], %[cyh]\n"
            "v_cmpx_ge_f32 vcc, %[a5], %[naP]\n"
            "v_cmpx_ge_f32 vcc, %[a6], %[nbP]\n"
            "s_mov_b64 %[h0], exec\n"
            "s_mov_b64 exec, %[cur]\n"
            "v_cmpx_ge_f32 vcc, %[b0], %[pz]\n"
            "v_cmpx_ge_f32 vcc, %[b1], %[cxl]\n"
            "v_cmpx_le_f32 vcc, %[b2], %[cxh]\n"
            "v_cmpx_ge_f32 vcc, %[b3], %[cyl]\n"
            "v_cmpx_le_f32 vcc, %[b4], %[cyh]\n"
            "v_cmpx_ge_f32 vcc, %[b5], %[naP]\n"
            "v_cmpx_ge_f32 vcc, %[b6], %[nbP]\n"
            "s_mov_b64 %[h1], exec\n"
            "s_mov_b64 exec, %[sv]\n"
            : [h0] "=&s"(h0), [h1] "=&s"(h1), [sv] "=&s"(sv)
            : [cur] "s"(cur), [pz] "v"(pz), [cxl] "v"(cxl), [cxh] "v"(cxh), [cyl] "v"(cyl), [cyh] "v"(cyh),
              [naP] "v"(naP), [nbP] "v"(nbP), [a0] "s"(nd.c[0][0]), [a1] "s"(nd.c[0][1]), [a2] "s"(nd.c[0][2]),
              [a3] "s"(nd.c[0][3]), [a4] "s"(nd.c[0][4]), [a5] "s"(nd.c[0][5]), [a6] "s"(nd.c[0][6]),
              [b0] "s"(nd.c[1][0]), [b1] "s"(nd.c[1][1]), [b2] "s"(nd.c[1][2]), [b3] "s"(nd.c[1][3]),
              [b4] "s"(nd.c[1][4]), [b5] "s"(nd.c[1][5]), [b6] "s"(nd.c[1][6])
            : "vcc");
    }
};

// The box-only side of SegFan's inequalities for one child box.  The
// shifted edges are formed in double and rounded outward; the wedge
// projections are box_reach.  An absent child gets a box no
// lane passes.
__device__ __forceinline__ void seg_child(const FanGeom &f, float x0, float y0, float x1, float y1, float z1,
                                          bool present, float *c)
{
    if (!present) {
        c[0] = -INFINITY;  // z1 >= pz fails for every finite pz
        c[1] = c[3] = c[5] = c[6] = -INFINITY;
        c[2] = c[4] = INFINITY;
        return;
    }
    c[0] = z1;
    c[1] = round_up_rel((float)((double)x1 - (double)z1 * f.umnx));
    c[2] = round_dn_rel((float)((double)x0 - (double)z1 * f.umxx));
    c[3] = round_up_rel((float)((double)y1 - (double)z1 * f.umny));
    c[4] = round_dn_rel((float)((double)y0 - (double)z1 * f.umxy));
    c[5] = box_reach(x0, y0, x1, y1, f.nax, f.nay);
    c[6] = box_reach(x0, y0, x1, y1, f.nbx, f.nby);
}

// Packet traversal over the per-segment views (see packet_traverse): the
// children of a view are already in the segment's visit order, interior
// references are byte offsets of views (one scalar load with a register
// offset, no address arithmetic), and a leaf reference's vertex range
// comes from the hierarchy-order offsets `voff`.
// Liveness is a wave mask throughout: `leaf(prim, voff, m, want)` returns
// the mask of lanes it retires, so no per-lane flag is carried around the
// loop (each such flag costs scalar merges with the exec mask at every
// iteration).  All leaf handling sits behind one branch, taken only at
// nodes with a leaf child.
// `root` is the byte offset of the view the walk starts at.
template <bool kCount, class LeafFn>
__device__ __forceinline__ void packet_traverse_seg(cSegNode *nodes, cint *voff, StackEntry *stack, uint64_t alive,
                                                    const SegFan &ft, LeafFn leaf, Work &w, int root = 0)
{
    typedef __attribute__((address_space(4))) const char cchar;
    uint64_t cur = alive;
    int sp = 0, node = root;  // byte offset of the current view
    while (cur) {
        const SegNode nd = ld((cSegNode *)((cchar *)nodes + (uint32_t)node));
        if constexpr (kCount) {
            w.box += lane_in(cur) ? 2u : 0u;
            w.nodes += first_active_lane() ? 1u : 0u;
        }
        uint64_t h0, h1;
        ft.both(nd, cur, h0, h1);
        if ((nd.ref[0] | nd.ref[1]) < 0) {
            uint64_t out = 0;
            if (nd.ref[0] < 0) {
                if (h0) {
                    const int prim = ~nd.ref[0];
                    const int v0 = ld(voff + prim), v1 = ld(voff + prim + 1);
                    out |= leaf(prim, v0, v1 - v0, h0);
                }
                h0 = 0;
            }
            if (nd.ref[1] < 0) {
                if (h1) {
                    const int prim = ~nd.ref[1];
                    const int v0 = ld(voff + prim), v1 = ld(voff + prim + 1);
                    out |= leaf(prim, v0, v1 - v0, h1);
                }
                h1 = 0;
            }
            alive &= ~out;
            h0 &= alive;
            h1 &= alive;
        }
        // both children wanted: defer the second; go to the first wanted
        const uint64_t defer = defer_mask(h0, h1);
        if (defer) {
            stack[sp] = StackEntry{nd.ref[1], (uint32_t)defer, (uint32_t)(defer >> 32), 0u};
            ++sp;
        }
        descend(h0, h1, nd.ref[0], nd.ref[1], node, cur);
        if (!cur) {
            const uint64_t keep = alive;
            while (sp > 0) {
                --sp;
                const StackEntry e = stack[sp];
                node = uniform(e.node);
                cur = uniform64(e.lo, e.hi) & keep;
                if (cur) break;
            }
        }
    }
}

}  // namespace dev
}  // namespace sa
