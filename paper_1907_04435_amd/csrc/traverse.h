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

constexpr int kStackDepth = 64;

// Map a block index so that each XCD (blocks are dealt round-robin to the
// 8 XCDs) works on one contiguous range of tiles: neighbouring tiles share
// hierarchy nodes and prisms in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G)
{
    const int64_t x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Work a lane's own traversal needed (instrumented instantiations only).
struct Work {
    uint32_t box, prism, edges, inserts, nodes, units, spills;
};

__device__ __forceinline__ bool first_active_lane()
{
    const int lane = __lane_id();
    return __builtin_amdgcn_readfirstlane(lane) == lane;
}

// Packet traversal.  `bt(x0, y0, x1, y1, z1)` is the per-lane child-box
// test; `leaf(prim, voff, m, want)` processes a leaf for lanes with `want`
// and may clear `live`.  `key(x0,y0,x1,y1,z1)` orders two wanted children
// (smaller first).  The walk ends when no lane is live or the stack runs
// dry.  A lane only tests the children of nodes it reached itself (a
// per-lane bit per stack entry remembers whether the lane wanted the pushed
// node), so leaves no lane reached are skipped.  With kCount, `w`
// accumulates those box tests and the wave's node fetches.
template <bool kCount, class BoxTest, class LeafFn, class KeyFn>
__device__ __forceinline__ void packet_traverse(cNode *nodes, int *stack, bool &live, BoxTest bt, LeafFn leaf,
                                                KeyFn key, Work &w)
{
    int sp = 0, node = 0;
    bool want_cur = live;
    uint64_t want_stack = 0;
    while (ballot(live)) {
        const Node nd = ld(nodes + node);
        if constexpr (kCount) {
            w.box += (want_cur && live) ? 2u : 0u;
            w.nodes += first_active_lane() ? 1u : 0u;
        }
        const bool mine = live && want_cur;
        bool hl = mine && nd.left != kNone && bt(nd.lx0, nd.ly0, nd.lx1, nd.ly1, nd.lz1);
        bool hr = mine && nd.right != kNone && bt(nd.rx0, nd.ry0, nd.rx1, nd.ry1, nd.rz1);
        if (nd.left < 0 && nd.left != kNone) {
            if (ballot(hl)) leaf(~nd.left, nd.l_voff, nd.l_m, hl);
            hl = false;
        }
        if (nd.right < 0 && nd.right != kNone) {
            if (ballot(hr)) leaf(~nd.right, nd.r_voff, nd.r_m, hr);
            hr = false;
        }
        const bool gl = ballot(hl && live) != 0, gr = ballot(hr && live) != 0;
        if (gl && gr) {
            const bool lfirst = key(nd.lx0, nd.ly0, nd.lx1, nd.ly1, nd.lz1) <=
                                key(nd.rx0, nd.ry0, nd.rx1, nd.ry1, nd.rz1);
            stack[sp] = lfirst ? nd.right : nd.left;
            const bool far = lfirst ? hr : hl;
            want_stack = far ? (want_stack | (1ull << sp)) : (want_stack & ~(1ull << sp));
            want_cur = lfirst ? hl : hr;
            ++sp;
            node = uniform(lfirst ? nd.left : nd.right);
        } else if (gl) {
            want_cur = hl;
            node = uniform(nd.left);
        } else if (gr) {
            want_cur = hr;
            node = uniform(nd.right);
        } else {
            if (sp == 0) break;
            --sp;
            want_cur = (want_stack >> sp) & 1ull;
            node = uniform(stack[sp]);
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
        const float den = fmaf(v.z, dx, v.w * dy);
        const float s = num * __builtin_amdgcn_rcpf(den);
        if (den > 0.f) s_out = fminf(s_out, s);
        else if (den < 0.f) s_in = fmaxf(s_in, s);
        else if (num < 0.f) s_out = -INFINITY;
    }
    const float s0 = fmaxf(s_in, 0.f);
    return s_out >= s0 && fmaf(s0, dz, pz) <= H;
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
// is a convex polygon: the footprint (mapped by M to in-plane (u, v))
// clipped to heights <= H.  The directions from p that meet it form one
// angular interval of span < pi (p is outside); its ends are found by
// cross products over the clipped polygon's vertices (the kept footprint
// vertices and the two clip crossings), and intersected with the window.
// Returns 0: no overlap, 1: [a, b] written.
__device__ __forceinline__ int prism_interval(cfloat4 *verts, int voff, int m, float H, float px, float py,
                                              float pz, const SegConst &g, float w0, float w1, float W0u,
                                              float W0v, float W1u, float W1v, float &a, float &b)
{
    const float h = H - pz;
    bool have = false, inside = true;
    float lou = 0.f, lov = 0.f, hiu = 0.f, hiv = 0.f;
    float fu = 0.f, fv = 0.f, fz = 0.f, fwx = 0.f, fwy = 0.f;
    float pu = 0.f, pv = 0.f, pzv = 0.f, pwx = 0.f, pwy = 0.f;
    auto cand = [&](float cu, float cv, bool ok) {
        const bool first = ok && !have;
        const bool new_lo = ok && have && cross2(lou, lov, cu, cv) < 0.f;
        const bool new_hi = ok && have && cross2(hiu, hiv, cu, cv) > 0.f;
        lou = (first || new_lo) ? cu : lou;
        lov = (first || new_lo) ? cv : lov;
        hiu = (first || new_hi) ? cu : hiu;
        hiv = (first || new_hi) ? cv : hiv;
        have = have || ok;
    };
    for (int e = 0; e <= m; ++e) {
        float u, v, z, wx, wy;
        if (e < m) {
            const float4 q = ld(verts + voff + e);
            wx = q.x - px;
            wy = q.y - py;
            u = fmaf(g.m00, wx, g.m01 * wy);
            v = fmaf(g.m10, wx, g.m11 * wy);
            z = fmaf(g.e1z, u, g.e2z * v);
        } else {
            u = fu; v = fv; z = fz; wx = fwx; wy = fwy;
        }
        const bool in = z <= h;
        if (e == 0) {
            fu = u; fv = v; fz = z; fwx = wx; fwy = wy;
        } else {
            inside = inside && cross2(pwx, pwy, wx, wy) >= 0.f;
            const bool pin = pzv <= h;
            const float t = (h - pzv) * __builtin_amdgcn_rcpf(z - pzv);
            cand(fmaf(t, u - pu, pu), fmaf(t, v - pv, pv), pin != in);
        }
        if (e < m) cand(u, v, in);
        pu = u; pv = v; pzv = z; pwx = wx; pwy = wy;
    }
    if (inside) {
        if (h < 0.f) return 0;
        a = w0;
        b = w1;
        return 1;
    }
    if (!have) return 0;
    const bool in0 = cross2(lou, lov, W0u, W0v) >= 0.f && cross2(W0u, W0v, hiu, hiv) >= 0.f;
    const bool in1 = cross2(lou, lov, W1u, W1v) >= 0.f && cross2(W1u, W1v, hiu, hiv) >= 0.f;
    if (in0 && in1) {
        a = w0;
        b = w1;
        return 1;
    }
    if (in0) {
        a = w0;
        b = fminf(fmaxf(atan2f(hiv, hiu), w0), w1);
        return 1;
    }
    if (in1) {
        a = fminf(fmaxf(atan2f(lov, lou), w0), w1);
        b = w1;
        return 1;
    }
    const bool lo_in = cross2(W0u, W0v, lou, lov) >= 0.f && cross2(lou, lov, W1u, W1v) >= 0.f;
    if (!lo_in) return 0;
    a = fminf(fmaxf(atan2f(lov, lou), w0), w1);
    b = fminf(fmaxf(atan2f(hiv, hiu), w0), w1);
    return 1;
}

// Facade point whose wall faces away from the sun: n . d(phi) <= 0 with
// d(phi) = cos(phi) e1 + sin(phi) e2.  Over a window narrower than pi the
// set is one interval.  Returns 0 or 1 with [a, b].
__device__ __forceinline__ int backface_interval(float nx, float ny, const SegConst &g, float w0, float w1,
                                                 float &a, float &b)
{
    const float A = fmaf(nx, g.e1x, ny * g.e1y), B = fmaf(nx, g.e2x, ny * g.e2y);
    const float f0 = A * cosf(w0) + B * sinf(w0), f1 = A * cosf(w1) + B * sinf(w1);
    const bool s0 = f0 <= 0.f, s1 = f1 <= 0.f;
    if (s0 && s1) {
        a = w0;
        b = w1;
        return 1;
    }
    if (!s0 && !s1) return 0;
    // zero of A cos + B sin inside the window (|phi| < pi/2 there, B != 0)
    const float z = fminf(fmaxf(atanf(-A / B), w0), w1);
    if (s0) {
        a = w0;
        b = z;
    } else {
        a = z;
        b = w1;
    }
    return 1;
}

}  // namespace dev
}  // namespace sa
