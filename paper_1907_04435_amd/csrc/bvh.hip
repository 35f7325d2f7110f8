// Device construction of the building hierarchy: footprint boxes, Morton
// codes of their centres, an LSD radix sort, the binary radix tree of the
// sorted codes (Karras, HPG 2012), and a bottom-up refit of the boxes with
// per-node arrival counters.  Every step runs on the GPU; the host only
// validates the input and sizes the buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "sa_internal.h"
#include "traverse.h"

namespace sa {
namespace {
using dev::pad_hi;
using dev::pad_lo;

constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;
constexpr int kSortTile = kSortThreads * kSortItems;

#define SA_HIP(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            err = std::string(#call) + ": " + hipGetErrorString(e_);        \
            return e_ == hipErrorOutOfMemory ? SA_ERR_OOM : SA_ERR_DEVICE;  \
        }                                                                   \
    } while (0)


__global__ void k_prism_box(int n_b, const int32_t *__restrict__ voff, const float2 *__restrict__ xy,
                            float4 *__restrict__ box)
{
    int b = wg_id() * wg_size() + tid();
    if (b >= n_b) return;
    float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int v = voff[b]; v < voff[b + 1]; ++v) {
        float2 p = xy[v];
        x0 = fminf(x0, p.x);
        y0 = fminf(y0, p.y);
        x1 = fmaxf(x1, p.x);
        y1 = fmaxf(y1, p.y);
    }
    box[b] = make_float4(x0, y0, x1, y1);
}

// One block: bounds of all footprint boxes and the largest height.
__global__ void k_bounds(int n_b, const float4 *__restrict__ box, const float *__restrict__ h,
                         float *__restrict__ out)
{
    __shared__ float red[5][1024];
    float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY, hm = 0.f;
    for (int b = tid(); b < n_b; b += wg_size()) {
        float4 q = box[b];
        x0 = fminf(x0, q.x);
        y0 = fminf(y0, q.y);
        x1 = fmaxf(x1, q.z);
        y1 = fmaxf(y1, q.w);
        hm = fmaxf(hm, h[b]);
    }
    red[0][tid()] = x0;
    red[1][tid()] = y0;
    red[2][tid()] = x1;
    red[3][tid()] = y1;
    red[4][tid()] = hm;
    __syncthreads();
    for (int s = wg_size() / 2; s > 0; s >>= 1) {
        if ((int)tid() < s) {
            red[0][tid()] = fminf(red[0][tid()], red[0][tid() + s]);
            red[1][tid()] = fminf(red[1][tid()], red[1][tid() + s]);
            red[2][tid()] = fmaxf(red[2][tid()], red[2][tid() + s]);
            red[3][tid()] = fmaxf(red[3][tid()], red[3][tid() + s]);
            red[4][tid()] = fmaxf(red[4][tid()], red[4][tid() + s]);
        }
        __syncthreads();
    }
    if (tid() < 5) out[tid()] = red[tid()][0];
}

__device__ inline uint32_t spread16(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// 32-bit Morton code of the footprint-box centre on a square 65536^2 grid
// over the scene (one scale for both axes keeps cells square).
__global__ void k_morton(int n_b, const float4 *__restrict__ box, const float *__restrict__ bounds,
                         uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    int b = wg_id() * wg_size() + tid();
    if (b >= n_b) return;
    float ext = fmaxf(fmaxf(bounds[2] - bounds[0], bounds[3] - bounds[1]), 1e-6f);
    float4 q = box[b];
    float cx = 0.5f * (q.x + q.z), cy = 0.5f * (q.y + q.w);
    float sx = (cx - bounds[0]) / ext * 65535.0f, sy = (cy - bounds[1]) / ext * 65535.0f;
    uint32_t ix = (uint32_t)fminf(fmaxf(sx, 0.f), 65535.f);
    uint32_t iy = (uint32_t)fminf(fmaxf(sy, 0.f), 65535.f);
    key[b] = spread16(ix) | (spread16(iy) << 1);
    val[b] = b;
}

// ---- LSD radix sort, 8-bit digits, stable ----
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(int n, int shift, int nblk,
                                                            const uint32_t *__restrict__ key,
                                                            uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[tid()] = 0;
    __syncthreads();
    for (int j = 0; j < kSortItems; ++j) {
        int i = wg_id() * kSortTile + j * kSortThreads + tid();
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[tid() * nblk + wg_id()] = h[tid()];
}

// Exclusive scan of m uint32 in place, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan_u32(int m, uint32_t *__restrict__ a)
{
    __shared__ uint32_t part[1024];
    int per = (m + 1023) / 1024;
    int lo = tid() * per, hi = min(lo + per, m);
    uint32_t s = 0;
    for (int i = lo; i < hi; ++i) s += a[i];
    part[tid()] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = tid() >= (unsigned)off ? part[tid() - off] : 0u;
        __syncthreads();
        part[tid()] += v;
        __syncthreads();
    }
    uint32_t run = part[tid()] - s;
    for (int i = lo; i < hi; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    int n, int shift, int nblk, const uint32_t *__restrict__ key_in, const int32_t *__restrict__ val_in,
    const uint32_t *__restrict__ hist, uint32_t *__restrict__ key_out, int32_t *__restrict__ val_out)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t cnt[kSortThreads / 64][256];
    const int lane = tid() & 63, wave = tid() >> 6;
    base[tid()] = hist[tid() * nblk + wg_id()];
    for (int w = 0; w < kSortThreads / 64; ++w) cnt[w][tid()] = 0;
    __syncthreads();
    for (int j = 0; j < kSortItems; ++j) {
        int i = wg_id() * kSortTile + j * kSortThreads + tid();
        bool valid = i < n;
        uint32_t k = valid ? key_in[i] : 0u;
        uint32_t dgt = (k >> shift) & 255u;
        unsigned long long eq = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            unsigned long long bb = __ballot((dgt >> b) & 1u);
            eq &= ((dgt >> b) & 1u) ? bb : ~bb;
        }
        unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        uint32_t r_wave = (uint32_t)__popcll(eq & below);
        if (valid && (__ffsll((long long)eq) - 1) == lane) cnt[wave][dgt] = (uint32_t)__popcll(eq);
        __syncthreads();
        if (valid) {
            uint32_t r = base[dgt] + r_wave;
            for (int w = 0; w < wave; ++w) r += cnt[w][dgt];
            key_out[r] = k;
            val_out[r] = val_in[i];
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) {
            tot += cnt[w][tid()];
            cnt[w][tid()] = 0;
        }
        base[tid()] += tot;
        __syncthreads();
    }
}

__global__ void k_scatter_rank(int n_b, const int32_t *__restrict__ order, int32_t *__restrict__ rank,
                               const int32_t *__restrict__ voff_in, uint32_t *__restrict__ m_sorted)
{
    int j = wg_id() * wg_size() + tid();
    if (j > n_b) return;
    if (j == n_b) {
        m_sorted[j] = 0;
        return;
    }
    int b = order[j];
    rank[b] = j;
    m_sorted[j] = (uint32_t)(voff_in[b + 1] - voff_in[b]);
}

// Prisms in hierarchy order; per vertex (x, y, ey, -ex) with e the edge to
// the next vertex: the outward normal of that edge for a CCW footprint.
__global__ void k_gather_prisms(int n_b, const int32_t *__restrict__ order,
                                const int32_t *__restrict__ voff_in, const float2 *__restrict__ xy,
                                const float *__restrict__ h_in, const float4 *__restrict__ box_in,
                                const uint32_t *__restrict__ voff_sorted, int32_t *__restrict__ voff,
                                float4 *__restrict__ verts, float *__restrict__ h, float4 *__restrict__ pbox)
{
    int j = wg_id() * wg_size() + tid();
    if (j > n_b) return;
    voff[j] = (int32_t)voff_sorted[j];
    if (j == n_b) return;
    int b = order[j];
    int o = voff_in[b], m = voff_in[b + 1] - o, d = (int)voff_sorted[j];
    for (int i = 0; i < m; ++i) {
        float2 a = xy[o + i], c = xy[o + (i + 1 == m ? 0 : i + 1)];
        verts[d + i] = make_float4(a.x, a.y, c.y - a.y, -(c.x - a.x));
    }
    h[j] = h_in[b];
    pbox[j] = box_in[b];
}

__device__ inline int karras_delta(const uint32_t *__restrict__ k, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    uint32_t a = k[i], b = k[j];
    if (a == b) return 32 + __clz((unsigned)(i ^ j));
    return __clz(a ^ b);
}

// Binary radix tree over sorted codes (ties broken by index), one thread
// per interior node.
__global__ void k_karras(int n, const uint32_t *__restrict__ key, const int32_t *__restrict__ voff,
                         Node *__restrict__ nodes, int32_t *__restrict__ parent)
{
    int i = wg_id() * wg_size() + tid();
    if (i >= n - 1) return;
    int d = (karras_delta(key, n, i, i + 1) - karras_delta(key, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = karras_delta(key, n, i, i - d);
    int lmax = 2;
    while (karras_delta(key, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (karras_delta(key, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = karras_delta(key, n, i, j);
    int s = 0, div = 2, t;
    do {
        t = (l + div - 1) / div;
        if (karras_delta(key, n, i, i + (s + t) * d) > dnode) s += t;
        div *= 2;
    } while (t > 1);
    int g = i + s * d + min(d, 0);
    int n_int = n - 1;
    Node &nd = nodes[i];
    if (min(i, j) == g) {
        nd.left = ~g;
        nd.l_voff = voff[g];
        nd.l_m = voff[g + 1] - voff[g];
        parent[n_int + g] = 2 * i;
    } else {
        nd.left = g;
        nd.l_voff = nd.l_m = 0;
        parent[g] = 2 * i;
    }
    if (max(i, j) == g + 1) {
        nd.right = ~(g + 1);
        nd.r_voff = voff[g + 1];
        nd.r_m = voff[g + 2] - voff[g + 1];
        parent[n_int + g + 1] = 2 * i + 1;
    } else {
        nd.right = g + 1;
        nd.r_voff = nd.r_m = 0;
        parent[g + 1] = 2 * i + 1;
    }
    if (i == 0) parent[0] = -1;
}

__device__ inline void put_box(Node *nd, int side, float x0, float y0, float x1, float y1, float z1)
{
    if (side == 0) {
        nd->lx0 = x0; nd->ly0 = y0; nd->lx1 = x1; nd->ly1 = y1; nd->lz1 = z1;
    } else {
        nd->rx0 = x0; nd->ry0 = y0; nd->rx1 = x1; nd->ry1 = y1; nd->rz1 = z1;
    }
}

// Bottom-up refit: each leaf writes its (padded) box into its parent's slot
// and arrives; the second arrival at a node merges both child boxes and
// carries on upward.  Release/acquire at device scope orders the box
// writes of one thread before the reads of the other, across XCDs.
__global__ void k_refit(int n_b, int n_int, const float4 *__restrict__ pbox, const float *__restrict__ h,
                        const int32_t *__restrict__ parent, Node *nodes, int32_t *flags)
{
    int j = wg_id() * wg_size() + tid();
    if (j >= n_b) return;
    float4 b = pbox[j];
    float x0 = pad_lo(b.x), y0 = pad_lo(b.y), x1 = pad_hi(b.z), y1 = pad_hi(b.w), z1 = pad_hi(h[j]);
    int pp = parent[n_int + j];
    while (pp >= 0) {
        int node = pp >> 1;
        put_box(&nodes[node], pp & 1, x0, y0, x1, y1, z1);
        int old = __hip_atomic_fetch_add(&flags[node], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0) return;
        const Node *nd = &nodes[node];
        x0 = fminf(nd->lx0, nd->rx0);
        y0 = fminf(nd->ly0, nd->ry0);
        x1 = fmaxf(nd->lx1, nd->rx1);
        y1 = fmaxf(nd->ly1, nd->ry1);
        z1 = fmaxf(nd->lz1, nd->rz1);
        pp = parent[node];
    }
}

// Heights from device arrays (original ids); bad entries are skipped and
// flagged (bit 2, reported by sa_sync).
__global__ void k_set_heights(int32_t n, const int32_t *__restrict__ ids, const float *__restrict__ h,
                              const int32_t *__restrict__ rank, int32_t n_b, float *height, uint32_t *flag)
{
    const int k = wg_id() * wg_size() + tid();
    if (k >= n) return;
    const int32_t id = ids[k];
    const float v = h[k];
    if (id < 0 || id >= n_b || !(v > 0.f) || !(v <= 3.0e38f)) {
        atomicOr(flag, 4u);
        return;
    }
    height[rank[id]] = v;
}

__global__ void k_clear_i32(int32_t *p, int32_t n)
{
    const int k = wg_id() * wg_size() + tid();
    if (k < n) p[k] = 0;
}

__global__ void k_depth(int n_b, int n_int, const int32_t *__restrict__ parent, int32_t *depth)
{
    int j = wg_id() * wg_size() + tid();
    if (j >= n_b) return;
    int d = 1, pp = parent[n_int + j];
    while (pp >= 0 && d < 4096) {
        ++d;
        pp = parent[pp >> 1];
    }
    atomicMax(depth, d);
}

// A single prism: one node whose right child is absent.
__global__ void k_single(const int32_t *__restrict__ voff, Node *nodes, int32_t *parent)
{
    Node &nd = nodes[0];
    nd.left = ~0;
    nd.l_voff = voff[0];
    nd.l_m = voff[1] - voff[0];
    nd.right = dev::kNone;
    nd.rx0 = nd.ry0 = nd.rz1 = -INFINITY;
    nd.rx1 = nd.ry1 = -INFINITY;
    nd.r_voff = nd.r_m = 0;
    parent[0] = -1;
    parent[1] = 0;
}

template <class T>
sa_status dalloc(T *&p, size_t n, std::string &err)
{
    if (hipMalloc((void **)&p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
        err = "device allocation failed";
        p = nullptr;
        return SA_ERR_OOM;
    }
    return SA_OK;
}

int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void scene_free(DeviceScene &s)
{
    (void)hipFree(s.nodes);
    (void)hipFree(s.verts);
    (void)hipFree(s.voff);
    (void)hipFree(s.height);
    (void)hipFree(s.order);
    (void)hipFree(s.rank);
    (void)hipFree(s.parent);
    (void)hipFree(s.flags);
    (void)hipFree(s.pbox);
    s = DeviceScene();
}

sa_status scene_set_heights_device(DeviceScene &s, int32_t n, const int32_t *ids, const float *h, uint32_t *flag,
                                   hipStream_t st, std::string &err)
{
    if (n <= 0 || s.n_b < 1) return SA_OK;
    hipLaunchKernelGGL(k_set_heights, dim3(blocks(n, 256)), dim3(256), 0, st, n, ids, h, (const int32_t *)s.rank,
                       s.n_b, s.height, flag);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

sa_status scene_refit(DeviceScene &s, hipStream_t st, std::string &err)
{
    if (s.n_b < 1) return SA_OK;
    if (s.n_b == 1) {
        hipLaunchKernelGGL(k_single, dim3(1), dim3(1), 0, st, s.voff, s.nodes, s.parent);
    }
    // arrival counters cleared by a fill kernel (capturable, unlike a memset node)
    hipLaunchKernelGGL(k_clear_i32, dim3(blocks(s.n_nodes, 256)), dim3(256), 0, st, s.flags, s.n_nodes);
    const int n_int = s.n_b == 1 ? 1 : s.n_b - 1;
    hipLaunchKernelGGL(k_refit, dim3(blocks(s.n_b, 256)), dim3(256), 0, st, s.n_b, n_int,
                       (const float4 *)s.pbox, (const float *)s.height, (const int32_t *)s.parent,
                       s.nodes, s.flags);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

sa_status scene_build(DeviceScene &s, hipStream_t st, int32_t n_b, const int32_t *voff_h,
                      const float *xy_h, const float *h_h, std::string &err)
{
    s = DeviceScene();
    s.n_b = n_b;
    if (n_b == 0) return SA_OK;
    const int n_vert = voff_h[n_b];
    s.n_vert = n_vert;
    s.n_nodes = n_b == 1 ? 1 : n_b - 1;
    sa_status rc;
    // raw input
    int32_t *voff_in = nullptr;
    float2 *xy_in = nullptr;
    float *h_in = nullptr;
    float4 *box_in = nullptr;
    uint32_t *keys[2] = {nullptr, nullptr}, *hist = nullptr, *m_sorted = nullptr;
    int32_t *vals[2] = {nullptr, nullptr}, *depth_d = nullptr;
    float *bounds_d = nullptr;
    const int nblk = blocks(n_b, kSortTile);
    auto cleanup = [&]() {
        (void)hipFree(voff_in); (void)hipFree(xy_in); (void)hipFree(h_in); (void)hipFree(box_in);
        (void)hipFree(keys[0]); (void)hipFree(keys[1]); (void)hipFree(vals[0]); (void)hipFree(vals[1]);
        (void)hipFree(hist); (void)hipFree(m_sorted); (void)hipFree(depth_d); (void)hipFree(bounds_d);
    };
#define SA_TRY(x)              \
    do {                       \
        rc = (x);              \
        if (rc != SA_OK) {     \
            cleanup();         \
            scene_free(s);     \
            return rc;         \
        }                      \
    } while (0)
    SA_TRY(dalloc(voff_in, n_b + 1, err));
    SA_TRY(dalloc(xy_in, n_vert, err));
    SA_TRY(dalloc(h_in, n_b, err));
    SA_TRY(dalloc(box_in, n_b, err));
    SA_TRY(dalloc(keys[0], n_b, err));
    SA_TRY(dalloc(keys[1], n_b, err));
    SA_TRY(dalloc(vals[0], n_b, err));
    SA_TRY(dalloc(vals[1], n_b, err));
    SA_TRY(dalloc(hist, (size_t)256 * nblk, err));
    SA_TRY(dalloc(m_sorted, n_b + 1, err));
    SA_TRY(dalloc(depth_d, 1, err));
    SA_TRY(dalloc(bounds_d, 8, err));
    SA_TRY(dalloc(s.nodes, s.n_nodes, err));
    SA_TRY(dalloc(s.verts, n_vert, err));
    SA_TRY(dalloc(s.voff, n_b + 1, err));
    SA_TRY(dalloc(s.height, n_b, err));
    SA_TRY(dalloc(s.order, n_b, err));
    SA_TRY(dalloc(s.rank, n_b, err));
    SA_TRY(dalloc(s.parent, s.n_nodes + n_b, err));
    SA_TRY(dalloc(s.flags, s.n_nodes, err));
    SA_TRY(dalloc(s.pbox, n_b, err));
#undef SA_TRY
    auto fail = [&](hipError_t e, const char *what) -> sa_status {
        err = std::string(what) + ": " + hipGetErrorString(e);
        cleanup();
        scene_free(s);
        return SA_ERR_DEVICE;
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(voff_in, voff_h, sizeof(int32_t) * (n_b + 1), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(xy_in, xy_h, sizeof(float) * 2 * n_vert, hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(h_in, h_h, sizeof(float) * n_b, hipMemcpyHostToDevice, st)) ||
        (e = hipMemsetAsync(s.nodes, 0, sizeof(Node) * s.n_nodes, st)) ||
        (e = hipMemsetAsync(depth_d, 0, sizeof(int32_t), st)))
        return fail(e, "scene upload copy");

    hipLaunchKernelGGL(k_prism_box, dim3(blocks(n_b, 256)), dim3(256), 0, st, n_b,
                       (const int32_t *)voff_in, (const float2 *)xy_in, box_in);
    hipLaunchKernelGGL(k_bounds, dim3(1), dim3(1024), 0, st, n_b, (const float4 *)box_in,
                       (const float *)h_in, bounds_d);
    hipLaunchKernelGGL(k_morton, dim3(blocks(n_b, 256)), dim3(256), 0, st, n_b, (const float4 *)box_in,
                       (const float *)bounds_d, keys[0], vals[0]);
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(kSortThreads), 0, st, n_b, shift, nblk,
                           (const uint32_t *)keys[cur], hist);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, 256 * nblk, hist);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(kSortThreads), 0, st, n_b, shift, nblk,
                           (const uint32_t *)keys[cur], (const int32_t *)vals[cur], (const uint32_t *)hist,
                           keys[cur ^ 1], vals[cur ^ 1]);
        cur ^= 1;
    }
    if ((e = hipMemcpyAsync(s.order, vals[cur], sizeof(int32_t) * n_b, hipMemcpyDeviceToDevice, st)))
        return fail(e, "order copy");
    hipLaunchKernelGGL(k_scatter_rank, dim3(blocks(n_b + 1, 256)), dim3(256), 0, st, n_b,
                       (const int32_t *)s.order, s.rank, (const int32_t *)voff_in, m_sorted);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, n_b + 1, m_sorted);
    hipLaunchKernelGGL(k_gather_prisms, dim3(blocks(n_b + 1, 256)), dim3(256), 0, st, n_b,
                       (const int32_t *)s.order, (const int32_t *)voff_in, (const float2 *)xy_in,
                       (const float *)h_in, (const float4 *)box_in, (const uint32_t *)m_sorted, s.voff,
                       s.verts, s.height, s.pbox);
    if (n_b > 1) {
        hipLaunchKernelGGL(k_karras, dim3(blocks(n_b - 1, 256)), dim3(256), 0, st, n_b,
                           (const uint32_t *)keys[cur], (const int32_t *)s.voff, s.nodes, s.parent);
    }
    if ((e = hipGetLastError())) return fail(e, "hierarchy kernels");
    rc = scene_refit(s, st, err);
    if (rc != SA_OK) {
        cleanup();
        scene_free(s);
        return rc;
    }
    const int n_int = n_b == 1 ? 1 : n_b - 1;
    hipLaunchKernelGGL(k_depth, dim3(blocks(n_b, 256)), dim3(256), 0, st, n_b, n_int,
                       (const int32_t *)s.parent, depth_d);
    float bh[8];
    if ((e = hipMemcpyAsync(bh, bounds_d, sizeof(float) * 5, hipMemcpyDeviceToHost, st)) ||
        (e = hipMemcpyAsync(&s.depth, depth_d, sizeof(int32_t), hipMemcpyDeviceToHost, st)) ||
        (e = hipStreamSynchronize(st)))
        return fail(e, "scene build");
    for (int i = 0; i < 4; ++i) s.bounds[i] = bh[i];
    s.max_h = bh[4];
    cleanup();
    // structural check of the tree before any traversal may use it: every
    // child reference in range, every node and leaf reached exactly once
    if (n_b > 1) {
        std::vector<Node> hn(s.n_nodes);
        if ((e = hipMemcpy(hn.data(), s.nodes, sizeof(Node) * s.n_nodes, hipMemcpyDeviceToHost))) {
            err = std::string("tree check copy: ") + hipGetErrorString(e);
            scene_free(s);
            return SA_ERR_DEVICE;
        }
        std::vector<int> seen_int(s.n_nodes, 0), seen_leaf(n_b, 0);
        bool ok = true;
        for (int i = 0; i < s.n_nodes && ok; ++i) {
            for (int c : {hn[i].left, hn[i].right}) {
                if (c >= 0) {
                    ok = ok && c < s.n_nodes && c != 0;
                    if (ok) ++seen_int[c];
                } else {
                    ok = ok && c != dev::kNone && ~c < n_b;
                    if (ok) ++seen_leaf[~c];
                }
            }
        }
        for (int i = 1; i < s.n_nodes && ok; ++i) ok = seen_int[i] == 1;
        for (int j = 0; j < n_b && ok; ++j) ok = seen_leaf[j] == 1;
        if (!ok) {
            err = "hierarchy construction produced an invalid tree";
            scene_free(s);
            return SA_ERR_DEVICE;
        }
    }
    if (s.depth > 63) {
        err = "hierarchy deeper than 63 levels";
        scene_free(s);
        return SA_ERR_CAPACITY;
    }
    return SA_OK;
}

}  // namespace sa
