// Gross shadow by raster shadow accrual maps (Sec. 4): per great-circle
// segment, a map of one depth slice per sample instant over a texel grid on
// a plane normal to the segment's start direction.  Step 1 fills every
// slice in one pass over (slice, prism) pairs: the depth at a texel is the
// largest distance along the light at which the ray from the texel centre
// toward the sun leaves a prism (its face nearest the sun).  Step 2 puts
// each point's shadow on every slice and counts the instants whose stored
// depth exceeds the point's own by more than the bias.  A map word holds an
// 8-bit segment stamp above a 24-bit depth (rounded down to a quantum of
// 1 / 2^24 of the segment's largest possible depth, about a millimetre for
// a city), so an integer maximum keeps the current segment's
// nearest-to-sun depth over any stale word, and the map is cleared only
// when it is allocated or after 255 segments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "sa_internal.h"

namespace sa {
namespace {

constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / 64;

__global__ void k_sam_clear(uint32_t *p, int64_t n)
{
    const int64_t stride = (int64_t)n_wg() * wg_size();
    for (int64_t t = (int64_t)wg_id() * wg_size() + tid(); t < n; t += stride) p[t] = 0u;
}

// One wave per (slice, prism): the wave covers the texels of the prism's
// shadow on the plane (the box of its vertices' projections, clamped to the
// grid) in 8 x 8 tiles, kTilesPerPass at a time in row order, each lane
// clipping the ray from its texel centre against the prism (height slab
// and every footprint edge's inner half-plane).  Within the box every
// clipping bound is an affine function of the texel's offset (i', j') from
// the box corner: the lanes first project one vertex each and form one
// edge's three coefficients each, then every pass reads an edge's
// coefficients from its lane and pays two FMAs and a min or max per texel.
// Depths are positive (the plane lies behind every prism) and quantised
// downward; with the segment's stamp above them a 32-bit integer maximum
// keeps the nearest-to-sun face of this segment.
constexpr int kTilesPerPass = 4;

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float lane_value(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

__global__ __launch_bounds__(kThreads) void k_sam_build(const float4 *__restrict__ verts,
                                                        const int32_t *__restrict__ voff,
                                                        const float *__restrict__ height, int n_b, SamGrid g,
                                                        const SamSlice *__restrict__ slices, int K,
                                                        uint32_t *__restrict__ map, uint32_t stamp)
{
    const int lane = tid() & 63;
    const int lx = lane & 7, ly = lane >> 3;
    const uint32_t tag = stamp << 24;
    const int64_t items = (int64_t)K * n_b;
    const int64_t T = (int64_t)g.nu * g.nv;
    const int64_t nw = (int64_t)n_wg() * kWavesPerBlock;
    const int64_t w0 = (int64_t)wg_id() * kWavesPerBlock + __builtin_amdgcn_readfirstlane(tid() >> 6);
    for (int64_t it = w0; it < items; it += nw) {
        const int k = (int)(it / n_b);
        const int b = (int)(it - (int64_t)k * n_b);
        const SamSlice s = slices[k];
        const int e0 = voff[b], ne = voff[b + 1] - e0;
        const float H = height[b];
        const float zlo = -g.oz, zhi = H - g.oz;
        // the prism's shadow: hull of its 2 x ne vertices' projections, a
        // vertex per lane
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        for (int c = 0; c < ne; c += 64) {
            if (c + lane < ne) {
                const float4 q = verts[e0 + c + lane];
                const float rx = q.x - g.ox, ry = q.y - g.oy;
#pragma unroll
                for (int top = 0; top < 2; ++top) {
                    const float rz = top ? zhi : zlo;
                    const float lam = (rx * g.ax + ry * g.ay + rz * g.az - g.c) * s.inv_da;
                    const float px = rx - lam * s.dx, py = ry - lam * s.dy, pz = rz - lam * s.dz;
                    const float pu = px * g.ux + py * g.uy + pz * g.uz;
                    const float pv = px * g.vx + py * g.vy + pz * g.vz;
                    umin = fminf(umin, pu);
                    umax = fmaxf(umax, pu);
                    vmin = fminf(vmin, pv);
                    vmax = fmaxf(vmax, pv);
                }
            }
        }
        umin = wave_min(umin);
        umax = wave_max(umax);
        vmin = wave_min(vmin);
        vmax = wave_max(vmax);
        // a centimetre of slack against the rounding of the projections;
        // clamped in float before the conversion to integers
        const float fi0 = fmaxf(floorf((umin - 0.01f - g.u0) * g.inv_h), 0.f);
        const float fi1 = fminf(floorf((umax + 0.01f - g.u0) * g.inv_h), (float)(g.nu - 1));
        const float fj0 = fmaxf(floorf((vmin - 0.01f - g.v0) * g.inv_h), 0.f);
        const float fj1 = fminf(floorf((vmax + 0.01f - g.v0) * g.inv_h), (float)(g.nv - 1));
        if (!(fi0 <= fi1 && fj0 <= fj1)) continue;
        const int i0 = __builtin_amdgcn_readfirstlane((int)fi0), j0 = __builtin_amdgcn_readfirstlane((int)fj0);
        const int W = __builtin_amdgcn_readfirstlane((int)fi1) - i0 + 1;
        const int Hh = __builtin_amdgcn_readfirstlane((int)fj1) - j0 + 1;
        const int tx_n = (W + 7) >> 3, ty_n = (Hh + 7) >> 3;
        uint32_t *slice = map + (int64_t)k * T;
        // the ray from the centre of texel (i0 + i', j0 + j'):
        // X0 + i' h u + j' h v + lam d
        const float cu0 = g.u0 + ((float)i0 + 0.5f) * g.h, cv0 = g.v0 + ((float)j0 + 0.5f) * g.h;
        const float X0 = g.c * g.ax + cu0 * g.ux + cv0 * g.vx;
        const float Y0 = g.c * g.ay + cu0 * g.uy + cv0 * g.vy;
        const float Z0 = g.c * g.az + cu0 * g.uz + cv0 * g.vz;
        // height slab: lam in [(zlo - Z) / dz, (zhi - Z) / dz]; the sun is
        // above the horizon (dz > 0)
        const float inv_dz = 1.f / s.dz;
        const float zl0 = (zlo - Z0) * inv_dz, zh0 = (zhi - Z0) * inv_dz;
        const float zi = -g.h * g.uz * inv_dz, zj = -g.h * g.vz * inv_dz;
        const int n_tiles = tx_n * ty_n;
        const float fi = (float)lx, fj = (float)ly;
        const float zl = fmaf(zj, fj, fmaf(zi, fi, zl0)), zh = fmaf(zj, fj, fmaf(zi, fi, zh0));
        // edge c + lane: along the ray its inner-side function is
        // f0 + fu i' + fv j' + lam gd (n.(x - p0) with n the outward normal;
        // inside where <= 0).  kind 1: gd > 0, the crossing
        // lam = A + B i' + C j' bounds lam from above; kind -1: from below;
        // kind 0: parallel, (A, B, C) = (f0, fu, fv) must stay <= 0.
        auto edge_coef = [&](int c, float &eA, float &eB, float &eC, int &kind) {
            eA = eB = eC = 0.f;
            kind = 0;
            if (c + lane < ne) {
                const float4 q = verts[e0 + c + lane];
                const float f0 = q.z * (X0 - (q.x - g.ox)) + q.w * (Y0 - (q.y - g.oy));
                const float fu = g.h * (q.z * g.ux + q.w * g.uy), fv = g.h * (q.z * g.vx + q.w * g.vy);
                const float gd = q.z * s.dx + q.w * s.dy;
                if (gd != 0.f) {
                    const float rg = -1.f / gd;
                    eA = f0 * rg;
                    eB = fu * rg;
                    eC = fv * rg;
                    kind = gd > 0.f ? 1 : -1;
                } else {
                    eA = f0;
                    eB = fu;
                    eC = fv;
                }
            }
        };
        float eA0, eB0, eC0;
        int kind0;
        edge_coef(0, eA0, eB0, eC0, kind0);  // the first 64 edges, once per (slice, prism)
        for (int t0 = 0; t0 < n_tiles; t0 += kTilesPerPass) {
            // the pass's tiles in row order: offsets (in texels) of each
            // tile's corner, the same for every lane
            float ox[kTilesPerPass], oy[kTilesPerPass];
            int tx = t0 % tx_n, ty = t0 / tx_n;
#pragma unroll
            for (int r = 0; r < kTilesPerPass; ++r) {
                ox[r] = (float)(8 * tx);
                oy[r] = (float)(8 * ty);
                if (++tx == tx_n) {
                    tx = 0;
                    ++ty;
                }
            }
            float lo[kTilesPerPass], hi[kTilesPerPass];
#pragma unroll
            for (int r = 0; r < kTilesPerPass; ++r) {
                lo[r] = fmaxf(0.f, fmaf(zj, oy[r], fmaf(zi, ox[r], zl)));
                hi[r] = fmaf(zj, oy[r], fmaf(zi, ox[r], zh));
            }
            for (int c = 0; c < ne; c += 64) {
                float eA = eA0, eB = eB0, eC = eC0;
                int kind = kind0;
                if (c > 0) edge_coef(c, eA, eB, eC, kind);  // footprints beyond 64 vertices
                const int m_n = min(64, ne - c);
                for (int m = 0; m < m_n; ++m) {
                    const float A = lane_value(eA, m), B = lane_value(eB, m), Cv = lane_value(eC, m);
                    const int kd = __builtin_amdgcn_readlane(kind, m);
                    const float base = fmaf(B, fi, fmaf(Cv, fj, A));
                    if (kd > 0) {
#pragma unroll
                        for (int r = 0; r < kTilesPerPass; ++r)
                            hi[r] = fminf(hi[r], fmaf(Cv, oy[r], fmaf(B, ox[r], base)));
                    } else if (kd < 0) {
#pragma unroll
                        for (int r = 0; r < kTilesPerPass; ++r)
                            lo[r] = fmaxf(lo[r], fmaf(Cv, oy[r], fmaf(B, ox[r], base)));
                    } else {
                        // parallel to the edge: outside it, no hit
#pragma unroll
                        for (int r = 0; r < kTilesPerPass; ++r)
                            if (fmaf(Cv, oy[r], fmaf(B, ox[r], base)) > 0.f) lo[r] = INFINITY;
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < kTilesPerPass; ++r) {
                const int ii = (int)ox[r] + lx, jj = (int)oy[r] + ly;
                if (t0 + r < n_tiles && ii < W && jj < Hh && lo[r] <= hi[r])
                    atomicMax(slice + (int64_t)(j0 + jj) * g.nu + (i0 + ii),
                              tag | (uint32_t)fminf(hi[r] * g.inv_dq, 16777215.f));
            }
        }
    }
}

// One thread per point: its shadow on each slice, the stored depth there
// (if written for this segment) against its own depth plus the bias; the
// segment's counts and minutes added to the point's bin.
__global__ __launch_bounds__(kThreads) void k_sam_query(const float *__restrict__ px, const float *__restrict__ py,
                                                        const float *__restrict__ pz, int64_t n, SamGrid g,
                                                        const SamSlice *__restrict__ slices, int K,
                                                        const uint32_t *__restrict__ map, uint32_t stamp,
                                                        int bin, float scale,
                                                        int32_t *__restrict__ counts, float *__restrict__ minutes)
{
    const int64_t T = (int64_t)g.nu * g.nv;
    const int64_t stride = (int64_t)n_wg() * wg_size();
    for (int64_t i = (int64_t)wg_id() * wg_size() + tid(); i < n; i += stride) {
        const float rx = px[i] - g.ox, ry = py[i] - g.oy, rz = pz[i] - g.oz;
        const float ra = rx * g.ax + ry * g.ay + rz * g.az - g.c;
        int cnt = 0;
        float mins = 0.f;
        for (int k = 0; k < K; ++k) {
            const SamSlice s = slices[k];
            const float lam = ra * s.inv_da;
            const float qx = rx - lam * s.dx, qy = ry - lam * s.dy, qz = rz - lam * s.dz;
            const float fu = floorf((qx * g.ux + qy * g.uy + qz * g.uz - g.u0) * g.inv_h);
            const float fv = floorf((qx * g.vx + qy * g.vy + qz * g.vz - g.v0) * g.inv_h);
            if (fu >= 0.f && fu < (float)g.nu && fv >= 0.f && fv < (float)g.nv) {
                // a word of an earlier segment (another stamp) is empty here
                const uint32_t m = map[(int64_t)k * T + (int64_t)fv * g.nu + (int64_t)fu];
                if ((m >> 24) == stamp && (float)(m & 0xffffffu) * g.dq > lam + g.bias) {
                    ++cnt;
                    mins += s.w;
                }
            }
        }
        if (counts) counts[(int64_t)bin * n + i] += cnt;
        if (minutes) minutes[(int64_t)bin * n + i] += mins * scale;
    }
}

// Plane and grid of one segment, FP64 (the float32 copy is relative to o):
// normal a; u = z x a normalised (east at the zenith), v = a x u; the plane
// 1 m behind the box corner farthest from the sun; the grid covers the
// box's projections along a and b (those along every direction between them
// lie in between) with a texel of margin.
bool sam_grid(const double box[6], const double *a, const double *b, double h, double bias, SamGrid &g)
{
    double u[3] = {-a[1], a[0], 0.0};
    const double ul = std::sqrt(u[0] * u[0] + u[1] * u[1]);
    if (ul > 1e-9) {
        u[0] /= ul;
        u[1] /= ul;
    } else {
        u[0] = 1.0;
        u[1] = 0.0;
    }
    const double v[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2], a[0] * u[1] - a[1] * u[0]};
    double c = INFINITY;
    double X[8][3];
    for (int q = 0; q < 8; ++q) {
        X[q][0] = box[(q & 4) ? 3 : 0];
        X[q][1] = box[(q & 2) ? 4 : 1];
        X[q][2] = box[(q & 1) ? 5 : 2];
        c = std::min(c, X[q][0] * a[0] + X[q][1] * a[1] + X[q][2] * a[2]);
    }
    c -= 1.0;
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    for (const double *d : {a, b}) {
        const double da = d[0] * a[0] + d[1] * a[1] + d[2] * a[2];
        for (int q = 0; q < 8; ++q) {
            const double lam = (X[q][0] * a[0] + X[q][1] * a[1] + X[q][2] * a[2] - c) / da;
            const double p[3] = {X[q][0] - lam * d[0], X[q][1] - lam * d[1], X[q][2] - lam * d[2]};
            const double pu = p[0] * u[0] + p[1] * u[1] + p[2] * u[2];
            const double pv = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
            umin = std::min(umin, pu);
            umax = std::max(umax, pu);
            vmin = std::min(vmin, pv);
            vmax = std::max(vmax, pv);
        }
    }
    const double u0 = std::floor(umin / h) * h - h, v0 = std::floor(vmin / h) * h - h;
    const double nu = std::ceil((umax - u0) / h) + 1.0, nv = std::ceil((vmax - v0) / h) + 1.0;
    if (!(nu >= 1.0 && nv >= 1.0 && nu < 2e9 && nv < 2e9)) return false;
    const double o[3] = {0.5 * (box[0] + box[3]), 0.5 * (box[1] + box[4]), 0.5 * (box[2] + box[5])};
    g.ax = (float)a[0];
    g.ay = (float)a[1];
    g.az = (float)a[2];
    g.ux = (float)u[0];
    g.uy = (float)u[1];
    g.uz = (float)u[2];
    g.vx = (float)v[0];
    g.vy = (float)v[1];
    g.vz = (float)v[2];
    g.c = (float)(c - (o[0] * a[0] + o[1] * a[1] + o[2] * a[2]));
    g.u0 = (float)(u0 - (o[0] * u[0] + o[1] * u[1] + o[2] * u[2]));
    g.v0 = (float)(v0 - (o[0] * v[0] + o[1] * v[1] + o[2] * v[2]));
    g.h = (float)h;
    g.inv_h = (float)(1.0 / h);
    g.nu = (int32_t)nu;
    g.nv = (int32_t)nv;
    g.ox = (float)o[0];
    g.oy = (float)o[1];
    g.oz = (float)o[2];
    g.bias = (float)bias;
    // every slice direction d lies on the arc from a to b, so d.a >= a.b and
    // no depth exceeds (max corner.a - c) / (a.b); 1 % of slack
    double cmax = -INFINITY;
    for (int q = 0; q < 8; ++q) cmax = std::max(cmax, X[q][0] * a[0] + X[q][1] * a[1] + X[q][2] * a[2]);
    const double ab = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    if (!(ab > 0.0)) return false;
    const double lam_max = 1.01 * (cmax - c) / ab;
    g.dq = (float)(lam_max / 16777215.0);
    g.inv_dq = (float)(16777215.0 / lam_max);
    return true;
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

sa_status launch_sam(const DeviceScene &s, const DevicePath &p, const PointsView &pts, double texel,
                     double bias, const double box[6], int64_t max_texels, float scale, int32_t *counts,
                     float *minutes, Scratch &scr, uint32_t &stamp, hipStream_t st, std::string &err)
{
    if (s.n_b == 0 || pts.n == 0 || p.n_samples == 0) return SA_OK;
    if (!p.sam_slices || p.seg_host.size() != (size_t)p.n_segs) {
        err = "sa_sam_accumulate: path has no raster slices";
        return SA_ERR_INVALID_ARG;
    }
    // every segment's grid first: the map buffer is sized for the largest
    std::vector<SamGrid> grids(p.seg_host.size());
    int64_t most = 0;
    for (size_t j = 0; j < p.seg_host.size(); ++j) {
        const SamSegHost &sh = p.seg_host[j];
        if (sh.ns == 0) continue;
        if (!sam_grid(box, sh.a, sh.b, texel, bias, grids[j])) {
            err = "sa_sam_accumulate: texel grid out of range";
            return SA_ERR_CAPACITY;
        }
        // in floating point first: nu * nv * ns may not fit 64 bits
        const double texels = (double)grids[j].nu * (double)grids[j].nv * (double)sh.ns;
        if (texels > (double)max_texels) {
            err = "sa_sam_accumulate: a segment's map needs " + std::to_string(texels) +
                  " texels, above the cap (larger texels, or a higher cap)";
            return SA_ERR_CAPACITY;
        }
        most = std::max(most, (int64_t)grids[j].nu * grids[j].nv * sh.ns);
    }
    const size_t need = (size_t)most * sizeof(uint32_t);
    auto clear_all = [&]() {
        const int64_t words = (int64_t)(scr.bytes / sizeof(uint32_t));
        hipLaunchKernelGGL(k_sam_clear, dim3((unsigned)std::min<int64_t>((words + kThreads - 1) / kThreads, 65536)),
                           dim3(kThreads), 0, st, (uint32_t *)scr.ptr, words);
        stamp = 0;
    };
    if (scr.bytes < need) {
        // the previous contents may still be read by queued kernels
        (void)hipStreamSynchronize(st);
        (void)hipFree(scr.ptr);
        scr.ptr = nullptr;
        scr.bytes = 0;
        if (hipMalloc(&scr.ptr, need) != hipSuccess) {
            (void)hipGetLastError();
            err = "raster map allocation failed";
            return SA_ERR_OOM;
        }
        scr.bytes = need;
        clear_all();
        SA_CHECK_LAUNCH("raster map clear");
    }
    uint32_t *map = (uint32_t *)scr.ptr;
    const unsigned qblocks = (unsigned)std::min<int64_t>((pts.n + kThreads - 1) / kThreads, 16384);
    for (size_t j = 0; j < p.seg_host.size(); ++j) {
        const SamSegHost &sh = p.seg_host[j];
        if (sh.ns == 0) continue;
        const SamGrid &g = grids[j];
        const SamSlice *sl = p.sam_slices + sh.first;
        if (stamp >= 255u) {
            clear_all();
            SA_CHECK_LAUNCH("raster map clear");
        }
        ++stamp;
        const int64_t items = (int64_t)sh.ns * s.n_b;
        hipLaunchKernelGGL(k_sam_build,
                           dim3((unsigned)std::min<int64_t>((items + kWavesPerBlock - 1) / kWavesPerBlock, 32768)),
                           dim3(kThreads), 0, st, (const float4 *)s.verts, (const int32_t *)s.voff,
                           (const float *)s.height, s.n_b, g, sl, sh.ns, map, stamp);
        SA_CHECK_LAUNCH("raster map build");
        hipLaunchKernelGGL(k_sam_query, dim3(qblocks), dim3(kThreads), 0, st, pts.x, pts.y, pts.z, pts.n, g, sl,
                           sh.ns, (const uint32_t *)map, stamp, sh.bin, scale, counts, minutes);
        SA_CHECK_LAUNCH("raster map query");
    }
    return SA_OK;
}

}  // namespace sa
