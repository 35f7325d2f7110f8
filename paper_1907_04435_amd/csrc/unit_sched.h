// Persistent launches of the per-tile kernels (accrual, sampled,
// continuous shadow, contributions, adjoint).
//
// Their work is a list of units (64-point tile, part) in tile-major order.
// A part is a run of the launch's items (segments or instants): one output
// bin's run, a fixed-size chunk, or all of them.  The units are cut into
// eight contiguous ranges, one per XCD (block b runs on XCD b mod 8), each
// with its own counter; a wave takes one unit per atomic from its XCD's
// range, then from the others'.  Neighbouring tiles share hierarchy nodes
// and prisms in their XCD's L2, and the waves stay resident until the work
// runs out: no SIMD idles behind a long tile, and a launch's tail is one
// unit long.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "sa_internal.h"
#include "traverse.h"

namespace sa {

constexpr int kSchedThreads = 256;               // threads per block of every persistent launch
constexpr int kSchedWaves = kSchedThreads / 64;  // waves per block
constexpr int kGrabStride = 32;                  // words between the eight counters (one 128-byte line each)

struct Sched {
    const int32_t *part_start;  // first item of each bin run of the launch (clipped to it), or null
    uint32_t *grab;             // eight counters, kGrabStride words apart, zero at launch
    uint32_t n_tiles;
    uint32_t n_parts;
    int32_t chunk;  // without part_start: items per part (0: one part, every item)
    int32_t sub;    // with part_start: equal pieces each run is cut into (0 or 1: whole runs)
};

namespace dev {

struct Unit {
    uint32_t tile;
    uint32_t part;
    int a, b;  // the unit's items [a, b)
};

// The next unit of the launch whose Sched is parked at s_W, for items
// [a0, a1); false when none is left.  k counts the XCD ranges already
// drained (0 at the start).  Callers pass the unit's bounds through
// uniform(): set inside this loop, they would otherwise count as per-lane
// values and could not address scalar loads.
__device__ __forceinline__ bool next_unit(const lds_int *s_W, int a0, int a1, int &k, Unit &un)
{
    const Sched W = lds_uniform<Sched>(s_W);
    const uint32_t n_units = W.n_tiles * W.n_parts;
    const int xcd = wg_id() & 7;
    for (; k < 8; ++k) {
        const int x = (xcd + k) & 7;
        const uint32_t lo = (uint32_t)((uint64_t)n_units * x >> 3);
        const uint32_t hi = (uint32_t)((uint64_t)n_units * (x + 1) >> 3);
        uint32_t got = 0;
        if ((tid() & 63) == 0) got = atomicAdd(W.grab + kGrabStride * x, 1u);
        got = (uint32_t)__builtin_amdgcn_readlane((int)got, 0);
        if (got < hi - lo) {
            const uint32_t u = lo + got;
            // the division runs on the vector unit: its result is made
            // scalar again for the scalar loads it addresses
            const uint32_t tile = (uint32_t)uniform((int)(u / W.n_parts));
            const uint32_t part = u - tile * W.n_parts;
            un.tile = tile;
            un.part = part;
            if (W.part_start) {
                const uint32_t sub = W.sub > 1 ? (uint32_t)W.sub : 1u;
                const uint32_t run = part / sub, piece = part - run * sub;
                const int ra = max(ld((cint *)W.part_start + run), a0);
                const int rb = min(ld((cint *)W.part_start + run + 1), a1);
                un.a = ra + (int)((int64_t)(rb - ra) * piece / sub);
                un.b = ra + (int)((int64_t)(rb - ra) * (piece + 1) / sub);
            } else if (W.chunk > 0) {
                un.a = a0 + (int)part * W.chunk;
                un.b = min(un.a + W.chunk, a1);
            } else {
                un.a = a0;
                un.b = a1;
            }
            return true;
        }
    }
    return false;
}

}  // namespace dev

// How a persistent launch may cut a tile's items into parts.
enum class Split {
    kNone,        // one part per tile
    kUniqueBins,  // a part per bin run when no bin has two runs in the launch
                  // (each (tile, bin) is then one unit's: plain stores)
    kBinRuns,     // a part per bin run (outputs added atomically)
    kChunks,      // parts of a fixed number of items, enough units to keep every
                  // wave busy (outputs added atomically)
    kRunPieces,   // as kUniqueBins, each run cut into equal pieces, enough units to
                  // keep every wave busy (per-piece sums, added in a fixed order after)
};

// Blocks of a persistent launch of `kern`: the tuned count, else as many
// as the device holds at once.
template <class Kern>
static int64_t resident_blocks(Kern kern, const TileLaunch &L)
{
    if (L.grid_blocks > 0) return L.grid_blocks;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kSchedThreads, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    return (int64_t)per_cu * std::max(L.n_cu, 1);
}

// The units of a persistent launch over items [a0, a1) (segments or
// instants, whose bin runs are R) for `tiles` 64-point tiles; `blocks` is
// the launch size (the chunk mode aims at eight units per wave).
static inline Sched plan_units(const BinRuns &R, int a0, int a1, int64_t tiles, Split split, int64_t blocks,
                               uint32_t *grab, int64_t max_parts = 1)
{
    Sched W{nullptr, grab, (uint32_t)tiles, 1u, 0, 0};
    if (split == Split::kNone || a1 <= a0) return W;
    if (split == Split::kChunks) {
        const int64_t items = a1 - a0;
        const int64_t want = std::max<int64_t>(1, (8 * blocks * kSchedWaves + tiles - 1) / tiles);
        int64_t parts = std::min(items, want);
        while (parts > 1 && (uint64_t)tiles * (uint64_t)parts >= (1ull << 31)) parts /= 2;
        const int64_t chunk = (items + parts - 1) / parts;
        W.chunk = (int32_t)chunk;
        W.n_parts = (uint32_t)((items + chunk - 1) / chunk);
        return W;
    }
    if (R.dev == nullptr || R.start.size() < 2) return W;
    const auto &rs = R.start;
    const int r0 = (int)(std::upper_bound(rs.begin(), rs.end(), a0) - rs.begin()) - 1;
    const int r1 = (int)(std::upper_bound(rs.begin(), rs.end(), a1 - 1) - rs.begin()) - 1;
    if ((r1 <= r0 && split != Split::kRunPieces) || (uint64_t)tiles * (uint64_t)(r1 - r0 + 1) >= (1ull << 31))
        return W;
    if (split == Split::kUniqueBins || split == Split::kRunPieces) {
        std::vector<int32_t> bins(R.bin.begin() + r0, R.bin.begin() + r1 + 1);
        std::sort(bins.begin(), bins.end());
        if (std::adjacent_find(bins.begin(), bins.end()) != bins.end()) return W;
    }
    W.part_start = R.dev + r0;
    const int64_t runs = r1 - r0 + 1;
    W.n_parts = (uint32_t)runs;
    if (split == Split::kRunPieces) {
        // pieces per run: eight units per resident wave, no piece shorter
        // than one item, no more parts than the caller can hold
        int shortest = a1 - a0;
        for (int r = r0; r <= r1; ++r) shortest = std::min(shortest, std::min(rs[r + 1], a1) - std::max(rs[r], a0));
        const int64_t want = (8 * blocks * kSchedWaves + tiles * runs - 1) / (tiles * runs);
        int64_t sub = std::min<int64_t>(std::min<int64_t>(want, shortest), std::max<int64_t>(1, max_parts / runs));
        while (sub > 1 && (uint64_t)tiles * (uint64_t)(runs * sub) >= (1ull << 31)) sub /= 2;
        if (sub > 1) {
            W.sub = (int32_t)sub;
            W.n_parts = (uint32_t)(runs * sub);
        }
    }
    return W;
}

// Blocks to launch: never more than the units need.
static inline int64_t unit_blocks(int64_t blocks, const Sched &W)
{
    const int64_t units = (int64_t)W.n_tiles * W.n_parts;
    return std::max<int64_t>(1, std::min<int64_t>(blocks, (units + kSchedWaves - 1) / kSchedWaves));
}

// Tiles of n points, refused beyond what the unit counters address.
static inline bool tile_count(int64_t n, int64_t &tiles, std::string &err)
{
    tiles = (n + 63) / 64;
    if (tiles >= (1ll << 31)) {
        err = "too many points";
        return false;
    }
    return true;
}

}  // namespace sa
