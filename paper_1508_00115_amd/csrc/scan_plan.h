// Launch plan of the device-wide exclusive scan: the tile sums of every level
// laid out in one scratch buffer, and the grid of every launch. Plain C++ (no
// HIP), so the geometry can be checked on the host.
//
// A tile is SCAN_TILE consecutive elements, one 256-thread block. Level 0
// holds one sum per tile of the input, level k + 1 one sum per tile of level
// k; the last level fits one tile. The scan reduces down the levels, scans
// the last level in one block, then applies the scanned sums back up: the
// launch over level k (or over the input) takes one block per tile of it,
// and block b reads sum b of the level above.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace sph {

constexpr int SCAN_BS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_ITEMS;

inline int64_t scan_tiles(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

struct ScanLevel {
    int64_t offset;  // first word of the level in the scratch buffer
    int64_t count;   // sums it holds = tiles of the level below (or of the input)
};

struct ScanPlan {
    int64_t tiles = 0;            // tiles of the input: the grid of the first and last launch
    std::vector<ScanLevel> lv;    // empty when the input is one tile
    int64_t scratch_words = 0;    // words of scratch the levels need
};

inline ScanPlan scan_plan(int64_t n)
{
    ScanPlan P;
    P.tiles = n > 0 ? scan_tiles(n) : 0;
    if (P.tiles <= 1) return P;
    int64_t m = P.tiles;
    for (;;) {
        P.lv.push_back({P.scratch_words, m});
        P.scratch_words += m + 64;  // levels 256 bytes apart
        if (m <= SCAN_TILE) break;
        m = scan_tiles(m);
    }
    return P;
}

// Grid of the launch that applies the sums of level k + 1 to level k: one
// block per tile of level k (which is the number of sums level k + 1 holds).
inline int64_t scan_apply_grid(const ScanPlan& P, std::size_t k) { return scan_tiles(P.lv[k].count); }

// A plan of one level (at most SCAN_TILE tiles) takes two launches: the
// reduce, then the apply over the input, in which block b adds up the raw
// tile sums 0 .. b - 1 itself (they fit one block's pass) instead of reading
// sum b of a scanned level.
inline bool scan_one_level(const ScanPlan& P) { return P.lv.size() == 1; }

}  // namespace sph
