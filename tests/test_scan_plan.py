"""Host-side checks of the device-wide scan's launch geometry.

The scan that numbers tree nodes, leaves and neighbour lists runs over tile
sums in levels (csrc/scan_plan.h). A small C++ program, built here with g++
against that header, walks every launch the plan makes, block by block, and
checks that each block reads and writes only inside its input, its output and
its level of the scratch buffer; it also carries the plan out on the host
with bounds-checked arrays and compares the result with a plain exclusive
prefix sum. Lengths cover one tile, one level (two launches: each apply block adds up
the raw tile sums before it), the step to a second level
(more than 2048 * 2048 elements, where the apply launches once used one block
per element instead of one per tile and read past the scratch buffer) and the
largest particle count the library accepts."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1508_00115_amd", "csrc")

PROGRAM = r"""
#include "scan_plan.h"
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
using namespace sph;

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { ++fails; std::printf("FAIL n=%lld: ", (long long)n); \
    std::printf(__VA_ARGS__); std::printf("\n"); return; } } while (0)

// Block b of a reduce or apply launch over `count` elements touches elements
// [b * TILE, min(count, (b + 1) * TILE)) and sum b, unless b * TILE >= count
// (the kernels return at once then).
static void geometry(long long n)
{
    const ScanPlan P = scan_plan(n);
    CHECK(P.tiles == (n + SCAN_TILE - 1) / SCAN_TILE, "tiles");
    if (P.tiles <= 1) { CHECK(P.lv.empty(), "one tile needs no levels"); return; }
    CHECK(!P.lv.empty(), "levels missing");
    int64_t below = n;  // elements of the level below
    for (size_t k = 0; k < P.lv.size(); ++k) {
        const ScanLevel& L = P.lv[k];
        CHECK(L.count == scan_tiles(below), "level %zu count", k);
        CHECK(L.offset >= 0 && L.offset + L.count <= P.scratch_words, "level %zu outside scratch", k);
        if (k > 0) CHECK(L.offset >= P.lv[k - 1].offset + P.lv[k - 1].count, "levels overlap");
        // reduce launch producing level k: one block per tile below, block b writes sum b
        const int64_t grid = k == 0 ? P.tiles : P.lv[k].count;
        CHECK(grid == L.count, "reduce grid of level %zu", k);
        below = L.count;
    }
    CHECK(P.lv.back().count <= SCAN_TILE, "last level must fit one block");
    if (scan_one_level(P)) {
        // block b of the apply reads raw sums 0 .. b - 1, one pass of a block (SCAN_TILE words)
        CHECK(P.tiles <= SCAN_TILE && P.lv[0].count == P.tiles, "one-level plan beyond one block's pass");
        return;
    }
    for (size_t k = 0; k + 1 < P.lv.size(); ++k) {
        const int64_t grid = scan_apply_grid(P, k);
        // exactly one block per tile: a surplus block would read a sum past level k + 1
        CHECK(grid == scan_tiles(P.lv[k].count) && grid == P.lv[k + 1].count, "apply grid of level %zu is %lld",
              k, (long long)grid);
        for (int64_t b = 0; b < grid; ++b)
            if (b * SCAN_TILE < P.lv[k].count)
                CHECK(b < P.lv[k + 1].count, "apply of level %zu reads sum %lld of %lld", k, (long long)b,
                      (long long)P.lv[k + 1].count);
    }
    CHECK(P.tiles <= P.lv[0].count, "final apply reads past level 0");
}

// The plan carried out on the host (tile-by-tile exactly as the kernels do)
// against a plain exclusive prefix sum.
static void numeric(long long n, unsigned seed)
{
    const ScanPlan P = scan_plan(n);
    std::mt19937 rng(seed);
    std::vector<uint32_t> in(n), out(n), ref(n);
    for (auto& v : in) v = rng() % 3;
    uint32_t acc = 0;
    for (long long i = 0; i < n; ++i) { ref[i] = acc; acc += in[i]; }
    std::vector<uint32_t> scratch(P.scratch_words, 0xdeadbeefu);
    auto reduce = [&](const uint32_t* src, int64_t cnt, const ScanLevel& dst, int64_t grid) {
        for (int64_t b = 0; b < grid; ++b) {
            if (b * SCAN_TILE >= cnt) continue;
            uint32_t s = 0;
            for (int64_t i = b * SCAN_TILE; i < std::min<int64_t>(cnt, (b + 1) * SCAN_TILE); ++i) s += src[i];
            scratch.at(dst.offset + b) = s;
        }
    };
    auto apply = [&](const uint32_t* src, uint32_t* dst, int64_t cnt, const ScanLevel* sums, int64_t grid,
                     uint32_t* total) {
        for (int64_t b = 0; b < grid; ++b) {
            if (b * SCAN_TILE >= cnt) continue;
            uint32_t run = sums ? scratch.at(sums->offset + b) : 0u;
            for (int64_t i = b * SCAN_TILE; i < (b + 1) * SCAN_TILE; ++i) {
                const uint32_t v = i < cnt ? src[i] : 0u;
                if (i < cnt) dst[i] = run;
                run += v;
            }
            if (total && b == grid - 1) *total = run;
        }
    };
    uint32_t total = 0;
    if (P.lv.empty()) {
        apply(in.data(), out.data(), n, nullptr, 1, &total);
    } else if (scan_one_level(P)) {
        // two launches: block b of the apply adds the raw tile sums before it
        reduce(in.data(), n, P.lv[0], P.tiles);
        for (int64_t b = 0; b < P.tiles; ++b) {
            if (b * SCAN_TILE >= n) continue;
            uint32_t run = 0;
            for (int64_t t = 0; t < b; ++t) run += scratch.at(P.lv[0].offset + t);
            for (int64_t i = b * SCAN_TILE; i < (b + 1) * SCAN_TILE; ++i) {
                const uint32_t v = i < n ? in[i] : 0u;
                if (i < n) out[i] = run;
                run += v;
            }
            if (b == P.tiles - 1) total = run;
        }
    } else {
        reduce(in.data(), n, P.lv[0], P.tiles);
        for (size_t k = 1; k < P.lv.size(); ++k)
            reduce(scratch.data() + P.lv[k - 1].offset, P.lv[k - 1].count, P.lv[k], P.lv[k].count);
        const size_t top = P.lv.size() - 1;
        uint32_t* t = scratch.data() + P.lv[top].offset;
        apply(t, t, P.lv[top].count, nullptr, 1, nullptr);
        for (size_t k = top; k-- > 0;) {
            uint32_t* l = scratch.data() + P.lv[k].offset;
            apply(l, l, P.lv[k].count, &P.lv[k + 1], scan_apply_grid(P, k), nullptr);
        }
        apply(in.data(), out.data(), n, &P.lv[0], P.tiles, &total);
    }
    for (long long i = 0; i < n; ++i)
        if (out[i] != ref[i]) { ++fails; std::printf("FAIL n=%lld: element %lld\n", n, i); return; }
    if (total != acc) { ++fails; std::printf("FAIL n=%lld: total\n", n); }
}

int main()
{
    const long long T = SCAN_TILE;
    const long long geo[] = {1, 2, T - 1, T, T + 1, 3 * T + 5, T * T - 1, T * T, T * T + 1, 16777216,
                             T * T * 7 + 3, T * T * T - 1, T * T * T, T * T * T + 1, (1ll << 31) - 2};
    for (long long n : geo) geometry(n);
    const long long num[] = {1, 5, T - 1, T, T + 1, 5 * T + 17, T * T, T * T + 1, T * T + T + 3};
    unsigned seed = 1;
    for (long long n : num) numeric(n, seed++);
    std::printf("%s\n", fails ? "FAILED" : "OK");
    return fails ? 1 : 0;
}
"""


def test_scan_launch_geometry(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "scan_plan_check.cpp"
    exe = tmp_path / "scan_plan_check"
    src.write_text(PROGRAM)
    subprocess.run([gxx, "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("OK")
