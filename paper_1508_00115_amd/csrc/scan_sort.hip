// Device-wide exclusive scan and stable LSD radix sort used by the cell build.
//
// Both work on wave64 primitives: lane-shuffle scans inside a wavefront and
// ballot-based digit matching for the sort's stable local ranking.
#include "common.h"
#include "scan_plan.h"

#include <algorithm>

namespace {

using sph::SCAN_BS;
using sph::SCAN_ITEMS;
using sph::SCAN_TILE;

// Inclusive scan inside one wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan over a 256-thread block; returns the block total in *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds4, uint32_t& total)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds4[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BS / 64; ++k) {
        uint32_t t = lds4[k];
        if (k < w) base += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

__global__ void __launch_bounds__(SCAN_BS) k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                         uint32_t* __restrict__ sums)
{
    __shared__ uint32_t lds4[4];
    if ((int64_t)blockIdx.x * SCAN_TILE >= n) return;  // whole block: no tile here
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, lds4, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scans each tile and adds the scanned tile offset. sums may be null when there
// is a single tile. With raw_sums > 0, sums holds the raw sums of the
// raw_sums (<= SCAN_TILE) tiles, and block b adds up sums 0 .. b - 1 itself.
// Writes the grand total from the last tile.
__global__ void __launch_bounds__(SCAN_BS) k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                        const uint32_t* __restrict__ sums,
                                                        uint32_t* __restrict__ total, int64_t raw_sums)
{
    __shared__ uint32_t lds4[4];
    if ((int64_t)blockIdx.x * SCAN_TILE >= n) return;  // whole block: no tile, no sum to read
    uint32_t tile_off = 0;
    if (raw_sums > 0) {
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const int64_t t = (int64_t)threadIdx.x * SCAN_ITEMS + k;
            if (t < (int64_t)blockIdx.x && t < raw_sums) s += sums[t];
        }
        block_excl_scan(s, lds4, tile_off);  // the block total: sums before this tile
    } else if (sums) {
        tile_off = sums[blockIdx.x];
    }
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, lds4, tot) + tile_off;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BS - 1) *total = run;
}

// ---- radix sort ------------------------------------------------------------------

// A tile is `rows` rows of RS_BS keys (one workgroup); rows goes from 1 to
// RS_ROWS_MAX so that a small sort still has a few tiles per CU and a large
// one fewer, longer tiles (smaller histograms to scan).
constexpr int RS_BS = 256;
constexpr int RS_ROWS_MAX = 8;

__global__ void __launch_bounds__(RS_BS) k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                   uint32_t* __restrict__ hist, int n_tiles, int rows)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_BS * rows;
    for (int r = 0; r < rows; ++r) {
        int64_t i = base + r * RS_BS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];  // digit-major
}

// Stable scatter: keys of a tile are ranked in position order. Within each row
// of 256 keys a wavefront finds the lanes holding the same digit with eight
// ballots; per-wave digit counts in LDS order the four waves; a running
// per-digit count orders the rows.
__global__ void __launch_bounds__(RS_BS) k_rs_scatter(const uint64_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, int64_t n,
                                                      int shift, const uint32_t* __restrict__ offs,
                                                      int n_tiles, int rows, uint64_t* __restrict__ keys_out,
                                                      uint32_t* __restrict__ vals_out)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[RS_BS / 64][256];
    __shared__ uint32_t goff[256];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = t >> 6;
    run[t] = 0;
    goff[t] = offs[(int64_t)t * n_tiles + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * RS_BS * rows;
    for (int r = 0; r < rows; ++r) {
        const int64_t i = base + r * RS_BS + t;
        const bool valid = i < n;
        uint64_t k = valid ? keys[i] : ~0ull;
        uint32_t v = valid ? vals[i] : 0u;
        const uint32_t d = valid ? (uint32_t)((k >> shift) & 255u) : 255u;
#pragma unroll
        for (int q = 0; q < RS_BS / 64; ++q) wcnt[q][t] = 0;
        __syncthreads();
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        uint32_t pos = run[d] + rank;
        for (int q = 0; q < w; ++q) pos += wcnt[q][d];
        __syncthreads();
        {
            uint32_t add = 0;
#pragma unroll
            for (int q = 0; q < RS_BS / 64; ++q) add += wcnt[q][t];
            run[t] += add;
        }
        if (valid) {
            const uint32_t dst = goff[d] + pos;
            keys_out[dst] = k;
            vals_out[dst] = v;
        }
        __syncthreads();
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

namespace sph {

void fill_u32(void* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    k_fill_u32<<<blocks_for(n, 256), 256, 0, s>>>(static_cast<uint32_t*>(p), v, n);
    SPH_HIP(hipGetLastError());
}

void scan_exclusive(sph_ctx* c, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                    hipStream_t s)
{
    if (n <= 0) {
        if (total) SPH_HIP(hipMemsetAsync(total, 0, sizeof(uint32_t), s));
        return;
    }
    const ScanPlan P = scan_plan(n);
    if (P.lv.empty()) {
        k_scan_apply<<<1, SCAN_BS, 0, s>>>(in, out, n, nullptr, total, 0);
        SPH_HIP(hipGetLastError());
        return;
    }
    uint32_t* sums = ensure<uint32_t>(c, c->scan_tmp, (size_t)P.scratch_words);
    auto level = [&](size_t k) { return sums + P.lv[k].offset; };
    // reduce down: level 0 holds the tile sums of `in`, level k those of level k - 1
    k_scan_reduce<<<(unsigned)P.tiles, SCAN_BS, 0, s>>>(in, n, level(0));
    SPH_HIP(hipGetLastError());
    if (scan_one_level(P)) {
        k_scan_apply<<<(unsigned)P.tiles, SCAN_BS, 0, s>>>(in, out, n, level(0), total, P.lv[0].count);
        SPH_HIP(hipGetLastError());
        return;
    }
    for (size_t k = 1; k < P.lv.size(); ++k) {
        k_scan_reduce<<<(unsigned)P.lv[k].count, SCAN_BS, 0, s>>>(level(k - 1), P.lv[k - 1].count, level(k));
        SPH_HIP(hipGetLastError());
    }
    // the last level fits one tile; then apply each level's scanned sums to
    // the level below, one block per tile of it
    const size_t top = P.lv.size() - 1;
    k_scan_apply<<<1, SCAN_BS, 0, s>>>(level(top), level(top), P.lv[top].count, nullptr, nullptr, 0);
    SPH_HIP(hipGetLastError());
    for (size_t k = top; k-- > 0;) {
        k_scan_apply<<<(unsigned)scan_apply_grid(P, k), SCAN_BS, 0, s>>>(level(k), level(k), P.lv[k].count,
                                                                         level(k + 1), nullptr, 0);
        SPH_HIP(hipGetLastError());
    }
    k_scan_apply<<<(unsigned)P.tiles, SCAN_BS, 0, s>>>(in, out, n, level(0), total, 0);
    SPH_HIP(hipGetLastError());
}

void radix_sort(sph_ctx* c, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                int64_t n, int bits, hipStream_t s, int lo_bit)
{
    if (n <= 1 || bits <= lo_bit) return;
    // about 1024 tiles (four per CU) while a tile holds at most RS_ROWS_MAX rows
    const int rows = (int)std::min<int64_t>(RS_ROWS_MAX, std::max<int64_t>(1, n / (1024 * RS_BS)));
    const int64_t tile = (int64_t)RS_BS * rows;
    const int n_tiles = (int)((n + tile - 1) / tile);
    const int64_t hn = (int64_t)n_tiles * 256;
    uint32_t* hist = ensure<uint32_t>(c, c->sort_hist, (size_t)hn);
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys_alt;
    uint32_t* vb = vals_alt;
    const int passes = (bits - lo_bit + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = lo_bit + 8 * p;
        k_rs_hist<<<n_tiles, RS_BS, 0, s>>>(ka, n, shift, hist, n_tiles, rows);
        SPH_HIP(hipGetLastError());
        scan_exclusive(c, hist, hist, hn, nullptr, s);
        k_rs_scatter<<<n_tiles, RS_BS, 0, s>>>(ka, va, n, shift, hist, n_tiles, rows, kb, vb);
        SPH_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        SPH_HIP(hipMemcpyAsync(keys, ka, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        SPH_HIP(hipMemcpyAsync(vals, va, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace sph
