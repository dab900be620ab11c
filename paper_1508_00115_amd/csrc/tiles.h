// Wavefront-level helpers shared by the hot kernels: the per-XCD work queues
// and the staging of a cell's neighbour particles into LDS.
#pragma once

#include "common.h"

// Work sources of the hot kernels. Items are schedule slots: either cells
// ranked by decreasing cost (particles x candidates) and dealt out to the 8
// XCDs (xcd_start), so the longest cells start first and every XCD gets an
// equal share of each cost class, or cells in Morton order, so each XCD runs a
// contiguous range of neighbouring cells whose particles its L2 keeps.
//   hardware dispatch: one item per wavefront; consecutive workgroups are
//     placed round-robin on the 8 XCDs and workgroup b is remapped to the next
//     slot of its XCD's run, which is rank b;
//   persistent: a grid sized to the machine pops batches of items from eight
//     per-XCD queues (one atomic per batch) and steals from the other queues
//     when its own is empty.
struct WorkSched {
    int persistent;   // 0: hardware dispatch, 1: per-XCD queues
    int batch;        // items per pop (persistent)
    int n_items;
    int q_begin[9];   // queue q covers items [q_begin[q], q_begin[q+1])
};

// Workgroup index with the XCD round-robin undone: blocks that land on the
// same XCD get consecutive indices.
__device__ __forceinline__ int xcd_block_index()
{
    const int nb = gridDim.x;
    const int q = nb / 8, r = nb % 8;
    const int x = blockIdx.x % 8, l = blockIdx.x / 8;
    return x * q + min(x, r) + l;
}

// Next item range [a, a_end) of this wavefront; false when the work is done.
__device__ __forceinline__ bool next_items(const WorkSched& W, int64_t* ctr, int waves_per_block, int& state,
                                           int& a, int& a_end)
{
    if (!W.persistent) {
        if (state) return false;
        state = 1;
        a = xcd_block_index() * waves_per_block + (int)(threadIdx.x >> 6);
        a_end = min(a + 1, W.n_items);
        return a < a_end;
    }
    int lo = -1, hi = -1;
    if ((threadIdx.x & 63) == 0) {
        const int xcd = blockIdx.x & 7;
        while (state < 8) {
            const int q = (xcd + state) & 7;
            const int size = W.q_begin[q + 1] - W.q_begin[q];
            const int64_t k = atomicAdd((unsigned long long*)&ctr[CT_QUEUE + 8 * q], (unsigned long long)W.batch);
            if (k < size) {
                lo = W.q_begin[q] + (int)k;
                hi = W.q_begin[q] + (int)min<int64_t>(k + W.batch, size);
                break;
            }
            ++state;
        }
    }
    a = __shfl(lo, 0, 64);
    a_end = __shfl(hi, 0, 64);
    state = __shfl(state, 0, 64);
    return a >= 0;
}

// Lanes per particle for a cell of ni particles and nj candidates: the power
// of two (at least lpi_min) that minimises passes x (candidate tests + list
// work per particle + fixed work of a pass, per lane), plus the re-staging of
// every pass when the candidates cannot stay resident in LDS (chunks of
// `chunk`). Weights are VALU costs in units of one candidate test: list work
// is given per particle (`list_work`), a pass costs ~25, staging a chunk ~20.
__device__ __forceinline__ int choose_lpi(int ni, int nj, int lpi_min, float list_work, bool resident, int chunk)
{
    const int nchunks = (nj + chunk - 1) / chunk;
    int best = 16;
    float best_cost = 3.0e38f;
#pragma unroll
    for (int lg = 1; lg <= 4; ++lg) {  // l = 2, 4, 8, 16: every division below is a shift or a constant
        const int l = 1 << lg;
        if (l < lpi_min) continue;
        const int per = 64 >> lg;
        const float passes = (float)((ni + per - 1) >> (6 - lg));
        float cost = passes * (((float)nj + list_work) * (1.0f / (float)l) + 25.0f);
        if (!resident) cost += passes * (float)nchunks * 20.0f;
        if (cost < best_cost) {
            best_cost = cost;
            best = l;
        }
    }
    return best;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A 32-bit value of another lane of the same row of 16, by a DPP pattern:
// 0xB1 = quad_perm [1,0,3,2], 0x4E = quad_perm [2,3,0,1], 0x141 =
// row_half_mirror (lane i of 8 reads 7 - i), 0x140 = row_mirror (lane i of
// 16 reads 15 - i). Every lane of the row must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}

// Sum over aligned groups of lpi lanes (1, 2, 4, 8 or 16), returned to every
// lane of the group; the whole wavefront must be active. The two quad
// patterns add the partners at distance 1 and 2; once each quad holds its
// sum, the half-row mirror brings in the other quad of the 8 and the row
// mirror the other half of the 16. The partners of a group add the same two
// values at every step, so every lane ends with the same bits (the same sums
// as exchanges at distance 1, 2, 4 and 8). One VALU operation per step.
__device__ __forceinline__ float group_sum(float v, int lpi)
{
    if (lpi >= 2) v += dpp_f<0xB1>(v);
    if (lpi >= 4) v += dpp_f<0x4E>(v);
    if (lpi >= 8) v += dpp_f<0x141>(v);
    if (lpi >= 16) v += dpp_f<0x140>(v);
    return v;
}
// Largest value over aligned groups of lpi lanes, with the same patterns.
__device__ __forceinline__ float group_max(float v, int lpi)
{
    if (lpi >= 2) v = fmaxf(v, dpp_f<0xB1>(v));
    if (lpi >= 4) v = fmaxf(v, dpp_f<0x4E>(v));
    if (lpi >= 8) v = fmaxf(v, dpp_f<0x141>(v));
    if (lpi >= 16) v = fmaxf(v, dpp_f<0x140>(v));
    return v;
}
__device__ __forceinline__ int group_sum_i(int v, int lpi)
{
    if (lpi >= 2) v += dpp_i<0xB1>(v);
    if (lpi >= 4) v += dpp_i<0x4E>(v);
    if (lpi >= 8) v += dpp_i<0x141>(v);
    if (lpi >= 16) v += dpp_i<0x140>(v);
    return v;
}

// Even out the list lengths of the lpi lanes of each particle (aligned groups
// of lanes; lane l's list is lists[l], lists[l + 64], ...), whose phase B
// trip count is the longest list in the wavefront: at distance m = 1, 2, ...
// the lane of each pair with more entries hands the surplus half to its
// partner, which copies them from the end of the giver's list to the end of
// its own (the giver only shortens its count, so no lane reads a slot that
// is being written). After log2(lpi) steps the lists of a particle differ by
// at most one entry; the set of entries, and so every sum, is unchanged (only
// the order in which the lanes add them, as with any split of the
// candidates). No list grows beyond the longest one. Returns the lane's new
// length; the whole wavefront must be active.
template <class T>
__device__ __forceinline__ int balance_lists(T* lists, int nl, int lpi)
{
    const int lane = threadIdx.x & 63;
    for (int m = 1; m < lpi; m <<= 1) {
        const int nl_p = __shfl_xor(nl, m, 64);
        const int tot = nl + nl_p;
        const int mine = (lane & m) ? (tot >> 1) : tot - (tot >> 1);
        const int take = mine - nl;  // > 0: copy that many from the partner's end
        const T* src = lists + (lane ^ m) + (nl_p - take) * 64;
        T* dst = lists + lane + nl * 64;
        for (int t = 0; t < take; ++t) dst[t * 64] = src[t * 64];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        nl = mine;
    }
    return nl;
}

// Number of lanes for which c holds (a scalar bit count of the ballot).
__device__ __forceinline__ int wave_count(bool c)
{
    return __popcll(__ballot(c));
}

// Number of candidates of a cell: the particles of every cell in its list.
__device__ __forceinline__ int count_candidates(const int2* __restrict__ p_rec, int pb0, int np_all)
{
    const int lane = threadIdx.x & 63;
    int nj = 0;
    for (int b0 = 0; b0 < np_all; b0 += 64) {
        const int q = b0 + lane;
        int cnt = q < np_all ? p_rec[pb0 + q].y : 0;
        for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        nj += cnt;
    }
    return nj;
}

// Neighbour-cell records of a cell with at most 64 neighbour cells, one per
// lane: first particle, count, exclusive prefix of the counts (the cell's
// offset in the flattened candidate list) and the shift into the cell frame.
// A record holds its cell's first particle and count itself (p_rec, written
// by the build), so the staging is one load away from the cell's record list.
struct NbrLanes {
    int bs, bc, off;
    float sx, sy, sz;
    int np, nj;
};

// The records already in registers (lane q: record q, zero beyond np).
__device__ __forceinline__ NbrLanes nbr_from(int2 rec, float4 sh, int np)
{
    const int lane = threadIdx.x & 63;
    NbrLanes nb;
    nb.bs = rec.x;
    nb.bc = rec.y;
    nb.sx = sh.x;
    nb.sy = sh.y;
    nb.sz = sh.z;
    int inc = nb.bc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    nb.off = inc - nb.bc;
    nb.nj = __shfl(inc, 63, 64);
    nb.np = np;
    return nb;
}

__device__ __forceinline__ NbrLanes load_nbr(const int2* __restrict__ p_rec, const float4* __restrict__ p_shift,
                                             int pb0, int np)
{
    const int lane = threadIdx.x & 63;
    NbrLanes nb;
    nb.bs = 0;
    nb.bc = 0;
    nb.sx = nb.sy = nb.sz = 0.f;
    if (lane < np) {
        const int2 rec = p_rec[pb0 + lane];
        const float4 sh = p_shift[pb0 + lane];
        nb.bs = rec.x;
        nb.bc = rec.y;
        nb.sx = sh.x;
        nb.sy = sh.y;
        nb.sz = sh.z;
    }
    int inc = nb.bc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    nb.off = inc - nb.bc;
    nb.nj = __shfl(inc, 63, 64);
    nb.np = np;
    return nb;
}

// The flattened candidate list of a cell, walked in increasing order: the
// neighbour-cell records are held 64 at a time (one NbrLanes block), and a
// chunk never spans two blocks, so any number of neighbour cells is staged
// with the independent loads of fetch_chunk / stage_fast and every record is
// read once per sweep. Candidates before the current block: off0.
struct NbrCursor {
    NbrLanes nb;
    int b0, off0;  // first record of the block, candidates before it
    int pb0, np_all;
};

__device__ __forceinline__ void cursor_init(NbrCursor& cu, const int2* __restrict__ p_rec,
                                            const float4* __restrict__ p_shift, int pb0, int np_all)
{
    cu.pb0 = pb0;
    cu.np_all = np_all;
    cu.b0 = 0;
    cu.off0 = 0;
    cu.nb = load_nbr(p_rec, p_shift, pb0, min(np_all, 64));
}

// The cursor on a cell whose first block of records is already in registers.
__device__ __forceinline__ void cursor_init_from(NbrCursor& cu, const NbrLanes& nb, int pb0, int np_all)
{
    cu.pb0 = pb0;
    cu.np_all = np_all;
    cu.b0 = 0;
    cu.off0 = 0;
    cu.nb = nb;
}

// Move the cursor to the block holding candidate c (c at or after the
// current block's start; back to the first block when c is before it).
__device__ __forceinline__ void cursor_seek(NbrCursor& cu, const int2* __restrict__ p_rec,
                                            const float4* __restrict__ p_shift, int c)
{
    if (c < cu.off0) cursor_init(cu, p_rec, p_shift, cu.pb0, cu.np_all);
    while (c >= cu.off0 + cu.nb.nj && cu.b0 + 64 < cu.np_all) {
        cu.off0 += cu.nb.nj;
        cu.b0 += 64;
        cu.nb = load_nbr(p_rec, p_shift, cu.pb0 + cu.b0, min(cu.np_all - cu.b0, 64));
    }
}

// Length of the chunk that starts at candidate c (cursor on c's block).
__device__ __forceinline__ int cursor_chunk(const NbrCursor& cu, int c, int cap)
{
    return min(cap, cu.off0 + cu.nb.nj - c);
}

// A chunk of candidates in flight: the loads of stage_fast split from the LDS
// stores, so a kernel can fetch chunk c + 1 while it computes chunk c.
template <int NF, int CAP>
struct ChunkRegs {
    float4 v[CAP / 64][NF];
    float s[CAP / 64][3];
    int len;
};

// Lanes of the wavefront below this one whose bit is set in mask.
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Load candidates [c0, c0 + len) of the cursor's block (len <= CAP) into R.
// The neighbour record (lane of nb) of each slot is found without a search:
// the record holding c0 is the last one starting at or before it (a ballot
// over the record lanes), each record starting inside the chunk marks its
// first slot in mk (CAP bytes of LDS), and a slot's record is that first one
// plus the marks up to the slot (a ballot of the marks and a lane count).
// Every record holds at least one particle, so no two records start at the
// same slot. The loads of the chunk are independent and issue back to back.
template <int NF, int CAP, int STRIDE = NF>
__device__ __forceinline__ void fetch_chunk(ChunkRegs<NF, CAP>& R, const float4* __restrict__ jd,
                                            const NbrLanes& nb, int c0, int len, uint8_t* mk)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = CAP / 64;
    R.len = len;
    const int q0 = __popcll(__ballot(lane < nb.np && nb.off <= c0)) - 1;
#pragma unroll
    for (int r = 0; r < PER; ++r) mk[lane + 64 * r] = 0;
    wave_sync_lds();
    const int s = nb.off - c0;
    if (lane < nb.np && s > 0 && s < len) mk[s] = 1;
    wave_sync_lds();
    int q = q0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        const bool start = mk[t] != 0;
        const uint64_t m = __ballot(start);
        const int qt = t < len ? q + lanes_below(m) + (start ? 1 : 0) : q0;
        q += __popcll(m);
        const int kg = c0 + (t < len ? t : 0);
        const int src = __shfl(nb.bs, qt, 64) + (kg - __shfl(nb.off, qt, 64));
        R.s[r][0] = __shfl(nb.sx, qt, 64);
        R.s[r][1] = __shfl(nb.sy, qt, 64);
        R.s[r][2] = __shfl(nb.sz, qt, 64);
#pragma unroll
        for (int f = 0; f < NF; ++f) R.v[r][f] = jd[(int64_t)STRIDE * src + f];
    }
}

// True on every lane when a candidate of the fetched chunk has a mass other
// than m.
template <int NF, int CAP>
__device__ __forceinline__ bool chunk_mass_differs(const ChunkRegs<NF, CAP>& R, float m)
{
    const int lane = threadIdx.x & 63;
    bool d = false;
#pragma unroll
    for (int r = 0; r < CAP / 64; ++r) d |= (lane + 64 * r < R.len) && (R.v[r][0].w != m);
    return __any(d);
}

// Store a fetched one-float4 chunk into the tile (shifted into the cell
// frame), its unused slots [len, CAP) filled with a position far outside any
// search radius: a loop over the chunk may then run to a multiple of its
// stride without a bounds test.
template <int CAP>
__device__ __forceinline__ void commit_chunk_padded(float4* sj, const ChunkRegs<1, CAP>& R)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = CAP / 64;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        float4 a = make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.0f);
        if (t < R.len) {
            a = R.v[r][0];
            a.x += R.s[r][0];
            a.y += R.s[r][1];
            a.z += R.s[r][2];
        }
        sj[t] = a;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// Culling of staged candidates. A candidate farther from a box than every
// search radius of the particles inside it (and, for the force, than its own
// h) pairs with none of them: the 3x3x3 block of cells is a cube, the region
// within reach of a cell a rounded box about a quarter smaller, and that of
// a pass's particles smaller still. The force tests its candidates against
// the box of each pass; the density only on non-uniform cells, against the
// box of the cell's particles (on a uniform grid the compaction costs more
// than the tests it saves); the re-scanning kernel against the box of each
// group of particles. An axis-aligned box in the cell frame: the cell's own
// box (centre 0, half width hw in every axis, widened by the drift bound) or
// the bounding box of a set of particles.
struct CullBox {
    float cx, cy, cz, hx, hy, hz;
};

__device__ __forceinline__ CullBox cell_box(float hw)
{
    CullBox b;
    b.cx = b.cy = b.cz = 0.0f;
    b.hx = b.hy = b.hz = hw;
    return b;
}

// A value every active lane holds alike, moved to a scalar register: it then
// costs no vector register while it stays live across a loop.
__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Lane 0's double (the first active lane's), in scalar registers.
__device__ __forceinline__ double lane0_d(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b & 0xffffffffull));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ float wave_min(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v);

// Bounding box of the positions of the lanes with `in` set (every lane must
// take part). The half widths are rounded up by a relative 1e-6 of the
// coordinates, so that the FP32 centre and widths still contain every
// position; the cull's reach has its own margin.
__device__ __forceinline__ CullBox pass_box(float x, float y, float z, bool in)
{
    const float BIG = 3.0e38f;
    const float lx = wave_min(in ? x : BIG), hx = wave_max(in ? x : -BIG);
    const float ly = wave_min(in ? y : BIG), hy = wave_max(in ? y : -BIG);
    const float lz = wave_min(in ? z : BIG), hz = wave_max(in ? z : -BIG);
    CullBox b;
    b.cx = uniform_f(0.5f * (lx + hx));
    b.cy = uniform_f(0.5f * (ly + hy));
    b.cz = uniform_f(0.5f * (lz + hz));
    b.hx = uniform_f(0.5f * (hx - lx) * 1.000001f + 1.0e-6f * fmaxf(fabsf(lx), fabsf(hx)));
    b.hy = uniform_f(0.5f * (hy - ly) * 1.000001f + 1.0e-6f * fmaxf(fabsf(ly), fabsf(hy)));
    b.hz = uniform_f(0.5f * (hz - lz) * 1.000001f + 1.0e-6f * fmaxf(fabsf(lz), fabsf(hz)));
    return b;
}

__device__ __forceinline__ float box_dist2(float x, float y, float z, const CullBox& b)
{
    const float gx = fmaxf(fabsf(x - b.cx) - b.hx, 0.0f), gy = fmaxf(fabsf(y - b.cy) - b.hy, 0.0f),
                gz = fmaxf(fabsf(z - b.cz) - b.hz, 0.0f);
    return fmaf(gx, gx, fmaf(gy, gy, gz * gz));
}

__device__ __forceinline__ float box_dist2(float x, float y, float z, float hw)
{
    const float gx = fmaxf(fabsf(x) - hw, 0.0f), gy = fmaxf(fabsf(y) - hw, 0.0f), gz = fmaxf(fabsf(z) - hw, 0.0f);
    return fmaf(gx, gx, fmaf(gy, gy, gz * gz));
}

// Margins of the cell-box test: FP32 positions in the cell frame carry
// relative errors near 1e-7, so the box grows by 1e-6 of its half width and
// the radii by 1e-5 (a candidate near the reach is kept, never dropped).
__device__ __forceinline__ float cull_half_width(float hw) { return hw * 1.000001f; }
__device__ __forceinline__ float cull_reach2(float reach) { return (reach * 1.00001f) * (reach * 1.00001f); }

// Store a fetched chunk (NF float4 per candidate, slot 0 = x, y, z, h^2) with
// the cell-box test: a candidate is kept when the box lies within
// max(reach, h_j) of it (OWN_H false: within reach). Returns how many were
// kept (packed from slot 0).
template <int NF, int CAP, bool OWN_H = true>
__device__ __forceinline__ int commit_chunk_culled(float4* sj, const ChunkRegs<NF, CAP>& R, const CullBox& box,
                                                   float reach2)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = CAP / 64;
    int n = 0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        float4 a = R.v[r][0];
        a.x += R.s[r][0];
        a.y += R.s[r][1];
        a.z += R.s[r][2];
        const bool keep = t < R.len && box_dist2(a.x, a.y, a.z, box) < (OWN_H ? fmaxf(reach2, a.w * 1.00002f) : reach2);
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int d = n + lanes_below(m);
            sj[d] = a;
#pragma unroll
            for (int f = 1; f < NF; ++f) sj[f * CAP + d] = R.v[r][f];
        }
        n += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return n;
}

// Store a fetched one-float4 chunk (x, y, z, m; shifted into the cell frame)
// keeping only the candidates within reach of the cell's box (box_dist2 <
// reach2), packed from slot 0, and fill the rest of the CAP slots with a far
// position, so a loop may run to a multiple of its stride without a bounds
// test. Returns how many were kept. A candidate farther from the box than
// every search radius of the cell pairs with none of its particles.
template <int CAP>
__device__ __forceinline__ int commit_chunk_culled_padded(float4* sj, const ChunkRegs<1, CAP>& R, const CullBox& box,
                                                          float reach2)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = CAP / 64;
    int n = 0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        float4 a = R.v[r][0];
        a.x += R.s[r][0];
        a.y += R.s[r][1];
        a.z += R.s[r][2];
        const bool keep = t < R.len && box_dist2(a.x, a.y, a.z, box) < reach2;
        const uint64_t m = __ballot(keep);
        if (keep) sj[n + lanes_below(m)] = a;
        n += __popcll(m);
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        if (t >= n) sj[t] = make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.0f);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return n;
}

// Largest v over the wavefront (every lane active).
__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Stage candidates [c0, c0 + len) (len <= CAP) into the tile: every lane finds
// the neighbour cell of each of its candidates by a binary search over the
// lane-held prefix offsets, so all global loads of the chunk are independent
// and issue back to back.
template <int NF, int CAP>
__device__ __forceinline__ void stage_fast(float4* sj, const float4* __restrict__ jd, const NbrLanes& nb, int c0,
                                           int len)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = CAP / 64;
    int src[PER];
    float s3[PER][3];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        const int kg = c0 + (t < len ? t : 0);
        int q = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int cand = q + step;
            const int v = __shfl(nb.off, cand < nb.np ? cand : nb.np - 1, 64);
            if (cand < nb.np && v <= kg) q = cand;
        }
        src[r] = __shfl(nb.bs, q, 64) + (kg - __shfl(nb.off, q, 64));
        s3[r][0] = __shfl(nb.sx, q, 64);
        s3[r][1] = __shfl(nb.sy, q, 64);
        s3[r][2] = __shfl(nb.sz, q, 64);
    }
    float4 v[PER][NF];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        if (lane + 64 * r < len) {
#pragma unroll
            for (int f = 0; f < NF; ++f) v[r][f] = jd[(int64_t)NF * src[r] + f];
        }
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        if (t < len) {
            float4 a = v[r][0];
            a.x += s3[r][0];
            a.y += s3[r][1];
            a.z += s3[r][2];
            sj[t] = a;
#pragma unroll
            for (int f = 1; f < NF; ++f) sj[f * CAP + t] = v[r][f];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// stage_fast keeping only the candidates within reach of `box` (distance to
// it below sqrt(reach2)), packed from slot 0 in candidate order; returns how
// many it kept.
template <int NF, int CAP>
__device__ __forceinline__ int stage_fast_culled(float4* sj, const float4* __restrict__ jd, const NbrLanes& nb,
                                                 int c0, int len, const CullBox& box, float reach2)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = CAP / 64;
    int src[PER];
    float s3[PER][3];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int t = lane + 64 * r;
        const int kg = c0 + (t < len ? t : 0);
        int q = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int cand = q + step;
            const int v = __shfl(nb.off, cand < nb.np ? cand : nb.np - 1, 64);
            if (cand < nb.np && v <= kg) q = cand;
        }
        src[r] = __shfl(nb.bs, q, 64) + (kg - __shfl(nb.off, q, 64));
        s3[r][0] = __shfl(nb.sx, q, 64);
        s3[r][1] = __shfl(nb.sy, q, 64);
        s3[r][2] = __shfl(nb.sz, q, 64);
    }
    float4 v[PER][NF];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        if (lane + 64 * r < len) {
#pragma unroll
            for (int f = 0; f < NF; ++f) v[r][f] = jd[(int64_t)NF * src[r] + f];
        }
    }
    int n = 0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        float4 a = v[r][0];
        a.x += s3[r][0];
        a.y += s3[r][1];
        a.z += s3[r][2];
        const bool keep = lane + 64 * r < len && box_dist2(a.x, a.y, a.z, box) < reach2;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int d = n + lanes_below(m);
            sj[d] = a;
#pragma unroll
            for (int f = 1; f < NF; ++f) sj[f * CAP + d] = v[r][f];
        }
        n += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return n;
}

