// Cell build: the cells of section 3.1 of the Swift paper.
//
// Particles are binned into a uniform top grid per box whose cells are at
// least as wide as the largest search radius in the box (so every neighbour of
// a particle lies in the same or one of the 26 adjacent top cells, Fig. 1),
// then each top cell is refined as an octree: a cell is split when it holds
// more than leaf_target particles and at most one in eight of them has
// cell_ratio times its search radius wider than half the cell (the mesh
// "needs to be adaptive", section 3.1; pairs of cells are then found by box
// distance with each cell's own largest radius, so the few wide particles
// only give their small cells a longer reach). Leaves hold contiguous ranges
// of the Morton-sorted particles. For every leaf the tree is walked from the 27 surrounding top
// cells to collect each leaf within reach -- the cell-pair tasks, found with a
// tree as the end of section 3.1 describes -- with the periodic image of each.
//
// All of it runs on the GPU: integer keys, a radix sort, one pass of small
// kernels per tree level, and a stack-based walk per (leaf, surrounding top
// cell). The host only reads back counts to size buffers.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int BS = 256;

__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

struct KeyLayout {
    int bits_top;  // bits of the top-cell index
    int levels;    // octree levels below the top grid (3 key bits each)
};

// Raise base[key] to v over a workgroup of WBS threads (valid lanes only).
// Each wavefront reduces first; when every wavefront of the group holds one
// key (a single box, or the inside of a box) a single atomic per group
// remains, otherwise each wavefront adds its own. Same-address atomics
// serialise at the L2, so one per 64 lanes still cost tens of microseconds
// for a million particles. Every thread of the group must call it.
constexpr int WBS = 1024;
__device__ __forceinline__ void block_atomic_max_u32(unsigned* base, int key, unsigned v, bool valid)
{
    __shared__ int wkey[WBS / 64];
    __shared__ unsigned wmax[WBS / 64];
    __shared__ int wstate[WBS / 64];  // 0: no valid lane, 1: one key, 2: several keys
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    const bool any = __any(valid);
    const int kref = __shfl(valid ? key : 0x7fffffff, __ffsll((unsigned long long)__ballot(valid)) - 1, 64);
    const bool uni = __all(!valid || key == kref);
    unsigned m = valid ? v : 0u;
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
    if (lane == 0) {
        wkey[w] = kref;
        wmax[w] = m;
        wstate[w] = !any ? 0 : (uni ? 1 : 2);
    }
    __syncthreads();
    bool one = true;  // every wavefront with a valid lane holds one and the same key
    int k0 = -1;
    unsigned mm = 0u;
    for (int q = 0; q < nw; ++q) {
        if (wstate[q] == 0) continue;
        if (wstate[q] == 2 || (k0 >= 0 && wkey[q] != k0)) one = false;
        k0 = k0 < 0 ? wkey[q] : k0;
        mm = max(mm, wmax[q]);
    }
    if (one) {
        if (threadIdx.x == 0 && k0 >= 0) atomicMax(&base[k0], mm);
    } else if (uni) {
        if (lane == 0 && any) atomicMax(&base[kref], m);
    } else if (valid) {
        atomicMax(&base[key], v);
    }
}

__global__ void k_wrap(int64_t n, const double* __restrict__ pos, const int64_t* __restrict__ box_first,
                       int n_boxes, const double* __restrict__ box_len, const float* __restrict__ hg,
                       double* __restrict__ pos_w, float* __restrict__ hg_copy,
                       unsigned* __restrict__ box_hmax, float margin, int64_t* __restrict__ ctr)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in_range = p < n;
    int b = 0;
    bool bad = false;
    float h = 0.0f;
    if (in_range) {
        b = box_of(box_first, n_boxes, p);
        const double L = box_len[b];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * p + a];
            bad |= !isfinite(x);
            double y = x - L * floor(x / L);
            if (!(y < L) || !(y >= 0.0)) y = 0.0;
            pos_w[3 * p + a] = y;
        }
        h = hg[p];
        bad |= !(h > 0.0f) || !isfinite(h);
        hg_copy[p] = h;
        if (bad) atomicAdd((unsigned long long*)&ctr[CT_BAD_INPUT], 1ull);
    }
    block_atomic_max_u32(box_hmax, b, __float_as_uint(margin * h), in_range && !bad);
}

// Largest search radius per box from the stored (caller-order) h guesses.
__global__ void k_box_hmax(int64_t n, const int64_t* __restrict__ box_first, int n_boxes,
                           const float* __restrict__ hg, unsigned* __restrict__ box_hmax, float margin,
                           int64_t* __restrict__ ctr)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in_range = p < n;
    float h = 0.0f;
    int b = 0;
    bool ok = false;
    if (in_range) {
        h = hg[p];
        b = box_of(box_first, n_boxes, p);
        ok = (h > 0.0f) && isfinite(h);
        if (!ok) atomicAdd((unsigned long long*)&ctr[CT_BAD_INPUT], 1ull);
    }
    block_atomic_max_u32(box_hmax, b, __float_as_uint(margin * h), ok);
}

__global__ void k_keys(int64_t n, const double* __restrict__ pos_w, const int64_t* __restrict__ box_first,
                       int n_boxes, const double* __restrict__ box_len, const int* __restrict__ box_G,
                       KeyLayout kl, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int b = box_of(box_first, n_boxes, p);
    const int G = box_G[b];
    const double wtop = box_len[b] / G;
    const uint32_t nsub = 1u << kl.levels;
    uint32_t tc[3], sc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double y = pos_w[3 * p + a];
        double c = floor(y / wtop);
        int ci = (int)c;
        ci = ci < 0 ? 0 : (ci >= G ? G - 1 : ci);
        double s = (y - ci * wtop) / wtop * (double)nsub;
        long si = (long)floor(s);
        si = si < 0 ? 0 : (si >= (long)nsub ? (long)nsub - 1 : si);
        tc[a] = (uint32_t)ci;
        sc[a] = (uint32_t)si;
    }
    const uint64_t top = ((uint64_t)tc[0] * G + tc[1]) * G + tc[2];
    const uint64_t mort = (spread3(sc[0]) << 2) | (spread3(sc[1]) << 1) | spread3(sc[2]);
    keys[p] = ((uint64_t)b << (kl.bits_top + 3 * kl.levels)) | (top << (3 * kl.levels)) | mort;
    vals[p] = (uint32_t)p;
}

__global__ void k_sorted_H(int64_t n, const uint32_t* __restrict__ perm, const float* __restrict__ hg,
                           float margin, float* __restrict__ Hs, int* __restrict__ leaf_tmp)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    Hs[p] = margin * hg[perm[p]];
    if (leaf_tmp) leaf_tmp[p] = -1;
}

__global__ void k_fill_int(int64_t n, int* __restrict__ a, int v)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) a[p] = v;
}

__global__ void k_lvl_head(int64_t n, const uint64_t* __restrict__ keys, const int* __restrict__ leaf_tmp,
                           int shift, uint32_t* __restrict__ head)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint32_t h = 0;
    if (leaf_tmp[p] < 0) {
        h = (p == 0) || (leaf_tmp[p - 1] >= 0) || ((keys[p] >> shift) != (keys[p - 1] >> shift));
    }
    head[p] = h;
}

// Node of every unassigned particle at level l; node start, count, largest
// search radius, and the number of particles whose search radius is too wide
// for half the node (cell_ratio * H > w / 2).
__global__ void k_lvl_nodes(int64_t n, const uint64_t* __restrict__ keys, const int* __restrict__ leaf_tmp,
                            const uint32_t* __restrict__ head, const uint32_t* __restrict__ excl,
                            const float* __restrict__ Hs, int level, KeyLayout kl, int64_t node_base,
                            int* __restrict__ nid, int* __restrict__ nd_start, int* __restrict__ nd_count,
                            unsigned* __restrict__ nd_hmax, int* __restrict__ nd_wide, int* __restrict__ nd_box,
                            int* __restrict__ nd_level, int* __restrict__ nd_coord,
                            const int* __restrict__ box_G, const double* __restrict__ box_len, float cell_ratio)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < n && leaf_tmp[p] < 0;
    int id = -1;
    unsigned hb = 0u;
    int wide = 0;
    if (valid) {
        id = (int)(node_base + (int64_t)excl[p] + head[p] - 1);
        nid[p] = id;
        const uint64_t k = keys[p];
        const int b = (int)(k >> (kl.bits_top + 3 * kl.levels));
        const double w = box_len[b] / box_G[b] / (double)(1u << level);
        const float H = Hs[p];
        hb = __float_as_uint(H);
        wide = (double)(cell_ratio * H) > 0.5 * w ? 1 : 0;
    }
    // The particles of a node are consecutive among the valid lanes (sorted
    // order; lanes of assigned particles only sit between nodes), so a scan
    // that combines equal ids gives each run's totals in its last lane, and
    // one atomic per run and array remains instead of one per particle.
    const int lane = threadIdx.x & 63;
    int cnt = valid ? 1 : 0, wsum = wide;
    unsigned hmx = hb;
    for (int o = 1; o < 64; o <<= 1) {
        const int id_o = __shfl_up(id, o, 64);
        const int c_o = __shfl_up(cnt, o, 64);
        const int w_o = __shfl_up(wsum, o, 64);
        const unsigned h_o = (unsigned)__shfl_up((int)hmx, o, 64);
        if (valid && lane >= o && id_o == id) {
            cnt += c_o;
            wsum += w_o;
            hmx = max(hmx, h_o);
        }
    }
    const int id_next = __shfl_down(id, 1, 64);
    if (valid && (lane == 63 || id_next != id)) {
        atomicAdd(&nd_count[id], cnt);
        atomicMax(&nd_hmax[id], hmx);
        if (wsum) atomicAdd(&nd_wide[id], wsum);
    }
    if (valid && head[p]) {
        const uint64_t k = keys[p];
        const int b = (int)(k >> (kl.bits_top + 3 * kl.levels));
        const uint64_t top = (k >> (3 * kl.levels)) & ((1ull << kl.bits_top) - 1);
        const int G = box_G[b];
        const uint64_t pre = (k & ((1ull << (3 * kl.levels)) - 1)) >> (3 * (kl.levels - level));
        const uint32_t mx = compact3(pre >> 2), my = compact3(pre >> 1), mz = compact3(pre);
        const uint32_t tz = (uint32_t)(top % G), ty = (uint32_t)((top / G) % G), tx = (uint32_t)(top / ((uint64_t)G * G));
        nd_start[id] = (int)p;
        nd_box[id] = b;
        nd_level[id] = level;
        nd_coord[3 * id + 0] = (int)((tx << level) | mx);
        nd_coord[3 * id + 1] = (int)((ty << level) | my);
        nd_coord[3 * id + 2] = (int)((tz << level) | mz);
    }
}

// A node is split when it holds more than leaf_target particles and at most
// one in eight of them has a search radius too wide for half its width. The
// wide few then sit in small cells with a long reach (pairs are found by box
// distance with each cell's own largest radius), instead of a few outliers
// keeping every particle of a dense region in one huge cell.
// The per-level kernels below run over a bound on the level's node count
// that the host knows (the launch), and take the count itself (*dM) from the
// device: slots k in [*dM, bound) hold no node.
__global__ void k_lvl_clear(int64_t node_base, int64_t bound, int* __restrict__ nd_count,
                            unsigned* __restrict__ nd_hmax, int* __restrict__ nd_wide)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= bound) return;
    nd_count[node_base + k] = 0;
    nd_hmax[node_base + k] = 0u;
    nd_wide[node_base + k] = 0;
}

__global__ void k_lvl_decide(int64_t bound, const uint32_t* __restrict__ dM, int64_t node_base, int level,
                             int max_level, int leaf_target, const int* __restrict__ nd_count,
                             const int* __restrict__ nd_wide, uint32_t* __restrict__ nflag,
                             int* __restrict__ nd_child0, int* __restrict__ nd_child1)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= bound) return;
    if (k >= (int64_t)*dM) {  // no node: not a leaf either (the scan of nflag counts the leaves)
        nflag[k] = 0u;
        return;
    }
    const int64_t id = node_base + k;
    const int cnt = nd_count[id];
    const bool split = level < max_level && cnt > leaf_target && 8 * nd_wide[id] <= cnt;
    nflag[k] = split ? 0u : 1u;
    nd_child0[id] = -1;
    nd_child1[id] = -1;
}

__global__ void k_lvl_leaves(int64_t bound, const uint32_t* __restrict__ dM, int64_t node_base, int64_t leaf_base,
                             const uint32_t* __restrict__ nflag, const uint32_t* __restrict__ nscan,
                             int* __restrict__ nd_leaf, int* __restrict__ lo2node)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= bound || k >= (int64_t)*dM) return;
    const int64_t id = node_base + k;
    if (nflag[k]) {
        const int64_t lo = leaf_base + nscan[k];
        nd_leaf[id] = (int)lo;
        lo2node[lo] = (int)id;
    } else {
        nd_leaf[id] = -1;
    }
}

__global__ void k_lvl_assign(int64_t n, const int* __restrict__ nid, const int* __restrict__ nd_leaf,
                             int* __restrict__ leaf_tmp)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || leaf_tmp[p] >= 0) return;
    const int lf = nd_leaf[nid[p]];
    if (lf >= 0) leaf_tmp[p] = lf;
}

// Children of the split nodes of the previous level: the level-l nodes holding
// the first and last particle of each split parent (level-l nodes are
// numbered in particle order, so a parent's children are the ids between),
// and each child's parent.
__global__ void k_lvl_children(int64_t Mprev, int64_t base_prev, const int* __restrict__ nd_leaf,
                               const int* __restrict__ nd_start, const int* __restrict__ nd_count,
                               const int* __restrict__ nid, int* __restrict__ nd_child0,
                               int* __restrict__ nd_child1, int* __restrict__ nd_parent)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mprev) return;
    const int64_t id = base_prev + k;
    if (nd_leaf[id] >= 0) return;
    const int s = nd_start[id];
    const int c0 = nid[s], c1 = nid[s + nd_count[id] - 1];
    nd_child0[id] = c0;
    nd_child1[id] = c1;
    for (int c = c0; c <= c1; ++c) nd_parent[c] = (int)id;
}

__global__ void k_top_table(int64_t bound, const uint32_t* __restrict__ dM, const int* __restrict__ nd_box,
                            const int* __restrict__ nd_coord, const int* __restrict__ box_G,
                            const int64_t* __restrict__ box_top_base, int* __restrict__ top)
{
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= bound || id >= (int64_t)*dM) return;
    const int b = nd_box[id];
    const int G = box_G[b];
    const int64_t t = ((int64_t)nd_coord[3 * id] * G + nd_coord[3 * id + 1]) * G + nd_coord[3 * id + 2];
    top[box_top_base[b] + t] = (int)id;
}

__global__ void k_leaf_head(int64_t n, const int* __restrict__ leaf_tmp, uint32_t* __restrict__ head)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    head[p] = (p == 0) || (leaf_tmp[p] != leaf_tmp[p - 1]);
}

__global__ void k_leaf_fill(int64_t n, const uint32_t* __restrict__ head, const uint32_t* __restrict__ excl,
                            const int* __restrict__ leaf_tmp, const int* __restrict__ lo2node,
                            int* __restrict__ leaf_of, int* __restrict__ lf_start, int* __restrict__ lf_node)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int L = (int)(excl[p] + head[p]) - 1;
    leaf_of[p] = L;
    if (head[p]) {
        lf_start[L] = (int)p;
        lf_node[L] = lo2node[leaf_tmp[p]];
    }
}

// First leaf of each box: leaves follow the sorted particles, whose boxes are
// contiguous blocks, so box b owns leaves [box_leaf[b], box_leaf[b + 1]).
__global__ void k_box_leaf(int n_boxes, int64_t n, int64_t nl, const int64_t* __restrict__ box_first,
                           const int* __restrict__ leaf_of, int* __restrict__ box_leaf)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > n_boxes) return;
    const int64_t p = box_first[b];
    box_leaf[b] = p < n ? leaf_of[p] : (int)nl;
}

// Particles of each leaf of 2 to 64 particles in decreasing order of search
// radius (ties by input index), one wavefront per leaf, a bitonic network
// over the 64 lanes; a leaf whose radii are all equal is left as it is. The hot kernels take a leaf's particles a pass at a
// time and cull the staged candidates to the pass's largest radius, which
// this order makes as small as it can be for every pass but the first.
// Only the order inside each leaf changes: leaves, nodes and lists stay.
__global__ void __launch_bounds__(256) k_leaf_sort_h(int64_t nl, const int* __restrict__ lf_start,
                                                     const int* __restrict__ lf_count, uint32_t* __restrict__ perm,
                                                     float* __restrict__ Hs)
{
    const int64_t leaf = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (leaf >= nl) return;  // whole wavefronts
    const int n = lf_count[leaf];
    if (n < 2 || n > 64) return;
    const int p0 = lf_start[leaf];
    // key: H descending, then index ascending; empty lanes last
    float k = lane < n ? Hs[p0 + lane] : -INFINITY;
    // a leaf whose radii are all equal keeps its order (every pass has the
    // same reach), without the network
    float lo = lane < n ? k : INFINITY, hi = k;
    for (int o = 32; o >= 1; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o, 64));
        hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    }
    if (lo == hi) return;  // whole wavefront
    uint32_t v = lane < n ? perm[p0 + lane] : 0xffffffffu;
    for (int size = 2; size <= 64; size <<= 1) {
        for (int stride = size >> 1; stride >= 1; stride >>= 1) {
            const float ko = __shfl_xor(k, stride, 64);
            const uint32_t vo = (uint32_t)__shfl_xor((int)v, stride, 64);
            const bool before = (ko > k) || (ko == k && vo < v);  // the partner sorts first
            const bool lower = (lane & stride) == 0;              // this lane keeps the first of the pair
            const bool desc_block = (lane & size) == 0;           // blocks alternate in bitonic order
            const bool take = (lower == desc_block) ? before : !before;
            if (take) {
                k = ko;
                v = vo;
            }
        }
    }
    if (lane < n) {
        Hs[p0 + lane] = k;
        perm[p0 + lane] = v;
    }
}

__global__ void k_leaf_fix(int64_t nl, const int* __restrict__ lf_node, const int* __restrict__ nd_count,
                           const unsigned* __restrict__ nd_hmax, int* __restrict__ nd_leaf,
                           int* __restrict__ lf_count, float* __restrict__ lf_hmax)
{
    int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= nl) return;
    const int id = lf_node[L];
    nd_leaf[id] = (int)L;
    lf_count[L] = nd_count[id];
    lf_hmax[L] = __uint_as_float(nd_hmax[id]);
}

__device__ __forceinline__ void node_geom(int id, const int* nd_coord, const int* nd_level, double wtop,
                                          double c[3], double& w)
{
    const int l = nd_level[id];
    w = wtop / (double)(1u << l);
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = ((double)nd_coord[3 * id + a] + 0.5) * w;
}

// The 27 top cells around a leaf's own, in the order its partner list visits
// them: three classes of (dx + dy + dz) mod 3, nine cells each, every class
// spread over the whole 3x3x3 block. The hot kernels stage a list in
// consecutive chunks, and a chunk that samples the whole neighbourhood gives
// every particle a similar share of its neighbours (even lane lists).
__constant__ signed char NB27[27][3] = {
    {-1, -1, -1}, {-1, 0, 1}, {-1, 1, 0}, {0, -1, 1}, {0, 0, 0}, {0, 1, -1}, {1, -1, 0}, {1, 0, -1}, {1, 1, 1},
    {-1, -1, 0}, {-1, 0, -1}, {-1, 1, 1}, {0, -1, -1}, {0, 0, 1}, {0, 1, 0}, {1, -1, 1}, {1, 0, 0}, {1, 1, -1},
    {-1, -1, 1}, {-1, 0, 0}, {-1, 1, -1}, {0, -1, 0}, {0, 0, -1}, {0, 1, 1}, {1, -1, -1}, {1, 0, 1}, {1, 1, 0}};

struct TreeView {
    const int* nd_coord;
    const int* nd_level;
    const unsigned* nd_hmax;
    const int* nd_leaf;
    const int* nd_child0;
    const int* nd_child1;
    const int* nd_parent;
    int n_nodes;
};

struct RecordOut {
    int* p_leaf;
    float4* p_shift;
    int* p_code;
    int2* p_rec;
    const int* lf_start;
    const int* lf_count;
};

// Depth-first walk below top cell T (seen through the periodic image shift S)
// for the leaves of partner lists of leaf a (centre cA, width wA, largest
// search radius HA): every leaf whose box lies within max(HA, its own largest
// radius) of a's box. nd counts those within HA, nf the others. FILL writes
// them from od and of on, and nj adds up their particles. The walk needs no
// stack: a split node's children have consecutive ids, so after a node the
// walk goes to its next sibling, or climbs to the first ancestor below T that
// has one. Children come in increasing id order. A tree that would take more
// steps than it has nodes is reported (CT_BAD_INPUT) and the walk ends.
template <bool FILL>
__device__ __forceinline__ void walk_top(int T, const double S[3], int code, const double cA[3], double wA,
                                         double wtop, float HA, const TreeView& tv, const RecordOut& ro,
                                         uint32_t od, uint32_t of, uint32_t& nd, uint32_t& nf, int& nj,
                                         int64_t* __restrict__ ctr)
{
    const double eps = 1e-9 * wtop;
    int X = T;
    for (int steps = 0;; ++steps) {
        if (steps > tv.n_nodes) {
            atomicAdd((unsigned long long*)&ctr[CT_BAD_INPUT], 1ull);
            return;
        }
        double cX[3], wX;
        node_geom(X, tv.nd_coord, tv.nd_level, wtop, cX, wX);
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double g = fabs(cX[k] + S[k] - cA[k]) - 0.5 * (wA + wX) - eps;
            g = g > 0.0 ? g : 0.0;
            d2 += g * g;
        }
        const double R = (double)fmaxf(HA, __uint_as_float(tv.nd_hmax[X]));
        if (d2 < R * R) {
            const int lf = tv.nd_leaf[X];
            if (lf < 0) {  // split: its first child next
                X = tv.nd_child0[X];
                continue;
            }
            const bool dens = d2 < (double)HA * (double)HA;
            if (FILL) {
                const uint32_t o = dens ? od + nd : of + nf;
                const int cnt = ro.lf_count[lf];
                ro.p_leaf[o] = lf;
                ro.p_rec[o] = make_int2(ro.lf_start[lf], cnt);
                ro.p_shift[o] = make_float4((float)(cX[0] + S[0] - cA[0]), (float)(cX[1] + S[1] - cA[1]),
                                            (float)(cX[2] + S[2] - cA[2]), 0.0f);
                ro.p_code[o] = code;
                nj += cnt;
            }
            nd += dens ? 1u : 0u;
            nf += dens ? 0u : 1u;
        }
        while (X != T && X == tv.nd_child1[tv.nd_parent[X]]) X = tv.nd_parent[X];
        if (X == T) return;
        ++X;
    }
}

// Sums over the 32 lanes of a half-wavefront.
__device__ __forceinline__ uint32_t half_sum(uint32_t v)
{
    for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive prefix sum over the 32 lanes of a half-wavefront.
__device__ __forceinline__ uint32_t half_excl_scan(uint32_t v)
{
    const int q = threadIdx.x & 31;
    uint32_t s = v;
    for (int o = 1; o < 32; o <<= 1) {
        const uint32_t t = __shfl_up(s, o, 32);
        if (q >= o) s += t;
    }
    return s - v;
}

constexpr int PBS = 256;

// Counters k0 + k of the workgroup's values v[k]: the total for k < n_sum,
// the largest value for the others. One atomic per counter and workgroup,
// into its spread slot (one per wavefront would be 10^5 atomics on a few
// cache lines for the largest sets). Every thread of the group must call it.
template <int NV>
__device__ __forceinline__ void block_counters(const int64_t (&v)[NV], int64_t (&red)[4][PBS / 64],
                                               int64_t* __restrict__ ctr, int k0, int n_sum)
{
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        int64_t x = v[k];
        for (int o = 32; o >= 1; o >>= 1) {
            const int64_t y = __shfl_xor(x, o, 64);
            x = k < n_sum ? x + y : max(x, y);
        }
        if ((threadIdx.x & 63) == 0) red[k][w] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        int64_t x = red[k][0];
        for (int q = 1; q < PBS / 64; ++q) x = k < n_sum ? x + red[k][q] : max(x, red[k][q]);
        unsigned long long* slot = (unsigned long long*)&ctr_slot(ctr)[k0 + k];
        if (k < n_sum) {
            if (x != 0) atomicAdd(slot, (unsigned long long)x);
        } else {
            atomicMax(slot, (unsigned long long)x);
        }
    }
}

// The cell-pair tasks (section 3.1: the neighbouring cells of each leaf, found
// with a tree), one half-wavefront per leaf and one lane per surrounding top
// cell. fill == 0 counts each leaf's records (all into p_cnt, the density's
// into p_cntd). fill == 1 writes the list at p_start[a], in two parts: first
// the leaves within Hmax_a of a's box (p_cntd[a] of them), then those that
// reach a only with their own radius. The density of a's particles (a gather
// over j inside h_i <= Hmax_a) needs only the first part; the force (pairs
// inside max(h_i, h_j)) takes both. Within each part the records follow the
// NB27 order of their top cells, depth-first below each, so each lane writes
// from the sum of the counts of the lanes before it (it walks its subtree
// twice: to count, then to write). The fill also writes the leaf's schedule
// key (sk != null), its cost particles x candidates as 12 bits of its float
// (exponent and four bits of mantissa) in decreasing order, prefixed with
// the XCD whose Morton range holds the leaf when xcd_local; and the build's
// shape counters (CT_B_*).
__global__ void __launch_bounds__(PBS) k_partners(int64_t nl, int fill, const int* __restrict__ lf_node,
                                                  TreeView tv, const int* __restrict__ nd_box,
                                                  const int* __restrict__ top,
                                                  const int64_t* __restrict__ box_top_base,
                                                  const int* __restrict__ box_G, const double* __restrict__ box_len,
                                                  uint32_t* __restrict__ p_cnt, uint32_t* __restrict__ p_cntd,
                                                  const uint32_t* __restrict__ p_start, RecordOut ro,
                                                  uint64_t* __restrict__ sk, uint32_t* __restrict__ sv,
                                                  int xcd_local, int64_t* __restrict__ ctr)
{
    const int q = threadIdx.x & 31;
    const int64_t a = ((int64_t)blockIdx.x * PBS + threadIdx.x) >> 5;
    const bool leaf_ok = a < nl;
    uint32_t nd = 0, nf = 0;
    int T = -1, code = 0;
    double S[3] = {0.0, 0.0, 0.0}, cA[3] = {0.0, 0.0, 0.0}, wA = 0.0, wtop = 1.0;
    float HA = 0.0f;
    if (leaf_ok && q < 27) {
        const int A = lf_node[a];
        const int b = nd_box[A];
        const int G = box_G[b];
        const double L = box_len[b];
        wtop = L / G;
        node_geom(A, tv.nd_coord, tv.nd_level, wtop, cA, wA);
        HA = __uint_as_float(tv.nd_hmax[A]);
        const int lA = tv.nd_level[A];
        int t[3], s[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            t[k] = (tv.nd_coord[3 * A + k] >> lA) + NB27[q][k];
            s[k] = 0;
            if (t[k] < 0) { t[k] += G; s[k] = -1; }
            else if (t[k] >= G) { t[k] -= G; s[k] = 1; }
            S[k] = s[k] * L;
        }
        T = top[box_top_base[b] + ((int64_t)t[0] * G + t[1]) * G + t[2]];
        code = image_code(s[0], s[1], s[2]);
    }
    int nj = 0;
    if (T >= 0) walk_top<false>(T, S, code, cA, wA, wtop, HA, tv, ro, 0u, 0u, nd, nf, nj, ctr);
    __shared__ int64_t red[4][PBS / 64];
    if (!fill) {
        const uint32_t td = half_sum(nd), tf = half_sum(nf);
        if (leaf_ok && q == 0) {
            p_cnt[a] = td + tf;
            p_cntd[a] = td;
        }
        // the records of all leaves in 64 bits: the list offsets are a 32-bit scan
        const int64_t v = (leaf_ok && q == 0) ? (int64_t)(td + tf) : 0;
        const int64_t r[1] = {v};
        block_counters<1>(r, red, ctr, CT_B_PAIRS64, 1);
        return;
    }
    const uint32_t sd = half_excl_scan(nd), sf = half_excl_scan(nf);
    if (T >= 0) {
        const uint32_t base = p_start[a];
        uint32_t cd = 0, cf = 0;
        walk_top<true>(T, S, code, cA, wA, wtop, HA, tv, ro, base + sd, base + p_cntd[a] + sf, cd, cf, nj, ctr);
    }
    nj = (int)half_sum((uint32_t)nj);
    int ni = 0, np = 0;
    if (leaf_ok) {
        ni = ro.lf_count[a];
        np = (int)(p_start[a + 1] - p_start[a]);
        if (sk && q == 0) {
            const float cost = (float)ni * (float)nj;
            uint64_t x = 0;
            if (xcd_local)
                while (x < 7 && a >= sph::xcd_start(nl, (int)x + 1)) ++x;
            sk[a] = (x << 12) | (uint64_t)(0xfffu - (__float_as_uint(cost) >> 19));
            sv[a] = (uint32_t)a;
        }
    }
    const bool lead = leaf_ok && q == 0;
    // CT_B_CAND_PAIRS, then the maxima CT_B_MAX_NI, _NP, _NJ
    const int64_t r[4] = {lead ? (int64_t)ni * nj : 0, lead ? ni : 0, lead ? np : 0, lead ? nj : 0};
    block_counters<4>(r, red, ctr, CT_B_CAND_PAIRS, 1);
}

// Schedule slots. by_cost != null and deal: the leaf of cost rank r goes to
// slot xcd_start(nl, r % 8) + r / 8. by_cost != null, no deal: slot r holds
// the leaf of rank r (the ranks already group each XCD's range). by_cost ==
// null: slot r holds leaf r (Morton order, so each XCD takes a contiguous
// range of neighbouring cells).
// cell_geom: half the leaf's width and its largest search radius, for the
// hot kernels' cell-box test on staged candidates.
__global__ void k_sched_fill(int64_t nl, const uint32_t* __restrict__ by_cost, int deal, const int* __restrict__ lf_start,
                             const int* __restrict__ lf_count, const uint32_t* __restrict__ p_start,
                             const int* __restrict__ lf_node, const int* __restrict__ nd_box,
                             const int* __restrict__ nd_level, const int* __restrict__ box_G,
                             const double* __restrict__ box_len, const float* __restrict__ lf_hmax,
                             const uint32_t* __restrict__ p_cntd, int4* __restrict__ cells,
                             int2* __restrict__ cell_aux, float2* __restrict__ cell_geom, int4* __restrict__ cells_d)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nl) return;
    const int a = by_cost ? (int)by_cost[r] : (int)r;
    const int64_t slot = by_cost && deal ? sph::xcd_start(nl, (int)(r & 7)) + (r >> 3) : r;
    const int node = lf_node[a];
    const int b = nd_box[node];
    cells[slot] = make_int4(lf_start[a], lf_count[a], (int)p_start[a], (int)(p_start[a + 1] - p_start[a]));
    cell_aux[slot] = make_int2(a, b);
    cells_d[slot] = make_int4(lf_start[a], lf_count[a], (int)p_start[a], (int)p_cntd[a]);
    const double w = box_len[b] / box_G[b] / (double)(1u << nd_level[node]);
    cell_geom[slot] = make_float2((float)(0.5 * w), lf_hmax[a]);
}

// Bounding box of each leaf's particles at their current offsets (sixteen
// lanes per schedule slot), for the density loop's culling of staged
// candidates: centre and the leaf's largest search radius, then the half
// widths, rounded up by a relative 1e-6 of the coordinates so that the FP32
// centre and widths still contain every particle.
__global__ void __launch_bounds__(256) k_cell_pbox(int64_t nl, const int4* __restrict__ cells,
                                                   const float4* __restrict__ xrel,
                                                   const float2* __restrict__ cell_geom, float4* __restrict__ pbox)
{
    // sixteen lanes per leaf (a leaf holds about that many particles); every
    // lane takes part in the shuffles, a group past the last leaf with no data
    const int64_t slot = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int sub = threadIdx.x & 15;
    const bool live = slot < nl;
    const int4 ci = live ? cells[slot] : make_int4(0, 0, 0, 0);
    const float BIG = 3.0e38f;
    float lx = BIG, ly = BIG, lz = BIG, hx = -BIG, hy = -BIG, hz = -BIG;
    for (int k = sub; k < ci.y; k += 16) {
        const float4 x = xrel[ci.x + k];
        lx = fminf(lx, x.x);
        ly = fminf(ly, x.y);
        lz = fminf(lz, x.z);
        hx = fmaxf(hx, x.x);
        hy = fmaxf(hy, x.y);
        hz = fmaxf(hz, x.z);
    }
    for (int o = 8; o >= 1; o >>= 1) {  // within the group of 16
        lx = fminf(lx, __shfl_xor(lx, o, 64));
        ly = fminf(ly, __shfl_xor(ly, o, 64));
        lz = fminf(lz, __shfl_xor(lz, o, 64));
        hx = fmaxf(hx, __shfl_xor(hx, o, 64));
        hy = fmaxf(hy, __shfl_xor(hy, o, 64));
        hz = fmaxf(hz, __shfl_xor(hz, o, 64));
    }
    if (live && sub == 0) {
        pbox[2 * slot] = make_float4(0.5f * (lx + hx), 0.5f * (ly + hy), 0.5f * (lz + hz), cell_geom[slot].y);
        pbox[2 * slot + 1] = make_float4(0.5f * (hx - lx) * 1.000001f + 1.0e-6f * fmaxf(fabsf(lx), fabsf(hx)),
                                         0.5f * (hy - ly) * 1.000001f + 1.0e-6f * fmaxf(fabsf(ly), fabsf(hy)),
                                         0.5f * (hz - lz) * 1.000001f + 1.0e-6f * fmaxf(fabsf(lz), fabsf(hz)), 0.0f);
    }
}

// Sorted FP64 positions and FP32 offsets from the centre of each particle's leaf.
__global__ void k_sorted_fill(int64_t n, const uint32_t* __restrict__ perm, const double* __restrict__ pos_w,
                              const int* __restrict__ leaf_of, const int* __restrict__ lf_node,
                              const int* __restrict__ nd_coord, const int* __restrict__ nd_level,
                              const int* __restrict__ nd_box, const int* __restrict__ box_G,
                              const double* __restrict__ box_len, double* __restrict__ pos_s,
                              float4* __restrict__ xrel)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    const int id = lf_node[leaf_of[p]];
    const int b = nd_box[id];
    double c[3], w;
    node_geom(id, nd_coord, nd_level, box_len[b] / box_G[b], c, w);
    const double L = box_len[b];
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // the image of the particle nearest its leaf: itself at a build; after
        // a drift across the box boundary, the one on the leaf's side
        const double x = pos_w[3 * (int64_t)o + a];
        const double img = L * rint((x - c[a]) / L);
        pos_s[3 * p + a] = x - img;
        d[a] = (x - c[a]) - img;
    }
    xrel[p] = make_float4((float)d[0], (float)d[1], (float)d[2], 0.0f);
}

// Smallest search radius (float bits; non-negative floats order like their bits).
__global__ void __launch_bounds__(BS) k_min_H(int64_t n, const float* __restrict__ Hs, unsigned* __restrict__ out)
{
    __shared__ float wm[BS / 64];
    float m = INFINITY;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        m = fminf(m, Hs[p]);
    for (int o = 32; o >= 1; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {  // one atomic per workgroup
        for (int q = 1; q < BS / 64; ++q) m = fminf(m, wm[q]);
        atomicMin(out, __float_as_uint(m));
    }
}

// The build's shape counters folded over their spread slots, and the
// smallest search radius, into out (BUILD_OUT_WORDS words): a buffer no other
// kernel writes, so its copy to the host can wait for the next synchronisation.
__global__ void k_build_out(const int64_t* __restrict__ ctr, const unsigned* __restrict__ hmin,
                            int64_t* __restrict__ out)
{
    const int k = threadIdx.x;  // CT_B_CAND_PAIRS + k
    if (k < 4) {
        int64_t v = ctr[CT_B_CAND_PAIRS + k];
        for (int sl = 0; sl < CT_SPREAD_SLOTS; ++sl) {
            const int64_t x = ctr[CT_SPREAD + sl * CT_SUMS + CT_B_CAND_PAIRS + k];
            v = k == 0 ? v + x : max(v, x);
        }
        out[k] = v;
    } else if (k == 4) {
        out[4] = (int64_t)*hmin;
    }
}

int ceil_log2(uint64_t v)
{
    int b = 0;
    while ((1ull << b) < v) ++b;
    return b;
}

}  // namespace

namespace sph {

// Everything after the positions are wrapped: keys, sort, tree, leaves, lists.
static void build_from_wrapped(sph_ctx* c, hipStream_t s)
{
    const int64_t n = c->n;
    const int nb = c->n_boxes;
    const float margin = (float)c->prm.h_margin;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);

    // ---- largest search radius per box (k_wrap / k_box_hmax ran) -> top grid --------
    unsigned* box_hmax = static_cast<unsigned*>(c->box_hmax.p);
    std::vector<unsigned> hm(nb);
    int64_t bad = 0;
    SPH_HIP(hipMemcpyAsync(hm.data(), box_hmax, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
    SPH_HIP(hipMemcpyAsync(&bad, &ctr[CT_BAD_INPUT], 8, hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    SPH_REQUIRE(bad == 0, SPH_E_ARG, "non-finite position or non-positive/non-finite h_guess");
    c->h_box_G.assign(nb, 0);
    c->h_box_top_base.assign(nb + 1, 0);
    uint64_t maxG3 = 1;
    for (int b = 0; b < nb; ++b) {
        const int64_t cnt = c->h_box_first[b + 1] - c->h_box_first[b];
        float H;
        std::memcpy(&H, &hm[b], 4);
        const double L = c->h_box_len[b];
        int G = 3;
        if (cnt > 0) {
            SPH_REQUIRE(3.0 * (double)H <= L, SPH_E_H_TOO_LARGE,
                        "box " + std::to_string(b) + ": search radius " + std::to_string(H) +
                            " exceeds a third of the box side " + std::to_string(L));
            G = (int)std::floor(L / (double)H);
            // a top cell exactly one radius wide must still hold the radius after rounding
            while (G > 3 && L / G < (double)H) --G;
            G = std::max(3, std::min(G, 256));
        }
        c->h_box_G[b] = G;
        c->h_box_top_base[b + 1] = c->h_box_top_base[b] + (int64_t)G * G * G;
        maxG3 = std::max<uint64_t>(maxG3, (uint64_t)G * G * G);
    }
    c->n_top = c->h_box_top_base[nb];
    c->bits_box = nb > 1 ? ceil_log2((uint64_t)nb) : 0;
    c->bits_top = std::max(1, ceil_log2(maxG3));
    c->levels = std::min(10, (63 - c->bits_box - c->bits_top) / 3);
    SPH_REQUIRE(c->levels >= 1, SPH_E_ARG, "too many boxes or top cells for the key layout");
    int* box_G = ensure<int>(c, c->box_G, nb);
    int64_t* box_top_base = ensure<int64_t>(c, c->box_top_base, nb + 1);
    SPH_HIP(hipMemcpyAsync(box_G, c->h_box_G.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s));
    SPH_HIP(hipMemcpyAsync(box_top_base, c->h_box_top_base.data(), (size_t)(nb + 1) * 8,
                           hipMemcpyHostToDevice, s));

    // ---- keys and sort -------------------------------------------------------------------
    KeyLayout kl{c->bits_top, c->levels};
    uint64_t* keys = ensure<uint64_t>(c, c->keys, n);
    uint64_t* keys_alt = ensure<uint64_t>(c, c->keys_alt, n);
    uint32_t* perm = ensure<uint32_t>(c, c->perm, n);
    uint32_t* perm_alt = ensure<uint32_t>(c, c->perm_alt, n);
    const int64_t* box_first = static_cast<int64_t*>(c->box_first.p);
    const double* box_len = static_cast<double*>(c->box_len.p);
    k_keys<<<blocks_for(n, BS), BS, 0, s>>>(n, static_cast<double*>(c->pos_w.p), box_first, nb, box_len,
                                            box_G, kl, keys, perm);
    SPH_HIP(hipGetLastError());
    // Sorted by box and top cell first; the Morton bits below the top grid
    // matter only where a top cell splits, and uniform sets have none (the
    // particles of a top-cell leaf keep their input order). Where one does,
    // the whole key is sorted after level 0, below.
    const int key_bits = c->bits_box + c->bits_top + 3 * c->levels;
    radix_sort(c, keys, perm, keys_alt, perm_alt, n, key_bits, s, 3 * c->levels);

    float* Hs = ensure<float>(c, c->Hs, n);
    int* leaf_tmp = ensure<int>(c, c->lf_tmp, n);
    k_sorted_H<<<blocks_for(n, BS), BS, 0, s>>>(n, perm, static_cast<float*>(c->hguess.p), margin, Hs,
                                                leaf_tmp);
    SPH_HIP(hipGetLastError());

    // ---- tree, level by level ---------------------------------------------------------------
    // One read-back per level: its node count M and leaf count K (the two
    // halves of one counter word). The level's kernels run over a bound the
    // host already has: the top cells at level 0, eight children per split
    // node of the level above after that.
    uint32_t* head = ensure<uint32_t>(c, c->head, n + 1);
    uint32_t* excl = ensure<uint32_t>(c, c->scan1, n + 1);
    int* nid = ensure<int>(c, c->nid, n);
    uint32_t* d_M = reinterpret_cast<uint32_t*>(&ctr[CT_TOTAL]);
    uint32_t* d_K = d_M + 1;
    int* top = ensure<int>(c, c->top, (size_t)c->n_top);
    k_fill_int<<<blocks_for(c->n_top, BS), BS, 0, s>>>(c->n_top, top, -1);
    SPH_HIP(hipGetLastError());

    int64_t node_base = 0, leaf_base = 0, prev_base = 0, prev_M = 0;
    int64_t bound = std::min<int64_t>(n, c->n_top);
    // level-order leaf id -> node; parked in lf_start's buffer until the leaves
    // are renumbered in Morton order
    int* lo2node = ensure<int>(c, c->lf_start, n + 1);
    for (int level = 0; level <= c->levels && bound > 0; ++level) {
        const int shift = 3 * (c->levels - level);
        k_lvl_head<<<blocks_for(n, BS), BS, 0, s>>>(n, keys, leaf_tmp, shift, head);
        SPH_HIP(hipGetLastError());
        scan_exclusive(c, head, excl, n, d_M, s);
        const int64_t need = node_base + bound;
        // node ids are int and index 3 ints of nd_coord each
        SPH_REQUIRE(need <= (int64_t)(INT32_MAX / 3), SPH_E_ARG,
                    "the cell tree needs more than " + std::to_string(INT32_MAX / 3) + " nodes");
        if (need > c->node_cap) {
            const int64_t cap = std::max<int64_t>(need + need / 2, 1024);
            grow_keep<int>(c, c->nd_start, cap, node_base, s);
            grow_keep<int>(c, c->nd_count, cap, node_base, s);
            grow_keep<unsigned>(c, c->nd_hmax, cap, node_base, s);
            grow_keep<int>(c, c->nd_wide, cap, node_base, s);
            grow_keep<int>(c, c->nd_child0, cap, node_base, s);
            grow_keep<int>(c, c->nd_child1, cap, node_base, s);
            grow_keep<int>(c, c->nd_parent, cap, node_base, s);
            grow_keep<int>(c, c->nd_leaf, cap, node_base, s);
            grow_keep<int>(c, c->nd_box, cap, node_base, s);
            grow_keep<int>(c, c->nd_level, cap, node_base, s);
            grow_keep<int>(c, c->nd_coord, 3 * cap, 3 * node_base, s);
            c->node_cap = cap;
        }
        int* nd_start = static_cast<int*>(c->nd_start.p);
        int* nd_count = static_cast<int*>(c->nd_count.p);
        unsigned* nd_hmax = static_cast<unsigned*>(c->nd_hmax.p);
        int* nd_wide = static_cast<int*>(c->nd_wide.p);
        int* nd_child0 = static_cast<int*>(c->nd_child0.p);
        int* nd_child1 = static_cast<int*>(c->nd_child1.p);
        int* nd_parent = static_cast<int*>(c->nd_parent.p);
        int* nd_leaf = static_cast<int*>(c->nd_leaf.p);
        int* nd_box = static_cast<int*>(c->nd_box.p);
        int* nd_level = static_cast<int*>(c->nd_level.p);
        int* nd_coord = static_cast<int*>(c->nd_coord.p);
        const unsigned gb = (unsigned)blocks_for(bound, BS);
        k_lvl_clear<<<gb, BS, 0, s>>>(node_base, bound, nd_count, nd_hmax, nd_wide);
        SPH_HIP(hipGetLastError());
        k_lvl_nodes<<<blocks_for(n, BS), BS, 0, s>>>(n, keys, leaf_tmp, head, excl, Hs, level, kl, node_base,
                                                     nid, nd_start, nd_count, nd_hmax, nd_wide, nd_box, nd_level,
                                                     nd_coord, box_G, box_len, (float)c->prm.cell_ratio);
        SPH_HIP(hipGetLastError());
        if (level == 0) {
            k_top_table<<<gb, BS, 0, s>>>(bound, d_M, nd_box, nd_coord, box_G, box_top_base, top);
            SPH_HIP(hipGetLastError());
        } else {
            k_lvl_children<<<blocks_for(prev_M, BS), BS, 0, s>>>(prev_M, prev_base, nd_leaf, nd_start,
                                                                 nd_count, nid, nd_child0, nd_child1,
                                                                 nd_parent);
            SPH_HIP(hipGetLastError());
        }
        uint32_t* nflag = ensure<uint32_t>(c, c->nflag, bound + 1);
        uint32_t* nscan = ensure<uint32_t>(c, c->nscan, bound + 1);
        k_lvl_decide<<<gb, BS, 0, s>>>(bound, d_M, node_base, level, c->levels, c->prm.leaf_target, nd_count,
                                       nd_wide, nflag, nd_child0, nd_child1);
        SPH_HIP(hipGetLastError());
        scan_exclusive(c, nflag, nscan, bound, d_K, s);
        k_lvl_leaves<<<gb, BS, 0, s>>>(bound, d_M, node_base, leaf_base, nflag, nscan, nd_leaf, lo2node);
        SPH_HIP(hipGetLastError());
        k_lvl_assign<<<blocks_for(n, BS), BS, 0, s>>>(n, nid, nd_leaf, leaf_tmp);
        SPH_HIP(hipGetLastError());
        uint32_t mk[2] = {0u, 0u};
        SPH_HIP(hipMemcpyAsync(mk, d_M, sizeof(mk), hipMemcpyDeviceToHost, s));
        SPH_HIP(hipStreamSynchronize(s));
        const int64_t M = mk[0], K = mk[1];
        if (level == 0) c->cells_refined = K < M;
        // every particle not yet in a leaf heads or joins a node of this level,
        // so the bound (its parents' children) holds them; a larger count is a bug
        SPH_REQUIRE(M <= bound && K <= M, SPH_E_HIP, "cell tree level outside its bound");
        if (level == 0 && K < M) {
            // A top cell splits: order the particles by the whole key. The
            // sort is stable and keeps every top cell's range, so the level-0
            // nodes, their sums and each particle's node and leaf stay as
            // they are; only the sorted search radii follow the new order.
            radix_sort(c, keys, perm, keys_alt, perm_alt, n, key_bits, s);
            k_sorted_H<<<blocks_for(n, BS), BS, 0, s>>>(n, perm, static_cast<float*>(c->hguess.p), margin, Hs,
                                                        nullptr);
            SPH_HIP(hipGetLastError());
        }
        prev_base = node_base;
        prev_M = M;
        node_base += M;
        leaf_base += K;
        bound = std::min<int64_t>(8 * (M - K), n);  // children of this level's split nodes
    }
    c->n_nodes = node_base;

    // ---- leaves in Morton (particle) order ---------------------------------------------------
    k_leaf_head<<<blocks_for(n, BS), BS, 0, s>>>(n, leaf_tmp, head);
    SPH_HIP(hipGetLastError());
    scan_exclusive(c, head, excl, n, nullptr, s);
    const int64_t nl = leaf_base;  // the leaves of all levels, one per run of leaf_tmp
    c->n_leaves = nl;
    int* leaf_of = ensure<int>(c, c->leaf_of, n);
    // lo2node lives in lf_start's buffer; move it aside before lf_start is written
    int* lo2 = ensure<int>(c, c->nid, std::max<int64_t>(n, nl));
    SPH_HIP(hipMemcpyAsync(lo2, lo2node, (size_t)nl * 4, hipMemcpyDeviceToDevice, s));
    int* lf_start = ensure<int>(c, c->lf_start, nl + 1);
    int* lf_node = ensure<int>(c, c->lf_node, nl);
    int* lf_count = ensure<int>(c, c->lf_count, nl);
    float* lf_hmax = ensure<float>(c, c->lf_hmax, nl);
    k_leaf_fill<<<blocks_for(n, BS), BS, 0, s>>>(n, head, excl, leaf_tmp, lo2, leaf_of, lf_start, lf_node);
    SPH_HIP(hipGetLastError());
    k_leaf_fix<<<blocks_for(nl, BS), BS, 0, s>>>(nl, lf_node, static_cast<int*>(c->nd_count.p),
                                                 static_cast<unsigned*>(c->nd_hmax.p),
                                                 static_cast<int*>(c->nd_leaf.p), lf_count, lf_hmax);
    SPH_HIP(hipGetLastError());
    k_leaf_sort_h<<<(unsigned)blocks_for(nl * 64, 256), 256, 0, s>>>(nl, lf_start, lf_count, perm, Hs);
    SPH_HIP(hipGetLastError());
    {
        int* box_leaf = ensure<int>(c, c->box_leaf, c->n_boxes + 1);
        k_box_leaf<<<blocks_for(c->n_boxes + 1, BS), BS, 0, s>>>(c->n_boxes, n, nl,
                                                                  static_cast<int64_t*>(c->box_first.p), leaf_of,
                                                                  box_leaf);
        SPH_HIP(hipGetLastError());
    }

    // ---- neighbour lists ------------------------------------------------------------------------
    uint32_t* p_cnt = ensure<uint32_t>(c, c->p_cnt, nl + 1);
    uint32_t* p_cntd = ensure<uint32_t>(c, c->p_cntd, nl + 1);
    uint32_t* p_start = ensure<uint32_t>(c, c->p_start, nl + 1);
    const int* nd_coord = static_cast<int*>(c->nd_coord.p);
    const int* nd_level = static_cast<int*>(c->nd_level.p);
    const int* nd_box = static_cast<int*>(c->nd_box.p);
    const unsigned* nd_hmax = static_cast<unsigned*>(c->nd_hmax.p);
    const int* nd_leaf = static_cast<int*>(c->nd_leaf.p);
    const int* nd_child0 = static_cast<int*>(c->nd_child0.p);
    const int* nd_child1 = static_cast<int*>(c->nd_child1.p);
    const TreeView tv{nd_coord, nd_level, nd_hmax, nd_leaf, nd_child0, nd_child1,
                      static_cast<int*>(c->nd_parent.p), (int)c->n_nodes};
    const unsigned p_blocks = (unsigned)blocks_for(nl * 32, PBS);
    k_partners<<<p_blocks, PBS, 0, s>>>(nl, 0, lf_node, tv, nd_box, top, box_top_base, box_G, box_len, p_cnt,
                                        p_cntd, nullptr, RecordOut{}, nullptr, nullptr, 0, ctr);
    SPH_HIP(hipGetLastError());
    scan_exclusive(c, p_cnt, p_start, nl, p_start + nl, s);
    uint32_t np = 0;
    SPH_HIP(hipMemcpyAsync(&np, p_start + nl, 4, hipMemcpyDeviceToHost, s));
    const int64_t* hc0 = read_counters(c, s);  // synchronises: np is in
    const int64_t bad2 = hc0[CT_BAD_INPUT], np64 = hc0[CT_B_PAIRS64];
    SPH_REQUIRE(bad2 == 0, SPH_E_HIP, "inconsistent cell tree: a walk took more steps than the tree has nodes");
    SPH_REQUIRE(np64 <= (int64_t)UINT32_MAX && (int64_t)np == np64, SPH_E_ARG,
                std::to_string(np64) + " (cell, neighbour cell) records: more than 2^32 - 1 cannot be indexed");
    c->n_pairs = np;
    int* p_leaf = ensure<int>(c, c->p_leaf, np);
    float4* p_shift = ensure<float4>(c, c->p_shift, np);
    int* p_code = ensure<int>(c, c->p_code, np);
    int2* p_rec = ensure<int2>(c, c->p_rec, np);
    const int order = c->prm.cell_order;
    const bool by_cost = order != 1;
    uint64_t* sk = ensure<uint64_t>(c, c->sched_key, nl);
    uint32_t* sv = ensure<uint32_t>(c, c->sched_val, nl);
    k_partners<<<p_blocks, PBS, 0, s>>>(nl, 1, lf_node, tv, nd_box, top, box_top_base, box_G, box_len, p_cnt,
                                        p_cntd, p_start, RecordOut{p_leaf, p_shift, p_code, p_rec, lf_start, lf_count},
                                        by_cost ? sk : nullptr, sv, order == 2 ? 1 : 0, ctr);
    SPH_HIP(hipGetLastError());

    // ---- work schedule: leaves by decreasing cost dealt out to the XCDs, Morton ranges, or Morton
    //      ranges each ordered by decreasing cost --------------------------------------------------
    {
        uint64_t* ska = ensure<uint64_t>(c, c->sched_key_alt, nl);
        uint32_t* sva = ensure<uint32_t>(c, c->sched_val_alt, nl);
        if (by_cost) radix_sort(c, sk, sv, ska, sva, nl, order == 2 ? 15 : 12, s);
        int4* cells = ensure<int4>(c, c->cells, nl);
        int2* cell_aux = ensure<int2>(c, c->cell_aux, nl);
        float2* cell_geom = ensure<float2>(c, c->cell_geom, nl);
        int4* cells_d = ensure<int4>(c, c->cells_d, nl);
        k_sched_fill<<<blocks_for(nl, BS), BS, 0, s>>>(nl, by_cost ? sv : nullptr, order == 0 ? 1 : 0, lf_start,
                                                       lf_count, p_start, lf_node, nd_box, nd_level,
                                                       static_cast<int*>(c->box_G.p),
                                                       static_cast<double*>(c->box_len.p), lf_hmax, p_cntd, cells,
                                                       cell_aux, cell_geom, cells_d);
        SPH_HIP(hipGetLastError());
    }

    // ---- sorted particle streams ------------------------------------------------------------------
    double* pos_s = ensure<double>(c, c->pos_s, 3 * n);
    float4* xrel = ensure<float4>(c, c->xrel, n);
    k_sorted_fill<<<blocks_for(n, BS), BS, 0, s>>>(n, perm, static_cast<double*>(c->pos_w.p), leaf_of, lf_node,
                                                   nd_coord, nd_level, nd_box, box_G, box_len, pos_s, xrel);
    SPH_HIP(hipGetLastError());
    cell_boxes(c, s);
    // no drift since this build; the smallest search radius bounds how far
    // the particles may drift before the cells are rebuilt
    unsigned* drift = ensure<unsigned>(c, c->drift, 4);
    fill_u32(drift, 0u, 4, s);               // bound, step maximum, (minimum below), non-finite flag
    fill_u32(drift + 2, 0x7f800000u, 1, s);  // +inf before the minimum
    k_min_H<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n, BS), 256)), BS, 0, s>>>(n, Hs,
                                                                                                 drift + 2);
    SPH_HIP(hipGetLastError());
    // the shape counters and the smallest radius come back behind an event;
    // the next synchronisation (or finish_build_read) picks them up
    int64_t* bo = ensure<int64_t>(c, c->build_out, BUILD_OUT_WORDS);
    k_build_out<<<1, 64, 0, s>>>(ctr, drift + 2, bo);
    SPH_HIP(hipGetLastError());
    SPH_HIP(hipMemcpyAsync(c->h_build, bo, BUILD_OUT_WORDS * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipEventRecord(c->ev_build, s));
    c->build_read_pending = true;
    c->binfo.n_cells = nl;
    c->binfo.n_pairs = c->n_pairs;
    c->built = true;
    ++c->tm.builds;
    c->drift_pending = false;
    c->vsig_valid = false;  // signal velocities belong to the cells of the last force pass
    c->bal_valid = false;
    c->div_valid = false;   // and the divergences to its particle order
    ++c->layout_serial;  // cell arrays and grid sizes changed
    c->density_done = false;
    c->density64_done = false;
}

void finish_build_read(sph_ctx* c)
{
    if (!c->build_read_pending) return;
    SPH_HIP(hipEventSynchronize(c->ev_build));
    c->build_read_pending = false;
    const int64_t* hb = c->h_build;
    c->binfo.candidate_pairs = hb[0];
    c->binfo.max_cell_particles = hb[1];
    c->binfo.max_neighbour_cells = hb[2];
    c->binfo.max_candidates = hb[3];
    const uint32_t bits = (uint32_t)hb[4];
    std::memcpy(&c->h_min, &bits, 4);
}

void build_cells(sph_ctx* c, int32_t n_boxes, const int64_t* box_first, const double* box_len, int64_t n,
                 const double* pos, const float* h_guess, hipStream_t s)
{
    c->built = false;
    c->density_done = false;
    c->density64_done = false;
    c->n = n;
    c->n_boxes = n_boxes;
    c->h_box_first.assign(box_first, box_first + n_boxes + 1);
    c->h_box_len.assign(box_len, box_len + n_boxes);
    int64_t* bf = ensure<int64_t>(c, c->box_first, n_boxes + 1);
    double* bl = ensure<double>(c, c->box_len, n_boxes);
    SPH_HIP(hipMemcpyAsync(bf, box_first, (size_t)(n_boxes + 1) * 8, hipMemcpyHostToDevice, s));
    SPH_HIP(hipMemcpyAsync(bl, box_len, (size_t)n_boxes * 8, hipMemcpyHostToDevice, s));
    ensure<int64_t>(c, c->counters, CT_COUNT);
    double* pw = ensure<double>(c, c->pos_w, 3 * n);
    float* hg = ensure<float>(c, c->hguess, n);
    unsigned* box_hmax = ensure<unsigned>(c, c->box_hmax, n_boxes);
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    SPH_HIP(hipMemsetAsync(box_hmax, 0, (size_t)n_boxes * 4, s));
    SPH_HIP(hipMemsetAsync(ctr, 0, CT_COUNT * 8, s));
    k_wrap<<<blocks_for(n, WBS), WBS, 0, s>>>(n, pos, bf, n_boxes, bl, h_guess, pw, hg, box_hmax,
                                            (float)c->prm.h_margin, ctr);
    SPH_HIP(hipGetLastError());
    c->rebuilds = 0;
    build_from_wrapped(c, s);
}

// Offsets of every particle from its leaf centre (and the sorted FP64
// positions) from the current positions, keeping the cells: after a drift.
void refresh_offsets(sph_ctx* c, hipStream_t s)
{
    const int64_t n = c->n;
    k_sorted_fill<<<blocks_for(n, BS), BS, 0, s>>>(
        n, static_cast<uint32_t*>(c->perm.p), static_cast<double*>(c->pos_w.p), static_cast<int*>(c->leaf_of.p),
        static_cast<int*>(c->lf_node.p), static_cast<int*>(c->nd_coord.p), static_cast<int*>(c->nd_level.p),
        static_cast<int*>(c->nd_box.p), static_cast<int*>(c->box_G.p), static_cast<double*>(c->box_len.p),
        static_cast<double*>(c->pos_s.p), static_cast<float4*>(c->xrel.p));
    SPH_HIP(hipGetLastError());
    cell_boxes(c, s);
}

// The particle boxes of every leaf (k_cell_pbox) from the current offsets.
void cell_boxes(sph_ctx* c, hipStream_t s)
{
    const int64_t nl = c->n_leaves;
    float4* pbox = ensure<float4>(c, c->cell_pbox, 2 * nl);
    if (nl == 0) return;
    k_cell_pbox<<<blocks_for(16 * nl, 256), 256, 0, s>>>(nl, static_cast<int4*>(c->cells.p),
                                                        static_cast<float4*>(c->xrel.p),
                                                        static_cast<float2*>(c->cell_geom.p), pbox);
    SPH_HIP(hipGetLastError());
}

// Rebuild around new smoothing lengths (caller order) keeping the positions.
void rebuild_cells(sph_ctx* c, const float* h_caller, hipStream_t s)
{
    float* hg = static_cast<float*>(c->hguess.p);
    unsigned* box_hmax = static_cast<unsigned*>(c->box_hmax.p);
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    if (h_caller && h_caller != hg)  // null: the guesses of the last build
        SPH_HIP(hipMemcpyAsync(hg, h_caller, (size_t)c->n * 4, hipMemcpyDeviceToDevice, s));
    SPH_HIP(hipMemsetAsync(box_hmax, 0, (size_t)c->n_boxes * 4, s));
    SPH_HIP(hipMemsetAsync(ctr, 0, CT_COUNT * 8, s));
    k_box_hmax<<<blocks_for(c->n, WBS), WBS, 0, s>>>(c->n, static_cast<int64_t*>(c->box_first.p), c->n_boxes, hg,
                                                   box_hmax, (float)c->prm.h_margin, ctr);
    SPH_HIP(hipGetLastError());
    build_from_wrapped(c, s);
}

}  // namespace sph
