// Wavefront-level helpers shared by the hot kernels: the per-XCD work queues
// and the staging of a cell's neighbour particles into LDS.
#pragma once

#include "common.h"

// Pop the next cell for this wavefront; -1 when all queues are drained.
__device__ __forceinline__ int pop_item(int64_t* ctr, const int* q_begin, int xcd, int& q_skip)
{
    int item = -1;
    if ((threadIdx.x & 63) == 0) {
        while (q_skip < 8) {
            const int q = (xcd + q_skip) & 7;
            const int size = q_begin[q + 1] - q_begin[q];
            const int64_t k = atomicAdd((unsigned long long*)&ctr[CT_QUEUE + q], 1ull);
            if (k < size) {
                item = q_begin[q] + (int)k;
                break;
            }
            ++q_skip;
        }
    }
    item = __shfl(item, 0, 64);
    q_skip = __shfl(q_skip, 0, 64);
    return item;
}

__device__ __forceinline__ float group_sum(float v, int lpi)
{
    for (int o = 1; o < lpi; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int group_sum_i(int v, int lpi)
{
    for (int o = 1; o < lpi; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Number of candidates of a cell: the particles of every cell in its list.
__device__ __forceinline__ int count_candidates(const int* __restrict__ p_leaf, const int* __restrict__ lf_count,
                                                int pb0, int np_all)
{
    const int lane = threadIdx.x & 63;
    int nj = 0;
    for (int b0 = 0; b0 < np_all; b0 += 64) {
        const int q = b0 + lane;
        int cnt = q < np_all ? lf_count[p_leaf[pb0 + q]] : 0;
        for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
        nj += cnt;
    }
    return nj;
}

// Copy candidates [c0, c0 + len) of the cell's flattened neighbour list into
// the wave's tile, shifted into the cell's frame. Each particle occupies NF
// float4 slots (tile layout [slot][candidate]); only slot 0's xyz is shifted.
// Partner records are read 64 at a time, one per lane, and broadcast with lane
// shuffles.
template <int NF>
__device__ __forceinline__ void stage_tile(float4* sj, const float4* __restrict__ jd, const int* __restrict__ p_leaf,
                                           const float4* __restrict__ p_shift, const int* __restrict__ lf_start,
                                           const int* __restrict__ lf_count, int pb0, int np_all, int c0, int len,
                                           int cap = 0)
{
    const int lane = threadIdx.x & 63;
    int off = 0;
    for (int b0 = 0; b0 < np_all && off < c0 + len; b0 += 64) {
        const int q = b0 + lane;
        int bs = 0, bc = 0;
        float4 sh = make_float4(0.f, 0.f, 0.f, 0.f);
        if (q < np_all) {
            const int bl = p_leaf[pb0 + q];
            bs = lf_start[bl];
            bc = lf_count[bl];
            sh = p_shift[pb0 + q];
        }
        const int npb = min(64, np_all - b0);
        for (int k = 0; k < npb; ++k) {
            const int bck = __shfl(bc, k, 64);
            const int lo = max(c0, off), hi = min(c0 + len, off + bck);
            if (lo < hi) {
                const int bsk = __shfl(bs, k, 64);
                const float sx = __shfl(sh.x, k, 64);
                const float sy = __shfl(sh.y, k, 64);
                const float sz = __shfl(sh.z, k, 64);
                for (int t = lo + lane; t < hi; t += 64) {
                    const int64_t src = (int64_t)NF * (bsk + (t - off));
                    float4 v = jd[src];
                    v.x += sx;
                    v.y += sy;
                    v.z += sz;
                    sj[t - c0] = v;
#pragma unroll
                    for (int f = 1; f < NF; ++f) sj[f * cap + (t - c0)] = jd[src + f];
                }
            }
            off += bck;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

