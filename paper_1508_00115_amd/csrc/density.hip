// FP32 density loop with the smoothing-length solve (section 2, Eq. 1 of the
// Swift paper, and the choice of h for a fixed weighted neighbour number).
//
// Work unit: one leaf cell, handled by one wavefront. The particles of every
// cell within reach (the cell's self task and its pair tasks, section 3.1) are
// copied into the wavefront's LDS tile once, shifted into the cell's
// FP32 frame. Each particle of the cell then iterates Newton's method on h
// entirely against that tile: the density sums of a particle depend only on
// its own h and the fixed positions, so no global sweep or ghost pass is
// needed between iterations. A particle whose root lies beyond its search
// radius is flagged; the host rebuilds the cells around a larger guess and
// solves it again.
//
// Cells with few particles give several lanes to each particle (lanes of a
// group stride over the tile; their partial sums meet through lane shuffles),
// so a 64-lane wavefront stays busy on cells of 8 to 64 particles.
//
// Cells are popped from eight work queues, one per XCD, each holding a
// contiguous Morton range so an XCD's L2 sees neighbouring cells; a wave whose
// queue is empty takes work from the next queue.
#include "common.h"
#include "tiles.h"

#include <cmath>

namespace {

constexpr int BS = 256;
constexpr int WAVES = BS / 64;

struct DensArgs {
    const float4* jd;        // sorted (x, y, z) in the leaf frame, m
    const float* Hs;         // sorted search radii
    float* hs;               // sorted h: in, start value; out, result
    float* rhos;
    float* fs;
    uint8_t* st_s;           // sorted state
    const int* lf_start;
    const int* lf_count;
    const uint32_t* p_start;
    const int* p_leaf;
    const float4* p_shift;
    const uint32_t* perm;
    float* h_out;
    float* rho_out;
    float* f_out;
    float* nw_out;
    uint8_t* status;
    int64_t* ctr;
    int q_begin[9];          // queue q covers leaves [q_begin[q], q_begin[q+1])
    float target;            // S0 = sum w(q) at the root: 3 n_ngb / 32
    float tol;               // on |S0 / target - 1|
    int max_iter;
};

__global__ void k_dens_prologue(int64_t n, const uint32_t* __restrict__ perm, const float4* __restrict__ xrel,
                                const float* __restrict__ mass, const float* __restrict__ h_in,
                                const uint8_t* __restrict__ status, float4* __restrict__ jd,
                                float* __restrict__ hs, uint8_t* __restrict__ st_s, int64_t* __restrict__ ctr)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    const float m = mass[o];
    const float h = h_in[o];
    const float4 x = xrel[p];
    jd[p] = make_float4(x.x, x.y, x.z, m);
    hs[p] = h;
    uint8_t st = status[o];
    st_s[p] = st == ST_OVERFLOW ? (uint8_t)ST_ACTIVE : st;
    if (!(m > 0.0f) || !isfinite(m) || !(h > 0.0f) || !isfinite(h))
        atomicAdd((unsigned long long*)&ctr[CT_BAD_INPUT], 1ull);
}

// Sorted copies of the final h, rho and f after the cells were rebuilt (the
// caller-order outputs hold every particle's final values).
__global__ void k_dens_regather(int64_t n, const uint32_t* __restrict__ perm, const float* __restrict__ h,
                                const float* __restrict__ rho, const float* __restrict__ f,
                                float* __restrict__ hs, float* __restrict__ rhos, float* __restrict__ fs)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    hs[p] = h[o];
    rhos[p] = rho[o];
    fs[p] = f[o];
}

template <int CAP>
__global__ void __launch_bounds__(BS) k_density(DensArgs A)
{
    __shared__ float4 tile[WAVES][CAP];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    float4* sj = tile[wv];
    const int xcd = blockIdx.x & 7;
    int q_skip = 0;
    int64_t cand_acc = 0, inter_acc = 0, sweep_acc = 0;
    int max_ev = 0;
    int64_t n_over = 0, n_unconv = 0;

    for (;;) {
        const int a = pop_item(A.ctr, A.q_begin, xcd, q_skip);
        if (a < 0) break;
        const int i0 = A.lf_start[a];
        const int ni = A.lf_count[a];
        const int pb0 = (int)A.p_start[a];
        const int np_all = (int)A.p_start[a + 1] - pb0;

        const int nj = count_candidates(A.p_leaf, A.lf_count, pb0, np_all);
        const int lpi = ni <= 8 ? 8 : (ni <= 16 ? 4 : (ni <= 32 ? 2 : 1));
        const int sub = lane & (lpi - 1);
        const int per_pass = 64 / lpi;
        const bool single_tile = nj <= CAP;
        bool loaded = false;

        for (int ib = 0; ib < ni; ib += per_pass) {
            const int gi = ib + lane / lpi;
            const bool valid = gi < ni;
            const int i = i0 + (valid ? gi : 0);
            const float4 xi = A.jd[i];
            const float Hi = A.Hs[i];
            float h = A.hs[i];
            const uint8_t st0 = A.st_s[i];
            bool done = !valid || st0 != ST_ACTIVE;
            if (!(h > 0.0f) || h > Hi) h = Hi;
            float lo = 0.0f, hi = Hi;
            bool hi_known = false;
            uint8_t state = st0;
            int nev = 0;
            float S0 = 0.f, S1 = 0.f, M0 = 0.f, M1 = 0.f;
            int cnt = 0;
            while (__any(!done)) {
                const float h2 = h * h;
                const float hinv = 1.0f / h;
                S0 = S1 = M0 = M1 = 0.f;
                cnt = 0;
                int active_groups = (!done && sub == 0) ? 1 : 0;
                for (int c0 = 0; c0 < nj; c0 += CAP) {
                    const int len = min(CAP, nj - c0);
                    if (!(single_tile && loaded)) {
                        stage_tile<1>(sj, A.jd, A.p_leaf, A.p_shift, A.lf_start, A.lf_count, pb0, np_all, c0, len);
                        loaded = true;
                    }
#pragma unroll 4
                    for (int k = sub; k < len; k += lpi) {
                        const float4 pj = sj[k];
                        const float dx = xi.x - pj.x, dy = xi.y - pj.y, dz = xi.z - pj.z;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const bool in = r2 < h2;
                        const float q = in ? sqrtf(r2) * hinv : 1.0f;
                        float w, dw;
                        spline_w_dw(q, w, dw);
                        const float qdw = q * dw;
                        S0 += w;
                        S1 += qdw;
                        M0 = fmaf(pj.w, w, M0);
                        M1 = fmaf(pj.w, qdw, M1);
                        cnt += in ? 1 : 0;
                    }
                    if (!single_tile) {
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                S0 = group_sum(S0, lpi);
                S1 = group_sum(S1, lpi);
                M0 = group_sum(M0, lpi);
                M1 = group_sum(M1, lpi);
                cnt = group_sum_i(cnt, lpi);
                // count tested pairs once per group
                for (int o = 32; o >= 1; o >>= 1) active_groups += __shfl_xor(active_groups, o, 64);
                cand_acc += (int64_t)active_groups * nj;
                if (!done && sub == 0) sweep_acc += cnt;
                if (done) continue;
                ++nev;
                const float ratio = S0 / A.target;
                if (fabsf(ratio - 1.0f) <= A.tol) {
                    done = true;
                    state = ST_DONE;
                    continue;
                }
                if (ratio < 1.0f) {
                    lo = h;
                } else {
                    hi = h;
                    hi_known = true;
                }
                if (ratio < 1.0f && h >= Hi) {
                    // the root lies beyond the search radius: ask for a rebuild,
                    // proposing the radius at which a uniform density would hold
                    // the target count
                    done = true;
                    state = ST_OVERFLOW;
                    continue;
                }
                const float slope = -S1 / S0;  // d ln S0 / d ln h
                float hn = slope > 0.05f ? h * __expf(-__logf(ratio) / slope) : 2.0f * h;
                if (hn >= hi) hn = hi_known ? 0.5f * (h + hi) : Hi;
                if (hn <= lo) hn = 0.5f * (lo + h);
                if (fabsf(hn - h) <= 2.5e-7f * h) {
                    // the next step is below FP32 resolution of h: h is the root
                    done = true;
                    state = ST_DONE;
                    continue;
                }
                if (nev >= A.max_iter) {
                    done = true;
                    state = ST_UNCONVERGED;
                    continue;
                }
                h = hn;
            }
            // results
            if (valid && sub == 0 && st0 == ST_ACTIVE) {
                const uint32_t o = A.perm[i];
                float h_report = h;
                if (state == ST_OVERFLOW) {
                    const float grow = cbrtf(A.target / S0);
                    h_report = h * fmaxf(grow, 1.0f) * 1.05f;
                    ++n_over;
                } else if (state == ST_UNCONVERGED) {
                    ++n_unconv;
                }
                const float hinv = 1.0f / h;
                const float rho = (8.0f / SPH_PI_F) * M0 * hinv * hinv * hinv;
                const float f = M1 < 0.0f ? -3.0f * M0 / M1 : 1.0f;
                A.hs[i] = h;
                A.rhos[i] = rho;
                A.fs[i] = f;
                A.st_s[i] = state;
                A.h_out[o] = h_report;
                A.rho_out[o] = rho;
                A.f_out[o] = f;
                if (A.nw_out) A.nw_out[o] = (32.0f / 3.0f) * S0;
                A.status[o] = state;
                if (state == ST_DONE) inter_acc += cnt - 1;
                max_ev = max(max_ev, nev);
            }
        }
    }
    // per-wave totals
    for (int o = 32; o >= 1; o >>= 1) {
        inter_acc += __shfl_xor(inter_acc, o, 64);
        sweep_acc += __shfl_xor(sweep_acc, o, 64);
        n_over += __shfl_xor(n_over, o, 64);
        n_unconv += __shfl_xor(n_unconv, o, 64);
        max_ev = max(max_ev, __shfl_xor(max_ev, o, 64));
    }
    if (lane == 0) {
        atomicAdd((unsigned long long*)&A.ctr[CT_DENS_INTER], (unsigned long long)inter_acc);
        atomicAdd((unsigned long long*)&A.ctr[CT_DENS_CAND], (unsigned long long)cand_acc);
        atomicAdd((unsigned long long*)&A.ctr[CT_DENS_SWEEP_INTER], (unsigned long long)sweep_acc);
        if (n_over) atomicAdd((unsigned long long*)&A.ctr[CT_OVERFLOW], (unsigned long long)n_over);
        if (n_unconv) atomicAdd((unsigned long long*)&A.ctr[CT_UNCONV], (unsigned long long)n_unconv);
        atomicMax((unsigned long long*)&A.ctr[CT_SWEEPS], (unsigned long long)max_ev);
    }
}

constexpr int DENS_CAP = 768;

}  // namespace

namespace sph {

void queue_bounds(int64_t n_items, int* q_begin)
{
    for (int q = 0; q <= 8; ++q) q_begin[q] = (int)((n_items * q) / 8);
}

int persistent_blocks(sph_ctx* c, int blocks_per_cu, int64_t n_items, int waves_per_block)
{
    int64_t want = (int64_t)c->n_cu * blocks_per_cu;
    int64_t cap = (n_items + waves_per_block - 1) / waves_per_block;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)want;
}

void density_f32(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw, sph_stats* st,
                 hipStream_t s)
{
    SPH_REQUIRE(c->built, SPH_E_STATE, "sph_density before sph_build_cells");
    SPH_REQUIRE(mass && h && rho && f, SPH_E_ARG, "null mass/h/rho/f");
    const int64_t n = c->n;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    uint8_t* status = ensure<uint8_t>(c, c->status, n);
    SPH_HIP(hipMemsetAsync(status, ST_ACTIVE, (size_t)n, s));
    int64_t tot_inter = 0, tot_cand = 0;
    int32_t sweeps = 0;
    c->rebuilds = 0;
    c->density_done = false;
    c->tm.density_kernel_ms = 0.0;
    c->tm.density_launches = 0;
    int64_t tot_sweep_inter = 0;
    ev_record(c, EV_DENS_C0, s);
    for (int pass = 0;; ++pass) {
        float4* jd = ensure<float4>(c, c->jd, n);
        float* hs = ensure<float>(c, c->hs, n);
        float* rhos = ensure<float>(c, c->rhos, n);
        float* fs = ensure<float>(c, c->fs, n);
        uint8_t* st_s = ensure<uint8_t>(c, c->st_s, n);
        SPH_HIP(hipMemsetAsync(ctr, 0, CT_COUNT * 8, s));
        k_dens_prologue<<<blocks_for(n, BS), BS, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p),
                                                          static_cast<float4*>(c->xrel.p), mass, h, status, jd,
                                                          hs, st_s, ctr);
        SPH_HIP(hipGetLastError());
        DensArgs A;
        A.jd = jd;
        A.Hs = static_cast<float*>(c->Hs.p);
        A.hs = hs;
        A.rhos = rhos;
        A.fs = fs;
        A.st_s = st_s;
        A.lf_start = static_cast<int*>(c->lf_start.p);
        A.lf_count = static_cast<int*>(c->lf_count.p);
        A.p_start = static_cast<uint32_t*>(c->p_start.p);
        A.p_leaf = static_cast<int*>(c->p_leaf.p);
        A.p_shift = static_cast<float4*>(c->p_shift.p);
        A.perm = static_cast<uint32_t*>(c->perm.p);
        A.h_out = h;
        A.rho_out = rho;
        A.f_out = f;
        A.nw_out = nw;
        A.status = status;
        A.ctr = ctr;
        queue_bounds(c->n_leaves, A.q_begin);
        A.target = (float)(3.0 * c->prm.n_ngb / 32.0);
        A.tol = (float)c->prm.n_tol;
        A.max_iter = c->prm.max_iter;
        const int grid = persistent_blocks(c, 3, c->n_leaves, WAVES);
        ev_record(c, EV_DENS_K0, s);
        k_density<DENS_CAP><<<grid, BS, 0, s>>>(A);
        SPH_HIP(hipGetLastError());
        ev_record(c, EV_DENS_K1, s);
        int64_t hc[CT_COUNT];
        SPH_HIP(hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
        SPH_HIP(hipStreamSynchronize(s));
        c->tm.density_kernel_ms += ev_ms(c, EV_DENS_K0, EV_DENS_K1);
        c->tm.density_launches += 1;
        tot_sweep_inter += hc[CT_DENS_SWEEP_INTER];
        SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "non-positive or non-finite mass or h");
        tot_inter += hc[CT_DENS_INTER];
        tot_cand += hc[CT_DENS_CAND];
        sweeps = std::max<int32_t>(sweeps, (int32_t)hc[CT_SWEEPS]);
        if (hc[CT_OVERFLOW] == 0) {
            if (st) {
                st->sweeps = sweeps;
                st->rebuilds = c->rebuilds;
                st->unconverged = hc[CT_UNCONV];
                st->interactions_density = tot_inter;
                st->interactions_force = 0;
                st->candidates_density = tot_cand;
                st->candidates_force = 0;
                st->sweep_interactions_density = tot_sweep_inter;
                st->n_cells = c->n_leaves;
                st->n_pairs = c->n_pairs;
            }
            if (c->rebuilds > 0) {
                k_dens_regather<<<blocks_for(n, BS), BS, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p), h, rho, f,
                                                                  hs, rhos, fs);
                SPH_HIP(hipGetLastError());
            }
            ev_record(c, EV_DENS_C1, s);
            c->tm.density_call_ms = ev_ms(c, EV_DENS_C0, EV_DENS_C1);
            SPH_REQUIRE(hc[CT_UNCONV] == 0, SPH_E_NOT_CONVERGED,
                        std::to_string(hc[CT_UNCONV]) + " smoothing lengths did not converge");
            c->density_done = true;
            return;
        }
        SPH_REQUIRE(c->rebuilds < 16, SPH_E_NOT_CONVERGED, "smoothing lengths keep outgrowing their cells");
        // cells around the current h (the overflowed particles report a larger
        // guess); converged particles keep their results and are skipped
        rebuild_cells(c, h, s);
        c->rebuilds += 1;
    }
}

}  // namespace sph
