// FP32 force loop: the pressure-gradient sum of the Swift paper (section 2,
// Eq. 2) in the grad-h form of Gadget-2 that Swift implements, with a
// signal-velocity artificial viscosity, in the internal-energy variable.
//
// The ghost step (after the density, section 3.1's dependency) turns rho, f
// and u into the per-particle pressure term Phi = f P / rho^2 and sound speed,
// packed with position, h^2, velocity, mass and 1/h into three float4 per
// particle: (x, y, z, h^2), (v, m), (rho, Phi, c, 1/h).
// The loop then runs one wavefront per leaf cell exactly like the density
// loop: the cell's neighbour particles are staged into LDS in chunks and each
// particle of the cell (several lanes per particle for small cells) gathers
// the terms of every pair inside max(h_i, h_j). The gather form evaluates each
// pair from both sides, so no two waves write the same particle and the result
// does not depend on scheduling. Per-box momentum and energy rates are summed
// in FP64: each wave stores its cell's share (plain stores, no atomics) and a
// second kernel adds the shares of each box's cells in a fixed order, so the
// sums are also reproducible.
//
// With the Balsara switch (not in the paper; the Gadget-2 form) the same loop
// first runs in a gather mode that sums the velocity divergence and curl of
// each particle over its neighbours inside h_i (staging only position and
// velocity, testing only r < h_i) and stores the factor
// B = |div v| / (|div v| + |curl v| + 1e-4 c / h) in place of 1/h in the
// particle's third float4, (rho, Phi, c, B); the force loop then takes 1/h
// from h^2 (a reciprocal square root) and scales each pair's viscosity by
// (B_i + B_j) / 2.
//
// sph_params.force_form = 1 swaps the grad-h pressure terms for the sum the
// paper prints as its illustration (Eq. 2): (P_i / rho_i^2 + P_j / rho_j^2)
// times the gradient of particle i's kernel, with no grad-h factor (the
// prologue then stores Phi = P / rho^2).
#include <type_traits>

#include "common.h"
#include "tiles.h"

namespace {

constexpr int BS = 64;     // one wavefront per block (finest LDS allocation)
constexpr int WAVES = BS / 64;
constexpr int FCAP = 128;  // candidates per LDS chunk (3 float4 each)
constexpr int FSLOTS = FCAP / 4;  // a lane (4+ lanes per particle) tests at most every fourth candidate
static_assert(FCAP % (2 * 4) == 0, "the phase-A stride (two candidates per lane, four lanes) divides a chunk");

__global__ void k_force_prologue(int64_t n, const uint32_t* __restrict__ perm, const float4* __restrict__ jd,
                                 const float* __restrict__ hs, const float* __restrict__ rhos,
                                 const float* __restrict__ fs, const float* __restrict__ vel,
                                 const float* __restrict__ u, float gamma, int with_f,
                                 float4* __restrict__ jf, int64_t* __restrict__ ctr)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    const float4 x = jd[p];
    const float h = hs[p];
    const float rho = rhos[p];
    const float uu = u[o];
    const float vx = vel[3 * (int64_t)o], vy = vel[3 * (int64_t)o + 1], vz = vel[3 * (int64_t)o + 2];
    if (!(uu >= 0.0f) || !isfinite(uu) || !isfinite(vx) || !isfinite(vy) || !isfinite(vz))
        atomicAdd((unsigned long long*)&ctr_slot(ctr)[CT_BAD_INPUT], 1ull);
    const float P = (gamma - 1.0f) * rho * uu;
    const float c = sqrtf(gamma * (gamma - 1.0f) * uu);
    const float phi = (with_f ? fs[p] : 1.0f) * P / (rho * rho);
    jf[3 * p + 0] = make_float4(x.x, x.y, x.z, h * h);
    jf[3 * p + 1] = make_float4(vx, vy, vz, x.w);
    jf[3 * p + 2] = make_float4(rho, phi, c, 1.0f / h);
}

struct ForceArgs {
    const float4* jf;
    float4* jf_w;             // the same array, written by the divergence pass (B in place of 1/h)
    const int4* cells;     // per schedule slot: first particle, count, first neighbour entry, entries
    const int2* cell_aux;  // per schedule slot: leaf, box
    const int2* p_rec;       // per (cell, neighbour cell) record: first particle and count of the neighbour
    const float4* p_shift;
    const uint32_t* perm;
    float* acc;
    float* dudt;
    double* cons_part;  // 4 per leaf, may be null
    float* vsig;        // sorted: signal velocity per particle (k_force<true> only)
    float* divv;        // sorted: velocity divergence per particle (k_force<true> only)
    float* bal;         // sorted: Balsara factor per particle (written in the FM_DIVCURL mode)
    const float* drift; // [0]: bound on the drift since the build (cell boxes widen by it)
    int64_t* ctr;
    WorkSched W;
    float alpha;
};

// Phase A of one chunk for the lanes of one particle: the lane with index sub
// in its group tests candidates sub, sub + LPI, ... (slot 0 of the tile: x,
// y, z, h^2) and appends the chunk index of every candidate inside
// max(h_i, h_j), except the particle itself, to its byte list (row e of the
// lists holds entry e of every lane; o is the byte offset of this lane's next
// entry). The chunk is padded with far positions to its full size
// (pad_tile), two tile reads are in flight (four, or eight, measured slower:
// the registers they hold) and the appends are branch-free.
// A lane (four per particle) tests at most FCAP / 4 candidates of a chunk,
// so its list of FSLOTS cannot overflow.
// OWN_H false (the divergence and curl): only the pairs inside h_i.
template <int LPI, bool OWN_H>
__device__ __forceinline__ int force_scan(const float4* sj, int len, int sub, float xx, float xy, float xz,
                                          float h2_i, uint8_t* lists)
{
    const int len_pad = (len + 2 * LPI - 1) & ~(2 * LPI - 1);
    const unsigned o0 = threadIdx.x & 63;
    unsigned o = o0;
    for (int k0 = sub; k0 < len_pad; k0 += 2 * LPI) {
        float4 pj[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) pj[u] = sj[k0 + u * LPI];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float dx = xx - pj[u].x, dy = xy - pj[u].y, dz = xz - pj[u].z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const bool in = (r2 < (OWN_H ? fmaxf(h2_i, pj[u].w) : h2_i)) & (r2 > 0.0f);
            lists[o] = (uint8_t)(k0 + u * LPI);
            o += in ? 64u : 0u;
        }
    }
    return (int)((o - o0) >> 6);
}

// Slot 0 of the unused tile entries [len, CAP): a far position with a tiny
// h^2, so no pair test passes there.
__device__ __forceinline__ void pad_tile(float4* sj, int len, int cap)
{
    for (int t = len + (int)(threadIdx.x & 63); t < cap; t += 64) sj[t] = make_float4(1.0e18f, 1.0e18f, 1.0e18f, 1.0e-12f);
    wave_sync_lds();
}

// What a pass of k_force computes: the force; the force with the Balsara
// switch (4 float4 per particle); the Balsara factors (3 float4 per particle,
// no force, no counters); the force in the Eq. 2 form.
enum { FM_FORCE = 0, FM_BALSARA = 1, FM_DIVCURL = 2, FM_EQ2 = 3 };
// With FM_BALSARA the third float4 of a particle holds (rho, Phi, c, B).

// Input-order copy of the sorted Balsara factors.
__global__ void k_unsort_f32(int64_t n, const uint32_t* __restrict__ perm, const float* __restrict__ src,
                             float* __restrict__ dst)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) dst[perm[p]] = src[p];
}

// VSIG: also record each particle's signal velocity max(c_i, max_j (c_i +
// c_j - 3 w_ij)) over its pairs, for the Courant time step, and its velocity
// divergence, rho_i div v_i = -sum_j m_j (v_i - v_j) . grad_i W(r_ij, h_i)
// (the pairs inside h_i; grad_i W = D_i rhat), from which the next step's
// smoothing length is predicted (continuity: dh/dt = h div v / 3).
// ONEBLK: every cell has at most 64 neighbour records (a layout of top cells
// only has 27), so the multi-block paths of the record cursor drop out.
template <bool VSIG, int MODE, bool ONEBLK>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) k_force(ForceArgs A)
{
    constexpr bool DC = MODE == FM_DIVCURL;
    constexpr int NF = DC ? 2 : 3;  // float4 staged per candidate (of the 3 per particle)
    __shared__ float4 tile[NF * FCAP];
    __shared__ uint8_t lists[FSLOTS * 64];
    __shared__ uint8_t marks[FCAP];  // record starts of the chunk being fetched
    const int lane = threadIdx.x & 63;
    float4* sj = tile;
    uint8_t* lst = lists + lane;
    int wstate = 0, a_cur = 0, a_end = 0;
    int64_t cand_acc = 0, inter_acc = 0;
    const float K8PI = 8.0f / SPH_PI_F;

    for (;;) {
        if (a_cur >= a_end && !next_items(A.W, A.ctr, WAVES, wstate, a_cur, a_end)) break;
        const int slot = a_cur++;
        const int4 ci = A.cells[slot];
        const int i0 = ci.x, ni = ci.y, pb0 = ci.z, np_all = ONEBLK ? min(ci.w, 64) : ci.w;
        NbrCursor cu;  // neighbour records 64 at a time
        cursor_init(cu, A.p_rec, A.p_shift, pb0, np_all);
        const int nj = np_all <= 64 ? cu.nb.nj : count_candidates(A.p_rec, pb0, np_all);
        // four lanes per particle on every cell: a lane's byte list (one
        // chunk's hits) cannot overflow, and the fixed count lets the
        // compiler specialise every loop (measured faster on every set than
        // a per-cell choice, even where leaves hold few particles)
        constexpr int lpi = 4;
        constexpr int lg = 2;
        constexpr int per_pass = 64 >> lg;
        const int g = lane >> lg;
        const int sub = lane & (lpi - 1);
        // this cell's share of the box sums: lane 0's totals, kept in scalar
        // registers across the passes (every lane is active where they change)
        double cm_cell[4] = {0.0, 0.0, 0.0, 0.0};
        for (int ib = 0; ib < ni; ib += per_pass) {
            const int gi = ib + g;
            const bool valid = gi < ni;
            const int i = i0 + (valid ? gi : 0);
            const float4 i0v = A.jf[3 * (int64_t)i + 0];
            const float4 i1v = A.jf[3 * (int64_t)i + 1];
            const float4 i2v = A.jf[3 * (int64_t)i + 2];
            const uint32_t o_i = DC ? 0u : A.perm[i];  // loaded here so the stores wait for nothing
            const float bal_i = MODE == FM_BALSARA ? i2v.w : 1.0f;
            const float h2_i = i0v.w;
            const float hinv_i = MODE == FM_BALSARA ? __builtin_amdgcn_rsqf(h2_i) : i2v.w;
            // every pass stages its own candidates (with four lanes a cell of
            // up to 16 particles takes one pass, so a tile kept across passes
            // would save little, and dropping it frees registers): those within
            // the pass's largest h, or their own, of the box around its
            // particles
            const float reach2 = uniform_f(cull_reach2(sqrtf(wave_max(valid ? h2_i : 0.0f))));
            const CullBox box = pass_box(i0v.x, i0v.y, i0v.z, valid);
            const float hinv2_i = hinv_i * hinv_i;
            const float Ki = K8PI * hinv2_i * hinv2_i;
            const float rho_i = i2v.x, phi_i = i2v.y, c_i = i2v.z;
            float ax = 0.f, ay = 0.f, az = 0.f, du = 0.f;
            float vmax = 0.f;  // (VSIG) largest c_i + c_j - 3 w_ij of this lane's pairs
            float dvr = 0.f;   // (VSIG) sum_j m_j D_i (v_ij . rhat) = -rho_i div v_i
            int cnt = 0;
            ChunkRegs<NF, FCAP> R;
            int len, kept = 0;  // candidates of this chunk; kept by the box test (all chunks)
            for (int c0 = 0; c0 < nj; c0 += len) {
                // stage this chunk's candidates within reach of the pass
                // (loaded and stored here rather than one chunk ahead: the
                // registers a fetch in flight would hold cost a wavefront per
                // SIMD, and the other wavefronts cover the loads)
                cursor_seek(cu, A.p_rec, A.p_shift, c0);
                fetch_chunk<NF, FCAP, 3>(R, A.jf, cu.nb, c0 - cu.off0, cursor_chunk(cu, c0, FCAP), marks);
                len = R.len;
                const int slen = commit_chunk_culled<NF, FCAP, !DC>(sj, R, box, reach2);
                pad_tile(sj, slen, FCAP);
                kept += slen;
                // phase A: compact the candidates inside max(h_i, h_j) of this chunk
                int nl = force_scan<lpi, !DC>(sj, slen, sub, i0v.x, i0v.y, i0v.z, h2_i, lists);
                if (!valid) nl = 0;
                cnt += nl;
                // phase B: the pair terms of the compacted neighbours only (not
                // unrolled: the lanes' list lengths differ, and a second copy of
                // the body measured 2% slower on every set)
#pragma unroll 1
                for (int e = 0; e < nl; ++e) {
                    const int k = lst[e * 64];
                    const float4 p0 = sj[k];
                    const float4 p1 = sj[FCAP + k];
                    const float4 p2 = DC ? p1 : sj[2 * FCAP + k];  // (not staged for the divergence)
                    const float dx = i0v.x - p0.x, dy = i0v.y - p0.y, dz = i0v.z - p0.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    if constexpr (DC) {
                        // rho_i div v_i = -sum m_j D_i (v_i - v_j) . rhat, rho_i curl v_i =
                        // sum m_j D_i (v_i - v_j) x rhat; D_i is 0 from r = h_i on
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float mD = p1.w * Ki * spline_dw_r(r2 * rinv, hinv_i) * rinv;
                        const float wx = i1v.x - p1.x, wy = i1v.y - p1.y, wz = i1v.z - p1.z;
                        du = fmaf(mD, fmaf(wx, dx, fmaf(wy, dy, wz * dz)), du);
                        ax = fmaf(mD, wy * dz - wz * dy, ax);
                        ay = fmaf(mD, wz * dx - wx * dz, ay);
                        az = fmaf(mD, wx * dy - wy * dx, az);
                        continue;
                    }
                    const float hinv_j = MODE == FM_BALSARA ? __builtin_amdgcn_rsqf(p0.w) : p2.w;
                    const float hinv2_j = hinv_j * hinv_j;
                    const float rinv = __builtin_amdgcn_rsqf(r2);  // r2 > 0 (phase A), far from denormal
                    const float r = r2 * rinv;
                    const float Di = Ki * spline_dw_r(r, hinv_i);
                    const float Dj = K8PI * hinv2_j * hinv2_j * spline_dw_r(r, hinv_j);
                    const float vr = ((i1v.x - p1.x) * dx + (i1v.y - p1.y) * dy + (i1v.z - p1.z) * dz) * rinv;
                    const float wv_ = fminf(vr, 0.0f);
                    const float vsig_ij = c_i + p2.z - 3.0f * wv_;
                    float visc = -A.alpha * vsig_ij * wv_ * __builtin_amdgcn_rcpf(rho_i + p2.x);
                    if constexpr (MODE == FM_BALSARA) visc *= 0.5f * (bal_i + p2.w);
                    if constexpr (VSIG) {
                        vmax = fmaxf(vmax, vsig_ij);
                        dvr = fmaf(p1.w * Di, vr, dvr);
                    }
                    const float Dbar = 0.5f * (Di + Dj);
                    const float G = MODE == FM_EQ2 ? fmaf(phi_i + p2.y, Di, visc * Dbar)
                                                   : fmaf(phi_i, Di, fmaf(p2.y, Dj, visc * Dbar));
                    const float mGr = p1.w * G * rinv;
                    ax = fmaf(-mGr, dx, ax);
                    ay = fmaf(-mGr, dy, ay);
                    az = fmaf(-mGr, dz, az);
                    du = fmaf(p1.w * fmaf(phi_i, Di, 0.5f * visc * Dbar), vr, du);
                }
                // every lane is done with the tile before the next chunk is staged
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            ax = group_sum(ax, lpi);
            ay = group_sum(ay, lpi);
            az = group_sum(az, lpi);
            du = group_sum(du, lpi);
            cnt = group_sum_i(cnt, lpi);
            if constexpr (VSIG) {
                vmax = group_max(vmax, lpi);
                dvr = group_sum(dvr, lpi);
            }
            const bool leader = valid && sub == 0;
            if constexpr (DC) {
                if (leader) {
                    const float ad = fabsf(du) / rho_i;
                    const float den = ad + sqrtf(fmaf(ax, ax, fmaf(ay, ay, az * az))) / rho_i +
                                      1.0e-4f * c_i * hinv_i;
                    const float B = den > 0.0f ? ad / den : 0.0f;  // no motion and no sound: no viscosity
                    A.bal[i] = B;
                    // B replaces 1/h in the particle's third float4 for the force
                    // pass (the candidates of this pass read only the first two)
                    A.jf_w[3 * (int64_t)i + 2] = make_float4(rho_i, phi_i, c_i, B);
                }
                continue;
            }
            cand_acc += (int64_t)wave_count(leader) * kept;
            double cm[4] = {0.0, 0.0, 0.0, 0.0};
            if (leader) {
                A.acc[3 * (int64_t)o_i + 0] = ax;
                A.acc[3 * (int64_t)o_i + 1] = ay;
                A.acc[3 * (int64_t)o_i + 2] = az;
                A.dudt[o_i] = du;
                if constexpr (VSIG) {
                    A.vsig[i] = fmaxf(vmax, c_i);
                    A.divv[i] = -dvr / rho_i;
                }
                inter_acc += cnt;
                const double m = i1v.w;
                cm[0] = m * ax;
                cm[1] = m * ay;
                cm[2] = m * az;
                cm[3] = m * ((double)i1v.x * ax + (double)i1v.y * ay + (double)i1v.z * az + (double)du);
            }
            if (A.cons_part) {
                // only the group leaders (lanes g * lpi) hold terms: the
                // exchanges at distances below lpi would add zeros
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    for (int o = 32; o >= lpi; o >>= 1) cm[k] += __shfl_xor(cm[k], o, 64);
                    cm_cell[k] = lane0_d(cm_cell[k] + cm[k]);
                }
            }
        }
        if (!DC && A.cons_part && lane == 0) {
            const int leaf = A.cell_aux[slot].x;
#pragma unroll
            for (int k = 0; k < 4; ++k) A.cons_part[4 * (int64_t)leaf + k] = cm_cell[k];
        }
    }
    if constexpr (!DC) {
        ctr_wave_add(A.ctr, CT_FORCE_INTER, inter_acc);
        ctr_add_uniform(A.ctr, CT_FORCE_CAND, cand_acc);  // already a wavefront total
    }
}

// Per-box sums of the cells' shares: block b adds the shares of its leaves
// [box_leaf[b], box_leaf[b + 1]) in a fixed order (strided partial sums, then
// a tree in LDS), so the result does not depend on scheduling.
constexpr int CR_BS = 1024;

__global__ void __launch_bounds__(CR_BS) k_cons_reduce(const int* __restrict__ box_leaf,
                                                       const double* __restrict__ cons_part, double* __restrict__ cons)
{
    __shared__ double red[4][CR_BS];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const int l0 = box_leaf[b], l1 = box_leaf[b + 1];
    // two partial sums per thread (leaves t, t + 2 CR_BS, ... and t + CR_BS,
    // t + 3 CR_BS, ...): two loads in flight, one fixed order
    double v[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = l0 + t; l < l1; l += 2 * CR_BS) {
        const bool second = l + CR_BS < l1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] += cons_part[4 * (int64_t)l + k];
            w[k] += second ? cons_part[4 * (int64_t)(l + CR_BS) + k] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][t] = v[k] + w[k];
    __syncthreads();
    for (int half = CR_BS / 2; half >= 1; half >>= 1) {
        if (t < half) {
#pragma unroll
            for (int k = 0; k < 4; ++k) red[k][t] += red[k][t + half];
        }
        __syncthreads();
    }
    if (t < 4) cons[4 * (int64_t)b + t] = red[t][0];
}

}  // namespace

namespace sph {

int make_sched(sph_ctx* c, int64_t n_items, int waves_per_block, int blocks_per_cu, WorkSched& W);

void mark_force_outputs(sph_ctx* c)
{
    c->vsig_valid = c->prm.signal_velocity != 0;
    c->div_valid = c->prm.signal_velocity != 0;
    c->bal_valid = c->prm.balsara != 0 && c->prm.alpha_visc > 0;
}

void force_enqueue(sph_ctx* c, const float* vel, const float* u, float* acc, float* dudt, double* cons_d,
                   bool clear_all, bool events, hipStream_t s, bool prologue)
{
    const int64_t n = c->n;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    float4* jf = static_cast<float4*>(c->jf.p);
    // all counters, or (after a density pass whose counters are still to be
    // read) only the work-queue heads, which only the persistent schedule uses
    if (clear_all)
        fill_u32(ctr, 0u, 2 * (int64_t)CT_COUNT, s);
    else if (c->prm.schedule == 1)
        fill_u32(ctr + CT_QUEUE, 0u, 2 * 64, s);
    const bool eq2 = c->prm.force_form == 1;
    if (prologue || eq2) {  // else the density kernels wrote the streams (ghost step fused)
        k_force_prologue<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p),
                                                             static_cast<float4*>(c->jd.p),
                                                             static_cast<float*>(c->hs.p),
                                                             static_cast<float*>(c->rhos.p),
                                                             static_cast<float*>(c->fs.p), vel, u,
                                                             (float)c->prm.gamma, eq2 ? 0 : 1, jf, ctr);
        SPH_HIP(hipGetLastError());
    }
    ForceArgs A;
    A.jf = jf;
    A.jf_w = jf;
    A.cells = static_cast<int4*>(c->cells.p);
    A.cell_aux = static_cast<int2*>(c->cell_aux.p);
    A.p_rec = static_cast<int2*>(c->p_rec.p);
    A.p_shift = static_cast<float4*>(c->p_shift.p);
    A.perm = static_cast<uint32_t*>(c->perm.p);
    A.acc = acc;
    A.dudt = dudt;
    A.cons_part = cons_d ? static_cast<double*>(c->cons_part.p) : nullptr;
    const bool vsig = c->prm.signal_velocity != 0;
    A.vsig = vsig ? static_cast<float*>(c->vsig_s.p) : nullptr;
    A.divv = vsig ? static_cast<float*>(c->divv_s.p) : nullptr;
    A.bal = static_cast<float*>(c->bal_s.p);
    A.drift = static_cast<float*>(c->drift.p);
    A.ctr = ctr;
    const int grid = make_sched(c, c->n_leaves, WAVES, 16, A.W);
    A.alpha = c->prm.alpha_visc > 0 ? (float)c->prm.alpha_visc : 0.0f;
    if (events) ev_record(c, EV_FORCE_K0, s);
    const bool bal = c->prm.balsara != 0 && A.alpha > 0.0f;
    // a layout of top cells only (no split) has at most 27 records per cell
    const bool one_block = !c->cells_refined;
    auto go = [&](auto vs, auto md) {
        constexpr bool V = decltype(vs)::value;
        constexpr int M = decltype(md)::value;
        if (one_block)
            k_force<V, M, true><<<grid, BS, 0, s>>>(A);
        else
            k_force<V, M, false><<<grid, BS, 0, s>>>(A);
    };
    using T = std::true_type;
    using F = std::false_type;
    if (bal) {
        go(F{}, std::integral_constant<int, FM_DIVCURL>{});
        SPH_HIP(hipGetLastError());
        if (c->prm.schedule == 1) fill_u32(ctr + CT_QUEUE, 0u, 2 * 64, s);  // the force pass pops the queues again
        if (vsig)
            go(T{}, std::integral_constant<int, FM_BALSARA>{});
        else
            go(F{}, std::integral_constant<int, FM_BALSARA>{});
    } else if (eq2) {
        if (vsig)
            go(T{}, std::integral_constant<int, FM_EQ2>{});
        else
            go(F{}, std::integral_constant<int, FM_EQ2>{});
    } else if (vsig) {
        go(T{}, std::integral_constant<int, FM_FORCE>{});
    } else {
        go(F{}, std::integral_constant<int, FM_FORCE>{});
    }
    SPH_HIP(hipGetLastError());
    if (events) ev_record(c, EV_FORCE_K1, s);
    if (cons_d) {
        k_cons_reduce<<<c->n_boxes, CR_BS, 0, s>>>(static_cast<int*>(c->box_leaf.p), A.cons_part, cons_d);
        SPH_HIP(hipGetLastError());
    }
}

double* force_buffers(sph_ctx* c, bool cons)
{
    SPH_REQUIRE(c->prm.force_form == 0 || c->prm.force_form == 1, SPH_E_ARG, "sph_params.force_form must be 0 or 1");
    SPH_REQUIRE(!(c->prm.force_form == 1 && c->prm.balsara), SPH_E_ARG,
                "the Eq. 2 force form (force_form = 1) has no Balsara switch");
    ensure<float4>(c, c->jf, 3 * c->n);
    if (c->prm.signal_velocity) {
        ensure<float>(c, c->vsig_s, c->n);
        ensure<float>(c, c->divv_s, c->n);
    }
    if (c->prm.balsara) ensure<float>(c, c->bal_s, c->n);
    if (!cons) return nullptr;
    ensure<double>(c, c->cons_part, (size_t)4 * c->n_leaves);
    return ensure<double>(c, c->cons_d, (size_t)4 * c->n_boxes);
}

void force_f32(sph_ctx* c, const float* vel, const float* u, float* acc, float* dudt, double* cons,
               sph_stats* st, hipStream_t s)
{
    SPH_REQUIRE(c->built && c->density_done, SPH_E_STATE, "sph_force needs a successful sph_density first");
    SPH_REQUIRE(vel && u && acc && dudt, SPH_E_ARG, "null vel/u/acc/dudt");
    double* cons_d = force_buffers(c, cons != nullptr);
    // the sorted signal velocities and Balsara factors are rewritten below:
    // they are valid again only once this pass has succeeded
    c->vsig_valid = c->bal_valid = c->div_valid = false;
    ev_record(c, EV_FORCE_C0, s);
    force_enqueue(c, vel, u, acc, dudt, cons_d, true, true, s);
    if (cons || st) {
        const int64_t* hc = read_counters(c, s, cons_d, cons);
        SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "negative or non-finite u, or non-finite velocity");
        if (st) {
            st->interactions_force = hc[CT_FORCE_INTER];
            st->candidates_force = hc[CT_FORCE_CAND];
            st->n_cells = c->n_leaves;
            st->n_pairs = c->n_pairs;
        }
    }
    mark_force_outputs(c);
    ev_record(c, EV_FORCE_C1, s);
    if (c->prm.timing) {
        c->tm.force_kernel_ms = ev_ms(c, EV_FORCE_K0, EV_FORCE_K1);
        c->tm.force_call_ms = ev_ms(c, EV_FORCE_C0, EV_FORCE_C1);
    }
}

void balsara_unsort(sph_ctx* c, float* out, hipStream_t s)
{
    SPH_REQUIRE(out, SPH_E_ARG, "null output");
    SPH_REQUIRE(c->built && c->bal_valid, SPH_E_STATE,
                "sph_get_balsara needs a force pass with sph_params.balsara (and viscosity) since the last build or drift");
    if (c->n == 0) return;
    k_unsort_f32<<<blocks_for(c->n, 256), 256, 0, s>>>(c->n, static_cast<uint32_t*>(c->perm.p),
                                                      static_cast<float*>(c->bal_s.p), out);
    SPH_HIP(hipGetLastError());
}

}  // namespace sph
