// Near-field gravity, particle-particle: Newton's pull of section 2, Eq. 3 of
// the Swift paper, summed directly over the pairs of neighbouring cells, the
// part that the tree code of section 3.2 evaluates particle by particle:
//
//   g_i = -G sum_{j != i} m_j r_ij (r_ij^2 + eps^2)^(-3/2) S(r_ij / r_cut),
//
// r_ij the minimum image of x_i - x_j, eps a Plummer softening and
// S(x) = (1 - x^2)^2 below 1, 0 beyond: the window takes the pull to zero
// with zero slope at the cutoff, so the sum is continuous in the positions
// (the remaining 1 - S belongs to a far field of multipoles, not computed
// here). Coincident pairs add nothing.
//
// Work unit: one leaf cell per wavefront, as in the density loop. Its
// candidates are the particles of the leaves within the cell's own largest
// search radius (the first part of its neighbour records), which the cutoff
// may not exceed, so every pair inside r_cut is among them. They are staged
// through LDS in chunks of GCH, shifted into the cell frame, keeping only
// those within r_cut of the bounding box of the particles in the pass (the
// cutoff is usually well inside the search radius the lists were built for);
// the lanes of each particle split the kept candidates and add up their
// pairs, then meet in a group sum. It is a gather: each particle sums its own
// pairs, so there are no atomics and the result has the same bits on every
// run.
#include <cmath>

#include "common.h"
#include "tiles.h"

namespace {

constexpr int GBS = 64;   // one wavefront per block
constexpr int GCH = 256;  // candidates per staged chunk

struct GravArgs {
    const float4* jg;       // sorted (x, y, z) in the leaf frame, m
    const uint32_t* perm;   // sorted index -> caller index
    const int4* cells;      // per schedule slot: first particle, count, first record, density records
    const int2* p_rec;      // per record: first particle and count of the neighbour leaf
    const float4* p_shift;  // per record: frame shift of the neighbour leaf
    float* acc;             // caller order, 3 per particle
    int64_t* ctr;
    int n_slots;
    float G, eps2, rc2, inv_rc2;
};

// Sorted copies of position (leaf frame) and mass; counts non-positive or
// non-finite masses.
__global__ void __launch_bounds__(256) k_grav_prologue(int64_t n, const uint32_t* __restrict__ perm,
                                                       const float4* __restrict__ xrel,
                                                       const float* __restrict__ mass, float4* __restrict__ jg,
                                                       int64_t* __restrict__ ctr)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (p < n) {
        const float m = mass[perm[p]];
        const float4 x = xrel[p];
        jg[p] = make_float4(x.x, x.y, x.z, m);
        bad = !(m > 0.0f) || !isfinite(m);
    }
    const int n_bad = __syncthreads_count(bad);
    if (threadIdx.x == 0 && n_bad) atomicAdd((unsigned long long*)&ctr_slot(ctr)[CT_BAD_INPUT], (unsigned long long)n_bad);
}

// Store a fetched chunk (x, y, z, m in the cell frame) keeping only the
// candidates within reach of `box`, packed from slot 0; the slots after them
// up to GCH get a massless candidate far outside r_cut, so the pair loop may
// run to a multiple of its stride without a bounds test. Returns how many
// were kept.
__device__ __forceinline__ int commit_culled(float4* sj, const ChunkRegs<1, GCH>& R, const CullBox& box,
                                             float reach2)
{
    const int lane = threadIdx.x & 63;
    constexpr int PER = GCH / 64;
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
    wave_sync_lds();
    return n;
}

// The pairs of one particle with the staged candidates sub, sub + LPI, ...
// below len (rounded up to a multiple of 4 LPI: the padding adds nothing),
// four tile reads in flight at once. The pull on i is -m_j S (r^2 + eps^2)^(-3/2)
// r_ij per pair inside r_cut; a pair outside (or at r = 0) is selected away,
// so the far padding's overflows never reach the sums. rc2 is the lane's:
// below zero on a lane without a particle. The pairs inside are counted for
// the whole wavefront (a ballot of the same test, in scalar registers).
template <int LPI>
__device__ __forceinline__ void pair_chunk(const float4* tc, int len, const float4& xi, float rc2, float inv_rc2,
                                           float eps2, float& ax, float& ay, float& az, int& wcnt)
{
    const int len_pad = (len + 4 * LPI - 1) & ~(4 * LPI - 1);
    for (int k0 = 0; k0 < len_pad; k0 += 4 * LPI, tc += 4 * LPI) {
        float4 pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pj[u] = tc[u * LPI];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float dx = xi.x - pj[u].x, dy = xi.y - pj[u].y, dz = xi.z - pj[u].z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            const bool in = r2 < rc2 && r2 > 0.0f;
            const float s = fmaf(-r2, inv_rc2, 1.0f);                 // 1 - x^2
            const float inv = __builtin_amdgcn_rsqf(r2 + eps2);      // (r^2 + eps^2)^(-1/2)
            const float f = in ? pj[u].w * (s * s) * (inv * inv * inv) : 0.0f;
            ax = fmaf(-f, dx, ax);
            ay = fmaf(-f, dy, ay);
            az = fmaf(-f, dz, az);
            wcnt += __popcll(__ballot(in));
        }
    }
}

// ONEBLK: every cell has at most 64 records (a layout of top cells only has
// 27), so the multi-block paths of the record cursor drop out.
template <bool ONEBLK>
__global__ void __launch_bounds__(GBS) k_gravity(GravArgs A)
{
    __shared__ float4 tile[GCH];
    __shared__ uint8_t marks[GCH];  // record starts of the chunk being fetched
    const int lane = threadIdx.x & 63;
    const int slot = xcd_block_index();  // each XCD takes its own run of slots
    if (slot >= A.n_slots) return;       // whole wavefront
    const int4 ci = A.cells[slot];
    const int i0 = ci.x, ni = ci.y, pb0 = ci.z, np = ONEBLK ? min(ci.w, 64) : ci.w;
    NbrCursor cu;
    cursor_init(cu, A.p_rec, A.p_shift, pb0, np);
    const int nj = np <= 64 ? cu.nb.nj : count_candidates(A.p_rec, pb0, np);
    // lanes per particle: the cell's particles spread over the wavefront
    int lpi = 1;
    while (lpi < 16 && 2 * lpi * ni <= 64) lpi *= 2;
    const int per_pass = 64 / lpi;
    const int g = lane / lpi, sub = lane & (lpi - 1);
    const float reach2 = cull_reach2(uniform_f(sqrtf(A.rc2)));
    int pairs = 0;  // wave-uniform
    int64_t tested = 0;
    for (int ib = 0; ib < ni; ib += per_pass) {
        const int gi = ib + g;
        const bool valid = gi < ni;
        const int i = i0 + (valid ? gi : 0);
        const float4 xi = A.jg[i];
        // only the candidates within r_cut of the pass's bounding box can pair
        const CullBox box = pass_box(xi.x, xi.y, xi.z, valid);
        const int n_valid = min(per_pass, ni - ib);
        const float rc2 = valid ? A.rc2 : -1.0f;
        float ax = 0.0f, ay = 0.0f, az = 0.0f;
        ChunkRegs<1, GCH> R;
        cursor_seek(cu, A.p_rec, A.p_shift, 0);
        fetch_chunk(R, A.jg, cu.nb, 0, cursor_chunk(cu, 0, GCH), marks);
        int len;
        for (int c0 = 0; c0 < nj; c0 += len) {
            len = R.len;
            const int kept = commit_culled(tile, R, box, reach2);
            // the next chunk's loads are in flight while this one is summed
            const int nx = c0 + len;
            if (nx < nj) {
                cursor_seek(cu, A.p_rec, A.p_shift, nx);
                fetch_chunk(R, A.jg, cu.nb, nx - cu.off0, cursor_chunk(cu, nx, GCH), marks);
            }
            tested += (int64_t)n_valid * kept;
            const float4* tc = tile + sub;
            if (lpi == 1)
                pair_chunk<1>(tc, kept, xi, rc2, A.inv_rc2, A.eps2, ax, ay, az, pairs);
            else if (lpi == 2)
                pair_chunk<2>(tc, kept, xi, rc2, A.inv_rc2, A.eps2, ax, ay, az, pairs);
            else if (lpi == 4)
                pair_chunk<4>(tc, kept, xi, rc2, A.inv_rc2, A.eps2, ax, ay, az, pairs);
            else if (lpi == 8)
                pair_chunk<8>(tc, kept, xi, rc2, A.inv_rc2, A.eps2, ax, ay, az, pairs);
            else
                pair_chunk<16>(tc, kept, xi, rc2, A.inv_rc2, A.eps2, ax, ay, az, pairs);
            wave_sync_lds();  // every lane is done with the tile before it is staged again
        }
        ax = group_sum(ax, lpi);
        ay = group_sum(ay, lpi);
        az = group_sum(az, lpi);
        if (valid && sub == 0) {
            const uint32_t o = A.perm[i];
            A.acc[3 * (int64_t)o + 0] = A.G * ax;
            A.acc[3 * (int64_t)o + 1] = A.G * ay;
            A.acc[3 * (int64_t)o + 2] = A.G * az;
        }
    }
    // the gravity call has the counters to itself
    ctr_add_uniform(A.ctr, CT_FORCE_INTER, pairs);
    ctr_add_uniform(A.ctr, CT_FORCE_CAND, tested);
}

}  // namespace

namespace sph {

void gravity_p2p(sph_ctx* c, const float* mass, double G, double eps, double r_cut, float* acc,
                 int64_t* counts, hipStream_t s)
{
    SPH_REQUIRE(c->built, SPH_E_STATE, "sph_gravity_p2p before sph_build_cells");
    SPH_REQUIRE(mass && acc, SPH_E_ARG, "null mass or acc");
    SPH_REQUIRE(std::isfinite(G) && std::isfinite(eps) && eps >= 0.0, SPH_E_ARG,
                "G must be finite and eps finite and >= 0");
    SPH_REQUIRE(std::isfinite(r_cut) && r_cut > 0.0, SPH_E_ARG, "r_cut must be finite and > 0");
    // after drifts that used up the margin of the cells, rebuild them around
    // the guesses of the last build (as the density would)
    check_drift(c, nullptr, s);
    finish_build_read(c);  // the smallest search radius of the build
    // the lists hold every pair closer than the search radius less twice the
    // distance the particles may have moved since the build. A search radius
    // is at most a third of its box (a build condition), so no two periodic
    // images of one particle both lie inside r_cut.
    unsigned w[4] = {0u, 0u, 0u, 0u};
    SPH_HIP(hipMemcpyAsync(w, c->drift.p, sizeof(w), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    float delta;
    std::memcpy(&delta, &w[0], 4);
    SPH_REQUIRE(r_cut + 2.0 * (double)delta <= (double)c->h_min, SPH_E_ARG,
                "r_cut " + std::to_string(r_cut) + " exceeds the smallest search radius of the cells (" +
                    std::to_string(c->h_min) + ", less twice the drift since the build)");
    const int64_t n = c->n;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    float4* jg = ensure<float4>(c, c->jg, n);
    fill_u32(ctr, 0u, 2 * (int64_t)CT_COUNT, s);
    k_grav_prologue<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p),
                                                       static_cast<float4*>(c->xrel.p), mass, jg, ctr);
    SPH_HIP(hipGetLastError());
    GravArgs A;
    A.jg = jg;
    A.perm = static_cast<uint32_t*>(c->perm.p);
    A.cells = static_cast<int4*>(c->cells_d.p);
    A.p_rec = static_cast<int2*>(c->p_rec.p);
    A.p_shift = static_cast<float4*>(c->p_shift.p);
    A.acc = acc;
    A.ctr = ctr;
    A.n_slots = (int)c->n_leaves;
    A.G = (float)G;
    A.eps2 = (float)(eps * eps);
    A.rc2 = (float)(r_cut * r_cut);
    A.inv_rc2 = (float)(1.0 / (r_cut * r_cut));
    ev_record(c, EV_GRAV_K0, s);
    const unsigned grid = (unsigned)std::max<int64_t>(c->n_leaves, 1);
    if (!c->cells_refined)
        k_gravity<true><<<grid, GBS, 0, s>>>(A);
    else
        k_gravity<false><<<grid, GBS, 0, s>>>(A);
    SPH_HIP(hipGetLastError());
    ev_record(c, EV_GRAV_K1, s);
    const int64_t* hc = read_counters(c, s);
    SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "non-positive or non-finite mass");
    if (counts) {
        counts[0] = hc[CT_FORCE_INTER];
        counts[1] = hc[CT_FORCE_CAND];
    }
    c->tm.gravity_kernel_ms = ev_ms(c, EV_GRAV_K0, EV_GRAV_K1);
}

}  // namespace sph
