// FP32 density loop with the smoothing-length solve (section 2, Eq. 1 of the
// Swift paper, and the choice of h for a fixed weighted neighbour number).
//
// Work unit: one leaf cell, handled by one wavefront. The cell's candidates
// are the particles of every cell within reach (its self task and its pair
// tasks, section 3.1); they are staged through the wavefront's LDS tile in
// chunks of 128, shifted into the cell's FP32 frame, and the next chunk is in
// flight while the current one is used.
//
// Two phases per particle of the cell (k_density):
//   A. every candidate is tested once against the particle's search radius H
//      (the radius the cells were built for) and the squared distances of the
//      hits are appended, branch-free, to a per-lane list in LDS;
//   B. Newton's method on h runs against that list only: each evaluation
//      reads one float per entry instead of re-testing every candidate. The
//      density sums of a particle depend only on its own h and the fixed
//      positions, so the whole iteration stays inside the wavefront: no
//      global sweep and no ghost pass between iterations.
// Lists hold distances only, so they serve cells whose candidates all share
// one mass (checked on the staged chunks); they are sized for the common case
// so many wavefronts fit on a CU. A particle whose list does not fit, or every
// particle of a cell with mixed masses, is left to k_density_scan: k_density
// queues such cells, and the re-scanning kernel (launched after it on the
// same stream, idle when the queue is empty) solves them over longer lists of
// distances and masses, 16 lanes per particle. A particle whose root lies
// beyond its search radius is flagged; the host rebuilds the cells around a
// larger guess and solves it again.
//
// Lanes: a cell's particles are spread over the 64 lanes, 2 to 16 lanes per
// particle; the lanes of a particle split the candidates and meet through lane
// shuffles.
#include "common.h"
#include "tiles.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace {

constexpr int BS = 64;         // one wavefront per block (finest LDS allocation)
constexpr int WAVES = BS / 64;
constexpr int DCH = 128;       // candidates per staged chunk (list kernel)
constexpr int DSLOTS = 30;     // list entries per lane, plus one spare slot that
                               // takes the stores of misses once a list is full
                               // (with a 128-candidate tile: < 10 KB of LDS per
                               // wavefront, 16 wavefronts per CU)
constexpr int DCH_U = 192;     // candidates per chunk of the persistent list kernel without
                               // culling, which streams every chunk: fewer, longer chunks per
                               // cell (batched list kernel -1.1%). At three wavefronts per SIMD
                               // the LDS allows it; the hardware-dispatch instance, at four,
                               // would lose wavefronts (Sedov +5%), and keeps DCH
constexpr int SCAP = 512;      // candidates per LDS chunk (re-scanning kernel)
static_assert(DCH % (4 * 16) == 0 && DCH_U % (8 * 4) == 0 && DCH_U % 64 == 0, "every phase-A stride divides a chunk");

struct DensArgs {
    const float4* jd;        // sorted (x, y, z) in the leaf frame, m
    const float* Hs;         // sorted search radii
    float* hs;               // sorted h: in, start value; out, result
    float* rhos;
    float* fs;
    uint8_t* st_s;           // sorted state
    const uint32_t* perm;    // sorted index -> caller index
    float* h_out;            // caller order: h (on an overflow, the larger guess
                             // the rebuild starts from)
    float* rho_out;
    float* f_out;
    float* nw_out;           // weighted neighbour count (null: not wanted)
    uint8_t* status;         // caller order
    const int4* cells;       // per schedule slot: first particle, count, first neighbour entry, and
                             // the entries within the leaf's largest search radius (a prefix of its
                             // list: the density needs no others)
    const float4* cell_pbox; // per schedule slot, 2: bounding box of the leaf's particles (centre, largest
                             // search radius; half widths, 0), at their current offsets
    const int2* p_rec;       // per (cell, neighbour cell) record: first particle and count of the neighbour
    const float4* p_shift;
    int64_t* ctr;
    int* scan_cells;         // schedule slots queued for k_density_scan (ctr[CT_SCAN_CELLS] of them)
    WorkSched W;             // which wavefront takes which cell
    float target;            // S0 = sum w(q) at the root: 3 n_ngb / 32
    float inv_target;        // 1 / target
    float tol;               // on |S0 / target - 1|
    int max_iter;
    int lpi_min;             // fewest lanes per particle (a power of two): spreads a list over enough slots
    float nl_est;            // expected list length of a particle: n_ngb * h_margin^3
    // ghost step fused into the outputs (null jf: not fused): the force
    // loop's three float4 per particle from the final h, rho, f and the
    // caller-order velocity and u
    const float* vel_in;
    const float* u_in;
    float4* jf;
    float gamma;
    const float* drift;      // [0]: bound on the drift since the build (search Hs - 2 drift)
    int detail;              // count the list-building tests and the listed candidates
                             // (sph_params.timing = 2; the list kernel's DETAIL instance)
};

// Sorted copies of position (cell frame), mass, h and state. fresh: every
// particle starts active; otherwise the caller-order state of the previous
// pass is kept (an overflowed particle starts again). The pass's fused ghost
// step reads velocity and u itself, by caller index, where it writes the
// particle's force streams: copying them here would gather them once more.
__global__ void __launch_bounds__(256) k_dens_prologue(int64_t n, const uint32_t* __restrict__ perm,
                                                       const float4* __restrict__ xrel,
                                                       const float* __restrict__ mass,
                                                       const float* __restrict__ h_in,
                                                       const uint8_t* __restrict__ status, int fresh,
                                                       float4* __restrict__ jd, float* __restrict__ hs,
                                                       uint8_t* __restrict__ st_s, int64_t* __restrict__ ctr)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (p < n) {
        const uint32_t o = perm[p];
        const float m = mass[o];
        const float h = h_in[o];
        const float4 x = xrel[p];
        jd[p] = make_float4(x.x, x.y, x.z, m);
        hs[p] = h;
        const uint8_t st = fresh ? (uint8_t)ST_ACTIVE : status[o];
        st_s[p] = st == ST_OVERFLOW ? (uint8_t)ST_ACTIVE : st;
        bad = !((m > 0.0f) && isfinite(m) && (h > 0.0f) && isfinite(h));
    }
    // one count per block instead of per-particle atomics on a shared counter
    const int n_bad = __syncthreads_count(bad);
    if (threadIdx.x == 0 && n_bad) atomicAdd((unsigned long long*)&ctr_slot(ctr)[CT_BAD_INPUT], (unsigned long long)n_bad);
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

// Newton state of one particle's h.
struct HSolve {
    float h, lo, hi, Hi;
    bool hi_known, done;
    uint8_t state;
    int nev;
};

__device__ __forceinline__ HSolve hsolve_init(float h, float Hi, bool done, uint8_t st0)
{
    HSolve s;
    s.Hi = Hi;
    s.h = (!(h > 0.0f) || h > Hi) ? Hi : h;
    s.lo = 0.0f;
    s.hi = Hi;
    s.hi_known = false;
    s.done = done;
    s.state = st0;
    s.nev = 0;
    return s;
}

// One Newton update from the sums at the current h: bracketed step on ln S0
// against ln h (exact where S0 ~ h^slope), bisection when the step leaves the
// bracket. Stops on |S0/target - 1| <= tol, on a step below FP32 resolution of
// h, on a root beyond the search radius (overflow) or after max_iter.
// Quotients use the hardware reciprocal (1 ulp): they only steer the steps,
// and the tests above are far coarser.
__device__ __forceinline__ void hsolve_step(HSolve& s, float S0, float S1, float inv_target, float tol, int max_iter)
{
    ++s.nev;
    const float ratio = S0 * inv_target;
    if (fabsf(ratio - 1.0f) <= tol) {
        s.done = true;
        s.state = ST_DONE;
        return;
    }
    if (ratio < 1.0f) {
        s.lo = s.h;
    } else {
        s.hi = s.h;
        s.hi_known = true;
    }
    if (ratio < 1.0f && s.h >= s.Hi) {
        s.done = true;
        s.state = ST_OVERFLOW;
        return;
    }
    const float slope = -S1 * __builtin_amdgcn_rcpf(S0);  // d ln S0 / d ln h
    float hn = slope > 0.05f ? s.h * __expf(-__logf(ratio) * __builtin_amdgcn_rcpf(slope)) : 2.0f * s.h;
    if (hn >= s.hi) hn = s.hi_known ? 0.5f * (s.h + s.hi) : s.Hi;
    if (hn <= s.lo) hn = 0.5f * (s.lo + s.h);
    if (fabsf(hn - s.h) <= 2.5e-7f * s.h) {
        s.done = true;  // the next step is below FP32 resolution of h: h is the root
        s.state = ST_DONE;
        return;
    }
    if (s.nev >= max_iter) {
        s.done = true;
        s.state = ST_UNCONVERGED;
        return;
    }
    s.h = hn;
}

// Outputs of one particle at its final h (sums M0 = sum m w, M1 = sum m q w'):
// sorted copies for the force loop, caller-order outputs at o = perm[i]
// (loaded with the particle, so the stores wait for nothing). SORTED_STATE
// false leaves the sorted state as it is: the re-scanning kernel's wavefronts
// that share a cell number its flagged particles from it, and nothing reads it
// after that kernel (the caller-order state carries over to the next pass).
template <bool SORTED_STATE = true, class I>
__device__ __forceinline__ void write_result(const DensArgs& A, int i, uint32_t o, const HSolve& s, float S0,
                                             float M0, float M1, int cnt, I& inter_acc, I& n_over,
                                             I& n_unconv, int& max_ev)
{
    float h_report = s.h;
    if (s.state == ST_OVERFLOW) {
        // propose the radius at which a uniform density would hold the target
        // (the rebuild starts this particle from there)
        h_report = s.h * fmaxf(cbrtf(A.target / S0), 1.0f) * 1.05f;
    }
    // (selects, not branches: a branch here makes the compiler keep the two
    // counters in a scratch array behind a pointer select)
    n_over += s.state == ST_OVERFLOW ? 1 : 0;
    n_unconv += s.state == ST_UNCONVERGED ? 1 : 0;
    const float hinv = __builtin_amdgcn_rcpf(s.h);
    const float rho = (8.0f / SPH_PI_F) * M0 * hinv * hinv * hinv;
    const float f = M1 < 0.0f ? -3.0f * M0 * __builtin_amdgcn_rcpf(M1) : 1.0f;
    A.hs[i] = s.h;
    A.rhos[i] = rho;
    A.fs[i] = f;
    if (SORTED_STATE) A.st_s[i] = s.state;
    A.h_out[o] = h_report;
    A.rho_out[o] = rho;
    A.f_out[o] = f;
    if (A.nw_out) A.nw_out[o] = (32.0f / 3.0f) * S0;
    A.status[o] = s.state;
    if (s.state == ST_DONE) inter_acc += cnt - 1;
    max_ev = max(max_ev, s.nev);
    if (A.jf) {
        // the ghost step of this particle (the same arithmetic as the force
        // loop's ghost kernel, so both give the same bits), with the checks
        // of its velocity and u: every particle of the pass passes here once
        const float4 x = A.jd[i];
        const float h = s.h;
        const float uu = A.u_in[o];
        const float vx = A.vel_in[3 * (int64_t)o], vy = A.vel_in[3 * (int64_t)o + 1],
                    vz = A.vel_in[3 * (int64_t)o + 2];
        if (!(uu >= 0.0f) || !isfinite(uu) || !isfinite(vx) || !isfinite(vy) || !isfinite(vz))
            atomicAdd((unsigned long long*)&ctr_slot(A.ctr)[CT_BAD_INPUT], 1ull);
        const float gamma = A.gamma;
        const float P = (gamma - 1.0f) * rho * uu;
        const float c = sqrtf(gamma * (gamma - 1.0f) * uu);
        const float phi = f * P / (rho * rho);
        A.jf[3 * (int64_t)i + 0] = make_float4(x.x, x.y, x.z, h * h);
        A.jf[3 * (int64_t)i + 1] = make_float4(vx, vy, vz, x.w);
        A.jf[3 * (int64_t)i + 2] = make_float4(rho, phi, c, 1.0f / h);
    }
}

__device__ __forceinline__ void flush_counters(const DensArgs& A, int64_t cand_acc, int64_t list_acc,
                                               int64_t inter_acc, int64_t sweep_acc, int64_t n_over,
                                               int64_t n_unconv, int max_ev, int64_t n_scan,
                                               int64_t listed_acc)
{
    // cand_acc and listed_acc are wavefront totals already
    ctr_add_uniform(A.ctr, CT_DENS_CAND, cand_acc);
    if (A.detail) {
        ctr_add_uniform(A.ctr, CT_DENS_TESTS, cand_acc);
        ctr_add_uniform(A.ctr, CT_DENS_LISTED, listed_acc);
    }
    ctr_wave_add(A.ctr, CT_DENS_CAND, list_acc);
    ctr_wave_add(A.ctr, CT_DENS_INTER, inter_acc);
    ctr_wave_add(A.ctr, CT_DENS_SWEEP_INTER, sweep_acc);
    ctr_wave_add(A.ctr, CT_OVERFLOW, n_over);
    ctr_wave_add(A.ctr, CT_UNCONV, n_unconv);
    ctr_wave_add(A.ctr, CT_NEED_SCAN, n_scan);
    ctr_wave_max_sweeps(A.ctr, max_ev);
}

// Flag the still-active particles [first, ni) of the cell starting at i0 for
// the re-scanning kernel; returns how many of them this lane flagged.
__device__ __forceinline__ int flag_for_scan(const DensArgs& A, int i0, int first, int ni)
{
    int n = 0;
    for (int gi = first + (int)(threadIdx.x & 63); gi < ni; gi += 64) {
        if (A.st_s[i0 + gi] == ST_ACTIVE) {
            A.st_s[i0 + gi] = ST_SCAN;
            ++n;
        }
    }
    return n;
}

// Queue schedule slot `slot` for the re-scanning kernel when any lane flagged
// a particle of its cell.
__device__ __forceinline__ void enqueue_scan(const DensArgs& A, int slot, int n_flag)
{
    if (__any(n_flag > 0) && (threadIdx.x & 63) == 0) {
        const int64_t k = (int64_t)atomicAdd((unsigned long long*)&A.ctr[CT_SCAN_CELLS], 1ull);
        A.scan_cells[k] = slot;
    }
}

// ---- the list kernel ----------------------------------------------------------------

// Phase A over one staged chunk for the lanes of one particle: the lane with
// index sub in its group tests candidates sub, sub + LPI, ... (tc points at
// candidate sub) and appends the squared distance of every hit inside H to
// its list. The chunk is padded with far positions to its full size
// (commit_chunk_padded), so there is no bounds test; U tile reads (x, y, z
// only) are in flight at once (eight where the lanes per particle are fixed
// at four: 0.7% faster; four where they vary, since eight wide groups pad
// more) and the appends are branch-free
// (the store always happens, the slot only advances on a hit). The slot is
// kept as a byte offset into the lists (o, advancing by one row of 64
// floats per hit) and clamped to the lane's spare slot (o_cap).
template <int LPI, int U = 4>
__device__ __forceinline__ void scan_chunk(const float4* tc, int len, float xx, float xy, float xz, float H2,
                                           float* lists, unsigned& o, unsigned o_cap)
{
    const int len_pad = (len + U * LPI - 1) & ~(U * LPI - 1);
    char* base = reinterpret_cast<char*>(lists);
    for (int k0 = 0; k0 < len_pad; k0 += U * LPI, tc += U * LPI) {
        float3 pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pj[u] = *reinterpret_cast<const float3*>(tc + u * LPI);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float dx = xx - pj[u].x, dy = xy - pj[u].y, dz = xz - pj[u].z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            *reinterpret_cast<float*>(base + min(o, o_cap)) = r2;
            o += r2 < H2 ? 256u : 0u;
        }
    }
}

// The first 64 neighbour records of a cell (lane q: record q), loaded with
// independent loads. A wavefront with a next cell loads them for that cell
// while it computes the current one; the particles of a cell are loaded
// together with its first chunk of candidates. So the chain cell -> records
// -> candidates costs about one memory latency per cell, not three.
struct CellRecs {
    int4 ci;      // first particle, count, first record, records
    int2 rec;     // p_rec of record `lane`
    float4 sh;    // p_shift of record `lane`
};

__device__ __forceinline__ void cell_recs(const DensArgs& A, CellRecs& P)
{
    const int lane = threadIdx.x & 63;
    const int pb0 = P.ci.z, np = P.ci.w;
    P.rec = make_int2(0, 0);
    P.sh = make_float4(0.f, 0.f, 0.f, 0.f);
    if (lane < np) {
        P.rec = A.p_rec[pb0 + lane];
        P.sh = A.p_shift[pb0 + lane];
    }
}

// One evaluation of the sums over a lane's list at 1/h = hinv. w(q) = 2 t^3 -
// 8 u^3 and q w'(q) = q (24 u^2 - 6 t^2) with t = max(1 - q, 0), u =
// max(1/2 - q, 0): the cubic spline as truncated powers, no branch and no
// select (both clamps are the FMA's clamp to [0, 1]). FIRST: the list still
// holds r^2; each entry is replaced by r as it is read.
template <bool FIRST>
__device__ __forceinline__ void eval_list(float* lst, int len, float hinv, float& S0, float& S1, int& cnt)
{
    float At = 0.f, Au = 0.f, Bt = 0.f, Bu = 0.f;
    int c = 0;
#pragma unroll 2
    for (int e = 0; e < len; ++e) {
        float r = lst[e * 64];
        if (FIRST) {
            r = __builtin_amdgcn_sqrtf(r);
            lst[e * 64] = r;
        }
        const float q = r * hinv;
        const float t = __builtin_amdgcn_fmed3f(fmaf(-r, hinv, 1.0f), 0.0f, 1.0f);
        const float u = __builtin_amdgcn_fmed3f(fmaf(-r, hinv, 0.5f), 0.0f, 1.0f);
        const float t2 = t * t, u2 = u * u;
        At = fmaf(t2, t, At);
        Au = fmaf(u2, u, Au);
        Bt = fmaf(q, t2, Bt);
        Bu = fmaf(q, u2, Bu);
        c += t > 0.0f ? 1 : 0;  // r < h
    }
    S0 = fmaf(2.0f, At, -8.0f * Au);
    S1 = fmaf(24.0f, Bu, -6.0f * Bt);
    cnt = c;
}

// One wavefront per cell. TCAP: candidates the LDS tile holds; a cell with at
// most TCAP candidates stages them once and keeps them for all its passes,
// a larger one streams them through the first DCH slots in every pass.
// PERSIST (the per-XCD queues): a wavefront takes cell after cell and loads
// the next cell's records while it computes the current one; the registers
// that takes leave three wavefronts per SIMD, which then cover the memory
// latency the prefetch does not. Hardware dispatch (one cell per wavefront)
// has no next cell: at most 128 VGPRs, four wavefronts per SIMD.
// DETAIL: also count the candidates listed (sph_params.timing = 2); a
// separate instance, since the counter costs the hot loop registers.
// CULL: the culling of staged candidates and the per-cell choice of lanes
// per particle (layouts that split a top cell, or whose lists need more
// than four lanes); without it, four lanes per particle and no culling,
// which lets the compiler specialise every loop on the lane count.
template <int TCAP, bool PERSIST, bool DETAIL, bool CULL>
__global__ void __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(PERSIST ? 3 : 4))) k_density(DensArgs A)
{
    constexpr int CH = (CULL || !PERSIST) ? DCH : DCH_U;  // candidates per streamed chunk
    __shared__ float4 tile[CULL ? TCAP : CH];  // (no resident tiles without CULL)
    __shared__ float lists[(DSLOTS + 1) * 64];
    __shared__ uint8_t marks[CH];  // record starts of the chunk being fetched
    __shared__ float4 box_lds[2];   // the cell's particle box (cull_pbox), culling cells only
    const int lane = threadIdx.x & 63;
    float4* sj = tile;
    float* lst = lists + lane;
    const unsigned o_lane = 4u * (unsigned)lane, o_cap = o_lane + 256u * DSLOTS;
    const float two_delta = 2.0f * A.drift[0];  // the cells are searched to Hs - 2 drift
    int wstate = 0, a_cur = 0, a_end = 0;
    int64_t cand_acc = 0;  // wave-uniform
    // per-lane counts (far below 2^31 for any particle count that fits a GPU)
    int inter_acc = 0, sweep_acc = 0, n_over = 0, n_unconv = 0, n_scan = 0, list_acc = 0;
    int max_ev = 0;
    int64_t listed_acc = 0;  // wave-uniform

    // the next schedule slot of this wavefront (wave-uniform), if any
    auto next_slot = [&](int& sl) -> bool {
        if (a_cur >= a_end && !next_items(A.W, A.ctr, WAVES, wstate, a_cur, a_end)) return false;
        sl = __builtin_amdgcn_readfirstlane(a_cur++);
        return true;
    };

    int slot = 0;
    bool have = next_slot(slot);
    CellRecs cur;
    if (have) {
        cur.ci = A.cells[slot];
        cell_recs(A, cur);
    }
    while (have) {
        int nslot = 0;
        const bool have_next = PERSIST && next_slot(nslot);
        CellRecs nxt;
        if (have_next) nxt.ci = A.cells[nslot];  // in flight while this cell is staged
        // (a leaf of a layout of top cells only has at most the 27 records of
        // its block, within one block of 64: telling the compiler drops the
        // multi-block paths)
        const int i0 = cur.ci.x, ni = cur.ci.y, pb0 = cur.ci.z, np_all = CULL ? cur.ci.w : min(cur.ci.w, 64);
        // the cell's first 64 particles, one per lane (in flight with the first chunk)
        float4 px = make_float4(0.f, 0.f, 0.f, 0.f);
        float ph = 0.f, pH = 0.f;
        int pst = ST_DONE;
        uint32_t pperm = 0;
        if (lane < ni) {
            px = A.jd[i0 + lane];
            ph = A.hs[i0 + lane];
            pH = A.Hs[i0 + lane] - two_delta;
            pst = A.st_s[i0 + lane];
            pperm = A.perm[i0 + lane];
        }
        int n_flag = 0;  // this lane's particles of the cell left to the re-scan
        NbrCursor cu;
        cursor_init_from(cu, nbr_from(cur.rec, cur.sh, min(np_all, 64)), pb0, np_all);
        const int nj = np_all <= 64 ? cu.nb.nj : count_candidates(A.p_rec, pb0, np_all);
        // resident: one block of neighbour records and at most TCAP candidates,
        // staged once at fixed tile slots of DCH
        // (the instance without culling always streams: with four lanes a
        // cell of up to 16 particles takes one pass, where a resident tile
        // saves nothing, and dropping that path frees registers)
        const bool resident = CULL && np_all <= 64 && nj <= TCAP;
        // a layout of top cells only runs with four lanes per particle (its
        // cells hold similar numbers of particles, for which the choice is
        // four, and the fixed count lets the compiler specialise every loop)
        const int lpi = CULL ? choose_lpi(ni, nj, A.lpi_min, 5.0f * A.nl_est, resident, CH) : 4;
        const int lg = __builtin_ctz(lpi);
        const int per_pass = 64 >> lg;
        const int g = lane >> lg;
        const int sub = lane & (lpi - 1);
        bool loaded = false;  // (resident) every candidate is in the tile
        bool mixed = false;   // a candidate with another mass was staged
        bool pre_issued = false;
        float m0 = 0.0f;      // the mass of the cell's first particle
        unsigned kept_pack = 0;  // (resident) candidates kept of each staged chunk, 8 bits each
        // neighbour cells of other sizes than the cell's own (only where a
        // top cell was split: CULL)
        const bool cull = CULL && np_all > 27;
        // the bounding box of the cell's particles at their current offsets
        // and the cell's largest search radius; the box waits in LDS for the
        // commits (held in registers across the passes it would cost the hot
        // loops)
        float geom_y = 0.0f;
        if (cull) {
            const float4 b = A.cell_pbox[2 * slot + (lane & 1)];
            if (lane < 2) box_lds[lane] = b;
            geom_y = uniform_f(__shfl(b.w, 0, 64));
        }

        for (int ib = 0; ib < ni; ib += per_pass) {
            const int gi = ib + g;
            const bool valid = gi < ni;
            const int i = i0 + (valid ? gi : 0);
            float4 xi;
            float h_start, H_i;
            int st_i;
            uint32_t o_i;
            if (ib + per_pass <= 64) {
                // the particles of this pass were loaded with the cell
                const int src = valid ? gi : 0;
                xi.x = __shfl(px.x, src, 64);
                xi.y = __shfl(px.y, src, 64);
                xi.z = __shfl(px.z, src, 64);
                h_start = __shfl(ph, src, 64);
                H_i = __shfl(pH, src, 64);
                st_i = __shfl(pst, src, 64);
                o_i = (uint32_t)__shfl((int)pperm, src, 64);
            } else {
                xi = A.jd[i];
                h_start = A.hs[i];
                H_i = A.Hs[i] - two_delta;
                st_i = A.st_s[i];
                o_i = A.perm[i];
            }
            const uint8_t st0 = (uint8_t)st_i;
            HSolve s = hsolve_init(h_start, H_i, !valid || st0 != ST_ACTIVE, st0);
            const int active_groups = wave_count(!s.done && sub == 0);
            if (active_groups == 0) continue;

            // ---- phase A: squared distances inside the search radius -----------
            unsigned o = o_lane;  // byte offset of this lane's next list slot
            {
                const float H2 = s.done ? -1.0f : s.Hi * s.Hi;
                const bool stream = !(resident && loaded);
                // staging keeps only the candidates within reach of the box of
                // the cell's particles (cell_pbox, at their current offsets):
                // the largest search radius of this pass, or of the whole cell
                // when the tile stays for later passes. A cell of a uniform
                // grid (27 neighbour cells, all as wide as the reach) loses
                // only the block's corners, which costs about what it saves,
                // so it keeps every candidate.
                const float reach2 = !cull ? 0.0f : cull_reach2(resident ? geom_y : wave_max(s.done ? 0.0f : s.Hi));
                int kept_tot = 0;
                ChunkRegs<1, CH> R;
                if (stream) {
                    cursor_seek(cu, A.p_rec, A.p_shift, 0);
                    fetch_chunk(R, A.jd, cu.nb, 0, cursor_chunk(cu, 0, CH), marks);
                }
                if (have_next && !pre_issued) {
                    // the next cell's records, in flight from here on
                    cell_recs(A, nxt);
                    pre_issued = true;
                }
                // the cell's own particles are among its candidates: when
                // every candidate has this mass, so has every particle of it
                m0 = __shfl(px.w, 0, 64);
                int len;
                for (int c0 = 0; c0 < nj; c0 += len) {
                    len = stream ? R.len : min(CH, nj - c0);
                    const float4* tc = resident ? sj + c0 : sj;
                    int slen;  // candidates of this chunk within reach
                    if (stream) {
                        mixed |= chunk_mass_differs(R, m0);
                        // store this chunk's candidates within reach (padded to
                        // DCH), put the next chunk in flight
                        if (cull) {
                            const float4 b0 = box_lds[0], b1 = box_lds[1];
                            CullBox cbox;
                            cbox.cx = b0.x;
                            cbox.cy = b0.y;
                            cbox.cz = b0.z;
                            cbox.hx = b1.x;
                            cbox.hy = b1.y;
                            cbox.hz = b1.z;
                            slen = commit_chunk_culled_padded(sj + (resident ? c0 : 0), R, cbox, reach2);
                        } else {
                            commit_chunk_padded(sj + (resident ? c0 : 0), R);
                            slen = len;
                        }
                        // (a resident tile is scanned again by later passes)
                        if (resident) kept_pack |= (unsigned)slen << (8 * (c0 / CH));
                        const int nx = c0 + len;
                        if (nx < nj) {
                            cursor_seek(cu, A.p_rec, A.p_shift, nx);
                            fetch_chunk(R, A.jd, cu.nb, nx - cu.off0, cursor_chunk(cu, nx, CH), marks);
                        }
                    } else {
                        slen = (int)((kept_pack >> (8 * (c0 / CH))) & 0xffu);
                    }
                    kept_tot += slen;
                    if (lpi == 2)
                        scan_chunk<2>(tc + sub, slen, xi.x, xi.y, xi.z, H2, lists, o, o_cap);
                    else if (lpi == 4)
                        scan_chunk<4, CULL ? 4 : 8>(tc + sub, slen, xi.x, xi.y, xi.z, H2, lists, o, o_cap);
                    else if (lpi == 8)
                        scan_chunk<8>(tc + sub, slen, xi.x, xi.y, xi.z, H2, lists, o, o_cap);
                    else
                        scan_chunk<16>(tc + sub, slen, xi.x, xi.y, xi.z, H2, lists, o, o_cap);
                    if (!resident) wave_sync_lds();
                }
                loaded = true;
                cand_acc += (int64_t)active_groups * kept_tot;
            }
            int nl = (int)((o - o_lane) >> 8);
            if (mixed) {
                // lists hold no masses: the cell's remaining particles re-scan
                // (every candidate is staged in the first pass that streams,
                // and earlier passes had no active particle)
                n_flag += flag_for_scan(A, i0, ib, ni);
                break;
            }
            // a group whose list does not fit goes to the re-scanning kernel
            const bool fits = group_sum_i(nl > DSLOTS ? 1 : 0, lpi) == 0;
            if (!s.done && !fits) {
                s.done = true;
                if (sub == 0) {
                    A.st_s[i] = ST_SCAN;
                    ++n_flag;
                }
            }
            if (s.done) nl = 0;
            wave_sync_lds();
            nl = balance_lists(lists, nl, lpi);  // phase B's trip count follows the mean, not the longest list

            // ---- phase B: Newton iteration on h over the list --------------------
            // (fS0, fS1, fcnt: the sums of this particle's last evaluation; a
            // finished particle skips its list while others still iterate; the
            // first evaluation also turns r^2 into r)
            float fS0 = 0.f, fS1 = 0.f;
            int fcnt = 0;
            bool first = true;
            while (__any(!s.done)) {
                const float hinv = __builtin_amdgcn_rcpf(s.h);
                const int len_l = s.done ? 0 : nl;
                float S0, S1;
                int cnt;
                if (first)
                    eval_list<true>(lst, len_l, hinv, S0, S1, cnt);
                else
                    eval_list<false>(lst, len_l, hinv, S0, S1, cnt);
                first = false;
                list_acc += len_l;
                S0 = group_sum(S0, lpi);
                S1 = group_sum(S1, lpi);
                cnt = group_sum_i(cnt, lpi);
                if (s.done) continue;
                if (sub == 0) sweep_acc += cnt;
                fS0 = S0;
                fS1 = S1;
                fcnt = cnt;
                hsolve_step(s, S0, S1, A.inv_target, A.tol, A.max_iter);
            }
            if constexpr (DETAIL) {
                // the candidates listed in this pass (balancing moved entries
                // between a particle's lanes but kept their number): one wave sum
                int v = nl;
                for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
                listed_acc += __builtin_amdgcn_readfirstlane(v);
            }
            if (valid && sub == 0 && st0 == ST_ACTIVE && fits)
                write_result(A, i, o_i, s, fS0, m0 * fS0, m0 * fS1, fcnt, inter_acc, n_over, n_unconv, max_ev);
        }
        if (have_next && !pre_issued) cell_recs(A, nxt);  // (no pass had an active particle)
        enqueue_scan(A, slot, n_flag);
        n_scan += n_flag;
        cur = nxt;
        slot = nslot;
        have = have_next;
    }
    flush_counters(A, cand_acc, list_acc, inter_acc, sweep_acc, n_over, n_unconv, max_ev, n_scan, listed_acc);
}

// ---- the re-scanning kernel: particles flagged ST_SCAN -------------------------------
// Persistent wavefronts take the queued cells one at a time (or, when the
// queue is short, a share of a cell's groups: see `split`); a wavefront with
// no queued cell left exits at once, so the launch costs little when nothing
// was queued. The flagged particles of a cell are compacted and taken four at
// a time, RLPI = 16 lanes each. Phase A walks the cell's candidates once and
// appends the distance and the mass of every hit inside the search radius to
// the lane's lists (room for RLPI * RSLOTS hits per particle, four times what
// the list kernel gives its widest groups); phase B runs Newton's method over
// the lists with mass-weighted sums, so mixed masses need no other path. A
// particle with still more hits re-tests every candidate at each evaluation
// (rewalk_solve).
constexpr int RLPI = 16;
constexpr int RSLOTS = 32;

// One evaluation over a lane's list (r and m at stride 64) at 1/h = hinv:
// S0 = sum w, S1 = sum q w', M0 = sum m w, M1 = sum m q w', and the entries
// inside h. The cubic spline as truncated powers, as in the list kernel:
// w = 2 t^3 - 8 u^3 and q w' = q (24 u^2 - 6 t^2).
struct ListSums {
    float S0, S1, M0, M1;
    int cnt;
};

__device__ __forceinline__ ListSums list_sums(const float* lr, const float* lm, int len, float hinv)
{
    float At = 0.f, Au = 0.f, Bt = 0.f, Bu = 0.f, mAt = 0.f, mAu = 0.f, mBt = 0.f, mBu = 0.f;
    int cnt = 0;
    for (int e = 0; e < len; ++e) {
        const float r = lr[e * 64];
        const float m = lm[e * 64];
        const float q = r * hinv;
        const float t = __builtin_amdgcn_fmed3f(fmaf(-r, hinv, 1.0f), 0.0f, 1.0f);
        const float u = __builtin_amdgcn_fmed3f(fmaf(-r, hinv, 0.5f), 0.0f, 1.0f);
        const float t2 = t * t, u2 = u * u;
        const float a = t2 * t, b = u2 * u, c = q * t2, d = q * u2;
        At += a;
        Au += b;
        Bt += c;
        Bu += d;
        mAt = fmaf(m, a, mAt);
        mAu = fmaf(m, b, mAu);
        mBt = fmaf(m, c, mBt);
        mBu = fmaf(m, d, mBu);
        cnt += t > 0.0f ? 1 : 0;
    }
    ListSums L;
    L.S0 = fmaf(2.0f, At, -8.0f * Au);
    L.S1 = fmaf(24.0f, Bu, -6.0f * Bt);
    L.M0 = fmaf(2.0f, mAt, -8.0f * mAu);
    L.M1 = fmaf(24.0f, mBu, -6.0f * mBt);
    L.cnt = cnt;
    return L;
}

// Stage the chunk of candidates starting at c0 into the tile (unless a
// single-tile cell already holds them all); returns its length.
// Candidates [c0, c0 + len) into the tile; returns len. A cell whose
// candidates fit one tile stages them once for all its groups of particles
// (kept = every candidate). Otherwise only those within reach2 of the
// group's box are kept, packed from slot 0 (kept of them): a particle of the
// group pairs with no other.
__device__ __forceinline__ int rescan_stage(const DensArgs& A, NbrCursor& cu, float4* tile, int c0, int nj,
                                            bool single_tile, bool& loaded, const CullBox& box, float reach2,
                                            int& kept)
{
    if (single_tile && loaded) {
        kept = nj;
        return nj;
    }
    cursor_seek(cu, A.p_rec, A.p_shift, c0);
    const int len = cursor_chunk(cu, c0, SCAP);
    if (single_tile) {
        stage_fast<1, SCAP>(tile, A.jd, cu.nb, c0 - cu.off0, len);
        kept = len;
    } else {
        kept = stage_fast_culled<1, SCAP>(tile, A.jd, cu.nb, c0 - cu.off0, len, box, reach2);
    }
    loaded = true;
    return len;
}

// Newton's method re-testing every candidate at each evaluation, for the
// lanes whose particle (active) has more hits than its lists hold.
template <class I>
__device__ __forceinline__ void rewalk_solve(const DensArgs& A, NbrCursor& cu, float4* tile, int nj, bool single_tile,
                                             bool& loaded, bool active, int i, float4 xi, int sub,
                                             const CullBox& box, float reach2, int64_t& cand_acc, I& inter_acc,
                                             I& sweep_acc, I& n_over, I& n_unconv, int& max_ev)
{
    HSolve s = hsolve_init(A.hs[i], A.Hs[i] - 2.0f * A.drift[0], !active, ST_ACTIVE);
    float S0 = 0.f, S1 = 0.f, M0 = 0.f, M1 = 0.f;
    int cnt = 0;
    while (__any(!s.done)) {
        const float h2 = s.h * s.h;
        const float hinv = __builtin_amdgcn_rcpf(s.h);
        S0 = S1 = M0 = M1 = 0.f;
        cnt = 0;
        const int groups_now = wave_count(!s.done && sub == 0);
        int len, kept_tot = 0;
        for (int c0 = 0; c0 < nj; c0 += len) {
            int kept;
            len = rescan_stage(A, cu, tile, c0, nj, single_tile, loaded, box, reach2, kept);
            kept_tot += kept;
            for (int k = sub; k < kept; k += RLPI) {
                const float4 pj = tile[k];
                const float dx = xi.x - pj.x, dy = xi.y - pj.y, dz = xi.z - pj.z;
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const bool in = r2 < h2;
                const float q = in ? __builtin_amdgcn_sqrtf(r2) * hinv : 1.0f;
                float w, dw;
                spline_w_dw(q, w, dw);
                const float qdw = q * dw;
                S0 += w;
                S1 += qdw;
                M0 = fmaf(pj.w, w, M0);
                M1 = fmaf(pj.w, qdw, M1);
                cnt += in ? 1 : 0;
            }
            if (!single_tile) wave_sync_lds();
        }
        cand_acc += (int64_t)groups_now * kept_tot;
        S0 = group_sum(S0, RLPI);
        S1 = group_sum(S1, RLPI);
        M0 = group_sum(M0, RLPI);
        M1 = group_sum(M1, RLPI);
        cnt = group_sum_i(cnt, RLPI);
        if (s.done) continue;
        if (sub == 0) sweep_acc += cnt;
        hsolve_step(s, S0, S1, A.inv_target, A.tol, A.max_iter);
    }
    if (active && sub == 0)
        write_result<false>(A, i, A.perm[i], s, S0, M0, M1, cnt, inter_acc, n_over, n_unconv, max_ev);
}

__global__ void __launch_bounds__(BS) k_density_scan(DensArgs A)
{
    __shared__ float4 tile[SCAP];
    __shared__ float lr_all[(RSLOTS + 1) * 64];
    __shared__ float lm_all[(RSLOTS + 1) * 64];
    __shared__ int pidx[64];
    const int lane = threadIdx.x & 63;
    const int g = lane / RLPI, sub = lane & (RLPI - 1);
    float* lr = lr_all + lane;
    float* lm = lm_all + lane;
    char* br = reinterpret_cast<char*>(lr_all);
    char* bm = reinterpret_cast<char*>(lm_all);
    const unsigned o_lane = 4u * (unsigned)lane, o_cap = o_lane + 256u * RSLOTS;
    const float two_delta = 2.0f * A.drift[0];
    int64_t cand_acc = 0;  // wave-uniform
    int list_acc = 0, inter_acc = 0, sweep_acc = 0, n_over = 0, n_unconv = 0;
    int64_t listed_acc = 0;  // wave-uniform
    int max_ev = 0;
    const int n_queued = (int)A.ctr[CT_SCAN_CELLS];  // final: written by the list kernel
    // A short queue leaves most wavefronts idle while a few take long cells
    // (a blast's hot centre: thousands of candidates, groups taken one after
    // another). Each queued cell then becomes `split` items, and item `part`
    // takes the cell's groups of flagged particles whose number is part
    // modulo split. A group's arithmetic does not depend on which wavefront
    // runs it, so the results keep their bits.
    const int n_waves = (int)gridDim.x * WAVES;
    int split = 1;
    while (split < 16 && (int64_t)n_queued * split * 2 <= n_waves) split *= 2;
    const int n_items = n_queued * split;
    if ((int)blockIdx.x * WAVES + (int)(threadIdx.x >> 6) >= n_items) return;

    for (;;) {
        int k = 0;
        if (lane == 0) k = (int)atomicAdd((unsigned long long*)&A.ctr[CT_SCAN_POP], 1ull);
        k = __shfl(k, 0, 64);
        if (k >= n_items) break;
        const int kc = k / split, part = k - kc * split;
        const int slot = A.scan_cells[kc];
        const int4 ci = A.cells[slot];
        const int i0 = ci.x, ni = ci.y, pb0 = ci.z, np_all = ci.w;
        NbrCursor cu;  // neighbour records 64 at a time
        cursor_init(cu, A.p_rec, A.p_shift, pb0, np_all);
        const int nj = np_all <= 64 ? cu.nb.nj : count_candidates(A.p_rec, pb0, np_all);
        const bool single_tile = np_all <= 64 && nj <= SCAP;
        bool loaded = false;
        int gbase = 0;  // groups in the cell's earlier blocks
        for (int b0 = 0; b0 < ni; b0 += 64) {
            // the flagged particles of these 64, compacted into pidx
            const bool flag = b0 + lane < ni && A.st_s[i0 + b0 + lane] == ST_SCAN;
            const uint64_t fm = __ballot(flag);
            const int nflag = __popcll(fm);
            wave_sync_lds();  // the previous block's reads of pidx are done
            if (flag) pidx[lanes_below(fm)] = b0 + lane;
            wave_sync_lds();
            constexpr int GP = 64 / RLPI;  // particles per group
            const int ng = (nflag + GP - 1) / GP;
            // this item's groups q of the block: gbase + q = part (mod split)
            for (int q = (part - gbase) & (split - 1); q < ng; q += split) {
                const int p0 = q * GP;
                const bool valid = p0 + g < nflag;
                const int i = i0 + pidx[valid ? p0 + g : p0];
                const float4 xi = A.jd[i];
                HSolve s = hsolve_init(A.hs[i], A.Hs[i] - two_delta, !valid, ST_ACTIVE);

                // ---- phase A: every candidate once, hits inside H listed ----------
                const float H2 = valid ? s.Hi * s.Hi : -1.0f;
                // the staged candidates any particle of this group can pair with:
                // within its largest search radius of the box around the group
                const CullBox gbox = pass_box(xi.x, xi.y, xi.z, valid);
                const float greach2 = uniform_f(cull_reach2(wave_max(valid ? s.Hi : 0.0f)));
                unsigned o = o_lane;
                int len, kept_tot = 0;
                for (int c0 = 0; c0 < nj; c0 += len) {
                    int kept;
                    len = rescan_stage(A, cu, tile, c0, nj, single_tile, loaded, gbox, greach2, kept);
                    kept_tot += kept;
                    for (int kk = sub; kk < kept; kk += RLPI) {
                        const float4 pj = tile[kk];
                        const float dx = xi.x - pj.x, dy = xi.y - pj.y, dz = xi.z - pj.z;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const unsigned oo = min(o, o_cap);
                        *reinterpret_cast<float*>(br + oo) = r2;
                        *reinterpret_cast<float*>(bm + oo) = pj.w;
                        o += r2 < H2 ? 256u : 0u;
                    }
                    if (!single_tile) wave_sync_lds();
                }
                cand_acc += (int64_t)wave_count(valid && sub == 0) * kept_tot;
                const int nl = (int)((o - o_lane) >> 8);
                const bool fits = group_sum_i(nl > RSLOTS ? 1 : 0, RLPI) == 0;
                if (A.detail) {
                    int v = valid && fits ? nl : 0;
                    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
                    listed_acc += __builtin_amdgcn_readfirstlane(v);
                }

                // ---- phase B: Newton's method over the lists ---------------------
                const bool listed = valid && fits;
                if (!listed) s.done = true;
                const int len_l = listed ? nl : 0;
                for (int e = 0; e < len_l; ++e) lr[e * 64] = __builtin_amdgcn_sqrtf(lr[e * 64]);
                float fS0 = 0.f, fM0 = 0.f, fM1 = 0.f;
                int fcnt = 0;
                while (__any(!s.done)) {
                    const float hinv = __builtin_amdgcn_rcpf(s.h);
                    const int len_e = s.done ? 0 : len_l;
                    const ListSums L = list_sums(lr, lm, len_e, hinv);
                    list_acc += len_e;
                    const float S0 = group_sum(L.S0, RLPI);
                    const float S1 = group_sum(L.S1, RLPI);
                    const float M0 = group_sum(L.M0, RLPI);
                    const float M1 = group_sum(L.M1, RLPI);
                    const int cnt = group_sum_i(L.cnt, RLPI);
                    if (s.done) continue;
                    if (sub == 0) sweep_acc += cnt;
                    fS0 = S0;
                    fM0 = M0;
                    fM1 = M1;
                    fcnt = cnt;
                    hsolve_step(s, S0, S1, A.inv_target, A.tol, A.max_iter);
                }
                if (listed && sub == 0)
                    write_result<false>(A, i, A.perm[i], s, fS0, fM0, fM1, fcnt, inter_acc, n_over, n_unconv,
                                        max_ev);

                // ---- lists too short: re-test every candidate per evaluation -------
                const bool rewalk = valid && !fits;
                if (__any(rewalk))
                    rewalk_solve(A, cu, tile, nj, single_tile, loaded, rewalk, i, xi, sub, gbox, greach2, cand_acc,
                                 inter_acc, sweep_acc, n_over, n_unconv, max_ev);
            }
            gbase += ng;
        }
    }
    flush_counters(A, cand_acc, list_acc, inter_acc, sweep_acc, n_over, n_unconv, max_ev, 0, listed_acc);
}

}  // namespace

namespace sph {

// Work schedule of a hot kernel over n_items cells and the grid to launch:
// one wavefront per cell under hardware dispatch, or a machine-sized grid of
// persistent wavefronts popping batches from the per-XCD queues.
int make_sched(sph_ctx* c, int64_t n_items, int waves_per_block, int blocks_per_cu, WorkSched& W)
{
    W.persistent = c->prm.schedule == 1 ? 1 : 0;
    W.batch = c->prm.queue_batch > 0 ? c->prm.queue_batch : 4;
    W.n_items = (int)n_items;
    for (int q = 0; q <= 8; ++q) W.q_begin[q] = (int)xcd_start(n_items, q);
    const int64_t all = (n_items + waves_per_block - 1) / waves_per_block;
    int64_t grid = all;
    if (W.persistent) grid = std::min<int64_t>(all, (int64_t)c->n_cu * blocks_per_cu);
    return (int)std::max<int64_t>(grid, 1);
}

void density_enqueue(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw, bool fresh,
                     bool events, hipStream_t s, const float* ghost_vel, const float* ghost_u)
{
    const int64_t n = c->n;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    uint8_t* status = static_cast<uint8_t*>(c->status.p);
    float4* jd = static_cast<float4*>(c->jd.p);
    float* hs = static_cast<float*>(c->hs.p);
    float* rhos = static_cast<float*>(c->rhos.p);
    float* fs = static_cast<float*>(c->fs.p);
    uint8_t* st_s = static_cast<uint8_t*>(c->st_s.p);
    const bool ghost = ghost_vel && ghost_u;
    float4* jf = ghost ? static_cast<float4*>(c->jf.p) : nullptr;
    fill_u32(ctr, 0u, 2 * (int64_t)CT_COUNT, s);  // sums, spread slots, queue heads
    k_dens_prologue<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p),
                                                        static_cast<float4*>(c->xrel.p), mass, h, status,
                                                        fresh ? 1 : 0, jd, hs, st_s, ctr);
    SPH_HIP(hipGetLastError());
    DensArgs A;
    A.jd = jd;
    A.Hs = static_cast<float*>(c->Hs.p);
    A.hs = hs;
    A.rhos = rhos;
    A.fs = fs;
    A.st_s = st_s;
    A.perm = static_cast<uint32_t*>(c->perm.p);
    A.h_out = h;
    A.rho_out = rho;
    A.f_out = f;
    A.nw_out = nw;
    A.status = status;
    A.cells = static_cast<int4*>(c->cells_d.p);
    A.cell_pbox = static_cast<float4*>(c->cell_pbox.p);
    A.p_rec = static_cast<int2*>(c->p_rec.p);
    A.p_shift = static_cast<float4*>(c->p_shift.p);
    A.ctr = ctr;
    A.target = (float)(3.0 * c->prm.n_ngb / 32.0);
    A.inv_target = (float)(32.0 / (3.0 * c->prm.n_ngb));
    A.tol = (float)c->prm.n_tol;
    A.max_iter = c->prm.max_iter;
    // a particle with a good guess finds about n_ngb * h_margin^3 candidates
    // inside its search radius; a lane takes every lpi-th candidate, so give
    // the lanes room for 70% more than their share
    const double expect = c->prm.n_ngb * c->prm.h_margin * c->prm.h_margin * c->prm.h_margin;
    A.nl_est = (float)expect;
    A.lpi_min = 2;
    while (A.lpi_min < 16 && A.lpi_min * DSLOTS < 1.7 * expect) A.lpi_min *= 2;
    A.scan_cells = static_cast<int*>(c->scan_cells.p);
    A.vel_in = ghost ? ghost_vel : nullptr;
    A.u_in = ghost ? ghost_u : nullptr;
    A.jf = jf;
    A.gamma = (float)c->prm.gamma;
    A.drift = static_cast<float*>(c->drift.p);
    A.detail = c->prm.timing == 2 ? 1 : 0;
    const int grid = make_sched(c, c->n_leaves, WAVES, 12, A.W);
    // re-scan grid: enough wavefronts for a full queue; the surplus exits at once
    const int scan_grid = (int)std::max<int64_t>(std::min<int64_t>(c->n_leaves, (int64_t)c->n_cu * 8), 1);
    if (events) ev_record(c, EV_DENS_K0, s);
    const bool pers = A.W.persistent != 0;
    auto launch = [&](auto tcap, auto cullc) {
        constexpr int T = decltype(tcap)::value;
        constexpr bool C = decltype(cullc)::value;
        if (A.detail)
            pers ? k_density<T, true, true, C><<<grid, BS, 0, s>>>(A)
                 : k_density<T, false, true, C><<<grid, BS, 0, s>>>(A);
        else
            pers ? k_density<T, true, false, C><<<grid, BS, 0, s>>>(A)
                 : k_density<T, false, false, C><<<grid, BS, 0, s>>>(A);
    };
    auto launch_t = [&](auto cullc) {
        if (c->prm.tile_cap == 512)
            launch(std::integral_constant<int, 512>{}, cullc);
        else if (c->prm.tile_cap == 256)
            launch(std::integral_constant<int, 256>{}, cullc);
        else
            launch(std::integral_constant<int, 128>{}, cullc);
    };
    // a layout of top cells only (no split) has no cell with more than 27
    // neighbour cells, so its kernels carry no culling code, and take four
    // lanes per particle where four hold the expected lists
    if (c->cells_refined || A.lpi_min > 4)
        launch_t(std::true_type{});
    else
        launch_t(std::false_type{});
    SPH_HIP(hipGetLastError());
    if (events) ev_record(c, EV_DENS_KM, s);
    k_density_scan<<<scan_grid, BS, 0, s>>>(A);
    SPH_HIP(hipGetLastError());
    if (events) ev_record(c, EV_DENS_K1, s);
}

void density_buffers(sph_ctx* c)
{
    const int64_t n = c->n;
    ensure<uint8_t>(c, c->status, n);
    ensure<float4>(c, c->jd, n);
    ensure<float>(c, c->hs, n);
    ensure<float>(c, c->rhos, n);
    ensure<float>(c, c->fs, n);
    ensure<uint8_t>(c, c->st_s, n);
    ensure<int>(c, c->scan_cells, (size_t)c->n_leaves);
}

void density_f32(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw, sph_stats* st,
                 hipStream_t s)
{
    SPH_REQUIRE(c->built, SPH_E_STATE, "sph_density before sph_build_cells");
    SPH_REQUIRE(mass && h && rho && f, SPH_E_ARG, "null mass/h/rho/f");
    check_drift(c, h, s);
    int64_t tot_inter = 0, tot_cand = 0, tot_sweep_inter = 0, tot_scan = 0, tot_tests = 0, tot_listed = 0;
    int32_t sweeps = 0;
    c->rebuilds = 0;
    c->density_done = false;
    c->vsig_valid = c->bal_valid = c->div_valid = false;  // all belong to the h this call replaces
    c->tm.density_kernel_ms = 0.0;
    c->tm.density_rescan_ms = 0.0;
    c->tm.density_launches = 0;
    ev_record(c, EV_DENS_C0, s);
    for (;;) {
        density_buffers(c);
        // the first pass starts every particle afresh; after a rebuild the
        // particles solved earlier keep their results
        density_enqueue(c, mass, h, rho, f, nw, c->rebuilds == 0, true, s);
        const int64_t* hc = read_counters(c, s);
        c->tm.density_kernel_ms += ev_ms(c, EV_DENS_K0, EV_DENS_K1);
        c->tm.density_rescan_ms += ev_ms(c, EV_DENS_KM, EV_DENS_K1);
        c->tm.density_launches += 2;
        SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "non-positive or non-finite mass or h");
        tot_scan += hc[CT_NEED_SCAN];
        tot_inter += hc[CT_DENS_INTER];
        tot_cand += hc[CT_DENS_CAND];
        tot_tests += hc[CT_DENS_TESTS];
        tot_listed += hc[CT_DENS_LISTED];
        tot_sweep_inter += hc[CT_DENS_SWEEP_INTER];
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
                st->rescanned_density = tot_scan;
                st->tests_density = tot_tests;
                st->listed_density = tot_listed;
                st->n_cells = c->n_leaves;
                st->n_pairs = c->n_pairs;
            }
            if (c->rebuilds > 0) {
                // sorted copies of every particle's final values (those solved
                // before the last rebuild were not touched by its pass)
                k_dens_regather<<<blocks_for(c->n, 256), 256, 0, s>>>(
                    c->n, static_cast<uint32_t*>(c->perm.p), h, rho, f, static_cast<float*>(c->hs.p),
                    static_cast<float*>(c->rhos.p), static_cast<float*>(c->fs.p));
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
