// Internal declarations shared by the library's translation units: the
// context, device-buffer management, error plumbing and small device helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "sph.h"

namespace sph {

// ---- errors ------------------------------------------------------------------

struct Error : std::runtime_error {
    sph_status code;
    Error(sph_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SPH_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::sph::Error(SPH_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define SPH_REQUIRE(cond, code, msg)                        \
    do {                                                    \
        if (!(cond)) throw ::sph::Error((code), (msg));     \
    } while (0)

// ---- device buffers ----------------------------------------------------------

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace sph

// Per-particle state of one FP32 density solve: flags in the caller's order.
// ST_SCAN: the particle's neighbour list did not fit its LDS slots (or masses
// differ); it is solved by the re-scanning kernel instead.
enum : uint8_t { ST_ACTIVE = 0, ST_DONE = 1, ST_OVERFLOW = 2, ST_UNCONVERGED = 3, ST_SCAN = 4 };

// Device counters (int64 entries) written by the kernels.
enum {
    // sums (CT_SWEEPS: a maximum) that every wavefront adds to; the hot
    // kernels add into a spread slot (ctr_slot) and read_counters folds the
    // slots into these entries
    CT_DENS_INTER = 0,   // ordered density interactions at the final h
    CT_DENS_CAND = 1,    // candidate pairs tested by all density sweeps
    CT_FORCE_INTER = 2,  // ordered force interactions
    CT_FORCE_CAND = 3,   // candidate pairs tested by the force loop
    CT_SWEEPS = 4,       // most evaluations any particle needed (max)
    CT_OVERFLOW = 5,     // particles whose root lies beyond their search radius
    CT_UNCONV = 6,       // particles that hit max_iter
    CT_BAD_INPUT = 7,    // non-finite or non-positive inputs seen by a kernel
    CT_DENS_SWEEP_INTER = 8,  // pairs inside the trial h, summed over every evaluation
    CT_NEED_SCAN = 9,    // particles left to the re-scanning density kernel
    CT_B_CAND_PAIRS = 10,  // build: sum over leaves of particles x candidates
    CT_B_MAX_NI = 11,      // build: largest leaf (max)
    CT_B_MAX_NP = 12,      // build: longest neighbour-cell list (max)
    CT_B_MAX_NJ = 13,      // build: most candidates of a leaf (max)
    CT_B_PAIRS64 = 14,     // build: (cell, neighbour cell) records, counted in 64 bits
    CT_DENS_TESTS = 15,  // density: candidate pairs tested against the search radius (phase A)
    CT_DENS_LISTED = 16, // density: candidates listed (inside the search radius) by phase A
    CT_SUMS = 17,        // entries [0, CT_SUMS) have spread slots
    // single entries
    CT_SCAN_CELLS = 17,  // cells queued for the re-scanning density kernel
    CT_SCAN_POP = 18,    // next queued cell to take
    CT_TOTAL = 19,       // scratch for device-computed totals read by the host (two uint32)
    CT_DT_MIN = 20,      // sph_timestep: smallest h / v_sig (float bits in the low word)
    CT_QUEUE = 32,       // 8 work-queue heads (one per XCD), one 64-byte line each: CT_QUEUE + 8 q
    CT_SPREAD = 96,      // CT_SPREAD_SLOTS copies of the sums, CT_SUMS entries each
    CT_SPREAD_SLOTS = 64,
    CT_COUNT = CT_SPREAD + CT_SPREAD_SLOTS * CT_SUMS
};

// Spread slot of this workgroup's sums. Atomics on one address serialise at
// the L2 (about 10 ns each): a single counter that every wavefront of a
// launch adds to costs 0.1 to 1 ms, 64 copies on separate cache lines do not.
__device__ inline int64_t* ctr_slot(int64_t* ctr)
{
    return ctr + CT_SPREAD + (int64_t)(blockIdx.x % CT_SPREAD_SLOTS) * CT_SUMS;
}

// Add v (the same on every lane) to sum k once per wavefront.
__device__ inline void ctr_add_uniform(int64_t* ctr, int k, int64_t v)
{
    if ((threadIdx.x & 63) == 0 && v != 0) atomicAdd((unsigned long long*)&ctr_slot(ctr)[k], (unsigned long long)v);
}

// Sum v over the 64 lanes of the wavefront (all active) and add it to sum k.
__device__ inline void ctr_wave_add(int64_t* ctr, int k, int64_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    ctr_add_uniform(ctr, k, v);
}

// Per-box conservation sums of the plain FP64 form (4 doubles per box) are
// kept in CONS_SLOTS copies, picked by workgroup, for the same reason as the
// counters' spread slots. (The FP32 force loop writes one partial per cell
// and sums them per box in a second kernel instead.)
constexpr int CONS_SLOTS = 16;

__device__ inline double* cons_slot(double* cons, int n_boxes)
{
    return cons + (int64_t)(blockIdx.x % CONS_SLOTS) * 4 * n_boxes;
}

// Raise maximum k (CT_SWEEPS or a CT_B_MAX_* entry) to the largest v of the
// wavefront (all lanes active).
__device__ inline void ctr_wave_max(int64_t* ctr, int k, int64_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v = max(v, (int64_t)__shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long*)&ctr_slot(ctr)[k], (unsigned long long)v);
}

__device__ inline void ctr_wave_max_sweeps(int64_t* ctr, int64_t v) { ctr_wave_max(ctr, CT_SWEEPS, v); }

struct sph_ctx {
    sph_params prm{};
    int device = 0;
    std::string err;
    size_t allocated = 0;
    std::vector<sph::Buf*> bufs;

    // ---- build (sph_build_cells) ---------------------------------------------
    bool built = false;
    bool density_done = false;
    bool density64_done = false;
    int64_t n = 0;
    int32_t n_boxes = 0;
    std::vector<int64_t> h_box_first;
    std::vector<double> h_box_len;
    std::vector<int32_t> h_box_G;          // top-grid cells per side of each box
    std::vector<int64_t> h_box_top_base;   // offset of each box in the top-cell table
    int bits_box = 0, bits_top = 0, levels = 0;
    int64_t n_top = 0;                     // entries of the top-cell table
    int64_t n_nodes = 0, n_leaves = 0, n_pairs = 0;
    int32_t rebuilds = 0;

    sph::Buf box_first, box_len, box_G, box_top_base, box_hmax;  // per box
    sph::Buf pos_w;          // double3 AoS, wrapped, caller order
    sph::Buf hguess;         // float, caller order (copy of h_guess)
    sph::Buf keys, keys_alt, perm, perm_alt;  // sort
    sph::Buf pos_s;          // double3 AoS, sorted
    sph::Buf xrel;           // float4 (x, y, z, 0) offsets from the leaf centre, sorted
    sph::Buf Hs;             // float search radius h_margin * h_guess, sorted
    // Drift since the last build (the cells are kept across drifts), 4 words:
    // [0] float bound delta on how far any particle moved (the kernels search
    // Hs - 2 delta and widen cell boxes by delta), [1] float bits of the
    // largest |v dt| component of the current drift, [2] float bits of the
    // smallest Hs. Cleared by every build.
    sph::Buf drift;
    float h_min = 0.0f;           // smallest Hs of the last build (host copy; see finish_build_read)
    bool cells_refined = false;   // a top cell was split in the last build (leaves of several sizes)
    bool drift_pending = false;   // a drift since the last check of delta
    sph::Buf leaf_of;        // int, sorted particle -> leaf
    sph::Buf unassigned;     // int flags per particle during the level loop
    sph::Buf head, scan1;    // uint32 per particle
    sph::Buf nid;            // int per particle: node at the current level
    // nodes (all levels, level-major)
    sph::Buf build_out;
    sph::Buf nd_start, nd_count, nd_hmax, nd_wide, nd_child0, nd_child1, nd_parent, nd_leaf, nd_box, nd_level,
        nd_coord;
    int64_t node_cap = 0;
    sph::Buf nflag, nscan;   // per-node temporaries of one level
    sph::Buf top;            // int: node of each (box, top cell), -1 if empty
    // leaves (Morton order)
    sph::Buf lf_start, lf_count, lf_node, lf_hmax;
    sph::Buf lf_tmp;         // level-order leaf id per particle
    // neighbour lists
    sph::Buf p_start;        // uint32 n_leaves + 1
    sph::Buf p_cnt;          // uint32 n_leaves
    sph::Buf p_cntd;         // uint32 n_leaves: the first p_cntd[a] records of leaf a are
                             // within its largest search radius (all the density needs)
    sph::Buf p_leaf;         // int
    sph::Buf p_rec;          // int2 per record: first particle and count of the neighbour leaf
    sph::Buf p_shift;        // float4 (dx, dy, dz, 0): leaf-centre frame offset
    sph::Buf p_code;         // int: periodic image code (3 x 2 bits)
    // work schedule of the hot kernels (one slot per leaf, see xcd_start)
    sph::Buf cells;          // int4 per slot: first particle, count, first neighbour entry, neighbour entries
    sph::Buf cell_aux;       // int2 per slot: leaf index, box
    sph::Buf cell_geom;      // float2 per slot: half width of the leaf, largest search radius in it
    sph::Buf cell_pbox;      // float4 x 2 per slot: box of the leaf's particles at their current offsets
                             // (centre, largest search radius; half widths, 0)
    sph::Buf cells_d;        // int4 per slot as `cells`, with the density's record count (a prefix)
    sph::Buf sched_key, sched_key_alt, sched_val, sched_val_alt;  // cost sort
    sph::Buf scan_tmp;       // scan workspace
    sph::Buf sort_hist;      // radix-sort histograms

    // ---- density / force state (sorted order) ---------------------------------
    sph::Buf jd;             // float4 (x, y, z, m)
    sph::Buf jg;             // float4 (x, y, z, m) of the near-field gravity (its own masses)
    sph::Buf hs, rhos, fs;   // float, sorted
    sph::Buf status;         // uint8, caller order
    sph::Buf st_s;           // uint8, sorted copy of status
    sph::Buf scan_cells;     // int: leaves holding particles left to the re-scan
    sph::Buf jf;             // 3 float4 per particle for the force loop
    sph::Buf vsig_s;         // float, sorted: signal velocity of the last force pass
    bool vsig_valid = false; // vsig_s matches the current cells and h
    sph::Buf divv_s;         // float, sorted: velocity divergence of the last force pass with signal velocities
    bool div_valid = false;  // divv_s holds the last such pass of the current cells (kept across drifts)
    sph::Buf bal_s;          // float, sorted: Balsara factor of the last force pass
    bool bal_valid = false;  // bal_s matches the current cells and h
    sph::Buf counters;       // int64[CT_COUNT]
    sph::Buf cons_d;         // double, 4 per box (FP32 force loop)
    sph::Buf cons_part;      // double, 4 per leaf: each cell's share of cons_d
    sph::Buf box_leaf;       // int, n_boxes + 1: first leaf of each box (leaves follow the boxes)
    sph::Buf cons64_d;       // double, CONS_SLOTS x 4 per box (plain FP64 form)
    int64_t* h_counters = nullptr;  // pinned host mirror of counters
    // the build's shape counters and smallest search radius come back without
    // a wait of their own: folded on the device into build_out, copied into
    // this pinned buffer behind ev_build, read by finish_build_read
    int64_t* h_build = nullptr;
    hipEvent_t ev_build = nullptr;
    bool build_read_pending = false;
    double* h_cons = nullptr;       // pinned host landing buffer of the conservation sums
    size_t h_cons_cap = 0;          // doubles it holds

    // ---- FP64 plain form --------------------------------------------------------
    sph::Buf h64, rho64, f64, st64;     // sorted state of the FP64 solve
    sph::Buf m64s;                      // sorted masses of the FP64 solve
    sph::Buf jf64;                      // per particle: v, m, rho, Phi, c (8 doubles)
    sph::Buf hf_tmp;                    // FP32 guesses for a rebuild from FP64 h

    // ---- tuning and timing ------------------------------------------------------------
    int n_cu = 256;
    hipEvent_t ev[11] = {};
    sph_timings tm{};
    sph_build_info binfo{};

    // ---- the captured density + force pass (sph_pass) -----------------------------
    int64_t layout_serial = 0;           // bumped by every reallocation and every build
    hipStream_t cap_stream = nullptr;    // private stream the pass is captured on
    hipGraphExec_t pass_exec = nullptr;  // instantiated pass for pass_key
    std::vector<uint64_t> pass_key;      // pointers and sizes the captured pass was built for
    std::vector<uint64_t> pass_key_eager;  // those of the last pass launched directly
};

// Event pairs of the timing mode.
enum { EV_DENS_K0 = 0, EV_DENS_K1 = 1, EV_DENS_C0 = 2, EV_DENS_C1 = 3,
       EV_FORCE_K0 = 4, EV_FORCE_K1 = 5, EV_FORCE_C0 = 6, EV_FORCE_C1 = 7, EV_DENS_KM = 8,
       EV_GRAV_K0 = 9, EV_GRAV_K1 = 10 };

inline void ev_record(sph_ctx* c, int k, hipStream_t s)
{
    if (c->prm.timing) {
        hipError_t e = hipEventRecord(c->ev[k], s);
        if (e != hipSuccess) throw sph::Error(SPH_E_HIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
    }
}

// Milliseconds between two recorded events (waits for the second).
inline double ev_ms(sph_ctx* c, int k0, int k1)
{
    if (!c->prm.timing) return 0.0;
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(c->ev[k1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[k0], c->ev[k1]);
    if (e != hipSuccess) throw sph::Error(SPH_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
    return (double)ms;
}

namespace sph {

template <class T>
T* ensure(sph_ctx* c, Buf& b, size_t count)
{
    size_t need = count * sizeof(T);
    if (need == 0) need = sizeof(T);
    if (b.bytes >= need) return static_cast<T*>(b.p);
    if (b.p) {
        // kernels already enqueued may still read the old buffer
        SPH_HIP(hipDeviceSynchronize());
        hipFree(b.p);
        c->allocated -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = need + need / 8;  // slack for small regrowth
    if (c->prm.workspace_limit > 0 && c->allocated + want > (size_t)c->prm.workspace_limit) {
        want = need;
        if (c->allocated + want > (size_t)c->prm.workspace_limit)
            throw Error(SPH_E_NOMEM, "workspace_limit exceeded");
    }
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(SPH_E_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    b.p = p;
    b.bytes = want;
    c->allocated += want;
    ++c->layout_serial;
    return static_cast<T*>(p);
}

// Grow keeping the first `keep` elements.
template <class T>
T* grow_keep(sph_ctx* c, Buf& b, size_t count, size_t keep, hipStream_t s)
{
    size_t need = count * sizeof(T);
    if (b.bytes >= need) return static_cast<T*>(b.p);
    Buf nb;
    T* np = ensure<T>(c, nb, count + count / 2);
    if (b.p && keep) SPH_HIP(hipMemcpyAsync(np, b.p, keep * sizeof(T), hipMemcpyDeviceToDevice, s));
    SPH_HIP(hipStreamSynchronize(s));
    if (b.p) {
        hipFree(b.p);
        c->allocated -= b.bytes;
    }
    b = nb;
    return np;
}

inline void free_buf(sph_ctx* c, Buf& b)
{
    if (b.p) {
        hipFree(b.p);
        c->allocated -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// First schedule slot of XCD x when n slots are dealt out to the 8 XCDs:
// XCD x owns n / 8 slots, plus one if x < n % 8. Cells are ranked by
// decreasing cost and rank r goes to slot xcd_start(n, r % 8) + r / 8, so
// every XCD owns a cost-descending run and the runs are equally loaded. A
// hardware-dispatched workgroup b lands on XCD b % 8 and (after the remap
// of xcd_block_index) takes slot xcd_start(n, b % 8) + b / 8: rank b. The
// persistent queues use the same runs.
__host__ __device__ inline int64_t xcd_start(int64_t n, int x)
{
    return (int64_t)x * (n / 8) + (x < n % 8 ? x : n % 8);
}

// Sum the copies of the conservation sums (device, slots x 4 x n_boxes) into
// out (host, 4 x n_boxes) once the stream reaches this point.
inline void read_cons(const double* cons_d, double* out, int n_boxes, int slots, hipStream_t s)
{
    std::vector<double> h((size_t)slots * 4 * n_boxes);
    SPH_HIP(hipMemcpyAsync(h.data(), cons_d, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < 4 * n_boxes; ++k) {
        double v = 0.0;
        for (int sl = 0; sl < slots; ++sl) v += h[(size_t)sl * 4 * n_boxes + k];
        out[k] = v;
    }
}

// Pinned host room for n doubles of conservation sums (grown on demand,
// outside any capture).
inline double* cons_host(sph_ctx* c, size_t n)
{
    if (c->h_cons_cap < n) {
        if (c->h_cons) (void)hipHostFree(c->h_cons);
        c->h_cons = nullptr;
        c->h_cons_cap = 0;
        SPH_HIP(hipHostMalloc((void**)&c->h_cons, n * sizeof(double), hipHostMallocDefault));
        c->h_cons_cap = n;
    }
    return c->h_cons;
}

// Copy the device counters into the pinned mirror once the stream reaches
// this point, wait for them and fold the spread slots into the sums. With
// cons_d, the per-box conservation sums (4 per box) travel in the same
// synchronisation into the context's pinned buffer and then to cons_out.
inline const int64_t* read_counters(sph_ctx* c, hipStream_t s, const double* cons_d = nullptr,
                                    double* cons_out = nullptr)
{
    double* hc = nullptr;
    const size_t nc = (size_t)4 * c->n_boxes;
    if (cons_d && cons_out) {
        hc = cons_host(c, nc);
        SPH_HIP(hipMemcpyAsync(hc, cons_d, nc * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    SPH_HIP(hipMemcpyAsync(c->h_counters, c->counters.p, CT_COUNT * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    if (hc) std::memcpy(cons_out, hc, nc * sizeof(double));
    int64_t* h = c->h_counters;
    for (int sl = 0; sl < CT_SPREAD_SLOTS; ++sl) {
        const int64_t* p = h + CT_SPREAD + sl * CT_SUMS;
        for (int k = 0; k < CT_SUMS; ++k) {
            const bool is_max = k == CT_SWEEPS || k == CT_B_MAX_NI || k == CT_B_MAX_NP || k == CT_B_MAX_NJ;
            h[k] = is_max ? std::max(h[k], p[k]) : h[k] + p[k];
        }
    }
    return h;
}

// ---- host entry points of the other translation units ---------------------------

// Exclusive scan of n uint32 values (in may equal out). If total != nullptr the
// sum of all inputs is written there (device pointer).
void scan_exclusive(sph_ctx* c, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                    hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on bits [lo_bit, bits) of the
// keys (8-bit digits from lo_bit up). Results end in keys/vals (the alt
// buffers are scratch).
void radix_sort(sph_ctx* c, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                uint32_t* vals_alt, int64_t n, int bits, hipStream_t s, int lo_bit = 0);

// Waits for the build's deferred read-back (if any) and sets h_min and the
// build info from it.
void finish_build_read(sph_ctx* c);
constexpr int BUILD_OUT_WORDS = 5;  // candidate pairs, largest leaf, list, candidates; smallest H (bits)

void build_cells(sph_ctx* c, int32_t n_boxes, const int64_t* box_first, const double* box_len,
                 int64_t n, const double* pos, const float* h_guess, hipStream_t s);
void rebuild_cells(sph_ctx* c, const float* h_guess_caller_order /* null: the last guesses */, hipStream_t s);

// Fill n 32-bit words with v by a kernel (not a memset node, so that the
// call may be captured into a HIP graph).
void fill_u32(void* p, uint32_t v, int64_t n, hipStream_t s);

void density_f32(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw,
                 sph_stats* st, hipStream_t s);
// Near-field gravity over the pairs of the current cells (sph_gravity_p2p).
void gravity_p2p(sph_ctx* c, const float* mass, double G, double eps, double r_cut, float* acc,
                 int64_t* counts, hipStream_t s);
void force_f32(sph_ctx* c, const float* vel, const float* u, float* acc, float* dudt,
               double* cons, sph_stats* st, hipStream_t s);
// Allocate what one density pass / force pass needs (never under capture).
void density_buffers(sph_ctx* c);
double* force_buffers(sph_ctx* c, bool cons);
// Record on the host what a force pass leaves in the sorted arrays (signal
// velocities, Balsara factors). Every path that runs the force loop calls it,
// the replay of a captured pass included, which runs no host code of its own.
void mark_force_outputs(sph_ctx* c);
// Input-order Balsara factors of the last force pass into out (device, n).
void balsara_unsort(sph_ctx* c, float* out, hipStream_t s);
// Kernel launches only: no allocation, memset or host synchronisation, so
// they may run under stream capture. events: record the timing events.
// ghost (density_enqueue, with vel and u): the density kernels also write
// the force loop's particle streams, so force_enqueue(..., prologue = false)
// skips its ghost kernel.
void density_enqueue(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw, bool fresh,
                     bool events, hipStream_t s, const float* ghost_vel = nullptr, const float* ghost_u = nullptr);
void force_enqueue(sph_ctx* c, const float* vel, const float* u, float* acc, float* dudt, double* cons_d,
                   bool clear_all, bool events, hipStream_t s, bool prologue = true);
void pass_f32(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw, const float* vel,
              const float* u, float* acc, float* dudt, double* cons, sph_stats* st, hipStream_t s);
void density_f64(sph_ctx* c, const double* mass, double* h, double* rho, double* f, double* nw,
                 sph_stats* st, hipStream_t s);
// Leapfrog pieces (integrate.hip).
void kick(sph_ctx* c, double dt, const float* acc, const float* dudt, const float* vel_in, const float* u_in,
          float* vel_out, float* u_out, hipStream_t s);
void drift(sph_ctx* c, double dt, const float* vel, double* pos, hipStream_t s);
double timestep(sph_ctx* c, double courant, hipStream_t s);
// h *= exp(dt div v / 3) in caller order, from the last force pass's divergence.
void predict_h(sph_ctx* c, double dt, float* h, hipStream_t s);
// The same step with the reduction scratch in a static device array
// (noalloc.hip); scratch_setup takes that array's address on `device` (which
// must be current) once per device.
double timestep_noalloc(sph_ctx* c, double courant, hipStream_t s);
void scratch_setup(int device);
// Offsets from the leaf centres from the current positions (build.hip).
void refresh_offsets(sph_ctx* c, hipStream_t s);
// Bounding boxes of the leaves' particles at their current offsets (cell_pbox).
void cell_boxes(sph_ctx* c, hipStream_t s);
// Before a density pass after a drift: reject non-finite positions, and
// rebuild the cells (around h_caller, or the last guesses when null) once the
// drift bound eats into the margin of the search radii.
void check_drift(sph_ctx* c, const float* h_caller, hipStream_t s);
void force_f64(sph_ctx* c, const double* vel, const double* u, double* acc, double* dudt,
               double* cons, sph_stats* st, hipStream_t s);

}  // namespace sph

// ---- device helpers ----------------------------------------------------------------

// Cubic-spline shape w(q) and its derivative on 0 <= q < 1 (callers mask q >= 1).
// Both branches are evaluated and selected so a wavefront never diverges here.
__device__ __forceinline__ void spline_w_dw(float q, float& w, float& dw)
{
    const float t = 1.0f - q;
    const float w_in = fmaf(q * q, fmaf(6.0f, q, -6.0f), 1.0f);  // 1 - 6q^2 + 6q^3
    const float dw_in = q * fmaf(18.0f, q, -12.0f);              // -12q + 18q^2
    const float w_out = 2.0f * t * t * t;
    const float dw_out = -6.0f * t * t;
    const bool inner = q < 0.5f;
    w = inner ? w_in : w_out;
    dw = inner ? dw_in : dw_out;
}

// w'(q) at q = r hinv, zero from q = 1 on: 24 u^2 - 6 t^2 with t = max(1 - q, 0)
// and u = max(1/2 - q, 0), the cubic spline's derivative as truncated powers
// (no branch, no select; both clamps fold into the FMAs' clamp bit).
__device__ __forceinline__ float spline_dw_r(float r, float hinv)
{
    const float t = __builtin_amdgcn_fmed3f(fmaf(-r, hinv, 1.0f), 0.0f, 1.0f);
    const float u = __builtin_amdgcn_fmed3f(fmaf(-r, hinv, 0.5f), 0.0f, 1.0f);
    return fmaf(24.0f * u, u, -6.0f * (t * t));
}

__device__ __forceinline__ void spline_w_dw64(double q, double& w, double& dw)
{
    const double t = 1.0 - q;
    if (q < 0.5) {
        w = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
        dw = -12.0 * q + 18.0 * q * q;
    } else {
        w = 2.0 * t * t * t;
        dw = -6.0 * t * t;
    }
}

__device__ __forceinline__ double spline_dw64(double q)
{
    const double t = 1.0 - q;
    return q < 0.5 ? (-12.0 * q + 18.0 * q * q) : (-6.0 * t * t);
}

__device__ __forceinline__ int box_of(const int64_t* box_first, int n_boxes, int64_t p)
{
    int lo = 0, hi = n_boxes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (box_first[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Image code: 2 bits per axis, value 0 -> no shift, 1 -> +L, 2 -> -L.
__device__ __forceinline__ int image_code(int sx, int sy, int sz)
{
    auto e = [](int s) { return s == 0 ? 0 : (s > 0 ? 1 : 2); };
    return e(sx) | (e(sy) << 2) | (e(sz) << 4);
}
__device__ __forceinline__ double image_shift(int code, int axis, double L)
{
    int v = (code >> (2 * axis)) & 3;
    return v == 0 ? 0.0 : (v == 1 ? L : -L);
}

#define SPH_PI_F 3.14159265358979323846f
#define SPH_PI_D 3.14159265358979323846
