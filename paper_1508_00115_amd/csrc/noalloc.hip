// The Courant time step without any allocation: the same result as
// sph_timestep (section 2's march forward in time, the step from the signal
// velocities of the last force pass), with its reduction scratch in a
// file-scope device array instead of the context's counters, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops).
//
// The array holds DT_SLOTS per-workgroup minima and the result. Each GPU the
// library runs on has its own copy; its device address is taken once per
// device when a context is created there (hipGetSymbolAddress) and used for
// every kernel argument and copy afterwards: in host code the array's name is
// not a device address. Every call on one GPU uses that GPU's copy, so calls
// that overlap on one GPU (several streams or threads at once) race; each
// call writes every slot it reads, so nothing needs clearing.
#include "common.h"

#include <mutex>

namespace {

constexpr int DT_SLOTS = 4096;   // per-workgroup minima: at most this many workgroups
constexpr int DT_BS = 256;
constexpr int MAX_DEVICES = 64;

// DT_SLOTS partial minima, then the result at [DT_SLOTS] (16 KB in all)
static __device__ __align__(256) float scratch[DT_SLOTS + 64];

std::mutex g_mutex;
float* g_scratch[MAX_DEVICES] = {};

// Smallest h / v_sig over the particles of this workgroup's grid-stride range
// with v_sig > 0 (the arithmetic of sph_timestep's kernel), into part[block].
__global__ void __launch_bounds__(DT_BS) k_dt_partial(int64_t n, const float* __restrict__ hs,
                                                      const float* __restrict__ vsig, float* __restrict__ part)
{
    __shared__ float wm[DT_BS / 64];
    float m = INFINITY;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const float v = vsig[p];
        if (v > 0.0f) m = fminf(m, hs[p] / v);
    }
    for (int o = 32; o >= 1; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < DT_BS / 64; ++q) m = fminf(m, wm[q]);
        part[blockIdx.x] = m;
    }
}

// One workgroup: the smallest of the nb partial minima into *out.
__global__ void __launch_bounds__(DT_BS) k_dt_final(const float* __restrict__ part, int nb, float* __restrict__ out)
{
    __shared__ float wm[DT_BS / 64];
    float m = INFINITY;
    for (int b = threadIdx.x; b < nb; b += DT_BS) m = fminf(m, part[b]);
    for (int o = 32; o >= 1; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < DT_BS / 64; ++q) m = fminf(m, wm[q]);
        *out = m;
    }
}

}  // namespace

namespace sph {

void scratch_setup(int device)
{
    SPH_REQUIRE(device >= 0 && device < MAX_DEVICES, SPH_E_ARG, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_scratch[device]) return;
    void* p = nullptr;
    SPH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));  // the caller made `device` current
    SPH_REQUIRE(p != nullptr, SPH_E_HIP, "no device address for the static scratch");
    g_scratch[device] = static_cast<float*>(p);
}

double timestep_noalloc(sph_ctx* c, double courant, hipStream_t s)
{
    SPH_REQUIRE(std::isfinite(courant) && courant > 0.0, SPH_E_ARG, "courant must be finite and > 0");
    SPH_REQUIRE(c->built && c->vsig_valid, SPH_E_STATE,
                "sph_timestep_noalloc needs a force pass with sph_params.signal_velocity since the last build "
                "or drift");
    float* part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        part = c->device >= 0 && c->device < MAX_DEVICES ? g_scratch[c->device] : nullptr;
    }
    SPH_REQUIRE(part != nullptr, SPH_E_STATE, "the static scratch of this device was not set up");
    const int64_t n = c->n;
    // one partial per workgroup, at most DT_SLOTS workgroups (grid-stride beyond)
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(blocks_for(n, DT_BS), DT_SLOTS));
    k_dt_partial<<<nb, DT_BS, 0, s>>>(n, static_cast<float*>(c->hs.p), static_cast<float*>(c->vsig_s.p), part);
    SPH_HIP(hipGetLastError());
    k_dt_final<<<1, DT_BS, 0, s>>>(part, nb, part + DT_SLOTS);
    SPH_HIP(hipGetLastError());
    // into the context's pinned counter mirror (allocated at sph_create)
    float* host = reinterpret_cast<float*>(&c->h_counters[CT_DT_MIN]);
    SPH_HIP(hipMemcpyAsync(host, part + DT_SLOTS, sizeof(float), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    return courant * (double)*host;
}

}  // namespace sph
