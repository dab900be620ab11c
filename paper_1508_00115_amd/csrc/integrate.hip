// Time integration: the pieces of a kick-drift-kick leapfrog (section 2 of the
// Swift paper: particles are marched forward in time, positions with their
// velocities and velocities with their accelerations; the leapfrog is the
// Gadget-2 scheme whose force the paper uses) and the Courant time step from
// the signal velocities the force loop records.
//
// Kick and drift stream caller-order arrays once each (HBM-bound, one pass
// over the components, fully coalesced); the time step reduces h / v_sig
// over the sorted particles with one atomic per wavefront.
#include "common.h"

#include <cmath>

namespace {

// vel_out = vel_in + acc dt over the 3n components, u_out = u_in + dudt dt
// over the first n threads; FP64 arithmetic rounded once to FP32.
__global__ void k_kick(int64_t n, double dt, const float* __restrict__ acc, const float* __restrict__ dudt,
                       const float* vel_in, const float* u_in, float* vel_out, float* u_out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * n) vel_out[t] = (float)((double)vel_in[t] + (double)acc[t] * dt);
    if (t < n) u_out[t] = (float)((double)u_in[t] + (double)dudt[t] * dt);
}

// pos += vel dt over the 3n components, wrapped into the particle's box, also
// into the library's copy pos_w; the largest |v dt| of a component goes to
// drift[1] (float bits) and a non-finite result sets drift[3]. A grid-stride
// loop over one workgroup per CU: one atomic per workgroup (same-address
// atomics serialise at the L2; one per wavefront cost 140 us on 262k
// particles). The wrap multiplies by 1/L (the two corrections absorb its
// rounding) instead of an FP64 division per component.
constexpr int DRIFT_BS = 1024;
__global__ void __launch_bounds__(DRIFT_BS) k_drift(int64_t n, double dt, const float* __restrict__ vel,
                                               double* __restrict__ pos, double* __restrict__ pos_w,
                                               const int64_t* __restrict__ box_first, int n_boxes,
                                               const double* __restrict__ box_len, unsigned* __restrict__ drift)
{
    __shared__ float wm[DRIFT_BS / 64];
    __shared__ int wbad[DRIFT_BS / 64];
    float m = 0.0f;
    bool bad = false;
    const double L0 = box_len[0], inv0 = 1.0 / L0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double L = n_boxes > 1 ? box_len[box_of(box_first, n_boxes, t / 3)] : L0;
        const double inv = n_boxes > 1 ? 1.0 / L : inv0;
        const double step = (double)vel[t] * dt;
        const double x = pos[t] + step;
        double y = x - L * floor(x * inv);
        if (y < 0.0) y += L;  // the quotient rounded up to an integer
        if (y >= L) y -= L;   // the quotient rounded down below one, or y rounded up to L
        pos[t] = y;
        pos_w[t] = y;
        const bool b = !isfinite(y);
        bad |= b;
        m = b ? m : fmaxf(m, (float)fabs(step));
    }
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    const bool any_bad = __any(bad);
    if ((threadIdx.x & 63) == 0) {
        wm[threadIdx.x >> 6] = m;
        wbad[threadIdx.x >> 6] = any_bad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nbad = 0;
        for (int q = 0; q < DRIFT_BS / 64; ++q) {
            m = fmaxf(m, wm[q]);
            nbad += wbad[q];
        }
        if (m > 0.0f) atomicMax(&drift[1], __float_as_uint(m));
        if (nbad) atomicOr(&drift[3], 1u);
    }
}

// delta += sqrt(3) * (largest component step), rounded up; the step maximum
// is cleared for the next drift.
__global__ void k_drift_close(unsigned* __restrict__ drift)
{
    if (threadIdx.x != 0) return;
    const float d = __uint_as_float(drift[0]) + 1.7320509f * __uint_as_float(drift[1]);
    drift[0] = __float_as_uint(d * 1.000001f);
    drift[1] = 0u;
}

// Smallest h / v_sig over the particles with v_sig > 0, as float bits
// (non-negative floats order like their bit patterns) into *out, which holds
// +inf beforehand.
__global__ void __launch_bounds__(256) k_dt_min(int64_t n, const float* __restrict__ hs,
                                                const float* __restrict__ vsig, unsigned* __restrict__ out)
{
    __shared__ float wm[4];
    float m = INFINITY;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const float v = vsig[p];
        if (v > 0.0f) m = fminf(m, hs[p] / v);
    }
    for (int o = 32; o >= 1; o >>= 1) m = fminf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {  // one atomic per workgroup: same-address atomics serialise at the L2
        for (int q = 1; q < 4; ++q) m = fminf(m, wm[q]);
        atomicMin(out, __float_as_uint(m));
    }
}

// The smoothing length of each particle advanced by a step dt with the
// continuity equation: rho h^3 is constant at a fixed neighbour number, so
// d ln h / dt = -(1/3) d ln rho / dt = div v / 3, integrated as
// h exp(dt div v / 3) over the step (one thread per sorted particle, the
// caller's h at o = perm[p]). Only a starting guess for the next solve.
__global__ void k_predict_h(int64_t n, double dt, const uint32_t* __restrict__ perm,
                            const float* __restrict__ divv, float* __restrict__ h)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    const double f = exp(dt * (double)divv[p] / 3.0);
    const float hp = (float)((double)h[o] * f);
    if (isfinite(hp) && hp > 0.0f) h[o] = hp;
}

}  // namespace

namespace sph {

void predict_h(sph_ctx* c, double dt, float* h, hipStream_t s)
{
    SPH_REQUIRE(h, SPH_E_ARG, "null h");
    SPH_REQUIRE(std::isfinite(dt), SPH_E_ARG, "dt must be finite");
    SPH_REQUIRE(c->built && c->div_valid, SPH_E_STATE,
                "sph_predict_h needs a force pass with sph_params.signal_velocity since the last build");
    const int64_t n = c->n;
    if (n == 0) return;
    k_predict_h<<<blocks_for(n, 256), 256, 0, s>>>(n, dt, static_cast<uint32_t*>(c->perm.p),
                                                   static_cast<float*>(c->divv_s.p), h);
    SPH_HIP(hipGetLastError());
}

void kick(sph_ctx* c, double dt, const float* acc, const float* dudt, const float* vel_in, const float* u_in,
          float* vel_out, float* u_out, hipStream_t s)
{
    SPH_REQUIRE(c->n > 0, SPH_E_STATE, "sph_kick before sph_build_cells");
    SPH_REQUIRE(acc && dudt && vel_in && u_in && vel_out && u_out, SPH_E_ARG, "null acc/dudt/vel/u");
    SPH_REQUIRE(std::isfinite(dt), SPH_E_ARG, "dt must be finite");
    const int64_t n = c->n;
    k_kick<<<blocks_for(3 * n, 256), 256, 0, s>>>(n, dt, acc, dudt, vel_in, u_in, vel_out, u_out);
    SPH_HIP(hipGetLastError());
}

void drift(sph_ctx* c, double dt, const float* vel, double* pos, hipStream_t s)
{
    SPH_REQUIRE(c->built && c->drift.p, SPH_E_STATE, "sph_drift needs cells (sph_build_cells)");
    SPH_REQUIRE(vel && pos, SPH_E_ARG, "null vel/pos");
    SPH_REQUIRE(std::isfinite(dt), SPH_E_ARG, "dt must be finite");
    const int64_t n = c->n;
    unsigned* dr = static_cast<unsigned*>(c->drift.p);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_for(3 * n, DRIFT_BS), c->n_cu));
    k_drift<<<grid, DRIFT_BS, 0, s>>>(n, dt, vel, pos, static_cast<double*>(c->pos_w.p),
                                 static_cast<int64_t*>(c->box_first.p), c->n_boxes,
                                 static_cast<double*>(c->box_len.p), dr);
    SPH_HIP(hipGetLastError());
    k_drift_close<<<1, 64, 0, s>>>(dr);
    SPH_HIP(hipGetLastError());
    // the cells stay; the offsets from their centres follow the particles
    refresh_offsets(c, s);
    c->drift_pending = true;
    c->density_done = false;
    c->density64_done = false;
    c->vsig_valid = false;
    c->bal_valid = false;
}

void check_drift(sph_ctx* c, const float* h_caller, hipStream_t s)
{
    if (!c->drift_pending) return;
    unsigned w[4];
    SPH_HIP(hipMemcpyAsync(w, c->drift.p, sizeof(w), hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    c->drift_pending = false;
    SPH_REQUIRE(w[3] == 0u, SPH_E_ARG, "a drift produced a non-finite position");
    finish_build_read(c);  // h_min
    float delta;
    std::memcpy(&delta, &w[0], 4);
    // the kernels search Hs - 2 delta: keep that above Hs / h_margin, the
    // radius the starting guesses had at the build
    const double budget = (1.0 - 1.0 / c->prm.h_margin) * (double)c->h_min;
    if (!(2.0 * (double)delta <= budget)) rebuild_cells(c, h_caller, s);
}

double timestep(sph_ctx* c, double courant, hipStream_t s)
{
    SPH_REQUIRE(std::isfinite(courant) && courant > 0.0, SPH_E_ARG, "courant must be finite and > 0");
    SPH_REQUIRE(c->built && c->vsig_valid, SPH_E_STATE,
                "sph_timestep needs a force pass with sph_params.signal_velocity since the last build or drift");
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    unsigned* slot = reinterpret_cast<unsigned*>(&ctr[CT_DT_MIN]);
    fill_u32(slot, 0x7f800000u, 1, s);  // +inf
    const int64_t n = c->n;
    const int grid = (int)std::min<int64_t>(blocks_for(n, 256), (int64_t)c->n_cu);
    k_dt_min<<<std::max(grid, 1), 256, 0, s>>>(n, static_cast<float*>(c->hs.p), static_cast<float*>(c->vsig_s.p),
                                               slot);
    SPH_HIP(hipGetLastError());
    unsigned bits = 0;
    SPH_HIP(hipMemcpyAsync(&bits, slot, 4, hipMemcpyDeviceToHost, s));
    SPH_HIP(hipStreamSynchronize(s));
    float m;
    std::memcpy(&m, &bits, 4);
    return courant * (double)m;
}

}  // namespace sph
