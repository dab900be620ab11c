// Plain FP64 form of the density solve and force loop, the baseline the FP32
// path is measured against: one thread per particle, walking the neighbour
// cells of its own cell on FP64 positions with explicit periodic images, FP64
// arithmetic throughout, no LDS staging and no pair symmetry. Same cells,
// same definitions (section 2 of the Swift paper, Eq. 1 and the grad-h
// Gadget-2 force) as the FP32 path.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int BS = 128;

struct D64Args {
    const double* pos_s;      // sorted FP64 positions (AoS)
    const double* m_s;        // sorted masses
    const float* Hs;          // sorted search radii
    const float* drift;       // [0]: bound on the drift since the build (search Hs - 2 drift)
    double* hs;               // sorted h: in start, out result
    double* rhos;
    double* fs;
    uint8_t* st_s;
    const int* leaf_of;
    const int* lf_start;
    const int* lf_count;
    const int* lf_node;
    const int* nd_box;
    const double* box_len;
    const uint32_t* p_start;
    const uint32_t* p_cntd;   // per leaf: its records within its largest search radius (a prefix)
    const int* p_leaf;
    const int* p_code;
    const uint32_t* perm;
    double* h_out;
    double* rho_out;
    double* f_out;
    double* nw_out;
    uint8_t* status;
    int64_t* ctr;
    int64_t n;
    double target;
    double tol;
    int max_iter;
};

__global__ void k_d64_prologue(int64_t n, const uint32_t* __restrict__ perm, const double* __restrict__ mass,
                               const double* __restrict__ h_in, const uint8_t* __restrict__ status,
                               double* __restrict__ m_s, double* __restrict__ hs, uint8_t* __restrict__ st_s,
                               int64_t* __restrict__ ctr)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    const double m = mass[o], h = h_in[o];
    m_s[p] = m;
    hs[p] = h;
    const uint8_t st = status[o];
    st_s[p] = st == ST_OVERFLOW ? (uint8_t)ST_ACTIVE : st;
    if (!(m > 0.0) || !isfinite(m) || !(h > 0.0) || !isfinite(h))
        atomicAdd((unsigned long long*)&ctr[CT_BAD_INPUT], 1ull);
}

// Counts of one particle's solve, summed per wavefront by the kernel.
struct D64Count {
    int64_t inter = 0, cand = 0, over = 0, unconv = 0, nev = 0;
};

__device__ __forceinline__ void density64_one(const D64Args& A, int64_t i, D64Count& ct)
{
    const int a = A.leaf_of[i];
    const double L = A.box_len[A.nd_box[A.lf_node[a]]];
    const double xi = A.pos_s[3 * i], yi = A.pos_s[3 * i + 1], zi = A.pos_s[3 * i + 2];
    const double Hi = (double)A.Hs[i] - 2.0 * (double)A.drift[0];
    double h = A.hs[i];
    if (!(h > 0.0) || h > Hi) h = Hi;
    double lo = 0.0, hi = Hi;
    bool hi_known = false;
    uint8_t state = ST_ACTIVE;
    int nev = 0;
    double S0, S1, M0, M1;
    int64_t cnt;
    const uint32_t q0 = A.p_start[a], q1 = q0 + A.p_cntd[a];  // the density needs only this prefix
    int64_t cand = 0;
    for (;;) {
        S0 = S1 = M0 = M1 = 0.0;
        cnt = 0;
        const double h2 = h * h;
        for (uint32_t q = q0; q < q1; ++q) {
            const int b = A.p_leaf[q];
            const int code = A.p_code[q];
            const double sx = image_shift(code, 0, L), sy = image_shift(code, 1, L), sz = image_shift(code, 2, L);
            const int j0 = A.lf_start[b], j1 = j0 + A.lf_count[b];
            cand += j1 - j0;
            for (int j = j0; j < j1; ++j) {
                const double dx = xi - (A.pos_s[3 * (int64_t)j] + sx);
                const double dy = yi - (A.pos_s[3 * (int64_t)j + 1] + sy);
                const double dz = zi - (A.pos_s[3 * (int64_t)j + 2] + sz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < h2) {
                    const double qq = sqrt(r2) / h;
                    double w, dw;
                    spline_w_dw64(qq, w, dw);
                    const double m = A.m_s[j];
                    S0 += w;
                    S1 += qq * dw;
                    M0 += m * w;
                    M1 += m * qq * dw;
                    ++cnt;
                }
            }
        }
        ++nev;
        const double ratio = S0 / A.target;
        if (fabs(ratio - 1.0) <= A.tol) { state = ST_DONE; break; }
        if (ratio < 1.0) lo = h; else { hi = h; hi_known = true; }
        if (ratio < 1.0 && h >= Hi) { state = ST_OVERFLOW; break; }
        const double slope = -S1 / S0;
        double hn = slope > 0.05 ? h * exp(-log(ratio) / slope) : 2.0 * h;
        if (hn >= hi) hn = hi_known ? 0.5 * (h + hi) : Hi;
        if (hn <= lo) hn = 0.5 * (lo + h);
        if (fabs(hn - h) <= 1e-15 * h) { state = ST_DONE; break; }
        if (nev >= A.max_iter) { state = ST_UNCONVERGED; break; }
        h = hn;
    }
    const uint32_t o = A.perm[i];
    double h_report = h;
    if (state == ST_OVERFLOW) h_report = h * fmax(cbrt(A.target / S0), 1.0) * 1.05;
    ct.over = state == ST_OVERFLOW ? 1 : 0;
    ct.unconv = state == ST_UNCONVERGED ? 1 : 0;
    ct.inter = state == ST_DONE ? cnt - 1 : 0;
    ct.cand = cand;
    ct.nev = nev;
    const double rho = 8.0 / (SPH_PI_D * h * h * h) * M0;
    const double f = M1 < 0.0 ? -3.0 * M0 / M1 : 1.0;
    A.hs[i] = h;
    A.rhos[i] = rho;
    A.fs[i] = f;
    A.st_s[i] = state;
    A.h_out[o] = h_report;
    A.rho_out[o] = rho;
    A.f_out[o] = f;
    if (A.nw_out) A.nw_out[o] = 32.0 / 3.0 * S0;
    A.status[o] = state;
}

// One thread per particle; the counts go to the counters once per wavefront.
__global__ void __launch_bounds__(BS) k_density64(D64Args A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    D64Count ct;
    if (i < A.n && A.st_s[i] == ST_ACTIVE) density64_one(A, i, ct);
    ctr_wave_add(A.ctr, CT_DENS_INTER, ct.inter);
    ctr_wave_add(A.ctr, CT_DENS_CAND, ct.cand);
    ctr_wave_add(A.ctr, CT_OVERFLOW, ct.over);
    ctr_wave_add(A.ctr, CT_UNCONV, ct.unconv);
    ctr_wave_max_sweeps(A.ctr, ct.nev);
}

__global__ void k_d64_regather(int64_t n, const uint32_t* __restrict__ perm, const double* __restrict__ h,
                               const double* __restrict__ rho, const double* __restrict__ f,
                               double* __restrict__ hs, double* __restrict__ rhos, double* __restrict__ fs)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    hs[p] = h[o];
    rhos[p] = rho[o];
    fs[p] = f[o];
}

// Per sorted particle: velocity, mass, rho, Phi, c (FP64), 8 doubles.
__global__ void k_f64_prologue(int64_t n, const uint32_t* __restrict__ perm, const double* __restrict__ m_s,
                               const double* __restrict__ rhos, const double* __restrict__ fs,
                               const double* __restrict__ vel, const double* __restrict__ u, double gamma,
                               double* __restrict__ jf, int64_t* __restrict__ ctr)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t o = perm[p];
    const double uu = u[o];
    const double vx = vel[3 * (int64_t)o], vy = vel[3 * (int64_t)o + 1], vz = vel[3 * (int64_t)o + 2];
    if (!(uu >= 0.0) || !isfinite(uu) || !isfinite(vx) || !isfinite(vy) || !isfinite(vz))
        atomicAdd((unsigned long long*)&ctr[CT_BAD_INPUT], 1ull);
    const double rho = rhos[p];
    const double P = (gamma - 1.0) * rho * uu;
    double* d = jf + 8 * p;
    d[0] = vx;
    d[1] = vy;
    d[2] = vz;
    d[3] = m_s[p];
    d[4] = rho;
    d[5] = fs[p] * P / (rho * rho);
    d[6] = sqrt(gamma * (gamma - 1.0) * uu);
    d[7] = 0.0;
}

struct F64Args {
    const double* pos_s;
    const double* jf;
    const double* hs;
    const int* leaf_of;
    const int* lf_start;
    const int* lf_count;
    const int* lf_node;
    const int* nd_box;
    const double* box_len;
    const uint32_t* p_start;
    const int* p_leaf;
    const int* p_code;
    const uint32_t* perm;
    double* acc;
    double* dudt;
    double* cons;  // CONS_SLOTS copies of 4 per box, may be null
    int64_t* ctr;
    int64_t n;
    double alpha;
    int n_boxes;
};

// Counts and conservation terms of one particle, summed per wavefront by the kernel.
struct F64Out {
    int64_t inter = 0, cand = 0;
    int box = -1;
    double cm[4] = {0.0, 0.0, 0.0, 0.0};
};

__device__ __forceinline__ void force64_one(const F64Args& A, int64_t i, F64Out& out)
{
    const int a = A.leaf_of[i];
    const int box = A.nd_box[A.lf_node[a]];
    const double L = A.box_len[box];
    const double xi = A.pos_s[3 * i], yi = A.pos_s[3 * i + 1], zi = A.pos_s[3 * i + 2];
    const double* di = A.jf + 8 * i;
    const double vxi = di[0], vyi = di[1], vzi = di[2], mi = di[3], rhoi = di[4], phii = di[5], ci = di[6];
    const double hi = A.hs[i];
    const double K = 8.0 / SPH_PI_D;
    double ax = 0, ay = 0, az = 0, du = 0;
    int64_t cnt = 0, cand = 0;
    const uint32_t q0 = A.p_start[a], q1 = A.p_start[a + 1];
    for (uint32_t q = q0; q < q1; ++q) {
        const int b = A.p_leaf[q];
        const int code = A.p_code[q];
        const double sx = image_shift(code, 0, L), sy = image_shift(code, 1, L), sz = image_shift(code, 2, L);
        const int j0 = A.lf_start[b], j1 = j0 + A.lf_count[b];
        cand += j1 - j0;
        for (int j = j0; j < j1; ++j) {
            const double dx = xi - (A.pos_s[3 * (int64_t)j] + sx);
            const double dy = yi - (A.pos_s[3 * (int64_t)j + 1] + sy);
            const double dz = zi - (A.pos_s[3 * (int64_t)j + 2] + sz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double hj = A.hs[j];
            if (!(r2 < hi * hi || r2 < hj * hj) || r2 == 0.0) continue;
            ++cnt;
            const double r = sqrt(r2);
            const double ex = dx / r, ey = dy / r, ez = dz / r;
            const double Di = r < hi ? K / (hi * hi * hi * hi) * spline_dw64(r / hi) : 0.0;
            const double Dj = r < hj ? K / (hj * hj * hj * hj) * spline_dw64(r / hj) : 0.0;
            const double* dj = A.jf + 8 * (int64_t)j;
            const double vr = (vxi - dj[0]) * ex + (vyi - dj[1]) * ey + (vzi - dj[2]) * ez;
            const double wv = vr < 0.0 ? vr : 0.0;
            const double visc = -A.alpha * (ci + dj[6] - 3.0 * wv) * wv / (rhoi + dj[4]);
            const double Dbar = 0.5 * (Di + Dj);
            const double G = phii * Di + dj[5] * Dj + visc * Dbar;
            const double mj = dj[3];
            ax -= mj * G * ex;
            ay -= mj * G * ey;
            az -= mj * G * ez;
            du += mj * (phii * Di + 0.5 * visc * Dbar) * vr;
        }
    }
    const uint32_t o = A.perm[i];
    A.acc[3 * (int64_t)o] = ax;
    A.acc[3 * (int64_t)o + 1] = ay;
    A.acc[3 * (int64_t)o + 2] = az;
    A.dudt[o] = du;
    out.inter = cnt;
    out.cand = cand;
    out.box = box;
    out.cm[0] = mi * ax;
    out.cm[1] = mi * ay;
    out.cm[2] = mi * az;
    out.cm[3] = mi * (vxi * ax + vyi * ay + vzi * az + du);
}

// One thread per particle. Counts go to the counters once per wavefront; the
// conservation terms are summed over the wavefront when all its particles
// share a box (the usual case: particles are sorted by box).
__global__ void __launch_bounds__(BS) k_force64(F64Args A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    F64Out out;
    if (i < A.n) force64_one(A, i, out);
    ctr_wave_add(A.ctr, CT_FORCE_INTER, out.inter);
    ctr_wave_add(A.ctr, CT_FORCE_CAND, out.cand);
    if (A.cons) {
        const int b0 = __shfl(out.box, 0, 64);
        if (__all(out.box < 0 || out.box == b0)) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                double v = out.cm[k];
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
                if ((threadIdx.x & 63) == 0 && b0 >= 0) atomicAdd(&cons_slot(A.cons, A.n_boxes)[4 * b0 + k], v);
            }
        } else if (out.box >= 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) atomicAdd(&cons_slot(A.cons, A.n_boxes)[4 * out.box + k], out.cm[k]);
        }
    }
}

}  // namespace

namespace sph {

void density_f64(sph_ctx* c, const double* mass, double* h, double* rho, double* f, double* nw, sph_stats* st,
                 hipStream_t s)
{
    SPH_REQUIRE(c->built, SPH_E_STATE, "sph_density_f64 before sph_build_cells");
    SPH_REQUIRE(mass && h && rho && f, SPH_E_ARG, "null mass/h/rho/f");
    check_drift(c, nullptr, s);  // a rebuild after a drift uses the guesses of the last build
    const int64_t n = c->n;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    uint8_t* status = ensure<uint8_t>(c, c->status, n);
    SPH_HIP(hipMemsetAsync(status, ST_ACTIVE, (size_t)n, s));
    int64_t tot_inter = 0, tot_cand = 0;
    int32_t sweeps = 0;
    c->rebuilds = 0;
    c->density64_done = false;
    // the FP64 form sizes its cells from the FP64 h it is given (rounded)
    for (;;) {
        double* m_s = ensure<double>(c, c->m64s, n);
        double* hs = ensure<double>(c, c->h64, n);
        double* rhos = ensure<double>(c, c->rho64, n);
        double* fs = ensure<double>(c, c->f64, n);
        uint8_t* st_s = ensure<uint8_t>(c, c->st64, n);
        SPH_HIP(hipMemsetAsync(ctr, 0, CT_COUNT * 8, s));
        k_d64_prologue<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p), mass, h, status,
                                                          m_s, hs, st_s, ctr);
        SPH_HIP(hipGetLastError());
        D64Args A;
        A.pos_s = static_cast<double*>(c->pos_s.p);
        A.m_s = m_s;
        A.Hs = static_cast<float*>(c->Hs.p);
        A.drift = static_cast<float*>(c->drift.p);
        A.hs = hs;
        A.rhos = rhos;
        A.fs = fs;
        A.st_s = st_s;
        A.leaf_of = static_cast<int*>(c->leaf_of.p);
        A.lf_start = static_cast<int*>(c->lf_start.p);
        A.lf_count = static_cast<int*>(c->lf_count.p);
        A.lf_node = static_cast<int*>(c->lf_node.p);
        A.nd_box = static_cast<int*>(c->nd_box.p);
        A.box_len = static_cast<double*>(c->box_len.p);
        A.p_start = static_cast<uint32_t*>(c->p_start.p);
        A.p_cntd = static_cast<uint32_t*>(c->p_cntd.p);
        A.p_leaf = static_cast<int*>(c->p_leaf.p);
        A.p_code = static_cast<int*>(c->p_code.p);
        A.perm = static_cast<uint32_t*>(c->perm.p);
        A.h_out = h;
        A.rho_out = rho;
        A.f_out = f;
        A.nw_out = nw;
        A.status = status;
        A.ctr = ctr;
        A.n = n;
        A.target = 3.0 * c->prm.n_ngb / 32.0;
        A.tol = 1e-13;
        A.max_iter = std::max(c->prm.max_iter, 100);
        k_density64<<<blocks_for(n, BS), BS, 0, s>>>(A);
        SPH_HIP(hipGetLastError());
        const int64_t* hc = read_counters(c, s);
        SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "non-positive or non-finite mass or h");
        tot_inter += hc[CT_DENS_INTER];
        tot_cand += hc[CT_DENS_CAND];
        sweeps = std::max<int32_t>(sweeps, (int32_t)hc[CT_SWEEPS]);
        if (hc[CT_OVERFLOW] == 0) {
            if (c->rebuilds > 0) {
                k_d64_regather<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p), h, rho, f,
                                                                  hs, rhos, fs);
                SPH_HIP(hipGetLastError());
                // masses follow the new order too
                k_d64_prologue<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p), mass, h,
                                                                  status, m_s, hs, st_s, ctr);
                SPH_HIP(hipGetLastError());
            }
            if (st) {
                st->sweeps = sweeps;
                st->rebuilds = c->rebuilds;
                st->unconverged = hc[CT_UNCONV];
                st->interactions_density = tot_inter;
                st->interactions_force = 0;
                st->candidates_density = tot_cand;
                st->candidates_force = 0;
                st->n_cells = c->n_leaves;
                st->n_pairs = c->n_pairs;
            }
            SPH_REQUIRE(hc[CT_UNCONV] == 0, SPH_E_NOT_CONVERGED,
                        std::to_string(hc[CT_UNCONV]) + " smoothing lengths did not converge");
            c->density64_done = true;
            return;
        }
        SPH_REQUIRE(c->rebuilds < 16, SPH_E_NOT_CONVERGED, "smoothing lengths keep outgrowing their cells");
        // cells around the current h, rounded up to FP32
        float* hf = ensure<float>(c, c->hf_tmp, n);
        {
            // convert caller-order FP64 h to FP32 guesses (rounded up so the
            // search radius never shrinks below the FP64 value)
            std::vector<double> hh((size_t)n);
            SPH_HIP(hipMemcpyAsync(hh.data(), h, (size_t)n * 8, hipMemcpyDeviceToHost, s));
            SPH_HIP(hipStreamSynchronize(s));
            std::vector<float> hf_h((size_t)n);
            for (int64_t k = 0; k < n; ++k) hf_h[k] = std::nextafter((float)hh[k], 3.4e38f);
            SPH_HIP(hipMemcpyAsync(hf, hf_h.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
            SPH_HIP(hipStreamSynchronize(s));
        }
        rebuild_cells(c, hf, s);
        c->rebuilds += 1;
    }
}

void force_f64(sph_ctx* c, const double* vel, const double* u, double* acc, double* dudt, double* cons,
               sph_stats* st, hipStream_t s)
{
    SPH_REQUIRE(c->built && c->density64_done, SPH_E_STATE, "sph_force_f64 needs a successful sph_density_f64");
    SPH_REQUIRE(vel && u && acc && dudt, SPH_E_ARG, "null vel/u/acc/dudt");
    SPH_REQUIRE(c->prm.balsara == 0, SPH_E_ARG, "sph_force_f64 has no Balsara switch (sph_params.balsara)");
    SPH_REQUIRE(c->prm.force_form == 0, SPH_E_ARG, "sph_force_f64 has the grad-h form only (sph_params.force_form)");
    const int64_t n = c->n;
    int64_t* ctr = static_cast<int64_t*>(c->counters.p);
    double* m_s = static_cast<double*>(c->m64s.p);
    double* jf = ensure<double>(c, c->jf64, 8 * n);
    double* cons_d = nullptr;
    if (cons) {
        cons_d = ensure<double>(c, c->cons64_d, (size_t)CONS_SLOTS * 4 * c->n_boxes);
        SPH_HIP(hipMemsetAsync(cons_d, 0, (size_t)CONS_SLOTS * 32 * c->n_boxes, s));
    }
    SPH_HIP(hipMemsetAsync(ctr, 0, CT_COUNT * 8, s));
    k_f64_prologue<<<blocks_for(n, 256), 256, 0, s>>>(n, static_cast<uint32_t*>(c->perm.p), m_s,
                                                      static_cast<double*>(c->rho64.p), static_cast<double*>(c->f64.p),
                                                      vel, u, c->prm.gamma, jf, ctr);
    SPH_HIP(hipGetLastError());
    F64Args A;
    A.pos_s = static_cast<double*>(c->pos_s.p);
    A.jf = jf;
    A.hs = static_cast<double*>(c->h64.p);
    A.leaf_of = static_cast<int*>(c->leaf_of.p);
    A.lf_start = static_cast<int*>(c->lf_start.p);
    A.lf_count = static_cast<int*>(c->lf_count.p);
    A.lf_node = static_cast<int*>(c->lf_node.p);
    A.nd_box = static_cast<int*>(c->nd_box.p);
    A.box_len = static_cast<double*>(c->box_len.p);
    A.p_start = static_cast<uint32_t*>(c->p_start.p);
    A.p_leaf = static_cast<int*>(c->p_leaf.p);
    A.p_code = static_cast<int*>(c->p_code.p);
    A.perm = static_cast<uint32_t*>(c->perm.p);
    A.acc = acc;
    A.dudt = dudt;
    A.cons = cons_d;
    A.n_boxes = c->n_boxes;
    A.ctr = ctr;
    A.n = n;
    A.alpha = c->prm.alpha_visc > 0 ? c->prm.alpha_visc : 0.0;
    k_force64<<<blocks_for(n, BS), BS, 0, s>>>(A);
    SPH_HIP(hipGetLastError());
    if (cons || st) {
        if (cons) read_cons(cons_d, cons, c->n_boxes, CONS_SLOTS, s);
        const int64_t* hc = read_counters(c, s);
        SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "negative or non-finite u, or non-finite velocity");
        if (st) {
            st->interactions_force = hc[CT_FORCE_INTER];
            st->candidates_force = hc[CT_FORCE_CAND];
            st->n_cells = c->n_leaves;
            st->n_pairs = c->n_pairs;
        }
    }
}

}  // namespace sph
