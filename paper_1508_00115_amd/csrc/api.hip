// C ABI of the library (declared in include/sph.h). Every entry point
// validates its arguments before touching the GPU, converts internal
// exceptions to sph_status codes and records a message for sph_last_error.
#include "common.h"

#include <chrono>
#include <cmath>
#include <new>

namespace {

thread_local std::string g_create_error;

sph_params with_defaults(const sph_params* in)
{
    sph_params p{};
    if (in) p = *in;
    if (!(p.n_ngb > 0)) p.n_ngb = 48.0;
    if (!(p.gamma > 1.0)) p.gamma = 5.0 / 3.0;
    if (p.alpha_visc == 0.0) p.alpha_visc = 0.8;
    if (p.alpha_visc < 0.0) p.alpha_visc = 0.0;
    if (!(p.n_tol > 0)) p.n_tol = 1e-6;
    if (p.max_iter <= 0) p.max_iter = 64;
    if (!(p.h_margin > 1.0)) p.h_margin = 1.26;
    if (!(p.cell_ratio > 0)) p.cell_ratio = 0.5;
    if (p.leaf_target <= 0) p.leaf_target = 64;
    if (p.workspace_limit < 0) p.workspace_limit = 0;
    if (p.schedule != 1) p.schedule = 0;
    if (p.queue_batch <= 0) p.queue_batch = 4;
    if (p.tile_cap != 256 && p.tile_cap != 512) p.tile_cap = 128;
    if (p.cell_order != 1 && p.cell_order != 2) p.cell_order = 0;
    return p;
}

template <class F>
sph_status guarded(sph_ctx* c, F&& fn)
{
    try {
        fn();
        if (c) c->err.clear();
        return SPH_OK;
    } catch (const sph::Error& e) {
        if (c) c->err = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return SPH_E_NOMEM;
    } catch (const std::exception& e) {
        if (c) c->err = e.what();
        return SPH_E_HIP;
    }
}

void set_device(sph_ctx* c) { SPH_HIP(hipSetDevice(c->device)); }

}  // namespace

extern "C" {

sph_status sph_create(const sph_params* params, int hip_device, sph_ctx** out)
{
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is null";
        return SPH_E_ARG;
    }
    *out = nullptr;
    if (params) {
        const sph_params& p = *params;
        if (!std::isfinite(p.n_ngb) || p.n_ngb < 0 || !std::isfinite(p.gamma) || !std::isfinite(p.alpha_visc) ||
            !std::isfinite(p.n_tol) || p.n_tol < 0 || !std::isfinite(p.h_margin) || p.h_margin < 0 ||
            (p.h_margin > 0 && p.h_margin <= 1.0) || !std::isfinite(p.cell_ratio) || p.cell_ratio < 0 ||
            p.max_iter < 0 || p.leaf_target < 0 || p.workspace_limit < 0 || (p.gamma != 0 && p.gamma <= 1.0) ||
            (p.tile_cap != 0 && p.tile_cap != 128 && p.tile_cap != 256 && p.tile_cap != 512)) {
            g_create_error = "invalid sph_params field";
            return SPH_E_ARG;
        }
    }
    if (hip_device < 0) {
        g_create_error = "negative device";
        return SPH_E_ARG;
    }
    sph_ctx* c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_E_NOMEM;
    c->prm = with_defaults(params);
    c->device = hip_device;
    sph_status st = guarded(c, [&] {
        int count = 0;
        SPH_HIP(hipGetDeviceCount(&count));
        SPH_REQUIRE(hip_device < count, SPH_E_ARG, "no such HIP device");
        set_device(c);
        hipDeviceProp_t prop;
        SPH_HIP(hipGetDeviceProperties(&prop, hip_device));
        c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        if (c->prm.timing)
            for (auto& e : c->ev) SPH_HIP(hipEventCreate(&e));
        sph::ensure<int64_t>(c, c->counters, CT_COUNT);
        SPH_HIP(hipHostMalloc((void**)&c->h_counters, CT_COUNT * sizeof(int64_t), hipHostMallocDefault));
        SPH_HIP(hipHostMalloc((void**)&c->h_build, sph::BUILD_OUT_WORDS * sizeof(int64_t), hipHostMallocDefault));
        SPH_HIP(hipEventCreateWithFlags(&c->ev_build, hipEventDisableTiming));
        sph::scratch_setup(hip_device);  // the static scratch of sph_timestep_noalloc on this device
    });
    if (st != SPH_OK) {
        g_create_error = c->err;
        sph_destroy(c);
        return st;
    }
    *out = c;
    return SPH_OK;
}

void sph_destroy(sph_ctx* c)
{
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    sph::Buf* all[] = {&c->box_first, &c->box_len, &c->box_G, &c->box_top_base, &c->box_hmax, &c->pos_w,
                       &c->hguess, &c->keys, &c->keys_alt, &c->perm, &c->perm_alt, &c->pos_s, &c->xrel,
                       &c->Hs, &c->leaf_of, &c->unassigned, &c->head, &c->scan1, &c->nid, &c->nd_start,
                       &c->nd_count, &c->nd_hmax, &c->nd_wide, &c->nd_child0, &c->nd_child1, &c->nd_parent, &c->nd_leaf, &c->nd_box,
                       &c->nd_level, &c->nd_coord, &c->nflag, &c->nscan, &c->top, &c->lf_start, &c->lf_count,
                       &c->lf_node, &c->lf_hmax, &c->lf_tmp, &c->p_start, &c->p_cnt, &c->p_leaf, &c->p_shift,
                       &c->p_code, &c->scan_tmp, &c->sort_hist, &c->jd, &c->hs, &c->rhos, &c->fs, &c->status,
                       &c->st_s, &c->jf, &c->vsig_s, &c->bal_s, &c->drift, &c->p_rec, &c->counters, &c->cons_d, &c->cons_part, &c->box_leaf, &c->cons64_d, &c->h64, &c->rho64, &c->f64, &c->st64,
                       &c->m64s, &c->jf64, &c->hf_tmp, &c->scan_cells, &c->cells, &c->cell_aux, &c->cell_geom, &c->cell_pbox, &c->cells_d, &c->p_cntd, &c->divv_s,
                       &c->sched_key, &c->sched_key_alt, &c->sched_val, &c->sched_val_alt, &c->build_out, &c->jg};
    for (sph::Buf* b : all) sph::free_buf(c, *b);
    for (auto& e : c->ev)
        if (e) hipEventDestroy(e);
    if (c->h_counters) hipHostFree(c->h_counters);
    if (c->h_build) hipHostFree(c->h_build);
    if (c->ev_build) hipEventDestroy(c->ev_build);
    if (c->h_cons) hipHostFree(c->h_cons);
    if (c->pass_exec) hipGraphExecDestroy(c->pass_exec);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
}

sph_status sph_build_cells(sph_ctx* c, int32_t n_boxes, const int64_t* box_first, const double* box_len,
                           int64_t n, const double* pos, const float* h_guess, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(n_boxes >= 1 && n_boxes <= 1024, SPH_E_ARG, "n_boxes must be in 1..1024");
        SPH_REQUIRE(box_first && box_len && pos && h_guess, SPH_E_ARG, "null argument");
        SPH_REQUIRE(n >= 1 && n < (int64_t(1) << 31) - 1, SPH_E_ARG, "n must be in 1 .. 2^31 - 2");
        SPH_REQUIRE(box_first[0] == 0 && box_first[n_boxes] == n, SPH_E_ARG,
                    "box_first must start at 0 and end at n");
        for (int b = 0; b < n_boxes; ++b) {
            SPH_REQUIRE(box_first[b + 1] >= box_first[b], SPH_E_ARG, "box_first must be non-decreasing");
            SPH_REQUIRE(std::isfinite(box_len[b]) && box_len[b] > 0, SPH_E_ARG, "box_len must be > 0");
        }
        set_device(c);
        const auto t0 = std::chrono::steady_clock::now();
        sph::build_cells(c, n_boxes, box_first, box_len, n, pos, h_guess, (hipStream_t)stream);
        c->tm.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
}

sph_status sph_density(sph_ctx* c, const float* mass, float* h, float* rho, float* f_gradh, float* n_weighted,
                       sph_stats* stats, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(mass && h && rho && f_gradh, SPH_E_ARG, "null argument");
        SPH_REQUIRE(c->built, SPH_E_STATE, "sph_density before sph_build_cells");
        set_device(c);
        if (stats) *stats = sph_stats{};
        sph::density_f32(c, mass, h, rho, f_gradh, n_weighted, stats, (hipStream_t)stream);
    });
}

sph_status sph_force(sph_ctx* c, const float* vel, const float* u, float* acc, float* dudt, double* cons,
                     sph_stats* stats, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(vel && u && acc && dudt, SPH_E_ARG, "null argument");
        SPH_REQUIRE(c->built && c->density_done, SPH_E_STATE, "sph_force needs a successful sph_density first");
        set_device(c);
        if (stats) *stats = sph_stats{};
        sph::force_f32(c, vel, u, acc, dudt, cons, stats, (hipStream_t)stream);
    });
}

sph_status sph_kick(sph_ctx* c, double dt, const float* acc, const float* dudt, const float* vel_in,
                    const float* u_in, float* vel_out, float* u_out, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        set_device(c);
        sph::kick(c, dt, acc, dudt, vel_in, u_in, vel_out, u_out, (hipStream_t)stream);
    });
}

sph_status sph_drift(sph_ctx* c, double dt, const float* vel, double* pos, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        set_device(c);
        sph::drift(c, dt, vel, pos, (hipStream_t)stream);
    });
}

sph_status sph_timestep(sph_ctx* c, double courant, double* dt, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(dt, SPH_E_ARG, "null dt");
        set_device(c);
        *dt = sph::timestep(c, courant, (hipStream_t)stream);
    });
}

sph_status sph_predict_h(sph_ctx* c, double dt, float* h, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        set_device(c);
        sph::predict_h(c, dt, h, (hipStream_t)stream);
    });
}

sph_status sph_timestep_noalloc(sph_ctx* c, double courant, double* dt, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(dt, SPH_E_ARG, "null dt");
        set_device(c);
        *dt = sph::timestep_noalloc(c, courant, (hipStream_t)stream);
    });
}

sph_status sph_gravity_p2p(sph_ctx* c, const float* mass, double G, double eps, double r_cut, float* acc,
                           int64_t* counts, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        set_device(c);
        sph::gravity_p2p(c, mass, G, eps, r_cut, acc, counts, (hipStream_t)stream);
    });
}

sph_status sph_get_balsara(sph_ctx* c, float* balsara, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        set_device(c);
        sph::balsara_unsort(c, balsara, (hipStream_t)stream);
    });
}

sph_status sph_pass(sph_ctx* c, const float* mass, float* h, float* rho, float* f_gradh, float* n_weighted,
                    const float* vel, const float* u, float* acc, float* dudt, double* cons, sph_stats* stats,
                    void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(mass && h && rho && f_gradh && vel && u && acc && dudt, SPH_E_ARG, "null argument");
        SPH_REQUIRE(c->built, SPH_E_STATE, "sph_pass before sph_build_cells");
        set_device(c);
        if (stats) *stats = sph_stats{};
        sph::pass_f32(c, mass, h, rho, f_gradh, n_weighted, vel, u, acc, dudt, cons, stats, (hipStream_t)stream);
    });
}

sph_status sph_density_f64(sph_ctx* c, const double* mass, double* h, double* rho, double* f_gradh,
                           double* n_weighted, sph_stats* stats, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(mass && h && rho && f_gradh, SPH_E_ARG, "null argument");
        SPH_REQUIRE(c->built, SPH_E_STATE, "sph_density_f64 before sph_build_cells");
        set_device(c);
        if (stats) *stats = sph_stats{};
        sph::density_f64(c, mass, h, rho, f_gradh, n_weighted, stats, (hipStream_t)stream);
    });
}

sph_status sph_force_f64(sph_ctx* c, const double* vel, const double* u, double* acc, double* dudt, double* cons,
                         sph_stats* stats, void* stream)
{
    if (!c) return SPH_E_ARG;
    return guarded(c, [&] {
        SPH_REQUIRE(vel && u && acc && dudt, SPH_E_ARG, "null argument");
        SPH_REQUIRE(c->built && c->density64_done, SPH_E_STATE,
                    "sph_force_f64 needs a successful sph_density_f64 first");
        set_device(c);
        if (stats) *stats = sph_stats{};
        sph::force_f64(c, vel, u, acc, dudt, cons, stats, (hipStream_t)stream);
    });
}

sph_status sph_get_timings(const sph_ctx* c, sph_timings* out)
{
    if (!c || !out) return SPH_E_ARG;
    *out = c->tm;
    return SPH_OK;
}

sph_status sph_get_build_info(const sph_ctx* c, sph_build_info* out)
{
    if (!c || !out) return SPH_E_ARG;
    if (!c->built) return SPH_E_STATE;
    sph_ctx* cm = const_cast<sph_ctx*>(c);  // the deferred read-back lands in the context
    const sph_status st = guarded(cm, [&] { sph::finish_build_read(cm); });
    if (st != SPH_OK) return st;
    *out = c->binfo;
    return SPH_OK;
}

const char* sph_status_string(sph_status s)
{
    switch (s) {
    case SPH_OK: return "ok";
    case SPH_E_ARG: return "invalid argument";
    case SPH_E_HIP: return "HIP runtime error";
    case SPH_E_NOMEM: return "out of device memory or workspace limit";
    case SPH_E_H_TOO_LARGE: return "smoothing length too large for the box";
    case SPH_E_NOT_CONVERGED: return "smoothing length did not converge";
    case SPH_E_STATE: return "call out of order";
    }
    return "unknown status";
}

const char* sph_last_error(const sph_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

const char* sph_version(void) { return "sph-mi355x 0.1 (gfx950)"; }

int32_t sph_struct_size(int32_t which)
{
    switch (which) {
        case 0: return (int32_t)sizeof(sph_params);
        case 1: return (int32_t)sizeof(sph_stats);
        case 2: return (int32_t)sizeof(sph_timings);
        case 3: return (int32_t)sizeof(sph_build_info);
        default: return -1;
    }
}

}  // extern "C"
