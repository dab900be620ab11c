// One density + force pass as a single launch sequence (section 3.1's
// dependency chain: density, ghost, force), captured once into a HIP graph
// and replayed.
//
// sph_density needs the host between kernels only to learn whether some
// smoothing length outgrew its cell (then the cells are rebuilt). The pass
// runs density and force back to back without looking, reads the counters
// once at the end and, in the rare case of an overflow, solves the density
// again with the synchronous rebuild loop and repeats the force. The ghost
// step is folded into the density kernels: a particle's force-loop streams
// are written as soon as its h is final, so there is no ghost kernel between
// the loops. The kernel sequence never changes between calls with the same
// buffers, so it is captured on a private stream and the graph is launched
// on the caller's stream; the capture is redone when any pointer or size
// changes. A capture pays only when it is replayed: the first pass on new
// cells or buffers launches the kernels directly, the second captures them.
// (A time step that rebuilds its cells every step never captures.)
#include "common.h"

namespace sph {

namespace {

void drop_graph(sph_ctx* c)
{
    if (c->pass_exec) (void)hipGraphExecDestroy(c->pass_exec);
    c->pass_exec = nullptr;
    c->pass_key.clear();
}

}  // namespace

void pass_f32(sph_ctx* c, const float* mass, float* h, float* rho, float* f, float* nw, const float* vel,
              const float* u, float* acc, float* dudt, double* cons, sph_stats* st, hipStream_t s)
{
    SPH_REQUIRE(c->built, SPH_E_STATE, "sph_pass before sph_build_cells");
    SPH_REQUIRE(mass && h && rho && f && vel && u && acc && dudt, SPH_E_ARG, "null input or output");
    check_drift(c, h, s);
    c->density_done = false;
    // the pass rewrites the sorted h, signal velocities and Balsara factors:
    // they are valid again only once it has succeeded
    c->vsig_valid = c->bal_valid = c->div_valid = false;
    c->rebuilds = 0;
    density_buffers(c);
    double* cons_d = force_buffers(c, cons != nullptr);
    if (c->prm.timing) {
        // timing mode: the same sequence launched directly, with events
        ev_record(c, EV_DENS_C0, s);
        density_enqueue(c, mass, h, rho, f, nw, true, true, s, vel, u);
        force_enqueue(c, vel, u, acc, dudt, cons_d, false, true, s, false);
        ev_record(c, EV_FORCE_C1, s);
    } else {
        const std::vector<uint64_t> key = {
            (uint64_t)c->layout_serial, (uint64_t)(uintptr_t)mass, (uint64_t)(uintptr_t)h, (uint64_t)(uintptr_t)rho,
            (uint64_t)(uintptr_t)f,     (uint64_t)(uintptr_t)nw,   (uint64_t)(uintptr_t)vel,
            (uint64_t)(uintptr_t)u,     (uint64_t)(uintptr_t)acc,  (uint64_t)(uintptr_t)dudt,
            (uint64_t)(uintptr_t)cons_d};
        if ((!c->pass_exec || c->pass_key != key) && c->pass_key_eager != key) {
            // first pass with these cells and buffers: launched directly
            density_enqueue(c, mass, h, rho, f, nw, true, false, s, vel, u);
            force_enqueue(c, vel, u, acc, dudt, cons_d, false, false, s, false);
            c->pass_key_eager = key;
        } else if (!c->pass_exec || c->pass_key != key) {
            drop_graph(c);
            if (!c->cap_stream) SPH_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            SPH_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            try {
                density_enqueue(c, mass, h, rho, f, nw, true, false, c->cap_stream, vel, u);
                force_enqueue(c, vel, u, acc, dudt, cons_d, false, false, c->cap_stream, false);
            } catch (...) {
                (void)hipStreamEndCapture(c->cap_stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            SPH_HIP(hipStreamEndCapture(c->cap_stream, &g));
            hipGraphExec_t ex = nullptr;
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            SPH_HIP(e);
            c->pass_exec = ex;
            c->pass_key = key;
            SPH_HIP(hipGraphLaunch(c->pass_exec, s));
        } else {
            SPH_HIP(hipGraphLaunch(c->pass_exec, s));
        }
    }
    // counters and conservation sums in one synchronisation (the sums are
    // discarded below if the pass has to be repeated)
    const int64_t* hc = read_counters(c, s, cons_d, cons);
    SPH_REQUIRE(hc[CT_BAD_INPUT] == 0, SPH_E_ARG, "non-positive or non-finite mass or h, negative u, or "
                                                  "non-finite velocity");
    if (hc[CT_OVERFLOW] > 0 || hc[CT_UNCONV] > 0) {
        // some h outgrew its cell (or did not converge): the synchronous
        // density loop rebuilds the cells (or reports), then the force again
        sph_stats sd{};
        density_f32(c, mass, h, rho, f, nw, &sd, s);
        force_f32(c, vel, u, acc, dudt, cons, st, s);
        if (st) {
            const int64_t fi = st->interactions_force, fc = st->candidates_force;
            *st = sd;
            st->interactions_force = fi;
            st->candidates_force = fc;
            st->n_cells = c->n_leaves;
            st->n_pairs = c->n_pairs;
        }
        return;
    }
    if (st) {
        st->sweeps = (int32_t)hc[CT_SWEEPS];
        st->rebuilds = 0;
        st->unconverged = 0;
        st->interactions_density = hc[CT_DENS_INTER];
        st->interactions_force = hc[CT_FORCE_INTER];
        st->candidates_density = hc[CT_DENS_CAND];
        st->candidates_force = hc[CT_FORCE_CAND];
        st->sweep_interactions_density = hc[CT_DENS_SWEEP_INTER];
        st->rescanned_density = hc[CT_NEED_SCAN];
        st->tests_density = hc[CT_DENS_TESTS];
        st->listed_density = hc[CT_DENS_LISTED];
        st->n_cells = c->n_leaves;
        st->n_pairs = c->n_pairs;
    }
    if (c->prm.timing) {
        c->tm.density_kernel_ms = ev_ms(c, EV_DENS_K0, EV_DENS_K1);
        c->tm.density_rescan_ms = ev_ms(c, EV_DENS_KM, EV_DENS_K1);
        c->tm.density_launches = 2;
        c->tm.force_kernel_ms = ev_ms(c, EV_FORCE_K0, EV_FORCE_K1);
        c->tm.density_call_ms = 0.0;
        c->tm.force_call_ms = 0.0;
        c->tm.pass_call_ms = ev_ms(c, EV_DENS_C0, EV_FORCE_C1);
    }
    c->density_done = true;
    mark_force_outputs(c);  // a replayed graph ran force_enqueue's kernels, not its host code
}

}  // namespace sph
