/*
 * sph.h -- C ABI of the MI355X (gfx950) SPH neighbour-interaction library.
 *
 * The library computes the smoothed-particle-hydrodynamics sums of the Swift
 * paper (Theuns, Chalk, Schaller & Gonnet, "Swift: task-based hydrodynamics
 * and gravity for cosmological simulations"):
 *
 *   - cell binning: particles are grouped in cubic cells no smaller than the
 *     search radius of the particles they hold, refined adaptively
 *     (section 3.1, Fig. 1); neighbouring cells are found with a tree
 *     (end of section 3.1);
 *   - the density loop: rho_i = sum_j m_j W(|r_i - r_j|, h_i) over all j
 *     including i (section 2, Eq. 1), with h_i solved so that a fixed
 *     weighted number of neighbours contributes (section 2, after Eq. 2);
 *   - after the density (the dependency of section 3.1), the symmetric
 *     pressure-gradient loop in the grad-h form of Gadget-2 that the paper
 *     says Swift implements (section 2, after Eq. 2), with a signal-velocity
 *     artificial viscosity, giving accelerations and du/dt;
 *   - marching the particles forward in time (section 2): kick-drift-kick
 *     leapfrog steps with a Courant time step, the cells kept across steps
 *     while the particles stay within their margin.
 *
 * Kernel: cubic spline with compact support h, W(r, h) = 8 / (pi h^3) w(r/h),
 *   w(q) = 1 - 6 q^2 + 6 q^3 (q <= 1/2), 2 (1 - q)^3 (1/2 < q <= 1), 0 beyond.
 * h_i: (4 pi / 3) h_i^3 sum_j W(r_ij, h_i) = n_ngb.
 * Grad-h factor: f_i = [1 + h_i / (3 rho_i) d rho_i / d h_i]^-1.
 * Equation of state: P = (gamma - 1) rho u; sound speed c = sqrt(gamma (gamma - 1) u).
 * Force, for each pair with 0 < r < max(h_i, h_j), rhat = (r_i - r_j) / r,
 *   D_k = dW/dr(r, h_k),  Phi_k = f_k P_k / rho_k^2,
 *   w_ij = min((v_i - v_j) . rhat, 0),
 *   Pi_ij = -alpha (c_i + c_j - 3 w_ij) w_ij / (rho_i + rho_j),
 *   G_ij = Phi_i D_i + Phi_j D_j + Pi_ij (D_i + D_j) / 2,
 *   a_i = -sum_j m_j G_ij rhat,
 *   du_i/dt = sum_j m_j (Phi_i D_i + Pi_ij (D_i + D_j) / 4) (v_i - v_j) . rhat.
 *
 * Conventions for every entry point
 *   - Pointers marked "device" are HIP device (or managed) memory; "host"
 *     pointers are ordinary host memory. The caller owns every buffer it
 *     passes; the library never frees or keeps caller memory beyond the call,
 *     except where stated. Device inputs must stay valid and unchanged until
 *     the work enqueued on `stream` has finished.
 *   - Per-particle arrays are in the caller's particle order. Vectors are AoS
 *     (x, y, z) per particle.
 *   - Boxes: particles [box_first[b], box_first[b+1]) live in periodic cubic
 *     box b of side box_len[b]; boxes never interact.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, 0 = null
 *     stream). Calls return after enqueueing, except where a host output
 *     (stats, cons) or an internal decision (rebuild) needs a result: those
 *     calls synchronise `stream` once.
 *   - Errors: every call returns an sph_status. On error the outputs are
 *     unspecified and sph_last_error() describes the cause. A context stays
 *     usable after any error except SPH_E_HIP.
 *   - A context is not thread-safe; use one context per stream.
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;

typedef enum {
    SPH_OK = 0,
    SPH_E_ARG = 1,            /* invalid argument (null, size, non-finite, order) */
    SPH_E_HIP = 2,            /* a HIP runtime call failed */
    SPH_E_NOMEM = 3,          /* device allocation failed or workspace_limit exceeded */
    SPH_E_H_TOO_LARGE = 4,    /* a search radius reaches L/3 of its box */
    SPH_E_NOT_CONVERGED = 5,  /* some h did not converge within max_iter */
    SPH_E_STATE = 6           /* call out of order (e.g. force before density) */
} sph_status;

/* Parameters, copied by sph_create. Zero-initialise and set what you need;
 * a zero field takes the default shown. */
typedef struct {
    double  n_ngb;        /* weighted neighbour number the h solve targets (48) */
    double  gamma;        /* adiabatic index of the ideal-gas law (5/3) */
    double  alpha_visc;   /* artificial-viscosity strength (0.8); negative = off */
    double  n_tol;        /* h solve stops when |n_i / n_ngb - 1| <= n_tol (1e-6),
                             or when the Newton step is below FP32 resolution */
    int32_t max_iter;     /* Newton iterations per particle (64) */
    double  h_margin;     /* cells are built for search radii h_margin * h_guess
                             (1.26); h may grow by this factor before a rebuild */
    double  cell_ratio;   /* a cell below the top grid is split only while at
                             most one particle in eight of it has cell_ratio *
                             search radius above half its width (0.5); the
                             few wider ones keep a longer reach, never a
                             wrong result */
    int32_t leaf_target;  /* a cell with more particles than this is split when
                             the width rule allows it (64) */
    int64_t workspace_limit; /* device bytes the context may allocate; 0 = no limit */
    int32_t timing;       /* nonzero: record HIP events around the hot kernels
                             (read with sph_get_timings; adds one stream
                             synchronisation to sph_force); 2: also count the
                             density loop's list-building tests and listed
                             candidates (sph_stats.tests_density,
                             listed_density), in a kernel instance that takes
                             a few percent longer */
    int32_t schedule;     /* how cells reach wavefronts: 0 = hardware dispatch,
                             one cell per wavefront, XCD-contiguous blocks;
                             1 = persistent wavefronts popping per-XCD queues */
    int32_t queue_batch;  /* cells per queue pop when schedule = 1 (4) */
    int32_t tile_cap;     /* candidates of a cell the density kernel keeps in LDS
                             for all its passes: 128, 256 or 512 (128); a larger
                             tile means fewer reloads but fewer wavefronts per CU */
    int32_t cell_order;   /* order cells reach wavefronts: 0 = by decreasing cost,
                             dealt out to the 8 XCDs (balance; default);
                             1 = Morton order, a contiguous range per XCD
                             (neighbouring cells share an XCD's L2);
                             2 = the Morton ranges of 1, each ordered by
                             decreasing cost (L2 locality and a short tail);
                             other values mean 0 */
    int32_t signal_velocity; /* nonzero: the force loop also records each
                             particle's signal velocity, which sph_timestep
                             needs (0: not recorded, one operation less per
                             pair) */
    int32_t balsara;      /* nonzero: Balsara switch on the viscosity. The FP32
                             force pass first sums each particle's velocity
                             divergence and curl over its neighbours inside h
                             (rho div v = sum m_j (v_j - v_i) . grad_i W(h_i),
                             rho curl v = sum m_j (v_i - v_j) x grad_i W(h_i)),
                             forms B = |div v| / (|div v| + |curl v| +
                             1e-4 c / h) (0 where the denominator is 0), and
                             scales each pair's viscosity by (B_i + B_j) / 2.
                             The Gadget-2 form of the switch; the paper has
                             no switch. Not in sph_force_f64 (SPH_E_ARG). One
                             more pass over the pairs (0: off) */
    int32_t force_form;   /* pressure terms of the FP32 force: 0 = the grad-h
                             Gadget-2 form (default); 1 = the sum the paper
                             prints as its illustration (section 2, Eq. 2):
                             a_i -= sum_j m_j (P_i / rho_i^2 + P_j / rho_j^2)
                             grad_i W(r_ij, h_i), no grad-h factor, with
                             du_i/dt += sum_j m_j P_i / rho_i^2 grad_i W(h_i)
                             . v_ij and the same viscosity. Pairs with
                             h_i <= r < h_j add only viscosity to i.
                             interactions_force still counts the pairs
                             inside max(h_i, h_j). Not with balsara, not in
                             sph_force_f64 (SPH_E_ARG) */
} sph_params;

/* Durations of the last calls, in milliseconds of GPU time measured with HIP
 * events on the caller's stream (zero unless sph_params.timing was set), and
 * the number of cell builds. */
typedef struct {
    double density_kernel_ms;  /* FP32 density kernels (list and re-scan), summed
                                  over rebuild passes */
    double density_call_ms;    /* whole sph_density: prologues, kernels, copies */
    double force_kernel_ms;    /* FP32 force kernel */
    double force_call_ms;      /* whole sph_force: ghost step, kernel, copies */
    double build_ms;           /* host wall time of the last sph_build_cells (the
                                  call returns with its last few kernels, offsets
                                  and smallest search radius, still queued) */
    int32_t density_launches;  /* density kernel launches of the last sph_density
                                  (two per pass: list kernel, re-scan kernel) */
    double density_rescan_ms;  /* the re-scan kernel's share of density_kernel_ms */
    double pass_call_ms;       /* whole sph_pass */
    int64_t builds;            /* cell builds since sph_create: sph_build_cells
                                  calls and the rebuilds the library made after
                                  a drift or for an h that outgrew its cell
                                  (counted whatever sph_params.timing) */
    double gravity_kernel_ms;  /* near-field gravity kernel of the last
                                  sph_gravity_p2p */
} sph_timings;

typedef struct {
    int32_t sweeps;             /* most Newton evaluations any particle needed */
    int32_t rebuilds;           /* cell rebuilds forced by h outgrowing its cell */
    int64_t unconverged;        /* particles whose h did not converge */
    int64_t interactions_density; /* #{(i, j), j != i : r_ij < h_i} at the final h */
    int64_t interactions_force;   /* #{(i, j), j != i : 0 < r_ij < max(h_i, h_j)}: the
                                     pairs that carry a force term (a coincident
                                     pair has no direction and adds nothing; it
                                     still counts in interactions_density) */
    int64_t candidates_density; /* (i, j) candidate pairs tested, summed over sweeps */
    int64_t candidates_force;   /* (i, j) candidate pairs tested by the force loop
                                   (candidates staged within reach of i's cell) */
    int64_t n_cells;            /* leaf cells of the current build */
    int64_t n_pairs;            /* (cell, neighbour cell) entries, self included */
    int64_t sweep_interactions_density; /* pairs inside the trial h, summed over
                                           every Newton evaluation */
    int64_t rescanned_density;  /* particles whose solve re-tested every candidate
                                   at each evaluation (unequal masses or a
                                   neighbour list too long for its slots) */
    int64_t tests_density;      /* FP32 loops: (i, j) candidate pairs tested against
                                   i's search radius outside the Newton lists (the
                                   list-building scans, and the rare re-walks of a
                                   particle whose list did not fit): the part of
                                   candidates_density that culling decides.
                                   Counted with sph_params.timing = 2 (0
                                   otherwise, and in the FP64 form) */
    int64_t listed_density;     /* FP32 loops, sph_params.timing = 2: of those,
                                   the pairs inside the search radius, kept for
                                   the Newton iteration */
} sph_stats;

/* Create a context on HIP device `hip_device`. `params` (host) may be NULL
 * for all defaults. On success *out owns device memory until sph_destroy. */
sph_status sph_create(const sph_params* params, int hip_device, sph_ctx** out);

/* Free everything the context owns. Waits for its pending work. NULL is a no-op. */
void sph_destroy(sph_ctx* ctx);

/*
 * Bin particles into cells and build the cell-pair (self and pair task)
 * lists: section 3.1 and Fig. 1 (cells at least as wide as the search radius,
 * so neighbours lie in the same or adjacent cells; the mesh refined
 * adaptively; neighbouring cells found with a tree).
 *   n_boxes    number of periodic boxes (1 .. 1024)
 *   box_first  host, n_boxes + 1 entries, box_first[0] = 0, non-decreasing,
 *              box_first[n_boxes] = n
 *   box_len    host, n_boxes side lengths (> 0)
 *   n          number of particles (>= 1)
 *   pos        device, 3n doubles (AoS), any real values (wrapped into each box)
 *   h_guess    device, n floats (> 0): starting smoothing lengths; the cells
 *              are sized for search radii h_margin * h_guess
 * The context keeps a copy of the wrapped positions; `pos` and `h_guess` may
 * be reused once the stream reaches this call's end.
 * Errors: SPH_E_ARG, SPH_E_H_TOO_LARGE (h_margin * max h_guess of a box above
 * a third of its side), SPH_E_NOMEM, SPH_E_HIP. Synchronises `stream`.
 */
sph_status sph_build_cells(sph_ctx* ctx, int32_t n_boxes, const int64_t* box_first,
                           const double* box_len, int64_t n, const double* pos,
                           const float* h_guess, void* stream);

/*
 * Density loop (section 2, Eq. 1) with the smoothing length of every particle
 * solved for n_ngb weighted neighbours (section 2), FP32 arithmetic on FP32
 * cell-relative offsets of the FP64 positions.
 *   mass        device, n floats (> 0)
 *   h           device, n floats: in, starting h (usually the h_guess given
 *               to sph_build_cells); out, converged h
 *   rho         device, n floats out: density at the converged h
 *   f_gradh     device, n floats out: grad-h factor f
 *   n_weighted  device, n floats out, may be NULL: (4 pi / 3) h^3 sum_j W
 *   stats       host, may be NULL: filled on return
 * If some h outgrows its cell the cells are rebuilt around the current h and
 * the unconverged particles are solved again (counted in stats->rebuilds).
 * Errors: SPH_E_STATE (no build), SPH_E_ARG, SPH_E_NOT_CONVERGED (outputs of
 * the converged particles are valid), SPH_E_H_TOO_LARGE, SPH_E_HIP.
 * Synchronises `stream` once.
 */
sph_status sph_density(sph_ctx* ctx, const float* mass, float* h, float* rho, float* f_gradh,
                       float* n_weighted, sph_stats* stats, void* stream);

/*
 * Force loop after the density (section 3.1: the density of a cell and its
 * neighbours precedes its pressure gradient): the ghost step computes P, c and
 * Phi from the density and u, then each pair inside max(h_i, h_j) adds the
 * pressure and viscosity terms of the Gadget-2 grad-h form (section 2, after
 * Eq. 2) to a_i and du_i/dt. FP32 arithmetic and accumulation.
 *   vel    device, 3n floats (AoS)
 *   u      device, n floats (>= 0): specific internal energy
 *   acc    device, 3n floats out
 *   dudt   device, n floats out
 *   cons   host, may be NULL: 4 doubles per box, sum_i m_i a_i (x, y, z) and
 *          sum_i m_i (v_i . a_i + du_i/dt), accumulated in FP64
 *   stats  host, may be NULL: interaction counts of this call
 * Uses the h, rho and f of the last successful sph_density on this context.
 * Errors: SPH_E_STATE, SPH_E_ARG, SPH_E_HIP. Synchronises `stream` only when
 * cons or stats is given.
 */
sph_status sph_force(sph_ctx* ctx, const float* vel, const float* u, float* acc, float* dudt,
                     double* cons, sph_stats* stats, void* stream);

/*
 * One density + force pass (section 3.1: density tasks, then the ghost, then
 * the force tasks) as a single launch sequence: the same results as
 * sph_density followed by sph_force with the same arguments, with one host
 * synchronisation instead of one per step. The sequence is captured into a
 * HIP graph on first use and replayed while the buffers (this call's pointers
 * and the context's own) stay the same; with sph_params.timing the same
 * kernels run uncaptured with HIP events around them (sph_get_timings). The
 * ghost step is done by the density kernels as each smoothing length becomes
 * final. When a smoothing length outgrows its cell, the pass falls back to
 * sph_density's rebuild loop and repeats the force.
 *   mass, h, rho, f_gradh, n_weighted: as for sph_density
 *   vel, u, acc, dudt, cons: as for sph_force
 *   stats  host, may be NULL: density and force counts of this pass
 * Errors: those of sph_density and sph_force. Synchronises `stream` once (more
 * after a rebuild).
 */
sph_status sph_pass(sph_ctx* ctx, const float* mass, float* h, float* rho, float* f_gradh,
                    float* n_weighted, const float* vel, const float* u, float* acc, float* dudt,
                    double* cons, sph_stats* stats, void* stream);

/*
 * The same density solve and force in plain FP64: one thread per particle
 * walking its cell's neighbour list on FP64 positions, no LDS staging and no
 * pair symmetry. The baseline the FP32 path is measured against; same
 * arguments and errors as the FP32 calls, FP64 arrays.
 */
sph_status sph_density_f64(sph_ctx* ctx, const double* mass, double* h, double* rho,
                           double* f_gradh, double* n_weighted, sph_stats* stats, void* stream);
sph_status sph_force_f64(sph_ctx* ctx, const double* vel, const double* u, double* acc,
                         double* dudt, double* cons, sph_stats* stats, void* stream);

/*
 * Time integration. Section 2 marches the particles forward in time from
 * their initial positions and velocities, the velocities updating the
 * positions and the accelerations the velocities. These calls give the
 * kick-drift-kick leapfrog of the Gadget-2 scheme whose force the paper
 * uses. One step of length dt, with acc and dudt holding the rates at its
 * start:
 *
 *   sph_kick(dt/2, acc, dudt, vel, u -> vel, u)        half kick
 *   sph_drift(dt, vel, pos)                            positions at t + dt
 *   sph_kick(dt/2, acc, dudt, vel, u -> vel_p, u_p)    v and u predicted to t + dt
 *   sph_pass(mass, h, ..., vel_p, u_p, acc, dudt)      rates at t + dt
 *   sph_kick(dt/2, acc, dudt, vel, u -> vel, u)        closing half kick
 *
 * and sph_timestep after the pass gives the next dt. The force sees the
 * predicted v and u: its viscosity and pressure need both at t + dt. The
 * cells are kept across drifts (below); sph_build_cells is only needed for
 * new particles or new boxes.
 */

/*
 * vel_out = vel_in + acc dt and u_out = u_in + dudt dt for the n particles of
 * the last sph_build_cells, computed in FP64 and rounded to FP32.
 *   dt               step (finite, any sign)
 *   acc, dudt        device, 3n and n floats
 *   vel_in, u_in     device, 3n and n floats
 *   vel_out, u_out   device, 3n and n floats out; may be vel_in and u_in
 * Errors: SPH_E_ARG (null pointer, non-finite dt), SPH_E_STATE (no build yet),
 * SPH_E_HIP. Does not synchronise.
 */
sph_status sph_kick(sph_ctx* ctx, double dt, const float* acc, const float* dudt, const float* vel_in,
                    const float* u_in, float* vel_out, float* u_out, void* stream);

/*
 * pos += vel dt in FP64, each particle wrapped into its periodic box (the
 * boxes of the last sph_build_cells). The cells are kept. The library bounds
 * the distance every particle has moved since the cells were built by delta,
 * the sum over drifts of sqrt(3) max |v dt|. Its offsets from the cell
 * centres follow the particle, the density searches h_margin * h_guess -
 * 2 delta instead of h_margin * h_guess, and the force widens each cell box
 * by delta. Every pair within reach is still found. The next sph_density or
 * sph_pass rebuilds the cells first once 2 delta exceeds
 * (1 - 1/h_margin) times the smallest search radius, or when an h outgrows
 * the reduced radius. After a drift, sph_force and sph_timestep need a
 * density pass first.
 *   dt    step (finite, any sign)
 *   vel   device, 3n floats
 *   pos   device, 3n doubles, in and out
 * Errors: SPH_E_ARG (a non-finite position is reported by the next density
 * pass), SPH_E_STATE (no cells yet), SPH_E_HIP. Does not synchronise.
 */
sph_status sph_drift(sph_ctx* ctx, double dt, const float* vel, double* pos, void* stream);

/*
 * Courant time step from the last force pass: *dt = courant * min_i h_i /
 * v_sig,i, where v_sig,i = max(c_i, max_j (c_i + c_j - 3 w_ij)) over the
 * pairs of i in the force loop (the signal velocity of its viscosity term);
 * +inf when every v_sig is 0. Needs sph_params.signal_velocity.
 *   courant  > 0 (0.1 to 0.4 is usual)
 *   dt       host, out
 * Errors: SPH_E_ARG, SPH_E_STATE (no force pass with signal velocities since
 * the last build or drift), SPH_E_HIP. Synchronises `stream`.
 */
sph_status sph_timestep(sph_ctx* ctx, double courant, double* dt, void* stream);

/*
 * Starting smoothing lengths for the next density solve, advanced over a step
 * dt by the continuity equation (the density of a particle changes at the
 * rate -rho div v; at a fixed neighbour number rho h^3 is constant, so
 * d ln h / dt = div v / 3): h_i *= exp(dt (div v)_i / 3), with the velocity
 * divergence rho_i (div v)_i = -sum_j m_j (v_i - v_j) . grad_i W(r_ij, h_i)
 * that the last force pass with sph_params.signal_velocity recorded (over
 * the pairs inside h_i). Called after sph_drift in a leapfrog step, it saves
 * Newton sweeps; the solve's result does not depend on it (the root is
 * unique).
 *   dt  the step (finite, any sign)
 *   h   device, n floats, caller order: in, the last smoothing lengths; out,
 *       the predicted ones (a non-finite or non-positive prediction leaves h)
 * Errors: SPH_E_ARG, SPH_E_STATE (no force pass with signal velocities since
 * the last build), SPH_E_HIP. Does not synchronise.
 */
sph_status sph_predict_h(sph_ctx* ctx, double dt, float* h, void* stream);

/*
 * sph_timestep without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid it). Same arguments, result and errors as sph_timestep (bit for bit
 * the same dt). Its reduction scratch is a static device array of 16 KB per
 * GPU (4096 per-workgroup minima and the result), whose address the library
 * takes when a context is created on that GPU; any particle count fits (the
 * workgroups stride over the particles). All calls on one GPU share that
 * array: calls that overlap on one GPU (other streams or host threads at the
 * same time) race and must be serialised by the caller. Synchronises
 * `stream`.
 */
sph_status sph_timestep_noalloc(sph_ctx* ctx, double courant, double* dt, void* stream);

/*
 * Near-field gravity, particle-particle (the paper's section 2, Eq. 3:
 * Newton's pull summed over the other particles; section 3.2 evaluates the
 * pairs of neighbouring cells directly and the far field by multipoles, this
 * call computes the direct part over the current cells):
 *   g_i = -G sum_{j != i} m_j r_ij (|r_ij|^2 + eps^2)^(-3/2) S(|r_ij| / r_cut),
 * r_ij the minimum image of x_i - x_j in i's box, eps a Plummer softening and
 * S(x) = (1 - x^2)^2 for x < 1, 0 beyond (zero with zero slope at the cutoff,
 * so g is continuous in the positions; the part 1 - S is the far field's).
 * Coincident pairs add nothing. FP32 arithmetic; each particle sums its own
 * pairs (no atomics), so repeated calls give the same bits.
 *   mass    device, n floats, caller order, each finite and > 0 (not
 *           necessarily the masses of the density)
 *   G       finite
 *   eps     finite, >= 0
 *   r_cut   > 0 and at most the smallest search radius of the cells
 *           (sph_params.h_margin x the smallest h of the last build) less
 *           twice the distance the particles may have moved since the build:
 *           every pair closer than that is in the cells' neighbour lists (and
 *           r_cut is below a third of every box, so one image per pair)
 *   acc     device, n x 3 floats, caller order, out (caller-owned; the
 *           gravity alone, not added to anything)
 *   counts  host, nullable, 2 int64 out: [0] ordered pairs (i, j) with
 *           0 < r_ij < r_cut, [1] (particle, candidate) pairs the kernel
 *           tested (the particles of the neighbour cells within reach)
 * Uses the positions of the last sph_build_cells / sph_drift (after drifts
 * that used up the cells' margin it rebuilds them around the last build's
 * guesses first, as sph_density would). Errors: SPH_E_ARG (null, a bad value,
 * an r_cut beyond the limits above, a mass <= 0 or non-finite), SPH_E_STATE
 * (no cells), SPH_E_NOMEM, SPH_E_HIP. Synchronises `stream`.
 */
sph_status sph_gravity_p2p(sph_ctx* ctx, const float* mass, double G, double eps, double r_cut, float* acc,
                           int64_t* counts, void* stream);

/*
 * Balsara factors B of the last force pass (see sph_params.balsara), in the
 * caller's particle order.
 *   balsara  device, n floats, out (caller-owned)
 * Errors: SPH_E_ARG (null), SPH_E_STATE (no force pass with the switch since
 * the last build or drift), SPH_E_HIP. Does not synchronise.
 */
sph_status sph_get_balsara(sph_ctx* ctx, float* balsara, void* stream);

/* Copy the durations of the last calls into *out (host). Errors: SPH_E_ARG. */
sph_status sph_get_timings(const sph_ctx* ctx, sph_timings* out);

/* Shape of the last sph_build_cells (section 3.1's cells and pair tasks). A
 * density sweep tests candidate_pairs (particle, candidate) pairs. */
typedef struct {
    int64_t n_cells;             /* leaf cells */
    int64_t n_pairs;             /* (cell, neighbour cell) entries, self included */
    int64_t max_cell_particles;  /* particles of the largest leaf */
    int64_t max_neighbour_cells; /* longest neighbour-cell list */
    int64_t max_candidates;      /* most particles in one leaf's neighbour cells */
    int64_t candidate_pairs;     /* sum over leaves of particles x candidates */
} sph_build_info;

/* Copy the shape of the last build into *out (host). Errors: SPH_E_ARG,
 * SPH_E_STATE (no build yet). */
sph_status sph_get_build_info(const sph_ctx* ctx, sph_build_info* out);

/* Static description of a status code. */
const char* sph_status_string(sph_status s);

/* Message of the last error on this context ("" if none); ctx may be NULL for
 * errors of sph_create. The string stays valid until the next call. */
const char* sph_last_error(const sph_ctx* ctx);

/* Library version string. */
const char* sph_version(void);

/* sizeof of the structs above as this library was compiled, for bindings that
 * lay them out by hand: which = 0 sph_params, 1 sph_stats, 2 sph_timings,
 * 3 sph_build_info; -1 for any other value. */
int32_t sph_struct_size(int32_t which);

#ifdef __cplusplus
}
#endif

#endif /* SPH_MI355X_H */
