/*
 * sph_oracle.c -- plain FP64 reference for the SPH density and force sums.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or
 * load this file or the library built from it; only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark use it. It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * What it computes (Swift paper, section 2, Eq. 1 and the text after Eq. 2;
 * the force is the grad-h form of the Gadget-2 scheme the paper says Swift
 * implements, in the internal-energy variable):
 *
 *   kernel     W(r, h) = 8 / (pi h^3) * w(q),  q = r / h, support q < 1
 *              w(q) = 1 - 6 q^2 + 6 q^3   (0 <= q <= 1/2)
 *                   = 2 (1 - q)^3         (1/2 < q <= 1),  0 beyond
 *   density    rho_i = sum_j m_j W(r_ij, h_i), the sum including j = i (Eq. 1)
 *   h_i        the root of (4 pi / 3) h^3 sum_j W(r_ij, h) = N_ngb, i.e.
 *              S0(h) = sum_j w(r_ij / h) = 3 N_ngb / 32  (the "given weighted
 *              number of particles" of section 2)
 *   grad-h     f_i = [1 + h/(3 rho) d rho/dh]^-1 = -3 M0 / M1
 *              with M0 = sum m_j w, M1 = sum m_j q w'(q)
 *   ghost      P = (gamma - 1) rho u, c = sqrt(gamma (gamma - 1) u),
 *              Phi = f P / rho^2   (pressure from density and temperature
 *              through the equation of state, section 2)
 *   force      for each pair with 0 < r < max(h_i, h_j), rhat = (x_i - x_j)/r:
 *              D_k = 8 / (pi h_k^4) w'(r / h_k)   (0 when r >= h_k)
 *              w_ij = min(v_ij . rhat, 0)
 *              Pi_ij = -alpha (c_i + c_j - 3 w_ij) w_ij / (rho_i + rho_j)
 *              G = Phi_i D_i + Phi_j D_j + Pi_ij (D_i + D_j) / 2
 *              a_i    -= m_j G rhat
 *              du_i/dt += m_j (Phi_i D_i + Pi_ij (D_i + D_j) / 4) (v_ij . rhat)
 *   Eq. 2 form (optional, form = 1) the paper's own illustration of the
 *              pressure sum in place of the grad-h terms:
 *              G = (P_i / rho_i^2 + P_j / rho_j^2) D_i + Pi_ij (D_i + D_j) / 2
 *              and du_i/dt += m_j (P_i / rho_i^2 D_i + Pi_ij (D_i + D_j) / 4)
 *              (v_ij . rhat), the first law with the Eq. 1 density's rate at
 *              fixed h_i; f plays no part
 *   Balsara    (optional) Pi_ij is scaled by (B_i + B_j) / 2 with the
 *              Balsara factor B_k = |div v|_k / (|div v|_k + |curl v|_k +
 *              1e-4 c_k / h_k) (the Gadget-2 form; not in the paper), from
 *              rho_i (div v)_i  = sum_j m_j (v_j - v_i) . rhat D_i
 *              rho_i (curl v)_i = sum_j m_j (v_i - v_j) x rhat D_i
 *              over 0 < r_ij < h_i (orc_divcurl)
 *
 * Distances use the minimum image of a periodic cubic box of side L, which
 * needs every smoothing length below L / 2 (checked).
 *
 * Neighbour search: a uniform bucket grid of g^3 cells; the particles within
 * a radius R of a point are found by visiting every bucket the cube of half
 * side R touches. This is the oracle's own search and has nothing in common
 * with the cell/task structure of the library.
 *
 * h is found per particle by bracketed Newton iteration with bisection
 * fallback on S0(h) - target, which is continuous and non-decreasing in h
 * and strictly increasing once a second particle is inside h, so the root is
 * unique and does not depend on the starting value.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

enum { ORC_OK = 0, ORC_E_ARG = 1, ORC_E_NOMEM = 2, ORC_E_RADIUS = 3, ORC_E_ROOT = 4, ORC_E_MISSING = 5 };

/* ---- cubic-spline kernel (shape only, support 1) ---------------------- */

static double w_shape(double q)
{
    if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) { double t = 1.0 - q; return 2.0 * t * t * t; }
    return 0.0;
}

static double dw_shape(double q)
{
    if (q < 0.5) return -12.0 * q + 18.0 * q * q;
    if (q < 1.0) { double t = 1.0 - q; return -6.0 * t * t; }
    return 0.0;
}

/* ---- bucket grid ------------------------------------------------------- */

typedef struct {
    int64_t g;        /* buckets per side */
    double L, cw;     /* box side, bucket width */
    int64_t *start;   /* g^3 + 1 offsets into idx */
    int64_t *idx;     /* particle indices grouped by bucket */
} grid_t;

static double wrap(double x, double L)
{
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y = 0.0;
    return y;
}

static int64_t bucket_of(double x, const grid_t *gr)
{
    int64_t i = (int64_t)floor(wrap(x, gr->L) / gr->cw);
    if (i < 0) i = 0;
    if (i >= gr->g) i = gr->g - 1;
    return i;
}

static int grid_build(grid_t *gr, int64_t n, const double *pos, double L)
{
    int64_t g = (int64_t)cbrt((double)n);
    if (g < 1) g = 1;
    if (g > 256) g = 256;
    gr->g = g;
    gr->L = L;
    gr->cw = L / (double)g;
    int64_t nc = g * g * g;
    gr->start = (int64_t *)calloc((size_t)(nc + 1), sizeof(int64_t));
    gr->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *cell = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!gr->start || !gr->idx || !cell) { free(cell); return ORC_E_NOMEM; }
    for (int64_t p = 0; p < n; ++p) {
        int64_t ix = bucket_of(pos[3 * p + 0], gr);
        int64_t iy = bucket_of(pos[3 * p + 1], gr);
        int64_t iz = bucket_of(pos[3 * p + 2], gr);
        cell[p] = (ix * g + iy) * g + iz;
        gr->start[cell[p] + 1] += 1;
    }
    for (int64_t c = 0; c < nc; ++c) gr->start[c + 1] += gr->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
    if (!fill) { free(cell); return ORC_E_NOMEM; }
    memcpy(fill, gr->start, (size_t)nc * sizeof(int64_t));
    for (int64_t p = 0; p < n; ++p) gr->idx[fill[cell[p]]++] = p;
    free(fill);
    free(cell);
    return ORC_OK;
}

static void grid_free(grid_t *gr)
{
    free(gr->start);
    free(gr->idx);
}

/* Candidate list of one particle: every j with |r_ij| < R (minimum image). */
typedef struct {
    int64_t n, cap;
    int64_t *j;
    double *r;      /* |r_ij| */
    double *dx;     /* 3 components of the minimum-image r_i - r_j */
} cand_t;

static int cand_push(cand_t *c, int64_t j, double r, const double d[3])
{
    if (c->n == c->cap) {
        int64_t cap = c->cap ? 2 * c->cap : 256;
        int64_t *nj = (int64_t *)realloc(c->j, (size_t)cap * sizeof(int64_t));
        if (!nj) return ORC_E_NOMEM;
        c->j = nj;
        double *nr = (double *)realloc(c->r, (size_t)cap * sizeof(double));
        if (!nr) return ORC_E_NOMEM;
        c->r = nr;
        double *nd = (double *)realloc(c->dx, (size_t)cap * 3 * sizeof(double));
        if (!nd) return ORC_E_NOMEM;
        c->dx = nd;
        c->cap = cap;
    }
    c->j[c->n] = j;
    c->r[c->n] = r;
    c->dx[3 * c->n + 0] = d[0];
    c->dx[3 * c->n + 1] = d[1];
    c->dx[3 * c->n + 2] = d[2];
    c->n += 1;
    return ORC_OK;
}

static void cand_free(cand_t *c)
{
    free(c->j);
    free(c->r);
    free(c->dx);
}

/* Visit buckets within R of particle i along each axis. When the window would
 * wrap onto itself, every bucket of that axis is visited exactly once. */
static int gather(const grid_t *gr, const double *pos, int64_t i, double R, cand_t *c)
{
    const double L = gr->L;
    const int64_t g = gr->g;
    int64_t k = (int64_t)ceil(R / gr->cw);
    int64_t lo[3], hi[3], ci[3];
    int full[3];
    for (int a = 0; a < 3; ++a) {
        ci[a] = bucket_of(pos[3 * i + a], gr);
        full[a] = (2 * k + 1 >= g);
        lo[a] = full[a] ? 0 : ci[a] - k;
        hi[a] = full[a] ? g - 1 : ci[a] + k;
    }
    c->n = 0;
    const double R2 = R * R;
    for (int64_t ax = lo[0]; ax <= hi[0]; ++ax) {
        int64_t bx = ((ax % g) + g) % g;
        for (int64_t ay = lo[1]; ay <= hi[1]; ++ay) {
            int64_t by = ((ay % g) + g) % g;
            for (int64_t az = lo[2]; az <= hi[2]; ++az) {
                int64_t bz = ((az % g) + g) % g;
                int64_t b = (bx * g + by) * g + bz;
                for (int64_t t = gr->start[b]; t < gr->start[b + 1]; ++t) {
                    int64_t j = gr->idx[t];
                    double d[3], r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double e = pos[3 * i + a] - pos[3 * j + a];
                        e -= L * nearbyint(e / L);
                        d[a] = e;
                        r2 += e * e;
                    }
                    if (r2 < R2) {
                        if (cand_push(c, j, sqrt(r2), d)) return ORC_E_NOMEM;
                    }
                }
            }
        }
    }
    return ORC_OK;
}

/* S0 = sum w(r/h), S1 = sum q w'(q), over candidates with r < h. */
static void shape_sums(const cand_t *c, const double *mass, double h,
                       double *S0, double *S1, double *M0, double *M1, int64_t *cnt, int64_t self)
{
    double s0 = 0, s1 = 0, m0 = 0, m1 = 0;
    int64_t k = 0;
    for (int64_t t = 0; t < c->n; ++t) {
        double r = c->r[t];
        if (r >= h) continue;
        double q = r / h;
        double w = w_shape(q), dw = dw_shape(q);
        double m = mass[c->j[t]];
        s0 += w;
        s1 += q * dw;
        m0 += m * w;
        m1 += m * q * dw;
        if (c->j[t] != self) k += 1;
    }
    *S0 = s0; *S1 = s1; *M0 = m0; *M1 = m1; *cnt = k;
}

/*
 * Smoothing length, density, grad-h factor and neighbour counts of the
 * listed target particles (all particles when targets == NULL).
 *   h_start   optional starting radius per particle (only sets where the
 *             search begins; the result is the same root for any value)
 *   nw_out    weighted neighbour number (32/3) S0 at the root
 *   nngb_out  #{j != i : r_ij < h_i}
 * Returns ORC_OK or an error code; *bad is set to the first failing index.
 */
int orc_density(int64_t n, const double *pos, const double *mass, double L, double n_ngb,
                int64_t n_targets, const int64_t *targets, const double *h_start,
                double *h_out, double *rho_out, double *f_out, double *nw_out,
                int64_t *nngb_out, int nthreads, int64_t *bad)
{
    if (n <= 0 || !pos || !mass || !(L > 0) || !(n_ngb > 0) || !h_out || !rho_out || !f_out)
        return ORC_E_ARG;
    if (nthreads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(nthreads);
#endif
    }
    grid_t gr;
    int rc = grid_build(&gr, n, pos, L);
    if (rc) { grid_free(&gr); return rc; }
    const int64_t nt = targets ? n_targets : n;
    const double target = 3.0 * n_ngb / 32.0;
    const double r0 = cbrt(3.0 * n_ngb / (4.0 * ORC_PI * (double)n)) * L; /* uniform-density radius */
    int status = ORC_OK;
    *bad = -1;

#pragma omp parallel
    {
        cand_t c = {0, 0, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < nt; ++t) {
            int st;
#pragma omp atomic read
            st = status;
            if (st != ORC_OK) continue;
            int64_t i = targets ? targets[t] : t;
            double R = (h_start && h_start[i] > 0) ? h_start[i] : r0;
            double S0, S1, M0, M1;
            int64_t cnt;
            int err = ORC_OK;
            /* grow the search radius until it brackets the root */
            for (;;) {
                if (R >= 0.5 * L) R = 0.5 * L * (1.0 - 1e-12);
                if (gather(&gr, pos, i, R, &c)) { err = ORC_E_NOMEM; break; }
                shape_sums(&c, mass, R, &S0, &S1, &M0, &M1, &cnt, i);
                if (S0 >= target) break;
                if (R >= 0.5 * L * (1.0 - 1e-11)) { err = ORC_E_RADIUS; break; }
                R *= 1.5;
            }
            double h = R;
            if (!err) {
                double lo = 0.0, hi = R;
                h = (h_start && h_start[i] > 0 && h_start[i] < R) ? h_start[i] : 0.5 * R;
                int it;
                for (it = 0; it < 400; ++it) {
                    shape_sums(&c, mass, h, &S0, &S1, &M0, &M1, &cnt, i);
                    double gval = S0 - target;
                    if (fabs(gval) <= 1e-13 * target) break;
                    if (gval < 0) lo = h; else hi = h;
                    if (hi - lo <= 1e-15 * hi) break;
                    double hn = (S1 < 0) ? h + gval * h / S1 : -1.0; /* Newton: dS0/dh = -S1/h */
                    if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
                    h = hn;
                }
                if (it == 400) err = ORC_E_ROOT;
            }
            if (err) {
#pragma omp critical
                {
                    if (status == ORC_OK) { status = err; *bad = i; }
                }
                continue;
            }
            shape_sums(&c, mass, h, &S0, &S1, &M0, &M1, &cnt, i);
            h_out[i] = h;
            rho_out[i] = 8.0 / (ORC_PI * h * h * h) * M0;
            f_out[i] = (M1 != 0.0) ? -3.0 * M0 / M1 : 1.0;
            if (nw_out) nw_out[i] = 32.0 / 3.0 * S0;
            if (nngb_out) nngb_out[i] = cnt;
        }
        cand_free(&c);
    }
    grid_free(&gr);
    return status;
}

/*
 * Acceleration and du/dt of the listed targets (all when targets == NULL).
 * h, rho, f must be valid for every particle within reach of a target. A
 * particle with h <= 0 (or NaN) is treated as unknown: it is skipped when it
 * lies at or beyond h_i of the target (it then pairs only through its own h,
 * which the caller vouches is not the case), and it is an error
 * (ORC_E_MISSING, *bad = the target) when it lies inside h_i, where it pairs
 * whatever its h.
 *   gross_a_out   sum_j |m_j G|, the scale the acceleration error is judged by
 *   gross_u_out   sum_j |m_j (Phi_i D_i + Pi Dbar / 2)(v_ij . rhat)|
 *   scale_a_out   sum_j m_j (|Phi_i| Dm_i + |Phi_j| Dm_j + |Pi| (Dm_i + Dm_j) / 2), where
 *                 Dm_k = 8 / (pi h_k^4) max|w'| (max|w'| = 2) for r < h_k, else 0: the
 *                 pair terms at full kernel slope. Unlike the gross sum it does not
 *                 shrink where w'(q) -> 0 at the kernel edge, so errors are judged
 *                 against a scale that rounding in q cannot exceed.
 *   scale_u_out   sum_j m_j (|Phi_i| Dm_i + |Pi| (Dm_i + Dm_j) / 4) |v_ij . rhat|
 *   npair_out     #{j != i : 0 < r_ij < max(h_i, h_j)}: the pairs that carry a
 *                 force term (a coincident pair has no direction and adds
 *                 nothing, so it is not a force interaction)
 *   vsig_out      signal velocity max(c_i, max_j (c_i + c_j - 3 w_ij)) over the
 *                 pairs with 0 < r_ij < max(h_i, h_j): the speed in the Courant
 *                 condition of the time step (the Gadget-2 choice that the
 *                 paper's force form follows)
 *   balsara       per-particle Balsara factors B (see the header) scaling the
 *                 viscosity by (B_i + B_j) / 2; NULL: no switch
 *   form          0: the grad-h Gadget-2 pressure terms; 1: the Eq. 2 form
 */
int orc_force(int64_t n, const double *pos, const double *vel, const double *mass,
              const double *u, const double *h, const double *rho, const double *f,
              double L, double gamma, double alpha, int64_t n_targets, const int64_t *targets,
              double *acc_out, double *dudt_out, double *gross_a_out, double *gross_u_out,
              double *scale_a_out, double *scale_u_out, int64_t *npair_out, double *vsig_out,
              const double *balsara, int form, int nthreads, int64_t *bad)
{
    if (n <= 0 || !pos || !vel || !mass || !u || !h || !rho || !f || !acc_out || !dudt_out)
        return ORC_E_ARG;
    if (nthreads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(nthreads);
#endif
    }
    double hmax = 0.0;
    for (int64_t p = 0; p < n; ++p)
        if (h[p] > hmax) hmax = h[p];
    if (!(hmax < 0.5 * L)) return ORC_E_RADIUS;
    grid_t gr;
    int rc = grid_build(&gr, n, pos, L);
    if (rc) { grid_free(&gr); return rc; }
    const int64_t nt = targets ? n_targets : n;
    int status = ORC_OK;
    *bad = -1;

#pragma omp parallel
    {
        cand_t c = {0, 0, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < nt; ++t) {
            int st;
#pragma omp atomic read
            st = status;
            if (st != ORC_OK) continue;
            int64_t i = targets ? targets[t] : t;
            if (!(h[i] > 0)) {
#pragma omp critical
                { if (status == ORC_OK) { status = ORC_E_ARG; *bad = i; } }
                continue;
            }
            double R = h[i] > hmax ? h[i] : hmax;
            if (R >= 0.5 * L) R = 0.5 * L * (1.0 - 1e-12);
            if (gather(&gr, pos, i, R, &c)) {
#pragma omp critical
                { if (status == ORC_OK) { status = ORC_E_NOMEM; *bad = i; } }
                continue;
            }
            const double hi_ = h[i];
            const double Pi_ = (gamma - 1.0) * rho[i] * u[i];
            const double ci = sqrt(gamma * (gamma - 1.0) * u[i]);
            const double Phii = (form == 1 ? 1.0 : f[i]) * Pi_ / (rho[i] * rho[i]);
            double ax = 0, ay = 0, az = 0, du = 0, ga = 0, gu = 0, sa = 0, su = 0;
            double vsig = ci;
            int64_t np = 0;
            int missing = 0;
            for (int64_t k = 0; k < c.n; ++k) {
                int64_t j = c.j[k];
                double r = c.r[k];
                if (j == i) continue;
                if (!(h[j] > 0)) {
                    if (r < hi_) { missing = 1; break; } /* a partner whose h is unknown */
                    continue;
                }
                double hj = h[j];
                if (!(r < hi_ || r < hj)) continue;
                if (r == 0.0) continue; /* coincident: no direction, no force */
                np += 1;
                double ex = c.dx[3 * k + 0] / r, ey = c.dx[3 * k + 1] / r, ez = c.dx[3 * k + 2] / r;
                double Di = 8.0 / (ORC_PI * hi_ * hi_ * hi_ * hi_) * dw_shape(r / hi_);
                double Dj = 8.0 / (ORC_PI * hj * hj * hj * hj) * dw_shape(r / hj);
                double Pj = (gamma - 1.0) * rho[j] * u[j];
                double cj = sqrt(gamma * (gamma - 1.0) * u[j]);
                double Phij = (form == 1 ? 1.0 : f[j]) * Pj / (rho[j] * rho[j]);
                double vr = (vel[3 * i + 0] - vel[3 * j + 0]) * ex +
                            (vel[3 * i + 1] - vel[3 * j + 1]) * ey +
                            (vel[3 * i + 2] - vel[3 * j + 2]) * ez;
                double wv = vr < 0.0 ? vr : 0.0;
                double Pv = -alpha * (ci + cj - 3.0 * wv) * wv / (rho[i] + rho[j]);
                if (balsara) Pv *= 0.5 * (balsara[i] + balsara[j]);
                double vs = ci + cj - 3.0 * wv;
                if (vs > vsig) vsig = vs;
                double Dbar = 0.5 * (Di + Dj);
                double G = Phii * Di + Phij * (form == 1 ? Di : Dj) + Pv * Dbar;
                double mj = mass[j];
                ax -= mj * G * ex;
                ay -= mj * G * ey;
                az -= mj * G * ez;
                double e = mj * (Phii * Di + 0.5 * Pv * Dbar) * vr;
                du += e;
                ga += fabs(mj * G);
                gu += fabs(e);
                double Dmi = r < hi_ ? 2.0 * 8.0 / (ORC_PI * hi_ * hi_ * hi_ * hi_) : 0.0;
                double Dmj = r < hj ? 2.0 * 8.0 / (ORC_PI * hj * hj * hj * hj) : 0.0;
                sa += mj * (fabs(Phii) * Dmi + fabs(Phij) * (form == 1 ? Dmi : Dmj) + fabs(Pv) * 0.5 * (Dmi + Dmj));
                su += mj * (fabs(Phii) * Dmi + 0.25 * fabs(Pv) * (Dmi + Dmj)) * fabs(vr);
            }
            if (missing) {
#pragma omp critical
                { if (status == ORC_OK) { status = ORC_E_MISSING; *bad = i; } }
                continue;
            }
            acc_out[3 * i + 0] = ax;
            acc_out[3 * i + 1] = ay;
            acc_out[3 * i + 2] = az;
            dudt_out[i] = du;
            if (gross_a_out) gross_a_out[i] = ga;
            if (gross_u_out) gross_u_out[i] = gu;
            if (scale_a_out) scale_a_out[i] = sa;
            if (scale_u_out) scale_u_out[i] = su;
            if (npair_out) npair_out[i] = np;
            if (vsig_out) vsig_out[i] = vsig;
        }
        cand_free(&c);
    }
    grid_free(&gr);
    return status;
}

/*
 * Velocity divergence and curl of the listed targets (all when targets ==
 * NULL), the SPH estimates of the header's Balsara paragraph: the gather sums
 * over the neighbours j != i with 0 < r_ij < h_i, divided by rho_i.
 *   div_out       (div v)_i
 *   curl_out      (curl v)_i, 3 per particle
 *   scale_out     sum_j m_j |v_ij| Dm_i / rho_i with Dm_i = 16 / (pi h_i^4),
 *                 the terms at full kernel slope (max|w'| = 2): it bounds
 *                 both sums' terms and does not shrink at the kernel edge,
 *                 so it is the scale their rounding errors are judged by
 * h and rho must be valid for every particle within h of a target.
 */
int orc_divcurl(int64_t n, const double *pos, const double *vel, const double *mass,
                const double *h, const double *rho, double L, int64_t n_targets, const int64_t *targets,
                double *div_out, double *curl_out, double *scale_out, int nthreads, int64_t *bad)
{
    if (n <= 0 || !pos || !vel || !mass || !h || !rho || !div_out || !curl_out) return ORC_E_ARG;
    if (nthreads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(nthreads);
#endif
    }
    double hmax = 0.0;
    for (int64_t p = 0; p < n; ++p)
        if (h[p] > hmax) hmax = h[p];
    if (!(hmax < 0.5 * L)) return ORC_E_RADIUS;
    grid_t gr;
    int rc = grid_build(&gr, n, pos, L);
    if (rc) { grid_free(&gr); return rc; }
    const int64_t nt = targets ? n_targets : n;
    int status = ORC_OK;
    *bad = -1;

#pragma omp parallel
    {
        cand_t c = {0, 0, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < nt; ++t) {
            int st;
#pragma omp atomic read
            st = status;
            if (st != ORC_OK) continue;
            int64_t i = targets ? targets[t] : t;
            if (!(h[i] > 0) || !(rho[i] > 0) || gather(&gr, pos, i, h[i], &c)) {
#pragma omp critical
                { if (status == ORC_OK) { status = h[i] > 0 && rho[i] > 0 ? ORC_E_NOMEM : ORC_E_ARG; *bad = i; } }
                continue;
            }
            const double hi_ = h[i];
            double dv = 0, cx = 0, cy = 0, cz = 0, g = 0;
            for (int64_t k = 0; k < c.n; ++k) {
                int64_t j = c.j[k];
                double r = c.r[k];
                if (j == i || !(r > 0.0) || !(r < hi_)) continue;
                double ex = c.dx[3 * k + 0] / r, ey = c.dx[3 * k + 1] / r, ez = c.dx[3 * k + 2] / r;
                double Di = 8.0 / (ORC_PI * hi_ * hi_ * hi_ * hi_) * dw_shape(r / hi_);
                double wx = vel[3 * i + 0] - vel[3 * j + 0];  /* v_i - v_j */
                double wy = vel[3 * i + 1] - vel[3 * j + 1];
                double wz = vel[3 * i + 2] - vel[3 * j + 2];
                double mD = mass[j] * Di;
                dv -= mD * (wx * ex + wy * ey + wz * ez);
                cx += mD * (wy * ez - wz * ey);
                cy += mD * (wz * ex - wx * ez);
                cz += mD * (wx * ey - wy * ex);
                g += mass[j] * 16.0 / (ORC_PI * hi_ * hi_ * hi_ * hi_) * sqrt(wx * wx + wy * wy + wz * wz);
            }
            div_out[i] = dv / rho[i];
            curl_out[3 * i + 0] = cx / rho[i];
            curl_out[3 * i + 1] = cy / rho[i];
            curl_out[3 * i + 2] = cz / rho[i];
            if (scale_out) scale_out[i] = g / rho[i];
        }
        cand_free(&c);
    }
    grid_free(&gr);
    return status;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
