/* O1-1DH: literal FP64 hybrid DDMC / continuous-MC walker on 1D grids (slab cells along z,
 * or spherical shells) -- ORACLE, TEST INFRASTRUCTURE ONLY.  Plain C; shares nothing with
 * the GPU library.
 *
 * Packets carry a full 3D position and direction; the geometry enters through the cells'
 * boundaries (planes z = z_f, or spheres r = r_f), their outward normals (+-z, or +-r^), and
 * the bulk velocity field (slab: u_c along +z; shell: u_c along r^, u_c = v_c / v_th(T_c)).
 *
 *  - DDMC states (tau_ij = k_ij w_i >= tau_th): every step draws dl_X = -ln(xi_X) / k_X for
 *    EVERY leak X (two faces: eq. 10 or the thin/vacuum interface rate; two bins: eq. 11) and
 *    takes the smallest (eqs. 15-16);
 *      * through a face whose neighbour is thick at the shifted bin: move there, re-binned by
 *        the f_mu-averaged shift of eq. 20;
 *      * through a face into a thin state or vacuum: an MC packet at a uniform point of that
 *        face with an isotropic outward direction (mu uniform in (0, 1] about the face's
 *        outward normal), x uniform in the bin, moved to the neighbour's frame exactly,
 *        x' = (x + n.u) sqrt(T/T') - n.u' (both velocities at that point); through vacuum it
 *        escapes with the lab frequency x + n.u;
 *      * into a thin bin: an MC packet at a uniform point of the cell (uniform in volume),
 *        isotropic, x uniform in the new bin;
 *      * re-binned into a thin state after a spatial move: MC in the new cell at a uniform
 *        point, isotropic, with the shifted x.
 *  - MC packets: distance to the cell boundary along n against an exponential optical depth
 *    with opacity k0 H(a, x) (eq. 12) at the packet's comoving x;
 *      * scattering: the shared MC physics (atom velocity by rejection, eq. 41 without recoil,
 *        isotropic phase function, optional core-skipping above x_crit); if the state
 *        (cell, bin(x')) is thick the packet becomes DDMC there;
 *      * a boundary: vacuum -> escape at x + n.u; a neighbour at
 *        x' = (x + n.u) sqrt(T/T') - n.u'; if that state is thick the packet converts with
 *        P = 2/(k' w' + 2 lambda) (2/3 + mu) (eq. 39; mu the direction cosine to the face
 *        normal, w' the neighbour's width), else it is reflected from a uniform point of the
 *        interface with an isotropic direction back into its cell and x unchanged; if thin it
 *        flies on in the neighbour.
 *    In a shell the bulk velocity changes direction with position: the packet's comoving x
 *    is kept for the point where it is (the lab frequency x + n.u is constant along a flight,
 *    so x changes by n.(u(p0) - u(p1)) between its start p0 and end p1), and the opacity of
 *    a flight is that of its starting x (exact for slabs, where u is uniform in a cell).
 *  - Escapes are tallied by face (slab: 2 rows; sphere: 1), lab bin and time (c = 1).
 *  - Dust (Sec. 2.4): the tables' rates already use the total scattering coefficient; DDMC
 *    states have one more exponential distance, to absorption at rate k_a, and an absorbed
 *    packet is removed after that residence; MC flights meet Lya, dust scattering (k_s:
 *    isotropic, coherent in the comoving frame) and dust absorption (k_a) in proportion.
 *  - Frequency groups (Sec. 5.3, static isothermal clouds): with P->group the thin states
 *    carry a bin j instead of a continuous x; a flight meets the bin-averaged opacity k_ij
 *    (eq. 14), and a scattering takes its outgoing bin from the flat-in-bin law of eq. 42 by
 *    simulation: an x uniform in bin j, one scattering of the continuous law above (its own
 *    throwaway direction), and the bin of the outgoing x (bins 0 and nb-1 take everything
 *    below and above the grid); the packet's new direction is isotropic and independent of
 *    that frequency change.  Crossings keep j; escapes are tallied in bin j.
 *  - Dust by continuous weights (Sec. 2.4's second method, P->dust_weight): absorption is no
 *    event; the packet's weight w = exp(-L) decays with L += k_a dl over every stretch dl it
 *    travels (a DDMC step's interaction distance, an MC flight), the packet is dropped (counted
 *    as absorbed) once w < 1e-10, and escapes add w (and w^2) to the weighted spectra.  The
 *    census estimators take the weight along the path: w(t_e) at a census time and the
 *    integral of w over a residence, (w(a) - w(b)) / k_a; eq. 18 likewise.
 *  - Time-dependent estimators (eq. 17), unnormalised: at every census time t_e the packet's
 *    state is counted ('bin'), and its residence time in each state is summed per census
 *    interval ('path'); an MC packet's state is (cell, bin of its comoving x at the start of
 *    the flight).  Packets are emitted at t = 0, or uniformly over their source's window.
 *  - Acceleration estimator (eq. 18), per cell and census interval, along z (slab) or r
 *    (shells): a DDMC spatial leak of a step with residence [t0, t1) in state (c, j), moving
 *    along d = -1 (face 0) or +1 (face 1), adds k_{c,j} d times the step's residence in each
 *    interval to cell c (outward leakage), and k_{c',j'} d times the same to the cell c' it
 *    enters when it lands there in a DDMC state (c', j') (inward leakage): both carry the
 *    sign of the motion.  Leaks into continuous-MC states or vacuum count for c only.
 *
 * Random numbers: xoshiro256** per packet seeded by splitmix64(seed ^ id*golden).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "mcphys.h"

#define OH_TIME_BINS 128
#define OH_STEP_BINS 64

typedef struct {
    int32_t geometry;              /* 0 slab, 1 spherical shells */
    int32_t nc, nb;
    const double *faces;           /* nc+1 face coordinates (z, or r) */
    const double *edges;           /* nb+1 */
    const double *k;               /* [nc*nb] bin-averaged opacity (eq. 14) */
    const uint8_t *thick;          /* [nc*nb] */
    const double *rate_face;       /* [nc*nb*2] */
    const uint8_t *face_mc;        /* [nc*nb*2] the leak through this face uses the interface rate */
    const double *rate_dn, *rate_up;  /* [nc*nb] */
    const int64_t *nbr;            /* [nc*2]: >= 0 cell, -1 vacuum, -2 no face */
    const double *rho, *shift;     /* [nc*2] DDMC re-binning map into the neighbour */
    const double *k0, *a, *T;      /* [nc] */
    const double *u;               /* [nc] bulk speed along +z (slab) or +r^ (shell) / v_th(T_c) */
    double lambda, x_crit;
    int32_t n_src;
    const int64_t *src_state;      /* [n_src] */
    const double *src_pos;         /* [n_src] z, or r (a source at r > 0 is placed on the +z axis) */
    const double *src_x;           /* [n_src] */
    const double *src_cdf;         /* [n_src] */
    const double *k_abs, *k_sca;   /* [nc] dust absorption / scattering coefficients, or NULL */
    const double *src_t;           /* [n_src*2] emission windows, or NULL (flash at t = 0) */
    int32_t n_census;              /* census intervals (0 = none) */
    const double *census;          /* [n_census+1] increasing census times */
    int32_t group;                 /* 1: thin states use frequency groups (Sec. 5.3) */
    int32_t dust_weight;           /* 1: dust absorption by continuous weights (Sec. 2.4) */
} oh_problem;

typedef struct {
    int64_t *spectrum;     /* [rows*(nb+2)], rows = 2 (slab) or 1 (sphere) */
    int64_t *time_hist;    /* [OH_TIME_BINS+2] */
    int64_t *step_hist;    /* [OH_STEP_BINS] */
    double t_sum, t2_sum, steps_sum, mc_steps_sum, steps2_sum;
    int64_t escaped, capped, to_mc, to_ddmc, reflected, absorbed;
    double *e_bin;         /* [(n_census+1)*nc*nb] counts of packets in each state at each census time */
    double *e_path;        /* [n_census*nc*nb] residence time in each state per census interval */
    double *e_accel;       /* [n_census*nc] eq. 18 optical-depth sums (z or r component) */
    double *wspec, *wspec2;    /* [rows*(nb+2)] escaped weight and squared weight (dust_weight) */
    double wt_sum, wt2_sum, w_sum;
} oh_result;

static int locate(const double *e, int nb, double x)
{
    if (x < e[0]) return -1;
    if (x >= e[nb]) return nb;
    int lo = 0, hi = nb;
    while (hi - lo > 1) { int m = (lo + hi) >> 1; if (x >= e[m]) lo = m; else hi = m; }
    return lo;
}

static int time_bin(double t)
{
    if (!(t >= 1e-3)) return 0;
    double u = (log10(t) + 3.0) / 9.0 * OH_TIME_BINS;
    if (u >= OH_TIME_BINS) return OH_TIME_BINS + 1;
    return 1 + (int)u;
}

static int step_bin(uint64_t n) { int b = 0; while (n > 1) { n >>= 1; ++b; } return b; }

static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* unit vector along p (the +z axis at the origin) */
static void radial(const double p[3], double e[3])
{
    double r = sqrt(dot(p, p));
    if (r > 0.0) { e[0] = p[0] / r; e[1] = p[1] / r; e[2] = p[2] / r; }
    else { e[0] = 0.0; e[1] = 0.0; e[2] = 1.0; }
}

/* outward normal of a cell at face f (0 lower / inner, 1 upper / outer) at point p */
static void face_normal(const oh_problem *P, int f, const double p[3], double nrm[3])
{
    double s = f ? 1.0 : -1.0;
    if (P->geometry == 0) { nrm[0] = 0.0; nrm[1] = 0.0; nrm[2] = s; return; }
    radial(p, nrm);
    nrm[0] *= s; nrm[1] *= s; nrm[2] *= s;
}

/* n . u of cell c at point p */
static double n_dot_u(const oh_problem *P, int64_t c, const double p[3], const double n[3])
{
    if (P->geometry == 0) return n[2] * P->u[c];
    double e[3];
    radial(p, e);
    return P->u[c] * dot(n, e);
}

/* direction with cosine mu ~ U(0, 1] about the unit vector N, uniform azimuth */
static void hemi_about(rng_t *r, const double N[3], double n[3])
{
    double mu = ru(r), ph = 2.0 * M_PI * ru(r), s = sqrt(fmax(0.0, 1.0 - mu * mu));
    double t1[3], t2[3];
    /* an orthonormal pair perpendicular to N */
    if (fabs(N[2]) < 0.9) { t1[0] = -N[1]; t1[1] = N[0]; t1[2] = 0.0; }
    else { t1[0] = 0.0; t1[1] = -N[2]; t1[2] = N[1]; }
    double l = sqrt(dot(t1, t1));
    t1[0] /= l; t1[1] /= l; t1[2] /= l;
    t2[0] = N[1] * t1[2] - N[2] * t1[1];
    t2[1] = N[2] * t1[0] - N[0] * t1[2];
    t2[2] = N[0] * t1[1] - N[1] * t1[0];
    double c1 = s * cos(ph), c2 = s * sin(ph);
    for (int d = 0; d < 3; ++d) n[d] = mu * N[d] + c1 * t1[d] + c2 * t2[d];
}

/* uniform point of face f of cell c */
static void face_point(const oh_problem *P, int64_t c, int f, rng_t *r, double p[3])
{
    double rf = P->faces[c + f];
    if (P->geometry == 0) { p[0] = 0.0; p[1] = 0.0; p[2] = rf; return; }
    double w[3];
    iso_dir(r, w);
    p[0] = rf * w[0]; p[1] = rf * w[1]; p[2] = rf * w[2];
}

/* uniform point of cell c (uniform in volume) */
static void cell_point(const oh_problem *P, int64_t c, rng_t *r, double p[3])
{
    double lo = P->faces[c], hi = P->faces[c + 1];
    if (P->geometry == 0) { p[0] = 0.0; p[1] = 0.0; p[2] = lo + (hi - lo) * ru(r); return; }
    double rr = cbrt(lo * lo * lo + ru(r) * (hi * hi * hi - lo * lo * lo));
    double w[3];
    iso_dir(r, w);
    p[0] = rr * w[0]; p[1] = rr * w[1]; p[2] = rr * w[2];
}

/* distance along n to the boundary of cell c from p, and the face it reaches */
/* A flight that starts on the cell's inner sphere moving outward cannot meet that sphere again
 * (a line leaves a ball once): left_inner says so, where the sign of p . n cannot for a grazing
 * flight. */
static double wall_distance(const oh_problem *P, int64_t c, const double p[3], const double n[3], int left_inner,
                            int *face)
{
    double lo = P->faces[c], hi = P->faces[c + 1];
    if (P->geometry == 0) {
        if (n[2] > 0.0) { *face = 1; return fmax(0.0, (hi - p[2]) / n[2]); }
        if (n[2] < 0.0) { *face = 0; return fmax(0.0, (lo - p[2]) / n[2]); }
        *face = 1;
        return INFINITY;
    }
    double b = dot(p, n);
    /* the packet is inside its shell: a point put on a face can sit a rounding error outside,
     * which would turn the far root into a zero-length crossing back and forth */
    double rr = fmin(fmax(sqrt(dot(p, p)), lo), hi), pp = rr * rr;
    double s_out = -b + sqrt(fmax(0.0, b * b - pp + hi * hi));
    *face = 1;
    if (lo > 0.0 && b < 0.0 && !left_inner) {
        double disc = b * b - pp + lo * lo;
        if (disc > 0.0) {
            double s_in = -b - sqrt(disc);
            if (s_in < 0.0) s_in = 0.0;
            if (s_in < s_out) { *face = 0; return s_in; }
        }
    }
    return fmax(0.0, s_out);
}

/* the packet stays in state s over [t0, t1): census counts and residence times */
/* weight at time t of a packet with L = L0 at t0 decaying at rate ka (c = 1) */
static double weight_at(double t, double t0, double L0, double ka) { return exp(-(L0 + ka * (t - t0))); }

/* integral of that weight over [a, b) (the residence without weights: ka = 0, L0 = 0) */
static double weight_int(double a, double b, double t0, double L0, double ka)
{
    if (ka > 0.0) return (weight_at(a, t0, L0, ka) - weight_at(b, t0, L0, ka)) / ka;
    return exp(-L0) * (b - a);
}

static void census_add(const oh_problem *P, oh_result *R, int64_t s, double t0, double t1, double L0, double ka)
{
    if (P->n_census <= 0) return;
    const int64_t ns = (int64_t)P->nc * P->nb;
    for (int e = 0; e <= P->n_census; ++e)
        if (P->census[e] >= t0 && P->census[e] < t1)
            R->e_bin[(int64_t)e * ns + s] += P->dust_weight ? weight_at(P->census[e], t0, L0, ka) : 1.0;
    for (int n = 0; n < P->n_census; ++n) {
        double a = fmax(t0, P->census[n]), b = fmin(t1, P->census[n + 1]);
        if (b > a) R->e_path[(int64_t)n * ns + s] += P->dust_weight ? weight_int(a, b, t0, L0, ka) : b - a;
    }
}

/* eq. 18: a leak of a step that stayed over [t0, t1) adds v times its residence in each census
 * interval to cell c */
static void accel_add(const oh_problem *P, oh_result *R, int64_t c, double t0, double t1, double v, double L0,
                      double ka)
{
    if (P->n_census <= 0) return;
    for (int n = 0; n < P->n_census; ++n) {
        double a = fmax(t0, P->census[n]), b = fmin(t1, P->census[n + 1]);
        if (b > a) R->e_accel[(int64_t)n * P->nc + c] += v * (P->dust_weight ? weight_int(a, b, t0, L0, ka) : b - a);
    }
}

static int64_t mc_state(const oh_problem *P, int64_t c, double x)
{
    int j = locate(P->edges, P->nb, x);
    j = j < 0 ? 0 : (j > P->nb - 1 ? P->nb - 1 : j);
    return c * P->nb + j;
}

static void tally_escape(oh_result *R, const oh_problem *P, int f, double xlab, double t, double L)
{
    int nb = P->nb;
    int row = P->geometry == 0 ? f : 0;
    int slot = locate(P->edges, nb, xlab) + 1;
    R->spectrum[(int64_t)row * (nb + 2) + slot]++;
    if (P->dust_weight) {
        const double w = exp(-L);
        R->wspec[(int64_t)row * (nb + 2) + slot] += w;
        R->wspec2[(int64_t)row * (nb + 2) + slot] += w * w;
        R->w_sum += w;
        R->wt_sum += w * t;
        R->wt2_sum += w * t * t;
    }
    R->escaped++;
    R->t_sum += t;
    R->t2_sum += t * t;
    R->time_hist[time_bin(t)]++;
}

typedef struct {
    const oh_problem *p;
    uint64_t first, n, seed, max_steps;
    volatile uint64_t *next;
    pthread_mutex_t *lock;
    oh_result *out;
    uint64_t grain;                /* packets a thread takes at a time */
} job_t;

static void walk_packet(const oh_problem *P, uint64_t id, uint64_t seed, uint64_t max_steps, oh_result *R)
{
    rng_t r;
    uint64_t xs = seed ^ (id * 0x9E3779B97F4A7C15ull);
    for (int i = 0; i < 4; ++i) r.s[i] = sm64(&xs);
    const int nb = P->nb;
    double uu = ru(&r);
    int k = 0;
    while (k < P->n_src - 1 && uu >= P->src_cdf[k]) ++k;
    int64_t s = P->src_state[k];
    int64_t c = s / nb;
    int j = (int)(s % nb);
    int mc = !P->thick[s];
    double pos[3] = {0.0, 0.0, P->src_pos[k]};
    double n[3] = {0.0, 0.0, 1.0};
    double x = P->src_x[k];
    double t = 0.0;
    if (P->src_t) t = P->src_t[2 * k] + (P->src_t[2 * k + 1] - P->src_t[2 * k]) * ru(&r);
    int left_inner = 0;
    if (mc) iso_dir(&r, n);
    uint64_t steps = 0, mcsteps = 0;
    double L = 0.0;                 /* -ln(weight) with continuous dust weights */
    for (;;) {
        if (steps >= max_steps) { R->capped++; break; }
        ++steps;
        if (!mc) {
            s = c * nb + j;
            double best = INFINITY;
            int ev = -1;
            for (int f = 0; f < 2; ++f) {
                double rt = P->rate_face[s * 2 + f];
                if (rt > 0.0) { double l = -log(ru(&r)) / rt; if (l < best) { best = l; ev = f; } }
            }
            if (P->rate_dn[s] > 0.0) { double l = -log(ru(&r)) / P->rate_dn[s]; if (l < best) { best = l; ev = 2; } }
            if (P->rate_up[s] > 0.0) { double l = -log(ru(&r)) / P->rate_up[s]; if (l < best) { best = l; ev = 3; } }
            const double ka = P->k_abs ? P->k_abs[c] : 0.0;
            if (ka > 0.0 && !P->dust_weight) {
                double l = -log(ru(&r)) / ka;
                if (l < best) { best = l; ev = 4; }
            }
            const double L_prev = L;
            census_add(P, R, s, t, t + best, L, ka);
            const double t_prev = t;
            t += best;
            if (ev == 4) { R->absorbed++; break; }   /* removed by dust after that residence */
            if (P->dust_weight) {
                L += ka * best;
                if (L > -log(1e-10)) { R->absorbed++; break; }   /* negligible weight: dropped */
            }
            if (ev >= 2) {
                j += (ev == 2) ? -1 : 1;
                if (!P->thick[c * nb + j]) {   /* frequency leak into a thin bin */
                    cell_point(P, c, &r, pos);
                    iso_dir(&r, n);
                    left_inner = 0;
                    x = P->edges[j] + (P->edges[j + 1] - P->edges[j]) * ru(&r);
                    mc = 1;
                    R->to_mc++;
                }
                continue;
            }
            int f = ev;
            int64_t nc = P->nbr[c * 2 + f];
            const double dir = f ? 1.0 : -1.0;
            accel_add(P, R, c, t_prev, t, dir * P->k[s], L_prev, ka);   /* outward leakage from c */
            double xin = P->edges[j] + (P->edges[j + 1] - P->edges[j]) * ru(&r);
            if (P->face_mc[s * 2 + f] || nc < 0) {
                /* interface leak: MC at a uniform point of the face, isotropic outward */
                double N[3];
                face_point(P, c, f, &r, pos);
                face_normal(P, f, pos, N);
                hemi_about(&r, N, n);
                double nu = n_dot_u(P, c, pos, n);
                if (nc < 0) { tally_escape(R, P, f, xin + nu, t, L); break; }
                x = (xin + nu) * sqrt(P->T[c] / P->T[nc]) - n_dot_u(P, nc, pos, n);
                c = nc;
                left_inner = f == 1;
                mc = 1;
                R->to_mc++;
                continue;
            }
            double rho = P->rho[c * 2 + f], sh = P->shift[c * 2 + f];
            double xsh = rho * xin + sh;
            if (rho != 1.0 || sh != 0.0) {
                int jn = locate(P->edges, nb, xsh);
                j = jn < 0 ? 0 : (jn > nb - 1 ? nb - 1 : jn);
            }
            c = nc;
            if (P->thick[c * nb + j]) accel_add(P, R, c, t_prev, t, dir * P->k[c * nb + j], L_prev, ka);   /* inward */
            if (!P->thick[c * nb + j]) {   /* re-binned into a thin state */
                cell_point(P, c, &r, pos);
                iso_dir(&r, n);
                left_inner = 0;
                x = xsh;
                mc = 1;
                R->to_mc++;
            }
            continue;
        }
        /* ---- continuous MC ---- */
        ++mcsteps;
        int fexit;
        double dwall = wall_distance(P, c, pos, n, left_inner, &fexit);
        double kl = P->group ? P->k[c * nb + j] : P->k0[c] * mc_voigt(P->a[c], x);
        double ka = P->k_abs ? P->k_abs[c] : 0.0, ks = P->k_sca ? P->k_sca[c] : 0.0;
        double ka_ev = P->dust_weight ? 0.0 : ka;     /* absorption as an interaction, or as weight decay */
        double kx = kl + ks + ka_ev;
        double ds = -log(ru(&r)) / kx;
        double p0[3] = {pos[0], pos[1], pos[2]};
        double u0 = n_dot_u(P, c, p0, n);
        census_add(P, R, P->group ? c * nb + j : mc_state(P, c, x), t, t + fmin(ds, dwall), L, ka);
        if (P->dust_weight) {
            L += ka * fmin(ds, dwall);
            if (L > -log(1e-10)) { R->absorbed++; break; }
        }
        if (ds < dwall) {
            for (int d = 0; d < 3; ++d) pos[d] += ds * n[d];
            t += ds;
            x += u0 - n_dot_u(P, c, pos, n);
            if (ka_ev > 0.0 || ks > 0.0) {   /* which opacity interacted */
                double uu2 = ru(&r) * kx;
                if (uu2 < ka_ev) { R->absorbed++; break; }
                if (uu2 < ka_ev + ks) { iso_dir(&r, n); left_inner = 0; continue; }   /* dust: coherent, isotropic */
            }
            if (P->group) {   /* eq. 42: the outgoing bin of a scattering of a bin-j packet */
                double xg = P->edges[j] + (P->edges[j + 1] - P->edges[j]) * ru(&r);
                double nd[3] = {n[0], n[1], n[2]};
                int jg = locate(P->edges, nb, scatter(P->a[c], xg, nd, &r, 0.0));
                j = jg < 0 ? 0 : (jg > nb - 1 ? nb - 1 : jg);
                iso_dir(&r, n);
                left_inner = 0;
                if (P->thick[c * nb + j]) { mc = 0; R->to_ddmc++; }
                continue;
            }
            x = scatter(P->a[c], x, n, &r, P->x_crit);
            left_inner = 0;
            int jj = locate(P->edges, nb, x);
            if (jj >= 0 && jj < nb && P->thick[c * nb + jj]) { j = jj; mc = 0; R->to_ddmc++; }
            continue;
        }
        for (int d = 0; d < 3; ++d) pos[d] += dwall * n[d];
        t += dwall;
        int f = fexit;
        if (P->geometry == 0) {
            pos[2] = P->faces[c + f];
        } else {   /* put the point exactly on its sphere */
            double e[3];
            radial(pos, e);
            for (int d = 0; d < 3; ++d) pos[d] = P->faces[c + f] * e[d];
        }
        double nu = n_dot_u(P, c, pos, n);
        x += u0 - nu;                                   /* comoving x at the wall */
        int64_t nc = P->nbr[c * 2 + f];
        if (nc == -2) continue;                         /* no face (r = 0): cannot occur */
        if (nc < 0) {
            tally_escape(R, P, f, P->group ? 0.5 * (P->edges[j] + P->edges[j + 1]) : x + nu, t, L);
            break;
        }
        double xn = (x + nu) * sqrt(P->T[c] / P->T[nc]) - n_dot_u(P, nc, pos, n);
        int jn = P->group ? j : locate(P->edges, nb, xn);
        if (jn >= 0 && jn < nb && P->thick[nc * nb + jn]) {
            double N[3];
            face_normal(P, f, pos, N);
            double wn = P->faces[nc + 1] - P->faces[nc];
            double mu = fabs(dot(n, N));
            double Pacc = 2.0 / (P->k[nc * nb + jn] * wn + 2.0 * P->lambda) * (2.0 / 3.0 + mu);
            if (ru(&r) < Pacc) { c = nc; j = jn; mc = 0; R->to_ddmc++; continue; }
            /* reflected into c: uniform point of the interface, isotropic inward direction;
             * x unchanged at the new point */
            double Nin[3];
            face_point(P, c, f, &r, pos);
            face_normal(P, f, pos, N);
            Nin[0] = -N[0]; Nin[1] = -N[1]; Nin[2] = -N[2];
            hemi_about(&r, Nin, n);
            left_inner = f == 0;
            R->reflected++;
            continue;
        }
        c = nc;
        left_inner = f == 1;
        x = xn;
    }
    R->steps_sum += (double)steps;
    R->mc_steps_sum += (double)mcsteps;
    R->steps2_sum += (double)steps * (double)steps;
    R->step_hist[step_bin(steps ? steps : 1)]++;
}

static void *worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const oh_problem *P = jb->p;
    oh_result L;
    memset(&L, 0, sizeof L);
    size_t rows = P->geometry == 0 ? 2 : 1;
    size_t ns = rows * (size_t)(P->nb + 2);
    L.spectrum = calloc(ns, 8);
    L.time_hist = calloc(OH_TIME_BINS + 2, 8);
    L.step_hist = calloc(OH_STEP_BINS, 8);
    size_t nst = (size_t)P->nc * P->nb;
    size_t nbin = P->n_census > 0 ? (size_t)(P->n_census + 1) * nst : 0;
    size_t npath = P->n_census > 0 ? (size_t)P->n_census * nst : 0;
    L.e_bin = nbin ? calloc(nbin, 8) : NULL;
    L.e_path = npath ? calloc(npath, 8) : NULL;
    size_t nacc = P->n_census > 0 ? (size_t)P->n_census * P->nc : 0;
    L.e_accel = nacc ? calloc(nacc, 8) : NULL;
    L.wspec = P->dust_weight ? calloc(ns, 8) : NULL;
    L.wspec2 = P->dust_weight ? calloc(ns, 8) : NULL;
    for (;;) {
        uint64_t b = __sync_fetch_and_add(jb->next, jb->grain);
        if (b >= jb->n) break;
        uint64_t e = b + jb->grain < jb->n ? b + jb->grain : jb->n;
        for (uint64_t i = b; i < e; ++i) walk_packet(P, jb->first + i, jb->seed, jb->max_steps, &L);
    }
    pthread_mutex_lock(jb->lock);
    oh_result *R = jb->out;
    for (size_t i = 0; i < ns; ++i) R->spectrum[i] += L.spectrum[i];
    for (int i = 0; i < OH_TIME_BINS + 2; ++i) R->time_hist[i] += L.time_hist[i];
    for (int i = 0; i < OH_STEP_BINS; ++i) R->step_hist[i] += L.step_hist[i];
    R->t_sum += L.t_sum; R->t2_sum += L.t2_sum; R->steps_sum += L.steps_sum; R->mc_steps_sum += L.mc_steps_sum;
    R->steps2_sum += L.steps2_sum;
    R->escaped += L.escaped; R->capped += L.capped; R->to_mc += L.to_mc; R->to_ddmc += L.to_ddmc;
    R->reflected += L.reflected;
    R->absorbed += L.absorbed;
    for (size_t i = 0; i < nbin; ++i) R->e_bin[i] += L.e_bin[i];
    for (size_t i = 0; i < npath; ++i) R->e_path[i] += L.e_path[i];
    for (size_t i = 0; i < nacc; ++i) R->e_accel[i] += L.e_accel[i];
    if (P->dust_weight) {
        for (size_t i = 0; i < ns; ++i) { R->wspec[i] += L.wspec[i]; R->wspec2[i] += L.wspec2[i]; }
        R->w_sum += L.w_sum; R->wt_sum += L.wt_sum; R->wt2_sum += L.wt2_sum;
    }
    pthread_mutex_unlock(jb->lock);
    free(L.spectrum); free(L.time_hist); free(L.step_hist); free(L.e_bin); free(L.e_path); free(L.e_accel);
    free(L.wspec); free(L.wspec2);
    return NULL;
}

int oh_run(const oh_problem *p, uint64_t first, uint64_t n, uint64_t seed, uint64_t max_steps, int threads,
           oh_result *out)
{
    if (!p || !out || threads < 1) return -1;
    volatile uint64_t next = 0;
    pthread_mutex_t lock;
    pthread_mutex_init(&lock, NULL);
    /* small runs (few, long packets) hand out one packet at a time */
    job_t jb = {p, first, n, seed, max_steps, &next, &lock, out, n >= 64 * (uint64_t)threads ? 8u : 1u};
    pthread_t *th = malloc(sizeof(pthread_t) * threads);
    for (int i = 0; i < threads; ++i) pthread_create(&th[i], NULL, worker, &jb);
    for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&lock);
    return 0;
}
