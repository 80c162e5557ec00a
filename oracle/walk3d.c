/* O1-3D: literal FP64 hybrid DDMC / continuous-MC walker on a 3D Cartesian grid --
 * ORACLE, TEST INFRASTRUCTURE ONLY.  Plain C; shares nothing with the GPU library.
 *
 * Follows the paper's Monte Carlo procedure and hybrid scheme as written:
 *  - DDMC states (tau_ij >= tau_th): every step draws dl_X = -ln(xi_X)/k_X for EVERY
 *    leak X (6 faces, eq. 10 or the thin/vacuum interface rate; 2 bins, eq. 11) and takes
 *    the smallest (eqs. 15-16);
 *      * a leak through a face whose neighbour is thick at the shifted bin moves the packet
 *        there and re-bins x (Sec. 2.5, eq. 20);
 *      * a leak through a face to a thin neighbour turns the packet into an MC packet at a
 *        random point of the interface with an isotropic outward direction (mu uniform
 *        in (0,1]), x uniform in the bin, shifted into the neighbour's frame with the exact
 *        comoving formula; through a vacuum face it escapes;
 *      * a frequency leak into a thin bin turns it into an MC packet at a uniform position
 *        in the cell with an isotropic direction and x uniform in the new bin.
 *  - MC packets (continuous position, direction, comoving frequency): distance to the cell
 *    boundary vs an exponential optical depth with k = k0 H(a,x) (eq. 12);
 *      * scattering: atom velocity u_par ~ exp(-u^2)/(a^2+(x-u)^2) by rejection (the method
 *        of Zheng & Miralda-Escude 2002), u_perp ~ N(0,1/2), isotropic new direction,
 *        x' = x + u_par (mu - 1) + u_perp sqrt(1-mu^2) (recoil g = 0); then if the
 *        state (cell, bin(x')) is thick the packet becomes DDMC there;
 *      * crossing a face: into vacuum -> escape with x_lab = x + n.u; into a cell at
 *        x' = (x + n.u) sqrt(T/T') - n.u' (exact comoving shift); if that state is thick the
 *        packet converts with P = 2/(k' w' + 2 lambda) (2/3 + mu) (mu the direction cosine
 *        to the interface), else it is reflected: random point on the interface, isotropic
 *        inward direction, x unchanged; if thin it continues as MC in the new cell.
 *  - Time advances by the path length (c = 1); escapes are tallied by face, lab bin,
 *    boundary cell (pixel) and time.
 *
 * H(a,x) uses the paper's expansion (eq. 12) with Dawson's integral computed here from its
 * power series int_0^x e^{t^2} dt = sum x^(2n+1)/(n! (2n+1)) (positive terms) times e^{-x^2}
 * for |x| < 6, and from its asymptotic series (1/2x) sum (2k-1)!!/(2x^2)^k beyond.
 *
 * Random numbers: xoshiro256** per packet seeded by splitmix64(seed ^ id*golden).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O3_TIME_BINS 128
#define O3_STEP_BINS 64

typedef struct {
    int32_t nx, ny, nz, nb;
    const double *fx, *fy, *fz;    /* face coordinates per axis (n+1) */
    const double *edges;           /* nb+1 */
    const double *k;               /* [nc*nb] bin-averaged opacity (eq. 14) */
    const uint8_t *thick;          /* [nc*nb] */
    const double *rate_face;       /* [nc*nb*6] */
    const uint8_t *face_mc;        /* [nc*nb*6] the leak through this face uses the interface rate */
    const double *rate_dn, *rate_up;  /* [nc*nb] */
    const double *rho, *shift;     /* [nc*6] DDMC re-binning map into the neighbour */
    const double *k0;              /* [nc] line-centre opacity */
    const double *a;               /* [nc] damping parameter */
    const double *T;               /* [nc] temperature */
    const double *u;               /* [nc*3] bulk velocity in units of the cell's v_th */
    double lambda;
    int32_t n_src;
    const int64_t *src_state;      /* [n_src] */
    const double *src_pos;         /* [n_src*3] */
    const double *src_x;           /* [n_src] */
    const double *src_cdf;         /* [n_src] */
    double x_crit;                 /* core-skipping threshold of the scattering (0 = off) */
} o3_problem;

typedef struct {
    int64_t *spectrum;     /* [6*(nb+2)] */
    int64_t *pixels;       /* [2*(ny*nz + nx*nz + nx*ny)] escape counts per boundary cell */
    int64_t *time_hist;    /* [O3_TIME_BINS+2] */
    int64_t *step_hist;    /* [O3_STEP_BINS] */
    double t_sum, t2_sum, steps_sum, mc_steps_sum;
    int64_t escaped, capped, to_mc, to_ddmc, reflected;
    double steps2_sum, mc_steps2_sum;
} o3_result;

#include "mcphys.h"

/* exported for the pins of the line physics */
double o3_dawson(double x) { return mc_dawson(x); }
double o3_voigt(double a, double x) { return mc_voigt(a, x); }

/* isotropic over the hemisphere around axis `ax` with sign `sg`: mu uniform in (0,1] */
static void hemi_dir(rng_t *r, int ax, double sg, double n[3])
{
    double mu = ru(r), ph = 2.0 * M_PI * ru(r), s = sqrt(fmax(0.0, 1.0 - mu * mu));
    double t1 = s * cos(ph), t2 = s * sin(ph);
    n[ax] = sg * mu;
    n[(ax + 1) % 3] = t1;
    n[(ax + 2) % 3] = t2;
}

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
    double u = (log10(t) + 3.0) / 9.0 * O3_TIME_BINS;
    if (u >= O3_TIME_BINS) return O3_TIME_BINS + 1;
    return 1 + (int)u;
}

static int step_bin(uint64_t n) { int b = 0; while (n > 1) { n >>= 1; ++b; } return b; }

typedef struct {
    const o3_problem *p;
    uint64_t first, n, seed, max_steps;
    volatile uint64_t *next;
    pthread_mutex_t *lock;
    o3_result *out;
} job_t;

/* geometry helpers */
static void cell_ijk(const o3_problem *p, int64_t c, int *ix, int *iy, int *iz)
{
    *ix = (int)(c % p->nx); *iy = (int)((c / p->nx) % p->ny); *iz = (int)(c / ((int64_t)p->nx * p->ny));
}
static int64_t nbr_of(const o3_problem *p, int64_t c, int f)
{
    int ix, iy, iz; cell_ijk(p, c, &ix, &iy, &iz);
    int d = f >> 1, up = f & 1;
    int idx[3] = {ix, iy, iz}, nn[3] = {p->nx, p->ny, p->nz};
    int64_t st[3] = {1, p->nx, (int64_t)p->nx * p->ny};
    if (up) return idx[d] < nn[d] - 1 ? c + st[d] : -1;
    return idx[d] > 0 ? c - st[d] : -1;
}
static const double *axis_faces(const o3_problem *p, int d) { return d == 0 ? p->fx : (d == 1 ? p->fy : p->fz); }
static int64_t pixel_of(const o3_problem *p, int64_t c, int f)
{   /* escape pixel index: per face, the boundary cell's two other coordinates */
    int i[3]; cell_ijk(p, c, &i[0], &i[1], &i[2]);
    int64_t off = 0;
    int64_t sz[3] = {(int64_t)p->ny * p->nz, (int64_t)p->nx * p->nz, (int64_t)p->nx * p->ny};
    for (int g = 0; g < f; ++g) off += sz[g >> 1];
    int d = f >> 1;
    if (d == 0) return off + (int64_t)i[2] * p->ny + i[1];
    if (d == 1) return off + (int64_t)i[2] * p->nx + i[0];
    return off + (int64_t)i[1] * p->nx + i[0];
}
static void random_point_on_face(const o3_problem *p, int64_t c, int f, rng_t *r, double pos[3])
{
    int i[3]; cell_ijk(p, c, &i[0], &i[1], &i[2]);
    for (int d = 0; d < 3; ++d) {
        const double *fa = axis_faces(p, d);
        if (d == (f >> 1)) pos[d] = (f & 1) ? fa[i[d] + 1] : fa[i[d]];
        else pos[d] = fa[i[d]] + (fa[i[d] + 1] - fa[i[d]]) * ru(r);
    }
}

static void tally_escape(o3_result *R, const o3_problem *p, int f, int64_t c, double xlab, double t)
{
    int nb = p->nb;
    int slot = locate(p->edges, nb, xlab) + 1;
    R->spectrum[(int64_t)f * (nb + 2) + slot]++;
    R->pixels[pixel_of(p, c, f)]++;
    R->escaped++;
    R->t_sum += t;
    R->t2_sum += t * t;
    R->time_hist[time_bin(t)]++;
}

static void walk_packet(const o3_problem *p, uint64_t id, uint64_t seed, uint64_t max_steps, o3_result *R)
{
    rng_t r;
    uint64_t xs = seed ^ (id * 0x9E3779B97F4A7C15ull);
    for (int i = 0; i < 4; ++i) r.s[i] = sm64(&xs);
    const int nb = p->nb;
    double uu = ru(&r);
    int k = 0;
    while (k < p->n_src - 1 && uu >= p->src_cdf[k]) ++k;
    int64_t s = p->src_state[k];
    int64_t c = s / nb;
    int j = (int)(s % nb);
    int mc = !p->thick[s];
    double pos[3] = {p->src_pos[3 * k], p->src_pos[3 * k + 1], p->src_pos[3 * k + 2]};
    double n[3];
    double x = p->src_x[k];
    if (mc) iso_dir(&r, n);
    double t = 0.0;
    uint64_t steps = 0, mcsteps = 0;
    for (;;) {
        if (steps >= max_steps) { R->capped++; break; }
        ++steps;
        if (!mc) {
            s = c * nb + j;
            double best = INFINITY;
            int ev = -1;
            for (int f = 0; f < 6; ++f) {
                double rt = p->rate_face[s * 6 + f];
                if (rt > 0.0) { double l = -log(ru(&r)) / rt; if (l < best) { best = l; ev = f; } }
            }
            if (p->rate_dn[s] > 0.0) { double l = -log(ru(&r)) / p->rate_dn[s]; if (l < best) { best = l; ev = 6; } }
            if (p->rate_up[s] > 0.0) { double l = -log(ru(&r)) / p->rate_up[s]; if (l < best) { best = l; ev = 7; } }
            t += best;
            if (ev >= 6) {
                j += (ev == 6) ? -1 : 1;
                if (!p->thick[c * nb + j]) {   /* frequency leak into a thin bin: MC in this cell */
                    int i3[3]; cell_ijk(p, c, &i3[0], &i3[1], &i3[2]);
                    for (int d = 0; d < 3; ++d) {
                        const double *fa = axis_faces(p, d);
                        pos[d] = fa[i3[d]] + (fa[i3[d] + 1] - fa[i3[d]]) * ru(&r);
                    }
                    iso_dir(&r, n);
                    x = p->edges[j] + (p->edges[j + 1] - p->edges[j]) * ru(&r);
                    mc = 1;
                    R->to_mc++;
                }
                continue;
            }
            int f = ev;
            int64_t nc = nbr_of(p, c, f);
            double xin = p->edges[j] + (p->edges[j + 1] - p->edges[j]) * ru(&r);
            if (p->face_mc[s * 6 + f] || nc < 0) {
                /* interface leak: MC at a random point of the face, isotropic outward */
                random_point_on_face(p, c, f, &r, pos);
                hemi_dir(&r, f >> 1, (f & 1) ? 1.0 : -1.0, n);
                double nu = n[0] * p->u[3 * c] + n[1] * p->u[3 * c + 1] + n[2] * p->u[3 * c + 2];
                if (nc < 0) { tally_escape(R, p, f, c, xin + nu, t); break; }
                double nu2 = n[0] * p->u[3 * nc] + n[1] * p->u[3 * nc + 1] + n[2] * p->u[3 * nc + 2];
                x = (xin + nu) * sqrt(p->T[c] / p->T[nc]) - nu2;
                c = nc;
                mc = 1;
                R->to_mc++;
                continue;
            }
            /* thick neighbour: re-bin the comoving frequency (eq. 20 averaged) */
            double rho = p->rho[c * 6 + f], sh = p->shift[c * 6 + f];
            double xs = rho * xin + sh;
            if (rho != 1.0 || sh != 0.0) {
                int jn = locate(p->edges, nb, xs);
                j = jn < 0 ? 0 : (jn > nb - 1 ? nb - 1 : jn);
            }
            c = nc;
            if (!p->thick[c * nb + j]) {
                /* the re-binned state itself is thin: continue as MC in the new cell at a
                 * uniform position, isotropic direction, with the shifted frequency */
                int i3[3]; cell_ijk(p, c, &i3[0], &i3[1], &i3[2]);
                for (int d = 0; d < 3; ++d) {
                    const double *fa = axis_faces(p, d);
                    pos[d] = fa[i3[d]] + (fa[i3[d] + 1] - fa[i3[d]]) * ru(&r);
                }
                iso_dir(&r, n);
                x = xs;
                mc = 1;
                R->to_mc++;
            }
            continue;
        }
        /* ---- continuous MC ---- */
        ++mcsteps;
        int i3[3]; cell_ijk(p, c, &i3[0], &i3[1], &i3[2]);
        double dface = INFINITY;
        int fexit = -1;
        for (int d = 0; d < 3; ++d) {
            if (n[d] == 0.0) continue;
            const double *fa = axis_faces(p, d);
            double wall = n[d] > 0 ? fa[i3[d] + 1] : fa[i3[d]];
            double dd = (wall - pos[d]) / n[d];
            if (dd < 0) dd = 0;
            if (dd < dface) { dface = dd; fexit = 2 * d + (n[d] > 0); }
        }
        double kx = p->k0[c] * mc_voigt(p->a[c], x);
        double ds = -log(ru(&r)) / kx;
        if (ds < dface) {
            for (int d = 0; d < 3; ++d) pos[d] += ds * n[d];
            t += ds;
            x = scatter(p->a[c], x, n, &r, p->x_crit);
            int jj = locate(p->edges, nb, x);
            if (jj >= 0 && jj < nb && p->thick[c * nb + jj]) { j = jj; mc = 0; R->to_ddmc++; }
            continue;
        }
        for (int d = 0; d < 3; ++d) pos[d] += dface * n[d];
        t += dface;
        int f = fexit;
        pos[f >> 1] = axis_faces(p, f >> 1)[i3[f >> 1] + (f & 1)];
        int64_t nc = nbr_of(p, c, f);
        double nu = n[0] * p->u[3 * c] + n[1] * p->u[3 * c + 1] + n[2] * p->u[3 * c + 2];
        if (nc < 0) { tally_escape(R, p, f, c, x + nu, t); break; }
        double nu2 = n[0] * p->u[3 * nc] + n[1] * p->u[3 * nc + 1] + n[2] * p->u[3 * nc + 2];
        double xn = (x + nu) * sqrt(p->T[c] / p->T[nc]) - nu2;
        int jn = locate(p->edges, nb, xn);
        if (jn >= 0 && jn < nb && p->thick[nc * nb + jn]) {
            /* eq. 39 with the neighbour's optical width across the interface (its width
             * along the crossing axis, as in the DDMC -> MC rate of the same face) */
            int in3[3]; cell_ijk(p, nc, &in3[0], &in3[1], &in3[2]);
            const double *fn = axis_faces(p, f >> 1);
            double wn = fn[in3[f >> 1] + 1] - fn[in3[f >> 1]];
            double mu = fabs(n[f >> 1]);
            double P = 2.0 / (p->k[nc * nb + jn] * wn + 2.0 * p->lambda) * (2.0 / 3.0 + mu);
            if (ru(&r) < P) { c = nc; j = jn; mc = 0; R->to_ddmc++; continue; }
            /* reflect into c: random point of the interface, isotropic inward */
            random_point_on_face(p, c, f, &r, pos);
            hemi_dir(&r, f >> 1, (f & 1) ? -1.0 : 1.0, n);
            R->reflected++;
            continue;
        }
        c = nc;
        x = xn;
    }
    R->steps_sum += (double)steps;
    R->mc_steps_sum += (double)mcsteps;
    R->steps2_sum += (double)steps * (double)steps;
    R->mc_steps2_sum += (double)mcsteps * (double)mcsteps;
    R->step_hist[step_bin(steps ? steps : 1)]++;
}

static void *worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const o3_problem *p = jb->p;
    o3_result L;
    memset(&L, 0, sizeof L);
    size_t ns = 6 * (size_t)(p->nb + 2);
    size_t np = 2 * ((size_t)p->ny * p->nz + (size_t)p->nx * p->nz + (size_t)p->nx * p->ny);
    L.spectrum = calloc(ns, 8);
    L.pixels = calloc(np, 8);
    L.time_hist = calloc(O3_TIME_BINS + 2, 8);
    L.step_hist = calloc(O3_STEP_BINS, 8);
    for (;;) {
        uint64_t b = __sync_fetch_and_add(jb->next, 8);
        if (b >= jb->n) break;
        uint64_t e = b + 8 < jb->n ? b + 8 : jb->n;
        for (uint64_t i = b; i < e; ++i) walk_packet(p, jb->first + i, jb->seed, jb->max_steps, &L);
    }
    pthread_mutex_lock(jb->lock);
    o3_result *R = jb->out;
    for (size_t i = 0; i < ns; ++i) R->spectrum[i] += L.spectrum[i];
    for (size_t i = 0; i < np; ++i) R->pixels[i] += L.pixels[i];
    for (int i = 0; i < O3_TIME_BINS + 2; ++i) R->time_hist[i] += L.time_hist[i];
    for (int i = 0; i < O3_STEP_BINS; ++i) R->step_hist[i] += L.step_hist[i];
    R->t_sum += L.t_sum; R->t2_sum += L.t2_sum; R->steps_sum += L.steps_sum; R->mc_steps_sum += L.mc_steps_sum;
    R->escaped += L.escaped; R->capped += L.capped; R->to_mc += L.to_mc; R->to_ddmc += L.to_ddmc;
    R->reflected += L.reflected;
    R->steps2_sum += L.steps2_sum; R->mc_steps2_sum += L.mc_steps2_sum;
    pthread_mutex_unlock(jb->lock);
    free(L.spectrum); free(L.pixels); free(L.time_hist); free(L.step_hist);
    return NULL;
}

int o3_run(const o3_problem *p, uint64_t first, uint64_t n, uint64_t seed, uint64_t max_steps, int threads,
           o3_result *out)
{
    if (!p || !out || threads < 1) return -1;
    volatile uint64_t next = 0;
    pthread_mutex_t lock;
    pthread_mutex_init(&lock, NULL);
    job_t jb = {p, first, n, seed, max_steps, &next, &lock, out};
    pthread_t *th = malloc(sizeof(pthread_t) * threads);
    for (int i = 0; i < threads; ++i) pthread_create(&th[i], NULL, worker, &jb);
    for (int i = 0; i < threads; ++i) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&lock);
    return 0;
}

/* test hook: n samples of the atom-velocity sampler */
void o3_upar_samples(double a, double x, uint64_t seed, int64_t n, double *out)
{
    rng_t r;
    uint64_t xs = seed;
    for (int i = 0; i < 4; ++i) r.s[i] = sm64(&xs);
    for (int64_t i = 0; i < n; ++i) out[i] = mc_sample_upar(a, x, &r);
}

/* test hook: outgoing frequencies of n scatterings of a photon absorbed at x, each from a
 * fresh incoming direction along +z, through the walk's own scattering routine */
void o3_redistribution_samples(double a, double x, double x_crit, uint64_t seed, int64_t n, double *out)
{
    rng_t r;
    uint64_t xs = seed;
    for (int i = 0; i < 4; ++i) r.s[i] = sm64(&xs);
    for (int64_t i = 0; i < n; ++i) {
        double dir[3] = {0.0, 0.0, 1.0};
        out[i] = scatter(a, x, dir, &r, x_crit);
    }
}
