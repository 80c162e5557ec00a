/* O1: literal FP64 Monte Carlo walker for rDDMC -- ORACLE, TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, no GPU code, shares nothing with the library.  It follows the
 * paper's Monte Carlo procedure (Sec. 2.3) as written:
 *   - a packet is tracked by its cell and frequency bin;
 *   - at every step an exponential distance  dl_X = -ln(xi_X) / k_X  is drawn
 *     for EVERY possible leakage X (each face neighbour, eq. 10 or the
 *     thin/vacuum-face rate of the hybrid section, and each frequency
 *     neighbour, eq. 11) and the smallest one is executed (eqs. 15-16);
 *   - time advances by dl / c (c = 1);
 *   - a leak through a vacuum face removes the packet (Sec. 2.3) and its
 *     escape frequency, face and time are tallied;
 *   - with bulk velocity, a leak into a neighbour draws x uniformly in the
 *     bin, shifts it into the neighbour's frame, x' = rho x + shift (Sec. 2.5,
 *     eq. 20), and re-bins it (clamped to the grid's first/last bin); an
 *     escaping packet's lab frequency is x + mu u_n with mu uniform in (0, 1].
 *
 * Random numbers: one xoshiro256** stream per packet (Blackman & Vigna 2018),
 * its 256-bit state filled by splitmix64 (Steele, Lea & Flood 2014) started
 * at seed ^ (packet_id * 0x9E3779B97F4A7C15).  Both written here from their
 * published definitions.
 *
 * Threads: POSIX threads pull packet ids from a shared counter; every tally
 * except the FP64 moment sums is an exact integer, independent of threading.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O1_TIME_BINS 128
#define O1_STEP_BINS 64

typedef struct {
    int32_t nc, nb, nf, moving;
    const double *rate_face;   /* [nc*nb*nf] */
    const double *rate_dn;     /* [nc*nb] */
    const double *rate_up;     /* [nc*nb] */
    const int64_t *nbr;        /* [nc*nf]: >=0 neighbour cell, -1 vacuum, -2 no face */
    const double *rho;         /* [nc*nf] */
    const double *shift;       /* [nc*nf] */
    const double *u_n;         /* [nc*nf] outward normal velocity in thermal units */
    const double *edges;       /* [nb+1] */
    int32_t n_src;
    const int64_t *src_state;  /* [n_src] */
    const double *src_cdf;     /* [n_src] cumulative probabilities, last = 1 */
    int32_t n_rows;            /* number of escape-face rows in the spectrum */
    const int32_t *face_row;   /* [nf]: row of the spectrum for each face, -1 if none */
} o1_problem;

typedef struct {
    int64_t *spectrum;         /* [n_rows*(nb+2)] escape counts per face row and lab slot */
    int64_t *time_hist;        /* [O1_TIME_BINS+2] log10 bins over [1e-3, 1e6] + under/over */
    int64_t *step_hist;        /* [O1_STEP_BINS] floor(log2(steps)) buckets */
    double t_sum, t2_sum, steps_sum, steps2_sum;
    int64_t escaped, capped;
    uint64_t steps_max;
} o1_result;

/* ---- splitmix64 / xoshiro256** ---------------------------------------------------- */
static inline uint64_t sm64_next(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xo_state;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t xo_next(xo_state *st)
{
    uint64_t *s = st->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

static inline void xo_seed(xo_state *st, uint64_t seed, uint64_t id)
{
    uint64_t x = seed ^ (id * 0x9E3779B97F4A7C15ull);
    for (int i = 0; i < 4; ++i) st->s[i] = sm64_next(&x);
}

/* uniform in the open interval (0, 1) with 53 random bits */
static inline double xo_open01(xo_state *st)
{
    return ((double)(xo_next(st) >> 11) + 0.5) * 0x1.0p-53;
}

/* ---- helpers --------------------------------------------------------------------- */
static int locate(const double *e, int nb, double x)
{   /* bin j with e[j] <= x < e[j+1]; -1 below, nb at or above the top edge */
    if (x < e[0]) return -1;
    if (x >= e[nb]) return nb;
    int lo = 0, hi = nb;   /* e[lo] <= x < e[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (x >= e[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

static int time_bin(double t)
{
    if (!(t >= 1e-3)) return 0;
    double u = (log10(t) + 3.0) / 9.0 * O1_TIME_BINS;
    if (u >= O1_TIME_BINS) return O1_TIME_BINS + 1;
    return 1 + (int)u;
}

static int step_bin(uint64_t n)
{
    int b = 0;
    while (n > 1) { n >>= 1; ++b; }
    return b;
}

typedef struct {
    const o1_problem *p;
    uint64_t first_id, n_packets, seed, max_steps;
    volatile uint64_t *next;
    pthread_mutex_t *lock;
    o1_result *out;
} o1_job;

static void walk_one(const o1_problem *p, uint64_t id, uint64_t seed, uint64_t max_steps,
                     o1_result *r)
{
    xo_state rng;
    xo_seed(&rng, seed, id);
    const int nb = p->nb, nf = p->nf;
    /* emission: choose a source state by its probability */
    double u = xo_open01(&rng);
    int k = 0;
    while (k < p->n_src - 1 && u >= p->src_cdf[k]) ++k;
    int64_t s = p->src_state[k];
    double t = 0.0;
    uint64_t steps = 0;
    for (;;) {
        if (steps >= max_steps) {
            r->capped++;
            break;
        }
        const int64_t c = s / nb;
        const int j = (int)(s % nb);
        double best = INFINITY;
        int ev = -1;
        for (int f = 0; f < nf; ++f) {
            double rate = p->rate_face[s * nf + f];
            if (rate > 0.0) {
                double l = -log(xo_open01(&rng)) / rate;
                if (l < best) { best = l; ev = f; }
            }
        }
        if (p->rate_dn[s] > 0.0) {
            double l = -log(xo_open01(&rng)) / p->rate_dn[s];
            if (l < best) { best = l; ev = nf; }
        }
        if (p->rate_up[s] > 0.0) {
            double l = -log(xo_open01(&rng)) / p->rate_up[s];
            if (l < best) { best = l; ev = nf + 1; }
        }
        t += best;
        ++steps;
        if (ev == nf) { s -= 1; continue; }
        if (ev == nf + 1) { s += 1; continue; }
        /* spatial leak through face ev */
        const int64_t n = p->nbr[c * nf + ev];
        const double lo = p->edges[j], hi = p->edges[j + 1];
        if (n < 0) {   /* vacuum: escape */
            int slot = j + 1;
            double un = p->moving ? p->u_n[c * nf + ev] : 0.0;
            if (un != 0.0) {
                double x = lo + (hi - lo) * xo_open01(&rng);
                double mu = xo_open01(&rng);   /* outward direction cosine, uniform */
                double xl = x + mu * un;
                slot = locate(p->edges, nb, xl) + 1;
            }
            int row = p->face_row[ev];
            r->spectrum[(int64_t)row * (nb + 2) + slot]++;
            r->escaped++;
            r->t_sum += t;
            r->t2_sum += t * t;
            r->time_hist[time_bin(t)]++;
            break;
        }
        int jn = j;
        if (p->moving) {
            double rho = p->rho[c * nf + ev], sh = p->shift[c * nf + ev];
            if (rho != 1.0 || sh != 0.0) {
                double x = lo + (hi - lo) * xo_open01(&rng);
                jn = locate(p->edges, nb, rho * x + sh);
                if (jn < 0) jn = 0;
                if (jn > nb - 1) jn = nb - 1;
            }
        }
        s = n * nb + jn;
    }
    r->steps_sum += (double)steps;
    r->steps2_sum += (double)steps * (double)steps;
    if (steps > r->steps_max) r->steps_max = steps;
    r->step_hist[step_bin(steps ? steps : 1)]++;
}

static void *worker(void *arg)
{
    o1_job *jb = (o1_job *)arg;
    const o1_problem *p = jb->p;
    const int nb = p->nb;
    o1_result loc;
    memset(&loc, 0, sizeof loc);
    size_t nspec = (size_t)p->n_rows * (nb + 2);
    loc.spectrum = (int64_t *)calloc(nspec, sizeof(int64_t));
    loc.time_hist = (int64_t *)calloc(O1_TIME_BINS + 2, sizeof(int64_t));
    loc.step_hist = (int64_t *)calloc(O1_STEP_BINS, sizeof(int64_t));
    const uint64_t chunk = 16;
    for (;;) {
        uint64_t b = __sync_fetch_and_add(jb->next, chunk);
        if (b >= jb->n_packets) break;
        uint64_t e = b + chunk < jb->n_packets ? b + chunk : jb->n_packets;
        for (uint64_t i = b; i < e; ++i)
            walk_one(p, jb->first_id + i, jb->seed, jb->max_steps, &loc);
    }
    pthread_mutex_lock(jb->lock);
    o1_result *r = jb->out;
    for (size_t i = 0; i < nspec; ++i) r->spectrum[i] += loc.spectrum[i];
    for (int i = 0; i < O1_TIME_BINS + 2; ++i) r->time_hist[i] += loc.time_hist[i];
    for (int i = 0; i < O1_STEP_BINS; ++i) r->step_hist[i] += loc.step_hist[i];
    r->t_sum += loc.t_sum;
    r->t2_sum += loc.t2_sum;
    r->steps_sum += loc.steps_sum;
    r->steps2_sum += loc.steps2_sum;
    r->escaped += loc.escaped;
    r->capped += loc.capped;
    if (loc.steps_max > r->steps_max) r->steps_max = loc.steps_max;
    pthread_mutex_unlock(jb->lock);
    free(loc.spectrum);
    free(loc.time_hist);
    free(loc.step_hist);
    return NULL;
}

/* Walk packets first_id .. first_id + n_packets - 1.  ``out`` arrays must be zeroed
 * by the caller.  Returns 0, or -1 on a bad argument. */
int o1_run(const o1_problem *p, uint64_t first_id, uint64_t n_packets, uint64_t seed,
           uint64_t max_steps, int n_threads, o1_result *out)
{
    if (!p || !out || p->nb < 1 || p->nc < 1 || p->n_src < 1 || n_threads < 1) return -1;
    volatile uint64_t next = 0;
    pthread_mutex_t lock;
    pthread_mutex_init(&lock, NULL);
    o1_job jb = {p, first_id, n_packets, seed, max_steps, &next, &lock, out};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, worker, &jb);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&lock);
    return 0;
}
