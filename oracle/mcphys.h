/* Continuous-MC physics shared by the oracle walkers (walk3d.c, walk1dh.c) -- ORACLE,
 * TEST INFRASTRUCTURE ONLY.  Plain C, FP64; nothing here is shared with the GPU library.
 *
 *   - RNG: xoshiro256** (Blackman & Vigna 2018) seeded by splitmix64, from their published
 *     definitions;
 *   - the line profile H(a, x) of eq. 12 with Dawson's integral from its power series
 *     (|x| < 6) and its asymptotic series beyond;
 *   - the atom velocity along the photon, density ~ exp(-u^2) / (a^2 + (x - u)^2), by
 *     rejection from a split Lorentzian (the method of Zheng & Miralda-Escude 2002);
 *   - one scattering: eq. 41 with no recoil, isotropic phase function, optional
 *     core-skipping (x_crit; off when <= 0).
 */
#ifndef ORACLE_MCPHYS_H
#define ORACLE_MCPHYS_H

#include <math.h>
#include <stdint.h>

/* ---- RNG ------------------------------------------------------------------------- */
static inline uint64_t sm64(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
typedef struct { uint64_t s[4]; } rng_t;
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rnext(rng_t *r)
{
    uint64_t *s = r->s;
    const uint64_t res = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]; s[2] ^= t; s[3] = rotl(s[3], 45);
    return res;
}
static inline double ru(rng_t *r) { return ((double)(rnext(r) >> 11) + 0.5) * 0x1.0p-53; }

/* ---- line physics ---------------------------------------------------------------- */
static double mc_dawson(double x)
{
    double ax = fabs(x), sg = x < 0 ? -1.0 : 1.0;
    if (ax < 6.0) {
        double x2 = ax * ax, term = ax, sum = ax;     /* term_n = x^(2n+1)/n! */
        for (int n = 1; n < 200; ++n) {
            term *= x2 / n;
            double add = term / (2 * n + 1);
            sum += add;
            if (add < 1e-18 * sum) break;
        }
        return sg * exp(-x2) * sum;
    }
    double q = 1.0 / (2.0 * ax * ax), term = 1.0, sum = 1.0;
    for (int k = 1; k < 60; ++k) {
        double nt = term * (2 * k - 1) * q;
        if (nt > term) break;                         /* optimal truncation */
        term = nt;
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sg * sum / (2.0 * ax);
}

static double mc_voigt(double a, double x)
{
    double e = exp(-x * x);
    return e + 2.0 * a / sqrt(M_PI) * (2.0 * x * mc_dawson(x) - 1.0) + a * a * e * (1.0 - 2.0 * x * x);
}

/* Atom velocity along the photon direction: density ~ exp(-u^2) / (a^2 + (x-u)^2).
 * Rejection with a Lorentzian proposal split at u0 >= 0 (Zheng & Miralda-Escude 2002):
 * below u0 the proposal is the Lorentzian and the acceptance exp(-u^2); above u0 the
 * proposal is the Lorentzian times exp(-u0^2) and the acceptance exp(u0^2 - u^2).  Works
 * on |x| and mirrors the result. */
/* proposal mass (times a) of the split at u0: Lorentzian mass below u0 plus
 * exp(-u0^2) times the Lorentzian mass above it */
static double split_mass(double a, double ax, double u0)
{
    double th = atan((u0 - ax) / a);
    return (M_PI / 2 + th) + exp(-u0 * u0) * (M_PI / 2 - th);
}

/* any u0 >= 0 gives an exact sampler; take the one minimising the proposal mass
 * (golden-section search on [0, |x|]) so that the acceptance rate stays high */
static double mc_split_point(double a, double ax)
{
    double lo = 0.0, hi = ax;
    const double g = 0.6180339887498949;
    double c1 = hi - g * (hi - lo), c2 = lo + g * (hi - lo);
    double f1 = split_mass(a, ax, c1), f2 = split_mass(a, ax, c2);
    for (int it = 0; it < 40; ++it) {
        if (f1 < f2) { hi = c2; c2 = c1; f2 = f1; c1 = hi - g * (hi - lo); f1 = split_mass(a, ax, c1); }
        else { lo = c1; c1 = c2; f1 = f2; c2 = lo + g * (hi - lo); f2 = split_mass(a, ax, c2); }
    }
    return 0.5 * (lo + hi);
}

static double mc_sample_upar(double a, double x, rng_t *r)
{
    double sg = x < 0 ? -1.0 : 1.0, ax = fabs(x);
    double u0 = mc_split_point(a, ax);
    double th0 = atan((u0 - ax) / a), e0 = exp(-u0 * u0);
    double p = (th0 + M_PI / 2) / ((1.0 - e0) * th0 + (1.0 + e0) * M_PI / 2);
    for (;;) {
        double th, uu;
        if (ru(r) <= p) {
            th = -M_PI / 2 + (th0 + M_PI / 2) * ru(r);
            uu = a * tan(th) + ax;
            if (ru(r) <= exp(-uu * uu)) return sg * uu;
        } else {
            th = th0 + (M_PI / 2 - th0) * ru(r);
            uu = a * tan(th) + ax;
            if (ru(r) <= exp(u0 * u0 - uu * uu)) return sg * uu;
        }
    }
}

static void iso_dir(rng_t *r, double n[3])
{
    double mu = 2.0 * ru(r) - 1.0, ph = 2.0 * M_PI * ru(r), s = sqrt(fmax(0.0, 1.0 - mu * mu));
    n[0] = s * cos(ph); n[1] = s * sin(ph); n[2] = mu;
}

/* One scattering (the hybrid section's MC step, eq. 41 with g = 0): the atom's velocity
 * along the incoming direction n from mc_sample_upar, one perpendicular component, an
 * isotropic new direction written back into n; returns the new comoving x. */
static double scatter(double a, double x, double n[3], rng_t *r, double x_crit)
{
    double upar = mc_sample_upar(a, x, r);
    /* the perpendicular velocity in the scattering plane: a N(0, 1/2) component, i.e. the
     * projection of a 2D Maxwellian speed sqrt(-ln xi1) on a uniform azimuth; with
     * core-skipping, photons in the core (|x| < x_crit) take the speed from the tail
     * above x_crit, sqrt(x_crit^2 - ln xi1) */
    double xc = (x_crit > 0.0 && fabs(x) < x_crit) ? x_crit : 0.0;
    double uperp = sqrt(xc * xc - log(ru(r))) * cos(2.0 * M_PI * ru(r));
    double n2[3];
    iso_dir(r, n2);
    double mu = n[0] * n2[0] + n[1] * n2[1] + n[2] * n2[2];
    double xo = x + upar * (mu - 1.0) + uperp * sqrt(fmax(0.0, 1.0 - mu * mu));
    n[0] = n2[0]; n[1] = n2[1]; n[2] = n2[2];
    return xo;
}

#endif
