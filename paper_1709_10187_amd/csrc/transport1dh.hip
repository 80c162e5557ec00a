// Hybrid rDDMC walk on 1D grids (slab cells along z, or spherical shells): DDMC steps in
// thick states (Sec. 2.3, eqs. 15-16; the Doppler re-binning of Sec. 2.5) and continuous
// Monte Carlo in thin ones (the hybrid section: interface leaks, conversions both ways, the
// eq. 39 acceptance; the MC step with the Voigt opacity of eq. 12 and the redistribution of
// eq. 41, optionally with core-skipping).
//
// One lane carries one packet.  MC packets have a full 3D position and direction; the grid
// enters through its boundaries (planes z = z_f, or spheres r = r_f), their outward normals
// (+-z, or +-r^) and the bulk velocity (u along +z in a slab cell; u r^ in a shell, so its
// direction changes with position).  Per step:
//   DDMC state: the 16-byte hot record {ln2/K, D_hi, S_hi, flags} as on 3D grids; a spatial
//     leak picks face 0 or 1 from the state's 31-bit split; the flags say whether bin j-1 / j+1
//     is thin and whether a face leads into a thin state or vacuum.  Conversions: into a thin
//     bin, a uniform point of the cell (uniform in volume), isotropic, x uniform in the bin;
//     through an interface face, a uniform point of the face, mu uniform in (0, 1] about its
//     outward normal, x uniform in the bin moved to the neighbour's frame,
//     x' = (x + n.u) sqrt(T/T') - n.u' (both velocities at that point), or escape with the lab
//     frequency x + n.u through vacuum; a re-binning into a thin state, MC in the new cell at
//     a uniform point, isotropic, with the shifted x.
//   MC state: distance to the cell boundary along n (planes, or the quadratic for spheres,
//     in FP64) against an exponential optical depth at opacity k0 H(a, x); the comoving x is
//     that of the packet's current point (in a shell it changes by n.(u(p0) - u(p1)) over a
//     flight, the lab frequency being constant), and a flight's opacity is that of its
//     starting x.  Scattering and wall crossings as on 3D grids, with the neighbour's width
//     across the interface in eq. 39.
// Dust (Sec. 2.4): the tables already hold the total scattering coefficient; a DDMC step's
// event draw may land in the absorption band of its thresholds, and an MC flight meets Lya,
// dust scattering (isotropic, coherent in the comoving frame) and dust absorption in
// proportion to their opacities; absorbed packets are counted after their residence.
// Time-dependent estimators (eq. 17): every stretch of a packet's clock spent in a state adds
// its overlap with each census interval to that state's residence time (2^-24 units) and
// counts the packet in that state at every census time it spans.  Packets start at t = 0 or
// uniformly inside their source's emission window.
// Frequency groups (Sec. 5.3): in a cloud built with them, thin states carry a bin instead of
// a continuous frequency; flights meet the bin-averaged opacity and scatterings draw the
// outgoing bin from the eq. 42 alias table of the packet's bin.
// Escapes add face row (slab: face; sphere: one row), lab bin and time to the int64 tallies.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mc_dev.h"
#include "philox.h"
#include "rddmc_internal.h"

namespace rddmc {

namespace {

using namespace mc;

constexpr uint32_t kDom1DH = 0x60000000u;       // counter domain of the 1D hybrid walk's streams

struct Pk1 {
    int cl;
    int cell;
    int j;
    bool mc, active;
    bool left_inner;   // the current flight started on the cell's inner sphere, moving outward
    float3 pos, n;
    float x;
    double t;
    double lw;         // -ln(weight): optical depth of dust absorption so far (continuous weights)
    uint32_t cn;       // next way of the packet's census path cache to evict (round robin)
    int ci;            // first census time at or after the packet's clock (its clock only grows)
    double tn;         // that census time (-inf until the first full update)
    uint64_t steps;
    uint32_t mcs, tomc, toddmc, refl;
    Rng r;
};

__device__ __forceinline__ float dot3f(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

// unit vector along p (+z at the origin)
__device__ __forceinline__ float3 radial(float3 p)
{
    const float r2 = dot3f(p, p);
    if (!(r2 > 0.0f)) return make_float3(0.f, 0.f, 1.f);
    const float ir = rsqrtf(r2);
    return make_float3(p.x * ir, p.y * ir, p.z * ir);
}

// outward normal of a cell at face f (0 lower / inner, 1 upper / outer) at point p
template <bool SPH>
__device__ __forceinline__ float3 face_normal(int f, float3 p)
{
    const float s = f ? 1.0f : -1.0f;
    if (!SPH) return make_float3(0.f, 0.f, s);
    const float3 e = radial(p);
    return make_float3(s * e.x, s * e.y, s * e.z);
}

// n . u of a cell whose bulk speed (in its thermal units) is u, at point p
template <bool SPH>
__device__ __forceinline__ float n_dot_u(float u, float3 p, float3 n)
{
    if (!SPH) return n.z * u;
    return u * dot3f(n, radial(p));
}

// direction with cosine mu ~ U(0, 1] about the unit vector N, uniform azimuth
__device__ __forceinline__ float3 hemi_about(Rng &r, const McArgs &a, float3 N)
{
    const float mu = uf(draw(r, a));
    const float ph = kTwoPi * uf(draw(r, a));
    const float s = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
    float sn, cs;
    sincosf(ph, &sn, &cs);
    float3 t1 = fabsf(N.z) < 0.9f ? make_float3(-N.y, N.x, 0.f) : make_float3(0.f, -N.z, N.y);
    const float il = rsqrtf(dot3f(t1, t1));
    t1 = make_float3(t1.x * il, t1.y * il, t1.z * il);
    const float3 t2 = make_float3(N.y * t1.z - N.z * t1.y, N.z * t1.x - N.x * t1.z, N.x * t1.y - N.y * t1.x);
    const float c1 = s * cs, c2 = s * sn;
    return make_float3(fmaf(mu, N.x, fmaf(c1, t1.x, c2 * t2.x)), fmaf(mu, N.y, fmaf(c1, t1.y, c2 * t2.y)),
                       fmaf(mu, N.z, fmaf(c1, t1.z, c2 * t2.z)));
}

// uniform point of face f of cell `cell`
template <bool SPH>
__device__ __forceinline__ float3 face_point(const double *fz, int cell, int f, Rng &r, const McArgs &a)
{
    const float rf = (float)fz[cell + f];
    if (!SPH) return make_float3(0.f, 0.f, rf);
    const float3 w = iso_dir(r, a);
    return make_float3(rf * w.x, rf * w.y, rf * w.z);
}

// uniform point of cell `cell` (uniform in volume)
template <bool SPH>
__device__ __forceinline__ float3 cell_point(const double *fz, int cell, Rng &r, const McArgs &a)
{
    const double lo = fz[cell], hi = fz[cell + 1];
    const double u = (double)uf(draw(r, a));
    if (!SPH) return make_float3(0.f, 0.f, (float)(lo + (hi - lo) * u));
    const float rr = (float)cbrt(lo * lo * lo + u * (hi * hi * hi - lo * lo * lo));
    const float3 w = iso_dir(r, a);
    return make_float3(rr * w.x, rr * w.y, rr * w.z);
}

// distance along n to the boundary of cell `cell` from p, and the face it reaches.  A flight
// that starts on the inner sphere moving outward cannot meet that sphere again (a line leaves a
// ball once); `left_inner` says so, where the sign of p . n cannot for a grazing flight.
template <bool SPH>
__device__ __forceinline__ float wall_distance(const double *fz, int cell, float3 p, float3 n, bool left_inner,
                                               int &face)
{
    const double lo = fz[cell], hi = fz[cell + 1];
    if (!SPH) {
        if (n.z > 0.0f) { face = 1; return fmaxf(0.0f, (float)((hi - (double)p.z) / (double)n.z)); }
        if (n.z < 0.0f) { face = 0; return fmaxf(0.0f, (float)((lo - (double)p.z) / (double)n.z)); }
        face = 1;
        return INFINITY;
    }
    const double px = p.x, py = p.y, pz = p.z;
    const double b = px * n.x + py * n.y + pz * n.z;
    // the packet is inside its shell: a point put on a face in float can sit an ulp outside,
    // which would turn the far root into a zero-length crossing back and forth
    const double r = fmin(fmax(sqrt(px * px + py * py + pz * pz), lo), hi);
    double s = -b + sqrt(fmax(0.0, b * b + (hi - r) * (hi + r)));
    face = 1;
    if (lo > 0.0 && b < 0.0 && !left_inner) {
        const double disc = b * b + (lo - r) * (lo + r);
        if (disc > 0.0) {
            const double s_in = fmax(0.0, -b - sqrt(disc));
            if (s_in < s) {
                s = s_in;
                face = 0;
            }
        }
    }
    return (float)fmax(0.0, s);
}

__device__ __forceinline__ int time_bin1(double t)
{
    if (!(t >= 1e-3)) return 0;
    const double u = (log10(t) + 3.0) * (RDDMC_TIME_BINS / 9.0);
    if (u >= (double)RDDMC_TIME_BINS) return RDDMC_TIME_BINS + 1;
    return 1 + (int)u;
}

__device__ __forceinline__ int step_bin1(uint64_t n) { return n <= 1 ? 0 : 63 - __clzll((long long)n); }

// Integral over [a, b) of the weight exp(-(lw0 + ka (t - t0))) of a packet that had log-weight
// lw0 at t0 (c = 1): w(a) (1 - exp(-ka (b - a))) / ka, the residence times the path correction.
__device__ __forceinline__ double weight_integral(double a, double b, double t0, double lw0, double ka)
{
    const double wa = exp(-(lw0 + ka * (a - t0)));
    return ka > 0.0 ? wa * (-expm1(-ka * (b - a)) / ka) : wa * (b - a);
}

constexpr uint64_t kNoKey = ~0ull;
constexpr int kWays = 8;         // ways of a lane's census path cache
constexpr int kBlockMax = 256;   // lanes per block of the walk

// The 'path' estimator's sums go through an eight-way cache per lane, held in LDS (way-major,
// so a wave's accesses to one way are 64 consecutive words): a walk returns to the states it
// has just left (a frequency move and back), so most of its per-step residences add to a held
// sum instead of a device atomic.  Integer sums make the tallies identical to adding every
// residence at once, whatever the evictions.  Each lane touches only its own slots.
__shared__ uint64_t s_path_key[kWays * kBlockMax];
__shared__ uint64_t s_path_sum[kWays * kBlockMax];

__device__ __forceinline__ void path_init()
{
#pragma unroll
    for (int q = 0; q < kWays; ++q) {
        s_path_key[q * kBlockMax + threadIdx.x] = kNoKey;
        s_path_sum[q * kBlockMax + threadIdx.x] = 0ull;
    }
}

__device__ __forceinline__ void path_add(Pk1 &p, unsigned long long *__restrict__ wpath, uint64_t key, uint64_t v)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int q = 0; q < kWays; ++q)
        if (s_path_key[q * kBlockMax + l] == key) {
            s_path_sum[q * kBlockMax + l] += v;
            return;
        }
    const int e = (int)p.cn * kBlockMax + l;
    const uint64_t k0 = s_path_key[e], v0 = s_path_sum[e];
    if (k0 != kNoKey && v0) atomicAdd(&wpath[k0], (unsigned long long)v0);
    s_path_key[e] = key;
    s_path_sum[e] = v;
    p.cn = (p.cn + 1) & (kWays - 1);
}

__device__ __forceinline__ void path_flush(Pk1 &p, unsigned long long *__restrict__ wpath)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int q = 0; q < kWays; ++q) {
        const uint64_t k0 = s_path_key[q * kBlockMax + l], v0 = s_path_sum[q * kBlockMax + l];
        if (k0 != kNoKey && v0) atomicAdd(&wpath[k0], (unsigned long long)v0);
        s_path_key[q * kBlockMax + l] = kNoKey;
        s_path_sum[q * kBlockMax + l] = 0ull;
    }
    p.cn = 0;
}

// The packet stays in state s over [t0, t1): census counts and residence times.  With
// continuous dust weights (log-weight lw0 at t0, decay rate ka) the counts are the weights at
// the census times and the residences their integrals (2^-24 units both).
template <bool WGT>
__device__ __forceinline__ void census_add(Pk1 &p, const DevCloud &c, const uint8_t *__restrict__ tb,
                                           unsigned long long *__restrict__ tally, int64_t s, double t0, double t1,
                                           double lw0, double ka)
{
    const int n = c.n_census;
    if (p.ci > n) return;   // past the last census time: nothing to count
    unsigned long long *w = tally + c.tally_off;
    const uint64_t ns = c.n_states;
    if (t1 <= p.tn) {   // no census time in [t0, t1): the whole residence in interval ci - 1
        if (p.ci > 0 && t1 > t0) {
            const double r = (WGT && c.dust_weight) ? weight_integral(t0, t1, t0, lw0, ka) : t1 - t0;
            path_add(p, w + c.census_path_off, (uint64_t)(p.ci - 1) * ns + s, (uint64_t)rint(r * kPathFix));
        }
        return;
    }
    const double *ct = reinterpret_cast<const double *>(tb + c.off_census);
    int lo = p.ci;   // first census time >= t0: the packet's clock never goes back
    while (lo <= n && ct[lo] < t0) ++lo;
    p.ci = lo;
    p.tn = lo <= n ? ct[lo] : 0.0;
    for (int e = lo; e <= n && ct[e] < t1; ++e)
        atomicAdd(&w[c.census_bin_off + (uint64_t)e * ns + s],
                  (WGT && c.dust_weight) ? (unsigned long long)rint(exp(-(lw0 + ka * (ct[e] - t0))) * kPathFix) : 1ull);
    for (int i = lo > 0 ? lo - 1 : 0; i < n && ct[i] < t1; ++i) {
        const double a0 = fmax(t0, ct[i]), b0 = fmin(t1, ct[i + 1]);
        if (b0 > a0) {
            const double r = (WGT && c.dust_weight) ? weight_integral(a0, b0, t0, lw0, ka) : b0 - a0;
            path_add(p, w + c.census_path_off, (uint64_t)i * ns + s, (uint64_t)rint(r * kPathFix));
        }
    }
}

// Eq. 18: a leak of a step that stayed over [t0, t1) adds v times its residence in each census
// interval to `cell` (signed fixed point, 2^-24); with continuous dust weights, v times the
// weight's integral over the residence (the path correction).
// lo is the first census index whose time is >= t0 (the packet's index after census_add of
// the same residence).
template <bool WGT>
__device__ __forceinline__ void accel_add(const DevCloud &c, const uint8_t *__restrict__ tb, unsigned long long *__restrict__ tally,
                          int cell, double t0, double t1, double v, double lw0, double ka, int lo)
{
    const double *ct = reinterpret_cast<const double *>(tb + c.off_census);
    const int n = c.n_census;
    unsigned long long *w = tally + c.tally_off + c.census_accel_off;
    for (int i = lo > 0 ? lo - 1 : 0; i < n && ct[i] < t1; ++i) {
        const double a0 = fmax(t0, ct[i]), b0 = fmin(t1, ct[i + 1]);
        if (b0 > a0) {
            const double r = (WGT && c.dust_weight) ? weight_integral(a0, b0, t0, lw0, ka) : b0 - a0;
            atomicAdd(&w[(uint64_t)i * c.nc + cell], (unsigned long long)(long long)rint(v * r * kAccelFix));
        }
    }
}

// A weighted escape (continuous dust weights): weight and squared weight into slot q of the
// weighted spectra, w t and w t^2 into their 128-bit sums.
__device__ __forceinline__ void escape_weighted(const DevCloud &c, unsigned long long *w, uint64_t q, uint64_t nspec,
                                             double lw, double t)
{
    unsigned long long *ww = w + c.wspec_off;
    const double wt = exp(-lw);
    atomicAdd(&ww[4 + q], (unsigned long long)rint(wt * kWeightFix));
    atomicAdd(&ww[4 + nspec + q], (unsigned long long)rint(wt * wt * kWeightFix));
    const unsigned long long a1 = (unsigned long long)rint(wt * t * kWeightFix);
    if (atomicAdd(&ww[0], a1) + a1 < a1) atomicAdd(&ww[1], 1ull);
    const unsigned long long a2 = (unsigned long long)rint(wt * t * t * kTimeFix);
    if (atomicAdd(&ww[2], a2) + a2 < a2) atomicAdd(&ww[3], 1ull);
}

template <bool WGT, bool CEN>
__device__ __forceinline__ void finish1(Pk1 &p, const DevCloud &c, unsigned long long *__restrict__ tally, bool escaped, int row,
                        int slot, bool absorbed = false)
{
    unsigned long long *w = tally + c.tally_off;
    const uint64_t nspec = (uint64_t)c.n_rows * (c.nb + 2);
    if (absorbed) {
        atomicAdd(&w[TW_ABSORBED], 1ull);
    } else if (escaped) {
        atomicAdd(&w[TW_ESCAPED], 1ull);
        atomicAdd(&w[kTallyHeader + (uint64_t)row * (c.nb + 2) + slot], 1ull);
        atomicAdd(&w[TW_TSUM], (unsigned long long)rint(p.t * kTimeFix));
        const unsigned long long t2 = (unsigned long long)rint(p.t * p.t * kTimeFix);
        const unsigned long long old = atomicAdd(&w[TW_T2_LO], t2);
        if (old + t2 < old) atomicAdd(&w[TW_T2_HI], 1ull);
        atomicAdd(&w[kTallyHeader + nspec + time_bin1(p.t)], 1ull);
        if (WGT && c.dust_weight) escape_weighted(c, w, (uint64_t)row * (c.nb + 2) + slot, nspec, p.lw, p.t);
    } else {
        atomicAdd(&w[TW_CAPPED], 1ull);
    }
    if (CEN && c.n_census > 0) path_flush(p, w + c.census_path_off);
    atomicAdd(&w[kTallyHeader + nspec + RDDMC_TIME_BINS + 2 + step_bin1(p.steps)], 1ull);
    atomicAdd(&w[TW_STEPS], (unsigned long long)p.steps);
    atomicMax(&w[TW_STEPS_MAX], (unsigned long long)p.steps);
    if (p.mcs) atomicAdd(&w[TW_MC_STEPS], (unsigned long long)p.mcs);
    if (p.tomc) atomicAdd(&w[TW_TO_MC], (unsigned long long)p.tomc);
    if (p.toddmc) atomicAdd(&w[TW_TO_DDMC], (unsigned long long)p.toddmc);
    if (p.refl) atomicAdd(&w[TW_REFLECTED], (unsigned long long)p.refl);
    p.active = false;
}

// neighbour of `cell` through face f: -1 for vacuum (a sphere's r = 0 face has no leak)
__device__ __forceinline__ int neighbour1(const DevCloud &c, int cell, int f)
{
    if (f) return cell + 1 < c.nc ? cell + 1 : -1;
    return cell > 0 ? cell - 1 : -1;
}

// One DDMC step of a packet in a thick state.
template <bool SPH, bool WGT, bool CEN>
__device__ __forceinline__ void ddmc_step1(Pk1 &p, const DevCloud &c, const uint8_t *__restrict__ tb, const McArgs &a,
                           unsigned long long *__restrict__ tally)
{
    const int nb = c.nb;
    const int64_t s = (int64_t)p.cell * nb + p.j;
    const uint4 rec = reinterpret_cast<const uint4 *>(tb + c.off_hot)[s];
    const uint32_t tw = draw(p.r, a), ew = draw(p.r, a);
    const double dl = (double)ddmc_path(tw, __uint_as_float(rec.x));
    // continuous dust weights: the interaction distance dl carries optical depth k_a dl
    const double ka = (WGT && c.dust_weight) ? reinterpret_cast<const double *>(tb + c.off_dust)[2 * p.cell] : 0.0;
    const double lw0 = p.lw;
    if (CEN && c.n_census > 0) census_add<WGT>(p, c, tb, tally, s, p.t, p.t + dl, lw0, ka);
    const double t0 = p.t;
    p.t += dl;
    if (WGT && c.dust_weight) {
        p.lw += ka * dl;
        if (p.lw > kLogWMin) {   // negligible weight: eliminated
            finish1<WGT, CEN>(p, c, tally, false, 0, 0, true);
            return;
        }
    }
    int ev;
    bool have_lo = false;
    uint32_t lo_word = 0u;
    if (ew != rec.y && ew != rec.z) {
        ev = ew < rec.y ? 0 : (ew < rec.z ? 1 : 2);
    } else {   // the high words tie: compare the full u64
        const uint4 lw = reinterpret_cast<const uint4 *>(tb + c.off_lo_words)[s];
        lo_word = draw(p.r, a);
        have_lo = true;
        const uint64_t U = ((uint64_t)ew << 32) | lo_word;
        const uint64_t D = ((uint64_t)rec.y << 32) | lw.x;
        const uint64_t S = ((uint64_t)rec.z << 32) | lw.y;
        ev = U < D ? 0 : (U < S ? 1 : 2);
    }
    if (ev == 2 && c.dusty) {   // dust absorption band [A, 2^64) above the spatial leaks
        const uint4 lw = reinterpret_cast<const uint4 *>(tb + c.off_lo_words)[s];
        const uint64_t A = ((uint64_t)lw.w << 32) | lw.z;
        bool absorb;
        if (A == 0ull) {
            absorb = false;
        } else if (ew != lw.w) {
            absorb = ew > lw.w;
        } else {
            if (!have_lo) lo_word = draw(p.r, a);
            absorb = (((uint64_t)ew << 32) | lo_word) >= A;
        }
        if (absorb) {
            finish1<WGT, CEN>(p, c, tally, false, 0, 0, true);
            return;
        }
    }
    const double *fz = faces_of(c, tb, 0);
    if (ev < 2) {   // frequency leak (eq. 11)
        p.j += ev ? 1 : -1;
        if (rec.w & (ev ? kFlagUpThin : kFlagDnThin)) {   // into a thin bin: MC in this cell
            p.pos = cell_point<SPH>(fz, p.cell, p.r, a);
            p.n = iso_dir(p.r, a);
            p.left_inner = false;
            p.x = bin_x(c, tb, p.j, uf(draw(p.r, a)));
            p.mc = true;
            ++p.tomc;
        }
        return;
    }
    // spatial leak: face 0 or 1 from the state's split
    const uint32_t v = draw(p.r, a) >> 1;
    const int f = v >= reinterpret_cast<const uint32_t *>(tb + c.off_face_split)[s] ? 1 : 0;
    const double *kt = reinterpret_cast<const double *>(tb + c.off_k);
    const double dir = f ? 1.0 : -1.0;
    if (CEN && c.n_census > 0) accel_add<WGT>(c, tb, tally, p.cell, t0, p.t, dir * kt[s], lw0, ka, p.ci);   // outward leakage (eq. 18)
    const float xin = bin_x(c, tb, p.j, uf(draw(p.r, a)));
    const int nbc = neighbour1(c, p.cell, f);
    const float4 *mcell = reinterpret_cast<const float4 *>(tb + c.off_mcell);
    if (rec.w & (1u << (kFlagFaceShift + f))) {
        // interface leak into a thin state or vacuum: an MC packet leaving through face f
        p.pos = face_point<SPH>(fz, p.cell, f, p.r, a);
        p.n = hemi_about(p.r, a, face_normal<SPH>(f, p.pos));
        const float nu = n_dot_u<SPH>(mcell[2 * p.cell + 1].x, p.pos, p.n);
        if (nbc < 0) {
            const int slot = c.moving ? bin_of(c, tb, xin + nu) + 1 : p.j + 1;
            finish1<WGT, CEN>(p, c, tally, true, SPH ? 0 : f, slot);
            return;
        }
        const float4 m0 = mcell[2 * p.cell], m1 = mcell[2 * nbc];
        p.x = (xin + nu) * (m0.z / m1.z) - n_dot_u<SPH>(mcell[2 * nbc + 1].x, p.pos, p.n);
        p.cell = nbc;
        p.left_inner = f == 1;   // through the outer face of the old cell: the new one's inner
        p.mc = true;
        ++p.tomc;
        return;
    }
    // thick neighbour (vacuum faces always carry the interface bit)
    float xs = xin;
    if (c.moving) {
        const double *mp = reinterpret_cast<const double *>(tb + c.off_map) + 3 * (p.cell * 2 + f);
        const double rho = mp[0], sh = mp[1];
        if (rho != 1.0 || sh != 0.0) {
            xs = (float)(rho * (double)xin + sh);
            const int jn = bin_of(c, tb, xs);
            p.j = jn < 0 ? 0 : (jn > nb - 1 ? nb - 1 : jn);
        }
    }
    p.cell = nbc;
    bool ddmc_in = true;
    if (c.moving) {
        const uint4 rn = reinterpret_cast<const uint4 *>(tb + c.off_hot)[(int64_t)p.cell * nb + p.j];
        if (!(rn.w & kFlagThick)) {   // re-binned into a thin state: MC in the new cell
            p.pos = cell_point<SPH>(fz, p.cell, p.r, a);
            p.n = iso_dir(p.r, a);
            p.left_inner = false;
            p.x = xs;
            p.mc = true;
            ++p.tomc;
            ddmc_in = false;
        }
    }
    if (CEN && c.n_census > 0 && ddmc_in)   // inward leakage into a DDMC state (eq. 18)
        accel_add<WGT>(c, tb, tally, p.cell, t0, p.t, dir * kt[(int64_t)p.cell * nb + p.j], lw0, ka, p.ci);
}

// One continuous-MC event (a scattering or a boundary crossing) of a packet in a thin state.
template <bool SPH, bool WGT, bool CEN>
__device__ __forceinline__ void mc_step1(Pk1 &p, const DevCloud &c, const uint8_t *__restrict__ tb, const McArgs &a,
                         unsigned long long *__restrict__ tally, const float *__restrict__ vtab,
                         const float *__restrict__ u0tab)
{
    ++p.mcs;
    const float4 *mcell = reinterpret_cast<const float4 *>(tb + c.off_mcell);
    const double *fz = faces_of(c, tb, 0);
    const float4 m0 = mcell[2 * p.cell];   // k0, a, sqrt(T), width
    const float4 m1c = mcell[2 * p.cell + 1];   // u, and with dust k_s, k_a
    const float uc = m1c.x;
    int fexit = 1;
    const float dwall = wall_distance<SPH>(fz, p.cell, p.pos, p.n, p.left_inner, fexit);
    const float kl = m0.x * voigt_f32(m0.y, p.x, vtab);
    // dust absorption is an interaction, or (continuous weights) a decay of the weight
    const float kab = (WGT && c.dust_weight) ? 0.0f : m1c.z;
    const float kx = c.dusty ? kl + m1c.y + kab : kl;
    const float ds = -__logf(uf(draw(p.r, a))) / kx;
    const float u0 = n_dot_u<SPH>(uc, p.pos, p.n);
    const double fl = (double)fminf(ds, dwall);
    if (CEN && c.n_census > 0) {
        int jc = bin_of(c, tb, p.x);
        jc = jc < 0 ? 0 : (jc > c.nb - 1 ? c.nb - 1 : jc);
        census_add<WGT>(p, c, tb, tally, (int64_t)p.cell * c.nb + jc, p.t, p.t + fl, p.lw, (double)m1c.z);
    }
    if (WGT && c.dust_weight) {
        p.lw += (double)m1c.z * fl;
        if (p.lw > kLogWMin) {   // negligible weight: eliminated
            finish1<WGT, CEN>(p, c, tally, false, 0, 0, true);
            return;
        }
    }
    if (ds < dwall) {   // an interaction
        p.pos.x = fmaf(ds, p.n.x, p.pos.x);
        p.pos.y = fmaf(ds, p.n.y, p.pos.y);
        p.pos.z = fmaf(ds, p.n.z, p.pos.z);
        p.t += (double)ds;
        if (SPH && c.moving) p.x += u0 - n_dot_u<SPH>(uc, p.pos, p.n);
        if (c.dusty) {   // which opacity interacted: dust absorption, dust scattering or Lya
            const float v = uf(draw(p.r, a)) * kx;
            if (v < kab) {
                finish1<WGT, CEN>(p, c, tally, false, 0, 0, true);
                return;
            }
            if (v < kab + m1c.y) {   // dust: isotropic, coherent in the comoving frame
                p.n = iso_dir(p.r, a);
                p.left_inner = false;
                return;
            }
        }
        float upar;
        if (!sample_upar(m0.y, p.x, u0tab, p.r, a, upar)) {
            finish1<WGT, CEN>(p, c, tally, false, 0, 0);   // counted with the step-capped packets
            return;
        }
        // perpendicular velocity in the scattering plane: sqrt(xc^2 - ln xi) cos(phi), a
        // N(0, 1/2) component without core-skipping (xc = 0)
        const float xc = (c.x_crit > 0.0f && fabsf(p.x) < c.x_crit) ? c.x_crit : 0.0f;
        const float uperp = sqrtf(fmaf(xc, xc, -__logf(uf(draw(p.r, a))))) * cosf(kTwoPi * uf(draw(p.r, a)));
        const float3 n2 = iso_dir(p.r, a);
        const float mu = dot3f(p.n, n2);
        p.x = p.x + upar * (mu - 1.0f) + uperp * sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
        p.n = n2;
        p.left_inner = false;
        const int jj = bin_of(c, tb, p.x);
        if (jj >= 0 && jj < c.nb &&
            (reinterpret_cast<const uint4 *>(tb + c.off_hot)[(int64_t)p.cell * c.nb + jj].w & kFlagThick)) {
            p.j = jj;
            p.mc = false;
            ++p.toddmc;
        }
        return;
    }
    // boundary crossing: put the point exactly on its plane or sphere
    p.pos.x = fmaf(dwall, p.n.x, p.pos.x);
    p.pos.y = fmaf(dwall, p.n.y, p.pos.y);
    p.pos.z = fmaf(dwall, p.n.z, p.pos.z);
    const float rf = (float)fz[p.cell + fexit];
    if (SPH) {
        const float3 e = radial(p.pos);
        p.pos = make_float3(rf * e.x, rf * e.y, rf * e.z);
    } else {
        p.pos.z = rf;
    }
    p.t += (double)dwall;
    const float nu = n_dot_u<SPH>(uc, p.pos, p.n);
    if (SPH && c.moving) p.x += u0 - nu;
    const int nbc = neighbour1(c, p.cell, fexit);
    if (nbc < 0) {
        finish1<WGT, CEN>(p, c, tally, true, SPH ? 0 : fexit, bin_of(c, tb, p.x + nu) + 1);
        return;
    }
    const float4 m1 = mcell[2 * nbc];
    const float xn = (p.x + nu) * (m0.z / m1.z) - n_dot_u<SPH>(mcell[2 * nbc + 1].x, p.pos, p.n);
    const int jn = bin_of(c, tb, xn);
    if (jn >= 0 && jn < c.nb &&
        (reinterpret_cast<const uint4 *>(tb + c.off_hot)[(int64_t)nbc * c.nb + jn].w & kFlagThick)) {
        const float kn = (float)reinterpret_cast<const double *>(tb + c.off_k)[(int64_t)nbc * c.nb + jn];
        const float mu = fabsf(dot3f(p.n, face_normal<SPH>(fexit, p.pos)));
        const float P = 2.0f / fmaf(kn, m1.w, 2.0f * (float)c.lambda) * (0.666666667f + mu);   // eq. 39
        if (uf(draw(p.r, a)) < P) {
            p.cell = nbc;
            p.j = jn;
            p.mc = false;
            ++p.toddmc;
            return;
        }
        // reflected: uniform point of the interface, isotropic direction back into the cell
        p.pos = face_point<SPH>(fz, p.cell, fexit, p.r, a);
        const float3 N = face_normal<SPH>(fexit, p.pos);
        p.n = hemi_about(p.r, a, make_float3(-N.x, -N.y, -N.z));
        p.left_inner = fexit == 0;   // back off the inner sphere, outward
        ++p.refl;
        return;
    }
    p.cell = nbc;
    p.left_inner = fexit == 1;
    p.x = xn;
}

// One frequency-group Monte Carlo event (Sec. 5.3) of a packet in a thin state of a static,
// isothermal cloud: the packet carries bin j; a flight meets the bin-averaged opacity k_ij
// (eq. 14) plus any dust; a scattering takes the outgoing bin from row j of the cloud's alias
// table of eq. 42 (two 32-bit words) and an isotropic direction.  Boundaries as in mc_step1,
// with the bin unchanged across faces (no velocities, one temperature).
template <bool SPH, bool WGT, bool CEN>
__device__ __forceinline__ void grp_step1(Pk1 &p, const DevCloud &c, const uint8_t *__restrict__ tb, const McArgs &a,
                          unsigned long long *__restrict__ tally)
{
    ++p.mcs;
    const double *fz = faces_of(c, tb, 0);
    const double *kt = reinterpret_cast<const double *>(tb + c.off_k);
    const int64_t s = (int64_t)p.cell * c.nb + p.j;
    int fexit = 1;
    const float dwall = wall_distance<SPH>(fz, p.cell, p.pos, p.n, p.left_inner, fexit);
    const float kl = (float)kt[s];
    float ka = 0.0f, ks = 0.0f, kd = 0.0f;   // kd: dust absorption rate (either method)
    if (c.dusty) {
        const float4 m1c = reinterpret_cast<const float4 *>(tb + c.off_mcell)[2 * p.cell + 1];
        ks = m1c.y;
        kd = m1c.z;
        ka = (WGT && c.dust_weight) ? 0.0f : kd;
    }
    const float kx = kl + ks + ka;
    const float ds = -__logf(uf(draw(p.r, a))) / kx;
    const double fl = (double)fminf(ds, dwall);
    if (CEN && c.n_census > 0) census_add<WGT>(p, c, tb, tally, s, p.t, p.t + fl, p.lw, (double)kd);
    if (WGT && c.dust_weight) {
        p.lw += (double)kd * fl;
        if (p.lw > kLogWMin) {   // negligible weight: eliminated
            finish1<WGT, CEN>(p, c, tally, false, 0, 0, true);
            return;
        }
    }
    if (ds < dwall) {   // an interaction
        p.pos.x = fmaf(ds, p.n.x, p.pos.x);
        p.pos.y = fmaf(ds, p.n.y, p.pos.y);
        p.pos.z = fmaf(ds, p.n.z, p.pos.z);
        p.t += (double)ds;
        p.left_inner = false;
        if (c.dusty) {
            const float v = uf(draw(p.r, a)) * kx;
            if (v < ka) {
                finish1<WGT, CEN>(p, c, tally, false, 0, 0, true);
                return;
            }
            if (v < ka + ks) {   // dust: isotropic, the bin unchanged
                p.n = iso_dir(p.r, a);
                return;
            }
        }
        // eq. 42: the outgoing bin from the row's alias table
        const uint32_t w1 = draw(p.r, a), w2 = draw(p.r, a);
        const int col = (int)(((uint64_t)w1 * (uint32_t)c.nb) >> 32);
        const uint2 ent = reinterpret_cast<const uint2 *>(tb + c.off_grp_alias)[(int64_t)p.j * c.nb + col];
        const int jj = w2 < ent.x ? col : (int)ent.y;
        p.n = iso_dir(p.r, a);
        p.j = jj;
        if (reinterpret_cast<const uint4 *>(tb + c.off_hot)[(int64_t)p.cell * c.nb + jj].w & kFlagThick) {
            p.mc = false;
            ++p.toddmc;
        }
        return;
    }
    // boundary crossing: put the point exactly on its plane or sphere
    p.pos.x = fmaf(dwall, p.n.x, p.pos.x);
    p.pos.y = fmaf(dwall, p.n.y, p.pos.y);
    p.pos.z = fmaf(dwall, p.n.z, p.pos.z);
    const float rf = (float)fz[p.cell + fexit];
    if (SPH) {
        const float3 e = radial(p.pos);
        p.pos = make_float3(rf * e.x, rf * e.y, rf * e.z);
    } else {
        p.pos.z = rf;
    }
    p.t += (double)dwall;
    const int nbc = neighbour1(c, p.cell, fexit);
    if (nbc < 0) {
        finish1<WGT, CEN>(p, c, tally, true, SPH ? 0 : fexit, p.j + 1);
        return;
    }
    if (reinterpret_cast<const uint4 *>(tb + c.off_hot)[(int64_t)nbc * c.nb + p.j].w & kFlagThick) {
        const float4 m1 = reinterpret_cast<const float4 *>(tb + c.off_mcell)[2 * nbc];
        const float kn = (float)kt[(int64_t)nbc * c.nb + p.j];
        const float mu = fabsf(dot3f(p.n, face_normal<SPH>(fexit, p.pos)));
        const float P = 2.0f / fmaf(kn, m1.w, 2.0f * (float)c.lambda) * (0.666666667f + mu);   // eq. 39
        if (uf(draw(p.r, a)) < P) {
            p.cell = nbc;
            p.mc = false;
            ++p.toddmc;
            return;
        }
        // reflected: uniform point of the interface, isotropic direction back into the cell
        p.pos = face_point<SPH>(fz, p.cell, fexit, p.r, a);
        const float3 N = face_normal<SPH>(fexit, p.pos);
        p.n = hemi_about(p.r, a, make_float3(-N.x, -N.y, -N.z));
        p.left_inner = fexit == 0;
        ++p.refl;
        return;
    }
    p.cell = nbc;
    p.left_inner = fexit == 1;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = __shfl((int)(uint32_t)v, src);
    const uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <bool SPH, bool SINGLE, bool WGT, bool CEN>
__global__ __launch_bounds__(256) void walk1dh(const uint8_t *__restrict__ tb, McArgs a,
                                               unsigned long long *__restrict__ tally,
                                               unsigned long long *__restrict__ work)
{
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud *clouds = reinterpret_cast<const DevCloud *>(tb + H->off_clouds);
    const uint64_t *prefix = reinterpret_cast<const uint64_t *>(tb + H->off_prefix);
    const float *vtab = reinterpret_cast<const float *>(tb + H->off_voigt);
    const float *u0tab = reinterpret_cast<const float *>(tb + H->off_u0);
    const int lane = threadIdx.x & 63;

    Pk1 p;
    p.active = false;
    p.mc = false;
    p.left_inner = false;
    p.cl = 0;
    p.cell = 0;
    p.j = 0;
    p.pos = make_float3(0.f, 0.f, 0.f);
    p.n = make_float3(0.f, 0.f, 1.f);
    p.x = 0.f;
    p.t = 0.0;
    p.lw = 0.0;
    if (CEN) path_init();
    p.cn = 0;
    p.ci = 0;
    p.tn = -__builtin_inf();
    p.steps = 0;
    p.mcs = p.tomc = p.toddmc = p.refl = 0u;
    p.r = Rng{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 4u, false, 0u, 0u, 0u, 0u};
    bool exhausted = false;

    for (;;) {
        if (!exhausted) {
            const uint64_t need = __ballot(!p.active);
            if (need) {
                const int leader = __ffsll((unsigned long long)need) - 1;
                const int cnt = __popcll(need);
                uint64_t base = 0;
                if (lane == leader) base = atomicAdd(work, (unsigned long long)cnt);
                base = shfl64(base, leader);
                if (base + cnt >= a.count) exhausted = true;
                if (!p.active) {
                    const uint64_t q = base + __popcll(need & ((1ull << lane) - 1ull));
                    if (q < a.count) {
                        const uint64_t g = a.first + q;
                        int cl = 0;
                        if (!SINGLE) {
                            int lo = 0, hi = a.n_clouds;
                            while (hi - lo > 1) {
                                const int mid = (lo + hi) >> 1;
                                if (g >= prefix[mid]) lo = mid; else hi = mid;
                            }
                            cl = lo;
                        }
                        const DevCloud &c = clouds[cl];
                        p.cl = cl;
                        p.r = Rng{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 4u, false, 0u, 0u, (uint32_t)(g - prefix[cl]),
                                  c.stream};
                        // emission (Sec. 2.3): a source entry drawn by its probability
                        const double u = ud(draw(p.r, a));
                        const double *cdf = reinterpret_cast<const double *>(tb + c.off_src_cdf);
                        int lo = 0, hi = c.n_src - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (u < cdf[mid]) hi = mid; else lo = mid + 1;
                        }
                        const int64_t st = reinterpret_cast<const int32_t *>(tb + c.off_src_state)[lo];
                        p.cell = (int)(st / c.nb);
                        p.j = (int)(st - (int64_t)p.cell * c.nb);
                        p.t = 0.0;
                        p.lw = 0.0;
                        p.ci = 0;
                        p.tn = -__builtin_inf();
                        if (c.off_src_t) {   // emission uniform over the source's window
                            const double *tw = reinterpret_cast<const double *>(tb + c.off_src_t) + 2 * lo;
                            p.t = tw[0] + (tw[1] - tw[0]) * ud(draw(p.r, a));
                        }
                        p.steps = 0;
                        p.mcs = p.tomc = p.toddmc = p.refl = 0u;
                        p.active = true;
                        const uint4 rec = reinterpret_cast<const uint4 *>(tb + c.off_hot)[st];
                        p.mc = !(rec.w & kFlagThick);
                        if (p.mc) {   // a thin source state starts as an MC packet at the source
                            const float4 sp = reinterpret_cast<const float4 *>(tb + c.off_src_pos)[lo];
                            p.pos = make_float3(0.f, 0.f, sp.z);
                            p.x = sp.w;
                            p.n = iso_dir(p.r, a);
                            p.left_inner = false;
                        }
                        atomicAdd(&tally[c.tally_off + TW_LAUNCHED], 1ull);
                    }
                }
            }
        }
        if (!__any(p.active)) break;

        // Mode-batched passes, as on 3D grids: DDMC lanes take up to two steps, or MC lanes
        // one event; every packet's own sequence of steps and draws is unchanged by this.
        const DevCloud &c = clouds[SINGLE ? 0 : p.cl];
        for (int k = 0; k < a.chunk; ++k) {
            if (p.active && p.steps >= a.max_steps) finish1<WGT, CEN>(p, c, tally, false, 0, 0);
            const uint64_t bm = __ballot(p.active && p.mc);
            const uint64_t bd = __ballot(p.active && !p.mc);
            if (!(bm | bd)) break;
            const int nm = __popcll(bm), nd = __popcll(bd);
            const bool mc_pass = nm > 0 && (4 * nm >= nd || (k & 7) == 7);
            if (p.active && p.mc == mc_pass) {
                prefetch(p.r, a);
                ++p.steps;
                if (mc_pass) {
                    if (c.groups)
                        grp_step1<SPH, WGT, CEN>(p, c, tb, a, tally);
                    else
                        mc_step1<SPH, WGT, CEN>(p, c, tb, a, tally, vtab, u0tab);
                } else {
                    ddmc_step1<SPH, WGT, CEN>(p, c, tb, a, tally);
                    if (p.active && !p.mc && p.steps < a.max_steps) {
                        ++p.steps;
                        ddmc_step1<SPH, WGT, CEN>(p, c, tb, a, tally);
                    }
                }
            }
        }
    }
}

__global__ void reset_queue1(unsigned long long *work)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) work[0] = 0ull;
}

}  // namespace

hipError_t launch_walk1dh(const uint8_t *d_tables, const DevHeader &h, const rddmc_run &run, uint64_t first,
                          uint64_t count, unsigned long long *d_tally, unsigned long long *d_work, hipStream_t s)
{
    McArgs a;
    a.first = first;
    a.count = count;
    a.max_steps = run.max_steps;
    a.key0 = (uint32_t)run.seed;
    a.key1 = (uint32_t)(run.seed >> 32);
    a.chunk = run.chunk > 0 ? run.chunk : 64;
    a.n_clouds = h.n_clouds;
    a.dom = kDom1DH;
    const int block = run.block > 0 ? run.block : 256;
    uint64_t grid = run.grid > 0 ? (uint64_t)run.grid : 0;
    if (grid == 0) {
        const uint64_t want = (count + block - 1) / block;
        const uint64_t cap = (uint64_t)device_cu_count() * 8;
        grid = want < cap ? want : cap;
        if (grid < 1) grid = 1;
    }
    reset_queue1<<<1, 64, 0, s>>>(d_work);
    const bool sph = h.geometry == RDDMC_SPHERE;
    const bool single = h.n_clouds == 1;
    // batches with continuous dust weights or census estimators take instantiations of their
    // own, so that the others keep the registers (and occupancy) of a walk without them
    auto go = [&](auto wgt, auto cen) {
        constexpr bool W = decltype(wgt)::value, C = decltype(cen)::value;
        if (sph && single)
            walk1dh<true, true, W, C><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
        else if (sph)
            walk1dh<true, false, W, C><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
        else if (single)
            walk1dh<false, true, W, C><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
        else
            walk1dh<false, false, W, C><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    };
    if (h.dust_weight1d && h.census1d)
        go(std::true_type{}, std::true_type{});
    else if (h.dust_weight1d)
        go(std::true_type{}, std::false_type{});
    else if (h.census1d)
        go(std::false_type{}, std::true_type{});
    else
        go(std::false_type{}, std::false_type{});
    return hipGetLastError();
}

}  // namespace rddmc
