// Hybrid rDDMC walk on 3D Cartesian grids: DDMC steps in thick states (Sec. 2.3,
// eqs. 15-16; Doppler re-binning of Sec. 2.5) and continuous Monte Carlo in thin ones (the
// hybrid section: interface leaks, conversions both ways and the eq. 39 acceptance; the
// MC step with the Voigt opacity of eq. 12 and the frequency redistribution of eq. 41).
//
// One lane carries one packet: cloud, cell (and its three indices), bin, mode, FP32
// position / direction / comoving frequency of MC packets, FP64 clock, step counts and a
// per-packet counter-based random stream (Philox4x32-10 blocks counted per packet, words
// used in order).  Per step:
//   DDMC state: the 16-byte hot record {ln2/K, D_hi, S_hi, flags}; a time word gives the
//     exponential path length, an event word the high word of a u64 uniform against the
//     thresholds D = P(lower bin) 2^64 and S = (1 - P(spatial)) 2^64 (a tie takes the low
//     word from the stream); a spatial leak picks its face from the state's 31-bit face CDF.
//     The flags say whether bin j-1 / j+1 is thin (a frequency move there turns the packet
//     into an MC packet at a uniform point of the cell, isotropic, x uniform in the bin) and
//     whether a face leads into a thin state or vacuum (the packet leaves from a uniform
//     point of the face with an isotropic outward direction, mu uniform in (0,1], and x
//     uniform in the bin moved to the neighbour's frame: x' = (x + n.u) sqrt(T/T') - n.u');
//     otherwise it moves to the neighbour, re-binned by the f_mu-averaged shift of eq. 20.
//   MC state: distance to the cell wall along n against an exponential optical depth with
//     opacity k0 H(a, x); a scattering draws the atom's parallel velocity from
//     exp(-u^2) / (a^2 + (x - u)^2) by rejection from a Lorentzian split at u0 (the method of
//     Zheng & Miralda-Escude 2002; any u0 >= 0 is exact, a table holds the one minimising
//     the proposal mass), the perpendicular one from N(0, 1/2) (with core-skipping on, from
//     its tail above x_crit for photons in the core), an isotropic new direction
//     and x' = x + u_par (mu - 1) + u_perp sqrt(1 - mu^2) (eq. 41, no recoil); if (cell,
//     bin(x')) is thick the packet becomes DDMC there.  At a wall: vacuum -> escape with the
//     lab frequency x + n.u; a thick neighbour state accepts the packet with probability
//     2/(k' w' + 2 lambda) (2/3 + mu) (eq. 39), else it is reflected from a uniform point of
//     the face with an isotropic inward direction; a thin one continues the flight.
// Escapes add face, lab bin, boundary pixel and time to the exact int64 tallies.
#include <hip/hip_runtime.h>

#include "mc_dev.h"
#include "philox.h"
#include "rddmc_internal.h"

namespace rddmc {

namespace {

constexpr uint32_t kDom3D = 0x40000000u;        // counter domain of the 3D walk's streams

using namespace mc;
using Walk3Args = McArgs;

struct Pk {
    int cl;
    int ix, iy, iz;
    int64_t cell;
    int j;
    bool mc, active;
    bool pend;           // a DDMC step chose a spatial leak that has not been applied yet
    float3 pos, n;
    float x;
    double t;
    uint64_t steps;
    uint32_t mcs, tomc, toddmc, refl;
    Rng r;
};

// isotropic over the hemisphere of axis d with sign sg (mu uniform in (0, 1])
__device__ __forceinline__ float3 hemi_dir(Rng &r, const Walk3Args &a, int d, float sg)
{
    const float mu = uf(draw(r, a));
    const float ph = kTwoPi * uf(draw(r, a));
    const float s = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
    float sn, cs;
    sincosf(ph, &sn, &cs);
    const float t1 = s * cs, t2 = s * sn;
    float3 n;
    n.x = d == 0 ? sg * mu : (d == 1 ? t2 : t1);
    n.y = d == 1 ? sg * mu : (d == 2 ? t2 : t1);
    n.z = d == 2 ? sg * mu : (d == 0 ? t2 : t1);
    return n;
}

// uniform point of the current cell, optionally pinned to face f (f < 0: interior)
__device__ __forceinline__ float3 cell_point(const Pk &p, const DevCloud &c, const uint8_t *tb, int f, Rng &r,
                                             const Walk3Args &a)
{
    float3 q;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *fa = faces_of(c, tb, d);
        const int i = compi(p.ix, p.iy, p.iz, d);
        float v;
        if (f >= 0 && (f >> 1) == d) {
            v = (float)fa[i + (f & 1)];
        } else {
            const double lo = fa[i], hi = fa[i + 1];
            v = (float)(lo + (hi - lo) * (double)uf(draw(r, a)));
        }
        setc(q, d, v);
    }
    return q;
}

// neighbour through face f: false for vacuum
__device__ __forceinline__ bool neighbour(const Pk &p, const DevCloud &c, int f, int &nix, int &niy, int &niz,
                                          int64_t &ncell)
{
    const int d = f >> 1, up = f & 1;
    const int i = compi(p.ix, p.iy, p.iz, d);
    const int nn = compi(c.n[0], c.n[1], c.n[2], d);
    if (up ? (i + 1 >= nn) : (i == 0)) return false;
    const int step = up ? 1 : -1;
    nix = p.ix + (d == 0 ? step : 0);
    niy = p.iy + (d == 1 ? step : 0);
    niz = p.iz + (d == 2 ? step : 0);
    const int64_t stride = d == 0 ? 1 : (d == 1 ? (int64_t)c.n[0] : (int64_t)c.n[0] * c.n[1]);
    ncell = p.cell + step * stride;
    return true;
}

__device__ __forceinline__ uint64_t pixel_of(const Pk &p, const DevCloud &c, int f)
{
    const uint64_t nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const uint64_t sz0 = ny * nz, sz1 = nx * nz, sz2 = nx * ny;
    const int d = f >> 1;
    uint64_t off = 0;
    if (d >= 1) off += 2 * sz0;
    if (d >= 2) off += 2 * sz1;
    if (f & 1) off += d == 0 ? sz0 : (d == 1 ? sz1 : sz2);
    if (d == 0) return off + (uint64_t)p.iz * ny + p.iy;
    if (d == 1) return off + (uint64_t)p.iz * nx + p.ix;
    return off + (uint64_t)p.iy * nx + p.ix;
}

__device__ __forceinline__ int time_bin3(double t)
{
    if (!(t >= 1e-3)) return 0;
    const double u = (log10(t) + 3.0) * (RDDMC_TIME_BINS / 9.0);
    if (u >= (double)RDDMC_TIME_BINS) return RDDMC_TIME_BINS + 1;
    return 1 + (int)u;
}

__device__ __forceinline__ int step_bin3(uint64_t n) { return n <= 1 ? 0 : 63 - __clzll((long long)n); }

__device__ void finish(Pk &p, const DevCloud &c, unsigned long long *__restrict__ tally, bool escaped, int face,
                       int slot)
{
    unsigned long long *w = tally + c.tally_off;
    const uint64_t nspec = (uint64_t)c.n_rows * (c.nb + 2);
    if (escaped) {
        atomicAdd(&w[TW_ESCAPED], 1ull);
        atomicAdd(&w[kTallyHeader + (uint64_t)face * (c.nb + 2) + slot], 1ull);
        atomicAdd(&w[TW_TSUM], (unsigned long long)rint(p.t * kTimeFix));
        const unsigned long long t2 = (unsigned long long)rint(p.t * p.t * kTimeFix);
        const unsigned long long old = atomicAdd(&w[TW_T2_LO], t2);
        if (old + t2 < old) atomicAdd(&w[TW_T2_HI], 1ull);
        atomicAdd(&w[kTallyHeader + nspec + time_bin3(p.t)], 1ull);
        atomicAdd(&w[kTallyHeader + nspec + RDDMC_TIME_BINS + 2 + RDDMC_STEP_BINS + pixel_of(p, c, face)], 1ull);
    } else {
        atomicAdd(&w[TW_CAPPED], 1ull);
    }
    atomicAdd(&w[kTallyHeader + nspec + RDDMC_TIME_BINS + 2 + step_bin3(p.steps)], 1ull);
    atomicAdd(&w[TW_STEPS], (unsigned long long)p.steps);
    atomicMax(&w[TW_STEPS_MAX], (unsigned long long)p.steps);
    if (p.mcs) atomicAdd(&w[TW_MC_STEPS], (unsigned long long)p.mcs);
    if (p.tomc) atomicAdd(&w[TW_TO_MC], (unsigned long long)p.tomc);
    if (p.toddmc) atomicAdd(&w[TW_TO_DDMC], (unsigned long long)p.toddmc);
    if (p.refl) atomicAdd(&w[TW_REFLECTED], (unsigned long long)p.refl);
    p.active = false;
}

__device__ __forceinline__ void enter(Pk &p, int nix, int niy, int niz, int64_t ncell)
{
    p.ix = nix;
    p.iy = niy;
    p.iz = niz;
    p.cell = ncell;
}

// The draw and event of one DDMC step of a packet in a thick state: the path length, then a
// frequency leak (eq. 11) is applied at once; a spatial leak is only marked (pend) and applied
// by ddmc_leak, with the next random words of the packet's stream, before its next step.
__device__ void ddmc_event(Pk &p, const DevCloud &c, const uint8_t *__restrict__ tb, const Walk3Args &a)
{
    const int nb = c.nb;
    const int64_t s = p.cell * nb + p.j;
    const uint4 rec = reinterpret_cast<const uint4 *>(tb + c.off_hot)[s];
    const uint32_t tw = draw(p.r, a), ew = draw(p.r, a);
    p.t += (double)ddmc_path(tw, __uint_as_float(rec.x));
    int ev;
    if (ew != rec.y && ew != rec.z) {
        ev = ew < rec.y ? 0 : (ew < rec.z ? 1 : 2);
    } else {   // the high words tie: compare the full u64
        const uint4 lw = reinterpret_cast<const uint4 *>(tb + c.off_lo_words)[s];
        const uint64_t U = ((uint64_t)ew << 32) | draw(p.r, a);
        const uint64_t D = ((uint64_t)rec.y << 32) | lw.x;
        const uint64_t S = ((uint64_t)rec.z << 32) | lw.y;
        ev = U < D ? 0 : (U < S ? 1 : 2);
    }
    if (ev < 2) {   // frequency leak (eq. 11)
        p.j += ev ? 1 : -1;
        if (rec.w & (ev ? kFlagUpThin : kFlagDnThin)) {   // into a thin bin: MC in this cell
            p.pos = cell_point(p, c, tb, -1, p.r, a);
            p.n = iso_dir(p.r, a);
            p.x = bin_x(c, tb, p.j, uf(draw(p.r, a)));
            p.mc = true;
            ++p.tomc;
        }
        return;
    }
    p.pend = true;
}

// The spatial leak a DDMC step chose (p.pend): the face from the state's cumulative split, then
// the move into the neighbour (Doppler re-binning of eq. 20), a conversion to continuous MC
// through an interface face, or an escape.
__device__ void ddmc_leak(Pk &p, const DevCloud &c, const uint8_t *__restrict__ tb, const Walk3Args &a,
                          unsigned long long *__restrict__ tally)
{
    p.pend = false;
    const int nb = c.nb;
    const int64_t s = p.cell * nb + p.j;
    const uint4 rec = reinterpret_cast<const uint4 *>(tb + c.off_hot)[s];
    const uint32_t v = draw(p.r, a) >> 1;
    const uint32_t *fs = reinterpret_cast<const uint32_t *>(tb + c.off_face_split) + s * 5;
    int f = 0;
    while (f < 5 && v >= fs[f]) ++f;
    const float xin = bin_x(c, tb, p.j, uf(draw(p.r, a)));
    int nix = 0, niy = 0, niz = 0;
    int64_t ncell = 0;
    const bool inside = neighbour(p, c, f, nix, niy, niz, ncell);
    const float4 *mcell = reinterpret_cast<const float4 *>(tb + c.off_mcell);
    if (rec.w & (1u << (kFlagFaceShift + f))) {
        // interface leak into a thin state or vacuum: an MC packet leaving through face f
        p.pos = cell_point(p, c, tb, f, p.r, a);
        p.n = hemi_dir(p.r, a, f >> 1, (f & 1) ? 1.0f : -1.0f);
        const float4 uc = mcell[2 * p.cell + 1];
        const float nu = dot3(p.n, uc);
        if (!inside) {
            const int slot = c.moving ? bin_of(c, tb, xin + nu) + 1 : p.j + 1;
            finish(p, c, tally, true, f, slot);
            return;
        }
        const float4 m0 = mcell[2 * p.cell], m1 = mcell[2 * ncell], un = mcell[2 * ncell + 1];
        p.x = (xin + nu) * (m0.z / m1.z) - dot3(p.n, un);
        enter(p, nix, niy, niz, ncell);
        p.mc = true;
        ++p.tomc;
        return;
    }
    // thick neighbour (vacuum faces always carry the interface bit)
    float xs = xin;
    if (c.moving) {
        const double *mp = reinterpret_cast<const double *>(tb + c.off_map) + 3 * (p.cell * 6 + f);
        const double rho = mp[0], sh = mp[1];
        if (rho != 1.0 || sh != 0.0) {
            xs = (float)(rho * (double)xin + sh);
            const int jn = bin_of(c, tb, xs);
            p.j = jn < 0 ? 0 : (jn > nb - 1 ? nb - 1 : jn);
        }
    }
    enter(p, nix, niy, niz, ncell);
    if (c.moving) {
        const uint4 rn = reinterpret_cast<const uint4 *>(tb + c.off_hot)[p.cell * nb + p.j];
        if (!(rn.w & kFlagThick)) {   // re-binned into a thin state: MC in the new cell
            p.pos = cell_point(p, c, tb, -1, p.r, a);
            p.n = iso_dir(p.r, a);
            p.x = xs;
            p.mc = true;
            ++p.tomc;
        }
    }
}

// One continuous-MC event (a scattering or a wall crossing) of a packet in a thin state.
__device__ void mc_step(Pk &p, const DevCloud &c, const uint8_t *__restrict__ tb, const Walk3Args &a,
                        unsigned long long *__restrict__ tally, const float *__restrict__ vtab,
                        const float *__restrict__ u0tab, float lambda)
{
    ++p.mcs;
    const float4 *mcell = reinterpret_cast<const float4 *>(tb + c.off_mcell);
    const float4 m0 = mcell[2 * p.cell];   // k0, a, sqrt(T), w_min
    float dface = INFINITY;
    int fexit = 0;
    float wexit = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float nd = comp(p.n, d);
        if (nd != 0.0f) {
            const int up = nd > 0.0f ? 1 : 0;
            const float wall = (float)faces_of(c, tb, d)[compi(p.ix, p.iy, p.iz, d) + up];
            float dd = (wall - comp(p.pos, d)) / nd;
            dd = dd > 0.0f ? dd : 0.0f;
            if (dd < dface) {
                dface = dd;
                fexit = 2 * d + up;
                wexit = wall;
            }
        }
    }
    const float kx = m0.x * voigt_f32(m0.y, p.x, vtab);
    const float ds = -__logf(uf(draw(p.r, a))) / kx;
    if (ds < dface) {   // scattering
        p.pos.x = fmaf(ds, p.n.x, p.pos.x);
        p.pos.y = fmaf(ds, p.n.y, p.pos.y);
        p.pos.z = fmaf(ds, p.n.z, p.pos.z);
        p.t += (double)ds;
        float upar;
        if (!sample_upar(m0.y, p.x, u0tab, p.r, a, upar)) {
            finish(p, c, tally, false, 0, 0);   // counted with the step-capped packets
            return;
        }
        // perpendicular velocity in the scattering plane: sqrt(xc^2 - ln xi) cos(phi), a
        // N(0, 1/2) component without core-skipping (xc = 0)
        const float xc = (c.x_crit > 0.0f && fabsf(p.x) < c.x_crit) ? c.x_crit : 0.0f;
        const float uperp = sqrtf(fmaf(xc, xc, -__logf(uf(draw(p.r, a))))) * cosf(kTwoPi * uf(draw(p.r, a)));
        const float3 n2 = iso_dir(p.r, a);
        const float mu = fmaf(p.n.x, n2.x, fmaf(p.n.y, n2.y, p.n.z * n2.z));
        p.x = p.x + upar * (mu - 1.0f) + uperp * sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
        p.n = n2;
        const int jj = bin_of(c, tb, p.x);
        if (jj >= 0 && jj < c.nb &&
            (reinterpret_cast<const uint4 *>(tb + c.off_hot)[p.cell * c.nb + jj].w & kFlagThick)) {
            p.j = jj;
            p.mc = false;
            ++p.toddmc;
        }
        return;
    }
    // wall crossing
    p.pos.x = fmaf(dface, p.n.x, p.pos.x);
    p.pos.y = fmaf(dface, p.n.y, p.pos.y);
    p.pos.z = fmaf(dface, p.n.z, p.pos.z);
    const int d = fexit >> 1;
    setc(p.pos, d, wexit);
    p.t += (double)dface;
    const float4 uc = mcell[2 * p.cell + 1];
    const float nu = dot3(p.n, uc);
    int nix = 0, niy = 0, niz = 0;
    int64_t ncell = 0;
    if (!neighbour(p, c, fexit, nix, niy, niz, ncell)) {
        finish(p, c, tally, true, fexit, bin_of(c, tb, p.x + nu) + 1);
        return;
    }
    const float4 m1 = mcell[2 * ncell], un = mcell[2 * ncell + 1];
    const float xn = (p.x + nu) * (m0.z / m1.z) - dot3(p.n, un);
    const int jn = bin_of(c, tb, xn);
    if (jn >= 0 && jn < c.nb &&
        (reinterpret_cast<const uint4 *>(tb + c.off_hot)[ncell * c.nb + jn].w & kFlagThick)) {
        const float kn = (float)reinterpret_cast<const double *>(tb + c.off_k)[ncell * c.nb + jn];
        const float mu = fabsf(comp(p.n, d));
        // the neighbour's width across the interface (along the crossing axis), as in the
        // DDMC -> MC rate of the same face
        const double *fd = faces_of(c, tb, d);
        const int ind = compi(nix, niy, niz, d);
        const float wn = (float)(fd[ind + 1] - fd[ind]);
        const float P = 2.0f / fmaf(kn, wn, 2.0f * lambda) * (0.666666667f + mu);   // eq. 39
        if (uf(draw(p.r, a)) < P) {
            enter(p, nix, niy, niz, ncell);
            p.j = jn;
            p.mc = false;
            ++p.toddmc;
            return;
        }
        // reflected: uniform point of the interface, isotropic inward direction
        p.pos = cell_point(p, c, tb, fexit, p.r, a);
        p.n = hemi_dir(p.r, a, d, (fexit & 1) ? -1.0f : 1.0f);
        ++p.refl;
        return;
    }
    enter(p, nix, niy, niz, ncell);
    p.x = xn;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = __shfl((int)(uint32_t)v, src);
    const uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <bool SINGLE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void walk3d(const uint8_t *__restrict__ tb, Walk3Args a,
                                              unsigned long long *__restrict__ tally,
                                              unsigned long long *__restrict__ work)
{
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud *clouds = reinterpret_cast<const DevCloud *>(tb + H->off_clouds);
    const uint64_t *prefix = reinterpret_cast<const uint64_t *>(tb + H->off_prefix);
    const float *vtab = reinterpret_cast<const float *>(tb + H->off_voigt);
    const float *u0tab = reinterpret_cast<const float *>(tb + H->off_u0);
    const int lane = threadIdx.x & 63;

    Pk p;
    p.active = false;
    p.mc = false;
    p.pend = false;
    p.cl = 0; p.ix = p.iy = p.iz = 0; p.cell = 0; p.j = 0;
    p.pos = make_float3(0.f, 0.f, 0.f);
    p.n = make_float3(0.f, 0.f, 1.f);
    p.x = 0.f; p.t = 0.0; p.steps = 0;
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
                        p.r = Rng{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 4u, false, 0u, 0u,
                                  (uint32_t)(g - prefix[cl]), c.stream};
                        // emission (Sec. 2.3): a source entry drawn by its probability
                        const double u = ud(draw(p.r, a));
                        const double *cdf = reinterpret_cast<const double *>(tb + c.off_src_cdf);
                        int lo = 0, hi = c.n_src - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (u < cdf[mid]) hi = mid; else lo = mid + 1;
                        }
                        const int64_t st = reinterpret_cast<const int32_t *>(tb + c.off_src_state)[lo];
                        p.cell = st / c.nb;
                        p.j = (int)(st - p.cell * c.nb);
                        p.ix = (int)(p.cell % c.n[0]);
                        p.iy = (int)((p.cell / c.n[0]) % c.n[1]);
                        p.iz = (int)(p.cell / ((int64_t)c.n[0] * c.n[1]));
                        p.t = 0.0;
                        p.steps = 0;
                        p.mcs = p.tomc = p.toddmc = p.refl = 0u;
                        p.active = true;
                        p.pend = false;
                        const uint4 rec = reinterpret_cast<const uint4 *>(tb + c.off_hot)[st];
                        p.mc = !(rec.w & kFlagThick);
                        if (p.mc) {   // a thin source state starts as an MC packet at the source
                            const float4 sp = reinterpret_cast<const float4 *>(tb + c.off_src_pos)[lo];
                            p.pos = make_float3(sp.x, sp.y, sp.z);
                            p.x = sp.w;
                            p.n = iso_dir(p.r, a);
                        }
                        atomicAdd(&tally[c.tally_off + TW_LAUNCHED], 1ull);
                    }
                }
            }
        }
        if (!__any(p.active)) break;

        // Event-batched passes: a pass advances the wave's DDMC lanes by up to two steps, or
        // applies the spatial leaks its DDMC steps chose, or advances its continuous-MC lanes
        // by one event, never two of these, so a wave does not issue the long leak or MC path
        // for one lane.  A lane whose step chose a spatial leak waits for a leak pass (taken
        // once such lanes are a sixteenth of the stepping ones, or every 32nd pass); MC
        // lanes wait until they are at least an eighth as many as the DDMC lanes, or every
        // sixteenth pass.  (Thresholds measured on the 128^3 cube: leak passes at an eighth
        // 1 926 ms, a quarter 1 902, a sixteenth 1 867, a 32nd 1 865; MC passes at an eighth
        // with leak passes at a sixteenth 1 852.)  Each pass starts by generating every taking part lane's next random
        // block together (two frequency steps read one block).  Every packet still takes its
        // own steps in its own order from its own stream, so the results do not depend on
        // this schedule.
        const DevCloud &c = clouds[SINGLE ? 0 : p.cl];
        const float lambda = (float)c.lambda;
        for (int k = 0; k < a.chunk; ++k) {
            if (p.active && !p.pend && p.steps >= a.max_steps) finish(p, c, tally, false, 0, 0);
            const uint64_t bm = __ballot(p.active && p.mc);
            const uint64_t bl = __ballot(p.active && p.pend);
            const uint64_t bd = __ballot(p.active && !p.mc && !p.pend);
            if (!(bm | bd | bl)) break;
            const int nm = __popcll(bm), nl = __popcll(bl), nd = __popcll(bd);
            const int mode = (nm > 0 && (8 * nm >= nd + nl || (k & 15) == 15)) ? 2
                             : (nl > 0 && (16 * nl >= nd || (k & 31) == 31 || nd == 0)) ? 1 : 0;
            if (p.active && (mode == 2 ? p.mc : (mode == 1 ? p.pend : !p.mc && !p.pend))) {
                prefetch(p.r, a);
                if (mode == 2) {
                    ++p.steps;
                    mc_step(p, c, tb, a, tally, vtab, u0tab, lambda);
                } else if (mode == 1) {
                    ddmc_leak(p, c, tb, a, tally);
                } else {
                    ++p.steps;
                    ddmc_event(p, c, tb, a);
                    if (!p.mc && !p.pend && p.steps < a.max_steps) {
                        ++p.steps;
                        ddmc_event(p, c, tb, a);
                    }
                }
            }
        }
    }
}

__global__ void reset_queue(unsigned long long *work)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) work[0] = 0ull;
}

}  // namespace

hipError_t launch_walk3d(const uint8_t *d_tables, const DevHeader &h, const rddmc_run &run, uint64_t first,
                         uint64_t count, unsigned long long *d_tally, unsigned long long *d_work, hipStream_t s)
{
    Walk3Args a;
    a.first = first;
    a.count = count;
    a.max_steps = run.max_steps;
    a.key0 = (uint32_t)run.seed;
    a.key1 = (uint32_t)(run.seed >> 32);
    a.chunk = run.chunk > 0 ? run.chunk : 64;
    a.n_clouds = h.n_clouds;
    a.dom = kDom3D;
    const int block = run.block > 0 ? run.block : 256;
    uint64_t grid = run.grid > 0 ? (uint64_t)run.grid : 0;
    if (grid == 0) {
        const uint64_t want = (count + block - 1) / block;
        const uint64_t cap = (uint64_t)device_cu_count() * 8;
        grid = want < cap ? want : cap;
        if (grid < 1) grid = 1;
    }
    reset_queue<<<1, 64, 0, s>>>(d_work);
    if (h.n_clouds == 1)
        walk3d<true><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    else
        walk3d<false><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    return hipGetLastError();
}

}  // namespace rddmc
