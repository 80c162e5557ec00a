// Device helpers shared by the hybrid walks (3D Cartesian and 1D slab / shell grids): the
// per-packet counter-based random stream, uniform and exponential draws, the FP32 line
// profile of eq. 12 from its table, the atom-velocity sampler of the MC scattering,
// isotropic directions, and the frequency-bin lookup.
#pragma once

#include <hip/hip_runtime.h>

#include "philox.h"
#include "rddmc_internal.h"

namespace rddmc {
namespace mc {

constexpr float kPi = 3.14159265358979f;
constexpr float kHalfPi = 1.57079632679490f;
constexpr float kTwoPi = 6.28318530717959f;
constexpr int kUparMaxTries = 1 << 20;          // the sampler's acceptance is >= ~1e-3

// Launch arguments of the hybrid walks: packet range, step cap, Philox key (the run's seed),
// steps between refills, number of clouds, and the counter domain of the walk's streams.
struct McArgs {
    uint64_t first, count, max_steps;
    uint32_t key0, key1;
    int32_t chunk, n_clouds;
    uint32_t dom;
};

// Per-packet stream: block b is Philox4x32-10 of counter (b_lo, dom | b_hi, packet id,
// cloud key) under the run's seed; its four words are used in order, each once.  The block
// being read (c0..c3, next word at index `idx`) is followed by a block generated ahead of
// need (n0..n3, valid when `ahead`): a pass generates every lane's next block at its start,
// so the whole wave issues Philox together; a draw generates in place only when the lane
// ran through both.
struct Rng {
    uint32_t c0, c1, c2, c3;
    uint32_t n0, n1, n2, n3;
    uint32_t idx;
    bool ahead;
    uint32_t ctr, ctr_hi;
    uint32_t pid, key;
};

__device__ __forceinline__ u32x4 next_block(Rng &r, const McArgs &a)
{
    const u32x4 b = philox4x32_10(r.ctr, a.dom | r.ctr_hi, r.pid, r.key, a.key0, a.key1);
    if (++r.ctr == 0u) ++r.ctr_hi;
    return b;
}

// Generate the block after the current one unless it is already there.
__device__ __forceinline__ void prefetch(Rng &r, const McArgs &a)
{
    if (!r.ahead) {
        const u32x4 b = next_block(r, a);
        r.n0 = b.x;
        r.n1 = b.y;
        r.n2 = b.z;
        r.n3 = b.w;
        r.ahead = true;
    }
}

__device__ __forceinline__ uint32_t draw(Rng &r, const McArgs &a)
{
    if (r.idx == 4u) {
        if (r.ahead) {
            r.c0 = r.n0;
            r.c1 = r.n1;
            r.c2 = r.n2;
            r.c3 = r.n3;
            r.ahead = false;
        } else {
            const u32x4 b = next_block(r, a);
            r.c0 = b.x;
            r.c1 = b.y;
            r.c2 = b.z;
            r.c3 = b.w;
        }
        r.idx = 0u;
    }
    const uint32_t v = r.idx == 0u ? r.c0 : (r.idx == 1u ? r.c1 : (r.idx == 2u ? r.c2 : r.c3));
    ++r.idx;
    return v;
}

// 24-bit uniform in (0, 1) (exactly representable, never 0 or 1)
__device__ __forceinline__ float uf(uint32_t w) { return ((float)(w >> 8) + 0.5f) * 5.9604644775390625e-8f; }
__device__ __forceinline__ double ud(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386962890625e-10; }

__device__ __forceinline__ float ddmc_path(uint32_t tw, float ln2_over_K)
{   // -ln(xi) / K with xi = (tw + 1/2) 2^-32, as -log2(xi) ln2/K
    const float xi = __fmul_rn(__fadd_rn((float)tw, 0.5f), 2.3283064365386963e-10f);
    return __fmul_rn(-__log2f(xi), ln2_over_K);
}

__device__ __forceinline__ float comp(float3 v, int d) { return d == 0 ? v.x : (d == 1 ? v.y : v.z); }
__device__ __forceinline__ int compi(int a, int b, int c, int d) { return d == 0 ? a : (d == 1 ? b : c); }
__device__ __forceinline__ void setc(float3 &v, int d, float s)
{
    v.x = d == 0 ? s : v.x;
    v.y = d == 1 ? s : v.y;
    v.z = d == 2 ? s : v.z;
}
__device__ __forceinline__ float dot3(float3 a, float4 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }

__device__ __forceinline__ const double *faces_of(const DevCloud &c, const uint8_t *tb, int d)
{
    const uint64_t o = d == 0 ? c.off_faces[0] : (d == 1 ? c.off_faces[1] : c.off_faces[2]);
    return reinterpret_cast<const double *>(tb + o);
}

// lab-frame bin of frequency x: -1 below the grid, nb at or above its top edge
__device__ __forceinline__ int bin_of(const DevCloud &c, const uint8_t *tb, float x)
{
    if (c.uniform_bins) {
        const float f = (x - c.x0) * c.inv_dx;
        if (!(f >= 0.0f)) return -1;
        if (f >= (float)c.nb) return c.nb;
        const int j = (int)f;
        return j < c.nb - 1 ? j : c.nb - 1;
    }
    const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
    const double xd = (double)x;
    if (xd < e[0]) return -1;
    if (xd >= e[c.nb]) return c.nb;
    int lo = 0, hi = c.nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (xd >= e[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

// x uniform in bin j
__device__ __forceinline__ float bin_x(const DevCloud &c, const uint8_t *tb, int j, float u)
{
    if (c.uniform_bins) return fmaf((float)j + u, c.dx, c.x0);
    const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
    return (float)(e[j] + (e[j + 1] - e[j]) * (double)u);
}

// H(a, x) of eq. 12 in FP32: exp(-x^2)(1 + a^2 (1 - 2 x^2)) + a H1(|x|), H1 from the table
// below |x| = 16 and from its asymptotic series (1/sqrt(pi)) (1/x^2 + 3/(2x^4) + 15/(4x^6)
// + 105/(8x^8)) above.
__device__ __forceinline__ float voigt_f32(float a, float x, const float *__restrict__ tab)
{
    const float ax = fabsf(x);
    const float x2 = ax * ax;
    float h1;
    if (ax < 16.0f) {
        const float f = ax * kVoigtScale;
        int i = (int)f;
        i = i < kVoigtN - 2 ? i : kVoigtN - 2;
        const float fr = f - (float)i;
        const float t0 = tab[i], t1 = tab[i + 1];
        h1 = fmaf(fr, t1 - t0, t0);
    } else {
        const float q = 1.0f / x2;
        h1 = 0.564189583547756f * q * fmaf(q, fmaf(q, fmaf(q, 13.125f, 3.75f), 1.5f), 1.0f);
    }
    const float e = __expf(-x2);
    return fmaf(a, h1, e * fmaf(a * a, 1.0f - 2.0f * x2, 1.0f));
}

// bilinear split point u0(a, |x|) (clamped to the table; every u0 >= 0 is exact)
__device__ __forceinline__ float u0_of(float a, float ax, const float *__restrict__ tab)
{
    float fa = (__log10f(a) + 6.0f) * kU0Scale;
    fa = fminf(fmaxf(fa, 0.0f), (float)(kU0NA - 1));
    const float fx = fminf(ax * kU0Scale, (float)(kU0NX - 1));
    int ia = (int)fa, ix = (int)fx;
    ia = ia < kU0NA - 2 ? ia : kU0NA - 2;
    ix = ix < kU0NX - 2 ? ix : kU0NX - 2;
    const float ta = fa - (float)ia, tx = fx - (float)ix;
    const float *r0 = tab + ia * kU0NX + ix;
    const float *r1 = r0 + kU0NX;
    const float v0 = fmaf(tx, r0[1] - r0[0], r0[0]);
    const float v1 = fmaf(tx, r1[1] - r1[0], r1[0]);
    return fmaxf(fmaf(ta, v1 - v0, v0), 0.0f);
}

// Atom velocity along the photon direction, density ~ exp(-u^2) / (a^2 + (x - u)^2).
// Lorentzian proposals centred on |x| written as u = |x| - a cot(phi), phi uniform: below
// u0 (phi in (0, phi0)) accepted with exp(-u^2), above (phi in (phi0, pi)) with
// exp(u0^2 - u^2); the branch is chosen by its proposal mass.  Returns false if no
// proposal was accepted within the try limit.
__device__ inline bool sample_upar(float a, float x, const float *__restrict__ u0tab, Rng &r, const McArgs &A,
                            float &out)
{
    const float ax = fabsf(x);
    const float u0 = u0_of(a, ax, u0tab);
    const float phi0 = kHalfPi + atanf((u0 - ax) / a);
    const float e0 = __expf(-u0 * u0);
    const float pl = phi0 / fmaf(e0, kPi - phi0, phi0);
    for (int it = 0; it < kUparMaxTries; ++it) {
        const float r1 = uf(draw(r, A)), r2 = uf(draw(r, A)), r3 = uf(draw(r, A));
        const bool below = r1 <= pl;
        const float phi = below ? r2 * phi0 : fmaf(r2, kPi - phi0, phi0);
        float sn, cs;
        sincosf(phi, &sn, &cs);
        const float uu = ax - a * (cs / sn);
        const float acc = below ? __expf(-uu * uu) : __expf(u0 * u0 - uu * uu);
        if (r3 <= acc) {
            out = x < 0.0f ? -uu : uu;
            return true;
        }
    }
    return false;
}

__device__ __forceinline__ float3 iso_dir(Rng &r, const McArgs &a)
{
    const float mu = fmaf(2.0f, uf(draw(r, a)), -1.0f);
    const float ph = kTwoPi * uf(draw(r, a));
    const float s = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
    float sn, cs;
    sincosf(ph, &sn, &cs);
    return make_float3(s * cs, s * sn, mu);
}

}  // namespace mc
}  // namespace rddmc
