// FP64 leakage-table build (Sec. 2.2: eqs. 10, 11, 13, 14; the hybrid section's
// thin/vacuum-face rate; Sec. 2.5: comoving-frame shift across faces).
//
// Three passes, one thread per item, coalesced over the fastest index (the bin):
//   build_maps : per (cell, face) neighbour Doppler map x' = rho x + shift and the
//                outward normal velocity u_n (in thermal units) for escapes;
//   build_k    : per state the tophat bin-averaged opacity k_ij (eq. 14);
//   build_rates: per state the face and frequency leakage rates, packed into the
//                16-byte hot record and the face-split thresholds;
//   build_mcell: (3D and 1D hybrid) per cell the FP32 record of the continuous-MC step;
// and, once per buffer of a batch with MC states, the FP32 Voigt and sampler tables.
#include <hip/hip_runtime.h>

#include "linemath_dev.h"
#include "rddmc_internal.h"

namespace rddmc {

namespace {

__device__ __forceinline__ const double *f64p(const uint8_t *base, uint64_t off)
{
    return reinterpret_cast<const double *>(base + off);
}

// Geometry of a 1D or 3D cell across face f: neighbour code (>= 0 cell, -1 vacuum,
// -2 no face), the cell's width across the face and the face-area / volume ratio.
struct FaceGeom {
    int64_t nbr;
    double width, area_over_vol, normal_sign;
    int axis;
};

__device__ FaceGeom face_geom(const DevCloud &c, const uint8_t *tb, int64_t cell, int f)
{
    FaceGeom g;
    g.normal_sign = (f & 1) ? 1.0 : -1.0;
    if (c.geometry == RDDMC_SLAB || c.geometry == RDDMC_SPHERE) {
        const double *fz = f64p(tb, c.off_faces[0]);
        const double lo = fz[cell], hi = fz[cell + 1];
        g.axis = 0;
        g.width = hi - lo;
        if (f == 0) {
            g.nbr = cell > 0 ? cell - 1 : -1;
        } else {
            g.nbr = cell < c.nc - 1 ? cell + 1 : -1;
        }
        if (c.geometry == RDDMC_SLAB) {
            g.area_over_vol = 1.0 / g.width;
        } else {
            const double v3 = (hi * hi * hi - lo * lo * lo) / 3.0;
            const double r = (f == 0) ? lo : hi;
            g.area_over_vol = r * r / v3;
            if (f == 0 && cell == 0 && lo == 0.0) g.nbr = -2;
        }
        return g;
    }
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int64_t ix = cell % nx, iy = (cell / nx) % ny, iz = cell / ((int64_t)nx * ny);
    const int axis = f >> 1;
    const int64_t idx[3] = {ix, iy, iz};
    const int nn[3] = {nx, ny, nz};
    const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
    const double *fa = f64p(tb, c.off_faces[axis]);
    g.axis = axis;
    g.width = fa[idx[axis] + 1] - fa[idx[axis]];
    g.area_over_vol = 1.0 / g.width;
    if (f & 1) {
        g.nbr = idx[axis] < nn[axis] - 1 ? cell + stride[axis] : -1;
    } else {
        g.nbr = idx[axis] > 0 ? cell - stride[axis] : -1;
    }
    return g;
}

__device__ double min_width(const DevCloud &c, const uint8_t *tb, int64_t cell)
{
    if (c.geometry != RDDMC_CART3D) {
        const double *fz = f64p(tb, c.off_faces[0]);
        return fz[cell + 1] - fz[cell];
    }
    const int nx = c.n[0], ny = c.n[1];
    const int64_t ix = cell % nx, iy = (cell / nx) % ny, iz = cell / ((int64_t)nx * ny);
    const double wx = f64p(tb, c.off_faces[0])[ix + 1] - f64p(tb, c.off_faces[0])[ix];
    const double wy = f64p(tb, c.off_faces[1])[iy + 1] - f64p(tb, c.off_faces[1])[iy];
    const double wz = f64p(tb, c.off_faces[2])[iz + 1] - f64p(tb, c.off_faces[2])[iz];
    return fmin(wx, fmin(wy, wz));
}

// v . n for cell `cell` through face f (km/s).
__device__ double normal_velocity(const DevCloud &c, const uint8_t *tb, int64_t cell, int f)
{
    if (!c.moving) return 0.0;
    const double *v = f64p(tb, c.off_vel);
    const double sgn = (f & 1) ? 1.0 : -1.0;
    if (c.geometry != RDDMC_CART3D) return sgn * v[cell];
    return sgn * v[cell * 3 + (f >> 1)];
}

__global__ void build_maps(DevCloud c, uint8_t *tb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)c.nc * c.nf) return;
    const int64_t cell = t / c.nf;
    const int f = (int)(t % c.nf);
    const double *T = f64p(tb, c.off_T);
    double *map = reinterpret_cast<double *>(tb + c.off_map) + 3 * t;
    const FaceGeom g = face_geom(c, tb, cell, f);
    const double vn_c = normal_velocity(c, tb, cell, f);
    double rho = 1.0, shift = 0.0;
    if (g.nbr >= 0) {
        const double Tn = T[g.nbr];
        rho = sqrt(T[cell] / Tn);
        const double vn_n = normal_velocity(c, tb, g.nbr, f);
        shift = -c.f_mu * (vn_n - vn_c) / vth_dev(Tn);          // eq. 20 with f_mu
    }
    map[0] = rho;
    map[1] = shift;
    map[2] = vn_c / vth_dev(T[cell]);
    if (c.nf == 2) {   // compact per-cell copy read together with the hot record
        float *cm = reinterpret_cast<float *>(tb + c.off_cmap) + 4 * cell + 2 * f;
        cm[0] = (float)rho;
        cm[1] = (float)shift;
    }
}

__global__ void build_k(DevCloud c, uint8_t *tb, uint32_t *err)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (int64_t)c.n_states) return;
    const int64_t cell = s / c.nb;
    const int j = (int)(s % c.nb);
    const double *e = f64p(tb, c.off_edges);
    const double lo = e[j], hi = e[j + 1];
    const double a = damping_dev(f64p(tb, c.off_T)[cell]);
    double k = f64p(tb, c.off_k0)[cell] * hcal_diff_dev(a, lo, hi) / (hi - lo);
    if (c.dusty) k += f64p(tb, c.off_dust)[2 * cell + 1];   // total scattering: Lya + dust (Sec. 2.4)
    reinterpret_cast<double *>(tb + c.off_k)[s] = k;
    if (!(k > 0.0) || !isfinite(k)) atomicOr(err, (uint32_t)BE_NONFINITE);
}

__device__ __forceinline__ uint32_t frac_to_u31(double p)
{
    if (!(p > 0.0)) return 0u;
    if (p >= 1.0) return 0x80000000u;
    return (uint32_t)rint(p * 2147483648.0);
}

__device__ __forceinline__ uint64_t prob_to_u64(double p)
{   // round(p * 2^64), saturating at 2^64 - 1
    const double v = p * 18446744073709551616.0;
    if (!(v > 0.0)) return 0ull;
    if (!(v < 18446744073709551616.0)) return ~0ull;
    return (uint64_t)rint(v);
}

__global__ void build_rates(DevCloud c, uint8_t *tb, uint32_t *err)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (int64_t)c.n_states) return;
    const int nb = c.nb, nf = c.nf;
    const int64_t cell = s / nb;
    const int j = (int)(s % nb);
    const double *e = f64p(tb, c.off_edges);
    const double *kk = f64p(tb, c.off_k);
    const double *k0 = f64p(tb, c.off_k0);
    const double *T = f64p(tb, c.off_T);
    const double *map = f64p(tb, c.off_map);
    const double lo = e[j], hi = e[j + 1], dx = hi - lo;
    const double ks = kk[s];
    const bool hybrid = c.tau_th > 0.0;
    const bool flagged = c.flag_layout != 0;
    const bool thick = !hybrid || ks * min_width(c, tb, cell) >= c.tau_th;
    if (!thick) {
        if (!flagged) {   // the pure 1D walk has no continuous-MC states
            atomicOr(err, (uint32_t)BE_THIN);
            return;
        }
        // a continuous-MC state: no DDMC rates, flags = 0 (not thick)
        reinterpret_cast<HotRecord *>(tb + c.off_hot)[s] = HotRecord{0.0f, 0u, 0u, 0u};
        reinterpret_cast<uint4 *>(tb + c.off_lo_words)[s] = make_uint4(0u, 0u, 0u, 0u);
        uint32_t *fs = reinterpret_cast<uint32_t *>(tb + c.off_face_split) + s * (nf - 1);
        for (int f = 0; f < nf - 1; ++f) fs[f] = 0u;
        if (c.keep_rates) {
            double *rr = reinterpret_cast<double *>(tb + c.off_rates) + s * (nf + 2);
            for (int f = 0; f < nf + 2; ++f) rr[f] = 0.0;
        }
        return;
    }

    double rf[kMaxFaces];
    double rs = 0.0;
    uint32_t iface = 0u;     // faces whose leak enters a thin state or vacuum
    for (int f = 0; f < nf; ++f) {
        const FaceGeom g = face_geom(c, tb, cell, f);
        const double kw = ks * g.width;
        double r;
        if (g.nbr == -2) {
            r = 0.0;
        } else if (g.nbr == -1) {
            r = c.dirichlet ? g.area_over_vol * 2.0 / (3.0 * kw)
                            : g.area_over_vol * 2.0 / (3.0 * (kw + 2.0 * c.lambda));
            iface |= 1u << f;
        } else {
            const double rho = map[3 * (cell * nf + f)];
            const double sh = map[3 * (cell * nf + f) + 1];
            double kn;
            if (rho == 1.0 && sh == 0.0) {
                kn = kk[g.nbr * nb + j];
            } else {   // neighbour opacity over the shifted image of the bin (eq. 14 again)
                const double a_n = damping_dev(T[g.nbr]);
                const double l2 = rho * lo + sh, h2 = rho * hi + sh;
                kn = k0[g.nbr] * hcal_diff_dev(a_n, l2, h2) / (h2 - l2);
                if (c.dusty) kn += f64p(tb, c.off_dust)[2 * g.nbr + 1];
            }
            const FaceGeom gn = face_geom(c, tb, g.nbr, f ^ 1);
            const bool nb_thick = !hybrid || kn * min_width(c, tb, g.nbr) >= c.tau_th;
            r = nb_thick ? g.area_over_vol * 2.0 / (3.0 * (kw + kn * gn.width))      // eq. 10
                         : g.area_over_vol * 2.0 / (3.0 * (kw + 2.0 * c.lambda));
            if (!nb_thick) iface |= 1u << f;
        }
        rf[f] = r;
        rs += r;
    }
    double rd = 0.0, ru = 0.0;
    if (j > 0) {
        const double dxm = e[j] - e[j - 1];
        rd = 1.0 / (dx * (dx / ks + dxm / kk[s - 1]));                            // eq. 11
    }
    if (j < nb - 1) {
        const double dxp = e[j + 2] - e[j + 1];
        ru = 1.0 / (dx * (dx / ks + dxp / kk[s + 1]));
    }
    // dust absorption rate: one more exponential channel, unless absorption is carried by
    // continuous weights (then the walk's interaction distances ignore it)
    const double ka = (c.dusty && !c.dust_weight) ? f64p(tb, c.off_dust)[2 * cell] : 0.0;
    const double K = rs + rd + ru + ka;
    if (!(K > 0.0) || !isfinite(K)) atomicOr(err, (uint32_t)BE_NONFINITE);

    // categorical thresholds in units of 2^-64: D = P(lower), S = 1 - P(spatial) - P(absorb),
    // F = S + P(face 0) (the face-0 / face-1 boundary of 1D cells); with dust the spatial
    // leaks end at A = 1 - P(absorb) and absorption takes [A, 2^64)
    const uint64_t D = prob_to_u64(rd / K);
    const uint64_t Tab = prob_to_u64(ka / K);
    const uint64_t A = 0ull - Tab;                  // 2^64 - Tab (0 = no absorption)
    uint64_t Tsp = prob_to_u64(rs / K);
    uint64_t S;
    if (rs + ka >= K) {
        S = 0ull;                                   // every leak is spatial or an absorption (one bin)
    } else {
        if (Tsp == 0ull) Tsp = 1ull;                // keep the spatial leak reachable
        S = 0ull - Tsp - Tab;                       // 2^64 - Tsp - Tab
        if (S < D || ru <= 0.0) S = D;              // no upper move from the last bin, even by rounding
    }
    // face 1 gets [F, 2^64); saturate if rounding leaves it less than nothing
    uint64_t F = S + prob_to_u64(rf[0] / K);
    if (F < S || rf[1] <= 0.0) F = ~0ull;
    HotRecord h;
    h.ln2_over_K = (float)(0.69314718055994530942 / K);
    h.d_hi = (uint32_t)(D >> 32);
    h.s_hi = (uint32_t)(S >> 32);
    uint32_t flags = kFlagThick | (iface << kFlagFaceShift);
    if (flagged && hybrid) {
        const double wmin = min_width(c, tb, cell);
        if (j > 0 && kk[s - 1] * wmin < c.tau_th) flags |= kFlagDnThin;
        if (j < nb - 1 && kk[s + 1] * wmin < c.tau_th) flags |= kFlagUpThin;
    }
    h.f_hi = flagged ? flags : (uint32_t)(F >> 32);
    reinterpret_cast<HotRecord *>(tb + c.off_hot)[s] = h;
    uint32_t *lw = reinterpret_cast<uint32_t *>(tb + c.off_lo_words) + 4 * s;
    lw[0] = (uint32_t)D;
    lw[1] = (uint32_t)S;
    lw[2] = flagged ? (uint32_t)A : (uint32_t)F;
    lw[3] = flagged ? (uint32_t)(A >> 32) : 0u;

    // cumulative face split: thresholds for faces 0 .. nf-2
    uint32_t *fsplit = reinterpret_cast<uint32_t *>(tb + c.off_face_split) + s * (nf - 1);
    double cum = 0.0;
    for (int f = 0; f < nf - 1; ++f) {
        cum += rf[f];
        fsplit[f] = rs > 0.0 ? frac_to_u31(cum / rs) : 0x80000000u;
    }
    if (c.keep_rates) {
        double *rr = reinterpret_cast<double *>(tb + c.off_rates) + s * (nf + 2);
        for (int f = 0; f < nf; ++f) rr[f] = rf[f];
        rr[nf] = rd;
        rr[nf + 1] = ru;
    }
}

// Per-cell FP32 record of the continuous-MC step: {k0, a, sqrt(T), w_min} and the bulk
// velocity in units of the cell's own thermal speed (1D: its component along +z or +r).
__global__ void build_mcell(DevCloud c, uint8_t *tb)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)c.nc) return;
    const double T = f64p(tb, c.off_T)[cell];
    const double vth = vth_dev(T);
    float4 *mc = reinterpret_cast<float4 *>(tb + c.off_mcell) + 2 * cell;
    mc[0] = make_float4((float)f64p(tb, c.off_k0)[cell], (float)damping_dev(T), (float)sqrt(T),
                        (float)min_width(c, tb, cell));
    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c.moving && c.geometry == RDDMC_CART3D) {
        const double *v = f64p(tb, c.off_vel) + 3 * cell;
        u = make_float4((float)(v[0] / vth), (float)(v[1] / vth), (float)(v[2] / vth), 0.f);
    } else if (c.moving) {
        u.x = (float)(f64p(tb, c.off_vel)[cell] / vth);
    }
    if (c.dusty) {   // 1D: dust scattering and absorption coefficients of the MC flight
        u.y = (float)f64p(tb, c.off_dust)[2 * cell + 1];
        u.z = (float)f64p(tb, c.off_dust)[2 * cell];
    }
    mc[1] = u;
}

// H1(x) = (2/sqrt(pi)) (2 x F(x) - 1), the first-order term of eq. 12 in a, on x = i/256.
__global__ void build_voigt_table(float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kVoigtN) return;
    const double x = (double)i / (double)kVoigtScale;
    out[i] = (float)(1.12837916709551257390 * (2.0 * x * dawson_dev(x) - 1.0));
}

// Proposal mass of the atom-velocity sampler split at u0 (times pi/a): the Lorentzian
// centred on |x| below u0 plus exp(-u0^2) times the Lorentzian above u0.
__device__ double split_mass(double a, double ax, double u0)
{
    const double th = atan((u0 - ax) / a);
    return (1.57079632679489661923 + th) + exp(-u0 * u0) * (1.57079632679489661923 - th);
}

// Split point minimising the proposal mass over [0, |x|] (golden-section search).
__global__ void build_u0_table(float *out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kU0NA * kU0NX) return;
    const int ia = t / kU0NX, ix = t % kU0NX;
    const double a = pow(10.0, -6.0 + ia / (double)kU0Scale);
    const double ax = ix / (double)kU0Scale;
    const double g = 0.61803398874989484820;
    double lo = 0.0, hi = ax;
    double c1 = hi - g * (hi - lo), c2 = lo + g * (hi - lo);
    double f1 = split_mass(a, ax, c1), f2 = split_mass(a, ax, c2);
    for (int it = 0; it < 60; ++it) {
        if (f1 < f2) {
            hi = c2; c2 = c1; f2 = f1; c1 = hi - g * (hi - lo); f1 = split_mass(a, ax, c1);
        } else {
            lo = c1; c1 = c2; f1 = f2; c2 = lo + g * (hi - lo); f2 = split_mass(a, ax, c2);
        }
    }
    out[t] = (float)(0.5 * (lo + hi));
}

__global__ void zero_words(unsigned long long *d, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        d[i] = 0ull;
}

}  // namespace

hipError_t launch_build(const DevCloud &c, int cloud_index, uint8_t *d_tables, hipStream_t s)
{
    (void)cloud_index;
    uint32_t *err = &reinterpret_cast<DevHeader *>(d_tables)->error_flags;
    const int bs = 256;
    const int64_t nmap = (int64_t)c.nc * c.nf;
    build_maps<<<(unsigned)((nmap + bs - 1) / bs), bs, 0, s>>>(c, d_tables);
    const int64_t ns = (int64_t)c.n_states;
    const unsigned g = (unsigned)((ns + bs - 1) / bs);
    build_k<<<g, bs, 0, s>>>(c, d_tables, err);
    build_rates<<<g, bs, 0, s>>>(c, d_tables, err);
    if (c.off_mcell)
        build_mcell<<<(unsigned)((c.nc + bs - 1) / bs), bs, 0, s>>>(c, d_tables);
    return hipGetLastError();
}

hipError_t launch_build_line_tables(const DevHeader &h, uint8_t *d_tables, hipStream_t s)
{
    if (h.off_voigt == 0) return hipSuccess;
    build_voigt_table<<<(kVoigtN + 255) / 256, 256, 0, s>>>(reinterpret_cast<float *>(d_tables + h.off_voigt));
    build_u0_table<<<(kU0NA * kU0NX + 255) / 256, 256, 0, s>>>(reinterpret_cast<float *>(d_tables + h.off_u0));
    return hipGetLastError();
}

hipError_t launch_zero(void *d, size_t words64, hipStream_t s)
{
    if (words64 == 0) return hipSuccess;
    size_t blocks = (words64 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    zero_words<<<(unsigned)blocks, 256, 0, s>>>(reinterpret_cast<unsigned long long *>(d), words64);
    return hipGetLastError();
}

}  // namespace rddmc
