// Discrete frequency redistribution for frequency-group Monte Carlo (Sec. 5.3, eq. 42), with
// the redistribution function R_II-A of Appendix A (isotropic scattering, coherent in the
// atom's frame, no recoil), built in FP64 for one isothermal cloud.
//
// A packet of bin j' has its frequency uniform over the bin (eq. 42 averages flatly over both
// bins); the probability of outgoing bin j is
//     P(j | j') = (1 / dx_j') int_{bin j'} N_j(x') / N(x') dx',
// where N_j(x') is the appendix's u-integral taken over the outgoing x in [x1, x2] (bin 0 open
// below, bin nb-1 open above: the grid is closed by its edge bins) and N(x') the same over all
// x.  Exchanging the x- and u-integrations makes N_j one integral over u of elementary
// functions: with A(y) = int_0^y atan(t / a) dt = y atan(y / a) - (a / 2) ln(1 + (y / a)^2),
//     N_j(x') = int_0^inf exp(-u^2) G_j(u) du,
//     G_j(u) = [(hi - lo) atan((x' + u) / a) - A(hi - u) + A(lo - u)]  over x in [x', x' + 2u]
//            + [A(hi + u) - A(lo + u) - (hi - lo) atan((x' - u) / a)]  over x in [x' - 2u, x'),
// each part on its overlap [lo, hi] with [x1, x2]; over all x the A terms cancel and
//     N(x') = int_0^inf exp(-u^2) 2u [atan((x' + u) / a) - atan((x' - u) / a)] du = pi H(a, x'),
// so the normalisation of R_II-A comes out of the same quadrature, with no Voigt function.
//
// Quadrature: 20-point Gauss-Legendre rules on the segments between breakpoints, both for u and
// for the average over x'.  The breakpoints are the points where an integration domain changes
// (kinks) and the points where an arctangent's argument changes sign (steps ~a wide), the latter
// with graded neighbours at 1, 8, 64 and 512 a on either side.  u runs from where the domain
// opens (half the distance between the bins) to 6.5 beyond, where exp(-u^2) has fallen by more
// than e^-42; pairs of bins more than 13 apart get probability 0 (below e^-42).
//
// Sampling table: per incoming bin a Walker alias table (Vose's construction) over the row
// normalised by its computed sum: entry col = {threshold, alias} with threshold = q_col 2^32
// (rounded, capped at 2^32 - 1); a draw takes col from one 32-bit word (its product with nb,
// high half) and keeps col when a second word is below the threshold, else takes the alias.
#include <hip/hip_runtime.h>

#include "linemath_dev.h"
#include "rddmc_internal.h"

namespace rddmc {

namespace {

constexpr int kGl = 20;                 // Gauss-Legendre order
constexpr int kMaxPts = 64;             // breakpoints of one integral
constexpr double kUSpan = 6.5;          // u range beyond the opening point
constexpr double kFarBins = 13.0;       // bin distance beyond which P(j | j') < e^-42
constexpr int kGrades = 4;             // graded neighbours at 8^g a, g < kGrades
constexpr double kMaxSeg = 0.5;         // longest piece of one Gauss-Legendre rule

__device__ const double *f64c(const uint8_t *tb, uint64_t off) { return reinterpret_cast<const double *>(tb + off); }

// The positive nodes and weights of the kGl-point Gauss-Legendre rule, by Newton's method on
// the Legendre polynomial P_kGl (three-term recurrence) from Tricomi's initial guesses.
__device__ void gauss_legendre(double *x, double *w, int i)
{
    const int n = kGl;
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (fabs(dz) < 1e-17) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
}

// A(y) = int_0^y atan(t / a) dt
__device__ __forceinline__ double anti_atan(double y, double a)
{
    const double r = y / a;
    return y * atan(r) - 0.5 * a * log1p(r * r);
}

// The bracket of R_II-A integrated over the outgoing x in [x1, x2] at atom parameter u.
__device__ double g_bin(double u, double xp, double x1, double x2, double a)
{
    double g = 0.0;
    double lo = fmax(x1, xp), hi = fmin(x2, xp + 2.0 * u);
    if (hi > lo) g += (hi - lo) * atan((xp + u) / a) - (anti_atan(hi - u, a) - anti_atan(lo - u, a));
    lo = fmax(x1, xp - 2.0 * u);
    hi = fmin(x2, xp);
    if (hi > lo) g += (anti_atan(hi + u, a) - anti_atan(lo + u, a)) - (hi - lo) * atan((xp - u) / a);
    return g;
}

// Sorted breakpoints of [lo, hi]: the ends, the kinks, and the steps with their graded
// neighbours (those strictly inside).
struct Pts {
    double v[kMaxPts];
    int n;
    double lo, hi;
    __device__ void init(double l, double h)
    {
        lo = l;
        hi = h;
        v[0] = l;
        v[1] = h;
        n = 2;
    }
    __device__ void add(double q)
    {
        if (q > lo && q < hi && n < kMaxPts) v[n++] = q;
    }
    __device__ void step(double b, double a)
    {
        add(b);
        double d = a;
        for (int g = 0; g < kGrades; ++g, d *= 8.0) {
            add(b - d);
            add(b + d);
        }
    }
    __device__ void sort()
    {
        for (int i = 1; i < n; ++i) {
            const double t = v[i];
            int k = i - 1;
            while (k >= 0 && v[k] > t) {
                v[k + 1] = v[k];
                --k;
            }
            v[k + 1] = t;
        }
    }
};

// int over the segments of P of f(u) by the Gauss-Legendre rule (xg, wg: positive half), each
// segment cut into equal pieces of at most kMaxSeg (the integrands vary on the Doppler scale 1:
// exp(-u^2), or exp(x'^2) erfc(|x|) across a wide central bin)
template <typename F>
__device__ double integrate(const Pts &P, const double *xg, const double *wg, F f)
{
    double tot = 0.0;
    for (int s = 0; s + 1 < P.n; ++s) {
        const double p = P.v[s], q = P.v[s + 1];
        if (!(q > p)) continue;
        const int m = (int)ceil((q - p) / kMaxSeg);
        const double hw = (q - p) / m;
        for (int t = 0; t < m; ++t) {
            const double h = 0.5 * hw, c = p + (t + 0.5) * hw;
            double acc = 0.0;
            for (int i = 0; i < kGl / 2; ++i) acc += wg[i] * (f(c - h * xg[i]) + f(c + h * xg[i]));
            tot += h * acc;
        }
    }
    return tot;
}

__device__ bool finite_edge(double e) { return e > -1e300 && e < 1e300; }

// N_j(x') / N(x') for the outgoing bin [x1, x2] (x1 = -inf / x2 = +inf for the edge bins)
__device__ double bin_fraction(double xp, double x1, double x2, double a, const double *xg, const double *wg)
{
    const bool f1 = finite_edge(x1), f2 = finite_edge(x2);
    double umin = 0.0;
    if (f1) umin = fmax(umin, 0.5 * (x1 - xp));
    if (f2) umin = fmax(umin, 0.5 * (xp - x2));
    Pts P;
    P.init(umin, umin + kUSpan);
    P.step(xp, a);
    P.step(-xp, a);
    if (f1) {
        P.step(x1, a);
        P.step(-x1, a);
        P.add(0.5 * (x1 - xp));
        P.add(0.5 * (xp - x1));
    }
    if (f2) {
        P.step(x2, a);
        P.step(-x2, a);
        P.add(0.5 * (x2 - xp));
        P.add(0.5 * (xp - x2));
    }
    P.sort();
    const double nj = integrate(P, xg, wg, [&](double u) { return exp(-u * u) * g_bin(u, xp, x1, x2, a); });
    Pts Q;
    Q.init(0.0, kUSpan);
    Q.step(fabs(xp), a);
    Q.sort();
    const double nall = integrate(Q, xg, wg, [&](double u) {
        return exp(-u * u) * 2.0 * u * (atan((xp + u) / a) - atan((xp - u) / a));
    });
    return nj / nall;
}

// One wave per (incoming bin jp, outgoing bin j): P(j | jp) into prob[jp * nb + j].
__global__ __launch_bounds__(64) void redist_prob(DevCloud c, uint8_t *__restrict__ tb, uint32_t *__restrict__ err)
{
    __shared__ double xg[kGl / 2], wg[kGl / 2];
    const int lane = threadIdx.x;
    if (lane < kGl / 2) gauss_legendre(xg, wg, lane);
    __syncthreads();
    const int nb = c.nb;
    const int64_t e = blockIdx.x;
    const int jp = (int)(e / nb), j = (int)(e - (int64_t)jp * nb);
    double *prob = reinterpret_cast<double *>(tb + c.off_grp_prob);
    const double *ed = f64c(tb, c.off_edges);
    const double a = damping_dev(f64c(tb, c.off_T)[0]);
    const double p0 = ed[jp], p1 = ed[jp + 1];
    const double x1 = j == 0 ? -INFINITY : ed[j], x2 = j == nb - 1 ? INFINITY : ed[j + 1];
    const double gap = fmax(fmax(x1 - p1, p0 - x2), 0.0);
    if (gap > kFarBins) {
        if (lane == 0) prob[e] = 0.0;
        return;
    }
    Pts O;
    O.init(p0, p1);
    if (finite_edge(x1)) {
        O.add(x1);
        O.step(-x1, a);
    }
    if (finite_edge(x2)) {
        O.add(x2);
        O.step(-x2, a);
    }
    O.sort();
    // outer nodes (piece t of the segments cut as in integrate(), node k of kGl) spread over
    // the lanes in a fixed order
    int pieces[kMaxPts];
    int np = 0;
    for (int s = 0; s + 1 < O.n; ++s) {
        const double len = O.v[s + 1] - O.v[s];
        pieces[s] = len > 0.0 ? (int)ceil(len / kMaxSeg) : 0;
        np += pieces[s];
    }
    double part = 0.0;
    for (int q = lane; q < np * kGl; q += 64) {
        int t = q / kGl, s = 0;
        const int k = q - t * kGl;
        while (t >= pieces[s]) t -= pieces[s++];
        const double hw = (O.v[s + 1] - O.v[s]) / pieces[s];
        const double h = 0.5 * hw, cen = O.v[s] + (t + 0.5) * hw;
        const int i = k < kGl / 2 ? k : k - kGl / 2;
        const double xq = k < kGl / 2 ? cen - h * xg[i] : cen + h * xg[i];
        part += h * wg[i] * bin_fraction(xq, x1, x2, a, xg, wg);
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if (lane == 0) {
        const double v = part / (p1 - p0);
        if (!(v >= 0.0) || !(v <= 1.0 + 1e-9)) atomicOr(err, (uint32_t)BE_NONFINITE);
        prob[e] = v;
    }
}

constexpr int kMaxGroupBins = RDDMC_MAX_GROUP_BINS;

// One block per incoming bin: normalise the row and build its alias table (Vose), in LDS.
__global__ __launch_bounds__(64) void redist_alias(DevCloud c, uint8_t *__restrict__ tb, uint32_t *__restrict__ err)
{
    __shared__ double q[kMaxGroupBins];
    __shared__ int small[kMaxGroupBins], large[kMaxGroupBins];
    if (threadIdx.x != 0) return;
    const int nb = c.nb, jp = blockIdx.x;
    const double *prob = f64c(tb, c.off_grp_prob) + (int64_t)jp * nb;
    uint2 *al = reinterpret_cast<uint2 *>(tb + c.off_grp_alias) + (int64_t)jp * nb;
    double sum = 0.0;
    for (int j = 0; j < nb; ++j) sum += prob[j];
    if (!(sum > 0.5) || !(sum < 1.5)) {
        atomicOr(err, (uint32_t)BE_NONFINITE);
        sum = 1.0;
    }
    int ns = 0, nl = 0;
    for (int j = 0; j < nb; ++j) {
        q[j] = prob[j] / sum * nb;
        if (q[j] < 1.0) small[ns++] = j; else large[nl++] = j;
    }
    auto thr = [](double v) -> uint32_t {
        const double t = rint(v * 4294967296.0);
        return t >= 4294967295.0 ? 0xffffffffu : (t <= 0.0 ? 0u : (uint32_t)t);
    };
    while (ns > 0 && nl > 0) {
        const int s = small[--ns], l = large[--nl];
        al[s] = make_uint2(thr(q[s]), (uint32_t)l);
        q[l] = (q[l] + q[s]) - 1.0;
        if (q[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) {   // what is left is 1 up to rounding
        const int l = large[--nl];
        al[l] = make_uint2(0xffffffffu, (uint32_t)l);
    }
    while (ns > 0) {
        const int s = small[--ns];
        al[s] = make_uint2(0xffffffffu, (uint32_t)s);
    }
}

}  // namespace

hipError_t launch_build_redistribution(const DevCloud &c, uint8_t *d_tables, hipStream_t s)
{
    if (!c.groups) return hipSuccess;
    uint32_t *err = &reinterpret_cast<DevHeader *>(d_tables)->error_flags;
    const uint64_t elems = (uint64_t)c.nb * c.nb;
    redist_prob<<<(unsigned)elems, 64, 0, s>>>(c, d_tables, err);
    redist_alias<<<(unsigned)c.nb, 64, 0, s>>>(c, d_tables, err);
    return hipGetLastError();
}

}  // namespace rddmc
