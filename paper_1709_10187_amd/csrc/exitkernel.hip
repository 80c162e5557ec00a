// Exact per-cell exit kernel: the law of a DDMC packet's walk inside one cell of a 1D cloud
// (Sec. 2.3, eqs. 11 and 15-16) from its entry bin to its first spatial leak, tabulated per
// window state (cell i, entry bin j) so that the walk can replace that whole sub-walk by one
// draw (the same hook as the learned surrogate).
//
// Inside cell i the walk is a birth-death chain on the bins with jump probabilities
// q_dn(k) = D_k / 2^64, q_up(k) = (S_k - D_k) / 2^64 (the walk's own integer thresholds) and
// leak probabilities p_f(k) through face f, holding times of mean 1/K_k = (ln2/K)_k / ln2 (the
// walk's own f32 path-length factor).  With A = I - Q:
//   P(face f, exit bin j' | j)      = [A^-T e_j](j') p_f(j')                       (w1)
//   E[T 1{exit bin j'} | j]         = [A^-T D A^-T e_j](j') p_s(j')                (w2)
//   E[T^2 1{exit bin j'} | j]       = 2 [A^-T D A^-T D A^-T e_j](j') p_s(j')       (w3)
// with D = diag(1/K).  A is an M-matrix; its LU factors are computed with pivots in the form
// piv_k = psi_k + q_up(k), psi_k = p_s(k) + q_dn(k) psi_{k-1} / piv_{k-1}, so that every
// elimination and substitution adds non-negative terms: no cancellation even when p_s is
// 1e-12 (very thick cells).  FP64 throughout.
//
// A row keeps the exit bins [j_lo, j_lo + m) outside of which every bin's leak probability is
// below the caller's tail (the kept law is renormalised), as a CDF over (face 0, bins...),
// (face 1, bins...) and, per exit bin, the exact conditional mean m1 = E[T | j'] and squared
// coefficient of variation c2 = E[T^2 | j'] / m1^2 - 1 of the time spent.
#include <hip/hip_runtime.h>

#include "philox.h"
#include "rddmc_internal.h"
#include "surrogate_dev.h"

namespace rddmc {
namespace {

constexpr int kEkArrays = 7;   // per-bin arrays of a cell: q_dn, q_up, p_f0, p_f1, 1/K, piv, n_steps
constexpr int EK_QDN = 0, EK_QUP = 1, EK_PF0 = 2, EK_PF1 = 3, EK_INVK = 4, EK_PIV = 5, EK_NST = 6;

__device__ __forceinline__ double u64_frac(uint64_t v) { return (double)v * 5.421010862427522e-20; }   // 2^-64

// Per cell (one thread each): the chain's probabilities from the hot records, the GTH-form
// pivots and the expected number of steps before a spatial leak from every bin, n = A^-1 1.
// cb[(a * nb + k) * nc + i]: array a, bin k, cell i.
__global__ void ek_prep(const uint8_t *__restrict__ tb, DevCloud c, double *__restrict__ cb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = c.nc, nb = c.nb;
    if (i >= nc) return;
    const uint4 *hot = reinterpret_cast<const uint4 *>(tb + c.off_hot) + (int64_t)i * nb;
    const uint4 *low = reinterpret_cast<const uint4 *>(tb + c.off_lo_words) + (int64_t)i * nb;
    auto at = [&](int a, int k) -> double & { return cb[((int64_t)a * nb + k) * nc + i]; };
    double psi_prev = 0.0, piv_prev = 1.0;
    for (int k = 0; k < nb; ++k) {
        const uint4 h = hot[k], l = low[k];
        const uint64_t D = ((uint64_t)h.y << 32) | l.x;
        const uint64_t S = ((uint64_t)h.z << 32) | l.y;
        const uint64_t F = ((uint64_t)h.w << 32) | l.z;
        const double qdn = u64_frac(D), qup = u64_frac(S - D);
        const double pf0 = u64_frac(F - S);
        // 2^64 - F as the complement of F in 64 bits (F = 0 would mean a full face-1 band)
        const double pf1 = F == 0ull ? 1.0 - qdn - qup - pf0 : u64_frac((uint64_t)0 - F);
        const double ps = pf0 + pf1;
        const double psi = ps + (k > 0 ? qdn * psi_prev / piv_prev : 0.0);
        const double piv = psi + qup;
        at(EK_QDN, k) = qdn;
        at(EK_QUP, k) = qup;
        at(EK_PF0, k) = pf0;
        at(EK_PF1, k) = pf1;
        at(EK_INVK, k) = (double)__uint_as_float(h.x) * 1.4426950408889634;   // (ln2/K) / ln2
        at(EK_PIV, k) = piv;
        psi_prev = psi;
        piv_prev = piv;
    }
    // n = A^-1 1: forward y_k = 1 + q_dn(k) y_{k-1} / piv_{k-1}, back n_k = (y_k + q_up(k) n_{k+1}) / piv_k
    double y = 0.0;
    for (int k = 0; k < nb; ++k) {
        y = 1.0 + (k > 0 ? at(EK_QDN, k) * y / at(EK_PIV, k - 1) : 0.0);
        at(EK_NST, k) = y;
    }
    double nxt = 0.0;
    for (int k = nb - 1; k >= 0; --k) {
        nxt = (at(EK_NST, k) + (k < nb - 1 ? at(EK_QUP, k) * nxt : 0.0)) / at(EK_PIV, k);
        at(EK_NST, k) = nxt;
    }
}

// Per bin: the smallest expected sub-walk length over cells [i_lo, i_hi].
__global__ void ek_minsteps(const double *__restrict__ cb, int nc, int nb, int i_lo, int i_hi, double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    double m = INFINITY;
    for (int i = i_lo; i <= i_hi; ++i) m = fmin(m, cb[((int64_t)EK_NST * nb + k) * nc + i]);
    out[k] = m;
}

// w <- A^-T b in place (w holds b on entry), the thread's vector strided by `st`.
__device__ void solve_t(const double *__restrict__ cb, int nc, int nb, int i, double *w, int64_t st, int k0)
{
    auto at = [&](int a, int k) { return cb[((int64_t)a * nb + k) * nc + i]; };
    // U^T z = b: z_k = (b_k + q_up(k-1) z_{k-1}) / piv_k   (b_k = 0 below k0)
    double z = 0.0;
    for (int k = k0; k < nb; ++k) {
        z = (w[k * st] + (k > k0 ? at(EK_QUP, k - 1) * z : 0.0)) / at(EK_PIV, k);
        w[k * st] = z;
    }
    // L^T v = z: v_k = z_k + (q_dn(k+1) / piv_k) v_{k+1}
    double v = w[(int64_t)(nb - 1) * st];
    for (int k = nb - 2; k >= 0; --k) {
        v = (k >= k0 ? w[k * st] : 0.0) + at(EK_QDN, k + 1) / at(EK_PIV, k) * v;
        w[k * st] = v;
    }
}

// One thread per window state q of the chunk [q0, q0 + cnt): cell i = i_lo + q / nj, entry bin
// j = j_lo + q % nj.  Scratch: three vectors of nb doubles per thread, interleaved by thread.
// count mode (rows == nullptr): writes {j_lo', m} of the kept exit bins into span[q - q0];
// write mode: writes the row of state q at rows + recs[q].row_off.
__global__ void ek_rows(const double *__restrict__ cb, int nc, int nb, int i_lo, int j_lo, int nj, uint64_t q0,
                        uint64_t cnt, double tail, double *__restrict__ scratch, int2 *__restrict__ span,
                        const ExitRec *__restrict__ recs, uint8_t *__restrict__ rows)
{
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const uint64_t q = q0 + t;
    const int i = i_lo + (int)(q / nj), j = j_lo + (int)(q % nj);
    auto at = [&](int a, int k) { return cb[((int64_t)a * nb + k) * nc + i]; };
    const int64_t st = (int64_t)cnt;
    double *w1 = scratch + t;
    double *w2 = w1 + (int64_t)nb * st;
    double *w3 = w2 + (int64_t)nb * st;
    for (int k = 0; k < nb; ++k) w1[k * st] = k == j ? 1.0 : 0.0;
    solve_t(cb, nc, nb, i, w1, st, j);
    if (!rows) {
        int lo = nb, hi = -1;
        for (int k = 0; k < nb; ++k) {
            const double pk = w1[k * st] * (at(EK_PF0, k) + at(EK_PF1, k));
            if (pk >= tail) {
                lo = min(lo, k);
                hi = k;
            }
        }
        if (hi < lo) lo = hi = j;   // cannot happen for a law that sums to 1 over <= nb bins
        span[t] = make_int2(lo, hi - lo + 1);
        return;
    }
    for (int k = 0; k < nb; ++k) w2[k * st] = at(EK_INVK, k) * w1[k * st];
    solve_t(cb, nc, nb, i, w2, st, 0);
    for (int k = 0; k < nb; ++k) w3[k * st] = at(EK_INVK, k) * w2[k * st];
    solve_t(cb, nc, nb, i, w3, st, 0);
    const ExitRec r = recs[q];
    double *cdf = reinterpret_cast<double *>(rows + r.row_off);
    float2 *tp = reinterpret_cast<float2 *>(cdf + 2 * r.m);
    double z = 0.0;
    for (int f = 0; f < 2; ++f)
        for (int k = 0; k < r.m; ++k) z += w1[(int64_t)(r.j_lo + k) * st] * at(f ? EK_PF1 : EK_PF0, r.j_lo + k);
    double acc = 0.0;
    for (int f = 0; f < 2; ++f)
        for (int k = 0; k < r.m; ++k) {
            acc += w1[(int64_t)(r.j_lo + k) * st] * at(f ? EK_PF1 : EK_PF0, r.j_lo + k);
            cdf[f * r.m + k] = fmin(acc / z, 1.0);
        }
    cdf[2 * r.m - 1] = 1.0;
    for (int k = 0; k < r.m; ++k) {
        const int64_t o = (int64_t)(r.j_lo + k) * st;
        const double a1 = w1[o];
        float2 par = make_float2(0.0f, 0.0f);
        if (a1 > 0.0) {
            const double m1 = w2[o] / a1, m2 = 2.0 * w3[o] / a1;
            par = make_float2((float)m1, (float)fmax(0.0, m2 / (m1 * m1) - 1.0));
        }
        tp[k] = par;
    }
}

// Training samples of the learned surrogate drawn from the exact in-cell law (for cells whose
// sub-walks are too long to run): thread t owns pair t = (cloud pc[t], cell * nb + bin ps[t])
// and writes cnt[t] samples at rows off[t] .. off[t] + cnt[t] - 1 of x [., 16] (the state's
// features) and y [., 3] = (face, asinh(x_out / S), ln(dt / w)) with x_out uniform in the exit
// bin and dt from the moment-matched law of the walk's exit kernel.  Scratch: 11 nb doubles
// per thread (chain arrays, three solves, the CDF), interleaved.  Random words: Philox keyed by
// (seed, pair) with the sample index as counter.
__global__ void ek_samples(const uint8_t *__restrict__ tb, const int32_t *__restrict__ pc,
                           const int32_t *__restrict__ ps, const int32_t *__restrict__ cnt,
                           const int64_t *__restrict__ off, uint64_t n_pairs, uint32_t k0, uint32_t k1,
                           int nb_max, double *__restrict__ scratch, float *__restrict__ xo, float *__restrict__ yo)
{
    const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (t >= n_pairs) return;
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud &c = reinterpret_cast<const DevCloud *>(tb + H->off_clouds)[pc[t]];
    const int nb = c.nb;
    const int i = ps[t] / nb, j = ps[t] - i * nb;
    const int64_t st = (int64_t)n_pairs;
    auto arr = [&](int a) { return scratch + (int64_t)a * nb_max * st + t; };
    double *qdn = arr(0), *qup = arr(1), *pf0 = arr(2), *pf1 = arr(3), *ik = arr(4), *pv = arr(5);
    double *w1 = arr(6), *w2 = arr(7), *w3 = arr(8), *cdf = arr(9);   // cdf spans arrays 9 and 10
    const uint4 *hot = reinterpret_cast<const uint4 *>(tb + c.off_hot) + (int64_t)i * nb;
    const uint4 *low = reinterpret_cast<const uint4 *>(tb + c.off_lo_words) + (int64_t)i * nb;
    double psi_prev = 0.0, piv_prev = 1.0;
    for (int k = 0; k < nb; ++k) {
        const uint4 h = hot[k], l = low[k];
        const uint64_t D = ((uint64_t)h.y << 32) | l.x;
        const uint64_t S = ((uint64_t)h.z << 32) | l.y;
        const uint64_t F = ((uint64_t)h.w << 32) | l.z;
        const double a_dn = u64_frac(D), a_up = u64_frac(S - D), a0 = u64_frac(F - S);
        const double a1 = F == 0ull ? 1.0 - a_dn - a_up - a0 : u64_frac((uint64_t)0 - F);
        const double psi = a0 + a1 + (k > 0 ? a_dn * psi_prev / piv_prev : 0.0);
        qdn[k * st] = a_dn;
        qup[k * st] = a_up;
        pf0[k * st] = a0;
        pf1[k * st] = a1;
        ik[k * st] = (double)__uint_as_float(h.x) * 1.4426950408889634;
        pv[k * st] = psi + a_up;
        psi_prev = psi;
        piv_prev = psi + a_up;
    }
    // w <- A^-T b (b in w; zero below k0), as solve_t with this thread's arrays
    auto solve = [&](double *w, int kb) {
        double z = 0.0;
        for (int k = kb; k < nb; ++k) {
            z = (w[k * st] + (k > kb ? qup[(k - 1) * st] * z : 0.0)) / pv[k * st];
            w[k * st] = z;
        }
        double v = w[(int64_t)(nb - 1) * st];
        for (int k = nb - 2; k >= 0; --k) {
            v = (k >= kb ? w[k * st] : 0.0) + qdn[(k + 1) * st] / pv[k * st] * v;
            w[k * st] = v;
        }
    };
    for (int k = 0; k < nb; ++k) w1[k * st] = k == j ? 1.0 : 0.0;
    solve(w1, j);
    for (int k = 0; k < nb; ++k) w2[k * st] = ik[k * st] * w1[k * st];
    solve(w2, 0);
    for (int k = 0; k < nb; ++k) w3[k * st] = ik[k * st] * w2[k * st];
    solve(w3, 0);
    double acc = 0.0;
    for (int f = 0; f < 2; ++f)
        for (int k = 0; k < nb; ++k) {
            acc += w1[k * st] * (f ? pf1[k * st] : pf0[k * st]);
            cdf[((int64_t)f * nb + k) * st] = acc;
        }
    float feat[kSurrIn];
    float Sc, wd;
    surr_features(c, tb, i, j, feat, Sc, wd);
    const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
    for (int q = 0; q < cnt[t]; ++q) {
        const u32x4 r = philox4x32_10((uint32_t)q, 0x51u, (uint32_t)t, (uint32_t)(t >> 32), k0, k1);
        const double u = (double)r.x * 2.3283064365386962890625e-10 * acc;
        int lo = 0, hi = 2 * nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (u < cdf[(int64_t)mid * st]) hi = mid; else lo = mid + 1;
        }
        const int face = lo >= nb ? 1 : 0;
        const int jo = lo - face * nb;
        const double a1 = w1[(int64_t)jo * st];
        const double m1 = a1 > 0.0 ? w2[(int64_t)jo * st] / a1 : 0.0;
        const double c2 = a1 > 0.0 ? fmax(0.0, 2.0 * w3[(int64_t)jo * st] / (a1 * m1 * m1) - 1.0) : 0.0;
        const double ex = -log(((double)(r.w >> 8) + 0.5) * 5.9604644775390625e-8);
        double dt;
        if (c2 <= 1.0) {
            const double b = m1 * sqrt(c2);
            dt = (m1 - b) + b * ex;
        } else {
            const double qq = 1.0 / ((1.0 + c2) * (1.0 + sqrt((c2 - 1.0) / (c2 + 1.0))));
            const double uc = ((double)(r.y >> 8) + 0.5) * 5.9604644775390625e-8;
            dt = (uc < qq ? m1 / (2.0 * qq) : m1 / (2.0 * (1.0 - qq))) * ex;
        }
        const double xout = e[jo] + (e[jo + 1] - e[jo]) * (((double)(r.z >> 8) + 0.5) * 5.9604644775390625e-8);
        const int64_t row = off[t] + q;
        for (int f = 0; f < kSurrIn; ++f) xo[row * kSurrIn + f] = feat[f];
        yo[row * 3 + 0] = (float)face;
        yo[row * 3 + 1] = (float)asinh(xout / (double)Sc);
        yo[row * 3 + 2] = (float)log(fmax(dt, 1e-300) / (double)wd);
    }
}

}  // namespace

hipError_t launch_ek_samples(const uint8_t *d_tables, const int32_t *d_pc, const int32_t *d_ps, const int32_t *d_cnt,
                             const int64_t *d_off, uint64_t n_pairs, uint64_t seed, int nb_max, double *d_scratch,
                             float *d_x, float *d_y, hipStream_t s)
{
    ek_samples<<<(unsigned)((n_pairs + 63) / 64), 64, 0, s>>>(d_tables, d_pc, d_ps, d_cnt, d_off, n_pairs,
                                                              (uint32_t)seed, (uint32_t)(seed >> 32), nb_max,
                                                              d_scratch, d_x, d_y);
    return hipGetLastError();
}

hipError_t launch_ek_prep(const uint8_t *d_tables, const DevCloud &c, double *d_cb, hipStream_t s)
{
    ek_prep<<<(c.nc + 63) / 64, 64, 0, s>>>(d_tables, c, d_cb);
    return hipGetLastError();
}

hipError_t launch_ek_minsteps(const double *d_cb, int nc, int nb, int i_lo, int i_hi, double *d_out, hipStream_t s)
{
    ek_minsteps<<<(nb + 255) / 256, 256, 0, s>>>(d_cb, nc, nb, i_lo, i_hi, d_out);
    return hipGetLastError();
}

hipError_t launch_ek_rows(const double *d_cb, int nc, int nb, int i_lo, int j_lo, int nj, uint64_t q0, uint64_t cnt,
                          double tail, double *d_scratch, int2 *d_span, const ExitRec *d_recs, uint8_t *d_rows,
                          hipStream_t s)
{
    ek_rows<<<(unsigned)((cnt + 63) / 64), 64, 0, s>>>(d_cb, nc, nb, i_lo, j_lo, nj, q0, cnt, tail, d_scratch, d_span,
                                                        d_recs, d_rows);
    return hipGetLastError();
}

}  // namespace rddmc
