// FP64 device line physics for the table build (Sec. 2.1-2.2, eqs. 12-14).
//
// Dawson's integral F(x) = exp(-x^2) int_0^x exp(y^2) dy is evaluated from the
// mathematics:
//   |x| < 0.2 : its Maclaurin series  sum_n (-2)^n x^(2n+1) / (2n+1)!!
//   |x| > 50  : its asymptotic series (1/2x) sum_k (2k-1)!! / (2x^2)^k
//   otherwise : Rybicki's (1989) sampling-theorem representation
//               F(x) = lim_{h->0} pi^(-1/2) sum_{n odd} exp(-(x - n h)^2) / n,
//               with h = 1/4 (aliasing error ~ exp(-(pi/2h)^2) ~ 1e-17), the sum
//               centred on the even integer n0 nearest x/h and its exponentials built
//               from two by recurrence.
// erf/erfc are the HIP device library's.
#pragma once

#include <hip/hip_runtime.h>

namespace rddmc {

__device__ __forceinline__ double dawson_dev(double x)
{
    const double ax = fabs(x);
    const double sgn = x < 0.0 ? -1.0 : 1.0;
    if (ax < 0.2) {
        const double x2 = x * x;
        double term = x, sum = x;
        for (int n = 1; n < 14; ++n) {
            term *= -2.0 * x2 / (2.0 * n + 1.0);
            sum += term;
        }
        return sum;
    }
    if (ax > 50.0) {
        const double q = 1.0 / (2.0 * ax * ax);
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < 9; ++k) {
            term *= (2.0 * k - 1.0) * q;
            sum += term;
        }
        return sgn * sum / (2.0 * ax);
    }
    constexpr double h = 0.25;
    constexpr int M = 27;                        // odd offsets m = +-1 .. +-M: |m h| <= 6.75
    const double n0 = 2.0 * rint(0.5 * ax / h);  // nearest even integer to ax/h
    const double xp = ax - n0 * h;               // |xp| <= h
    const double e1 = exp(2.0 * h * xp);         // exp(2 h xp m) = e1^m
    const double e1sq = e1 * e1;
    const double hh = h * h;
    double up = e1, dn = 1.0 / e1;               // e1^m and e1^-m for m = 1
    double sum = 0.0;
    for (int m = 1; m <= M; m += 2) {
        const double g = exp(-(double)(m * m) * hh);
        sum += g * (up / (n0 + m) + dn / (n0 - m));
        up *= e1sq;
        dn /= e1sq;
    }
    return sgn * 0.56418958354775628695 * exp(-xp * xp) * sum;   // 1/sqrt(pi)
}

// calH(a, x) = int_0^x H(a, y) dy with H of eq. (12): eq. (13).
__device__ __forceinline__ double hcal_dev(double a, double x)
{
    return 0.88622692545275801365 * erf(x) - 1.12837916709551257390 * a * dawson_dev(x) +
           a * a * x * exp(-x * x);
}

// calH(a, hi) - calH(a, lo) for 0 <= lo <= hi; the Gaussian part through erfc in the wings.
__device__ __forceinline__ double hcal_diff_nonneg(double a, double lo, double hi)
{
    double g = (lo > 1.0) ? (erfc(lo) - erfc(hi)) : (erf(hi) - erf(lo));
    g *= 0.88622692545275801365;                         // sqrt(pi)/2
    const double d = -1.12837916709551257390 * a * (dawson_dev(hi) - dawson_dev(lo));   // 2/sqrt(pi)
    const double s = a * a * (hi * exp(-hi * hi) - lo * exp(-lo * lo));
    return g + d + s;
}

// calH(a, hi) - calH(a, lo) for lo <= hi of any signs (calH is odd).
__device__ __forceinline__ double hcal_diff_dev(double a, double lo, double hi)
{
    if (lo >= 0.0) return hcal_diff_nonneg(a, lo, hi);
    if (hi <= 0.0) return hcal_diff_nonneg(a, -hi, -lo);
    return hcal_dev(a, hi) + hcal_dev(a, -lo);
}

// a(T) and v_th(T) of Sec. 2.1.
__device__ __forceinline__ double damping_dev(double T) { return 4.702e-4 * sqrt(1.0e4 / T); }
__device__ __forceinline__ double vth_dev(double T) { return 12.85 * sqrt(T / 1.0e4); }

}  // namespace rddmc
