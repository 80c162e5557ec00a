// The learned escape surrogate's device-side definitions, shared by the data generator,
// the per-state table build and the walk: the network's input features of a DDMC state,
// the target scalings, and the layout of the sampling records.
//
// A state (cell i, bin j) of a 1D cloud is described by
//   f0 = (log10 tau_c - 6) / 1.5      tau_c = k0_i w_i, the cell's line-centre optical width
//   f1 = (log10 a + 3.3) / 0.6        Voigt damping parameter of the cell
//   f2 = x_j / 3                      centre of the entry bin (Doppler units)
//   f3 = log10(dx_j) / 0.7            width of the entry bin
//   f4, f5 = s_0, s_1                 Doppler shifts of eq. 20 into the neighbours across
//                                     faces 0 and 1 (the cell's own frame moves by them)
//   f6, f7 = 4 (g_f - 1)              face geometry g_f = (A_f / dV_i) w_i (1 for slabs)
// and the exit it learns as y1 = asinh(x_out / S), S = (a tau_c)^(1/3), x_out the exit
// frequency in the cell's frame (uniform in the exit bin), and y2 = ln(dt / w_i).
#pragma once

#include <hip/hip_runtime.h>

#include "linemath_dev.h"
#include "rddmc_internal.h"

namespace rddmc {

constexpr int kSurrIn = 16;
constexpr int kSurrRec = 128;      // floats per state record
// record: [0,16) component CDF, [16,32) P(face 0 | k), [32,48) mu1, [48,64) sigma1,
//         [64,80) mu2, [80,96) sigma2, [96,112) rho, [112] S, [113] w
constexpr int kRecCdf = 0, kRecPf0 = 16, kRecMu1 = 32, kRecSg1 = 48, kRecMu2 = 64, kRecSg2 = 80, kRecRho = 96,
              kRecS = 112, kRecW = 113;

// Surrogate window of one cloud: states (i, j) with i_lo <= i <= i_hi, j_lo <= j <= j_hi
// (empty when i_hi < i_lo); their records start at record index rec_off.
struct alignas(16) SurrCloud {
    int32_t i_lo, i_hi, j_lo, j_hi;
    uint64_t rec_off;
    uint64_t pad;
};

constexpr int32_t kSurrMdn = 0;     // records: learned mixture laws (kSurrRec floats each)
constexpr int32_t kSurrExact = 1;   // records: ExitRec headers of exact exit-kernel rows

struct alignas(16) SurrHeader {
    int32_t n_clouds;
    int32_t kind;            // kSurrMdn or kSurrExact
    uint64_t off_clouds;     // SurrCloud [n_clouds]
    uint64_t off_records;    // kSurrMdn: float [n_records * kSurrRec]; kSurrExact: ExitRec [n_records]
    uint64_t n_records;
    uint64_t off_rows;       // kSurrExact: the row pool (ExitRec.row_off is relative to it)
    uint64_t pad;
};

// Exact exit-kernel row of one window state: 2m doubles, the CDF over (face 0, exit bins
// j_lo .. j_lo+m-1) then (face 1, the same bins), then m float2 {mu, sigma} of the lognormal
// exit time given the exit bin.
struct ExitRec {
    uint64_t row_off;        // bytes from SurrHeader.off_rows
    int32_t j_lo, m;
};

// Exit-kernel builders (exitkernel.hip): per-cell chain arrays d_cb (7 nb nc doubles), the
// per-bin minimum of the expected sub-walk length over cells [i_lo, i_hi], and per window
// state either the kept exit-bin span (d_rows == nullptr) or the row.
hipError_t launch_ek_prep(const uint8_t *d_tables, const DevCloud &c, double *d_cb, hipStream_t s);
hipError_t launch_ek_minsteps(const double *d_cb, int nc, int nb, int i_lo, int i_hi, double *d_out, hipStream_t s);
hipError_t launch_ek_samples(const uint8_t *d_tables, const int32_t *d_pc, const int32_t *d_ps, const int32_t *d_cnt,
                             const int64_t *d_off, uint64_t n_pairs, uint64_t seed, int nb_max, double *d_scratch,
                             float *d_x, float *d_y, hipStream_t s);
hipError_t launch_ek_rows(const double *d_cb, int nc, int nb, int i_lo, int j_lo, int nj, uint64_t q0, uint64_t cnt,
                          double tail, double *d_scratch, int2 *d_span, const ExitRec *d_recs, uint8_t *d_rows,
                          hipStream_t s);

__device__ inline void surr_features(const DevCloud &c, const uint8_t *tb, int i, int j, float *f, float &S,
                                     float &w)
{
    const double *fz = reinterpret_cast<const double *>(tb + c.off_faces[0]);
    const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
    const double *map = reinterpret_cast<const double *>(tb + c.off_map);
    const double lo = fz[i], hi = fz[i + 1];
    const double wd = hi - lo;
    const double T = reinterpret_cast<const double *>(tb + c.off_T)[i];
    const double a = damping_dev(T);
    const double tau_c = reinterpret_cast<const double *>(tb + c.off_k0)[i] * wd;
    double g0 = 1.0, g1 = 1.0;
    if (c.geometry == RDDMC_SPHERE) {
        const double v3 = (hi * hi * hi - lo * lo * lo) / 3.0;
        g0 = lo * lo / v3 * wd;
        g1 = hi * hi / v3 * wd;
    }
    for (int q = 0; q < kSurrIn; ++q) f[q] = 0.0f;
    f[0] = (float)((log10(tau_c) - 6.0) / 1.5);
    f[1] = (float)((log10(a) + 3.3) / 0.6);
    f[2] = (float)(0.5 * (e[j] + e[j + 1]) / 3.0);
    f[3] = (float)(log10(e[j + 1] - e[j]) / 0.7);
    f[4] = (float)map[3 * (2 * (int64_t)i + 0) + 1];
    f[5] = (float)map[3 * (2 * (int64_t)i + 1) + 1];
    f[6] = (float)(4.0 * (g0 - 1.0));
    f[7] = (float)(4.0 * (g1 - 1.0));
    S = (float)cbrt(a * tau_c);
    w = (float)wd;
}

}  // namespace rddmc
