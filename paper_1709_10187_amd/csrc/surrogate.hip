// Per-state tables of the learned escape surrogate: the network's inputs for every state of
// every cloud's surrogate window, and, from the network's raw outputs, the sampling record
// the walk reads (component CDF, per-component face probability, Gaussian parameters of
// y1 and y2 with their correlation, and the state's scales S and w).
#include <hip/hip_runtime.h>

#include "rddmc_internal.h"
#include "surrogate_dev.h"

namespace rddmc {

namespace {

__global__ void surr_features_kernel(const uint8_t *__restrict__ tb, const uint8_t *__restrict__ surr,
                                     uint64_t first, uint64_t count, float *__restrict__ X,
                                     float *__restrict__ SW)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const uint64_t g = first + t;
    const SurrHeader *SH = reinterpret_cast<const SurrHeader *>(surr);
    const SurrCloud *sc = reinterpret_cast<const SurrCloud *>(surr + SH->off_clouds);
    int lo = 0, hi = SH->n_clouds;          // last cloud whose first record is <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sc[mid].rec_off <= g) lo = mid; else hi = mid;
    }
    const SurrCloud w = sc[lo];
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud &c = reinterpret_cast<const DevCloud *>(tb + H->off_clouds)[lo];
    const int nj = w.j_hi - w.j_lo + 1;
    const int64_t r = (int64_t)(g - w.rec_off);
    const int i = w.i_lo + (int)(r / nj), j = w.j_lo + (int)(r % nj);
    float f[kSurrIn], S, wd;
    surr_features(c, tb, i, j, f, S, wd);
    for (int k = 0; k < kSurrIn; ++k) X[t * kSurrIn + k] = f[k];
    SW[2 * t] = S;
    SW[2 * t + 1] = wd;
}

__global__ void surr_records_kernel(const float *__restrict__ o, const float *__restrict__ SW, uint64_t count,
                                    float *__restrict__ rec)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const float *q = o + t * 128;
    float *r = rec + t * kSurrRec;
    float amax = -INFINITY;
    for (int k = 0; k < 16; ++k) amax = fmaxf(amax, q[k]);
    float e[16], sum = 0.0f;
    for (int k = 0; k < 16; ++k) {
        e[k] = __expf(q[k] - amax);
        sum += e[k];
    }
    float cum = 0.0f;
    for (int k = 0; k < 16; ++k) {
        cum += e[k];
        r[kRecCdf + k] = k == 15 ? 1.0f : cum / sum;
        const float f0 = q[16 + 2 * k], f1 = q[17 + 2 * k];
        r[kRecPf0 + k] = 1.0f / (1.0f + __expf(f1 - f0));
        r[kRecMu1 + k] = q[48 + k];
        r[kRecSg1 + k] = __expf(fminf(fmaxf(q[64 + k], -6.0f), 4.0f));
        r[kRecMu2 + k] = q[80 + k];
        r[kRecSg2 + k] = __expf(fminf(fmaxf(q[96 + k], -6.0f), 4.0f));
        r[kRecRho + k] = 0.95f * tanhf(q[112 + k]);
    }
    r[kRecS] = SW[2 * t];
    r[kRecW] = SW[2 * t + 1];
    for (int k = kRecW + 1; k < kSurrRec; ++k) r[k] = 0.0f;
}

}  // namespace

hipError_t launch_surr_features(const uint8_t *d_tables, const uint8_t *d_surr, uint64_t first, uint64_t count,
                                float *d_x, float *d_sw, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    surr_features_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(d_tables, d_surr, first, count, d_x, d_sw);
    return hipGetLastError();
}

hipError_t launch_surr_records(const float *d_out, const float *d_sw, uint64_t count, float *d_rec, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    surr_records_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(d_out, d_sw, count, d_rec);
    return hipGetLastError();
}

}  // namespace rddmc
