// Persistent rDDMC walk (Sec. 2.3, eqs. 15-16; Sec. 2.5 for moving media).
//
// Every lane carries one packet in registers: cloud, packet id, cell, bin, FP64 clock
// and step count.  A step reads the state's 16-byte hot record and two 32-bit words of
// a Philox4x32-10 block keyed by (seed) and counted by (step pair, packet, cloud); one
// block serves two consecutive steps:
//   time word  -> exponential path length dl = -ln(xi) / K (xi in (0,1), f32 log2),
//   event word -> high word of a u64 uniform U compared with the state's categorical
//                 thresholds D = P(lower bin) 2^64 and S = (1 - P(spatial)) 2^64.
// When the high word decides (all but ~2^-31 of steps) the step is a frequency move;
// otherwise an auxiliary block supplies U's low word, the face choice and any
// re-binning draws.  This samples the same law as taking the smallest of independent
// exponential distances for every possible leak: the minimum is Exp(K) and the winner
// is X with probability k_X / K, independently -- exact to 2^-64 per event, which
// matters because spatial leaks from line-core bins have probabilities ~1e-10.
//
// Every `chunk` steps the wave refills lanes whose packet has finished from a global
// counter (one atomic per wave).  Escapes and step-capped packets add to exact int64
// tallies with device atomics; results depend only on (seed, cloud, packet id).
#include <hip/hip_runtime.h>

#include "philox.h"
#include "rddmc_internal.h"
#include "surrogate_dev.h"

namespace rddmc {

namespace {

struct WalkArgs {
    uint64_t first;        // first flattened packet index of this run
    uint64_t count;        // number of packets in this run
    uint64_t max_steps;
    uint32_t key0, key1;
    int32_t chunk;
    int32_t n_clouds;
    int32_t tail_lanes;    // export a wave's packets once the queue is empty and <= this many remain
    int32_t pad;
    uint64_t tail_capacity;
    const uint8_t *surr;   // learned escape surrogate (windows and records) or null
    uint32_t producer_blocks;   // blocks [0, producer_blocks) walk packets from the queue;
    uint32_t producer_waves;    // later blocks walk handed-over packets cooperatively
};

// Work area (u64 words, the polled ones on their own 128-byte lines): [0] packet queue
// counter, [16] export slots handed out, [17] slots claimed by consumer waves of the
// lane-walk launch, [18] producer waves finished, [24] slots claimed by the closing
// cooperative kernel; export slots start at byte kWorkHeaderBytes.
constexpr uint64_t kWorkHeaderBytes = 256;
constexpr int kWGiven = 16, kWClaimed = 17, kWDone = 18, kWSweep = 24;

// One exported packet.  `flag` moves empty -> ready (published by the exporting lane) ->
// taken (claimed by a walking wave), or empty -> abandoned (a consumer claimed the slot
// before its packet was published and moved on; the exporter then walks it itself).
struct TailPacket {        // 48 bytes
    uint32_t cl, pid;
    int32_t i, j;
    uint64_t steps;
    double t;
    uint32_t flag, surr_calls;   // slot state; surrogate exits the packet took before
    uint64_t pad1;
};
constexpr uint32_t kSlotEmpty = 0u, kSlotReady = 1u, kSlotTaken = 2u, kSlotAbandoned = 3u;
// A consumer wave with nothing to claim polls every 32 x s_sleep 127 (about 0.1 ms) and
// gives up after this many polls in a row (about 100 s); in normal operation it leaves
// much earlier, as soon as every producer wave has finished.
constexpr int kConsumerIdlePolls = 1000000;
// A consumer that claims a slot not yet published re-reads its flag at most this many times
// (s_sleep 2 apart, ~0.2 ms in all) before leaving the packet to its exporter.
constexpr int kPublishWaitPolls = 4096;

// Domain tags in the second counter word (high bits of the step index never reach them).
constexpr uint32_t kDomAux = 0x80000000u;   // extra draws inside step k (re-binning, escape)
constexpr uint32_t kDomEmit = 0xC0000000u;  // emission draw
constexpr uint32_t kDomSurr = 0x40000000u;  // surrogate exit draws (per pair slot)
constexpr uint32_t kDomSub = 0x20000000u;   // sub-walk data: exit frequency inside the exit bin

__device__ __forceinline__ double u01_open_low(uint32_t r)
{   // (r + 0.5) / 2^32 in (0, 1)
    return ((double)r + 0.5) * 2.3283064365386962890625e-10;
}

__device__ __forceinline__ int locate_bin(const double *e, int nb, double x)
{   // j with e[j] <= x < e[j+1]; -1 below the grid, nb at or above the top edge
    if (x < e[0]) return -1;
    if (x >= e[nb]) return nb;
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (x >= e[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int time_bin(double t)
{
    if (!(t >= 1e-3)) return 0;
    const double u = (log10(t) + 3.0) * (RDDMC_TIME_BINS / 9.0);
    if (u >= (double)RDDMC_TIME_BINS) return RDDMC_TIME_BINS + 1;
    return 1 + (int)u;
}

__device__ __forceinline__ int step_bin(uint64_t n)
{
    return n <= 1 ? 0 : 63 - __clzll((long long)n);
}

__device__ void tally_finish(unsigned long long *tally, const DevCloud &c, bool escaped, int row,
                             int slot, double t, uint64_t steps)
{
    unsigned long long *w = tally + c.tally_off;
    if (escaped) {
        atomicAdd(&w[TW_ESCAPED], 1ull);
        atomicAdd(&w[kTallyHeader + (uint64_t)row * (c.nb + 2) + slot], 1ull);
        const unsigned long long tf = (unsigned long long)rint(t * kTimeFix);
        atomicAdd(&w[TW_TSUM], tf);
        const unsigned long long t2 = (unsigned long long)rint(t * t * kTimeFix);
        const unsigned long long old = atomicAdd(&w[TW_T2_LO], t2);
        if (old + t2 < old) atomicAdd(&w[TW_T2_HI], 1ull);
        const uint64_t spec_words = (uint64_t)c.n_rows * (c.nb + 2);
        atomicAdd(&w[kTallyHeader + spec_words + time_bin(t)], 1ull);
    } else {
        atomicAdd(&w[TW_CAPPED], 1ull);
    }
    const uint64_t spec_words = (uint64_t)c.n_rows * (c.nb + 2);
    atomicAdd(&w[kTallyHeader + spec_words + RDDMC_TIME_BINS + 2 + step_bin(steps)], 1ull);
    atomicAdd(&w[TW_STEPS], (unsigned long long)steps);
    atomicMax(&w[TW_STEPS_MAX], (unsigned long long)steps);
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = __shfl((int)(uint32_t)v, src);
    const uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Path length of one step in length units: -ln(xi) / K with xi = (tw + 1/2) / 2^32, as
// -log2(xi) * (ln2 / K).  Written with explicit round-to-nearest operations so that the
// lane walk and the cooperative walk produce the same bits.
__device__ __forceinline__ float path_length(uint32_t tw, float ln2_over_K)
{
    const float xi = __fmul_rn(__fadd_rn((float)tw, 0.5f), 2.3283064365386963e-10f);
    return __fmul_rn(-__log2f(xi), ln2_over_K);
}

// Per-lane packet state of the 1D walk.
struct Packet1D {
    int cl, nb, nc, geom;
    uint32_t pid, key;         // packet id within its cloud; the cloud's stream key
    int i, j;
    double t;
    uint64_t steps;
    const uint4 *hot;          // HotRecord viewed as 4 words
    const float4 *cmap;        // per-cell Doppler maps {rho0, shift0, rho1, shift1}
    float x0, dx, inv_dx;      // uniform bin grid
    bool uniform;
    bool moving;               // the cloud has bulk velocity (one Philox block per step)
    bool active;
    uint32_t surr_calls;       // exits taken from the learned surrogate
};

// The cloud's surrogate window (empty: i_hi < i_lo).
struct SurrWin {
    int i_lo, i_hi, j_lo, j_hi;
    uint64_t rec_off;
};

__device__ __forceinline__ bool in_window(const Packet1D &p, const SurrWin &w)
{
    return (unsigned)(p.i - w.i_lo) <= (unsigned)(w.i_hi - w.i_lo) &&
           (unsigned)(p.j - w.j_lo) <= (unsigned)(w.j_hi - w.j_lo);
}

// Replace the rest of the packet's walk inside its cell by one exit drawn from the learned
// law of the state: mixture component, face, then (y1, y2) from the component's correlated
// Gaussian; x_out = S sinh(y1) in the cell's frame, dt = w exp(y2).  The exit crosses the
// face like a spatial leak (Doppler map of eq. 20 applied to x_out).  It takes a whole
// Philox pair slot (the step count is rounded up to even, then advanced by 2), drawn in
// its own counter domain.
template <bool MOVING>
__device__ void mdn_exit(Packet1D &p, const SurrWin &sw, const float *__restrict__ recs,
                         const uint8_t *__restrict__ tb, const DevCloud &c, const WalkArgs &a)
{
    p.steps = (p.steps + 1ull) & ~1ull;
    const uint64_t pair = p.steps >> 1;
    const u32x4 r = philox4x32_10((uint32_t)pair, kDomSurr | (uint32_t)(pair >> 32), p.pid, p.key, a.key0, a.key1);
    const int64_t idx = (int64_t)sw.rec_off + (int64_t)(p.i - sw.i_lo) * (sw.j_hi - sw.j_lo + 1) + (p.j - sw.j_lo);
    const float *q = recs + idx * kSurrRec;
    const float u0 = ((float)(r.x >> 8) + 0.5f) * 5.9604644775390625e-8f;
    int k = 0;
    while (k < 15 && u0 >= q[kRecCdf + k]) ++k;
    const float uf = ((float)(r.y >> 8) + 0.5f) * 5.9604644775390625e-8f;
    const int face = uf < q[kRecPf0 + k] ? 0 : 1;
    const float ua = ((float)(r.z >> 8) + 0.5f) * 5.9604644775390625e-8f;
    const float ub = ((float)(r.w >> 8) + 0.5f) * 5.9604644775390625e-8f;
    const float rad = sqrtf(-2.0f * __logf(ua));
    float sn, cs;
    sincosf(6.28318530717959f * ub, &sn, &cs);
    const float n1 = rad * cs, n2 = rad * sn;
    const float rho = q[kRecRho + k];
    float y1 = fmaf(q[kRecSg1 + k], n1, q[kRecMu1 + k]);
    float y2 = q[kRecMu2 + k] + q[kRecSg2 + k] * fmaf(rho, n1, sqrtf(fmaxf(0.0f, 1.0f - rho * rho)) * n2);
    y1 = fminf(fmaxf(y1, -20.0f), 20.0f);
    y2 = fminf(y2, 80.0f);
    const float xo = q[kRecS] * sinhf(y1);
    p.t += (double)(q[kRecW] * __expf(y2));
    float xn = xo;
    if (MOVING && p.moving) {
        const float4 cm = p.cmap[p.i];
        xn = fmaf(face ? cm.z : cm.x, xo, face ? cm.w : cm.y);
    }
    int jn;
    if (p.uniform) {
        const float fj = (xn - p.x0) * p.inv_dx;
        jn = !(fj >= 0.0f) ? 0 : (fj >= (float)(p.nb - 1) ? p.nb - 1 : (int)fj);
    } else {
        jn = locate_bin(reinterpret_cast<const double *>(tb + c.off_edges), p.nb, (double)xn);
        jn = jn < 0 ? 0 : (jn > p.nb - 1 ? p.nb - 1 : jn);
    }
    p.j = jn;
    p.i += face ? 1 : -1;
    p.steps += 2ull;
    ++p.surr_calls;
}

// Random words of one step.  Static clouds: one Philox block serves two steps (time and
// event words); moving clouds: one block per step (time, event, re-binning, escape mu).
// The layout is a property of the cloud, so a cloud's packets draw the same numbers in
// whichever kernel variant walks them.
struct StepWords {
    uint32_t t, e, z, w;
};

// Comoving re-binning across face `face` (Sec. 2.5, eq. 20): x uniform in bin j, mapped to
// the neighbour's frame x' = rho x + shift, re-binned and clamped to the grid.
// The neighbour's bin on a uniform grid (before clamping), with explicit rounding so that
// every walker computes the same bits.
__device__ __forceinline__ int rebin_uniform(const Packet1D &p, float rho, float sh, uint32_t zw)
{
    const float u = __fmul_rn(__fadd_rn((float)(zw >> 8), 0.5f), 5.9604644775390625e-8f);   // 24-bit uniform
    const float x = __fmaf_rn(__fadd_rn((float)p.j, u), p.dx, p.x0);
    return (int)floorf(__fmul_rn(__fsub_rn(__fmaf_rn(rho, x, sh), p.x0), p.inv_dx));
}

__device__ __forceinline__ void rebin(Packet1D &p, int face, float4 cm, uint32_t zw,
                                      const DevCloud &c, const uint8_t *__restrict__ tb)
{
    const float rho = face ? cm.z : cm.x;
    const float sh = face ? cm.w : cm.y;
    if (rho == 1.0f && sh == 0.0f) return;
    int jn;
    if (p.uniform) {
        jn = rebin_uniform(p, rho, sh, zw);
    } else {
        const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
        const double x = e[p.j] + (e[p.j + 1] - e[p.j]) * u01_open_low(zw);
        jn = locate_bin(e, p.nb, (double)rho * x + (double)sh);
    }
    p.j = jn < 0 ? 0 : (jn > p.nb - 1 ? p.nb - 1 : jn);
}

// Replace the rest of the packet's walk inside its cell by one exit drawn from the exact law of
// its in-cell walk (the exact exit kernel, same window and check points as the learned
// surrogate): (face, exit bin) from the state's row CDF with a 32-bit uniform, then the spatial
// leak from the exit bin exactly as a walk step takes it (x uniform in the bin and the Doppler
// map of eq. 20 in moving clouds).  The time has the exact conditional mean m1 and squared
// coefficient of variation c2: m1 (1 - sqrt(c2)) + m1 sqrt(c2) E for c2 <= 1, else a balanced
// mixture of two exponentials (probabilities q and 1 - q, means m1 / 2q and m1 / 2(1 - q),
// q = 1 / ((1 + c2)(1 + sqrt((c2 - 1) / (c2 + 1))))), with q on the 2^-24 grid of the uniform
// that picks the branch so that the mean stays m1 exactly.  E = -ln u with u a 24-bit uniform
// (its largest value, 17.3, leaves out 6e-7 of an exponential's mean).  One Philox block in the
// surrogate's counter domain per exit: x for the CDF, y for the branch, z for the re-binning, w
// for E.
template <bool MOVING>
__device__ void exact_exit(Packet1D &p, const SurrWin &sw, const uint8_t *__restrict__ tb, const DevCloud &c,
                           const WalkArgs &a)
{
    p.steps = (p.steps + 1ull) & ~1ull;
    const uint64_t pair = p.steps >> 1;
    const u32x4 r = philox4x32_10((uint32_t)pair, kDomSurr | (uint32_t)(pair >> 32), p.pid, p.key, a.key0, a.key1);
    const SurrHeader *SH = reinterpret_cast<const SurrHeader *>(a.surr);
    const int64_t idx = (int64_t)sw.rec_off + (int64_t)(p.i - sw.i_lo) * (sw.j_hi - sw.j_lo + 1) + (p.j - sw.j_lo);
    const ExitRec er = reinterpret_cast<const ExitRec *>(a.surr + SH->off_records)[idx];
    const double *cdf = reinterpret_cast<const double *>(a.surr + SH->off_rows + er.row_off);
    const double u = (double)r.x * 2.3283064365386962890625e-10;   // [0, 1) on the 2^-32 grid
    int lo = 0, hi = 2 * er.m - 1;   // first outcome whose CDF exceeds u (the last is 1)
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < cdf[mid]) hi = mid; else lo = mid + 1;
    }
    const int face = lo >= er.m ? 1 : 0;
    const int k = lo - face * er.m;
    const float2 tp = reinterpret_cast<const float2 *>(cdf + 2 * er.m)[k];   // {m1, c2}
    const float ex = -__logf(((float)(r.w >> 8) + 0.5f) * 5.9604644775390625e-8f);
    float dt;
    if (tp.y <= 1.0f) {
        const float b = tp.x * sqrtf(tp.y);
        dt = fmaf(b, ex, tp.x - b);
    } else {
        const float q = 1.0f / ((1.0f + tp.y) * (1.0f + sqrtf((tp.y - 1.0f) / (tp.y + 1.0f))));
        const uint32_t nq = (uint32_t)fminf(fmaxf(rintf(q * 16777216.0f), 1.0f), 8388608.0f);
        const float qk = (float)nq * 5.9604644775390625e-8f;
        dt = ((r.y >> 8) < nq ? tp.x / (2.0f * qk) : tp.x / (2.0f * (1.0f - qk))) * ex;
    }
    p.t += (double)dt;
    p.j = er.j_lo + k;
    if (MOVING && p.moving) rebin(p, face, p.cmap[p.i], r.z, c, tb);
    p.i += face ? 1 : -1;
    p.steps += 2ull;
    ++p.surr_calls;
}

// A cell exit from the surrogate buffer: the learned law or the exact kernel.
template <bool MOVING>
__device__ __forceinline__ void surrogate_exit(Packet1D &p, const SurrWin &sw, const float *__restrict__ recs,
                                               const uint8_t *__restrict__ tb, const DevCloud &c, const WalkArgs &a)
{
    if (reinterpret_cast<const SurrHeader *>(a.surr)->kind == kSurrExact)
        exact_exit<MOVING>(p, sw, tb, c, a);
    else
        mdn_exit<MOVING>(p, sw, recs, tb, c, a);
}

// Rare path of a step: the event word tied with a threshold's high word (resolved with an
// auxiliary low word) or an escape.  Returns false when the packet escaped.
template <bool MOVING>
__device__ __forceinline__ bool slow_step(Packet1D &p, StepWords w, uint4 rec, float4 cm,
                                          const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                                          const WalkArgs &a, unsigned long long *__restrict__ tally)
{
    const DevCloud &c = clouds[p.cl];
    const int s = p.i * p.nb + p.j;
    const u32x4 aux = philox4x32_10((uint32_t)p.steps, kDomAux | (uint32_t)(p.steps >> 32), p.pid, p.key,
                                    a.key0, a.key1);
    const uint4 lw = reinterpret_cast<const uint4 *>(tb + c.off_lo_words)[s];
    const uint64_t U = ((uint64_t)w.e << 32) | aux.x;
    const uint64_t D = ((uint64_t)rec.y << 32) | lw.x;
    const uint64_t S = ((uint64_t)rec.z << 32) | lw.y;
    const uint64_t F = ((uint64_t)rec.w << 32) | lw.z;
    if (U < D) { --p.j; ++p.steps; return true; }
    if (U < S) { ++p.j; ++p.steps; return true; }
    // spatial leak: face 0 (lower / inner) or face 1 (upper / outer)
    const int face = (U < F) ? 0 : 1;
    const int ni = face ? p.i + 1 : p.i - 1;
    ++p.steps;
    if (ni < 0 || ni >= p.nc) {
        int slot = p.j + 1;
        if (MOVING && p.moving) {   // lab frame: x uniform in the bin, outward mu uniform in (0, 1]
            const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
            const double un = reinterpret_cast<const double *>(tb + c.off_map)[3 * (p.i * 2 + face) + 2];
            if (un != 0.0) {
                const double x = e[p.j] + (e[p.j + 1] - e[p.j]) * u01_open_low(w.z);
                slot = locate_bin(e, p.nb, x + u01_open_low(w.w) * un) + 1;
            }
        }
        tally_finish(tally, c, true, (p.geom == RDDMC_SLAB) ? face : 0, slot, p.t, p.steps);
        p.active = false;
        return false;
    }
    if (MOVING && p.moving) rebin(p, face, cm, w.z, c, tb);
    p.i = ni;
    return true;
}

// One step with its random words, the state's hot record and (moving media) the cell's
// Doppler map.  Returns -1 / +1 for a frequency move and 2 for a spatial move decided on
// the fast path, 0 for a step that took the slow path.
template <bool MOVING>
__device__ __forceinline__ int one_step(Packet1D &p, StepWords w, uint4 rec, float4 cm,
                                        const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                                        const WalkArgs &a, unsigned long long *__restrict__ tally)
{
    p.t += (double)path_length(w.t, __uint_as_float(rec.x));
    const uint32_t ew = w.e;
    const bool tie = (ew == rec.y) | (ew == rec.z) | (ew == rec.w);
    if (__builtin_expect(!tie, 1)) {
        if (ew < rec.z) {
            const int d = (ew < rec.y) ? -1 : 1;
            p.j += d;
            ++p.steps;
            return d;
        }
        const int face = (ew < rec.w) ? 0 : 1;
        const int ni = face ? p.i + 1 : p.i - 1;
        if ((unsigned)ni < (unsigned)p.nc) {
            if (MOVING && p.moving) rebin(p, face, cm, w.z, clouds[p.cl], tb);
            p.i = ni;
            ++p.steps;
            return 2;
        }
    }
    slow_step<MOVING>(p, w, rec, cm, tb, clouds, a, tally);
    return 0;
}

template <bool MOVING>
__device__ __forceinline__ StepWords words_of_step(const Packet1D &p, uint64_t step, const WalkArgs &a)
{
    if (MOVING && p.moving) {
        const u32x4 r = philox4x32_10((uint32_t)step, (uint32_t)(step >> 32), p.pid, p.key, a.key0, a.key1);
        return {r.x, r.y, r.z, r.w};
    }
    const uint64_t pr = step >> 1;
    const u32x4 r = philox4x32_10((uint32_t)pr, (uint32_t)(pr >> 32), p.pid, p.key, a.key0, a.key1);
    return (step & 1) ? StepWords{r.z, r.w, 0u, 0u} : StepWords{r.x, r.y, 0u, 0u};
}

// A few single steps of one packet (lane-walk arithmetic), used by the cooperative walk on
// static media where spatial leaks dominate (moving media use moving_steps).
template <bool MOVING>
__device__ void single_steps(Packet1D &p, int n, const uint8_t *__restrict__ tb,
                             const DevCloud *__restrict__ clouds, const WalkArgs &a,
                             unsigned long long *__restrict__ tally)
{
    for (int k = 0; k < n && p.active && p.steps < a.max_steps; ++k) {
        const StepWords w = words_of_step<MOVING>(p, p.steps, a);
        const uint4 rec = p.hot[p.i * p.nb + p.j];
        const float4 cm = (MOVING && p.moving) ? p.cmap[p.i] : make_float4(1.f, 0.f, 1.f, 0.f);
        one_step<MOVING>(p, w, rec, cm, tb, clouds, a, tally);
    }
}

// Single steps of one packet with the lane walk's surrogate exits (a step that starts in the
// window is replaced by one exit, at the lane walk's check points), used by the cooperative
// walk where spatial leaks dominate.
template <bool MOVING>
__device__ void surr_single_steps(Packet1D &p, int n, const SurrWin &sw, const float *__restrict__ recs,
                                  const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                                  const WalkArgs &a, unsigned long long *__restrict__ tally)
{
    for (int k = 0; k < n && p.active && p.steps < a.max_steps; ++k) {
        const bool chk = (MOVING && p.moving) || !(p.steps & 1ull);
        if (chk && p.steps + 3ull <= a.max_steps && in_window(p, sw)) {
            surrogate_exit<MOVING>(p, sw, recs, tb, clouds[p.cl], a);
            continue;
        }
        const StepWords w = words_of_step<MOVING>(p, p.steps, a);
        const uint4 rec = p.hot[p.i * p.nb + p.j];
        const float4 cm = (MOVING && p.moving) ? p.cmap[p.i] : make_float4(1.f, 0.f, 1.f, 0.f);
        one_step<MOVING>(p, w, rec, cm, tb, clouds, a, tally);
    }
}

// One step's fast path as selects (no branches): the clock advances for every enabled lane;
// a frequency move or a spatial move inside the grid is applied; returns true when the step
// needs the slow path (a tie with a threshold's high word, or a leak out of the grid), which
// the caller runs.  Disabled lanes change nothing.  The arithmetic is that of one_step.
__device__ __forceinline__ bool select_step(Packet1D &p, bool en, uint32_t tw, uint32_t ew, uint4 rec, int &d)
{
    const double tn = p.t + (double)path_length(tw, __uint_as_float(rec.x));
    p.t = en ? tn : p.t;
    const bool tie = (ew == rec.y) | (ew == rec.z) | (ew == rec.w);
    const bool freq = ew < rec.z;
    const int dj = ew < rec.y ? -1 : 1;
    const int ni = ew < rec.w ? p.i - 1 : p.i + 1;
    const bool inside = (unsigned)ni < (unsigned)p.nc;
    const bool slow = en & (tie | (!freq & !inside));
    const bool fast = en & !slow;
    p.j = (fast & freq) ? p.j + dj : p.j;
    p.i = (fast & !freq) ? ni : p.i;
    p.steps += fast ? 1ull : 0ull;
    d = slow ? 0 : (freq ? dj : 2);
    return slow;
}

// Pairs of static-medium steps with wave-uniform control flow: every lane evaluates both
// steps of a pair with selects, lanes that are done or past their budget are disabled, and
// the slow path and record reloads run under masks only when some lane needs them.  Same
// records, random words and arithmetic as one_step, so the same bits.
template <bool MOVING, bool SURR = false>
__device__ __forceinline__ void static_pairs(Packet1D &p, int budget, int last_state,
                                             const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                                             const WalkArgs &a, unsigned long long *__restrict__ tally,
                                             const SurrWin *sw = nullptr, const float *__restrict__ recs = nullptr)
{
    const float4 nomap = make_float4(1.f, 0.f, 1.f, 0.f);
    for (int k = 0; k < a.chunk; ++k) {
        bool en = p.active && k < budget && (!SURR || p.steps < a.max_steps);
        if (!__any(en)) break;
        if (SURR) {   // a pair that starts in the surrogate window is replaced by one exit
            const bool sx = en && p.steps + 3ull <= a.max_steps && in_window(p, *sw);
            if (__any(sx)) {
                if (sx) surrogate_exit<MOVING>(p, *sw, recs, tb, clouds[p.cl], a);
            }
            en = en && !sx;
        }
        // disabled lanes read the first records of the table buffer (always mapped; unused)
        const uint4 *h = en ? p.hot : reinterpret_cast<const uint4 *>(tb);
        const int s = en ? p.i * p.nb + p.j : 0;
        const uint4 rm = h[s > 0 ? s - 1 : 0];
        const uint4 r0 = h[s];
        const uint4 rp = h[en && s < last_state ? s + 1 : s];
        const uint64_t pair = p.steps >> 1;
        const u32x4 r = philox4x32_10((uint32_t)pair, (uint32_t)(pair >> 32), p.pid, p.key, a.key0, a.key1);
        int d;
        const bool s1 = select_step(p, en, r.x, r.y, r0, d);
        if (__any(s1)) {
            if (s1) slow_step<MOVING>(p, StepWords{r.x, r.y, 0u, 0u}, r0, nomap, tb, clouds, a, tally);
        }
        const bool en2 = en && p.active && p.steps < a.max_steps;
        uint4 rb = d == -1 ? rm : rp;
        const bool reload = en2 && (d == 0 || d == 2);   // after a spatial move or a slow step
        if (__any(reload)) {
            if (reload) rb = p.hot[p.i * p.nb + p.j];
        }
        const bool s2 = select_step(p, en2, r.z, r.w, rb, d);
        if (__any(s2)) {
            if (s2) slow_step<MOVING>(p, StepWords{r.z, r.w, 0u, 0u}, rb, nomap, tb, clouds, a, tally);
        }
    }
}

// One moving-medium step as selects: like select_step, with the Doppler re-binning of a
// spatial move (eq. 20) computed inline on uniform grids; on other grids the lanes that
// moved spatially re-bin under a mask.  The arithmetic is that of one_step.
__device__ __forceinline__ bool select_step_moving(Packet1D &p, bool en, StepWords w, uint4 rec, float4 cm,
                                                   const DevCloud *__restrict__ clouds,
                                                   const uint8_t *__restrict__ tb)
{
    const double tn = p.t + (double)path_length(w.t, __uint_as_float(rec.x));
    p.t = en ? tn : p.t;
    const uint32_t ew = w.e;
    const bool tie = (ew == rec.y) | (ew == rec.z) | (ew == rec.w);
    const bool freq = ew < rec.z;
    const int dj = ew < rec.y ? -1 : 1;
    const bool up = ew >= rec.w;   // face 1 (upper / outer)
    const int ni = up ? p.i + 1 : p.i - 1;
    const bool inside = (unsigned)ni < (unsigned)p.nc;
    const bool slow = en & (tie | (!freq & !inside));
    const bool fast = en & !slow;
    const bool spatial = fast & !freq;
    const float rho = up ? cm.z : cm.x;
    const float sh = up ? cm.w : cm.y;
    const bool ident = (rho == 1.0f) & (sh == 0.0f);
    int jn = rebin_uniform(p, rho, sh, w.z);
    jn = jn < 0 ? 0 : (jn > p.nb - 1 ? p.nb - 1 : jn);
    const bool other_grid = spatial & !ident & !p.uniform;
    p.j = (fast & freq) ? p.j + dj : ((spatial & !ident & p.uniform) ? jn : p.j);
    if (__any(other_grid)) {
        if (other_grid) rebin(p, up ? 1 : 0, cm, w.z, clouds[p.cl], tb);
    }
    p.i = spatial ? ni : p.i;
    p.steps += fast ? 1ull : 0ull;
    return slow;
}

// Moving-medium steps (one Philox block each) with wave-uniform control flow: at most
// `lim` iterations, lanes past their own `budget` disabled; with the surrogate, a step that
// starts in the window is replaced by one exit.
template <bool SURR = false>
__device__ __forceinline__ void moving_steps(Packet1D &p, int budget, int lim, const uint8_t *__restrict__ tb,
                                             const DevCloud *__restrict__ clouds, const WalkArgs &a,
                                             unsigned long long *__restrict__ tally, const SurrWin *sw = nullptr,
                                             const float *__restrict__ recs = nullptr)
{
    for (int k = 0; k < lim; ++k) {
        bool en = p.active && k < budget && (!SURR || p.steps < a.max_steps);
        if (!__any(en)) break;
        if (SURR) {
            const bool sx = en && p.steps + 3ull <= a.max_steps && in_window(p, *sw);
            if (__any(sx)) {
                if (sx) surrogate_exit<true>(p, *sw, recs, tb, clouds[p.cl], a);
            }
            en = en && !sx;
        }
        // disabled lanes read the first words of the table buffer (always mapped; unused)
        const uint4 rec = (en ? p.hot : reinterpret_cast<const uint4 *>(tb))[en ? p.i * p.nb + p.j : 0];
        const float4 cm = (en ? p.cmap : reinterpret_cast<const float4 *>(tb))[en ? p.i : 0];
        const u32x4 r = philox4x32_10((uint32_t)p.steps, (uint32_t)(p.steps >> 32), p.pid, p.key, a.key0, a.key1);
        const StepWords w{r.x, r.y, r.z, r.w};
        const bool slow = select_step_moving(p, en, w, rec, cm, clouds, tb);
        if (__any(slow)) {
            if (slow) slow_step<true>(p, w, rec, cm, tb, clouds, a, tally);
        }
    }
}

// 1D walk (slab or sphere), pure DDMC; MOVING enables Doppler re-binning and lab-frame
// escape frequencies.  Static media take one Philox block per pair of steps ((x, y) for the
// even step and (z, w) for the odd one; all active lanes of a wave are at even step counts
// between pairs); moving media take one block per step.
template <bool MOVING, bool SURR>
__device__ void coop_walk(Packet1D &q, const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                          const WalkArgs &a, unsigned long long *__restrict__ tally, int lane);

__device__ __forceinline__ uint32_t rl(uint32_t v, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

__device__ __forceinline__ TailPacket *slots_of(unsigned long long *work)
{
    return reinterpret_cast<TailPacket *>(reinterpret_cast<uint8_t *>(work) + kWorkHeaderBytes);
}

// The packet of an export slot as a wave-uniform state.
__device__ Packet1D load_slot(const TailPacket *ts, const uint8_t *__restrict__ tb,
                              const DevCloud *__restrict__ clouds)
{
    const TailPacket tk = *ts;
    Packet1D q;
    q.cl = (int)rl(tk.cl, 0);
    const DevCloud &c = clouds[q.cl];
    q.pid = rl(tk.pid, 0);
    q.key = c.stream;
    q.i = (int)rl((uint32_t)tk.i, 0);
    q.j = (int)rl((uint32_t)tk.j, 0);
    q.steps = ((uint64_t)rl((uint32_t)(tk.steps >> 32), 0) << 32) | rl((uint32_t)tk.steps, 0);
    const uint64_t tb64 = ((uint64_t)rl((uint32_t)(__double_as_longlong(tk.t) >> 32), 0) << 32) |
                          rl((uint32_t)__double_as_longlong(tk.t), 0);
    q.t = __longlong_as_double((long long)tb64);
    q.nb = c.nb;
    q.nc = c.nc;
    q.geom = c.geometry;
    q.hot = reinterpret_cast<const uint4 *>(tb + c.off_hot);
    q.cmap = reinterpret_cast<const float4 *>(tb + c.off_cmap);
    q.x0 = c.x0;
    q.dx = c.dx;
    q.inv_dx = c.inv_dx;
    q.uniform = c.uniform_bins != 0;
    q.moving = c.moving != 0;
    q.active = true;
    q.surr_calls = rl(tk.surr_calls, 0);
    return q;
}

// A consumer wave (a block past the producers) walks handed-over packets cooperatively,
// one after another.  It claims only slot indices already handed out (a CAS on the claim
// counter bounded by the hand-out counter: each failed CAS means another wave claimed one,
// so the retries end); a claimed slot whose packet is not yet published is marked abandoned
// (its exporter walks it).  With nothing to claim it exits once every producer wave has
// finished, or after kConsumerIdlePolls polls; what it leaves, the closing kernel walks.
template <bool MOVING, bool SURR>
__device__ void consume_exported(const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                                 const WalkArgs &a, unsigned long long *__restrict__ tally,
                                 unsigned long long *__restrict__ work, int lane)
{
    TailPacket *slots = slots_of(work);
    constexpr uint64_t kNone = ~0ull;
    int idle = 0;
    for (;;) {
        uint64_t idx = kNone;
        uint32_t done = 0u;
        if (lane == 0) {
            for (;;) {
                const uint64_t taken = __hip_atomic_load(&work[kWClaimed], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t given = __hip_atomic_load(&work[kWGiven], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (taken >= given || taken >= a.tail_capacity) {
                    done = __hip_atomic_load(&work[kWDone], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                   (unsigned long long)a.producer_waves
                               ? 1u
                               : 0u;
                    break;
                }
                unsigned long long expect = taken;
                if (__hip_atomic_compare_exchange_strong(&work[kWClaimed], &expect, taken + 1ull, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    idx = taken;
                    break;
                }
            }
        }
        idx = shfl_u64(idx, 0);
        if (idx == kNone) {
            if (rl(done, 0) != 0u || ++idle > kConsumerIdlePolls) return;
            for (int z = 0; z < 32; ++z) __builtin_amdgcn_s_sleep(127);
            continue;
        }
        idle = 0;
        uint32_t got = 0u;
        if (lane == 0) {
            // the exporter hands the slot out just before it writes and publishes it: give it
            // a bounded moment, then take the packet or leave it to the exporter
            uint32_t *f = &slots[idx].flag;
            int tries = 0;
            while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == kSlotEmpty &&
                   ++tries < kPublishWaitPolls)
                __builtin_amdgcn_s_sleep(2);
            uint32_t expect = kSlotEmpty;
            if (!__hip_atomic_compare_exchange_strong(f, &expect, kSlotAbandoned, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                      __HIP_MEMORY_SCOPE_AGENT) &&
                expect == kSlotReady) {
                got = __hip_atomic_compare_exchange_strong(f, &expect, kSlotTaken, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                          ? 1u
                          : 0u;
            }
        }
        if (rl(got, 0) == 0u) continue;
        Packet1D q = load_slot(slots + idx, tb, clouds);
        coop_walk<MOVING, SURR>(q, tb, clouds, a, tally, lane);
    }
}

template <bool MOVING, bool SURR>
__global__ __launch_bounds__(256) void walk1d(const uint8_t *__restrict__ tb, WalkArgs a,
                                              unsigned long long *__restrict__ tally,
                                              unsigned long long *__restrict__ work)
{
    const SurrHeader *SH = SURR ? reinterpret_cast<const SurrHeader *>(a.surr) : nullptr;
    const float *recs = SURR ? reinterpret_cast<const float *>(a.surr + SH->off_records) : nullptr;
    SurrWin sw{0, -1, 0, -1, 0ull};
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud *clouds = reinterpret_cast<const DevCloud *>(tb + H->off_clouds);
    const uint64_t *prefix = reinterpret_cast<const uint64_t *>(tb + H->off_prefix);
    const int lane = threadIdx.x & 63;
    if (blockIdx.x >= a.producer_blocks) {   // a consumer block
        consume_exported<MOVING, SURR>(tb, clouds, a, tally, work, lane);
        return;
    }

    Packet1D p;
    p.active = false;
    p.cl = 0; p.nb = 1; p.nc = 1; p.geom = 0; p.pid = 0; p.key = 0; p.i = 0; p.j = 0; p.t = 0.0; p.steps = 0;
    p.hot = nullptr;
    p.cmap = nullptr;
    p.x0 = 0.f; p.dx = 1.f; p.inv_dx = 1.f; p.uniform = false; p.moving = false;
    p.surr_calls = 0u;
    int last_state = 0;
    bool exhausted = false;       // wave-uniform: the queue is empty

    for (;;) {
        // ---- refill finished lanes (one atomic per wave) -----------------------------
        if (!exhausted) {
            const uint64_t need = __ballot(!p.active);
            if (need) {
                const int leader = __ffsll((unsigned long long)need) - 1;
                const int cnt = __popcll(need);
                uint64_t base = 0;
                if (lane == leader) base = atomicAdd(work, (unsigned long long)cnt);
                base = shfl_u64(base, leader);
                if (base + cnt >= a.count) exhausted = true;
                if (!p.active) {
                    const int rank = __popcll(need & ((1ull << lane) - 1ull));
                    const uint64_t q = base + rank;
                    if (q < a.count) {
                        const uint64_t g = a.first + q;
                        int lo = 0, hi = a.n_clouds;      // prefix[lo] <= g < prefix[hi]
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (g >= prefix[mid]) lo = mid; else hi = mid;
                        }
                        p.cl = lo;
                        const DevCloud &c = clouds[lo];
                        p.pid = (uint32_t)(g - prefix[lo]);
                        p.key = c.stream;
                        p.nb = c.nb;
                        p.nc = c.nc;
                        p.geom = c.geometry;
                        p.hot = reinterpret_cast<const uint4 *>(tb + c.off_hot);
                        p.cmap = reinterpret_cast<const float4 *>(tb + c.off_cmap);
                        p.x0 = c.x0;
                        p.dx = c.dx;
                        p.inv_dx = c.inv_dx;
                        p.uniform = c.uniform_bins != 0;
                        p.moving = c.moving != 0;
                        last_state = (int)c.n_states - 1;
                        // emission (Sec. 2.3): a source state drawn by its probability
                        const u32x4 r = philox4x32_10(0u, kDomEmit, p.pid, p.key, a.key0, a.key1);
                        const double u = u01_open_low(r.x);
                        const int32_t *ss = reinterpret_cast<const int32_t *>(tb + c.off_src_state);
                        const double *cdf = reinterpret_cast<const double *>(tb + c.off_src_cdf);
                        int k = 0;
                        while (k < c.n_src - 1 && u >= cdf[k]) ++k;
                        const int32_t st = ss[k];
                        p.i = st / p.nb;
                        p.j = st - p.i * p.nb;
                        p.t = 0.0;
                        p.steps = 0;
                        p.active = true;
                        p.surr_calls = 0u;
                        if (SURR) {
                            const SurrCloud *scl = reinterpret_cast<const SurrCloud *>(a.surr + SH->off_clouds) + lo;
                            sw = SurrWin{scl->i_lo, scl->i_hi, scl->j_lo, scl->j_hi, scl->rec_off};
                        }
                        atomicAdd(&tally[c.tally_off + TW_LAUNCHED], 1ull);
                    }
                }
            }
        }
        if (!__any(p.active)) break;

        // ---- tail: hand the last few packets of this wave to the cooperative walk ----
        if (exhausted && a.tail_lanes > 0) {
            const uint64_t live = __ballot(p.active);
            if (__popcll(live) <= a.tail_lanes) {
                const int leader = __ffsll((unsigned long long)live) - 1;
                uint64_t base = 0;
                if (lane == leader) base = atomicAdd(&work[kWGiven], (unsigned long long)__popcll(live));
                base = shfl_u64(base, leader);
                bool keep = false;
                if (p.active) {
                    const uint64_t slot = base + __popcll(live & ((1ull << lane) - 1ull));
                    TailPacket *tp = slots_of(work) + slot;
                    tp->cl = (uint32_t)p.cl;
                    tp->pid = p.pid;
                    tp->i = p.i;
                    tp->j = p.j;
                    tp->steps = p.steps;
                    tp->t = p.t;
                    tp->surr_calls = p.surr_calls;
                    __threadfence();
                    uint32_t expect = kSlotEmpty;
                    keep = !__hip_atomic_compare_exchange_strong(&tp->flag, &expect, kSlotReady, __ATOMIC_RELEASE,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    p.active = false;
                }
                // slots a consumer claimed before they were published: walk them here
                uint64_t mine = __ballot(keep);
                while (mine) {
                    const int l = __ffsll((unsigned long long)mine) - 1;
                    mine &= mine - 1ull;
                    const uint64_t slot = base + __popcll(live & ((1ull << l) - 1ull));
                    Packet1D q = load_slot(slots_of(work) + slot, tb, clouds);
                    coop_walk<MOVING, SURR>(q, tb, clouds, a, tally, lane);
                }
                break;
            }
        }

        // ---- walk up to `chunk` pairs of steps ---------------------------------------
        const bool was_active = p.active;
        const uint64_t left = p.active ? (a.max_steps - p.steps) : 0ull;
        if (!(MOVING && p.moving)) {
            const uint64_t pairs = (left + 1) >> 1;
            const int budget = pairs < (uint64_t)a.chunk ? (int)pairs : a.chunk;
            static_pairs<MOVING, SURR>(p, budget, last_state, tb, clouds, a, tally, &sw, recs);
        }
        if (MOVING && p.moving) {
            const uint64_t lim = 2ull * (uint64_t)a.chunk;
            const int budget = left < lim ? (int)left : (int)lim;
            moving_steps<SURR>(p, budget, (int)lim, tb, clouds, a, tally, &sw, recs);
        }
        if (p.active && p.steps >= a.max_steps) {
            tally_finish(tally, clouds[p.cl], false, 0, 0, p.t, p.steps);
            p.active = false;
        }
        if (SURR && was_active && !p.active && p.surr_calls)
            atomicAdd(&tally[clouds[p.cl].tally_off + TW_SURR_CALLS], (unsigned long long)p.surr_calls);
    }
    if (lane == 0) __hip_atomic_fetch_add(&work[kWDone], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Cooperative walk of ONE packet by a whole wave (the packet state is wave-uniform).
//   * The 64 lanes hold the hot records of 64 consecutive bins of the packet's cell (the
//     band); each block of up to 64 steps walks a 15-bin window of it, centred on the
//     packet's bin.
//   * Lane l draws the Philox words of step steps+l and builds the step's transition table
//     over the window: 4 bits per window position giving the next position, or 15 ("stop")
//     for a slow-path step (a tie with a threshold, a spatial leak), a move out of the
//     window, or (with the surrogate) a step that starts in the surrogate window at one of
//     the lane walk's check points; position 15 maps to itself.
//   * Each even lane composes its table with the next lane's (two steps per table); the
//     sequential part is a scalar chain of two instructions per pair of steps (a 4-bit
//     field extract addressed by the position, a shift-add back to an address); even
//     lanes receive the position their step starts from, odd lanes take one step from it.
//   * The lane whose step stops classifies it: a move out of the window completes; a
//     surrogate exit or a slow-path step runs in lane 0 with the lane walk's arithmetic.
// The clock gives the bits of the lane walk's ordered FP64 additions (clock_parallel, else
// in order), so every tally is bit-identical to walking the packet in a single lane.
constexpr int kCoopWin = 15;
// scan state: 4 x window position in bits 0..5, field width 4 in bits 16..22 (the operand
// layout of s_bfe_u64); kScanStop is the state of the stop position
constexpr uint32_t kScanWidth = 4u << 16;
constexpr uint32_t kScanStop = kScanWidth | (15u << 2);

// Step L of the chain: hand lane L its starting state, then move to the next position.
template <int L>
__device__ __forceinline__ void scan_step(uint32_t &st, int &vst, uint32_t tlo, uint32_t thi)
{
    const uint64_t tab = ((uint64_t)rl(thi, L) << 32) | rl(tlo, L);
    uint64_t f;
    asm("v_writelane_b32 %0, %1, %2" : "+v"(vst) : "s"(st), "n"(L));
    asm("s_bfe_u64 %0, %1, %2" : "=s"(f) : "s"(tab), "s"(st) : "scc");
    asm("s_lshl2_add_u32 %0, %1, %2" : "=s"(st) : "s"((uint32_t)f), "s"(kScanWidth) : "scc");
}

// The chain over two-step tables held by the even lanes (lane 2k: steps 2k and 2k+1),
// eight steps per group, leaving once the stop is reached.
template <int G>
__device__ __forceinline__ void scan_from(uint32_t &st, int &vst, uint32_t tlo, uint32_t thi)
{
    scan_step<8 * G + 0>(st, vst, tlo, thi);
    scan_step<8 * G + 2>(st, vst, tlo, thi);
    scan_step<8 * G + 4>(st, vst, tlo, thi);
    scan_step<8 * G + 6>(st, vst, tlo, thi);
    if constexpr (G < 7) {
        if (st != kScanStop) scan_from<G + 1>(st, vst, tlo, thi);
    }
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double rl_f64(double v, int lane)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)(((uint64_t)rl((uint32_t)(b >> 32), lane) << 32) | rl((uint32_t)b, lane)));
}

// Clock of a block without the sequential chain, where that gives the same bits.  With
// t0 in [2^e, 2^(e+1)), ulp = 2^(e-52), and every partial sum below 2^(e+1), each
// addition t + d (d >= 0) rounds to t + ulp * rint(d / ulp), unless d / ulp lies exactly
// halfway between integers (then the rounding depends on the running sum).  Without such
// a tie the block's result is t0 + ulp * (sum of the rint values): an exact integer sum,
// reduced across the wave in any order.  Returns false (t unchanged) where the premises
// fail; the caller then adds in order.
__device__ __forceinline__ bool clock_parallel(double &t, double dd)
{
    const uint64_t tbits = (uint64_t)__double_as_longlong(t);
    const int be = (int)((tbits >> 52) & 0x7ffu);
    if (be == 0 || be >= 0x7fe) return false;        // zero, subnormal or near the top
    const int e = be - 1023;
    const double qv = ldexp(dd, 52 - e);               // exact: a power-of-two scaling
    const double n = rint(qv);
    const bool tie = (qv - floor(qv)) == 0.5;
    if (__any(tie)) return false;
    double s = n;                                      // integers below 2^53: exact sums
    s += dpp_f64<0xb1>(s);                             // quad_perm [1,0,3,2]
    s += dpp_f64<0x4e>(s);                             // quad_perm [2,3,0,1]
    s += dpp_f64<0x124>(s);                            // row_ror:4
    s += dpp_f64<0x128>(s);                            // row_ror:8
    const double S = (rl_f64(s, 0) + rl_f64(s, 16)) + (rl_f64(s, 32) + rl_f64(s, 48));
    const double tf = t + ldexp(S, e - 52);
    if (!(tf < ldexp(1.0, e + 1))) return false;       // left the binade: add in order
    t = tf;
    return true;
}

// Clock of a block: t += the FP64 path lengths of lanes 0, 1, ... in order (lanes at or
// beyond `done` hold +0, which leaves t unchanged).
template <int G>
__device__ __forceinline__ void clock_from(double &t, uint32_t dlo, uint32_t dhi, int done)
{
    double v[8];   // read the group's eight values first, then add them in order
#pragma unroll
    for (int u = 0; u < 8; ++u)
        v[u] = __longlong_as_double((long long)(((uint64_t)rl(dhi, 8 * G + u) << 32) | rl(dlo, 8 * G + u)));
#pragma unroll
    for (int u = 0; u < 8; ++u) t += v[u];
    if constexpr (G < 7) {
        if (done > 8 * (G + 1)) clock_from<G + 1>(t, dlo, dhi, done);
    }
}

template <bool MOVING, bool SURR>
__device__ void coop_walk(Packet1D &q, const uint8_t *__restrict__ tb, const DevCloud *__restrict__ clouds,
                          const WalkArgs &a, unsigned long long *__restrict__ tally, int lane)
{
    // the cloud's surrogate window: a step that starts in it is replaced by one exit, at the
    // same points as in the lane walk (every step in moving media, even step counts in
    // static media, and only with room for three more steps)
    SurrWin sw{0, -1, 0, -1, 0ull};
    const float *recs = nullptr;
    if (SURR) {
        const SurrHeader *SH = reinterpret_cast<const SurrHeader *>(a.surr);
        recs = reinterpret_cast<const float *>(a.surr + SH->off_records);
        const SurrCloud *scl = reinterpret_cast<const SurrCloud *>(a.surr + SH->off_clouds) + q.cl;
        sw = SurrWin{scl->i_lo, scl->i_hi, scl->j_lo, scl->j_hi, scl->rec_off};
    }
    int wi = -1, jb = 0;
    int short_run = 0;   // consecutive blocks stopped by a slow-path step within 16 steps
    uint32_t v_lk = 0u, v_dhi = 0u, v_shi = 0u, v_fhi = 0u;
    while (q.active) {
        const uint64_t left = a.max_steps - q.steps;
        if (left == 0) {
            if (lane == 0) tally_finish(tally, clouds[q.cl], false, 0, 0, q.t, q.steps);
            q.active = false;
            break;
        }
        const int m = left < 64 ? (int)left : 64;
        // band of 64 bins around the packet (reloaded on a new cell or near its edges)
        if (q.i != wi || (q.j - jb < kCoopWin / 2 && jb > 0) ||
            (q.j - jb > 63 - kCoopWin / 2 && jb < q.nb - 64)) {
            jb = q.j - 32;
            if (jb > q.nb - 64) jb = q.nb - 64;
            if (jb < 0) jb = 0;
            wi = q.i;
            // bins beyond the grid: every event there is "slow" (never reached)
            v_lk = 0u;
            v_dhi = 0u;
            v_shi = 0u;
            v_fhi = 0u;
            if (jb + lane < q.nb) {
                const uint4 r = q.hot[q.i * q.nb + jb + lane];
                v_lk = r.x;
                v_dhi = r.y;
                v_shi = r.z;
                v_fhi = r.w;
            }
        }
        int jw = q.j - kCoopWin / 2;
        if (jw > jb + 64 - kCoopWin) jw = jb + 64 - kCoopWin;
        if (jw < jb) jw = jb;
        const int wb = jw - jb;   // band lane of window position 0
        const StepWords wl = words_of_step<MOVING>(q, q.steps + (uint64_t)lane, a);
        const uint32_t ew = wl.e;
        // surrogate stops: window positions inside the surrogate window, for the steps that
        // check it
        uint32_t smask = 0u;
        bool chk = false;
        if (SURR && (unsigned)(q.i - sw.i_lo) <= (unsigned)(sw.i_hi - sw.i_lo)) {
#pragma unroll
            for (int b = 0; b < kCoopWin; ++b)
                smask |= ((unsigned)(jw + b - sw.j_lo) <= (unsigned)(sw.j_hi - sw.j_lo) ? 1u : 0u) << b;
            const uint64_t st_l = q.steps + (uint64_t)lane;
            chk = ((MOVING && q.moving) || !(st_l & 1ull)) && st_l + 3ull <= a.max_steps;
        }
        // the window's thresholds rotated into lanes 0..14
        const uint32_t wdh = (uint32_t)__shfl((int)v_dhi, (wb + lane) & 63);
        const uint32_t wsh = (uint32_t)__shfl((int)v_shi, (wb + lane) & 63);
        // the step's table: field b = next window position from position b
        uint32_t tlo = 0u, thi = 15u << 28;
#pragma unroll
        for (int b = 0; b < kCoopWin; ++b) {
            const uint32_t dh = rl(wdh, b), sh = rl(wsh, b);
            const bool dn = ew < dh;
            const bool slow = (ew >= sh) || (ew == dh) || (SURR && chk && ((smask >> b) & 1u));
            const uint32_t mv = dn ? (b == 0 ? 15u : (uint32_t)(b - 1)) : (b == kCoopWin - 1 ? 15u : (uint32_t)(b + 1));
            const uint32_t nx = slow ? 15u : mv;
            if (b < 8) tlo |= nx << (4 * b);
            else thi |= nx << (4 * (b - 8));
        }
        if (lane >= m) {   // no step: stop there
            tlo = 0xffffffffu;
            thi = 0xffffffffu;
        }
        // even lanes: the table of two steps (this lane's, then the next lane's)
        const uint64_t tab = ((uint64_t)thi << 32) | tlo;
        const uint64_t nxt = ((uint64_t)(uint32_t)__shfl_down((int)thi, 1) << 32) | (uint32_t)__shfl_down((int)tlo, 1);
        uint32_t clo = 0u, chi = 0u;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const uint32_t mid = (uint32_t)(tab >> (4 * b)) & 15u;
            const uint32_t two = (uint32_t)(nxt >> (4 * mid)) & 15u;
            if (b < 8) clo |= two << (4 * b);
            else chi |= two << (4 * (b - 8));
        }
        // sequential part: the chain of positions, in scalar registers, two steps at a time
        uint32_t st = kScanWidth | ((uint32_t)(q.j - jw) << 2);
        int vst = (int)kScanStop;
        scan_from<0>(st, vst, clo, chi);
        // each lane's starting position (odd lanes: one step from the even lane before);
        // the first lane whose step stops
        const int pe = (int)(((uint32_t)vst & 63u) >> 2);
        const uint32_t ne = (uint32_t)(tab >> (4 * pe)) & 15u;
        const uint32_t from_even = (uint32_t)__shfl_up((int)ne, 1);
        const int pl = (lane & 1) ? (int)from_even : pe;
        const bool stops = pl != 15 && ((uint32_t)(tab >> (4 * pl)) & 15u) == 15u;
        const uint64_t sb = __ballot(stops);
        const int ls = sb ? __ffsll((unsigned long long)sb) - 1 : 64;
        // the records of the lane's bin
        const int src = (wb + (pl < 15 ? pl : 0)) & 63;
        const uint32_t lk = (uint32_t)__shfl((int)v_lk, src);
        const uint32_t dhl = (uint32_t)__shfl((int)v_dhi, src);
        const uint32_t shl = (uint32_t)__shfl((int)v_shi, src);
        int done, pos;
        bool special = false, surr_stop = false;
        if (ls >= m) {                         // m steps, no stop
            done = m;
            pos = ls < 64 ? (int)rl((uint32_t)pl, ls) : (int)((st & 63u) >> 2);
        } else {
            const bool sstop = SURR && chk && pl < 15 && ((smask >> pl) & 1u);
            surr_stop = SURR && rl(sstop ? 1u : 0u, ls) != 0u;
            const uint32_t slow = (sstop || (ew >= shl) || (ew == dhl)) ? 1u : 0u;
            const int p = (int)rl((uint32_t)pl, ls);
            if (rl(slow, ls)) {                // step ls takes the slow path
                special = true;
                done = ls;
                pos = p;
            } else {                           // step ls leaves the window: it is done
                done = ls + 1;
                pos = p + (rl(ew < dhl ? 1u : 0u, ls) ? -1 : 1);
            }
        }
        const float dl = lane < done ? path_length(wl.t, __uint_as_float(lk)) : 0.0f;
        const double dd = (double)dl;
        const uint32_t dlo = (uint32_t)__double_as_longlong(dd);
        const uint32_t dhi = (uint32_t)((uint64_t)__double_as_longlong(dd) >> 32);
        double t = q.t;                    // the lane walk's FP64 additions, same bits
        if (done > 0 && !clock_parallel(t, dd)) clock_from<0>(t, dlo, dhi, done);
        q.t = t;
        q.steps += (uint64_t)done;
        const int jj = jw + pos;
        q.j = jj;
        short_run = special && done < 16 ? short_run + 1 : 0;
        if (special) {
            // the step at `done` in lane 0 with the lane walk's arithmetic; then, if several
            // blocks in a row stopped early (spatial leaks dominate here), a run of single
            // steps in lane 0, twice as long (up to 1024) for every further such block
            const int b = (jj - jb) & 63;
            const StepWords ws = {rl(wl.t, done), rl(ew, done), rl(wl.z, done), rl(wl.w, done)};
            const uint4 rec = make_uint4(rl(v_lk, b), rl(v_dhi, b), rl(v_shi, b), rl(v_fhi, b));
            Packet1D s1 = q;
            if (lane == 0 && SURR && surr_stop) {
                surrogate_exit<MOVING>(s1, sw, recs, tb, clouds[s1.cl], a);
            } else if (lane == 0) {
                const float4 cm = (MOVING && s1.moving) ? s1.cmap[s1.i] : make_float4(1.f, 0.f, 1.f, 0.f);
                one_step<MOVING>(s1, ws, rec, cm, tb, clouds, a, tally);
                if (SURR && short_run >= 3) {
                    surr_single_steps<MOVING>(s1, 64 << (short_run - 3 < 4 ? short_run - 3 : 4), sw, recs, tb,
                                              clouds, a, tally);
                } else if (short_run >= 3) {
                    const int n = 64 << (short_run - 3 < 4 ? short_run - 3 : 4);
                    if (MOVING && s1.moving) {
                        const uint64_t left = s1.active ? a.max_steps - s1.steps : 0ull;
                        const int budget = left < (uint64_t)n ? (int)left : n;
                        moving_steps(s1, budget, budget, tb, clouds, a, tally);
                    } else {
                        single_steps<MOVING>(s1, n, tb, clouds, a, tally);
                    }
                }
            }
            q.i = (int)rl((uint32_t)s1.i, 0);
            q.j = (int)rl((uint32_t)s1.j, 0);
            q.steps = ((uint64_t)rl((uint32_t)(s1.steps >> 32), 0) << 32) | rl((uint32_t)s1.steps, 0);
            const uint64_t tbits = (uint64_t)__double_as_longlong(s1.t);
            q.t = __longlong_as_double((long long)(((uint64_t)rl((uint32_t)(tbits >> 32), 0) << 32) |
                                                   rl((uint32_t)tbits, 0)));
            q.active = rl(s1.active ? 1u : 0u, 0) != 0u;
            if (SURR) q.surr_calls = rl(s1.surr_calls, 0);
        }
    }
    if (SURR && lane == 0 && q.surr_calls)
        atomicAdd(&tally[clouds[q.cl].tally_off + TW_SURR_CALLS], (unsigned long long)q.surr_calls);
}

template <bool MOVING, bool SURR>
__global__ __launch_bounds__(64) void walk1d_coop(const uint8_t *__restrict__ tb, WalkArgs a,
                                                  unsigned long long *__restrict__ tally,
                                                  unsigned long long *__restrict__ work)
{
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud *clouds = reinterpret_cast<const DevCloud *>(tb + H->off_clouds);
    const int lane = threadIdx.x & 63;
    const uint64_t n = work[kWGiven] < a.tail_capacity ? work[kWGiven] : a.tail_capacity;
    TailPacket *slots = slots_of(work);
    for (;;) {   // the packets still published once the lane-walk launch has ended
        uint64_t idx = 0;
        if (lane == 0) idx = atomicAdd(&work[kWSweep], 1ull);
        idx = shfl_u64(idx, 0);
        if (idx >= n) break;
        uint32_t got = 0u;
        if (lane == 0) {
            uint32_t expect = kSlotReady;
            got = __hip_atomic_compare_exchange_strong(&slots[idx].flag, &expect, kSlotTaken, __ATOMIC_ACQ_REL,
                                                       __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
                      ? 1u
                      : 0u;
        }
        if (rl(got, 0) == 0u) continue;
        Packet1D q = load_slot(slots + idx, tb, clouds);
        coop_walk<MOVING, SURR>(q, tb, clouds, a, tally, lane);
    }
}

// Sub-walks for the surrogate's training data: sample q starts in state s_state[q] of
// cloud s_cloud[q] (a cell with two neighbours) and takes DDMC steps until its first
// spatial leak.  Writes the state's features X[q, 16] and the exit Y[q] = (face, y1, y2),
// face -1 when max_steps ran out first, and the number of steps.
template <bool MOVING>
__global__ __launch_bounds__(256) void subwalk1d(const uint8_t *__restrict__ tb, WalkArgs a,
                                                 const int32_t *__restrict__ s_cloud,
                                                 const int32_t *__restrict__ s_state, int64_t n,
                                                 float *__restrict__ X, float *__restrict__ Y,
                                                 unsigned long long *__restrict__ steps_out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const DevHeader *H = reinterpret_cast<const DevHeader *>(tb);
    const DevCloud *clouds = reinterpret_cast<const DevCloud *>(tb + H->off_clouds);
    const int cl = s_cloud[q];
    const DevCloud &c = clouds[cl];
    Packet1D p;
    p.cl = cl;
    p.nb = c.nb;
    p.nc = c.nc;
    p.geom = c.geometry;
    p.pid = (uint32_t)q;
    p.key = c.stream;
    p.i = s_state[q] / c.nb;
    p.j = s_state[q] - p.i * c.nb;
    p.t = 0.0;
    p.steps = 0;
    p.hot = reinterpret_cast<const uint4 *>(tb + c.off_hot);
    p.cmap = reinterpret_cast<const float4 *>(tb + c.off_cmap);
    p.x0 = c.x0;
    p.dx = c.dx;
    p.inv_dx = c.inv_dx;
    p.uniform = c.uniform_bins != 0;
    p.moving = c.moving != 0;
    p.active = true;
    p.surr_calls = 0u;
    float f[kSurrIn], S, w;
    surr_features(c, tb, p.i, p.j, f, S, w);
    for (int k = 0; k < kSurrIn; ++k) X[q * kSurrIn + k] = f[k];
    int face = -1, jexit = p.j;
    while (p.steps < a.max_steps) {
        const int i0 = p.i, j0 = p.j;
        const StepWords wd = words_of_step<MOVING>(p, p.steps, a);
        const uint4 rec = p.hot[p.i * p.nb + p.j];
        const float4 cm = (MOVING && p.moving) ? p.cmap[p.i] : make_float4(1.f, 0.f, 1.f, 0.f);
        one_step<MOVING>(p, wd, rec, cm, tb, clouds, a, nullptr);
        if (p.i != i0) {
            face = p.i > i0 ? 1 : 0;
            jexit = j0;
            break;
        }
    }
    const double *e = reinterpret_cast<const double *>(tb + c.off_edges);
    const u32x4 r = philox4x32_10((uint32_t)q, kDomSub | (uint32_t)((uint64_t)q >> 32), p.pid, p.key, a.key0, a.key1);
    const double xo = e[jexit] + (e[jexit + 1] - e[jexit]) * u01_open_low(r.x);
    Y[3 * q] = (float)face;
    Y[3 * q + 1] = (float)asinh(xo / (double)S);
    Y[3 * q + 2] = (float)log(p.t / (double)w);
    steps_out[q] = p.steps;
}

__global__ void philox_fill_kernel(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                   uint32_t c3, uint64_t n, uint32_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const u32x4 r = philox4x32_10(c0 + (uint32_t)i, c1, c2, c3, k0, k1);
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

// Clears the counters and every export slot's flag (a kernel, so that the call can be
// captured in a graph).
__global__ void reset_work(unsigned long long *work, uint64_t capacity)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kWorkHeaderBytes / 8) work[i] = 0ull;
    if (i < capacity) slots_of(work)[i].flag = kSlotEmpty;
}

}  // namespace

int device_cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return n > 0 ? n : 256;
}

hipError_t launch_walk(const uint8_t *d_tables, const DevHeader &h, const DevCloud *host_clouds,
                       const rddmc_run &run, uint64_t first, uint64_t count,
                       unsigned long long *d_tally, unsigned long long *d_work, uint64_t work_bytes,
                       hipStream_t s)
{
    WalkArgs a;
    a.first = first;
    a.count = count;
    a.max_steps = run.max_steps;
    a.key0 = (uint32_t)run.seed;
    a.key1 = (uint32_t)(run.seed >> 32);
    a.chunk = run.chunk > 0 ? (run.chunk + 1) / 2 : 32;   // in pairs of steps
    a.n_clouds = h.n_clouds;
    a.tail_lanes = run.tail_lanes == 0 ? 16 : (run.tail_lanes < 0 ? 0 : run.tail_lanes);
    a.pad = 0;
    a.tail_capacity = work_bytes > kWorkHeaderBytes ? (work_bytes - kWorkHeaderBytes) / sizeof(TailPacket) : 0;
    if (a.tail_capacity == 0) a.tail_lanes = 0;
    const int block = run.block > 0 ? run.block : 256;
    uint64_t grid = run.grid > 0 ? (uint64_t)run.grid : 0;
    if (grid == 0) {
        const uint64_t want = (count + block - 1) / block;
        const uint64_t cap = (uint64_t)device_cu_count() * 8;   // 8 blocks of 256 per CU
        grid = want < cap ? want : cap;
        if (grid < 1) grid = 1;
    }
    const uint64_t lanes = grid * (uint64_t)block;
    if (a.tail_lanes > 0 && (lanes < count ? lanes : count) > a.tail_capacity) {
        // every exported packet (at most one per lane, at most `count`) needs a slot
        grid = a.tail_capacity / block;
        if (grid < 1) {
            grid = 1;
            a.tail_lanes = 0;
        }
    }
    bool moving = false;
    for (int c = 0; c < h.n_clouds; ++c) moving |= host_clouds[c].moving != 0;
    a.surr = static_cast<const uint8_t *>(run.surrogate);
    a.producer_blocks = (uint32_t)grid;
    a.producer_waves = (uint32_t)(grid * (uint64_t)(block / 64));
    // consumer blocks after the producers: 16 waves per CU walk handed-over packets as soon
    // as lane-walk blocks finish and free their slots
    const uint64_t consumers = a.tail_lanes > 0 ? ((uint64_t)device_cu_count() * 16 * 64 + block - 1) / block : 0;
    {
        const uint64_t n = a.tail_capacity > kWorkHeaderBytes / 8 ? a.tail_capacity : kWorkHeaderBytes / 8;
        reset_work<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d_work, a.tail_capacity);
    }
    grid += consumers;
    if (moving && a.surr)
        walk1d<true, true><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    else if (moving)
        walk1d<true, false><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    else if (a.surr)
        walk1d<false, true><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    else
        walk1d<false, false><<<(unsigned)grid, block, 0, s>>>(d_tables, a, d_tally, d_work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.tail_lanes == 0) return e;
    const unsigned cgrid = (unsigned)device_cu_count() * 16;   // one wave per block
    if (moving && a.surr)
        walk1d_coop<true, true><<<cgrid, 64, 0, s>>>(d_tables, a, d_tally, d_work);
    else if (moving)
        walk1d_coop<true, false><<<cgrid, 64, 0, s>>>(d_tables, a, d_tally, d_work);
    else if (a.surr)
        walk1d_coop<false, true><<<cgrid, 64, 0, s>>>(d_tables, a, d_tally, d_work);
    else
        walk1d_coop<false, false><<<cgrid, 64, 0, s>>>(d_tables, a, d_tally, d_work);
    return hipGetLastError();
}

hipError_t launch_subwalk(const uint8_t *d_tables, bool moving, uint64_t seed, uint64_t max_steps,
                          const int32_t *d_cloud, const int32_t *d_state, int64_t n, float *d_x, float *d_y,
                          unsigned long long *d_steps, hipStream_t s)
{
    WalkArgs a{};
    a.max_steps = max_steps;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (moving)
        subwalk1d<true><<<grid, 256, 0, s>>>(d_tables, a, d_cloud, d_state, n, d_x, d_y, d_steps);
    else
        subwalk1d<false><<<grid, 256, 0, s>>>(d_tables, a, d_cloud, d_state, n, d_x, d_y, d_steps);
    return hipGetLastError();
}

hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                              uint32_t c3, uint64_t n, uint32_t *d_out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    philox_fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(k0, k1, c0, c1, c2, c3, n, d_out);
    return hipGetLastError();
}

}  // namespace rddmc
