// Internal layout shared by the library's translation units (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rddmc.h"

namespace rddmc {

constexpr int kMaxFaces = 6;
constexpr double kTimeFix = 1048576.0;          // escape-time fixed point: 2^-20 length/c per unit
constexpr int kTallyHeader = 16;                // int64 words before the spectrum

// Tally header words (per cloud)
enum TallyWord {
    TW_ESCAPED = 0,
    TW_CAPPED = 1,
    TW_STEPS = 2,
    TW_STEPS_MAX = 3,
    TW_TSUM = 4,      // sum of round(t * 2^20)
    TW_T2_LO = 5,     // 128-bit sum of round(t^2 * 2^20): low word
    TW_T2_HI = 6,     //                                   high word
    TW_LAUNCHED = 7,
    TW_TO_MC = 8,     // hybrid: DDMC -> continuous MC conversions
    TW_TO_DDMC = 9,   //         MC -> DDMC conversions
    TW_REFLECTED = 10,//         MC packets reflected at a thick interface
    TW_MC_STEPS = 11, //         MC events (scatterings and face crossings)
    TW_SURR_CALLS = 12, // exits drawn from the learned surrogate
    TW_ABSORBED = 13,   // packets absorbed by dust
};

// 3D cells: the fourth word of the hot record holds flags instead of F.
constexpr uint32_t kFlagThick = 1u;             // the state is a DDMC state (tau >= tau_th)
constexpr int kFlagFaceShift = 1;               // bit 1+f: a leak through face f enters a thin
                                                // state or vacuum (interface rate, conversion)
constexpr uint32_t kFlagDnThin = 1u << 7;       // bin j-1 of the cell is thin
constexpr uint32_t kFlagUpThin = 1u << 8;       // bin j+1 of the cell is thin

// Shared FP32 line tables for the continuous-MC states (built once per table buffer).
//   voigt: H1(x) = (2/sqrt(pi)) (2 x F(x) - 1) on x = i/256, i < kVoigtN (F = Dawson), so
//          that H(a,x) = exp(-x^2)(1 + a^2 (1 - 2x^2)) + a H1(|x|) (eq. 12);
//   u0:    split point of the atom-velocity rejection sampler on log10(a) = -6 + i/8,
//          |x| = k/8 (any u0 >= 0 is exact; the table's minimises the proposal mass).
constexpr int kVoigtN = 4097;
constexpr float kVoigtScale = 256.0f;
constexpr int kU0NA = 49, kU0NX = 257;
constexpr float kU0Scale = 8.0f;

// The per-state record every DDMC step reads: one 16-byte load.  A uniform u64 U picks the
// event against three u64 thresholds D <= S <= F:
//   U < D -> lower bin,  D <= U < S -> upper bin,  S <= U < F -> face 0,  U >= F -> face 1
// (1D geometries; 3D uses the first two and a separate face CDF), with
// D = P(lower bin) 2^64, S = (1 - P(spatial)) 2^64, F = S + P(face 0) 2^64.
// Only the high words live here; the low words (needed only when U's high word ties with a
// threshold's, probability ~3 * 2^-32) live in the cold `lo_words` array.
struct alignas(16) HotRecord {
    float ln2_over_K;      // ln(2) / K, K = total leakage rate of the state [1/length]
    uint32_t d_hi;         // high word of D
    uint32_t s_hi;         // high word of S
    uint32_t f_hi;         // high word of F (1D); flags (3D: kFlagThick, face bits)
};
static_assert(sizeof(HotRecord) == 16, "hot record must be 16 bytes");

// Device-resident per-cloud descriptor.  Offsets are bytes from the table base.
struct alignas(16) DevCloud {
    int32_t geometry, nb, nc, nf;
    int32_t n[3];
    int32_t moving;
    int32_t n_src, keep_rates, n_rows, dirichlet;
    uint32_t stream, pad0;
    uint64_t n_packets;
    uint64_t packet_base;        // flattened index of this cloud's first packet
    uint64_t n_states;
    uint64_t off_edges;          // f64 [nb+1]
    uint64_t off_faces[3];       // f64 [n[d]+1]
    uint64_t off_k0, off_T, off_vel;   // f64 [nc], [nc], [nc * (1 or 3)]
    uint64_t off_src_state;      // i32 [n_src]
    uint64_t off_src_cdf;        // f64 [n_src]
    uint64_t off_k;              // f64 [n_states]   eq. 14
    uint64_t off_hot;            // HotRecord [n_states]
    uint64_t off_lo_words;       // u32x4 [n_states]: low words of D, S, F and 0
    uint64_t off_face_split;     // u32 [n_states * (nf-1)]  P(face f | spatial) CDF * 2^31
    uint64_t off_rates;          // f64 [n_states * (nf+2)]  (only with keep_rates)
    uint64_t off_map;            // f64 [nc * nf * 3]: rho, shift, u_n per (cell, face)
    uint64_t off_cmap;           // f32x4 [nc] (1D): rho and shift of face 0, then of face 1
    uint64_t off_src_pos;        // f32x4 [n_src] (flag layout): source position (1D: {0, 0, z or r}) and frequency
    uint64_t off_mcell;          // f32x4 [2 nc] (flag layout): {k0, a, sqrt(T), w_min}, {u_x, u_y, u_z, 0}
                                 // (1D: u along +z or +r in the first component)
    uint64_t tally_off;          // int64 word offset of this cloud's tally block
    uint64_t tally_words;
    uint64_t n_pix;              // 3D: escape pixels 2 (ny nz + nx nz + nx ny), after the step histogram
    double tau_th, f_mu, lambda;
    float x0, dx, inv_dx;        // uniform bin grid: first edge, width, 1/width
    int32_t uniform_bins;        // 1 when every bin has the same width
    int32_t flag_layout;         // hot records carry flags and the face split lives in its own
                                 // array (3D grids and 1D hybrid batches); else w3 = F (1D pure)
    float x_crit;                // MC core-skipping threshold (0 = off)
    int32_t dusty;               // dust coefficients present (absorption threshold in lo_words[2..3])
    int32_t n_census;            // census intervals of the time-dependent estimators (0 = none)
    uint64_t off_dust;           // f64 [2 nc]: k_a, k_s per cell (dusty clouds)
    uint64_t off_src_t;          // f64 [2 n_src]: emission window per source entry (0 = flash)
    uint64_t off_census;         // f64 [n_census + 1] census times
    uint64_t census_bin_off;     // int64 word offsets (in the cloud's tally block) of the 'bin'
    uint64_t census_path_off;    //   counts [(n_census+1) n_states], 'path' times [n_census n_states]
    uint64_t census_accel_off;   //   and eq. 18 sums [n_census nc]
    uint64_t off_grp_prob;       // frequency groups: f64 [nb * nb] P(j | j') of eq. 42, row j'
    uint64_t off_grp_alias;      //   u32x2 [nb * nb] Walker alias table per row {threshold, alias}
    int32_t groups;              // thin states carry a frequency group (Sec. 5.3)
    int32_t dust_weight;         // dust absorption by continuous weights (Sec. 2.4)
    uint64_t wspec_off;          // (dust_weight) int64 word offset in the cloud's tally block:
                                 //   sum w t (128-bit, 2^-32 units), sum w t^2 (128-bit, 2^-20
                                 //   units), then the weighted and squared-weight spectra
                                 //   [n_rows (nb + 2)] each, 2^-32 units
};

constexpr double kPathFix = RDDMC_CENSUS_PATH_FIX;   // residence-time fixed point (2^24 per length/c)
constexpr double kWeightFix = RDDMC_WEIGHT_FIX;      // weighted escape tallies (2^32 per unit weight)
constexpr double kLogWMin = 23.025850929940457;      // ln(1 / RDDMC_DUST_WMIN)
constexpr double kAccelFix = RDDMC_CENSUS_ACCEL_FIX; // eq. 18 optical-depth fixed point (2^24)

struct alignas(16) DevHeader {
    int32_t n_clouds;
    int32_t geometry;            // common geometry of the batch
    uint64_t total_packets;
    uint64_t off_clouds;         // DevCloud [n_clouds]
    uint64_t off_prefix;         // u64 [n_clouds+1] flattened packet prefix
    uint32_t error_flags;        // set by the build kernels (see BuildError)
    uint32_t hybrid1d;           // 1D batch walked by the hybrid 1D walk (flag layout, MC tables)
    uint64_t off_voigt;          // f32 [kVoigtN] (3D batches)
    uint64_t off_u0;             // f32 [kU0NA * kU0NX] (3D batches)
    uint32_t dust_weight1d;      // a cloud of the 1D batch carries continuous dust weights
    uint32_t census1d;           // a cloud of the 1D batch has census estimators
};

enum BuildError : uint32_t {
    BE_NONFINITE = 1u,
    BE_THIN = 2u,
};

// ---- launchers (defined in the .hip translation units) ------------------------------
hipError_t launch_build(const DevCloud &c, int cloud_index, uint8_t *d_tables, hipStream_t s);
hipError_t launch_walk(const uint8_t *d_tables, const DevHeader &h, const DevCloud *host_clouds,
                       const rddmc_run &run, uint64_t first, uint64_t count,
                       unsigned long long *d_tally, unsigned long long *d_work, uint64_t work_bytes,
                       hipStream_t s);
hipError_t launch_zero(void *d, size_t words64, hipStream_t s);
hipError_t launch_subwalk(const uint8_t *d_tables, bool moving, uint64_t seed, uint64_t max_steps,
                          const int32_t *d_cloud, const int32_t *d_state, int64_t n, float *d_x, float *d_y,
                          unsigned long long *d_steps, hipStream_t s);
hipError_t launch_surr_features(const uint8_t *d_tables, const uint8_t *d_surr, uint64_t first, uint64_t count,
                                float *d_x, float *d_sw, hipStream_t s);
hipError_t launch_surr_records(const float *d_out, const float *d_sw, uint64_t count, float *d_rec, hipStream_t s);
// mixture-density network (mdn.hip)
uint64_t mdn_param_bytes();
uint64_t mdn_work_bytes(int64_t cap);
int64_t mdn_n_params();
hipError_t mdn_init(void *d_params, uint64_t seed, hipStream_t s);
hipError_t mdn_refresh(void *d_params, hipStream_t s);
hipError_t mdn_forward(void *d_params, void *d_work, int64_t cap, const float *d_x, int n, float *d_out,
                       hipStream_t s);
hipError_t mdn_loss_grad(void *d_params, void *d_work, int64_t cap, const float *d_x, const float *d_y, int n,
                         float *d_loss, hipStream_t s);
hipError_t mdn_adam(void *d_params, int64_t step, float lr, hipStream_t s);
const float *mdn_outputs(void *d_work, int64_t cap);
hipError_t launch_build_redistribution(const DevCloud &c, uint8_t *d_tables, hipStream_t s);
hipError_t launch_build_line_tables(const DevHeader &h, uint8_t *d_tables, hipStream_t s);
hipError_t launch_walk3d(const uint8_t *d_tables, const DevHeader &h, const rddmc_run &run, uint64_t first,
                         uint64_t count, unsigned long long *d_tally, unsigned long long *d_work, hipStream_t s);
hipError_t launch_walk1dh(const uint8_t *d_tables, const DevHeader &h, const rddmc_run &run, uint64_t first,
                          uint64_t count, unsigned long long *d_tally, unsigned long long *d_work, hipStream_t s);
hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                              uint32_t c3, uint64_t n, uint32_t *d_out, hipStream_t s);
int device_cu_count();

}  // namespace rddmc
