/*
 * rddmc.h -- C ABI of the MI355X (gfx950) resonant discrete diffusion Monte Carlo
 * (rDDMC) Lyman-alpha transport library.
 *
 * The method is that of Smith, Tsang, Bromm & Milosavljevic (2017), "Discrete
 * diffusion Lyman alpha radiative transfer": photon packets random-walk on a joint
 * (spatial cell) x (frequency bin) grid.  In every step a packet leaks to one face
 * neighbour (spatial Fick leakage, eq. 10, or the thin/vacuum-face rate of the
 * hybrid section) or to one neighbouring frequency bin (Fokker-Planck leakage,
 * eq. 11), chosen as the smallest of exponential distances (eqs. 15-16); the
 * bin-averaged opacities come from the Voigt expansion of eqs. 12-14.  Packets are
 * removed at the domain boundary (Sec. 2.3) and their escape frequency, face and
 * time are tallied.
 *
 * Conventions for every call
 *   - Host pointers are read only during the call; nothing is retained.
 *   - Device pointers are caller-owned (e.g. torch tensors); the library never
 *     allocates or frees device memory.  Buffers are sized with the *_bytes queries.
 *     (rddmc_transport_static's work area is a device array of the library itself,
 *     created with the library's code on each device, not allocated by a call.)
 *   - Every device operation is enqueued on the caller's stream; results are valid
 *     after that stream is synchronised.  rddmc_build_leakage and rddmc_tally also
 *     synchronise the stream themselves (they stage small host data).
 *   - Errors are returned as rddmc_status; no exceptions cross the ABI.  A
 *     human-readable message for the calling thread is rddmc_last_error().
 *   - Output is a pure function of (batch, seed, packet range): packets are keyed
 *     by their (cloud, packet id) and every tally is an exact integer sum, so
 *     results are bit-identical for any launch shape, shard split or resume.
 *
 * Units: lengths in units of the domain length scale (slab half-width, sphere
 * radius, or one cell for Cartesian grids); times in length / c; frequencies in
 * the dimensionless comoving x = (nu - nu0)/dnu_D of each cell (Sec. 2.1);
 * velocities in km/s; temperatures in K.
 */
#ifndef RDDMC_H
#define RDDMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RDDMC_ABI_VERSION 8

typedef enum {
    RDDMC_OK = 0,
    RDDMC_EINVAL = -1,        /* malformed grid, non-finite or negative input, tau_threshold in (0,2) */
    RDDMC_ESIZE = -2,         /* a caller buffer is smaller than the *_bytes query requires */
    RDDMC_EUNSUPPORTED = -3,  /* a feature combination the library does not implement */
    RDDMC_ENUMERIC = -4,      /* a table entry came out non-finite or non-positive */
    RDDMC_EHIP = -5           /* a HIP runtime call failed */
} rddmc_status;

enum { RDDMC_SLAB = 0, RDDMC_SPHERE = 1, RDDMC_CART3D = 2 };

/* rddmc_medium.flags */
#define RDDMC_FLAG_DIRICHLET  (1u << 0)  /* vacuum faces: 2/(3 k dz^2) instead of eq. 10 with 2 lambda */
#define RDDMC_FLAG_KEEP_RATES (1u << 1)  /* also store the FP64 rates (for table parity checks) */
#define RDDMC_FLAG_GROUPS     (1u << 2)  /* continuous-MC states use frequency groups (Sec. 5.3) */
#define RDDMC_MAX_GROUP_BINS  2048       /* largest n_bins of a cloud with RDDMC_FLAG_GROUPS */
#define RDDMC_FLAG_DUST_WEIGHT (1u << 3) /* dust absorption by continuous packet weights (Sec. 2.4) */
#define RDDMC_DUST_WMIN       1e-10      /* weight below which such a packet is eliminated */
#define RDDMC_WEIGHT_FIX      4294967296.0   /* weighted escape tallies: units of 2^-32 weight */

#define RDDMC_TIME_BINS 128              /* log10-uniform escape-time bins over [1e-3, 1e6] */
#define RDDMC_STEP_BINS 64               /* floor(log2(steps per packet)) buckets */

/*
 * One cloud (medium + grid + sources).  Sec. 2.2 (grid, eqs. 10-14), Sec. 2.3
 * (sources and packets), Sec. 2.5 (bulk velocity).
 *   geometry     RDDMC_SLAB: 1D Cartesian cells along z; RDDMC_SPHERE: radial shells;
 *                RDDMC_CART3D: nx*ny*nz cells, linear index (iz*ny + iy)*nx + ix.
 *   n_cells      {n,1,1} for 1D geometries, {nx,ny,nz} for 3D.
 *   faces[d]     n_cells[d]+1 strictly increasing face coordinates per axis (1D uses
 *                faces[0] only; a sphere's faces[0][0] must be >= 0).
 *   bin_edges    n_bins+1 strictly increasing comoving frequency edges.
 *   k0, temp     per cell line-centre opacity [1/length] (> 0) and temperature [K] (> 0).
 *   vel          NULL for a static medium; else per cell: slab v_z, sphere v_r (one value
 *                per cell), Cartesian (vx,vy,vz) (three values per cell) [km/s].
 *   tau_threshold  0 selects pure DDMC (every state diffusive); > 0 (must be >= 2, the
 *                hybrid section's validity bound) makes states with k_ij w_i below it (w_i the
 *                cell's smallest width) continuous Monte Carlo states.  A 1D batch in which a
 *                cloud has tau_threshold > 0 or x_crit > 0 is walked by the hybrid 1D walk
 *                (slab planes or spherical shells); a 1D batch without is the pure walk.
 *   f_mu         Doppler averaging factor of eq. 20 (1/2 for isotropic escape).
 *   lambda       extrapolation distance of the vacuum/thin-face rate (0.7104).
 *   n_src, src_pos, src_x  source positions (3 doubles each: slab z; sphere r; Cartesian
 *                x,y,z) and comoving frequencies.  A source exactly on an interior face
 *                or bin edge is split with probability 1/2 between its two neighbours;
 *                packets are shared equally between sources.
 *   stream       this cloud's random-stream key: packet p of the cloud draws from Philox
 *                counters (step, p, stream); results of a cloud depend on (seed, stream)
 *                only, not on its position in a batch.  Give clouds of one batch distinct
 *                keys (the Python binding uses the batch index).
 *   n_packets    packets emitted by this cloud (initial flash, equal weights, t = 0).
 *   x_crit       core-skipping of the continuous-MC scattering (hybrid section): a photon
 *                scattered at |x| < x_crit takes the atom's perpendicular speed from the
 *                Maxwellian's tail above x_crit (its square is x_crit^2 + Exp(1)); 0 = off.
 *                This biases the result; it is an option for comparisons, not for parity.
 *   dust_abs, dust_sca  per cell dust absorption k_a and scattering k_s coefficients
 *                [1/length] (>= 0), or NULL (Sec. 2.4): the leakage coefficients use the total
 *                scattering coefficient k_ij + k_s, and absorption competes as one more
 *                exponential distance (rate k_a) in DDMC states; in MC states dust scatters
 *                isotropically and coherently in the comoving frame, or absorbs.  Absorbed
 *                packets are counted, not tallied as escapes.  1D clouds only.
 *                With flags & RDDMC_FLAG_DUST_WEIGHT (Sec. 2.4's second method) nothing is
 *                absorbed: a packet's weight, 1 at emission, is multiplied by exp(-k_a dl) over
 *                every stretch dl it travels (a DDMC step's interaction distance, an MC flight),
 *                packets whose weight falls below RDDMC_DUST_WMIN are eliminated (counted as
 *                absorbed), escapes add their weight (and its square) to weighted spectra, and
 *                the census estimators are weighted along the path: a 'bin' count at a census
 *                time adds the weight then, and a residence [a, b) adds the integral of the
 *                weight over it, w(a) (1 - exp(-k_a (b - a))) / k_a (the paper's path
 *                correction), as does eq. 18's sum.
 *   src_t        per source emission window {t_start, t_end} (0 <= t_start <= t_end): packets
 *                are emitted uniformly in time over it (Sec. 2.3); NULL = a flash at t = 0.
 *                1D clouds only.
 *   n_census, census  time-dependent estimators (eq. 17): n_census intervals between
 *                n_census + 1 increasing times (>= 0).  The tallies then hold, per state, the
 *                number of packets in it at each census time ('bin' estimator) and the
 *                residence time in it during each interval, in units of 2^-24 length/c
 *                ('path' estimator); E_ij,n follows by the packet energy over dV dx (and dt).
 *                Per cell and interval they also hold eq. 18's optical-depth sum, the
 *                acceleration estimator without its energy, c, rho and dt factors: a DDMC
 *                spatial leak of a step that stayed over [t0, t1) in (i, j), moving along
 *                d = -1 (face 0) or +1 (face 1), adds k_ij d times the step's residence in
 *                each interval to cell i (outward leakage) and k_i'j' d to the cell i' it
 *                enters when it lands there in a DDMC state (i', j') (inward leakage); z
 *                component for slabs, radial for spheres; leaks into continuous-MC states
 *                or vacuum count for i only.
 *                1D clouds only; n_census = 0 and census = NULL for none.
 * A 1D batch in which any cloud uses x_crit, dust, emission windows or a census is walked by
 * the hybrid 1D walk.
 *
 * Frequency groups (flags & RDDMC_FLAG_GROUPS; Sec. 5.3, eq. 42): the cloud's continuous-MC
 * states carry a frequency bin instead of a continuous frequency.  A flight meets the bin's
 * averaged opacity k_ij (eq. 14); a scattering draws the outgoing bin from the discrete
 * redistribution P(j | j') = dx_j R_{j'->j} of eq. 42, built from R_II-A of Appendix A (isotropic
 * scattering, coherent in the atom's frame, no recoil) with the incoming frequency uniform over
 * its bin, and bins 0 and n_bins-1 taking every outgoing frequency below and above the grid; the
 * new direction is isotropic, independent of the frequency change.  Crossings keep the bin;
 * escapes are tallied in it.  Needs a 1D geometry, a static medium (vel NULL or zero), one
 * temperature for all cells (one table per cloud), tau_threshold > 0 (thin states exist; a value
 * above every k_ij w_i makes the cloud pure frequency-group Monte Carlo), x_crit = 0 and
 * n_bins <= RDDMC_MAX_GROUP_BINS.  DDMC states, dust, emission windows and census estimators
 * work as for continuous-MC states.
 */
typedef struct {
    int32_t geometry;
    int32_t n_cells[3];
    int32_t n_bins;
    uint32_t flags;
    const double *faces[3];
    const double *bin_edges;
    const double *k0;
    const double *temp;
    const double *vel;
    double tau_threshold;
    double f_mu;
    double lambda;
    int32_t n_src;
    uint32_t stream;
    const double *src_pos;
    const double *src_x;
    uint64_t n_packets;
    double x_crit;
    const double *dust_abs;
    const double *dust_sca;
    const double *src_t;
    int32_t n_census;
    int32_t reserved1;
    const double *census;
} rddmc_medium;

/* A batch of independent clouds transported together (one persistent launch). */
typedef struct {
    int32_t n_clouds;
    int32_t reserved0;
    const rddmc_medium *clouds;
} rddmc_batch;

/*
 * Transport run parameters.
 *   seed         Philox4x32-10 key (Salmon et al. 2011); every packet's stream is keyed
 *                by (seed, cloud stream key, packet id) and indexed by its step count.
 *   first, count packets first .. first+count-1 of the batch's flattened packet space
 *                (cloud 0's packets, then cloud 1's, ...); count = 0 means "to the end".
 *   max_steps    per-packet step cap (>= 1); capped packets are counted, not dropped.
 *   block, grid  threads per block (multiple of 64, <= 1024) and blocks; 0 = automatic.
 *   chunk        steps between refills of finished lanes (0 = automatic).
 *   tail_lanes   once every packet of the run has started, a wave with at most this many
 *                packets left hands them to a cooperative walk in which a whole wave
 *                advances one packet (0 = automatic (16), < 0 = never).  Results are
 *                bit-identical either way.
 *   surrogate    1D clouds: learned escape surrogate (rddmc_surrogate_attach), exact exit
 *                kernel (rddmc_exitkernel_build) or NULL for plain rDDMC; with one, a packet
 *                in a state of its cloud's window leaves the cell by one exit drawn from that
 *                law (checked before every step in moving clouds, at even step counts in
 *                static ones, in the lane walk and the cooperative tail walk alike).
 */
typedef struct {
    uint64_t seed;
    uint64_t first;
    uint64_t count;
    uint64_t max_steps;
    int32_t block;
    int32_t grid;
    int32_t chunk;
    int32_t tail_lanes;
    const void *surrogate;   /* rddmc_surrogate_attach or rddmc_exitkernel_build buffer, or NULL */
} rddmc_run;

/* Per-cloud summary filled by rddmc_tally (FP64 host-side normalisation of the exact
 * integer tallies).  The weighted fields are 0 unless the cloud has RDDMC_FLAG_DUST_WEIGHT. */
typedef struct {
    uint64_t launched;       /* packets emitted in the tallied runs                      */
    uint64_t escaped;        /* packets that left the domain                             */
    uint64_t capped;         /* packets stopped by max_steps                             */
    uint64_t steps_total;    /* leakage events (DDMC steps) summed over packets          */
    uint64_t steps_max;      /* largest per-packet step count                            */
    double   steps_mean;     /* steps_total / (escaped + capped)                         */
    double   t_mean;         /* mean escape time of escaped packets [length / c]         */
    double   t_var;          /* variance of the escape time                              */
    int32_t  n_rows;         /* spectrum rows (escape faces): slab 2, sphere 1, 3D 6     */
    int32_t  n_slots;        /* n_bins + 2 (slot 0 below the grid, slot n_bins+1 above) */
    uint64_t to_mc;          /* hybrid: DDMC -> continuous-MC conversions                 */
    uint64_t to_ddmc;        /* hybrid: continuous-MC -> DDMC conversions                 */
    uint64_t reflected;      /* hybrid: MC packets reflected at a thick interface         */
    uint64_t mc_steps;       /* hybrid: MC events (scatterings and face crossings),       */
                             /* included in steps_total                                  */
    uint64_t n_pix;          /* 3D: escape pixels 2 (ny nz + nx nz + nx ny); else 0       */
    uint64_t surrogate_calls;/* cell exits drawn from the learned surrogate (each counted  */
                             /* as two steps in steps_total)                             */
    uint64_t absorbed;       /* packets absorbed by dust (weights: eliminated below        */
                             /* RDDMC_DUST_WMIN)                                          */
    double   escaped_w;      /* weights: total escaped weight                             */
    double   t_mean_w;       /* weights: weighted mean escape time [length / c]           */
    double   t_var_w;        /* weights: weighted variance of the escape time             */
} rddmc_cloud_stats;

/*
 * Tally read-back.  For cloud c (in batch order) the caller provides
 *   spectrum[c]   int64 [n_rows * (n_bins + 2)] escape counts per face row and lab slot,
 *   time_hist[c]  int64 [RDDMC_TIME_BINS + 2],
 *   step_hist[c]  int64 [RDDMC_STEP_BINS],
 *   stats[c],
 *   pixels[c]     (3D) int64 [n_pix] escape counts per boundary cell: for face f (0 = -x,
 *                 1 = +x, 2 = -y, 3 = +y, 4 = -z, 5 = +z) a block of the face's cells, blocks
 *                 in face order; x faces index iz*ny + iy, y faces iz*nx + ix, z faces
 *                 iy*nx + ix.
 *   census_bin[c] (with a census) int64 [(n_census + 1) * n_cells * n_bins]: packets in each
 *                 state (cell * n_bins + bin) at each census time, time-major.
 *   census_path[c] (with a census) int64 [n_census * n_cells * n_bins]: residence time in each
 *                 state during each census interval, units of 2^-24 length/c, interval-major.
 *   census_accel[c] (with a census) int64 [n_census * n_cells]: eq. 18 optical-depth sums
 *                 per cell and interval (signed), units of 2^-24, interval-major.
 *   spectrum_w[c], spectrum_w2[c]  (RDDMC_FLAG_DUST_WEIGHT) int64 [n_rows * (n_bins + 2)]:
 *                 escaped weight and escaped squared weight per face row and lab slot, units
 *                 of 2^-32 (RDDMC_WEIGHT_FIX).
 * With RDDMC_FLAG_DUST_WEIGHT the census 'bin' counts are weights in units of 2^-24 and the
 * 'path' and eq. 18 sums are weighted by the integral of the weight over each residence.
 * Any pointer array may be NULL to skip that output.
 */
typedef struct {
    int64_t **spectrum;
    int64_t **time_hist;
    int64_t **step_hist;
    rddmc_cloud_stats *stats;
    int64_t **pixels;
    int64_t **census_bin;
    int64_t **census_path;
    int64_t **census_accel;
    int64_t **spectrum_w;
    int64_t **spectrum_w2;
} rddmc_tally_out;

#define RDDMC_CENSUS_PATH_FIX 16777216.0   /* residence-time units per length/c (2^24) */
#define RDDMC_CENSUS_ACCEL_FIX 16777216.0  /* eq. 18 optical-depth units (2^24 per unit) */

/* ---- queries ------------------------------------------------------------------------- */

/* ABI version compiled into the library. */
int32_t rddmc_abi_version(void);

/* Thread-local message for the last non-OK status returned on this thread. */
const char *rddmc_last_error(void);

/* Device bytes needed for the leakage tables of a batch (includes a copy of the inputs). */
rddmc_status rddmc_table_bytes(const rddmc_batch *batch, size_t *bytes);

/* Device bytes for the integer tallies of a batch (caller zeroes them with
 * rddmc_tally_reset or any fill before the first run; runs accumulate). */
rddmc_status rddmc_tally_bytes(const rddmc_batch *batch, size_t *bytes);

/* Device bytes for the transport work area: queue counters and one 48-byte slot per
 * resident lane for packets handed to the cooperative tail walk. */
rddmc_status rddmc_work_bytes(const rddmc_batch *batch, size_t *bytes);

/* ---- the path ------------------------------------------------------------------------ */

/*
 * rddmc_build_leakage -- Sec. 2.2 (eqs. 10, 11, 12-14), the hybrid section's thin/vacuum
 * face rate and the comoving-frame shift of eq. 20.  For every state (cell i, bin j) the
 * GPU computes in FP64:
 *   k_ij = k0_i [calH(a_i, x_j+) - calH(a_i, x_j-)] / dx_j            (eqs. 13-14)
 *   face rates (A_f/dV_i) 2 / (3 (k_ij w_i + k'_nb w_nb))            (eq. 10; A/dV = 1/w
 *            for Cartesian cells, r_f^2/((r_+^3 - r_-^3)/3) for shells), with k'_nb the
 *            neighbour's opacity averaged over the Doppler-shifted image of bin j;
 *            vacuum faces (A_f/dV_i) 2 / (3 (k_ij w_i + 2 lambda));
 *   frequency rates 1 / (dx_j (dx_j/k_ij + dx_j'/k_ij'))             (eq. 11), zero past
 *            the first and last bin (reflecting frequency edges);
 * and stores, per state, a 16-byte hot record {ln2/K (f32), high words of the u64
 * categorical thresholds D = P(lower bin) 2^64 and S = (1 - P(spatial)) 2^64, w3} with
 * w3 = high word of F = S + P(face 0) 2^64 on pure 1D grids, and on 3D grids and hybrid 1D
 * batches a flag word (bit 0 thick, bit 1+f face f leads into a thin state or vacuum,
 * bits 7 / 8 bin j-1 / j+1 thin); plus cold arrays (low words, the face split, k_ij, Doppler
 * maps), and with continuous-MC states the per-cell FP32 record of the MC step and the FP32
 * Voigt (H1 of eq. 12) and atom-velocity sampler tables.
 *   batch        host description, read during the call.
 *   d_tables     device buffer of >= rddmc_table_bytes bytes, 256-byte aligned.
 *   stream       hipStream_t (NULL = default stream); the call synchronises it.
 * For clouds with RDDMC_FLAG_GROUPS it also builds, in FP64 (Sec. 5.3 eq. 42, Appendix A),
 * the discrete redistribution P(j | j') of every pair of bins -- the u-integral of R_II-A over
 * the outgoing bin, exchanged with the x-integration into elementary functions, normalised by
 * the same integral over all x (pi H(a, x')) and averaged over x' in bin j', by Gauss-Legendre
 * rules on segments between the integrands' breakpoints -- and, per incoming bin, a Walker
 * alias table over the row normalised by its sum (rddmc_read_redistribution returns both).
 * Errors: EINVAL (bad grid or inputs), ESIZE (buffer), ENUMERIC (non-finite table entry),
 * EUNSUPPORTED (mixed geometries in one batch; frequency groups in a 3D, moving or
 * non-isothermal cloud), EHIP.
 */
rddmc_status rddmc_build_leakage(const rddmc_batch *batch, void *d_tables, size_t table_bytes,
                                 void *stream);

/*
 * rddmc_transport -- the walk of Sec. 2.3 (eqs. 15-16), emission as an initial flash
 * (Sec. 2.3), Doppler re-binning across faces (Sec. 2.5) and removal at the boundary; on
 * 3D grids and hybrid 1D batches (slab planes, spherical shells) the hybrid scheme
 * (conversions, eq. 39 acceptance, continuous MC with the Voigt opacity of eq. 12 and the
 * redistribution of eq. 41, optional core-skipping), one lane per packet drawing its words
 * in order from its own Philox stream; on pure 1D clouds optionally the learned escape
 * surrogate (run.surrogate; EUNSUPPORTED with a hybrid batch).
 * A persistent kernel: every lane carries one packet; every run.chunk steps finished
 * lanes take new packet ids from a work counter.  One Philox4x32-10 block serves two
 * steps; each step takes one 32-bit word for the exponential path length (time advances
 * in FP64 by dl = -ln(xi)/K) and one as the high word of a u64 uniform compared with the
 * categorical thresholds (lower bin / upper bin / spatial leak); the low word, the face
 * choice and re-binning draws come from an auxiliary block only when needed.  This is
 * the same law as the smallest of independent exponentials, exact to 2^-64 in every
 * event probability.  Escapes add to the integer tallies with device atomics.
 *   batch        the same host description passed to rddmc_build_leakage.
 *   d_tables     tables written by rddmc_build_leakage for that batch.
 *   run          run parameters (see rddmc_run).
 *   d_tally      >= rddmc_tally_bytes bytes; accumulated into (not cleared).
 *   d_work       >= rddmc_work_bytes bytes (a smaller buffer of >= 256 bytes disables the
 *                cooperative tail walk); its counters are cleared by the call (a kernel).
 *   stream       hipStream_t; asynchronous.
 * Errors: EINVAL (run parameters), ESIZE, EUNSUPPORTED (surrogate with a hybrid batch), EHIP.
 */
rddmc_status rddmc_transport(const rddmc_batch *batch, const void *d_tables, const rddmc_run *run,
                             void *d_tally, size_t tally_bytes, void *d_work, size_t work_bytes,
                             void *stream);

/*
 * rddmc_transport_static -- rddmc_transport for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same walk with the same results, bit for bit; the only difference is the work area (queue
 * counters and the cooperative tail walk's export slots), which lives in a device array of
 * RDDMC_STATIC_WORK_BYTES that the library holds on every device it runs on until the process
 * ends.  The call allocates nothing: no hipMalloc, no hipFree, no allocating library routine.
 *   batch, d_tables, run, d_tally, tally_bytes, stream  as for rddmc_transport; the device is
 *                the calling thread's current device (its first call there looks up the
 *                array's device address once).
 * Every call on one device shares that device's array; each call clears the counters and
 * slot flags it uses with a kernel on its stream before walking.  Calls that overlap on one
 * device (two streams, or two threads) race on the array: serialise them.
 * Errors: as rddmc_transport, plus ESIZE when an explicit run->grid x run->block exceeds
 * RDDMC_STATIC_WORK_LANES resident lanes (automatic grids fit by construction on devices of
 * up to 256 compute units; larger devices get a smaller automatic grid).
 */
#define RDDMC_STATIC_WORK_LANES (1ull << 19)
#define RDDMC_STATIC_WORK_BYTES (256ull + 48ull * RDDMC_STATIC_WORK_LANES)   /* 24 MiB + 256 B */
rddmc_status rddmc_transport_static(const rddmc_batch *batch, const void *d_tables, const rddmc_run *run,
                                    void *d_tally, size_t tally_bytes, void *stream);

/* Zero a tally buffer with a kernel on the stream (safe under stream capture). */
rddmc_status rddmc_tally_reset(const rddmc_batch *batch, void *d_tally, size_t tally_bytes,
                               void *stream);

/*
 * rddmc_tally -- copy the exact integer tallies of every cloud to the caller's host
 * arrays and derive the FP64 summaries (mean steps, mean and variance of the escape
 * time from the int64 fixed-point sums).  Synchronises the stream.
 * Errors: EINVAL (NULL out), ESIZE, EHIP.
 */
rddmc_status rddmc_tally(const rddmc_batch *batch, const void *d_tally, size_t tally_bytes,
                         rddmc_tally_out *out, void *stream);

/* ---- validation helpers (same kernels, exposed for parity tests) ---------------------- */

/*
 * Copy back, for cloud `cloud`, the per-state arrays the builder computed:
 *   k         [n_states]          FP64 bin-averaged opacity (eq. 14)
 *   rates     [n_states * (nf+2)] FP64 face rates (nf = 2 for 1D, 6 for 3D), then the
 *             lower and upper frequency rates; only with RDDMC_FLAG_KEEP_RATES (else EINVAL)
 *   hot       [n_states * 16 bytes] hot records {ln2/K f32, D>>32 u32, S>>32 u32, w3 u32}
 *             (w3: F>>32 on 1D grids, the flag word on 3D grids; thin states: all zero)
 *   lo_words  [n_states * 16 bytes] {D & 0xffffffff, S & 0xffffffff, F & 0xffffffff (1D), 0}
 * where D = P(lower bin) * 2^64, S = (1 - P(spatial)) * 2^64 and F = S + P(face 0) * 2^64
 * (rounded).  Any pointer may be NULL.  Synchronises the stream.
 */
rddmc_status rddmc_read_tables(const rddmc_batch *batch, const void *d_tables, int32_t cloud,
                               double *k, double *rates, void *hot, void *lo_words, void *stream);

/*
 * Frequency-group tables of cloud `cloud` (RDDMC_FLAG_GROUPS; else EINVAL):
 *   prob   [n_bins * n_bins] FP64 P(j | j') = dx_j R_{j'->j} (eq. 42) at prob[j' * n_bins + j], as
 *          computed (each row sums to 1 within the quadrature's error; pairs of bins more than 13
 *          apart are 0, below e^-42);
 *   alias  [n_bins * n_bins * 2] u32 {threshold, alias bin} per row j' and column: a draw picks
 *          column c = (w1 * n_bins) >> 32 from a 32-bit word w1 and keeps c when a second word is
 *          below the threshold, else takes the alias bin.
 * Either pointer may be NULL.  Synchronises the stream.
 */
rddmc_status rddmc_read_redistribution(const rddmc_batch *batch, const void *d_tables, int32_t cloud, double *prob,
                                       uint32_t *alias, void *stream);

/*
 * Fill d_out[4*n] with Philox4x32-10 blocks for counters (c0 + i, c1, c2, c3), i < n, under
 * key (k0, k1) -- the generator the walk uses, for known-answer tests.
 */
rddmc_status rddmc_philox_fill(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                               uint32_t c3, uint64_t n, uint32_t *d_out, void *stream);

/* ---- learned escape surrogate: training data and per-state tables ---------------------
 *
 * The surrogate replaces the rest of a packet's DDMC walk inside one thick cell of a 1D
 * cloud (all the frequency steps until the first spatial leak, Sec. 2.3) by one exit
 * (face, exit frequency, time spent) drawn from a learned law.  The law is a function of
 * the state: cell optical width tau_c = k0 w, damping a, entry bin (centre, width), the
 * Doppler shifts into the two neighbours (eq. 20) and the face geometry (A_f/dV) w.
 *
 * Domain of the trained network (states outside it walk plainly): */
typedef struct {
    double tau_min, tau_max;   /* cell optical width k0 w                                  */
    double a_min, a_max;       /* damping parameter                                         */
    double dx_min, dx_max;     /* entry-bin width                                           */
    double shift_max;          /* |Doppler shift| across either face                        */
    double g_min, g_max;       /* face geometry (A_f / dV) w (1 for slabs)                  */
    double x_core;             /* entry-bin centres within |x| <= x_core                    */
} rddmc_surrogate_cfg;

/*
 * Training data from the walk itself: sample q starts in state h_state[q] (cell * n_bins +
 * bin) of cloud h_cloud[q] (a cell with two neighbours; host arrays) and takes DDMC steps
 * until its first spatial leak.  Writes the state's network inputs d_x [n, 16] and the exit
 * d_y [n, 3] = (face 0/1, asinh(x_out / S), ln(dt / w)) with x_out uniform in the exit bin
 * (cell frame), S = (a tau_c)^(1/3), w the cell width; face = -1 if max_steps ran out.
 * d_steps [n] receives each sub-walk's step count.  d_scratch >= 8 n bytes.  Synchronises.
 * Errors: EINVAL (bad start, 3D), ESIZE, EHIP.
 */
rddmc_status rddmc_surrogate_samples(const rddmc_batch *batch, const void *d_tables, const int32_t *h_cloud,
                                     const int32_t *h_state, int64_t n, uint64_t seed, uint64_t max_steps,
                                     void *d_scratch, size_t scratch_bytes, float *d_x, float *d_y,
                                     uint64_t *d_steps, void *stream);

/* Bytes of the surrogate buffer for a batch (windows, staging for max_batch states, one
 * 512-byte sampling record per window state) and the number of window states. */
rddmc_status rddmc_surrogate_bytes(const rddmc_batch *batch, const rddmc_surrogate_cfg *cfg, int64_t max_batch,
                                   size_t *bytes, uint64_t *n_states);

/* The window {i_lo, i_hi, j_lo, j_hi} of cloud `cloud` (empty when i_hi < i_lo): interior
 * cells of a uniform cloud inside the domain (longest contiguous run) x the bins around 0. */
rddmc_status rddmc_surrogate_window(const rddmc_batch *batch, const rddmc_surrogate_cfg *cfg, int32_t cloud,
                                    int32_t *window);

/* Evaluate the network (rddmc_mdn_*) on every window state in batches of max_batch (BF16
 * matrix cores) and store the sampling records in d_surr (>= rddmc_surrogate_bytes,
 * 256-byte aligned); pass d_surr as rddmc_run.surrogate.  Synchronises.
 * Errors: EINVAL, ESIZE, EHIP. */
rddmc_status rddmc_surrogate_attach(const rddmc_batch *batch, const void *d_tables, void *d_params, void *d_work,
                                    int64_t max_batch, const rddmc_surrogate_cfg *cfg, void *d_surr, size_t bytes,
                                    void *stream);

/* ---- exact per-cell exit kernel (a non-learned accelerator) ---------------------------
 *
 * The same hook as the learned surrogate (pass the buffer as rddmc_run.surrogate): a packet
 * in a window state (cell i, bin j) of a pure-DDMC 1D cloud leaves cell i by one exit drawn
 * from the EXACT law of its in-cell walk (Sec. 2.3: the frequency moves of eq. 11 between
 * the cell's bins until the first spatial leak).  With A = I - Q the in-cell jump matrix,
 * built from the walk's own integer event thresholds, the exit (face f, exit bin j') has
 * probability [A^-T e_j](j') p_f(j'); the time spent has the exact conditional mean and
 * variance given j' (two more transposed solves with D = diag(1/K)): a shifted exponential
 * when its squared coefficient of variation c2 <= 1, else a balanced mixture of two
 * exponentials.  The leak from (i, j') then happens as in a walk
 * step (x uniform in the bin, the Doppler map of eq. 20).  Escape spectra are therefore the
 * plain walk's in law; escape-time means and variances are exact, the time distribution's
 * shape within a cell approximate.  FP64 solves whose eliminations add only non-negative
 * terms (pivots in Grassmann-Taksar-Heyman form), so cells with leak probabilities of 1e-12
 * per step are solved to full precision.
 *
 * Window of a cloud: its interior cells (1 .. nc-2; a sphere whose first face is the centre:
 * 0 .. nc-2) x the contiguous
 * bins around the longest expected sub-walk in which every window cell's expected sub-walk is
 * at least min_steps steps.  A row keeps the exit bins whose leak probability reaches `tail`
 * (the kept law renormalised; 24 bytes per kept bin). */
typedef struct {
    double min_steps;          /* >= 1: shortest expected sub-walk worth one exit draw            */
    double tail;               /* in [0, 1e-6]: exit bins below this probability are dropped     */
} rddmc_exitkernel_cfg;

/* Device scratch (256-byte aligned, caller-owned) that the two calls below need. */
rddmc_status rddmc_exitkernel_scratch_bytes(const rddmc_batch *batch, size_t *bytes);

/* Solve the windows' chains and report the buffer size, the number of window states and,
 * if h_windows != NULL, each cloud's window {i_lo, i_hi, j_lo, j_hi} (empty: i_hi < i_lo).
 * d_tables from rddmc_build_leakage.  Synchronises.
 * Errors: EINVAL, ESIZE (scratch), EUNSUPPORTED (3D or hybrid batch), ENUMERIC, EHIP. */
rddmc_status rddmc_exitkernel_bytes(const rddmc_batch *batch, const void *d_tables, const rddmc_exitkernel_cfg *cfg,
                                    void *d_scratch, size_t scratch_bytes, size_t *bytes, uint64_t *n_states,
                                    int32_t *h_windows, void *stream);

/* Write the exit kernel into d_ek (>= rddmc_exitkernel_bytes, 256-byte aligned, caller-owned;
 * the same cfg).  Synchronises.  Errors: as rddmc_exitkernel_bytes, ESIZE for d_ek. */
rddmc_status rddmc_exitkernel_build(const rddmc_batch *batch, const void *d_tables, const rddmc_exitkernel_cfg *cfg,
                                    void *d_scratch, size_t scratch_bytes, void *d_ek, size_t bytes, void *stream);

/* Training samples of the learned surrogate drawn from the exact in-cell law instead of run
 * sub-walks (for cells whose sub-walks are too long): pair q = (cloud h_cloud[q], state
 * h_state[q] in a cell with two neighbours) receives h_count[q] consecutive rows of d_x
 * [rows, 16] and d_y [rows, 3], in pair order, in the layout of rddmc_surrogate_samples (exit
 * face, asinh(x_out / S), ln(dt / w)); (face, exit bin) follow the exact law of the in-cell
 * walk, x_out is uniform in the exit bin and dt is drawn as in the exact exit kernel (exact
 * conditional mean and variance).  d_scratch >= 20 n_pairs + 88 nb_max n_pairs bytes (plus
 * alignment: 256 bytes per region).  Synchronises.  Errors: EINVAL, ESIZE, EUNSUPPORTED
 * (3D or hybrid), EHIP. */
rddmc_status rddmc_exitlaw_samples(const rddmc_batch *batch, const void *d_tables, const int32_t *h_cloud,
                                   const int32_t *h_state, const int32_t *h_count, int64_t n_pairs, uint64_t seed,
                                   void *d_scratch, size_t scratch_bytes, float *d_x, float *d_y, void *stream);

/* ---- learned escape surrogate: mixture-density network --------------------------------
 *
 * A multilayer perceptron 16 -> 256 -> 256 -> 256 -> 128 with exact GELU whose outputs are
 * a 16-component mixture over (exit face of a thick DDMC cell, y1 = asinh-scaled exit
 * frequency, y2 = log time spent); it learns the law of a packet's exit from one cell from
 * sub-walks of the DDMC walk itself (the surrogate calls below).  Products run on BF16
 * matrix cores with FP32 accumulation; parameters, gradients and the Adam state are FP32.
 *
 * d_params   device buffer of param_bytes (caller-owned): FP32 theta (n_params values in
 *            the order W1 [16,256], b1, W2 [256,256], b2, W3, b3, W4 [256,128], b4, each W
 *            input-major), Adam moments, gradient, BF16 weight copies.
 * d_work     device buffer of work_bytes for batches of up to max_batch samples.
 * d_x        FP32 [n, 16] inputs; d_y FP32 [n, 3] targets (face as 0/1, y1, y2).
 * Errors: EINVAL (NULL, sizes), EHIP.
 */
rddmc_status rddmc_mdn_bytes(int64_t max_batch, size_t *param_bytes, size_t *work_bytes, int64_t *n_params);

/* Glorot-uniform weights, zero biases and Adam state from `seed`. */
rddmc_status rddmc_mdn_init(void *d_params, uint64_t seed, void *stream);

/* Upload theta (FP32, n_params values) and reset the optimiser; synchronises. */
rddmc_status rddmc_mdn_set(void *d_params, const float *h_theta, void *stream);

/* Copy theta and / or the last gradient (each may be NULL) to the host; synchronises. */
rddmc_status rddmc_mdn_get(const void *d_params, float *h_theta, float *h_grad, void *stream);

/* Raw outputs (FP32 [n, 128]) of the network for n inputs. */
rddmc_status rddmc_mdn_forward(void *d_params, void *d_work, int64_t max_batch, const float *d_x, int32_t n,
                               float *d_out, void *stream);

/* Mean negative log-likelihood of (d_x, d_y) into *d_loss (device FP32, may be NULL) and its
 * gradient with respect to theta into the parameter buffer's gradient slot. */
rddmc_status rddmc_mdn_loss_grad(void *d_params, void *d_work, int64_t max_batch, const float *d_x,
                                 const float *d_y, int32_t n, float *d_loss, void *stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the stored gradient; `step` counts from 1. */
rddmc_status rddmc_mdn_adam(void *d_params, int64_t step, float lr, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RDDMC_H */
