/* sse.h -- C ABI of the MI355X scatter-estimation library (libsse.so).
 *
 * The library computes Monte Carlo scatter estimates for PET in the way of
 * Noe et al., "Object independent scatter sensitivities for PET, applied to
 * scatter estimation through fast Monte Carlo simulation" (arXiv 2509.05047):
 * annihilation pairs are transported through a voxel attenuation / activity
 * phantom to a plain detection cylinder; every detected single gets a
 * detection probability from a 5D LUT; each coincidence adds p1 * p2 to its
 * TOF sinogram bin; the resulting "LUT scatter" sinogram is multiplied by a
 * LUT-specific scatter-sensitivity sinogram (Methods, "Scatter simulation",
 * Fig. 3) and may be Gaussian-smoothed first (Methods, "Known activity
 * distribution, very limited simulation time").
 *
 * Conventions for every call:
 *  - Units: mm, keV.  Positions are relative to the scanner centre, z along
 *    the scanner axis.
 *  - Sinograms are C-order arrays [tof][plane][view][rad] (radial fastest).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it and is asynchronous unless stated.
 *  - Pointers marked "device" must point to device memory of the context's
 *    GPU; "host" to ordinary host memory.  `mem` arguments (SSE_MEM_HOST or
 *    SSE_MEM_DEVICE) say which kind an input is.
 *  - Inputs are borrowed for the duration of the call and copied; the library
 *    owns everything it allocates; outputs are caller-owned.
 *  - No C++ exception crosses the ABI.  Every call returns an sse_status;
 *    sse_last_error() gives a thread-local message for the last failure.
 *    Device errors of asynchronous work surface at the next synchronising
 *    call as SSE_EDEVICE.
 */
#ifndef SSE_H
#define SSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSE_ABI_VERSION 1

typedef enum {
  SSE_OK = 0,
  SSE_EINVAL = 1,  /* invalid argument or descriptor */
  SSE_ENOMEM = 2,  /* device or host allocation failed */
  SSE_EDEVICE = 3, /* HIP runtime error */
  SSE_ESTATE = 4,  /* call not valid in the current state (e.g. no LUT loaded) */
  SSE_EBUSY = 5    /* resource in use */
} sse_status;

typedef enum { SSE_F32 = 0, SSE_F16 = 1, SSE_BF16 = 2 } sse_dtype;
typedef enum { SSE_MEM_HOST = 0, SSE_MEM_DEVICE = 1 } sse_mem;

typedef struct sse_ctx sse_ctx;
typedef uint32_t sse_phantom_id;

/* Scanner: a cylinder of radius radius_mm and length length_mm on which every
 * crossing photon is detected (Methods, "Scatter simulator description").
 * Crystal c covers azimuth [2 pi c / n, 2 pi (c+1) / n); rings tile
 * [-L/2, L/2) (Methods, "Signa PET/MR description": 448 crystals in 28
 * modules of 16, 45 rings in 5 blocks of 9).  max_ring_diff < 0 keeps all. */
typedef struct {
  int32_t n_crystals;          /* even, > 0 */
  int32_t n_rings;             /* > 0 */
  float radius_mm;             /* > 0 */
  float length_mm;             /* > 0 */
  int32_t crystals_per_module; /* > 0; transaxial LUT axis bins c mod this */
  int32_t rings_per_block;     /* > 0; axial LUT axis bins r mod this */
  int32_t max_ring_diff;
} sse_scanner_desc;

/* TOF sinogram: n_view = n_crystals / 2, n_plane = 2 n_rings - 1 (plane =
 * r1 + r2), n_rad odd <= n_crystals - 1 (radial index rho + (n_rad-1)/2),
 * TOF bin = floor(tau / tof_bin_mm + n_tof / 2) of the offset tau along the
 * LOR; tof_sigma_mm is the Gaussian jitter of tau (0 = none).  The paper
 * takes the TOF bin from the photons' time difference (Methods, "Scatter
 * simulator description") with 380 ps FWHM resolution (Methods, "Simulated
 * scans in GATE"). */
typedef struct {
  int32_t n_rad, n_view, n_plane, n_tof;
  float tof_bin_mm;            /* > 0 */
  float tof_sigma_mm;          /* >= 0 */
} sse_sino_desc;

/* Photon physics.  Window [e_lo, e_hi] keV (the paper: 300-650 keV with the
 * LUT at 0.1 % resolution, 425-650 keV without, Methods, "Scatter simulator
 * description"); photons below e_kill are dropped; e_fwhm_frac is the energy
 * blur FWHM at 511 keV (0 = none).  Attenuation is separable,
 * mu(x, E) = mu511(x) g(E), with g(E) = f_compton KN(E)/KN(511) +
 * f_rayleigh (511/E)^2 + f_photo (511/E)^3; Rayleigh angles follow the
 * Thomson factor times (1 + beta (E/511)^2 (1 - cos))^-2.  mu_majorant = 0
 * uses the phantom maximum as the Woodcock majorant at 511 keV. */
typedef struct {
  float e_lo_kev, e_hi_kev, e_kill_kev, e_fwhm_frac;
  float f_compton, f_rayleigh, f_photo; /* >= 0, sum > 0 */
  float rayleigh_beta;                  /* > 0 */
  float mu_majorant;                    /* 0 or >= max mu511 (1/mm) */
  int32_t max_interactions;             /* >= 1 */
} sse_physics_desc;

/* Voxel phantom: nx * ny * nz voxels, x fastest (index (z*ny + y)*nx + x),
 * box [lo, lo + n * voxel); air outside.  The box's transaxial corners must
 * lie inside the cylinder. */
typedef struct {
  int32_t nx, ny, nz;
  float voxel_mm[3];
  float lo_mm[3];
} sse_phantom_desc;

/* 5D detection-probability LUT, row-major [E][theta_t][theta_a][ct][ca]
 * (Methods, "Photon detection probability LUT"): energy bins of
 * (e_max - e_min) / dims[0] keV from e_min (clamped), transaxial and axial
 * incidence angle bins of 180/dims deg over [-90, 90] (Fig. 5 caption).
 * Plain cylinder: in-module crystal ct = (c mod crystals_per_module) *
 * dims[3] / crystals_per_module, in-block ring ca = (r mod rings_per_block) *
 * dims[4] / rings_per_block.  With gaps (sse_set_gaps) the crystal axes
 * carry the virtual gap indices instead: dims[3] = crystals_per_module + 2,
 * dims[4] = n_blocks (rings_per_block + 2), or 1 to ignore the axis.  Values
 * in [0, 1]. */
typedef struct {
  int32_t dims[5];
  float e_min_kev, e_max_kev;
} sse_lut_desc;

/* Statistics counters (unsigned 64-bit each), accumulated by sse_simulate. */
enum {
  SSE_ST_HISTORIES = 0, SSE_ST_STEPS, SSE_ST_REAL, SSE_ST_COMPTON, SSE_ST_RAYLEIGH,
  SSE_ST_ABSORBED, SSE_ST_KILLED, SSE_ST_CAPPED, SSE_ST_ESCAPED, SSE_ST_DETECTED,
  SSE_ST_IN_WINDOW, SSE_ST_SCATTER, SSE_ST_TRUE, SSE_ST_REJ_WINDOW, SSE_ST_REJ_SAME,
  SSE_ST_REJ_RING, SSE_ST_REJ_RADIAL, SSE_ST_REJ_TOF, SSE_ST_RNG_BLOCKS,
  SSE_ST_REJ_GAP,       /* coincidences discarded for a photon in a gap */
  SSE_ST_GAP_ASSIGNED,  /* gap hits of evaluated coincidences given an edge crystal or ring */
  SSE_ST_COUNT
};

/* Per-history record (128 bytes), for parity checks and list-mode style
 * inspection.  Word layout:
 *   0 outcome: 0 scatter, 1 true, 2 a photon undetected, 3 outside the energy
 *     window, 4 same crystal, 5 ring difference, 6 outside the radial FOV,
 *     7 outside the TOF range, 8 a photon in a gap (discard policy); bit 8
 *     set if either photon scattered
 *   1,2 flat sinogram bin (low, high word; all ones if none)
 *   3 emission voxel   4 weight p_A p_B (float)   5 TOF offset tau (float, mm)
 *   6 Woodcock tentative steps of both photons    7 zero
 *   8..19 photon A, 20..31 photon B: hit x, y, z, direction x, y, z, energy,
 *     blurred energy, path length (floats), crystal | ring << 16 (for a hit
 *     in a gap the nearest edge crystal and ring, before any edge-LUT draw),
 *     flat LUT index (both all ones if the photon is not detected in the
 *     window),
 *     n_compton | n_rayleigh << 8 | fate << 16 (fate 0 detected, 1 absorbed,
 *     2 dropped below e_kill, 3 interaction/step cap, 4 missed the cylinder). */
typedef struct { uint32_t w[32]; } sse_history_record;

/* Outputs of sse_simulate (all device pointers, caller-owned, accumulated
 * into: zero them before the first call of a run).  scatter_counts and
 * scatter_weights are required (n_bins entries each, 4- and 8-byte aligned);
 * the rest may be NULL.  records, if given, receives one record for every
 * history h with (h - h_offset) % record_stride == 0, at index
 * (h - h_offset) / record_stride. */
typedef struct {
  uint32_t* scatter_counts;
  double* scatter_weights;
  uint32_t* true_counts;
  double* true_weights;
  unsigned long long* stats;     /* SSE_ST_COUNT entries */
  sse_history_record* records;
  uint64_t record_stride;        /* >= 1 when records != NULL */
} sse_outputs;

/* Version of this ABI (SSE_ABI_VERSION). */
int sse_abi_version(void);

/* Thread-local message of the last failed call ("" if none).  The pointer is
 * valid until the next call on the same thread. */
const char* sse_last_error(void);

/* Create a context on HIP device `device`.  Descriptors are validated and
 * copied.  *out receives the context (library-owned; free with
 * sse_destroy).  Errors: SSE_EINVAL for a bad descriptor (odd crystal count,
 * n_view != n_crystals/2, n_plane != 2 n_rings - 1, even or too large n_rad,
 * non-positive sizes, invalid physics), SSE_EDEVICE. */
sse_status sse_create(sse_ctx** out, int device, const sse_scanner_desc* scanner,
                      const sse_sino_desc* sino, const sse_physics_desc* physics);

/* Wait for the context's pending work and free everything it owns.
 * Errors: SSE_EBUSY while a server runs on the context (stop it first). */
sse_status sse_destroy(sse_ctx* ctx);

/* Load a phantom: mu511_per_mm (attenuation at 511 keV, 1/mm) and activity
 * (any unit, >= 0, not all zero), nx*ny*nz floats each, host or device
 * (`mem`).  The emission sampler (an integer alias table over voxels) is
 * built on the host.  The activity and attenuation images are the
 * simulator's inputs (Fig. 3 caption).  *out receives the phantom id.
 * Synchronous with respect to the host inputs.  Allowed while a server runs
 * on the context (thread-safe against its scheduler; the new phantom's
 * device memory counts against the server's HBM budget).  Errors:
 * SSE_EINVAL (bad descriptor, negative or non-finite values, all-zero
 * activity, box outside the cylinder), SSE_ENOMEM. */
sse_status sse_load_phantom(sse_ctx* ctx, const sse_phantom_desc* desc, const float* mu511_per_mm,
                            const float* activity, int mem, void* stream, sse_phantom_id* out);

/* Replace a loaded phantom's activity (rebuilds its emission sampler); the
 * iterative estimation loop re-simulates with updated activity (Methods,
 * "Unknown activity distribution, very limited simulation time").  The call
 * first waits for every sse_simulate / sse_simulate_noalloc enqueued earlier
 * on the context, on any stream (they read the sampler), and returns with
 * the new sampler in place.  Errors: SSE_EINVAL, SSE_EBUSY while a server
 * runs on the context (its requests read the sampler). */
sse_status sse_update_activity(sse_ctx* ctx, sse_phantom_id id, const float* activity, int mem,
                               void* stream);

/* Free a phantom.  Errors: SSE_EINVAL (unknown id), SSE_EBUSY while a
 * server runs on the context. */
sse_status sse_unload_phantom(sse_ctx* ctx, sse_phantom_id id);

/* Load the 5D LUT (see sse_lut_desc) in F32, F16 or BF16 (`dtype`), host or
 * device.  Values are checked to lie in [0, 1].  Replaces any previous LUT.
 * Errors: SSE_EINVAL (bad dims, range or values), SSE_ENOMEM, SSE_EBUSY
 * while a server runs on the context (its requests hold the LUT). */
sse_status sse_load_lut(sse_ctx* ctx, const sse_lut_desc* desc, const void* values, int dtype,
                        int mem, void* stream);

/* ------------------------------------------------------------------------ */
/* Gaps between modules and blocks                                           */
/* ------------------------------------------------------------------------ */
/* The paper's scanner has gaps between its transaxial modules (given by the
 * angle they subtend) and its axial blocks (given by their width); a photon
 * crossing the detection cylinder in a gap is discarded with its
 * coincidence, assigned to the nearest edge crystal, or assigned at random
 * to one of the two edge crystals by an edge-crystal LUT, depending on the
 * LUT in use (Methods, "Scatter simulator description", "Photon detection
 * probability LUT", "Edge crystal assignment LUT").
 *
 * Geometry.  Module m of n_modules = n_crystals / crystals_per_module covers
 * azimuth [m D, (m + 1) D), D = 2 pi / n_modules, with half a gap at either
 * end and its crystals sharing the rest equally.  Block b of n_blocks =
 * n_rings / rings_per_block holds rings of pitch (L - (n_blocks - 1) w) /
 * n_rings, blocks separated by gaps of width w, none at the scanner's ends.
 * A hit in the half of a gap next to a module (block) takes that module's
 * (block's) virtual LUT index and, as nearest edge crystal, its edge crystal.
 * All of this is evaluated in binary64.
 *
 * Edge LUTs.  For the edge-LUT policy, one table for the transaxial gaps and
 * one for the axial gaps, row-major [angle][position], edge_n_angle bins of
 * the incidence angle over [-90, 90] degrees (the LUT's transaxial resp.
 * axial angle, positive towards the upper side: larger azimuth, larger z)
 * and edge_n_pos bins of the position across the gap (from the lower side's
 * edge); each entry is the probability that the photon goes to the lower
 * side's edge crystal (sse_build_edge_lut computes them).  A uniform from
 * the history's stream (after photon B's transport: photon A's transaxial,
 * then axial gap, then photon B's; before the TOF jitter) below the entry
 * picks the lower side.  The LUT probability of a gap photon is the one of
 * its virtual index, whichever crystal it goes to. */
typedef enum { SSE_GAP_DISCARD = 0, SSE_GAP_NEAREST = 1, SSE_GAP_EDGE_LUT = 2 } sse_gap_policy;

typedef struct {
  float transaxial_gap_rad;    /* 0 <= angle < 2 pi / n_modules */
  float axial_gap_mm;          /* >= 0, (n_blocks - 1) * width < length */
  int32_t policy;              /* sse_gap_policy */
  int32_t edge_n_angle;        /* edge LUT bins (EDGE_LUT policy; >= 1) */
  int32_t edge_n_pos;
  int32_t reserved;            /* 0 */
} sse_gap_desc;

/* Switch the gap model on (desc != NULL) or off (desc == NULL, the plain
 * cylinder).  n_crystals must be a multiple of crystals_per_module and
 * n_rings of rings_per_block; a loaded LUT must have the gap layout on its
 * crystal axes (see sse_lut_desc).  edge_transaxial / edge_axial (host or
 * device per `mem`, edge_n_angle * edge_n_pos floats in [0, 1] each) are
 * read for the EDGE_LUT policy only and copied.  Errors: SSE_EINVAL,
 * SSE_EBUSY while a server runs on the context. */
sse_status sse_set_gaps(sse_ctx* ctx, const sse_gap_desc* desc, const float* edge_transaxial,
                        const float* edge_axial, int mem, void* stream);

/* Geometry of one kind of gap for the edge-crystal LUT: two crystal blocks
 * depth_mm deep either side of a gap gap_mm wide (for transaxial gaps, the
 * gap angle times the detection radius: the angle between the two modules
 * is neglected, as in the paper), the detection cylinder doi_mm below their
 * front faces, crystal attenuation mu_per_mm (LYSO at 511 keV: about
 * 0.087 / mm). */
typedef struct {
  float gap_mm, depth_mm, doi_mm, mu_per_mm;
  int32_t n_angle, n_pos;
} sse_edge_geom;

/* Host helper: the edge-crystal LUT of Eq. (1)-(3) ("Edge crystal assignment
 * LUT").  For a ray through the detection surface at position x across the
 * gap and incidence angle theta (the bin centres), l1 and l2 are its path
 * lengths in the two blocks (taken as unbounded away from the gap); the
 * block the ray meets first absorbs it with p_first = 1 - exp(-mu l_first),
 * the other with p_second = exp(-mu l_first) (1 - exp(-mu l_second)) (the
 * paper prints the first factor as a transmission; this is the reading that
 * makes both probabilities of detection); out = p_lower / (p_lower +
 * p_upper), or the nearer side (0.5 at the centre) for a ray through
 * neither block.  out: host, n_angle * n_pos floats, [angle][position].
 * Errors: SSE_EINVAL. */
sse_status sse_build_edge_lut(const sse_edge_geom* geom, float* out);

/* Self-check of the device division: the transport forms its binary32
 * quotients as the hardware reciprocal refined by one Newton step, then one
 * remainder correction (Markstein 1990), which is the correctly rounded
 * quotient when the refined reciprocal is the correctly rounded 1/b.  This
 * call checks that premise for all 2^23 significands and compares n_random
 * quotients of hashed operands (exponents -20..20; `seed` varies them) with
 * the IEEE operator on the context's GPU.  Both counts are 0 on a conforming
 * device.  Synchronous.  Errors: SSE_EINVAL, SSE_EDEVICE. */
sse_status sse_check_division(sse_ctx* ctx, uint64_t n_random, uint32_t seed, uint64_t* reciprocal_mismatches,
                              uint64_t* quotient_mismatches);

/* Load the scatter-sensitivity sinogram (float, >= 0), with the full
 * sinogram shape (has_tof_axis = 1) or without the TOF axis (shared by all
 * TOF bins).  Methods, "Scatter sensitivity sinogram". */
sse_status sse_load_sensitivity(sse_ctx* ctx, const float* sens, int has_tof_axis, int mem,
                                void* stream);

/* Simulate histories h_offset .. h_offset + n_histories - 1 of the run
 * `seed` and accumulate their coincidences into `out`.  A history is one
 * annihilation: two back-to-back 511 keV photons from a voxel drawn by
 * activity, uniform inside it.  Each photon is tracked with Woodcock steps,
 * Compton (Klein-Nishina), Rayleigh and photoabsorption until it leaves the
 * voxel box, then intersected with the cylinder; a detected single in the
 * window gets crystal, ring and LUT probability; a coincidence of two
 * singles in different crystals within the ring-difference, radial and TOF
 * ranges adds 1 to counts and p_A p_B (binary32 product) to weights
 * (binary64) of its bin, in the scatter pair if either photon scattered,
 * else in the trues pair (Methods, "Scatter simulator description";
 * Introduction, footnote on scatter).  Random numbers: Philox4x32-10 keyed
 * by the seed, counter (block, h, substream); history results do not depend
 * on the launch, so runs split over calls or GPUs sum to the same result.
 * Device memory: the context's pair buffer (sse_set_pair_buffer) and a few
 * words of work-list scratch, allocated on first use and grown for longer
 * runs up to the buffer's limit.  Asynchronous on `stream`.  Errors:
 * SSE_EINVAL (unknown phantom, null or misaligned outputs, record stride 0),
 * SSE_ESTATE (no LUT loaded), SSE_ENOMEM (no pair buffer of 2^22 records). */
sse_status sse_simulate(sse_ctx* ctx, sse_phantom_id id, uint64_t n_histories, uint64_t seed,
                        uint64_t h_offset, const sse_outputs* out, void* stream);

/* sse_simulate without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid it).  Same histories, arguments and results as sse_simulate
 * (counts bit for bit; weights up to the order of their binary64 sums), on
 * the production path only: out->stats and out->records must be NULL.  The
 * kernels' scratch (work-list parameters, counters and the pair buffer) is a
 * fixed 256 MiB device array of the library, one per GPU, held from the
 * first sse_create on that GPU until the process ends; runs longer than one
 * launch's share of it are split into launches, which costs a little speed.
 * The call allocates nothing and frees nothing.  Calls of one context are
 * ordered with its other simulations; calls of different contexts on one GPU
 * share the array and race if they overlap: order them (one stream).
 * Asynchronous on `stream`.  Errors: those of sse_simulate, SSE_EINVAL for
 * stats or records, or if the GPU's resident transport grid would need more
 * pair records than the array holds. */
sse_status sse_simulate_noalloc(sse_ctx* ctx, sse_phantom_id id, uint64_t n_histories, uint64_t seed,
                                uint64_t h_offset, const sse_outputs* out, void* stream);

/* Pair pruning (enable = 1; off after sse_create): photon B of a history is
 * not tracked when photon A ended outside the energy window (not detected,
 * or detected outside [e_lo, e_hi]).  Such a history adds to no sinogram
 * whatever photon B does, and every history keeps its own random stream, so
 * counts are unchanged bit for bit and weights up to the order of their
 * binary64 sums.  A history then costs about half the transport work when
 * A misses.  Calls that collect statistics or per-history records track
 * both photons whatever this setting, since both describe photon B.  Applies
 * to sse_simulate and to the requests of servers started afterwards.
 * Errors: SSE_EINVAL (enable not 0 or 1), SSE_EBUSY while a server runs on
 * the context. */
sse_status sse_set_pair_pruning(sse_ctx* ctx, int enable);

/* Size limit of the context's pair buffer, in records of 80 bytes (default
 * 2^27, 10.7 GB).  The buffer carries the in-window pairs from the transport
 * kernel to the coincidence kernel; sse_simulate allocates it on first use,
 * at most max_records and no more than a run needs.  A run whose pairs do not
 * fit goes through several launches, each of which stops taking histories
 * when the buffer is nearly full, so a smaller buffer costs launches, not
 * results: counts are the same bit for bit and weights up to the order of
 * their binary64 sums.  The current buffer is freed (after the device is
 * idle) and the next sse_simulate allocates one under the new limit.
 * Errors: SSE_EINVAL (max_records outside 2^22 .. 2^31), SSE_EBUSY while a
 * server runs on the context. */
sse_status sse_set_pair_buffer(sse_ctx* ctx, uint64_t max_records);

/* Per-kernel timing of the production launches, for measurement.  With
 * enable = 1, every later sse_simulate on its production path (no
 * statistics, no records) records HIP events on its stream before and after
 * each transport kernel and each coincidence kernel it launches, for up to
 * max_launches launches (1 .. 2^20; events created here); enable = 0 frees
 * them.  The call first waits for the context's earlier simulations.
 * sse_read_kernel_timing waits for the recorded launches, returns the
 * launches recorded (and those beyond max_launches, not recorded) and the
 * summed kernel durations in milliseconds, and starts a new count.
 * Errors: SSE_EINVAL, SSE_ESTATE (timing off), SSE_EDEVICE. */
typedef struct {
  uint64_t launches;           /* launches recorded */
  uint64_t dropped;            /* launches after max_launches were reached */
  double transport_ms;         /* summed transport kernel durations */
  double coincidence_ms;       /* summed coincidence kernel durations */
} sse_kernel_timing;

sse_status sse_set_kernel_timing(sse_ctx* ctx, int enable, uint32_t max_launches);
sse_status sse_read_kernel_timing(sse_ctx* ctx, sse_kernel_timing* out);

/* Expected annihilations per simulated history: sum(activity) * voxel volume
 * (ml) * acq_seconds * factor / n_histories (binary64).  The simulator's
 * output is absolutely scaled (Discussion); `factor` carries a global
 * correction such as the paper's real-scan factors (Methods, "Real scans").
 * Errors: SSE_EINVAL. */
sse_status sse_emission_scale(sse_ctx* ctx, sse_phantom_id id, uint64_t n_histories,
                              double acq_seconds, double factor, double* scale);

/* out[b] = (float)(scale * W[b] * sens[b]) computed in binary64 (device
 * pointers, n_bins each; W and out must not overlap).  Methods, "Scatter
 * sensitivity sinogram".  Errors: SSE_EINVAL, SSE_ESTATE (no sensitivity). */
sse_status sse_apply_sensitivity(sse_ctx* ctx, const double* W, double scale, float* out,
                                 void* stream);

/* Total scatter of the estimate in binary64: total[0] = sum over bins of
 * (scale * W[b]) * sens[b] (the sensitivity broadcast over TOF when it has
 * no TOF axis), reduced on the device in a fixed order, so repeated calls
 * give the same bits.  With a smoothed estimate the paper's smoothing keeps
 * the total of the LUT scatter but not of its product with the
 * sensitivity; this is the total of the unsmoothed estimate (Methods,
 * "Scatter sensitivity sinogram": the LUT scatter times the sensitivity is
 * the absolutely scaled scatter estimate).  W: device, n_bins binary64;
 * total: device, one binary64 (caller-owned).  Asynchronous on stream.
 * Errors: SSE_EINVAL, SSE_ESTATE (no sensitivity), SSE_ENOMEM. */
sse_status sse_total_scatter(sse_ctx* ctx, const double* W, double scale, double* total, void* stream);

/* Separable Gaussian smoothing of a float sinogram (device, n_bins each;
 * in == out allowed) with sigma_bins = {radial, view, plane} (0 skips an
 * axis), kernel truncated at floor(truncate * sigma + 0.5) bins and
 * normalised.  Radial and plane edges reflect (edge bin repeated); views are
 * periodic over 180 degrees, continuing across the seam on the same LORs
 * seen from the other end (radial and TOF indices reversed); TOF bins are
 * not smoothed.  Methods, "Known activity distribution, very limited
 * simulation time" (the paper uses FWHM [9, 6, 10.5] bins).  Uses
 * library-owned scratch.  Errors: SSE_EINVAL. */
sse_status sse_gaussian_smooth(sse_ctx* ctx, const float* in, float* out, const float sigma_bins[3],
                               float truncate, void* stream);

/* Fused post-processing: with sigma_bins NULL, out = scale * W * sens as
 * sse_apply_sensitivity; otherwise out = sens * G(float(scale * W)), the
 * smoothed LUT scatter times the sensitivity sinogram (the paper multiplies
 * by the sensitivity after smoothing, Methods, "Known activity distribution,
 * very limited simulation time").  Errors: as the two calls above. */
sse_status sse_finalize(sse_ctx* ctx, const double* W, double scale, const float* sigma_bins,
                        float truncate, float* out, void* stream);

/* Smoothing normalisation sinogram (Methods, "Known activity distribution,
 * very limited simulation time"): the simulated LUT scatter of a reference
 * object (the paper: a 40 cm cylinder), heavily smoothed and divided by its
 * unsmoothed self, N[b] = G_heavy(S)[b] / S[b] with S = float(scale * W) and
 * G_heavy the smoothing of sse_gaussian_smooth with sigma_bins.  Bins where
 * S or G_heavy(S) is not positive get N = 1 (a reading: the paper does not
 * say).  W: device, n_bins binary64 weights of the reference simulation;
 * norm_out: device, n_bins binary32, caller-owned.  Asynchronous on stream.
 * Errors: as sse_gaussian_smooth. */
sse_status sse_smoothing_normalisation(sse_ctx* ctx, const double* W, double scale, const float sigma_bins[3],
                                       float truncate, float* norm_out, void* stream);

/* Normalised finalize: out = sens * G(S * N) / N with S = float(scale * W),
 * N a smoothing normalisation sinogram (entries <= 0 count as 1) and G the
 * smoothing of sse_gaussian_smooth: the simulator output is multiplied by N
 * to remove the LUT's high-frequency structures, smoothed, divided by N to
 * re-apply them, and multiplied by the scatter-sensitivity sinogram (same
 * passage).  The paper smooths with FWHM [9, 6, 10.5] radial, view and plane
 * bins (sigma = FWHM / 2.35482).  One fused three-pass run over all planes.
 * W, norm, out: device, n_bins each; out must not overlap W or norm.
 * Errors: SSE_EINVAL, SSE_ESTATE (no sensitivity). */
sse_status sse_finalize_normalised(sse_ctx* ctx, const double* W, double scale, const float* norm,
                                   const float sigma_bins[3], float truncate, float* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Reconstruction for the joint activity / scatter estimation loop           */
/* ------------------------------------------------------------------------ */
/* The paper estimates scatter iteratively when the activity is unknown:
 * reconstruct the activity with the current scatter estimate (TOF-OSEM, 1
 * iteration of 28 subsets per loop iteration), simulate scatter from it with
 * the known attenuation map, smooth, repeat (Methods, "Unknown activity
 * distribution, very limited simulation time"); the attenuation sinogram is
 * a forward projection of the attenuation map (Methods, "Evaluation
 * metrics").  The projector is not specified in the paper; this one:
 *  - image: n_plane slices [plane][y][x] of float on the transaxial grid of
 *    a loaded phantom (`grid`: its nx, ny, voxel and lo in x and y), slice p
 *    at sinogram plane p;
 *  - LOR of bin (view, rad): the line joining the centres (azimuth
 *    2 pi (c + 1/2) / n_crystals on the detection cylinder) of the crystal
 *    pair the simulator bins there; plane p at the mean z of its two rings;
 *  - Joseph sampling: one sample per pixel column (row) along the LOR's
 *    major axis, linear interpolation between the two nearest pixels along
 *    the minor axis, weight = pixel size / |major direction component|;
 *  - TOF: a sample at signed distance s from the LOR midpoint towards the
 *    simulator's TOF-positive crystal adds to TOF bin j with weight
 *    Phi((hi_j - s) / sigma) - Phi((lo_j - s) / sigma) (sigma the context's
 *    tof_sigma_mm), for bins within 5 sigma of s; with sigma = 0 the bin
 *    holding s gets weight 1.
 * Views are taken in subsets: view v belongs to subset v mod n_subsets.
 * Binary32 arithmetic.  All pointers device, caller-owned; asynchronous on
 * stream.  Errors: SSE_EINVAL (null pointers, unknown grid phantom, subset
 * out of range, tof not 0 / 1, more than 48 TOF bins for the TOF
 * projector), SSE_ENOMEM. */

/* Forward projection of the subset's views: sino is [tof][plane][view][rad]
 * (tof = 1) or [plane][view][rad] (tof = 0, the plain line integral); the
 * bins of other views are not written. */
sse_status sse_project(sse_ctx* ctx, sse_phantom_id grid, const float* image, float* sino, int tof, int subset,
                       int n_subsets, void* stream);

/* Back projection (the transpose of sse_project up to the order of binary32
 * sums) of the subset's views of sino into image (overwritten). */
sse_status sse_backproject(sse_ctx* ctx, sse_phantom_id grid, const float* sino, float* image, int tof,
                           int subset, int n_subsets, void* stream);

/* n_iter iterations of TOF-OSEM (Hudson and Larkin 1994) with n_subsets
 * subsets, in place on image: for each subset s in order,
 *   image_j <- image_j (P_s^T (m y / (m P_s image + a)))_j / (P_s^T m)_j
 * with prompts y and additive sinogram a (scatter) of the TOF shape, and the
 * multiplicative sinogram m (attenuation factors times detector
 * sensitivity) without TOF axis, shared by the TOF bins.  Ratios with a
 * non-positive denominator count 0, and denominators below 1e-20 count as
 * 1e-20; pixels with zero sensitivity in a subset keep their value.  The library holds projection scratch for one subset. */
sse_status sse_osem(sse_ctx* ctx, sse_phantom_id grid, const float* prompts, const float* mult, const float* additive,
                    const float* sens, float* image, int n_iter, int n_subsets, void* stream);

/* The subset sensitivity images P_s^T m of sse_osem (m broadcast over TOF),
 * for n_subsets subsets: sens holds n_subsets images back to back (device,
 * n_subsets * n_plane * ny * nx floats, caller-owned).  Passing them to
 * sse_osem (sens != NULL) saves one back projection per subset when m stays
 * the same over many calls, as in the estimation loop; with sens == NULL
 * sse_osem computes each subset's image itself. */
sse_status sse_osem_sensitivity(sse_ctx* ctx, sse_phantom_id grid, const float* mult, int n_subsets, float* sens,
                                void* stream);

/* Attenuation factors of the multiplicative sinogram: out[plane][view][rad]
 * = exp(-line integral of mu511) along each LOR, by the projector above
 * (without TOF) over phantom id's own attenuation map; plane p reads the
 * voxel slice that holds its z (the paper derives its attenuation sinogram
 * from a forward projection of the attenuation map, Methods, "Evaluation
 * metrics").  out: device, n_plane n_view n_rad floats.  Synchronous.
 * Errors: SSE_EINVAL, SSE_ENOMEM. */
sse_status sse_attenuation_factors(sse_ctx* ctx, sse_phantom_id id, float* out, void* stream);

/* Replace phantom id's activity by a reconstructed image (device, on the
 * phantom's own transaxial grid, n_plane slices): voxel slice iz takes the
 * image slice of the plane nearest its centre; negative or non-finite values
 * count 0.  Then as sse_update_activity (synchronous).  Errors: SSE_EINVAL
 * (also for an all-zero image), SSE_EBUSY while a server runs. */
sse_status sse_image_to_activity(sse_ctx* ctx, sse_phantom_id id, const float* image, void* stream);

/* Host helper: the integer alias table the library samples emission voxels
 * with.  Activity is quantised to integer masses q_i summing to n 2^32
 * (q_i = floor(a_i n 2^32 / sum a), remainder to the first largest voxel);
 * Vose's pairing with LIFO small/large stacks filled in index order.  A
 * column i keeps i for a 32-bit draw below thresh[i], else takes alias[i].
 * Host pointers, n entries each.  Errors: SSE_EINVAL. */
sse_status sse_build_alias_table(const float* activity, uint64_t n, uint32_t* thresh, uint32_t* alias);

/* ------------------------------------------------------------------------ */
/* Request server (continuous batching of scatter-estimate requests)         */
/* ------------------------------------------------------------------------ */
/* The iterative scatter estimation of the paper re-simulates scatter for a
 * new activity image at every iteration (Methods, "Unknown activity
 * distribution, very limited simulation time"); a serving system runs many
 * such requests (different phantoms and history budgets) on one GPU.  The
 * server admits requests first-in first-out while their output footprint
 * fits an HBM budget and a slot is free, and every scheduling tick launches
 * one kernel over a work list of history sub-chunks drawn from the active
 * requests (the request submitted first takes a quarter of the tick, the
 * rest goes by shortest remaining work first), so requests that arrive while
 * others run join the next tick and their work overlaps on the device.  Every random
 * number is keyed by the history index, so a request's sinograms are the
 * same alone or in any mix (counts exactly; weights up to the order of
 * binary64 sums).  Phantoms, LUT and sensitivity stay resident in the
 * context. */
typedef struct sse_server sse_server;

typedef struct {
  int32_t max_active;          /* requests simulated concurrently, 1..256 */
  int32_t reserved;
  uint64_t hbm_budget_bytes;   /* cap on library-allocated output buffers, with the device memory of phantoms
                                  loaded after the start; 0 = 90 % of the device memory free at the start */
  uint64_t tick_histories;     /* histories per tick over all active requests; 0 = 32 Mi */
  uint64_t chunk_histories;    /* histories per work-list sub-chunk (<= 2^31; the kernel balances its launches by
                                  claiming 256 histories at a time); 0 = a sixteenth of a tick, at least 256 */
} sse_server_cfg;

typedef struct {
  sse_phantom_id phantom;      /* loaded in the server's context */
  uint32_t reserved;
  uint64_t n_histories;        /* >= 1 */
  uint64_t seed;
  uint64_t h_offset;           /* histories h_offset .. h_offset + n - 1 */
  uint32_t* scatter_counts;    /* caller-owned device sinograms (zeroed by the server), or both */
  double* scatter_weights;     /* NULL: the server allocates them within the budget */
} sse_request;

/* Completion status.  SSE_REQ_FAILED: the server could not allocate the
 * request's output sinograms (the device had less free memory than the
 * budget allowed for) and no buffer it holds could come back; nothing was
 * simulated. */
enum { SSE_REQ_DONE = 0, SSE_REQ_CANCELLED = 1, SSE_REQ_FAILED = 2 };

typedef struct {
  uint64_t id;
  int32_t status;              /* SSE_REQ_DONE or SSE_REQ_CANCELLED */
  int32_t reserved;
  double t_submit, t_admit, t_complete;  /* seconds since sse_server_start (host steady clock) */
  uint64_t histories;          /* histories simulated */
  uint32_t* scatter_counts;    /* the result sinograms (device) */
  double* scatter_weights;
} sse_completion;

typedef struct {
  uint64_t submitted, completed, cancelled, ticks, histories;
  uint64_t max_active_seen;    /* largest number of requests active in one tick */
  uint64_t bytes_allocated;    /* library-allocated output buffers (in use or pooled) */
  uint64_t budget_bytes;
  uint64_t failed;             /* requests completed as SSE_REQ_FAILED */
} sse_server_stats;

/* Start a server on a context (the context must outlive it and have a LUT
 * loaded).  Spawns one host scheduler thread and one HIP stream. Errors:
 * SSE_EINVAL, SSE_ESTATE (no LUT), SSE_ENOMEM, SSE_EDEVICE. */
sse_status sse_server_start(sse_ctx* ctx, const sse_server_cfg* cfg, sse_server** out);

/* Queue a request; *id receives its id.  Thread-safe.  Errors: SSE_EINVAL
 * (unknown phantom, zero histories, one output pointer NULL, misaligned),
 * SSE_EBUSY (a request can never fit the budget), SSE_ESTATE (stopping). */
sse_status sse_server_submit(sse_server* s, const sse_request* req, uint64_t* id);

/* Move up to max completed requests into out (oldest first); *n receives
 * the count.  Waits up to wait_ms milliseconds for the first one (0: no
 * wait).  Thread-safe. */
sse_status sse_server_poll(sse_server* s, sse_completion* out, int32_t max, int32_t* n, int32_t wait_ms);

/* Stop simulating a queued or active request; it completes with status
 * SSE_REQ_CANCELLED once its work in flight has finished.  Errors:
 * SSE_EINVAL (unknown or already completed id). */
sse_status sse_server_cancel(sse_server* s, uint64_t id);

/* Return a completed request's server-allocated sinograms to the pool (the
 * pointers in its completion become invalid).  No-op for caller-owned
 * buffers.  Errors: SSE_EINVAL (unknown id or not completed). */
sse_status sse_server_release(sse_server* s, uint64_t id);

/* Counters of the server (a consistent snapshot). */
sse_status sse_server_stats_get(sse_server* s, sse_server_stats* out);

/* Drain and stop: waits until every submitted request has completed, joins
 * the scheduler thread and frees everything the server allocated
 * (including outputs not yet released). */
sse_status sse_server_stop(sse_server* s);

#ifdef __cplusplus
}
#endif
#endif
