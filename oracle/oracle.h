/* CPU oracle of the LUT-weighted Monte Carlo scatter estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path includes, links or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the HIP library.
 *
 * The oracle follows the paper's pipeline (Methods, "Scatter simulation",
 * Fig. 3): pairs are emitted from the activity map, transported through the
 * attenuation map until they cross a plain cylinder (the simulator keeps every
 * photon that crosses it), each detected single receives a probability from the
 * 5D detection-probability LUT ("Photon detection probability LUT"), each
 * coincidence adds p1 * p2 to its TOF sinogram bin ("Scatter simulator
 * description"), and the sinogram is later multiplied by the scatter
 * sensitivity sinogram ("Scatter sensitivity sinogram").
 */
#ifndef SSE_ORACLE_H
#define SSE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_crystals;          /* crystals per ring (even) */
  int32_t n_rings;
  float radius_mm;             /* detection cylinder radius */
  float length_mm;             /* axial length; rings tile [-L/2, L/2) */
  int32_t crystals_per_module; /* transaxial crystals per module */
  int32_t rings_per_block;     /* axial crystals per block */
  int32_t max_ring_diff;       /* < 0: all ring differences */
} orc_scanner;

typedef struct {
  int32_t n_rad, n_view, n_plane, n_tof;
  float tof_bin_mm;            /* width of a TOF bin in offset along the LOR */
  float tof_sigma_mm;          /* Gaussian TOF jitter on the offset; 0 = none */
} orc_sino;

typedef struct {
  float e_lo_kev, e_hi_kev;    /* energy window (inclusive) */
  float e_kill_kev;            /* photons below this energy are dropped */
  float e_fwhm_frac;           /* energy blur FWHM at 511 keV as a fraction; 0 = none */
  float f_compton, f_rayleigh, f_photo; /* split of mu at 511 keV, sum 1 */
  float rayleigh_beta;         /* analytic form-factor parameter (> 0) */
  float mu_majorant;           /* Woodcock majorant at 511 keV; 0 = phantom max */
  int32_t max_interactions;
} orc_physics;

typedef struct {
  int32_t nx, ny, nz;          /* voxel grid, x fastest: index (z*ny + y)*nx + x */
  float voxel_mm[3];
  float lo_mm[3];              /* minimum corner of the voxel box */
} orc_phantom;

typedef struct {
  int32_t dims[5];             /* n_e, n_theta_t, n_theta_a, n_ct, n_ca */
  float e_min_kev, e_max_kev;
} orc_lut;

/* Gaps between transaxial modules and axial blocks (Methods, "Scatter
 * simulator description": transaxial gaps are given by the angle they
 * subtend, axial gaps by their width) and what happens to a photon that hits
 * one: discarded with its coincidence (LUTs without crystal information, no
 * LUT), assigned to the nearest edge crystal (3D LUT with crystal
 * information), or assigned at random to one of the two edge crystals by the
 * edge-crystal LUT (5D LUT; "Edge crystal assignment LUT").
 *
 * Geometry.  Module m (n_crystals / crystals_per_module of them) covers
 * azimuth [m D, (m+1) D), D = 2 pi / n_modules; half a gap at each end, its
 * crystals_per_module crystals share the rest equally.  Block b (n_rings /
 * rings_per_block of them) covers rings_per_block rings of pitch
 * (L - (n_blocks - 1) w) / n_rings, blocks separated by gaps of width w, no
 * gap at the two ends of the scanner.  The LUT's crystal axes then carry the
 * virtual indices of the gap halves: ct in [0, crystals_per_module + 2)
 * (0: the gap before the module, crystals_per_module + 1: the gap after it)
 * and ca in [0, n_blocks (rings_per_block + 2)), block b's rings at
 * b (rings_per_block + 2) + 1 + k with the gap halves on either side (Methods,
 * "Photon detection probability LUT": 18 and 55 indices on the Signa).  A LUT
 * axis of size 1 ignores the coordinate. */
typedef struct {
  int32_t enabled;             /* 0: plain cylinder (the fields below are ignored) */
  float transaxial_gap_rad;    /* angle of each gap between modules, 0 <= g < 2 pi / n_modules */
  float axial_gap_mm;          /* width of each gap between blocks, >= 0 */
  int32_t policy;              /* ORC_GAP_* */
  int32_t edge_n_angle;        /* edge LUT incidence-angle bins over [-90, 90] degrees */
  int32_t edge_n_pos;          /* edge LUT position bins across the gap */
} orc_gaps;

enum { ORC_GAP_DISCARD = 0, ORC_GAP_NEAREST = 1, ORC_GAP_EDGE_LUT = 2 };

/* Geometry of one kind of gap for the edge-crystal LUT: two blocks of depth
 * depth_mm either side of a gap of width gap_mm, the detection surface
 * doi_mm below their front faces, crystal attenuation mu_per_mm. */
typedef struct {
  float gap_mm, depth_mm, doi_mm, mu_per_mm;
  int32_t n_angle, n_pos;
} orc_edge_geom;

/* Per-photon part of a history record (12 words). */
typedef struct {
  float hx, hy, hz;            /* hit point on the cylinder (0 if not detected) */
  float dx, dy, dz;            /* direction at the hit */
  float e_kev;                 /* photon energy at the cylinder */
  float e_det_kev;             /* after optional energy blur */
  float path_mm;               /* path length from emission to hit */
  uint32_t crystal_ring;       /* crystal | ring << 16 (0xffffffff if none); in a gap, the
                                  nearest edge crystal / ring (before any edge-LUT draw) */
  uint32_t lut_index;          /* flat LUT index (0xffffffff if none) */
  uint32_t inter;              /* n_compton | n_rayleigh << 8 | fate << 16 */
} orc_photon_rec;

/* One record per history (32 words). */
typedef struct {
  uint32_t outcome;            /* ORC_OUT_* */
  uint32_t bin_lo, bin_hi;     /* flat sinogram bin (0xffffffff,0xffffffff if none) */
  uint32_t voxel;              /* emission voxel */
  float weight;                /* p_A * p_B (0 if not binned) */
  float tau_mm;                /* TOF offset including jitter (0 if not computed) */
  uint32_t n_steps;            /* Woodcock tentative steps, both photons */
  uint32_t reserved;
  orc_photon_rec ph[2];        /* photon A (+d), photon B (-d) */
} orc_record;

/* photon fates */
enum { ORC_FATE_DETECTED = 0, ORC_FATE_ABSORBED = 1, ORC_FATE_KILLED = 2,
       ORC_FATE_CAPPED = 3, ORC_FATE_AXIAL = 4 };

/* coincidence outcomes */
enum { ORC_OUT_SCATTER = 0, ORC_OUT_TRUE = 1, ORC_OUT_UNDETECTED = 2,
       ORC_OUT_WINDOW = 3, ORC_OUT_SAME_CRYSTAL = 4, ORC_OUT_RING_DIFF = 5,
       ORC_OUT_RADIAL = 6, ORC_OUT_TOF = 7, ORC_OUT_GAP = 8 };

/* statistics counters */
enum { ORC_ST_HISTORIES = 0, ORC_ST_STEPS, ORC_ST_REAL, ORC_ST_COMPTON,
       ORC_ST_RAYLEIGH, ORC_ST_ABSORBED, ORC_ST_KILLED, ORC_ST_CAPPED,
       ORC_ST_ESCAPED, ORC_ST_DETECTED, ORC_ST_IN_WINDOW, ORC_ST_SCATTER,
       ORC_ST_TRUE, ORC_ST_REJ_WINDOW, ORC_ST_REJ_SAME, ORC_ST_REJ_RING,
       ORC_ST_REJ_RADIAL, ORC_ST_REJ_TOF, ORC_ST_RNG_BLOCKS, ORC_ST_REJ_GAP,
       ORC_ST_GAP_ASSIGNED, ORC_ST_COUNT };

/* Integer Vose alias table over the voxels (see the C file). Returns 0 on
 * success, -1 on invalid activity (negative, non-finite, or all zero). */
int orc_build_alias(const float* activity, uint64_t n, uint32_t* thresh, uint32_t* alias);

/* Run histories h0 .. h0+n-1 (or, if h_list is not NULL, the n histories it
 * lists).  gaps may be NULL (plain cylinder); with the edge-LUT policy,
 * edge_t and edge_a hold the transaxial and axial edge LUTs
 * ([angle][position], probability of the lower-side block).  Sinogram outputs (any may be NULL) are accumulated into; record
 * output (may be NULL) gets one record per processed history; stats (may be
 * NULL) gets ORC_ST_COUNT counters accumulated into. Returns 0 or -1 on bad
 * arguments. */
int orc_simulate(const orc_scanner* sc, const orc_sino* sn, const orc_physics* ph,
                 const orc_phantom* pd, const float* mu511,
                 const uint32_t* alias_thresh, const uint32_t* alias_idx,
                 const orc_lut* ld, const float* lut,
                 const orc_gaps* gaps, const float* edge_t, const float* edge_a,
                 uint64_t seed, uint64_t h0, uint64_t n, const uint64_t* h_list,
                 uint32_t* scatter_counts, double* scatter_weights,
                 uint32_t* true_counts, double* true_weights,
                 uint64_t* stats, orc_record* records);

/* Test hooks on the building blocks. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float orc_u01(uint32_t x);
/* -ln(u) for n uniforms as the transport's free-path sampling evaluates it
 * (binary32 build: the faithful binary32 logarithm; binary64: the library's). */
void orc_neg_log(const float* u, float* out, uint64_t n);
void orc_log_table(float* out); /* 129 x 3 floats */
/* (sin 2 pi u, cos 2 pi u) as the transport's azimuth sampling evaluates it. */
void orc_sincos_2pi(const float* u, float* sn, float* cs, uint64_t n);
/* The transport's coefficients g, fC, fC + fR at energy e_kev in the build's
 * precision (binary32 build: the binary32 energy model). */
void orc_transport_coefs(const orc_physics* ph, float e_kev, float out[3]);
/* Emission of history h: voxel, position and direction of photon A. */
void orc_emit(const orc_phantom* pd, const uint32_t* alias_thresh, const uint32_t* alias_idx,
              uint64_t seed, uint64_t h, uint32_t* voxel, double pos[3], double dir[3]);
/* n Compton samples at energy e_kev from stream (seed, h=index, s=1): writes
 * cos(theta) and the scattered energy. */
void orc_sample_compton(uint64_t seed, double e_kev, uint64_t n, double* cos_theta, double* e_out);
/* n Rayleigh samples of cos(theta) at energy e_kev. */
void orc_sample_rayleigh(uint64_t seed, double e_kev, float beta, uint64_t n, double* cos_theta);
/* The transport's change of direction: u turned by polar cosine ct and
 * azimuth (cos phi, sin phi) = (cp, sp), in the build's precision. */
void orc_rotate(const double u[3], double ct, double cp, double sp, double out[3]);
/* n photons, photon i from p0[3i..] along the unit dir[3i..] with energy
 * e_kev, each on its own stream (seed, h = i, substream 1), transported to
 * the cylinder as the simulation transports annihilation photons (out:
 * hit, direction, energy, path, interactions and fate; no crystal or LUT
 * index).  Returns -1 on bad arguments. */
int orc_transport_photons(const orc_scanner* sc, const orc_physics* ph, const orc_phantom* pd,
                          const float* mu, uint64_t seed, uint64_t n, const double* p0, const double* dir,
                          double e_kev, orc_photon_rec* out);
/* Attenuation model: g(E) = mu(E)/mu(511) and the Compton / Rayleigh parts. */
void orc_energy_model(const orc_physics* ph, double e_kev, double out[3]);
/* Sinogram coordinates of an LOR between crystals c1 (photon A) and c2
 * (photon B): view, signed radial index rho, and 1 if A is the TOF-positive end. */
void orc_lor(int32_t n_crystals, int32_t c1, int32_t c2, int32_t* view, int32_t* rho, int32_t* a_is_pos);

/* Edge-crystal LUT: probability that a gap photon is assigned to the block
 * on the lower side (Eq. (1)-(3), in the reading p1 = 1 - exp(-mu l1),
 * p2 = exp(-mu l1) (1 - exp(-mu l2)) for a photon meeting block 1 first),
 * at the centres of n_angle x n_pos bins, [angle][position]. */
void orc_edge_lut(const orc_edge_geom* g, float* out);
/* Path lengths of a ray in the two blocks: it crosses the detection surface
 * at x0 from the gap centre (positive towards block 2) at angle theta to the
 * depth axis (positive when it moves towards block 2). */
void orc_edge_paths(const orc_edge_geom* g, double theta, double x0, double* l1, double* l2);
/* p_rel of block 1 for one ray (the value orc_edge_lut tabulates). */
double orc_edge_prob(const orc_edge_geom* g, double theta, double x0);
/* Where a hit at (hx, hy, hz) falls: out = {crystal, ring, ct, ca,
 * transaxial gap (0/1), axial gap (0/1), lower-side crystal, upper-side
 * crystal, lower-side ring, upper-side ring}; frac = position across the
 * transaxial and axial gap (0 at the lower side's edge).  Returns -1 on bad
 * arguments. */
int orc_locate(const orc_scanner* sc, const orc_gaps* gaps, float hx, float hy, float hz,
               int32_t out[10], double frac[2]);

/* Reconstruction of the joint estimation loop (recon.c; binary64 whatever
 * the build): TOF Joseph projector on the simulator's sinogram geometry and
 * TOF-OSEM.  The image has n_plane slices [plane][y][x] on the transaxial
 * grid of pd (nx, ny, voxel_mm[0..1], lo_mm[0..1]; pd's nz is not used).
 * Sinograms [tof][plane][view][rad], or [plane][view][rad] without TOF.
 * project: bins of the subset's views (view mod n_subsets == subset; all
 * with n_subsets <= 1) are overwritten, others left; backproject: img is
 * overwritten with the transpose over the subset's views.  osem: n_iter
 * iterations of n_subsets subsets in place (mult without TOF axis, prompts
 * and add with it).  Each returns 0, or -1 on bad arguments.
 * lor_table: the crystal pair of each (view, rad), TOF-positive end in a. */
void orc_recon_lor_table(int32_t n_crystals, int32_t n_rad, int32_t* a, int32_t* b);
int orc_recon_project(const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd, const double* img,
                      double* sino, int tof, int subset, int n_subsets);
int orc_recon_backproject(const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd, const double* sino,
                          double* img, int tof, int subset, int n_subsets);
int orc_recon_osem(const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd, const double* prompts,
                   const double* mult, const double* add, double* img, int n_iter, int n_subsets);

/* Compiled-in transport precision: 4 (binary32) or 8 (binary64). */
int orc_real_size(void);

#ifdef __cplusplus
}
#endif
#endif
