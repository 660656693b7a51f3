/* CPU oracle of the LUT-weighted Monte Carlo PET scatter estimator.
 *
 * TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the HIP library.  It is plain, sequential and slow on purpose.
 *
 * What it computes (the paper's scatter-simulation pipeline, Methods,
 * "Scatter simulation", Fig. 3):
 *   1. emit an annihilation pair from the activity map (emission voxel is part
 *      of the simulator's list-mode record, "Scatter simulator description");
 *   2. transport both photons through the attenuation map (Woodcock tracking;
 *      Compton, Rayleigh, photoabsorption) until they cross the detection
 *      cylinder: the simulator detects every photon crossing a plain cylinder
 *      and models no detector physics ("Scatter simulator description");
 *   3. assign each detected single a transaxial crystal and a ring from its hit
 *      position ("Scatter simulator description", Fig. 4);
 *   4. look up its detection probability in the 5D LUT indexed by energy,
 *      transaxial and axial incidence angle, and in-module / in-block crystal
 *      ("Photon detection probability LUT", Fig. 5);
 *   5. a coincidence adds p1 * p2 (instead of one count) to its TOF sinogram
 *      bin; the TOF bin comes from the difference of the photons' times
 *      ("Scatter simulator description");
 *   6. a coincidence is scattered if at least one photon scattered in the
 *      object (Introduction, footnote on trues and scatters).
 * Every event is either weighted or dropped, never duplicated ("Edge crystal
 * assignment LUT", closing paragraph).
 *
 * The paper leaves the photon physics, the random number generator and the
 * sinogram conventions to its simulator; the readings used here are stated
 * at the steps below that follow them.
 *
 * Parity unpinned: the Rayleigh angular model (Thomson factor times an
 * analytic squared form factor) is a choice made here, not the paper's;
 * its sampler is pinned to its own pdf, but nothing fixes the model itself.
 *
 * Precision.  The file is compiled twice.  With ORACLE_REAL=float every step
 * of the transport that decides an integer (a voxel, an interaction, a
 * crystal, a bin) is taken in binary32, the kernel's precision, with correctly
 * rounded + - * / sqrt and no contraction; logarithms, arc tangents and the
 * cross-section formula are evaluated in binary64 and, where their result
 * feeds binary32 arithmetic, rounded once to binary32.  With
 * ORACLE_REAL=double the same steps run in binary64 (the "FP64 oracle" used to
 * state the error of binary32 transport).  Weights are always accumulated in
 * binary64, in history order.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_REAL
#define ORACLE_REAL float
#endif
typedef ORACLE_REAL real;
#define R(x) ((real)(x))

#define MEC2_KEV 510.99895          /* electron rest energy (CODATA 2018) */
#define PI_D 3.141592653589793
#define TWO_PI_D 6.283185307179586
#define HALF_PI_D 1.5707963267948966
#define MAX_STEPS 100000            /* tentative Woodcock steps per photon */
#define MAX_TRIES 1000              /* rejection-loop guard (never reached) */

int orc_real_size(void) { return (int)sizeof(real); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplications with   */
/* the Weyl key schedule.                                                     */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One random stream: history h, substream s.  Block j has counter
 * (j, h_lo, h_hi, s) and key (seed_lo, seed_hi); the stream's words are the
 * blocks' words in order.  A history draws everything from substream 0 (the
 * samplers' test hooks use substream 1). */
typedef struct {
  uint32_t key[2];
  uint32_t ctr[4];
  uint32_t buf[4];
  int pos;
  uint64_t blocks;
} rng_t;

static void rng_init(rng_t* r, uint64_t seed, uint64_t h, uint32_t s) {
  r->key[0] = (uint32_t)seed;
  r->key[1] = (uint32_t)(seed >> 32);
  r->ctr[0] = 0;
  r->ctr[1] = (uint32_t)h;
  r->ctr[2] = (uint32_t)(h >> 32);
  r->ctr[3] = s;
  r->pos = 4;
  r->blocks = 0;
}

static uint32_t next32(rng_t* r) {
  if (r->pos == 4) {
    orc_philox(r->ctr, r->key, r->buf);
    r->ctr[0] += 1;
    r->pos = 0;
    r->blocks += 1;
  }
  return r->buf[r->pos++];
}

/* Uniform in (0, 1): the top 24 bits with the lowest forced to one, times
 * 2^-24 (exact in binary32, never 0 or 1). */
float orc_u01(uint32_t x) { return (float)((x >> 8) | 1u) * 5.9604644775390625e-08f; }

static real u01(rng_t* r) { return (real)((next32(r) >> 8) | 1u) * R(5.9604644775390625e-08); }

/* -ln(u) for a positive normal binary32 u: the logarithm of the energy
 * model (Klein-Nishina total cross-section), a faithful binary32 logarithm
 * defined operation by operation, so that any IEEE binary32 arithmetic
 * without contraction gives the same bits:
 *   u = f 2^e with f in [sqrt(1/2), sqrt(2))         (frexp, exact)
 *   s = f - 1                                        (exact)
 *   r = s / (2 + s),  z = r^2,  ln f = 2 atanh(r)
 *   2 atanh(r) = 2 r + r R,  R = 2z/3 + 2z^2/5 + 2z^3/7 + 2z^4/9 (Taylor; the
 *     next term is below 2e-9 relative for |r| <= 0.172)
 *   ln f = s - (s^2/2 - r (s^2/2 + R))                (the same value,
 *     arranged so that the exact s is not rounded -- the split used by the
 *     fdlibm logarithm; it rests on 2 r = s - r s)
 *   -ln u = n ln2 - ln f,  n = -e,  ln 2 = hi + lo with n * hi exact. */
static float neg_log_f32(float u) {
  int e;
  float f = frexpf(u, &e);
  if (f < 0.70710678f) {
    f = f + f;
    e -= 1;
  }
  const float s = f - 1.0f;
  const float r = s / (2.0f + s);
  const float z = r * r;
  const float R = z * (2.0f / 3.0f + z * (2.0f / 5.0f + z * (2.0f / 7.0f + z * (2.0f / 9.0f))));
  const float hfsq = 0.5f * s * s;
  const float lnf = s - (hfsq - r * (hfsq + R));
  const float n = (float)(-e);
  return n * 0.693145751953125f + (n * 1.4286068e-06f - lnf);
}

/* -ln(u) of a transport uniform u in (0, 1), the free-path sample of the
 * Woodcock step (Methods, "Scatter simulator description").
 *
 * Binary64 build: the library logarithm.  Binary32 build: a faithful
 * logarithm (error below 0.85 units in the last place for every uniform the
 * generator can produce; 99.7 % correctly rounded), defined operation by
 * operation with fused multiply-adds (fmaf, correctly rounded), after the
 * table method of Tang (1990):
 *   u = F 2^k with F in [sqrt(1/2), sqrt(2))             (frexp, exact)
 *   i = (bits(F) - 0x3F348000) >> 16, 0 <= i <= 128: the table entry whose
 *     F range (2^16 consecutive binary32 values) holds F; entry 75 is the
 *     range around F = 1
 *   c_i = RN(1 / mid_i), mid_i the midpoint of the range, and c_i = 1 for
 *     entries 73..77 (|F - 1| < 0.02), so that no table term cancels a
 *     small result
 *   T_i = -ln(c_i) = hi_i + lo_i, hi_i = T_i rounded to a multiple of
 *     2^-16, lo_i = RN(T_i - hi_i)
 *   r = RN(F c_i - 1)                                    (one fused rounding)
 *   ln(1 + r) = r + r^2 (-1/2 + r (1/3 + r (-1/4 + r/5))) (|r| < 0.02 or
 *     below 2^-8: the next term is below 2^-27 relative)
 *   ln u = (k ln2_hi + hi_i) + ((ln(1 + r) + lo_i) + k ln2_lo), ln 2 split
 *     so that the first sum is exact (multiples of 2^-16 below 2^5). */
enum { kLogEntries = 129 };
static const uint32_t kLogBase = 0x3F348000u;  /* bits of 1.0 - 2^15 - 75 * 2^16 */
static float log_tab[kLogEntries][3];           /* c_i, hi_i, lo_i */
static pthread_once_t log_tab_once = PTHREAD_ONCE_INIT;

static float float_of_bits(uint32_t b) {
  float x;
  memcpy(&x, &b, sizeof x);
  return x;
}

static void build_log_tab(void) {
  for (int i = 0; i < kLogEntries; ++i) {
    const double a = float_of_bits(kLogBase + ((uint32_t)i << 16));
    const double b = float_of_bits(kLogBase + ((uint32_t)(i + 1) << 16));
    const float c = (i >= 73 && i <= 77) ? 1.0f : (float)(1.0 / (0.5 * (a + b)));
    const double t = -log((double)c);
    const double hi = nearbyint(t * 65536.0) / 65536.0;
    log_tab[i][0] = c;
    log_tab[i][1] = (float)hi;
    log_tab[i][2] = (float)(t - hi);
  }
}

static float free_path_log_f32(float u) {
  pthread_once(&log_tab_once, build_log_tab);
  int e;
  float f = frexpf(u, &e);
  if (f < 0.70710678f) {
    f = f + f;
    e -= 1;
  }
  uint32_t fb;
  memcpy(&fb, &f, sizeof fb);
  const float* t = log_tab[(fb - kLogBase) >> 16];
  const float r = fmaf(f, t[0], -1.0f);
  const float q0 = fmaf(r, 0.2f, -0.25f);
  const float q1 = fmaf(r, q0, 0.33333334f);
  const float q2 = fmaf(r, q1, -0.5f);
  const float r2 = r * r;
  const float l1p = fmaf(r2, q2, r);
  const float k = (float)e;
  const float hi = fmaf(k, 0.693145751953125f, t[1]);
  const float lo = fmaf(k, 1.4286068e-06f, l1p + t[2]);
  return -(hi + lo);
}

static real neg_log(real u) {
  return sizeof(real) == sizeof(float) ? (real)free_path_log_f32((float)u) : (real)(-log((double)u));
}

/* The table of the free-path logarithm (kLogEntries rows of c_i, hi_i,
 * lo_i). */
void orc_log_table(float* out) {
  pthread_once(&log_tab_once, build_log_tab);
  memcpy(out, log_tab, sizeof log_tab);
}

/* (sin 2 pi u, cos 2 pi u) for u in [0, 1): the azimuth of a direction.
 *
 * Binary64 build: the library sin and cos.  Binary32 build: fixed
 * operation by operation (error below 1.7 * 2^-24 for every uniform the
 * generator can produce), so every IEEE binary32 implementation agrees:
 *   4u = q + f, q in {0, 1, 2, 3} the quadrant, f in [0, 1)   (exact)
 *   h = f, or 1 - f when f > 1/2 (sine and cosine swap)        (exact)
 *   y = h pi/2 in [0, pi/4], z = y^2, and the Taylor series
 *   sin y = y + y z (-1/3! + z (1/5! + z (-1/7! + z / 9!)))
 *   cos y = 1 + z (-1/2! + z (1/4! + z (-1/6! + z (1/8! - z / 10!))))
 *   (the first omitted terms are below 2e-9), then the quadrant's signs. */
static void sincos_2pi_f32(float u, float* sn, float* cs) {
  const float v = 4.0f * u;
  const int q = (int)floorf(v);
  const float f = v - (float)q;
  const int swap = f > 0.5f;
  const float h = swap ? 1.0f - f : f;
  const float y = h * 1.5707963267948966f;
  const float z = y * y;
  const float s = y + (y * z) * (-1.0f / 6.0f + z * (1.0f / 120.0f + z * (-1.0f / 5040.0f + z * (1.0f / 362880.0f))));
  const float c = 1.0f + z * (-0.5f + z * (1.0f / 24.0f + z * (-1.0f / 720.0f + z * (1.0f / 40320.0f + z * (-1.0f / 3628800.0f)))));
  const float sf = swap ? c : s, cf = swap ? s : c;
  switch (q & 3) {
    case 0: *sn = sf; *cs = cf; break;
    case 1: *sn = cf; *cs = -sf; break;
    case 2: *sn = -sf; *cs = -cf; break;
    default: *sn = -cf; *cs = sf; break;
  }
}

static void sincos_2pi(real u, real* sn, real* cs) {
  if (sizeof(real) == sizeof(float)) {
    float a, b;
    sincos_2pi_f32((float)u, &a, &b);
    *sn = (real)a;
    *cs = (real)b;
  } else {
    const double ph = 6.283185307179586 * (double)u;
    *sn = (real)sin(ph);
    *cs = (real)cos(ph);
  }
}

void orc_sincos_2pi(const float* u, float* sn, float* cs, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    real a, b;
    sincos_2pi((real)u[i], &a, &b);
    sn[i] = (float)a;
    cs[i] = (float)b;
  }
}

void orc_neg_log(const float* u, float* out, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) out[i] = (float)neg_log((real)u[i]);
}

/* Standard normal by Marsaglia's polar method (Marsaglia & Bray 1964). */
static real std_normal(rng_t* r) {
  for (int i = 0; i < MAX_TRIES; ++i) {
    real a = R(2) * u01(r) - R(1);
    real b = R(2) * u01(r) - R(1);
    real s = a * a + b * b;
    if (s < R(1)) return a * (real)sqrt(-2.0 * log((double)s) / (double)s);
  }
  return R(0);
}

/* ------------------------------------------------------------------------ */
/* Integer alias table over voxels (Walker 1977; Vose 1991).                 */
/* Activity a_i becomes integer weights q_i summing to V * 2^32:              */
/*   S = sum a_i (binary64, ascending i), q_i = floor(a_i * (V 2^32 / S)),    */
/*   residual V 2^32 - sum q_i added to the first voxel of largest q.         */
/* Columns hold 2^32 each.  Vose's pairing with two LIFO stacks filled in     */
/* ascending index order: pop l from "small" and g from "large", column l     */
/* keeps q_l and aliases g, q_g -= 2^32 - q_l, g goes back to "small" if now  */
/* below 2^32 else to "large".  Leftover columns are full: threshold          */
/* 0xffffffff, alias = itself.  Sampling column i with a 32-bit draw x keeps i */
/* if x < thresh[i], else takes alias[i].                                    */
/* ------------------------------------------------------------------------ */
int orc_build_alias(const float* activity, uint64_t n, uint32_t* thresh, uint32_t* alias) {
  if (n == 0) return -1;
  double sum = 0.0;
  for (uint64_t i = 0; i < n; ++i) {
    double a = (double)activity[i];
    if (!(a >= 0.0) || isinf(a)) return -1;
    sum += a;
  }
  if (!(sum > 0.0) || isinf(sum)) return -1;
  const uint64_t T = (uint64_t)1 << 32;
  uint64_t* q = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* small = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* large = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!q || !small || !large) { free(q); free(small); free(large); return -1; }
  double scale = (double)n * 4294967296.0 / sum;
  uint64_t total = 0, imax = 0;
  for (uint64_t i = 0; i < n; ++i) {
    q[i] = (uint64_t)floor((double)activity[i] * scale);
    total += q[i];
    if (q[i] > q[imax]) imax = i;
  }
  q[imax] += n * T - total; /* modular: also right if total overshoots */
  uint64_t ns = 0, nl = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (q[i] < T) small[ns++] = i; else large[nl++] = i;
  }
  while (ns > 0 && nl > 0) {
    uint64_t l = small[--ns];
    uint64_t g = large[--nl];
    thresh[l] = (uint32_t)q[l];
    alias[l] = (uint32_t)g;
    q[g] = q[g] - (T - q[l]);
    if (q[g] < T) small[ns++] = g; else large[nl++] = g;
  }
  while (nl > 0) { uint64_t g = large[--nl]; thresh[g] = 0xffffffffu; alias[g] = (uint32_t)g; }
  while (ns > 0) { uint64_t l = small[--ns]; thresh[l] = 0xffffffffu; alias[l] = (uint32_t)l; }
  free(q); free(small); free(large);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry and physics context                                              */
/* ------------------------------------------------------------------------ */
typedef struct { real x, y, z; } vec3;

typedef struct {
  const orc_scanner* sc;
  const orc_sino* sn;
  const orc_physics* ph;
  const orc_phantom* pd;
  const float* mu;
  const uint32_t* thresh;
  const uint32_t* alias;
  const orc_lut* ld;
  const float* lut;
  uint64_t nvox;
  vec3 lo, hi, inv_vox, vox;
  real mu_maj;       /* Woodcock majorant at 511 keV */
  real RR, half_len, pitch, e_scale;
  /* gap model (gp NULL: plain cylinder) */
  const orc_gaps* gp;
  const float* edge_t;
  const float* edge_a;
} ctx_t;

/* Total Klein-Nishina cross section in units of 2 pi r_e^2, a = E / m_e c^2
 * (Klein & Nishina 1929). */
static double kn_total(double a) {
  double L = log(1.0 + 2.0 * a);
  double t1 = (1.0 + a) / (a * a) * (2.0 * (1.0 + a) / (1.0 + 2.0 * a) - L / a);
  double t2 = L / (2.0 * a);
  double t3 = (1.0 + 3.0 * a) / ((1.0 + 2.0 * a) * (1.0 + 2.0 * a));
  return t1 + t2 - t3;
}

/* Energy-dependent coefficients of the separable attenuation model
 * mu(x, E) = mu511(x) g(E), g(E) = fC KN(E)/KN(511) + fR (511/E)^2 + fP (511/E)^3. */
typedef struct { real E, alpha, g, cC, cCR, inv_maj; } ecoef_t;

static void model_parts(const orc_physics* ph, double a, double* fc, double* fr, double* fp) {
  double k = kn_total(a) / kn_total(1.0);
  *fc = (double)ph->f_compton * k;
  *fr = (double)ph->f_rayleigh * (1.0 / (a * a));
  *fp = (double)ph->f_photo * (1.0 / (a * a * a));
}

/* The Klein-Nishina total above evaluated in binary32 for the binary32
 * transport: ln(1 + 2a) by the faithful binary32 logarithm, the quotients
 * by 1/a and 1/(1 + 2a).  Relative error below 2e-5 for E >= 100 keV (the
 * lowest kill energy accepted; cancellation grows as a -> 0). */
static float kn_total_f32(float a) {
  const float ia = 1.0f / a;
  const float b = 1.0f + 2.0f * a;
  const float i12 = 1.0f / b;
  const float L = -neg_log_f32(b);
  const float t1 = (((1.0f + a) * ia) * ia) * ((2.0f * (1.0f + a)) * i12 - L * ia);
  const float t2 = (0.5f * L) * ia;
  const float t3 = ((1.0f + 3.0f * a) * i12) * i12;
  return (t1 + t2) - t3;
}

/* Transport coefficients at energy E.  Binary64 build: the model above,
 * rounded once.  Binary32 build: the same model in binary32,
 *   fC = (f_C / KN32(1)) KN32(a), fR = f_R / a^2, fP = f_P / a^3 (by 1/a). */
static void set_energy(ecoef_t* c, real E, const ctx_t* C) {
  c->E = E;
  c->alpha = E / R(MEC2_KEV);
  if (sizeof(real) == sizeof(float)) {
    const float a = (float)c->alpha;
    const float kc = C->ph->f_compton / kn_total_f32(1.0f);
    const float ia = 1.0f / a;
    const float fc = kc * kn_total_f32(a);
    const float fr = C->ph->f_rayleigh * ia * ia;
    const float fp = C->ph->f_photo * ia * ia * ia;
    c->g = (real)((fc + fr) + fp);
    c->cC = (real)fc;
    c->cCR = (real)(fc + fr);
  } else {
    double fc, fr, fp;
    model_parts(C->ph, (double)c->alpha, &fc, &fr, &fp);
    c->g = (real)(fc + fr + fp);
    c->cC = (real)fc;
    c->cCR = (real)(fc + fr);
  }
  c->inv_maj = R(1) / (C->mu_maj * c->g);
}

void orc_transport_coefs(const orc_physics* ph, float e_kev, float out[3]) {
  ctx_t C;
  memset(&C, 0, sizeof(C));
  C.ph = ph;
  C.mu_maj = R(1);
  ecoef_t c;
  set_energy(&c, (real)e_kev, &C);
  out[0] = (float)c.g;
  out[1] = (float)c.cC;
  out[2] = (float)c.cCR;
}

void orc_energy_model(const orc_physics* ph, double e_kev, double out[3]) {
  double fc, fr, fp;
  model_parts(ph, e_kev / MEC2_KEV, &fc, &fr, &fp);
  out[0] = fc + fr + fp;
  out[1] = fc;
  out[2] = fr;
}

/* Distance along d from p to the exit of the voxel box (slab method). */
static real box_exit(const ctx_t* C, vec3 p, vec3 d) {
  real t = R(INFINITY);
  real s;
  if (d.x > R(0)) { s = (C->hi.x - p.x) / d.x; if (s < t) t = s; }
  else if (d.x < R(0)) { s = (C->lo.x - p.x) / d.x; if (s < t) t = s; }
  if (d.y > R(0)) { s = (C->hi.y - p.y) / d.y; if (s < t) t = s; }
  else if (d.y < R(0)) { s = (C->lo.y - p.y) / d.y; if (s < t) t = s; }
  if (d.z > R(0)) { s = (C->hi.z - p.z) / d.z; if (s < t) t = s; }
  else if (d.z < R(0)) { s = (C->lo.z - p.z) / d.z; if (s < t) t = s; }
  return t;
}

static int clamp_index(real f, int n) {
  if (!(f >= R(0))) return 0;
  if (f >= (real)n) return n - 1;
  return (int)f;
}

static uint64_t voxel_of(const ctx_t* C, vec3 q) {
  int ix = clamp_index((real)floor((double)((q.x - C->lo.x) * C->inv_vox.x)), C->pd->nx);
  int iy = clamp_index((real)floor((double)((q.y - C->lo.y) * C->inv_vox.y)), C->pd->ny);
  int iz = clamp_index((real)floor((double)((q.z - C->lo.z) * C->inv_vox.z)), C->pd->nz);
  return ((uint64_t)iz * (uint64_t)C->pd->ny + (uint64_t)iy) * (uint64_t)C->pd->nx + (uint64_t)ix;
}

/* ------------------------------------------------------------------------ */
/* Emission: voxel by the alias table, uniform position inside it, isotropic */
/* direction with cos(theta) = 1 - 2 u1 (exact) and azimuth 2 pi u2; photon  */
/* B = -d.  No positron range, no acollinearity, no decay.                   */
/* ------------------------------------------------------------------------ */
static void emit(const ctx_t* C, rng_t* r, uint32_t* voxel, vec3* p, vec3* d) {
  uint64_t lo = next32(r);
  uint64_t hi = next32(r);
  uint64_t x0 = (hi << 32) | lo;
  uint64_t col = (uint64_t)(((unsigned __int128)x0 * (unsigned __int128)C->nvox) >> 64);
  uint32_t x1 = next32(r);
  uint32_t v = (x1 < C->thresh[col]) ? (uint32_t)col : C->alias[col];
  *voxel = v;
  uint32_t nx = (uint32_t)C->pd->nx, ny = (uint32_t)C->pd->ny;
  uint32_t ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
  real ux = u01(r);
  real uy = u01(r);
  real uz = u01(r);
  p->x = C->lo.x + ((real)ix + ux) * C->vox.x;
  p->y = C->lo.y + ((real)iy + uy) * C->vox.y;
  p->z = C->lo.z + ((real)iz + uz) * C->vox.z;
  const real cz = R(1) - R(2) * u01(r);
  const real st = (real)sqrt((double)((R(1) - cz) * (R(1) + cz)));
  real sp, cp;
  sincos_2pi(u01(r), &sp, &cp);
  d->x = st * cp;
  d->y = st * sp;
  d->z = cz;
}

/* Klein-Nishina sampling by Kahn's rejection method (Kahn 1954): samples
 * x = E / E' in [1, 1 + 2 alpha]. */
static int sample_kahn(rng_t* r, real alpha, real* x_out) {
  real twoa = R(2) * alpha;
  real b1 = R(1) + twoa;
  real b2 = R(9) + twoa;
  for (int i = 0; i < MAX_TRIES; ++i) {
    real r1 = u01(r);
    real r2 = u01(r);
    real r3 = u01(r);
    if (r1 * b2 <= b1) {
      real x = R(1) + twoa * r2;
      if (r3 * (x * x) <= R(4) * (x - R(1))) { *x_out = x; return 1; }
    } else {
      real x = b1 / (R(1) + twoa * r2);
      real c = R(1) + (R(1) - x) / alpha;
      if (R(2) * r3 <= c * c + R(1) / x) { *x_out = x; return 1; }
    }
  }
  return 0;
}

/* Rayleigh angle: Thomson factor (1 + cos^2)/2 times the analytic squared
 * form factor (1 + beta' (1 - cos))^-2 with beta' = beta (E/511)^2.  The form
 * factor part is sampled by inversion in t = 1 - cos, the Thomson factor by
 * rejection. */
static int sample_rayleigh(rng_t* r, real alpha, real beta, real* cos_out) {
  real bp = beta * (alpha * alpha);
  real C = (R(2) * bp) / (R(1) + R(2) * bp);
  for (int i = 0; i < MAX_TRIES; ++i) {
    real r1 = u01(r);
    real r2 = u01(r);
    real q = r1 * C;
    real t = q / ((R(1) - q) * bp);
    real c = R(1) - t;
    if (c < R(-1)) c = R(-1);
    if (R(2) * r2 <= R(1) + c * c) { *cos_out = c; return 1; }
  }
  return 0;
}

/* Uniform azimuth phi = 2 pi u as (cos phi, sin phi). */
static void azimuth(rng_t* r, real* cp, real* sp) { sincos_2pi(u01(r), sp, cp); }

/* New direction after scattering by polar cosine ct and azimuth (cp, sp)
 * about the old direction u: d' = ct u + st (cp e1 + sp e2) in the frame
 *   e1 = (ux uz / s, uy uz / s, -s),  e2 = (-uy / s, ux / s, 0),
 *   s = sqrt(ux^2 + uy^2),
 * which is orthogonal to u with |e1| = |u| and |e2| = 1 whatever the rounding
 * of u's norm, so d' . u = ct to rounding.  Only a direction within 1e-10 of
 * the axis (s^2 <= 1e-20) takes the axis itself as u, with (e1, e2) = (x, y)
 * for uz > 0 and (x, -y) for uz < 0 (limits of the frame above, so that
 * (e1, e2, u) stays right-handed); the angle that costs is below 1e-10. */
static void rotate(vec3* d, real ct, real cp, real sp) {
  real st = (real)sqrt((double)((R(1) - ct) * (R(1) + ct)));
  real ux = d->x, uy = d->y, uz = d->z;
  real tt = ux * ux + uy * uy;
  if (!(tt > R(1e-20))) {
    real sg = uz > R(0) ? R(1) : R(-1);
    d->x = st * cp;
    d->y = sg * st * sp;
    d->z = sg * ct;
  } else {
    real s = (real)sqrt((double)tt);
    d->x = ux * ct + st * (ux * uz * cp - uy * sp) / s;
    d->y = uy * ct + st * (uy * uz * cp + ux * sp) / s;
    d->z = uz * ct - s * st * cp;
  }
}

/* ------------------------------------------------------------------------ */
/* Transport of one photon to the detection cylinder                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  int fate;
  real E, Edet, path;
  real hx, hy, hz, dx, dy, dz;
  int nC, nR;
  uint32_t steps;
} photon_t;

/* Photon from p0 along unit d with energy e0 (511 keV for annihilation
 * photons). */
static void transport(const ctx_t* C, rng_t* r, vec3 p0, vec3 d, real e0, photon_t* o, uint64_t* st) {
  ecoef_t ec;
  set_energy(&ec, e0, C);
  real len = R(0);
  real t = R(0);
  real texit = box_exit(C, p0, d);
  int nC = 0, nR = 0, nint = 0;
  uint32_t steps = 0;
  int fate = -1;
  for (;;) {
    if (steps >= MAX_STEPS) { fate = ORC_FATE_CAPPED; break; }
    steps += 1;
    /* Woodcock tentative step with the majorant at the current energy */
    real s = neg_log(u01(r)) * ec.inv_maj;
    t = t + s;
    if (!(t < texit)) break; /* leaves the voxel box: straight to the cylinder */
    vec3 q;
    q.x = p0.x + t * d.x;
    q.y = p0.y + t * d.y;
    q.z = p0.z + t * d.z;
    real mu = (real)C->mu[voxel_of(C, q)];
    if (!(u01(r) * C->mu_maj < mu)) continue; /* null collision */
    st[ORC_ST_REAL] += 1;
    p0 = q;
    len = len + t;
    t = R(0);
    nint += 1;
    if (nint > C->ph->max_interactions) { fate = ORC_FATE_CAPPED; break; }
    real ug = u01(r) * ec.g;
    real ct;
    if (ug < ec.cC) {
      real x;
      if (!sample_kahn(r, ec.alpha, &x)) { fate = ORC_FATE_ABSORBED; break; }
      real E2 = ec.E / x;
      ct = R(1) - (x - R(1)) / ec.alpha;
      if (ct < R(-1)) ct = R(-1);
      if (ct > R(1)) ct = R(1);
      nC += 1;
      st[ORC_ST_COMPTON] += 1;
      if (E2 < (real)C->ph->e_kill_kev) { fate = ORC_FATE_KILLED; break; }
      set_energy(&ec, E2, C);
    } else if (ug < ec.cCR) {
      if (!sample_rayleigh(r, ec.alpha, (real)C->ph->rayleigh_beta, &ct)) { fate = ORC_FATE_ABSORBED; break; }
      nR += 1;
      st[ORC_ST_RAYLEIGH] += 1;
    } else {
      fate = ORC_FATE_ABSORBED;
      break;
    }
    real cp, sp;
    azimuth(r, &cp, &sp);
    rotate(&d, ct, cp, sp);
    texit = box_exit(C, p0, d);
  }
  st[ORC_ST_STEPS] += steps;
  o->steps = steps;
  o->nC = nC;
  o->nR = nR;
  o->E = ec.E;
  o->Edet = ec.E;
  o->path = R(0);
  o->hx = o->hy = o->hz = R(0);
  o->dx = d.x; o->dy = d.y; o->dz = d.z;
  if (fate >= 0) {
    o->fate = fate;
    if (fate == ORC_FATE_ABSORBED) st[ORC_ST_ABSORBED] += 1;
    else if (fate == ORC_FATE_KILLED) st[ORC_ST_KILLED] += 1;
    else st[ORC_ST_CAPPED] += 1;
    return;
  }
  st[ORC_ST_ESCAPED] += 1;
  /* Crossing of the cylinder x^2 + y^2 = R^2 ahead of p0 (the larger root of
   * a t^2 + 2 b t + c = 0, in the form without cancellation). */
  real a = d.x * d.x + d.y * d.y;
  if (!(a > R(0))) { o->fate = ORC_FATE_AXIAL; return; }
  real b = p0.x * d.x + p0.y * d.y;
  real c = p0.x * p0.x + p0.y * p0.y - C->RR;
  real D = b * b - a * c;
  real sq = (real)sqrt((double)D);
  real tc = (b > R(0)) ? (-c) / (b + sq) : (sq - b) / a;
  real hz = p0.z + tc * d.z;
  if (!(hz >= -C->half_len && hz < C->half_len)) { o->fate = ORC_FATE_AXIAL; return; }
  o->fate = ORC_FATE_DETECTED;
  o->hx = p0.x + tc * d.x;
  o->hy = p0.y + tc * d.y;
  o->hz = hz;
  o->path = len + tc;
  st[ORC_ST_DETECTED] += 1;
  if (C->ph->e_fwhm_frac > 0.0f) {
    real n = std_normal(r);
    real sig = ((real)C->ph->e_fwhm_frac / R(2.35482)) * (real)sqrt((double)(R(MEC2_KEV) / ec.E));
    o->Edet = ec.E * (R(1) + sig * n);
  }
}

/* ------------------------------------------------------------------------ */
/* Single -> crystal, ring, LUT entry                                        */
/* ------------------------------------------------------------------------ */
static int bin_angle(double th, int n) {
  double f = floor((th + HALF_PI_D) * (double)n / PI_D);
  if (!(f >= 0.0)) return 0;
  if (f >= (double)n) return n - 1;
  return (int)f;
}

/* ------------------------------------------------------------------------ */
/* Gaps between modules and blocks, edge crystals                           */
/* ------------------------------------------------------------------------ */
/* Where a hit falls with gaps ("Scatter simulator description", Fig. 4): the
 * crystal and ring it is assigned to (the nearest edge crystal / ring when it
 * lies in a gap), the LUT crystal coordinates with their virtual gap indices,
 * and for a gap hit the edge crystals on either side and the position across
 * the gap.  Evaluated in binary64. */
typedef struct {
  int crystal, ring;    /* assigned (nearest edge for a gap hit) */
  int ct, ca;           /* LUT coordinates: crystal in module, crystal along the axis */
  int tgap, agap;       /* 1 if in a transaxial / axial gap */
  int c_lo, c_hi;       /* transaxial gap: edge crystals of the lower / upper module */
  int r_lo, r_hi;       /* axial gap: edge rings of the lower / upper block */
  double tfrac, afrac;  /* position across the gap, 0 at the lower side, 1 at the upper */
} hit_t;

static int clamp_int(double f, int n) {
  if (!(f >= 0.0)) return 0;
  if (f >= (double)n) return n - 1;
  return (int)f;
}

static void locate(const orc_scanner* sc, const orc_gaps* gp, double hx, double hy, double hz, hit_t* h) {
  const int cm = sc->crystals_per_module, rb = sc->rings_per_block;
  const int nm = sc->n_crystals / cm, nb = sc->n_rings / rb;
  memset(h, 0, sizeof(*h));
  /* transaxial: module m spans azimuth [m D, (m + 1) D); half a gap of
   * angle g at either end, crystals of width (D - g) / cm in between */
  const double g = (double)gp->transaxial_gap_rad;
  const double D = TWO_PI_D / (double)nm;
  double phi = atan2(hy, hx);
  if (phi < 0.0) phi += TWO_PI_D;
  const int m = clamp_int(floor(phi / D), nm);
  const double loc = phi - (double)m * D;
  if (g > 0.0 && loc < 0.5 * g) {
    /* upper half of the gap between modules m - 1 and m */
    h->tgap = 1;
    h->ct = 0;
    h->c_lo = ((m + nm - 1) % nm) * cm + cm - 1;
    h->c_hi = m * cm;
    h->crystal = h->c_hi;
    h->tfrac = (loc + 0.5 * g) / g;
  } else if (g > 0.0 && loc >= D - 0.5 * g) {
    /* lower half of the gap between modules m and m + 1 */
    h->tgap = 1;
    h->ct = cm + 1;
    h->c_lo = m * cm + cm - 1;
    h->c_hi = ((m + 1) % nm) * cm;
    h->crystal = h->c_lo;
    h->tfrac = (loc - (D - 0.5 * g)) / g;
  } else {
    const int k = clamp_int(floor((loc - 0.5 * g) * (double)cm / (D - g)), cm);
    h->ct = k + 1;
    h->crystal = m * cm + k;
  }
  /* axial: blocks of rb rings of pitch pa, gaps of width w between them */
  const double L = (double)sc->length_mm, w = (double)gp->axial_gap_mm;
  const double pa = (L - (double)(nb - 1) * w) / (double)sc->n_rings;
  const double span = (double)rb * pa;
  const double period = span + w;
  const double z = hz + 0.5 * L;
  const int b = clamp_int(floor(z / period), nb);
  const double zl = z - (double)b * period;
  if (w > 0.0 && b < nb - 1 && zl >= span) {
    /* gap between blocks b and b + 1 */
    const double go = zl - span;
    h->agap = 1;
    h->r_lo = b * rb + rb - 1;
    h->r_hi = (b + 1) * rb;
    h->afrac = go / w;
    if (go < 0.5 * w) {
      h->ca = b * (rb + 2) + rb + 1;
      h->ring = h->r_lo;
    } else {
      h->ca = (b + 1) * (rb + 2);
      h->ring = h->r_hi;
    }
  } else {
    const int k = clamp_int(floor(zl / pa), rb);
    h->ca = b * (rb + 2) + 1 + k;
    h->ring = b * rb + k;
  }
}

/* Path lengths of a straight ray inside the two blocks either side of a gap
 * ("Edge crystal assignment LUT", Fig. 9).  Coordinates: x across the gap
 * (0 at its centre, block 1 at x <= -w/2, block 2 at x >= w/2), y the depth
 * below the blocks' front faces (blocks span 0 <= y <= depth); the ray
 * crosses the detection surface y = doi at x0 with angle theta to the y axis,
 * moving towards +x for theta > 0.  The blocks are taken as unbounded away
 * from the gap. */
void orc_edge_paths(const orc_edge_geom* g, double theta, double x0, double* l1, double* l2) {
  const double D = (double)g->depth_mm, d = (double)g->doi_mm, hw = 0.5 * (double)g->gap_mm;
  const double t = tan(theta), c = cos(theta);
  *l1 = 0.0;
  *l2 = 0.0;
  if (t == 0.0) {
    /* parallel to the gap walls: inside a block over the whole depth, or in neither */
    if (x0 <= -hw) *l1 = D;
    if (x0 >= hw) *l2 = D;
    return;
  }
  /* depths at which the ray crosses x = -w/2 and x = +w/2 */
  const double y1 = d + (-hw - x0) / t, y2 = d + (hw - x0) / t;
  double a1, b1, a2, b2;
  if (t > 0.0) {        /* x grows with depth: block 1 above y1, block 2 below y2 */
    a1 = 0.0; b1 = fmin(D, y1);
    a2 = fmax(0.0, y2); b2 = D;
  } else {              /* x falls with depth: block 2 above y2, block 1 below y1 */
    a1 = fmax(0.0, y1); b1 = D;
    a2 = 0.0; b2 = fmin(D, y2);
  }
  if (b1 > a1) *l1 = (b1 - a1) / c;
  if (b2 > a2) *l2 = (b2 - a2) / c;
}

/* Eq. (1)-(3) in the reading that makes them probabilities of detection:
 * the block the photon meets first absorbs it with probability
 * 1 - exp(-mu l_first); the second with exp(-mu l_first)(1 - exp(-mu l_second))
 * (the printed Eq. (1) reads as a transmission).  A ray through neither block
 * goes to the nearer one (0.5 at the gap centre). */
double orc_edge_prob(const orc_edge_geom* g, double theta, double x0) {
  double l1, l2;
  orc_edge_paths(g, theta, x0, &l1, &l2);
  const double mu = (double)g->mu_per_mm;
  double p1, p2;
  if (theta >= 0.0) {   /* block 1 first */
    p1 = -expm1(-mu * l1);
    p2 = exp(-mu * l1) * -expm1(-mu * l2);
  } else {              /* block 2 first */
    p2 = -expm1(-mu * l2);
    p1 = exp(-mu * l2) * -expm1(-mu * l1);
  }
  if (p1 + p2 > 0.0) return p1 / (p1 + p2);
  return x0 < 0.0 ? 1.0 : (x0 > 0.0 ? 0.0 : 0.5);
}

void orc_edge_lut(const orc_edge_geom* g, float* out) {
  const double w = (double)g->gap_mm;
  for (int a = 0; a < g->n_angle; ++a) {
    const double th = (-90.0 + ((double)a + 0.5) * 180.0 / (double)g->n_angle) * PI_D / 180.0;
    for (int j = 0; j < g->n_pos; ++j) {
      const double x0 = -0.5 * w + ((double)j + 0.5) * w / (double)g->n_pos;
      out[a * g->n_pos + j] = (float)orc_edge_prob(g, th, x0);
    }
  }
}

static void single_index(const ctx_t* C, const photon_t* o, hit_t* hit, uint32_t* lut_index) {
  const orc_scanner* sc = C->sc;
  int c, rg;
  if (C->gp) {
    locate(sc, C->gp, (double)o->hx, (double)o->hy, (double)o->hz, hit);
    c = hit->crystal;
    rg = hit->ring;
  } else {
    /* crystal c covers azimuth [2 pi c / Nc, 2 pi (c + 1) / Nc) */
    double phi = atan2((double)o->hy, (double)o->hx);
    if (phi < 0.0) phi += TWO_PI_D;
    double fc = floor(phi * (double)sc->n_crystals / TWO_PI_D);
    c = (fc >= (double)sc->n_crystals) ? sc->n_crystals - 1 : (fc < 0.0 ? 0 : (int)fc);
    /* rings tile [-L/2, L/2) */
    rg = clamp_index((real)floor((double)((o->hz + C->half_len) / C->pitch)), sc->n_rings);
    memset(hit, 0, sizeof(*hit));
    hit->crystal = c;
    hit->ring = rg;
  }
  /* LUT axes: energy, transaxial angle, axial angle, crystal in module,
   * crystal in block.  The angles are those between the path and the hit
   * point's position vector, projected in the transaxial and axial planes,
   * over [-90, 90] degrees (Fig. 5 caption). */
  const int* dm = C->ld->dims;
  int iE = clamp_index((real)floor((double)((o->E - (real)C->ld->e_min_kev) * C->e_scale)), dm[0]);
  double hx = (double)o->hx, hy = (double)o->hy;
  double rho = sqrt(hx * hx + hy * hy);
  double dr = (hx * (double)o->dx + hy * (double)o->dy) / rho;
  double tt = (hx * (double)o->dy - hy * (double)o->dx) / rho;
  int it = bin_angle(atan2(tt, dr), dm[1]);
  int ia = bin_angle(atan2((double)o->dz, dr), dm[2]);
  int ct, ca;
  if (C->gp) {
    /* axes of size 1 ignore the coordinate; otherwise the virtual-index layout */
    ct = dm[3] == 1 ? 0 : hit->ct;
    ca = dm[4] == 1 ? 0 : hit->ca;
  } else {
    ct = ((c % sc->crystals_per_module) * dm[3]) / sc->crystals_per_module;
    ca = ((rg % sc->rings_per_block) * dm[4]) / sc->rings_per_block;
  }
  *lut_index = (uint32_t)((((iE * dm[1] + it) * dm[2] + ia) * dm[3] + ct) * dm[4] + ca);
}

/* Edge-crystal assignment of a gap photon of a coincidence ("Edge crystal
 * assignment LUT"): with the edge-LUT policy a uniform draw from the
 * history's stream below the tabulated probability picks the lower side's
 * edge crystal, otherwise the upper side's; a photon in both kinds of gap
 * draws for the transaxial gap first.  With the nearest policy the hit keeps
 * its nearest edge crystal. */
static void resolve_gap(const ctx_t* C, rng_t* r, const photon_t* o, hit_t* h, uint64_t* st) {
  const orc_gaps* gp = C->gp;
  if (!h->tgap && !h->agap) return;
  double hx = (double)o->hx, hy = (double)o->hy;
  double rho = sqrt(hx * hx + hy * hy);
  double dr = (hx * (double)o->dx + hy * (double)o->dy) / rho;
  double tt = (hx * (double)o->dy - hy * (double)o->dx) / rho;
  const int na = gp->edge_n_angle, np = gp->edge_n_pos;
  if (h->tgap) {
    if (gp->policy == ORC_GAP_EDGE_LUT) {
      int ia = bin_angle(atan2(tt, dr), na);
      int ip = clamp_int(floor(h->tfrac * (double)np), np);
      double u = (double)u01(r);
      h->crystal = u < (double)C->edge_t[ia * np + ip] ? h->c_lo : h->c_hi;
    }
    st[ORC_ST_GAP_ASSIGNED] += 1;
  }
  if (h->agap) {
    if (gp->policy == ORC_GAP_EDGE_LUT) {
      int ia = bin_angle(atan2((double)o->dz, dr), na);
      int ip = clamp_int(floor(h->afrac * (double)np), np);
      double u = (double)u01(r);
      h->ring = u < (double)C->edge_a[ia * np + ip] ? h->r_lo : h->r_hi;
    }
    st[ORC_ST_GAP_ASSIGNED] += 1;
  }
}

/* Sinogram coordinates of the LOR between crystals c1 and c2: the view angle
 * is pi k / Nc with k = c1 + c2 + 1 folded into [0, Nc), the signed radial
 * index rho = Nc/2 - |c1 - c2| (sign flips with the fold), two neighbouring k
 * share one view.  The TOF-positive end is the crystal lying on the positive
 * side of the LOR direction (-sin, cos) of the view angle. */
void orc_lor(int32_t n, int32_t c1, int32_t c2, int32_t* view, int32_t* rho, int32_t* a_is_pos) {
  int k = c1 + c2 + 1;
  int dc = c1 > c2 ? c1 - c2 : c2 - c1;
  int rh = n / 2 - dc;
  if (k >= n) { k -= n; rh = -rh; }
  *view = k >> 1;
  *rho = rh;
  int m = ((2 * c1 + 1 - k) % (2 * n) + 2 * n) % (2 * n);
  *a_is_pos = (m > 0 && m < n) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* One history                                                               */
/* ------------------------------------------------------------------------ */
static void fill_photon_rec(orc_photon_rec* pr, const photon_t* o) {
  pr->hx = (float)o->hx; pr->hy = (float)o->hy; pr->hz = (float)o->hz;
  pr->dx = (float)o->dx; pr->dy = (float)o->dy; pr->dz = (float)o->dz;
  pr->e_kev = (float)o->E;
  pr->e_det_kev = (float)o->Edet;
  pr->path_mm = (float)o->path;
  pr->crystal_ring = 0xffffffffu;
  pr->lut_index = 0xffffffffu;
  pr->inter = (uint32_t)o->nC | ((uint32_t)o->nR << 8) | ((uint32_t)o->fate << 16);
}

static void history(const ctx_t* C, uint64_t seed, uint64_t h,
                    uint32_t* sc_n, double* sc_w, uint32_t* tr_n, double* tr_w,
                    uint64_t* st, orc_record* rec) {
  /* one stream per history, consumed in order: emission, photon A,
   * photon B, TOF jitter */
  rng_t r;
  rng_init(&r, seed, h, 0);
  uint32_t voxel;
  vec3 p, d, dm;
  emit(C, &r, &voxel, &p, &d);
  dm.x = -d.x; dm.y = -d.y; dm.z = -d.z;
  photon_t A, B;
  transport(C, &r, p, d, R(MEC2_KEV), &A, st);
  transport(C, &r, p, dm, R(MEC2_KEV), &B, st);
  st[ORC_ST_HISTORIES] += 1;

  uint32_t outcome;
  uint64_t bin = ~(uint64_t)0;
  real w = R(0), tau = R(0);
  int cA = -1, rA = -1, cB = -1, rB = -1;
  uint32_t lA = 0xffffffffu, lB = 0xffffffffu;
  hit_t hA, hB;
  int inwinA = A.fate == ORC_FATE_DETECTED && A.Edet >= (real)C->ph->e_lo_kev && A.Edet <= (real)C->ph->e_hi_kev;
  int inwinB = B.fate == ORC_FATE_DETECTED && B.Edet >= (real)C->ph->e_lo_kev && B.Edet <= (real)C->ph->e_hi_kev;
  if (inwinA) { single_index(C, &A, &hA, &lA); cA = hA.crystal; rA = hA.ring; st[ORC_ST_IN_WINDOW] += 1; }
  if (inwinB) { single_index(C, &B, &hB, &lB); cB = hB.crystal; rB = hB.ring; st[ORC_ST_IN_WINDOW] += 1; }
  /* the record keeps the nearest crystal and ring of each single */
  const uint32_t crA = inwinA ? (uint32_t)cA | ((uint32_t)rA << 16) : 0xffffffffu;
  const uint32_t crB = inwinB ? (uint32_t)cB | ((uint32_t)rB << 16) : 0xffffffffu;
  int scattered = (A.nC + A.nR + B.nC + B.nR) > 0;
  int gap_discard = 0;
  if (C->gp && A.fate == ORC_FATE_DETECTED && B.fate == ORC_FATE_DETECTED && inwinA && inwinB) {
    if (C->gp->policy == ORC_GAP_DISCARD) {
      gap_discard = hA.tgap || hA.agap || hB.tgap || hB.agap;
    } else {
      /* photon A's gaps draw first, then photon B's, before the TOF jitter */
      resolve_gap(C, &r, &A, &hA, st);
      resolve_gap(C, &r, &B, &hB, st);
      cA = hA.crystal; rA = hA.ring;
      cB = hB.crystal; rB = hB.ring;
    }
  }
  if (A.fate != ORC_FATE_DETECTED || B.fate != ORC_FATE_DETECTED) {
    outcome = ORC_OUT_UNDETECTED;
  } else if (!inwinA || !inwinB) {
    outcome = ORC_OUT_WINDOW;
    st[ORC_ST_REJ_WINDOW] += 1;
  } else if (gap_discard) {
    outcome = ORC_OUT_GAP;
    st[ORC_ST_REJ_GAP] += 1;
  } else if (cA == cB) {
    outcome = ORC_OUT_SAME_CRYSTAL;
    st[ORC_ST_REJ_SAME] += 1;
  } else if (C->sc->max_ring_diff >= 0 && abs(rA - rB) > C->sc->max_ring_diff) {
    outcome = ORC_OUT_RING_DIFF;
    st[ORC_ST_REJ_RING] += 1;
  } else {
    int view, rho, apos;
    orc_lor(C->sc->n_crystals, cA, cB, &view, &rho, &apos);
    int half = (C->sn->n_rad - 1) / 2;
    if (abs(rho) > half) {
      outcome = ORC_OUT_RADIAL;
      st[ORC_ST_REJ_RADIAL] += 1;
    } else {
      /* TOF offset toward the TOF-positive end: half the path difference */
      tau = apos ? (B.path - A.path) * R(0.5) : (A.path - B.path) * R(0.5);
      if (C->sn->tof_sigma_mm > 0.0f) tau = tau + (real)C->sn->tof_sigma_mm * std_normal(&r);
      real xt = tau / (real)C->sn->tof_bin_mm + (real)C->sn->n_tof * R(0.5);
      if (!(xt >= R(0)) || !(xt < (real)C->sn->n_tof)) {
        outcome = ORC_OUT_TOF;
        st[ORC_ST_REJ_TOF] += 1;
      } else {
        uint64_t tof = (uint64_t)floor((double)xt);
        uint64_t plane = (uint64_t)(rA + rB);
        uint64_t rad = (uint64_t)(rho + half);
        bin = ((tof * (uint64_t)C->sn->n_plane + plane) * (uint64_t)C->sn->n_view + (uint64_t)view)
              * (uint64_t)C->sn->n_rad + rad;
        w = (real)C->lut[lA] * (real)C->lut[lB];
        if (scattered) {
          outcome = ORC_OUT_SCATTER;
          st[ORC_ST_SCATTER] += 1;
          if (sc_n) sc_n[bin] += 1u;
          if (sc_w) sc_w[bin] += (double)w;
        } else {
          outcome = ORC_OUT_TRUE;
          st[ORC_ST_TRUE] += 1;
          if (tr_n) tr_n[bin] += 1u;
          if (tr_w) tr_w[bin] += (double)w;
        }
      }
    }
  }
  st[ORC_ST_RNG_BLOCKS] += r.blocks;
  if (rec) {
    rec->outcome = outcome | (scattered ? 0x100u : 0u);
    rec->bin_lo = (uint32_t)bin;
    rec->bin_hi = (uint32_t)(bin >> 32);
    rec->voxel = voxel;
    rec->weight = (float)w;
    rec->tau_mm = (float)tau;
    rec->n_steps = A.steps + B.steps;
    rec->reserved = 0;
    fill_photon_rec(&rec->ph[0], &A);
    fill_photon_rec(&rec->ph[1], &B);
    if (inwinA) { rec->ph[0].crystal_ring = crA; rec->ph[0].lut_index = lA; }
    if (inwinB) { rec->ph[1].crystal_ring = crB; rec->ph[1].lut_index = lB; }
  }
}

static int setup(ctx_t* C, const orc_scanner* sc, const orc_sino* sn, const orc_physics* ph,
                 const orc_phantom* pd, const float* mu, const uint32_t* th, const uint32_t* al,
                 const orc_lut* ld, const float* lut,
                 const orc_gaps* gaps, const float* edge_t, const float* edge_a) {
  if (!sc || !sn || !ph || !pd || !mu || !th || !al || !ld || !lut) return -1;
  C->gp = NULL;
  C->edge_t = edge_t;
  C->edge_a = edge_a;
  if (gaps && gaps->enabled) {
    const int cm = sc->crystals_per_module, rb = sc->rings_per_block;
    if (cm <= 0 || rb <= 0 || sc->n_crystals % cm || sc->n_rings % rb) return -1;
    const int nm = sc->n_crystals / cm, nb = sc->n_rings / rb;
    if (!(gaps->transaxial_gap_rad >= 0.0f) || !((double)gaps->transaxial_gap_rad < TWO_PI_D / (double)nm)) return -1;
    if (!(gaps->axial_gap_mm >= 0.0f) || !((double)(nb - 1) * (double)gaps->axial_gap_mm < (double)sc->length_mm)) return -1;
    if (ld->dims[3] != 1 && ld->dims[3] != cm + 2) return -1;
    if (ld->dims[4] != 1 && ld->dims[4] != nb * (rb + 2)) return -1;
    if (gaps->policy < ORC_GAP_DISCARD || gaps->policy > ORC_GAP_EDGE_LUT) return -1;
    if (gaps->policy == ORC_GAP_EDGE_LUT &&
        (!edge_t || !edge_a || gaps->edge_n_angle < 1 || gaps->edge_n_pos < 1)) return -1;
    C->gp = gaps;
  }
  if (sc->n_crystals <= 0 || sc->n_crystals % 2 || sc->n_rings <= 0) return -1;
  if (sn->n_view != sc->n_crystals / 2 || sn->n_plane != 2 * sc->n_rings - 1) return -1;
  if (sn->n_rad <= 0 || sn->n_rad % 2 == 0 || sn->n_rad > sc->n_crystals - 1 || sn->n_tof <= 0) return -1;
  if (pd->nx <= 0 || pd->ny <= 0 || pd->nz <= 0) return -1;
  if (!(ph->rayleigh_beta > 0.0f)) return -1;
  C->sc = sc; C->sn = sn; C->ph = ph; C->pd = pd; C->mu = mu; C->thresh = th; C->alias = al;
  C->ld = ld; C->lut = lut;
  C->nvox = (uint64_t)pd->nx * (uint64_t)pd->ny * (uint64_t)pd->nz;
  C->vox.x = (real)pd->voxel_mm[0]; C->vox.y = (real)pd->voxel_mm[1]; C->vox.z = (real)pd->voxel_mm[2];
  C->lo.x = (real)pd->lo_mm[0]; C->lo.y = (real)pd->lo_mm[1]; C->lo.z = (real)pd->lo_mm[2];
  C->hi.x = C->lo.x + (real)pd->nx * C->vox.x;
  C->hi.y = C->lo.y + (real)pd->ny * C->vox.y;
  C->hi.z = C->lo.z + (real)pd->nz * C->vox.z;
  C->inv_vox.x = R(1) / C->vox.x; C->inv_vox.y = R(1) / C->vox.y; C->inv_vox.z = R(1) / C->vox.z;
  float mmax = 0.0f;
  for (uint64_t i = 0; i < C->nvox; ++i) {
    if (!(mu[i] >= 0.0f)) return -1;
    if (mu[i] > mmax) mmax = mu[i];
  }
  if (ph->mu_majorant > 0.0f) {
    if (ph->mu_majorant < mmax) return -1;
    mmax = ph->mu_majorant;
  }
  C->mu_maj = (real)mmax;
  C->RR = (real)sc->radius_mm * (real)sc->radius_mm;
  C->half_len = R(0.5) * (real)sc->length_mm;
  C->pitch = (real)sc->length_mm / (real)sc->n_rings;
  C->e_scale = (real)ld->dims[0] / ((real)ld->e_max_kev - (real)ld->e_min_kev);
  return 0;
}

int orc_simulate(const orc_scanner* sc, const orc_sino* sn, const orc_physics* ph,
                 const orc_phantom* pd, const float* mu511,
                 const uint32_t* alias_thresh, const uint32_t* alias_idx,
                 const orc_lut* ld, const float* lut,
                 const orc_gaps* gaps, const float* edge_t, const float* edge_a,
                 uint64_t seed, uint64_t h0, uint64_t n, const uint64_t* h_list,
                 uint32_t* scatter_counts, double* scatter_weights,
                 uint32_t* true_counts, double* true_weights,
                 uint64_t* stats, orc_record* records) {
  ctx_t C;
  if (setup(&C, sc, sn, ph, pd, mu511, alias_thresh, alias_idx, ld, lut, gaps, edge_t, edge_a)) return -1;
  uint64_t local[ORC_ST_COUNT];
  memset(local, 0, sizeof(local));
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t h = h_list ? h_list[i] : h0 + i;
    history(&C, seed, h, scatter_counts, scatter_weights, true_counts, true_weights, local,
            records ? &records[i] : NULL);
  }
  if (stats)
    for (int k = 0; k < ORC_ST_COUNT; ++k) stats[k] += local[k];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Test hooks                                                                */
/* ------------------------------------------------------------------------ */
void orc_emit(const orc_phantom* pd, const uint32_t* th, const uint32_t* al,
              uint64_t seed, uint64_t h, uint32_t* voxel, double pos[3], double dir[3]) {
  ctx_t C;
  memset(&C, 0, sizeof(C));
  C.pd = pd; C.thresh = th; C.alias = al;
  C.nvox = (uint64_t)pd->nx * (uint64_t)pd->ny * (uint64_t)pd->nz;
  C.vox.x = (real)pd->voxel_mm[0]; C.vox.y = (real)pd->voxel_mm[1]; C.vox.z = (real)pd->voxel_mm[2];
  C.lo.x = (real)pd->lo_mm[0]; C.lo.y = (real)pd->lo_mm[1]; C.lo.z = (real)pd->lo_mm[2];
  rng_t r;
  rng_init(&r, seed, h, 0);
  vec3 p, d;
  emit(&C, &r, voxel, &p, &d);
  pos[0] = (double)p.x; pos[1] = (double)p.y; pos[2] = (double)p.z;
  dir[0] = (double)d.x; dir[1] = (double)d.y; dir[2] = (double)d.z;
}

void orc_sample_compton(uint64_t seed, double e_kev, uint64_t n, double* cos_theta, double* e_out) {
  real E = (real)e_kev;
  real alpha = E / R(MEC2_KEV);
  for (uint64_t i = 0; i < n; ++i) {
    rng_t r;
    rng_init(&r, seed, i, 1);
    real x = R(1);
    sample_kahn(&r, alpha, &x);
    real ct = R(1) - (x - R(1)) / alpha;
    if (ct < R(-1)) ct = R(-1);
    if (ct > R(1)) ct = R(1);
    cos_theta[i] = (double)ct;
    e_out[i] = (double)(E / x);
  }
}

void orc_sample_rayleigh(uint64_t seed, double e_kev, float beta, uint64_t n, double* cos_theta) {
  real alpha = (real)e_kev / R(MEC2_KEV);
  for (uint64_t i = 0; i < n; ++i) {
    rng_t r;
    rng_init(&r, seed, i, 1);
    real c = R(1);
    sample_rayleigh(&r, alpha, (real)beta, &c);
    cos_theta[i] = (double)c;
  }
}

void orc_rotate(const double u[3], double ct, double cp, double sp, double out[3]) {
  vec3 d;
  d.x = (real)u[0]; d.y = (real)u[1]; d.z = (real)u[2];
  rotate(&d, (real)ct, (real)cp, (real)sp);
  out[0] = (double)d.x; out[1] = (double)d.y; out[2] = (double)d.z;
}

int orc_transport_photons(const orc_scanner* sc, const orc_physics* ph, const orc_phantom* pd,
                          const float* mu, uint64_t seed, uint64_t n, const double* p0, const double* dir,
                          double e_kev, orc_photon_rec* out) {
  if (!sc || !ph || !pd || !mu || !p0 || !dir || !out) return -1;
  if (pd->nx <= 0 || pd->ny <= 0 || pd->nz <= 0 || !(ph->rayleigh_beta > 0.0f)) return -1;
  ctx_t C;
  memset(&C, 0, sizeof(C));
  C.sc = sc; C.ph = ph; C.pd = pd; C.mu = mu;
  C.nvox = (uint64_t)pd->nx * (uint64_t)pd->ny * (uint64_t)pd->nz;
  C.vox.x = (real)pd->voxel_mm[0]; C.vox.y = (real)pd->voxel_mm[1]; C.vox.z = (real)pd->voxel_mm[2];
  C.lo.x = (real)pd->lo_mm[0]; C.lo.y = (real)pd->lo_mm[1]; C.lo.z = (real)pd->lo_mm[2];
  C.hi.x = C.lo.x + (real)pd->nx * C.vox.x;
  C.hi.y = C.lo.y + (real)pd->ny * C.vox.y;
  C.hi.z = C.lo.z + (real)pd->nz * C.vox.z;
  C.inv_vox.x = R(1) / C.vox.x; C.inv_vox.y = R(1) / C.vox.y; C.inv_vox.z = R(1) / C.vox.z;
  float mmax = 0.0f;
  for (uint64_t i = 0; i < C.nvox; ++i) {
    if (!(mu[i] >= 0.0f)) return -1;
    if (mu[i] > mmax) mmax = mu[i];
  }
  if (ph->mu_majorant > 0.0f) {
    if (ph->mu_majorant < mmax) return -1;
    mmax = ph->mu_majorant;
  }
  C.mu_maj = (real)mmax;
  C.RR = (real)sc->radius_mm * (real)sc->radius_mm;
  C.half_len = R(0.5) * (real)sc->length_mm;
  uint64_t st[ORC_ST_COUNT];
  memset(st, 0, sizeof(st));
  for (uint64_t i = 0; i < n; ++i) {
    rng_t r;
    rng_init(&r, seed, i, 1);
    vec3 p, d;
    p.x = (real)p0[3 * i]; p.y = (real)p0[3 * i + 1]; p.z = (real)p0[3 * i + 2];
    d.x = (real)dir[3 * i]; d.y = (real)dir[3 * i + 1]; d.z = (real)dir[3 * i + 2];
    photon_t o;
    transport(&C, &r, p, d, (real)e_kev, &o, st);
    fill_photon_rec(&out[i], &o);
  }
  return 0;
}

int orc_locate(const orc_scanner* sc, const orc_gaps* gaps, float hx, float hy, float hz,
               int32_t out[10], double frac[2]) {
  if (!sc || !gaps || sc->crystals_per_module <= 0 || sc->rings_per_block <= 0 ||
      sc->n_crystals % sc->crystals_per_module || sc->n_rings % sc->rings_per_block) return -1;
  hit_t h;
  locate(sc, gaps, (double)hx, (double)hy, (double)hz, &h);
  out[0] = h.crystal; out[1] = h.ring; out[2] = h.ct; out[3] = h.ca; out[4] = h.tgap; out[5] = h.agap;
  out[6] = h.c_lo; out[7] = h.c_hi; out[8] = h.r_lo; out[9] = h.r_hi;
  frac[0] = h.tfrac;
  frac[1] = h.afrac;
  return 0;
}
