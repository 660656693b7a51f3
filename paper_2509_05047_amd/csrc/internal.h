// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sse {

constexpr float kMec2 = 510.99895f;          // electron rest energy, keV (CODATA 2018)
constexpr int kMaxSteps = 100000;            // tentative Woodcock steps per photon
constexpr int kMaxTries = 1000;              // rejection-loop guard (never reached)
constexpr int kRecordWords = 32;
constexpr int kStatCount = 21;

enum LutType { kLutF32 = 0, kLutF16 = 1, kLutBF16 = 2 };
// What happens to a single that hits a gap between modules or blocks (the
// values of sse_gap_policy).
enum GapPolicy { kGapDiscard = 0, kGapNearest = 1, kGapEdgeLut = 2 };

// A coincidence with both singles in the energy window, as the transport
// kernel hands it to the coincidence kernel: one 80-byte record per pair
// (written as five 16-byte stores).
// Per single: hit x, y, z, direction x, y, z, path length (floats) and the
// LUT energy bin; where the hit lies on the detector (crystal, ring, gap) is
// the coincidence kernel's work.
constexpr int kSingleWords = 8;
enum SingleWord { kSX = 0, kSY, kSZ, kSDx, kSDy, kSDz, kSPath, kSEbin };
enum PairWord {
  kPhLo = 0,   // history, low and high word
  kPhHi,
  kPPos,       // word of the history's stream where photon B ended
  kPFlags,     // scattered << 8 | request slot << 16, or kEmptyPair
  kPA,         // photon A, kSingleWords words
  kPB = kPA + kSingleWords,
  kPairWords = kPB + kSingleWords
};
static_assert(kPairWords % 4 == 0, "pair records are written as 16-byte stores");
constexpr uint32_t kEmptyPair = 0xffffffffu;  // flags of a padding record
// Wavefronts reserve the buffer in blocks of kPairBlock records (one atomic
// per block); the part of a block a wavefront cannot use is padded with
// empty records.
constexpr uint32_t kPairBlock = 512;
constexpr uint64_t kMaxPairCap = 1ull << 31;
// Records a launch of n histories may reserve when w wavefronts run it: one
// pair per history at most, each block padded by at most 63 records, plus
// one partly used block per wavefront.
inline uint64_t pair_records_needed(uint64_t n, uint64_t w) {
  return n + (n / (kPairBlock - 64) + 1) * 64 + w * kPairBlock;
}

// Energy-dependent transport coefficients of the separable attenuation model.
struct ECoef {
  float E, alpha, g, cC, cCR, inv_maj;
};

// Everything one transport launch reads; passed by value as the kernel argument.
struct TransportParams {
  // phantom
  const float* mu;          // mu at 511 keV, [nz][ny][nx] (binary32 map)
  const uint8_t* mu8;       // or palette indices (NULL if not used)
  const float* mu_table;    // 256-entry palette of exact mu values (NULL if not used)
  const uint2* alias;       // (threshold, alias) per column
  uint64_t nvox;
  int nx, ny, nz;
  float inv_nx, inv_nxy;   // binary32 reciprocals of nx and nx * ny
  float lox, loy, loz, hix, hiy, hiz;
  float ivx, ivy, ivz, vx, vy, vz;
  float fx_max, fy_max, fz_max;   // nx - 1, ny - 1, nz - 1
  int vox24;                      // ny nz <= 2^24: voxel indices by 24-bit multiplies
  int voxf;                       // nx ny nz <= 2^24: voxel indices by exact binary32 multiply-adds
  float fnx, fnxy;                // nx, nx ny
  float mu_maj;             // Woodcock majorant at 511 keV
  // scanner and sinogram
  int n_crystals, n_rings, cmod, rblk, max_ring_diff;
  float rr, half_len, pitch;
  int n_rad, n_view, n_plane, n_tof;
  float tof_bin, tof_sigma;
  // physics
  float e_lo, e_hi, e_kill, e_fwhm, rayleigh_beta;
  float kc, f_r, f_p;       // energy model: kc = f_C / KN(1), f_R, f_P
  int max_int;
  ECoef e511;               // coefficients at 511 keV (host-evaluated)
  // LUT
  const void* lut;
  int lut_type;
  int d0, d1, d2, d3, d4;
  float e_min, e_scale;
  // gaps between modules and blocks (gap_on = 0: plain cylinder): gap
  // policy, module and block counts, transaxial gap angle and module angle,
  // axial geometry in binary64 (half length, gap width, ring pitch, the rings
  // of a block, block period), and the edge-crystal LUTs
  int gap_on, gap_policy, n_mod, n_blk;
  double gap_t, mod_d;
  double half_len_d, gap_a, pitch_a, block_span, block_period;
  const float* edge_t;
  const float* edge_a;
  int edge_na, edge_np;
  // photon B of a history is not tracked when photon A ended outside the
  // energy window (production instantiation only)
  int prune_b;
  // run
  uint64_t seed, h0, n;
  // outputs
  uint32_t* sc_n;
  double* sc_w;
  uint32_t* tr_n;
  double* tr_w;
  unsigned long long* stats;
  uint32_t* rec;
  uint64_t rec_stride;
  uint64_t rec_h0;          // record k is history rec_h0 + k * rec_stride
  // pair buffer (device): pair_cap records of kPairWords words and the
  // count of records reserved
  uint32_t* pairs;
  uint32_t* pair_count;
  uint64_t pair_cap;
  uint32_t item;            // request slot, for the work-list form
};

// -ln(u) for a positive normal u, the logarithm of the energy model (the
// free-path sample uses the table logarithm in transport.hip): a faithful
// binary32 logarithm, fixed operation by operation so that host and device,
// and any IEEE binary32 arithmetic without contraction, give the same bits:
// u = f 2^e with f in [sqrt(1/2), sqrt(2)); s = f - 1 (exact);
// ln f = 2 atanh(r), r = s / (2 + s), whose Taylor series to z^4, z = r^2,
// is arranged as s - (s^2/2 - r (s^2/2 + R)) so the exact s is not rounded
// (the split of the fdlibm logarithm); -ln u = n ln 2 - ln f, n = -e, with
// ln 2 split so that n times its leading part is exact.
//
// Div is how the correctly rounded quotients of the binary32 model are
// formed: the IEEE operator on the host (IeeeDiv), an equivalent faster
// sequence on the device (the transport's DevDiv); both give the correctly
// rounded quotient for the operands these functions see.
struct IeeeDiv {
  __host__ __device__ static float div(float a, float b) { return a / b; }
};

template <class Div = IeeeDiv>
__host__ __device__ inline float neg_log32(float u) {
  int e;
  float f = frexpf(u, &e);
  if (f < 0.70710678f) {
    f = f + f;
    e -= 1;
  }
  const float s = f - 1.0f;
  const float r = Div::div(s, 2.0f + s);
  const float z = r * r;
  const float R = z * (2.0f / 3.0f + z * (2.0f / 5.0f + z * (2.0f / 7.0f + z * (2.0f / 9.0f))));
  const float hfsq = 0.5f * s * s;
  const float lnf = s - (hfsq - r * (hfsq + R));
  const float n = static_cast<float>(-e);
  return n * 0.693145751953125f + (n * 1.4286068e-06f - lnf);
}

// Total Klein-Nishina cross section in units of 2 pi r_e^2, a = E / m_e c^2
// (Klein and Nishina 1929), in binary32: ln(1 + 2a) by the logarithm above,
// the quotients through 1/a and 1/(1 + 2a).  Relative error below 2e-5 for
// E >= 100 keV, the lowest kill energy accepted (cancellation grows as
// a -> 0).
template <class Div = IeeeDiv>
__host__ __device__ inline float kn_total32(float a) {
  const float ia = Div::div(1.0f, a);
  const float b = 1.0f + 2.0f * a;
  const float i12 = Div::div(1.0f, b);
  const float L = -neg_log32<Div>(b);
  const float t1 = (((1.0f + a) * ia) * ia) * ((2.0f * (1.0f + a)) * i12 - L * ia);
  const float t2 = (0.5f * L) * ia;
  const float t3 = ((1.0f + 3.0f * a) * i12) * i12;
  return (t1 + t2) - t3;
}

// Coefficients of the separable attenuation model mu(x, E) = mu511(x) g(E),
// g = fC + fR + fP with fC = kc KN(a) (kc = f_C / KN(1)), fR = f_R / a^2 and
// fP = f_P / a^3, in binary32 (host and device evaluate it alike).  The
// majorant's reciprocal uses the IEEE operator: its divisor is 0 for a
// phantom of air.
template <class Div = IeeeDiv>
__host__ __device__ inline void energy_coefficients(ECoef& c, float E, float kc, float f_r, float f_p,
                                                    float mu_maj) {
  c.E = E;
  c.alpha = Div::div(E, kMec2);
  const float a = c.alpha;
  const float ia = Div::div(1.0f, a);
  const float fc = kc * kn_total32<Div>(a);
  const float fr = f_r * ia * ia;
  const float fp = f_p * ia * ia * ia;
  c.g = (fc + fr) + fp;
  c.cC = fc;
  c.cCR = fc + fr;
  c.inv_maj = 1.0f / (mu_maj * c.g);
}

// Transport and coincidence evaluation of histories [h0, h0 + n): launches
// sized to the pair buffer, each a pair-counter reset, the transport kernel
// and the coincidence kernel, in stream order.
hipError_t launch_transport(const TransportParams& p, hipStream_t stream);
// Pair-buffer capacity (records) one launch of n histories needs, and the
// most histories a launch may take with capacity cap (0 if none).
uint64_t transport_pairs_needed(uint64_t n);
uint64_t transport_max_histories(uint64_t cap);
uint64_t transport_batch_pairs_needed(uint64_t n);
uint64_t transport_batch_max_histories(uint64_t cap);

// The free-path logarithm's table, built on the host and copied to the
// current device's constant memory (once per context is enough; every copy
// is the same).
hipError_t upload_log_table();

// The device division check (counts: two zeroed device words).
hipError_t launch_check_division(uint64_t n, uint32_t seed, unsigned long long* counts, hipStream_t stream);

// One sub-chunk of a request: histories [h0, h0 + n) of items[item].
struct WorkChunk {
  uint64_t h0;
  uint32_t n;
  uint32_t item;
};

// Histories per claim of the work-list kernel; each chunk of a launch takes
// its length rounded up to a multiple of this in the claim positions.
constexpr uint32_t kBatchSlice = 256;

// A list of sub-chunks over several requests, simulated by one launch.
struct BatchParams {
  const TransportParams* items;  // device array, one per request slot
  const WorkChunk* chunks;       // device array
  uint32_t n_chunks;
  uint32_t n_positions;          // sum of the chunks' lengths rounded up to multiples of kBatchSlice
  uint32_t* counter;             // device claim cursor (positions), reset by the launcher
  uint64_t n_histories;          // sum of the chunks' lengths
  uint32_t* pairs;               // the items' common pair buffer
  uint32_t* pair_count;
  uint64_t pair_cap;
  int gap_on;                    // the items' gap model is on (they share one context)
  // No slice is claimed once the pair counter exceeds stop_at (a fill
  // launch: the launch ends early and the next one goes on from the claim
  // cursor); ~0 never stops.
  uint64_t stop_at = ~0ull;
  // Fill launches: a flag, in a cache line of its own, that the wavefront
  // finding the cursor at the end sets; while it is set no slice is claimed
  // (or NULL: not kept).
  uint32_t* done = nullptr;
};

// Words from the claim cursor to the fill launches' end flag (128 bytes: the
// flag lies in another cache line than the cursor's atomic adds); d_cursor of
// launch_transport_item holds at least kCursorWords words.
constexpr uint32_t kDoneOffsetWords = 32;
constexpr uint32_t kCursorWords = 64;

// HIP events recorded around the kernels of work-list launches (for
// measurement): launch i records ev[4i] / ev[4i + 1] before and after its
// transport kernel and ev[4i + 2] / ev[4i + 3] around its coincidence kernel,
// while n < cap; launches beyond cap are counted in dropped.
struct KernelTiming {
  hipEvent_t* ev;
  uint32_t cap;
  uint32_t n;
  uint64_t dropped;
};

// One work list (at most transport_batch_max_histories(pair_cap) histories
// in all): pair-counter reset, transport, coincidences (timed if kt).
hipError_t launch_transport_batch(const BatchParams& b, hipStream_t stream, KernelTiming* kt = nullptr);
// Histories [p.h0, p.h0 + p.n) of one request through the work-list kernels
// (the production path of a simulate call: no statistics, no records):
// fill launches when the pair buffer is large enough, else launches of at
// most transport_batch_max_histories(p.pair_cap) histories; d_item, d_chunk
// and d_cursor are device scratch of one parameter set, one chunk and the
// claim cursor with the fill launches' end flag (kCursorWords words).
hipError_t launch_transport_item(const TransportParams& p, TransportParams* d_item, WorkChunk* d_chunk,
                                 uint32_t* d_cursor, hipStream_t stream, KernelTiming* kt = nullptr);

// Allocation-free simulate (sse_simulate_noalloc): the kernels' scratch --
// work-list parameters, counters and pair buffer -- is a file-scope device
// array of kNoAllocScratchBytes.  noalloc_scratch_init looks its address up
// on `device` (which must be current) once per device; the launch then
// splits [p.h0, p.h0 + p.n) into work-list launches that fit it (p's pair
// buffer fields are replaced).  noalloc_max_histories: the most histories
// one launch takes (0 if the resident grid needs more than the scratch).
constexpr uint64_t kNoAllocScratchBytes = 256ull << 20;
hipError_t noalloc_scratch_init(int device);
uint64_t noalloc_max_histories();
hipError_t launch_transport_noalloc(int device, const TransportParams& p, hipStream_t stream);

}  // namespace sse
