// Monte Carlo pair transport, detection, LUT weighting and TOF sinogram
// accumulation on gfx950.
//
// One launch simulates histories h0 .. h0+n-1.  Each history: emission from
// the activity alias table, two photons tracked with Woodcock steps through
// the attenuation map (Compton by Kahn's method, Rayleigh with an analytic
// form factor, photoabsorption), crossing of the detection cylinder, crystal /
// ring / 5D-LUT indexing of each single (with the gaps between modules and
// blocks and the edge-crystal assignment when they are modelled), and one
// atomic update of the TOF sinogram bin with count 1 and weight p_A p_B
// (Methods, "Scatter simulator description", "Photon detection probability
// LUT" and "Edge crystal assignment LUT").
//
// Execution model: a persistent grid; every wavefront owns a contiguous range
// of histories and every lane runs a small state machine
//     EMIT -> TRACK (photon A) -> FINISH -> TRACK (photon B) -> FINISH -> EMIT
// advancing to its next event (a real interaction or the end of the photon)
// per loop iteration.  A lane whose history ends takes the next history of
// its wave immediately, so lanes never idle while the slowest lane of the
// wave finishes, and each expensive branch runs once per iteration for all
// lanes that need it.
//
// Numerics: binary32 transport with IEEE-rounded + - * / sqrt (no
// contraction); the free-path logarithm, the azimuth's sine and cosine and
// the cross-section model in binary32 by fixed operation sequences; the
// detector-side atan2 and the TOF jitter's logarithm in binary64, rounded
// once where they feed binary32 values.  Random numbers: one Philox4x32-10
// stream per history, keyed by the seed and countered by (block, history),
// consumed in order by the emission, photon A, photon B, the edge-crystal
// draws and the TOF jitter, so a history's result does not depend on the
// launch geometry.
#include "internal.h"
#include <cmath>
#include <cstring>
#include <mutex>

namespace sse {
namespace {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;
constexpr double kHalfPi = 1.5707963267948966;

// kCompton is a rejection sampling that may take several iterations of the
// wave's loop (a bounded number of rounds per iteration); kAzimuth draws the
// azimuth of a scattered photon and turns it.
enum Phase { kEmit = 0, kTrack = 1, kInteract = 2, kFinish = 3, kDone = 4, kCompton = 5, kAzimuth = 6 };
enum Fate { kDetected = 0, kAbsorbed = 1, kKilled = 2, kCapped = 3, kAxial = 4, kEscaped = 5 };
enum Stat {
  kStHist = 0, kStSteps, kStReal, kStCompton, kStRayleigh, kStAbsorbed, kStKilled, kStCapped, kStEscaped,
  kStDetected, kStInWindow, kStScatter, kStTrue, kStRejWindow, kStRejSame, kStRejRing, kStRejRadial,
  kStRejTof, kStRngBlocks, kStRejGap, kStGapAssigned
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                       uint32_t k1, uint32_t& o0, uint32_t& o1, uint32_t& o2, uint32_t& o3) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t a = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t b = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(b >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(a >> 32) ^ c3 ^ k1;
    c1 = static_cast<uint32_t>(b);
    c3 = static_cast<uint32_t>(a);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

// Statistics: at each counting site the lowest active lane adds the
// population count of the wave's ballot to a per-block LDS counter (a
// wave-uniform accumulator cannot live in a register that divergent lanes
// update separately).  The predicate is evaluated whether or not statistics
// are collected.
#define SSE_COUNT(idx, pred)                                                          \
  do {                                                                                \
    const bool v_ = (pred);                                                           \
    if (kInstr && p.stats) {                                                          \
      const uint64_t m_ = __ballot(static_cast<int>(v_));                            \
      if (m_ && lane == static_cast<uint32_t>(__builtin_ctzll(__builtin_amdgcn_read_exec()))) \
        atomicAdd(&s_stats[idx], static_cast<unsigned long long>(__popcll(m_)));      \
    }                                                                                 \
  } while (0)

// Wave votes over the active lanes.  A vote on a conjunction is taken as
// the AND of the two comparisons' lane masks: a ballot of a combined
// predicate is compiled as a value that is compared back into a mask (two
// more vector instructions, one of them a 4-cycle select).
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }
__device__ __forceinline__ bool wave_any(bool p, bool q) {
  return (__builtin_amdgcn_ballot_w64(p) & __builtin_amdgcn_ballot_w64(q)) != 0;
}
__device__ __forceinline__ bool wave_all(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

// A history's random stream: the 32-bit words of Philox blocks 0, 1, 2, ...
// with counter (block, h_lo, h_hi, 0), consumed in order.
//
// Lane streams keep up to kRngSlots words in LDS, in a column per lane (slot
// i of lane l at word 64 i + l, so a wave's accesses hit distinct banks).
// Block b goes to slots 4 (b mod kRngSlots/4) .. +3, and words are read
// from slot rd, advancing mod kRngSlots; a lane may generate its next block
// whenever it has room for four more words, so a refill that one lane needs
// is shared by every lane of the wave with room and Philox runs mostly
// converged.  Reading a word is one LDS load: no register shuffling and no
// dynamically indexed registers.
typedef __attribute__((address_space(3))) uint32_t LdsWord;
constexpr uint32_t kRngSlots = 8;

__device__ __forceinline__ float to_uniform(uint32_t x) {
  // uniform in (0, 1): 24 bits with the last forced odd, times 2^-24
  return static_cast<float>((x >> 8) | 1u) * 5.9604644775390625e-08f;
}

// ---------------------------------------------------------------------------
// free-path logarithm
// ---------------------------------------------------------------------------
// -ln(u) of a transport uniform u in (0, 1), the free-path sample of the
// Woodcock step (Methods, "Scatter simulator description"): a faithful
// binary32 logarithm (below 0.85 units in the last place for every uniform
// the generator can produce; 99.7 % correctly rounded), fixed operation by
// operation with fused multiply-adds, after the table method of Tang (1990):
//   u = F 2^k with F in [sqrt(1/2), sqrt(2))             (frexp, exact)
//   i = (bits(F) - kLogBase) >> 16, 0 <= i < kLogEntries: the row whose F
//     range (2^16 consecutive binary32 values) holds F; row 75 is the range
//     around F = 1
//   c_i = RN(1 / mid_i), mid_i the midpoint of the range, and c_i = 1 for
//     rows 73..77 (|F - 1| < 0.02), so that no table term cancels a small
//     result
//   T_i = -ln(c_i) = hi_i + lo_i, hi_i = T_i rounded to a multiple of
//     2^-16, lo_i = RN(T_i - hi_i)
//   r = RN(F c_i - 1)                                    (one fused rounding)
//   ln(1 + r) = r + r^2 (-1/2 + r (1/3 + r (-1/4 + r/5)))
//   ln u = (k ln2_hi + hi_i) + ((ln(1 + r) + lo_i) + k ln2_lo), ln 2 split
//     so that the first sum is exact (multiples of 2^-16 below 2^5).
// The table (c_i, hi_i, lo_i, 0 per row) is built on the host in binary64
// and kept in constant memory; each block stages it in LDS.
constexpr int kLogEntries = 129;
constexpr uint32_t kLogBase = 0x3F348000u;  // bits of 1.0, less 2^15 and 75 rows of 2^16
__constant__ float4 c_log_rows[kLogEntries];
// (a generic pointer to the block's LDS copy: the loads stay LDS loads once
// the kernel is inlined, as the pointer's origin is known)
typedef const float4 LdsLogRow;

__device__ __forceinline__ float free_path_log32(float u, LdsLogRow* rows) {
  int e;
  float f = frexpf(u, &e);
  if (f < 0.70710678f) {
    f = f + f;
    e -= 1;
  }
  const float4 t = rows[(__float_as_uint(f) - kLogBase) >> 16];
  const float r = __builtin_fmaf(f, t.x, -1.0f);
  const float q0 = __builtin_fmaf(r, 0.2f, -0.25f);
  const float q1 = __builtin_fmaf(r, q0, 0.33333334f);
  const float q2 = __builtin_fmaf(r, q1, -0.5f);
  const float r2 = r * r;
  const float l1p = __builtin_fmaf(r2, q2, r);
  const float k = static_cast<float>(e);
  const float hi = __builtin_fmaf(k, 0.693145751953125f, t.y);
  const float lo = __builtin_fmaf(k, 1.4286068e-06f, l1p + t.z);
  return -(hi + lo);
}

// the block's copy of the table (all threads; a barrier follows)
__device__ __forceinline__ void stage_log_rows(float4* rows) {
  for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(kLogEntries); i += blockDim.x) rows[i] = c_log_rows[i];
}

// ---------------------------------------------------------------------------
// division
// ---------------------------------------------------------------------------
// The correctly rounded binary32 quotient a / b without the general divide
// sequence (scaling, special cases): the hardware reciprocal (within one ulp)
// refined by one Newton step is the correctly rounded reciprocal RN(1/b) for
// every significand (sse_check_division verifies all 2^23 of them on the
// device), and with RN(1/b) one remainder correction of q = RN(a y) gives
// RN(a / b) (Markstein 1990).  Valid while b, 1/b and a/b are normal numbers,
// which holds for every quotient the transport forms (see the call sites);
// six instructions instead of about twelve.
struct DevDiv {
  __device__ static float div(float a, float b) {
    const float y0 = __builtin_amdgcn_rcpf(b);
    const float y = __builtin_fmaf(__builtin_fmaf(-b, y0, 1.0f), y0, y0);
    const float q = a * y;
    const float r = __builtin_fmaf(-b, q, a);
    return __builtin_fmaf(r, y, q);
  }
};
__device__ __forceinline__ float fdiv(float a, float b) { return DevDiv::div(a, b); }

// The key is the same for every lane of a transport wavefront.  Passed to
// Philox as an opaque scalar, its ten round keys are formed by scalar adds at
// each use: otherwise the compiler keeps all twenty of them live across the
// whole transport loop, spills them into vector-register lanes and reads
// them back with two extra vector instructions per round.
__device__ __forceinline__ void wave_uniform_key(uint32_t& k0, uint32_t& k1) {
  k0 = __builtin_amdgcn_readfirstlane(k0);
  k1 = __builtin_amdgcn_readfirstlane(k1);
  asm volatile("" : "+s"(k0), "+s"(k1));
}

struct LaneRng {
  LdsWord* col;  // this lane's column
  uint32_t hlo, hhi, blk, left, rd;

  __device__ __forceinline__ void start(uint64_t h) {
    hlo = static_cast<uint32_t>(h);
    hhi = static_cast<uint32_t>(h >> 32);
    blk = 0;
    left = 0;
    rd = 0;
  }
  // go on at block b with nothing buffered (the read slot follows the block)
  __device__ __forceinline__ void seek_block(uint32_t b) {
    blk = b;
    left = 0;
    rd = (b * 4u) & (kRngSlots - 1u);
  }
  __device__ __forceinline__ bool room() const { return left <= kRngSlots - 4u; }
  __device__ __forceinline__ void refill(uint32_t k0, uint32_t k1) {
    uint32_t b0, b1, b2, b3;
    wave_uniform_key(k0, k1);
    philox(blk, hlo, hhi, 0u, k0, k1, b0, b1, b2, b3);
    LdsWord* d = col + ((blk & (kRngSlots / 4u - 1u)) << 8);  // slots 4 (blk mod kRngSlots/4) .. +3
    d[0] = b0;
    d[64] = b1;
    d[128] = b2;
    d[192] = b3;
    ++blk;
    left += 4;
  }
  __device__ __forceinline__ uint32_t take() {
    const uint32_t x = col[rd << 6];
    rd = (rd + 1u) & (kRngSlots - 1u);
    --left;
    return x;
  }
  __device__ __forceinline__ float uniform() { return to_uniform(take()); }
  // word k ahead of the next one, not consumed (k < left for a valid word)
  __device__ __forceinline__ uint32_t peek(uint32_t k) const { return col[((rd + k) & (kRngSlots - 1u)) << 6]; }
  __device__ __forceinline__ void advance(uint32_t k) {
    rd = (rd + k) & (kRngSlots - 1u);
    left -= k;
  }
};

// A stream held in registers (a shift register w0..w7, w0 next, with the
// same refill rule): the re-positioned copy of a history's stream that the
// coincidence evaluation draws the TOF jitter from.
struct RegRng {
  uint32_t hlo, hhi, blk, left;
  uint32_t w0, w1, w2, w3, w4, w5, w6, w7;

  __device__ __forceinline__ void start(uint64_t h) {
    hlo = static_cast<uint32_t>(h);
    hhi = static_cast<uint32_t>(h >> 32);
    blk = 0;
    left = 0;
  }
  __device__ __forceinline__ bool room() const { return left <= 4u; }
  __device__ __forceinline__ void refill(uint32_t k0, uint32_t k1) {
    uint32_t b0, b1, b2, b3;
    philox(blk, hlo, hhi, 0u, k0, k1, b0, b1, b2, b3);
    ++blk;
    const uint32_t L = left;  // 0 .. 4: the new words go to slots L .. L+3
    w0 = L == 0 ? b0 : w0;
    w1 = L == 0 ? b1 : (L == 1 ? b0 : w1);
    w2 = L == 0 ? b2 : (L == 1 ? b1 : (L == 2 ? b0 : w2));
    w3 = L == 0 ? b3 : (L == 1 ? b2 : (L == 2 ? b1 : (L == 3 ? b0 : w3)));
    w4 = L == 1 ? b3 : (L == 2 ? b2 : (L == 3 ? b1 : (L == 4 ? b0 : w4)));
    w5 = L == 2 ? b3 : (L == 3 ? b2 : (L == 4 ? b1 : w5));
    w6 = L == 3 ? b3 : (L == 4 ? b2 : w6);
    w7 = L == 4 ? b3 : w7;
    left = L + 4;
  }
  __device__ __forceinline__ uint32_t take() {
    const uint32_t x = w0;
    w0 = w1; w1 = w2; w2 = w3; w3 = w4; w4 = w5; w5 = w6; w6 = w7;
    --left;
    return x;
  }
  __device__ __forceinline__ float uniform() { return to_uniform(take()); }
};

// Make sure every active lane holds at least k (<= 4) words: if any lane is
// short, all active lanes with room generate one block together.
#define RNG_NEED(k)                                  \
  do {                                               \
    if (wave_any(r.left < (k))) {                       \
      if (r.room()) r.refill(k0, k1);                \
    }                                                \
  } while (0)

// The statistics count the Philox blocks a history uses -- ceil(words
// consumed / 4), the blocks an on-demand generator would make -- not the
// ones generated ahead of need.
__device__ __forceinline__ uint64_t blocks_used(uint32_t words) { return (words + 3u) / 4u; }

// (sin 2 pi u, cos 2 pi u) for u in [0, 1), fixed operation by operation
// (error below 1.7 * 2^-24 for the transport's uniforms):
// 4u = q + f with q the quadrant and f in [0, 1) (exact); h = f, or 1 - f
// when f > 1/2 (sine and cosine swap; exact); y = h pi/2 in [0, pi/4],
// z = y^2, and the Taylor series of sin y to y^9 and of cos y to y^10 (the
// first omitted terms are below 2e-9); then the quadrant's signs.
__device__ __forceinline__ void sincos_2pi(float u, float& sn, float& cs) {
  const float v = 4.0f * u;
  const int q = static_cast<int>(floorf(v));
  const float f = v - static_cast<float>(q);
  const bool swap = f > 0.5f;
  const float h = swap ? 1.0f - f : f;
  const float y = h * 1.5707963267948966f;
  const float z = y * y;
  const float s = y + (y * z) * (-1.0f / 6.0f + z * (1.0f / 120.0f + z * (-1.0f / 5040.0f + z * (1.0f / 362880.0f))));
  const float c =
      1.0f + z * (-0.5f + z * (1.0f / 24.0f + z * (-1.0f / 720.0f + z * (1.0f / 40320.0f + z * (-1.0f / 3628800.0f)))));
  const float sf = swap ? c : s, cf = swap ? s : c;
  const int qq = q & 3;
  sn = qq == 0 ? sf : (qq == 1 ? cf : (qq == 2 ? -sf : -cf));
  cs = qq == 0 ? cf : (qq == 1 ? -sf : (qq == 2 ? -cf : sf));
}

// ---------------------------------------------------------------------------
// physics
// ---------------------------------------------------------------------------

// New direction after scattering by polar cosine ct and azimuth (cp, sp)
// about the old direction u: d' = ct u + st (cp e1 + sp e2) in the frame
// e1 = (ux uz / s, uy uz / s, -s), e2 = (-uy / s, ux / s, 0) with
// s = sqrt(ux^2 + uy^2), orthogonal to u whatever the rounding of u's norm.
// A direction within 1e-10 of the axis takes the axis itself as u, with
// (e1, e2) = (x, y) about +z and (x, -y) about -z (right-handed, as the
// frame's limits).  The quotients have s >= 1e-10 as divisor.
__device__ __forceinline__ void rotate(float& dx, float& dy, float& dz, float ct, float cp, float sp) {
  const float st = sqrtf((1.0f - ct) * (1.0f + ct));
  const float ux = dx, uy = dy, uz = dz;
  const float tt = ux * ux + uy * uy;
  if (!(tt > 1e-20f)) {
    const float sg = uz > 0.0f ? 1.0f : -1.0f;
    dx = st * cp;
    dy = sg * st * sp;
    dz = sg * ct;
  } else {
    const float s = sqrtf(tt);
    dx = ux * ct + fdiv(st * (ux * uz * cp - uy * sp), s);
    dy = uy * ct + fdiv(st * (uy * uz * cp + ux * sp), s);
    dz = uz * ct - s * st * cp;
  }
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
// Distance along d from p to the exit of the voxel box: the least of the
// per-axis quotients, all three computed (no branches) and those of axes
// the direction does not move along left out.
// The box's bounds are read as wave-uniform values before the per-lane
// select: a select between two parameter fields otherwise becomes a select
// of their addresses and a vector load, whose latency the few lanes that
// scatter in an iteration wait out.
__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ __forceinline__ float box_exit(const TransportParams& p, float px, float py, float pz, float dx,
                                          float dy, float dz) {
  const float lox = uniform_f(p.lox), loy = uniform_f(p.loy), loz = uniform_f(p.loz);
  const float hix = uniform_f(p.hix), hiy = uniform_f(p.hiy), hiz = uniform_f(p.hiz);
  // a quotient by a zero component is not used (its value does not matter)
  const float qx = fdiv(dx > 0.0f ? hix - px : lox - px, dx);
  const float qy = fdiv(dy > 0.0f ? hiy - py : loy - py, dy);
  const float qz = fdiv(dz > 0.0f ? hiz - pz : loz - pz, dz);
  float t = __builtin_huge_valf();
  t = dx != 0.0f ? fminf(t, qx) : t;
  t = dy != 0.0f ? fminf(t, qy) : t;
  t = dz != 0.0f ? fminf(t, qz) : t;
  return t;
}

// floor(f) clamped to [0, n - 1]; NaN gives 0 (maximum returns the number).
__device__ __forceinline__ int clamp_floor(float f, int n) {
  return static_cast<int>(fminf(fmaxf(floorf(f), 0.0f), static_cast<float>(n - 1)));
}

// Voxel of a point, clamped to the grid (a valid index for any finite
// point): the clamp is one median-of-three before the floor, which equals
// flooring first and clamping to [0, n - 1] after.  The index is formed from
// the floored coordinates by two binary32 multiply-adds when the grid has at
// most 2^24 voxels (every partial sum is then an integer below 2^24, exact),
// else by 24-bit multiplies when the grid's sizes allow them (vox24).
__device__ __forceinline__ uint32_t voxel_at(const TransportParams& p, float x, float y, float z) {
  const float fx = floorf(__builtin_amdgcn_fmed3f((x - p.lox) * p.ivx, 0.0f, p.fx_max));
  const float fy = floorf(__builtin_amdgcn_fmed3f((y - p.loy) * p.ivy, 0.0f, p.fy_max));
  const float fz = floorf(__builtin_amdgcn_fmed3f((z - p.loz) * p.ivz, 0.0f, p.fz_max));
  if (p.voxf) return static_cast<uint32_t>(__builtin_fmaf(fz, p.fnxy, __builtin_fmaf(fy, p.fnx, fx)));
  const uint32_t ix = static_cast<uint32_t>(fx), iy = static_cast<uint32_t>(fy), iz = static_cast<uint32_t>(fz);
  const uint32_t nx = static_cast<uint32_t>(p.nx), ny = static_cast<uint32_t>(p.ny);
  if (p.vox24) return __umul24(__umul24(iz, ny) + iy, nx) + ix;
  return (iz * ny + iy) * nx + ix;
}

__device__ __forceinline__ int angle_bin(double th, int n) {
  const double f = floor((th + kHalfPi) * static_cast<double>(n) / kPi);
  if (!(f >= 0.0)) return 0;
  if (f >= static_cast<double>(n)) return n - 1;
  return static_cast<int>(f);
}

__device__ __forceinline__ float lut_value(const TransportParams& p, uint32_t i) {
  if (p.lut_type == kLutF32) return static_cast<const float*>(p.lut)[i];
  const uint16_t b = static_cast<const uint16_t*>(p.lut)[i];
  if (p.lut_type == kLutF16) return static_cast<float>(__builtin_bit_cast(_Float16, b));
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

__device__ __forceinline__ int clamp_index_d(double f, int n) {
  if (!(f >= 0.0)) return 0;
  if (f >= static_cast<double>(n)) return n - 1;
  return static_cast<int>(f);
}

// Crystal of a single detected at (hx, hy) on the plain cylinder: azimuth in
// [0, 2 pi) in binary64.
__device__ __forceinline__ int crystal_of(const TransportParams& p, float hx, float hy) {
  double phi = atan2(static_cast<double>(hy), static_cast<double>(hx));
  if (phi < 0.0) phi += kTwoPi;
  const double fc = floor(phi * static_cast<double>(p.n_crystals) / kTwoPi);
  return fc >= static_cast<double>(p.n_crystals) ? p.n_crystals - 1 : (fc < 0.0 ? 0 : static_cast<int>(fc));
}

__device__ __forceinline__ int ring_of(const TransportParams& p, float hz) {
  return clamp_floor((hz + p.half_len) / p.pitch, p.n_rings);
}

__device__ __forceinline__ int energy_bin(const TransportParams& p, float E) {
  return clamp_floor((E - p.e_min) * p.e_scale, p.d0);
}

// Where a single falls on the detector (Methods, "Scatter simulator
// description", Fig. 4): the crystal and ring it is assigned to (for a hit in
// a gap, the nearest edge crystal and ring), its coordinates on the LUT's
// crystal axes, and for a gap hit the edge crystals / rings of the lower and
// upper side and the position across the gap (0 at the lower side).
struct Hit {
  int crystal, ring, ct, ca;
  int c_lo, c_hi, r_lo, r_hi;
  double tfrac, afrac;
  bool tgap, agap;
};

// The plain cylinder: the LUT's crystal axes bin the crystal in its module
// and the ring in its block.
__device__ __forceinline__ void locate_plain(const TransportParams& p, float hx, float hy, float hz, Hit& h) {
  h.tgap = false;
  h.agap = false;
  h.c_lo = h.c_hi = h.r_lo = h.r_hi = 0;
  h.tfrac = h.afrac = 0.0;
  h.crystal = crystal_of(p, hx, hy);
  h.ring = ring_of(p, hz);
  h.ct = ((h.crystal % p.cmod) * p.d3) / p.cmod;
  h.ca = ((h.ring % p.rblk) * p.d4) / p.rblk;
}

__device__ void locate(const TransportParams& p, float hx, float hy, float hz, Hit& h) {
  if (!p.gap_on) {
    locate_plain(p, hx, hy, hz, h);
    return;
  }
  h.tgap = false;
  h.agap = false;
  h.c_lo = h.c_hi = h.r_lo = h.r_hi = 0;
  h.tfrac = h.afrac = 0.0;
  const int cm = p.cmod, rb = p.rblk, nm = p.n_mod, nb = p.n_blk;
  // Transaxial: module m spans azimuth [m D, (m + 1) D) with half a gap of
  // angle g at either end and cm crystals of width (D - g) / cm between.
  // LUT index 0 is the gap half before the module, cm + 1 the one after it.
  const double g = p.gap_t, D = p.mod_d;
  double phi = atan2(static_cast<double>(hy), static_cast<double>(hx));
  if (phi < 0.0) phi += kTwoPi;
  const int m = clamp_index_d(floor(phi / D), nm);
  const double loc = phi - static_cast<double>(m) * D;
  if (g > 0.0 && loc < 0.5 * g) {
    h.tgap = true;
    h.c_lo = ((m + nm - 1) % nm) * cm + cm - 1;
    h.c_hi = m * cm;
    h.crystal = h.c_hi;
    h.ct = 0;
    h.tfrac = (loc + 0.5 * g) / g;
  } else if (g > 0.0 && loc >= D - 0.5 * g) {
    h.tgap = true;
    h.c_lo = m * cm + cm - 1;
    h.c_hi = ((m + 1) % nm) * cm;
    h.crystal = h.c_lo;
    h.ct = cm + 1;
    h.tfrac = (loc - (D - 0.5 * g)) / g;
  } else {
    const int k = clamp_index_d(floor((loc - 0.5 * g) * static_cast<double>(cm) / (D - g)), cm);
    h.crystal = m * cm + k;
    h.ct = k + 1;
  }
  // Axial: blocks of rb rings of pitch pitch_a separated by gaps of width w
  // (none at the scanner's ends).  Block b's rings have LUT indices
  // b (rb + 2) + 1 + k, the gap halves either side of it b (rb + 2) and
  // b (rb + 2) + rb + 1.
  const double w = p.gap_a;
  const double z = static_cast<double>(hz) + p.half_len_d;
  const int b = clamp_index_d(floor(z / p.block_period), nb);
  const double zl = z - static_cast<double>(b) * p.block_period;
  if (w > 0.0 && b < nb - 1 && zl >= p.block_span) {
    const double go = zl - p.block_span;
    h.agap = true;
    h.r_lo = b * rb + rb - 1;
    h.r_hi = (b + 1) * rb;
    h.afrac = go / w;
    const bool lower = go < 0.5 * w;
    h.ring = lower ? h.r_lo : h.r_hi;
    h.ca = lower ? b * (rb + 2) + rb + 1 : (b + 1) * (rb + 2);
  } else {
    const int k = clamp_index_d(floor(zl / p.pitch_a), rb);
    h.ring = b * rb + k;
    h.ca = b * (rb + 2) + 1 + k;
  }
  // a LUT axis of size 1 ignores the coordinate
  if (p.d3 == 1) h.ct = 0;
  if (p.d4 == 1) h.ca = 0;
}

// Transaxial and axial incidence angles of a single: the angles between its
// path and the hit point's position vector, projected in the transaxial and
// axial planes, in [-90, 90] degrees (Fig. 5 caption), binary64.
__device__ __forceinline__ void incidence(float hx_, float hy_, float dx, float dy, float dz, double& th_t,
                                          double& th_a) {
  const double hx = static_cast<double>(hx_), hy = static_cast<double>(hy_);
  const double rho = sqrt(hx * hx + hy * hy);
  const double dr = (hx * static_cast<double>(dx) + hy * static_cast<double>(dy)) / rho;
  const double tt = (hx * static_cast<double>(dy) - hy * static_cast<double>(dx)) / rho;
  th_t = atan2(tt, dr);
  th_a = atan2(static_cast<double>(dz), dr);
}

// Flat LUT index of a single: energy bin, incidence angles, crystal axes.
__device__ __forceinline__ uint32_t lut_index(const TransportParams& p, int ie, double th_t, double th_a, int ct,
                                              int ca) {
  const int it = angle_bin(th_t, p.d1);
  const int ia = angle_bin(th_a, p.d2);
  return static_cast<uint32_t>((((ie * p.d1 + it) * p.d2 + ia) * p.d3 + ct) * p.d4 + ca);
}

// crystal | ring << 16 (the nearest edge ones for a gap hit) and the flat LUT
// index of a single detected at (hx, hy, hz) with direction (dx, dy, dz) and
// energy E.
__device__ void index_single(const TransportParams& p, float hx, float hy, float hz, float dx, float dy, float dz,
                             float E, uint32_t& crystal_ring, uint32_t& lut) {
  Hit h;
  locate(p, hx, hy, hz, h);
  double th_t, th_a;
  incidence(hx, hy, dx, dy, dz, th_t, th_a);
  crystal_ring = static_cast<uint32_t>(h.crystal) | (static_cast<uint32_t>(h.ring) << 16);
  lut = lut_index(p, energy_bin(p, E), th_t, th_a, h.ct, h.ca);
}

// q = v / d for v < 2^24 and d >= 1: binary32 reciprocal estimate (off by at
// most one) and one integer correction.
__device__ __forceinline__ uint32_t udiv24(uint32_t v, uint32_t d, float inv_d) {
  uint32_t q = static_cast<uint32_t>(static_cast<float>(v) * inv_d);
  const int32_t rem = static_cast<int32_t>(v) - static_cast<int32_t>(q * d);
  if (rem < 0) --q;
  else if (rem >= static_cast<int32_t>(d)) ++q;
  return q;
}

// ---------------------------------------------------------------------------
// tuning of the transport loop
// ---------------------------------------------------------------------------
// Lanes left stepping when a wave moves on to its events (measured on the
// clinical workload: flat between 8 and 12, slower at 4 and 16).
constexpr int kStepTail = 10;
// Rejection rounds per iteration for the Compton sampler; a lane still
// rejecting goes on in the next iteration with its try count.
constexpr int kRounds = 2;
// Waves per SIMD the transport kernels are compiled for (registers, at most
// 102 each).  With eight random-word slots per lane the work-list kernel's
// LDS (about 31 KB per block) also admits five 256-thread blocks per CU:
// the loop waits on its gathers and LDS reads, and a fifth wave per SIMD
// hides more of that than the deeper word buffer of sixteen slots saved in
// refills (measured: 68.4 against 72.2 ms for 1e9 clinical histories).
constexpr int kTransportWavesPerEu = 5;
// The instrumented instantiation (statistics and records) keeps more state
// live; it is compiled for three.
constexpr int kInstrWavesPerEu = 3;

// ---------------------------------------------------------------------------
// coincidences
// ---------------------------------------------------------------------------
// Pairs with both singles in the energy window are rare (about one history
// in twenty) but their evaluation -- two crystal and LUT look-ups with
// binary64 atan2, the sinogram geometry, the TOF jitter and the atomic
// update -- is long and needs most of the detector and sinogram parameters.
// Inside the transport loop it would run with a few lanes active and keep
// those parameters live (and spilled) through every Woodcock step, so the
// transport kernel appends such pairs to a buffer in device memory and the
// coincidence kernel evaluates them, one pair per lane.  The jitter is drawn
// from the history's own stream at the position photon B left it, so the
// result is the one an in-place evaluation gives.

// Standard normal by Marsaglia's polar method from stream q (a lane's own,
// or a copy re-positioned in a history's stream).
template <class Q>
__device__ __forceinline__ float std_normal(Q& q, const TransportParams& p) {
  const uint32_t k0 = static_cast<uint32_t>(p.seed), k1 = static_cast<uint32_t>(p.seed >> 32);
  for (int i = 0; i < kMaxTries; ++i) {
    if (wave_any(q.left < 2u)) {
      if (q.room()) q.refill(k0, k1);
    }
    const float a = 2.0f * q.uniform() - 1.0f;
    const float b = 2.0f * q.uniform() - 1.0f;
    const float s = a * a + b * b;
    if (s < 1.0f) return a * static_cast<float>(sqrt(-2.0 * log(static_cast<double>(s)) / static_cast<double>(s)));
  }
  return 0.0f;
}

// Edge-crystal assignment of a gap hit of a coincidence (Methods, "Edge
// crystal assignment LUT"): with the edge-LUT policy a uniform from the
// history's stream below the table's probability (at the incidence-angle and
// position bin) picks the lower side's edge crystal or ring, otherwise the
// upper side's; a hit in both kinds of gap draws for the transaxial gap
// first.  The nearest policy keeps the nearest edge crystal.  Returns the
// number of gap assignments.
__device__ int resolve_gap(const TransportParams& p, RegRng& q, Hit& h, double th_t, double th_a) {
  const uint32_t k0 = static_cast<uint32_t>(p.seed), k1 = static_cast<uint32_t>(p.seed >> 32);
  const bool draw = p.gap_policy == kGapEdgeLut;
  const int np = p.edge_np;
  int n = 0;
  if (h.tgap) {
    if (draw) {
      const int ia = angle_bin(th_t, p.edge_na);
      const int ip = clamp_index_d(floor(h.tfrac * static_cast<double>(np)), np);
      if (q.left == 0u) q.refill(k0, k1);
      h.crystal = q.uniform() < p.edge_t[ia * np + ip] ? h.c_lo : h.c_hi;
    }
    ++n;
  }
  if (h.agap) {
    if (draw) {
      const int ia = angle_bin(th_a, p.edge_na);
      const int ip = clamp_index_d(floor(h.afrac * static_cast<double>(np)), np);
      if (q.left == 0u) q.refill(k0, k1);
      h.ring = q.uniform() < p.edge_a[ia * np + ip] ? h.r_lo : h.r_hi;
    }
    ++n;
  }
  return n;
}

// Pair i of the buffer: where both singles fall (crystals, rings, gaps), the
// gap policy, ring difference and radial acceptance, TOF bin with jitter, LUT
// weight, sinogram update (and record and counters in the instrumented
// form).  kGaps: the gap model is compiled in (it is used when p.gap_on);
// without it the plain cylinder's evaluation keeps fewer registers.
template <bool kInstr, bool kGaps>
__device__ __forceinline__ void evaluate_pair(const TransportParams& p, const uint32_t* pairs, uint64_t i,
                                              unsigned long long* s_stats) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t k0 = static_cast<uint32_t>(p.seed), k1 = static_cast<uint32_t>(p.seed >> 32);
  const uint4* rec4 = reinterpret_cast<const uint4*>(pairs + i * kPairWords);
  const uint4 q0 = rec4[0];
  if (q0.w == kEmptyPair) return;
  const uint4 q1 = rec4[1], q2 = rec4[2], q3 = rec4[3], q4 = rec4[4];
  const uint32_t words[kPairWords] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y,
                                      q2.z, q2.w, q3.x, q3.y, q3.z, q3.w, q4.x, q4.y, q4.z, q4.w};
  auto F = [&](int w) -> float { return __uint_as_float(words[w]); };
  {
    const uint64_t hh = static_cast<uint64_t>(words[kPhLo]) | (static_cast<uint64_t>(words[kPhHi]) << 32);
    const uint32_t pos = words[kPPos], flags = words[kPFlags];
    const bool scattered = (flags & 0x100u) != 0u;
    Hit ha, hb;
    if (kGaps) {
      locate(p, F(kPA + kSX), F(kPA + kSY), F(kPA + kSZ), ha);
      locate(p, F(kPB + kSX), F(kPB + kSY), F(kPB + kSZ), hb);
    } else {
      locate_plain(p, F(kPA + kSX), F(kPA + kSY), F(kPA + kSZ), ha);
      locate_plain(p, F(kPB + kSX), F(kPB + kSY), F(kPB + kSZ), hb);
    }
    double ta_t, ta_a, tb_t, tb_a;
    incidence(F(kPA + kSX), F(kPA + kSY), F(kPA + kSDx), F(kPA + kSDy), F(kPA + kSDz), ta_t, ta_a);
    incidence(F(kPB + kSX), F(kPB + kSY), F(kPB + kSDx), F(kPB + kSDy), F(kPB + kSDz), tb_t, tb_a);
    const bool any_gap = kGaps && (ha.tgap || ha.agap || hb.tgap || hb.agap);
    // the history's stream where photon B left it (word pos), for the edge
    // draws and the TOF jitter
    RegRng q;
    const bool qon = p.tof_sigma > 0.0f || (kGaps && p.gap_on && p.gap_policy == kGapEdgeLut && any_gap);
    if (qon) {
      q.start(hh);
      q.blk = pos >> 2;
      q.refill(k0, k1);
      for (uint32_t j = 0; j < (pos & 3u); ++j) q.take();
    }
    bool gap_drop = false;
    int assigned = 0;
    if (kGaps && p.gap_on) {
      if (p.gap_policy == kGapDiscard) {
        gap_drop = any_gap;
      } else {
        // photon A's gaps first, then photon B's, before the jitter
        assigned = resolve_gap(p, q, ha, ta_t, ta_a);
        assigned += resolve_gap(p, q, hb, tb_t, tb_a);
      }
    }
    const int cA = ha.crystal, cB = hb.crystal, rA = ha.ring, rB = hb.ring;
    uint32_t outcome;
    uint64_t bin = ~0ull;
    float w = 0.0f, tau = 0.0f;
    if (gap_drop) {
      outcome = 8;
    } else if (cA == cB) {
      outcome = 4;
    } else if (p.max_ring_diff >= 0 && abs(rA - rB) > p.max_ring_diff) {
      outcome = 5;
    } else {
      const int nc = p.n_crystals;
      int k = cA + cB + 1;
      int rho = nc / 2 - abs(cA - cB);
      if (k >= nc) { k -= nc; rho = -rho; }
      const int view = k >> 1;
      int m = (2 * cA + 1 - k) % (2 * nc);
      if (m < 0) m += 2 * nc;
      const bool a_pos = m > 0 && m < nc;
      const int half = (p.n_rad - 1) / 2;
      if (abs(rho) > half) {
        outcome = 6;
      } else {
        const float apath = F(kPA + kSPath), bpath = F(kPB + kSPath);
        tau = a_pos ? (bpath - apath) * 0.5f : (apath - bpath) * 0.5f;
        if (p.tof_sigma > 0.0f) tau = tau + p.tof_sigma * std_normal(q, p);
        const float xt = tau / p.tof_bin + static_cast<float>(p.n_tof) * 0.5f;
        if (!(xt >= 0.0f) || !(xt < static_cast<float>(p.n_tof))) {
          outcome = 7;
        } else {
          const uint64_t tof = static_cast<uint64_t>(floorf(xt));
          const uint64_t plane = static_cast<uint64_t>(rA + rB);
          bin = ((tof * static_cast<uint64_t>(p.n_plane) + plane) * static_cast<uint64_t>(p.n_view) +
                 static_cast<uint64_t>(view)) * static_cast<uint64_t>(p.n_rad) +
                static_cast<uint64_t>(rho + half);
          // detection probabilities at the hit positions (a gap hit keeps its
          // virtual LUT index whatever edge crystal it went to)
          const uint32_t la = lut_index(p, static_cast<int>(words[kPA + kSEbin]), ta_t, ta_a, ha.ct, ha.ca);
          const uint32_t lb = lut_index(p, static_cast<int>(words[kPB + kSEbin]), tb_t, tb_a, hb.ct, hb.ca);
          w = lut_value(p, la) * lut_value(p, lb);
          if (scattered) {
            outcome = 0;
            atomicAdd(p.sc_n + bin, 1u);
            unsafeAtomicAdd(p.sc_w + bin, static_cast<double>(w));
          } else {
            outcome = 1;
            if (p.tr_n) atomicAdd(p.tr_n + bin, 1u);
            if (p.tr_w) unsafeAtomicAdd(p.tr_w + bin, static_cast<double>(w));
          }
        }
      }
    }
    // blocks the edge draws and the jitter add to those counted when photon B ended
    if (kInstr && p.stats && qon)
      atomicAdd(&s_stats[kStRngBlocks], blocks_used(q.blk * 4u - q.left) - blocks_used(pos));
    if (kInstr && p.stats && assigned)
      atomicAdd(&s_stats[kStGapAssigned], static_cast<unsigned long long>(assigned));
    SSE_COUNT(kStScatter, outcome == 0);
    SSE_COUNT(kStTrue, outcome == 1);
    SSE_COUNT(kStRejSame, outcome == 4);
    SSE_COUNT(kStRejRing, outcome == 5);
    SSE_COUNT(kStRejRadial, outcome == 6);
    SSE_COUNT(kStRejTof, outcome == 7);
    SSE_COUNT(kStRejGap, outcome == 8);
    if (kInstr && p.rec) {
      const uint64_t off = hh - p.rec_h0;
      if (off % p.rec_stride == 0) {
        uint32_t* rc = p.rec + (off / p.rec_stride) * kRecordWords;
        rc[0] = outcome | (scattered ? 0x100u : 0u);
        rc[1] = static_cast<uint32_t>(bin);
        rc[2] = static_cast<uint32_t>(bin >> 32);
        rc[4] = __float_as_uint(w);
        rc[5] = __float_as_uint(tau);
      }
    }
  }
}

// Emission of history hh into column `lane` of the queue eq: voxel from the
// alias table (64-bit multiply-shift column, 32-bit alias decision), uniform
// point in it, isotropic direction with cos(theta) = 1 - 2 u (exact) and
// azimuth 2 pi u'.  It takes exactly the eight words of Philox blocks 0 and 1
// of the history's stream, in that order.  Columns: position, direction,
// voxel, distances to the exit of the voxel box along +d (photon A) and -d
// (photon B: computed here, with all lanes active, rather than when photon A
// ends).
__device__ __forceinline__ void emit_to_queue(const TransportParams& p, uint64_t hh, LdsWord* eq) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t k0 = static_cast<uint32_t>(p.seed), k1 = static_cast<uint32_t>(p.seed >> 32);
  const uint32_t hlo = static_cast<uint32_t>(hh), hhi = static_cast<uint32_t>(hh >> 32);
  uint32_t a0, a1, a2, a3, b0, b1, b2, b3;
  uint32_t q0 = k0, q1 = k1;
  wave_uniform_key(q0, q1);
  philox(0u, hlo, hhi, 0u, q0, q1, a0, a1, a2, a3);
  philox(1u, hlo, hhi, 0u, q0, q1, b0, b1, b2, b3);
  const uint64_t col = __umul64hi((static_cast<uint64_t>(a1) << 32) | a0, p.nvox);
  const uint2 al = p.alias[col];
  const uint32_t v = (a2 < al.x) ? static_cast<uint32_t>(col) : al.y;
  const uint32_t nx = static_cast<uint32_t>(p.nx), ny = static_cast<uint32_t>(p.ny);
  uint32_t ix, iy, iz;
  if (p.nvox < (1ull << 24)) {
    const uint32_t q = udiv24(v, nx, p.inv_nx);
    iz = udiv24(v, nx * ny, p.inv_nxy);
    ix = v - q * nx;
    iy = q - iz * ny;
  } else {
    ix = v % nx;
    iy = (v / nx) % ny;
    iz = v / (nx * ny);
  }
  const float ex = p.lox + (static_cast<float>(ix) + to_uniform(a3)) * p.vx;
  const float ey = p.loy + (static_cast<float>(iy) + to_uniform(b0)) * p.vy;
  const float ez = p.loz + (static_cast<float>(iz) + to_uniform(b1)) * p.vz;
  const float cz = 1.0f - 2.0f * to_uniform(b2);
  const float st = sqrtf((1.0f - cz) * (1.0f + cz));
  float sp, cp;
  sincos_2pi(to_uniform(b3), sp, cp);
  eq[lane] = __float_as_uint(ex);
  eq[64u + lane] = __float_as_uint(ey);
  eq[128u + lane] = __float_as_uint(ez);
  eq[192u + lane] = __float_as_uint(st * cp);
  eq[256u + lane] = __float_as_uint(st * sp);
  eq[320u + lane] = __float_as_uint(cz);
  eq[384u + lane] = v;
  eq[448u + lane] = __float_as_uint(box_exit(p, ex, ey, ez, st * cp, st * sp, cz));
  eq[512u + lane] = __float_as_uint(box_exit(p, ex, ey, ez, -(st * cp), -(st * sp), -cz));
}

// Columns of the emission queue.
constexpr int kEmitWords = 9;

// Mark records [from, to) of the wavefront's block empty (converged call).
__device__ __forceinline__ void pad_pairs(const TransportParams& p, uint64_t from, uint64_t to) {
  for (uint64_t k = from + (threadIdx.x & 63u); k < to; k += 64u)
    if (k < p.pair_cap) p.pairs[k * kPairWords + kPFlags] = kEmptyPair;
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
// kInstr = true: the instrumented instantiation (statistics counters and
// per-history records); false: the production path, with neither.
// Simulate histories [next, end) of one wavefront.  mu_tab is the palette
// (in LDS) when p.mu8 is set; s_stats the block's statistics counters (used
// only when kInstr); stash the wavefront's LDS area for photon A's hit data
// (kSingleWords columns of 64 lanes); eq its emission queue (kEmitWords
// columns).  With kExtends, more(next, end), called converged whenever the
// range is used up, may give the wavefront a further range of histories
// with the same parameters (the lanes then go on without draining); it
// leaves next >= end when there is none.
// The palette pointer is typed as LDS so that its reads are LDS reads even
// where the compiler merges them with the binary32-map path.
typedef const __attribute__((address_space(3))) float LdsFloat;

// The range of a single-stream launch: nothing beyond [next, end).
struct NoMore {
  __device__ void operator()(uint64_t&, uint64_t&) const {}
};

template <bool kInstr, bool kExtends, class More>
__device__ __forceinline__ void run_histories(const TransportParams& p, uint64_t next, uint64_t end,
                                              unsigned long long* s_stats, LdsFloat* mu_tab,
                                              LdsWord* stash, LdsWord* rng_buf, LdsWord* eq, LdsLogRow* log_rows,
                                              uint64_t& res_next, uint64_t& res_end, More&& more) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t k0 = static_cast<uint32_t>(p.seed), k1 = static_cast<uint32_t>(p.seed >> 32);
  const uint64_t below = (1ull << lane) - 1ull;

  int phase = kEmit;
  int side = 0;                       // 0 photon A, 1 photon B
  uint64_t h = 0;
  uint32_t* rec = nullptr;            // this history's record, if sampled
  float ex = 0.f, ey = 0.f, ez = 0.f, edx = 0.f, edy = 0.f, edz = 0.f;  // emission point, direction of A
  float texit_b = 0.f;                // distance to the voxel box's exit along -d
  // photon A summary (its in-window hit data wait in the stash)
  uint32_t a_steps = 0;
  bool a_det = false, a_win = false, a_scat = false;
  bool pushed = false;                // this lane appended a pair in this iteration
  // photon state
  float px = 0.f, py = 0.f, pz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f, t = 0.f, texit = 0.f, len = 0.f;
  ECoef ec = p.e511;
  int nC = 0, nR = 0, nint = 0, fate = kEscaped;
  uint32_t steps = 0;
  int tries = 0;                      // of the rejection sampling in progress
  float ct = 1.0f;                    // cosine of the scattering angle, until the azimuth is drawn
  LaneRng r;
  r.col = rng_buf + lane;
  r.start(0);
  // emission queue (wave-uniform): entries for histories qbase .. qbase +
  // qn - 1 in eq, the next unused at qhead; qnext the next history to queue
  uint64_t qnext = next, qbase = next;
  uint32_t qn = 0, qhead = 0;

  // Start history qbase + k from queue entry k: photon A at the emission
  // point; its stream goes on at block 2 (the emission used blocks 0 and 1).
  auto take_emission = [&](uint32_t k) {
    h = qbase + k;
    ex = __uint_as_float(eq[k]);
    ey = __uint_as_float(eq[64u + k]);
    ez = __uint_as_float(eq[128u + k]);
    edx = __uint_as_float(eq[192u + k]);
    edy = __uint_as_float(eq[256u + k]);
    edz = __uint_as_float(eq[320u + k]);
    r.start(h);
    r.seek_block(2u);
    rec = nullptr;
    if (kInstr && p.rec) {
      const uint64_t off = h - p.rec_h0;
      if (off % p.rec_stride == 0) {
        rec = p.rec + (off / p.rec_stride) * kRecordWords;
        rec[3] = eq[384u + k];
      }
    }
    side = 0;
    px = ex; py = ey; pz = ez;
    dx = edx; dy = edy; dz = edz;
    t = 0.0f; len = 0.0f;
    texit = __uint_as_float(eq[448u + k]);
    texit_b = __uint_as_float(eq[512u + k]);
    ec = p.e511;
    nC = nR = nint = 0;
    steps = 0;
    fate = kEscaped;
    phase = kTrack;
  };


  for (;;) {
    // ---------------- take new histories ---------------------------------
    // Lanes that need a history take the next emission of the wavefront's
    // queue; when it runs out, all lanes refill it together (every history's
    // emission is computed by one lane of a converged wave) and the remaining
    // lanes take from the new entries.
    const uint64_t needmask = __ballot(phase == kEmit);
    if (needmask) {
      const uint32_t want = static_cast<uint32_t>(__popcll(needmask));
      const uint32_t rank = static_cast<uint32_t>(__popcll(needmask & below));
      const uint32_t got = want < qn - qhead ? want : qn - qhead;
      if (phase == kEmit && rank < got) take_emission(qhead + rank);
      qhead += got;
      if (want > got && !kExtends) {
        if (qnext < end) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          emit_to_queue(p, qnext + lane, eq);
          qbase = qnext;
          qn = end - qnext < 64u ? static_cast<uint32_t>(end - qnext) : 64u;
          qnext += qn;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (phase == kEmit && rank >= got && rank - got < qn) take_emission(rank - got);
          qhead = want - got < qn ? want - got : qn;
        }
        if (phase == kEmit) phase = kDone;  // no history left for this lane
      } else if (want > got) {
        // Refill rounds, extending the range, until every waiting lane has a
        // history or none is left (each round serves at least one lane, or
        // ends the loop).
        uint32_t given = got;
        for (;;) {
          if (qnext >= end) more(qnext, end);
          if (qnext >= end) break;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          emit_to_queue(p, qnext + lane, eq);
          qbase = qnext;
          qn = end - qnext < 64u ? static_cast<uint32_t>(end - qnext) : 64u;
          qnext += qn;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const uint32_t take = want - given < qn ? want - given : qn;
          if (phase == kEmit && rank >= given && rank - given < take) take_emission(rank - given);
          qhead = take;
          given += take;
          if (given == want) break;
        }
        if (phase == kEmit) phase = kDone;  // no history left for this lane
      }
    }
    if (wave_all(phase == kDone)) break;
    // Converged top-up: two rounds in which every live lane with room
    // generates a block (a new history gets eight words, the whole buffer).
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (wave_any(phase != kDone, r.room())) {
        if (phase != kDone && r.room()) r.refill(k0, k1);
      }
    }

    // ---------------- Woodcock steps until most lanes have an event --------
    // The step is cheap; the expensive branches below (interaction, photon
    // end, emission) then run once per outer iteration for all lanes that
    // need them, instead of once per step.  The loop stops when at most
    // kStepTail lanes are still stepping (they go on in the next iteration)
    // rather than waiting for the longest run of steps in the wave -- unless
    // no lane has anything else to do.
    // The test is one wave-uniform flag, computed before the loop and at the
    // end of each step: with the condition at the loop's head the compiler
    // kept two copies of the photon state and moved eleven registers per step.
    auto keep_stepping = [&]() -> bool {
      const uint64_t trk_m = __ballot(phase == kTrack);
      if (!trk_m) return false;
      return __popcll(trk_m) > kStepTail || !wave_any(phase != kTrack, phase != kDone);
    };
    bool stepping = keep_stepping();
    while (stepping) {
      if (wave_any(phase == kTrack, r.left < 2u)) {
        if (phase != kDone && r.room()) r.refill(k0, k1);
      }
      // One tentative step per tracking lane, written with selects rather
      // than branches (a masked lane costs the same issue slot): the step's
      // two words are read ahead and consumed only as far as the step uses
      // them -- the distance word when it steps, the acceptance word when the
      // point is inside the voxel box.
      const bool trk = phase == kTrack;
      const bool go = trk && steps < static_cast<uint32_t>(kMaxSteps);
      const uint32_t x0 = r.peek(0u), x1 = r.peek(1u);
      const float tn = t + free_path_log32(to_uniform(x0), log_rows) * ec.inv_maj;
      const bool inside = go && tn < texit;
      const float qx = px + tn * dx;
      const float qy = py + tn * dy;
      const float qz = pz + tn * dz;
      const uint32_t vox = voxel_at(p, qx, qy, qz);  // clamped: a valid index for every lane
      float mu = 0.0f;
      if (inside) {
        if (p.mu8) mu = mu_tab[p.mu8[vox]];
        else mu = p.mu[vox];
      }
      const bool real = inside && to_uniform(x1) * p.mu_maj < mu;
      SSE_COUNT(kStSteps, go);
      SSE_COUNT(kStReal, real);
      r.advance((go ? 1u : 0u) + (inside ? 1u : 0u));
      steps += go ? 1u : 0u;
      fate = (trk && !go) ? static_cast<int>(kCapped) : fate;
      // capped or out of the voxel box: to the cylinder; real: interaction
      phase = trk ? (real ? kInteract : (inside ? kTrack : kFinish)) : phase;
      // the distance along d from the last interaction point; a real
      // interaction moves the point there (and adds the distance to the
      // path) in the interaction section, for its lanes only, with the same
      // products and sums as q: four selects per step fewer
      t = go ? tn : t;
      stepping = keep_stepping();
    }

    // ---------------- real interactions ----------------------------------
    if (phase == kInteract) {
      len = len + t;
      px = px + t * dx;
      py = py + t * dy;
      pz = pz + t * dz;
      t = 0.0f;
      if (++nint > p.max_int) {
        fate = kCapped;
        phase = kFinish;
      } else {
        RNG_NEED(4u);
        const float ug = r.uniform() * ec.g;
        tries = 0;
        if (ug < ec.cC) {
          phase = kCompton;
        } else if (ug < ec.cCR) {
          // Rayleigh: form factor by inversion, Thomson factor by rejection
          const float bp = p.rayleigh_beta * (ec.alpha * ec.alpha);
          const float cc = (2.0f * bp) / (1.0f + 2.0f * bp);
          bool ok = false;
          for (int i = 0; i < kMaxTries && !ok; ++i) {
            RNG_NEED(2u);
            const float r1 = r.uniform();
            const float r2 = r.uniform();
            const float q = r1 * cc;
            const float tq = q / ((1.0f - q) * bp);
            float c = 1.0f - tq;
            if (c < -1.0f) c = -1.0f;
            if (2.0f * r2 <= 1.0f + c * c) { ct = c; ok = true; }
          }
          if (!ok) {
            fate = kAbsorbed;
            phase = kFinish;
          } else {
            SSE_COUNT(kStRayleigh, true);
            ++nR;
            phase = kAzimuth;
          }
        } else {
          fate = kAbsorbed;
          phase = kFinish;
        }
      }
    }

    // ---------------- Compton: Klein-Nishina by Kahn's method --------------
    // x = E / E'; at most kMaxTries tries in all, kRounds per iteration.
    if (wave_any(phase == kCompton)) {
      bool acc = false;
      float x = 0.0f;
      for (int k = 0; k < kRounds; ++k) {
        if (!wave_any(phase == kCompton, !acc)) break;
        if (phase == kCompton && !acc) {
          if (tries >= kMaxTries) {
            fate = kAbsorbed;
            phase = kFinish;
          } else {
            ++tries;
            RNG_NEED(3u);
            const float twoa = 2.0f * ec.alpha;
            const float b1 = 1.0f + twoa;
            const float b2 = 9.0f + twoa;
            const float r1 = r.uniform();
            const float r2 = r.uniform();
            const float r3 = r.uniform();
            if (r1 * b2 <= b1) {
              const float xx = 1.0f + twoa * r2;
              if (r3 * (xx * xx) <= 4.0f * (xx - 1.0f)) { x = xx; acc = true; }
            } else {
              const float xx = fdiv(b1, 1.0f + twoa * r2);
              const float c = 1.0f + fdiv(1.0f - xx, ec.alpha);
              if (2.0f * r3 <= c * c + fdiv(1.0f, xx)) { x = xx; acc = true; }
            }
          }
        }
      }
      if (acc) {
        SSE_COUNT(kStCompton, true);
        const float e2 = fdiv(ec.E, x);
        ct = 1.0f - fdiv(x - 1.0f, ec.alpha);
        ct = fminf(fmaxf(ct, -1.0f), 1.0f);
        ++nC;
        if (e2 < p.e_kill) {
          fate = kKilled;
          phase = kFinish;
        } else {
          energy_coefficients<DevDiv>(ec, e2, p.kc, p.f_r, p.f_p, p.mu_maj);
          tries = 0;
          phase = kAzimuth;
        }
      }
    }

    // ---------------- azimuth, new direction -----------------------------
    if (phase == kAzimuth) {
      RNG_NEED(1u);
      float sp, cp;
      sincos_2pi(r.uniform(), sp, cp);
      rotate(dx, dy, dz, ct, cp, sp);
      texit = box_exit(p, px, py, pz, dx, dy, dz);
      phase = kTrack;
    }

    // ---------------- pair-buffer room (converged) ------------------------
    // Room in the wavefront's block for every lane whose photon B may end a
    // pair below; otherwise the rest of the block is padded and the next
    // block reserved.  res_next and res_end change only here and at the end
    // of the iteration, so they stay wave-uniform.
    {
      const uint64_t need = static_cast<uint64_t>(__popcll(__builtin_amdgcn_ballot_w64(phase == kFinish) &
                                                            __builtin_amdgcn_ballot_w64(side == 1) &
                                                            __builtin_amdgcn_ballot_w64(a_win)));
      if (res_end - res_next < need) {
        pad_pairs(p, res_next, res_end);
        uint32_t b0 = 0u;
        if (lane == 0u) b0 = atomicAdd(p.pair_count, kPairBlock);
        res_next = static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(b0))));
        res_end = res_next + kPairBlock;
      }
    }

    // ---------------- photon finished ------------------------------------
    if (phase == kFinish) {
      float hx = 0.0f, hy = 0.0f, hz = 0.0f, path = 0.0f, edet = ec.E;
      if (fate == kEscaped) {
        // crossing of x^2 + y^2 = R^2 ahead of the last point
        const float a = dx * dx + dy * dy;
        fate = kAxial;
        if (a > 0.0f) {
          const float b = px * dx + py * dy;
          const float c = px * px + py * py - p.rr;
          const float disc = b * b - a * c;
          const float sq = sqrtf(disc);
          // c < 0 (the voxel box lies inside the cylinder), a > 0: a positive quotient
          const float tc = (b > 0.0f) ? fdiv(-c, b + sq) : fdiv(sq - b, a);
          const float zz = pz + tc * dz;
          if (zz >= -p.half_len && zz < p.half_len) {
            fate = kDetected;
            hx = px + tc * dx;
            hy = py + tc * dy;
            hz = zz;
            path = len + tc;
            if (p.e_fwhm > 0.0f) {
              const float nrm = std_normal(r, p);
              const float sig = (p.e_fwhm / 2.35482f) * sqrtf(kMec2 / ec.E);
              edet = ec.E * (1.0f + sig * nrm);
            }
          }
        }
        SSE_COUNT(kStEscaped, true);
        SSE_COUNT(kStDetected, fate == kDetected);
      } else {
        SSE_COUNT(kStAbsorbed, fate == kAbsorbed);
        SSE_COUNT(kStKilled, fate == kKilled);
        SSE_COUNT(kStCapped, fate == kCapped);
      }
      const bool det = fate == kDetected;
      const bool win = det && edet >= p.e_lo && edet <= p.e_hi;
      SSE_COUNT(kStInWindow, win);
      if (kInstr && rec) {
        uint32_t cr = 0xffffffffu, lidx = 0xffffffffu;
        if (win) index_single(p, hx, hy, hz, dx, dy, dz, ec.E, cr, lidx);
        uint32_t* w = rec + 8 + 12 * side;
        w[0] = __float_as_uint(hx); w[1] = __float_as_uint(hy); w[2] = __float_as_uint(hz);
        w[3] = __float_as_uint(dx); w[4] = __float_as_uint(dy); w[5] = __float_as_uint(dz);
        w[6] = __float_as_uint(ec.E); w[7] = __float_as_uint(edet); w[8] = __float_as_uint(path);
        w[9] = cr;
        w[10] = lidx;
        w[11] = static_cast<uint32_t>(nC) | (static_cast<uint32_t>(nR) << 8) | (static_cast<uint32_t>(fate) << 16);
      }
      // the LUT energy bin of an in-window single
      const uint32_t ebin = win ? static_cast<uint32_t>(energy_bin(p, ec.E)) : 0u;
      if (side == 0) {
        a_det = det;
        a_win = win;
        a_scat = (nC + nR) > 0;
        a_steps = steps;
        if (win) {
          stash[64u * kSX + lane] = __float_as_uint(hx);
          stash[64u * kSY + lane] = __float_as_uint(hy);
          stash[64u * kSZ + lane] = __float_as_uint(hz);
          stash[64u * kSDx + lane] = __float_as_uint(dx);
          stash[64u * kSDy + lane] = __float_as_uint(dy);
          stash[64u * kSDz + lane] = __float_as_uint(dz);
          stash[64u * kSPath + lane] = __float_as_uint(path);
          stash[64u * kSEbin + lane] = ebin;
        }
        if (!kInstr && p.prune_b && !win) {
          // Photon A ended outside the energy window: the history adds to
          // no sinogram whatever photon B does, so with pruning on B is not
          // tracked and the lane takes the next history.  (The instrumented
          // instantiation, whose statistics and records describe photon B,
          // always tracks it.)
          phase = kEmit;
        } else {
          // photon B: back to back with A
          side = 1;
          px = ex; py = ey; pz = ez;
          dx = -edx; dy = -edy; dz = -edz;
          t = 0.0f; len = 0.0f;
          texit = texit_b;
          ec = p.e511;
          nC = nR = nint = 0;
          steps = 0;
          fate = kEscaped;
          phase = kTrack;
        }
      } else {
        // ---------------- coincidence -------------------------------------
        // Not both detected (outcome 2) or not both in the window (3) is
        // decided here; pairs in the window go to the queue -- in the
        // production instantiation without a trues sinogram, only the
        // scattered ones (an unscattered pair would add to nothing, and each
        // pair draws its coincidence numbers from its own stream).
        const bool scattered = a_scat || (nC + nR) > 0;
        const bool both = a_win && win;
        const bool queued = both && (kInstr || scattered || p.tr_n != nullptr);
        const uint64_t bm = __ballot(queued);
        if (queued) {
          const uint64_t slot = res_next + static_cast<uint64_t>(__popcll(bm & below));
          if (slot < p.pair_cap) {  // always, by the launch size; a guard for the memory
            uint4* w = reinterpret_cast<uint4*>(p.pairs + slot * kPairWords);
            w[0] = make_uint4(static_cast<uint32_t>(h), static_cast<uint32_t>(h >> 32), r.blk * 4u - r.left,
                              (scattered ? 0x100u : 0u) | (p.item << 16));
            w[1] = make_uint4(stash[lane], stash[64u + lane], stash[128u + lane], stash[192u + lane]);
            w[2] = make_uint4(stash[256u + lane], stash[320u + lane], stash[384u + lane], stash[448u + lane]);
            w[3] = make_uint4(__float_as_uint(hx), __float_as_uint(hy), __float_as_uint(hz), __float_as_uint(dx));
            w[4] = make_uint4(__float_as_uint(dy), __float_as_uint(dz), __float_as_uint(path), ebin);
          }
        }
        pushed = queued;
        SSE_COUNT(kStHist, true);
        if (kInstr && p.stats) atomicAdd(&s_stats[kStRngBlocks], blocks_used(r.blk * 4u - r.left));
        SSE_COUNT(kStRejWindow, a_det && det && !both);
        if (kInstr && rec) {
          if (!both) {
            rec[0] = ((a_det && det) ? 3u : 2u) | (scattered ? 0x100u : 0u);
            rec[1] = 0xffffffffu;
            rec[2] = 0xffffffffu;
            rec[4] = 0u;
            rec[5] = 0u;
          }
          rec[6] = a_steps + steps;
          rec[7] = 0u;
        }
        phase = kEmit;
      }
    }
    res_next += static_cast<uint64_t>(__popcll(__ballot(pushed)));
    pushed = false;
  }
}

// kInstr = true: the instrumented instantiation (statistics counters and
// per-history records); false: the production path, with neither.  Every
// wavefront owns a contiguous share of [h0, h0 + n).
template <bool kInstr>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kInstr ? kInstrWavesPerEu : kTransportWavesPerEu)))
transport_kernel(TransportParams p) {
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  const uint64_t per = p.n / nwaves, rem = p.n % nwaves;
  const uint64_t begin = p.h0 + wave * per + (wave < rem ? wave : rem);
  const uint64_t end = begin + per + (wave < rem ? 1 : 0);
  __shared__ unsigned long long s_stats[kStatCount];
  __shared__ float s_mu_table[256];
  __shared__ uint32_t s_stash[4][kSingleWords * 64];
  __shared__ uint32_t s_rng[4][kRngSlots * 64];
  __shared__ uint32_t s_emit[4][kEmitWords * 64];
  __shared__ float4 s_log[kLogEntries];
  if (kInstr && threadIdx.x < kStatCount) s_stats[threadIdx.x] = 0;
  if (p.mu_table) s_mu_table[threadIdx.x] = p.mu_table[threadIdx.x];
  stage_log_rows(s_log);
  __syncthreads();
  uint64_t res_next = 0, res_end = 0;
  run_histories<kInstr, false>(p, begin, end, s_stats, (LdsFloat*)(s_mu_table), (LdsWord*)(s_stash[threadIdx.x >> 6]),
                               (LdsWord*)(s_rng[threadIdx.x >> 6]), (LdsWord*)(s_emit[threadIdx.x >> 6]),
                               (LdsLogRow*)(s_log), res_next, res_end, NoMore{});
  pad_pairs(p, res_next, res_end);
  if (kInstr) {
    __syncthreads();
    if (p.stats && threadIdx.x < kStatCount && s_stats[threadIdx.x])
      atomicAdd(p.stats + threadIdx.x, s_stats[threadIdx.x]);
  }
}

typedef const __attribute__((address_space(4))) WorkChunk ConstChunk;
typedef const __attribute__((address_space(4))) TransportParams ConstParams;

// Work-list form: the request server's launches, and the production path of
// a simulate call (one request, one chunk per launch).  The launch's chunks
// (request, history range) are laid end to end, each padded to a multiple
// of kBatchSlice, and wavefronts claim slices of kBatchSlice positions from
// a device cursor until it passes the end; a slice lies in one chunk, so it
// carries that request's parameters.  A wavefront whose range runs out
// claims the next slice at once: one of the same request extends the range
// and the lanes go on without draining; one of another request waits until
// the lanes have finished (the parameters are wave-uniform).  The small
// slices balance the launch's end, at one drain per request change.  The
// palette table is per wavefront because neighbouring wavefronts may work
// on different requests.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kTransportWavesPerEu)))
transport_batch_kernel(BatchParams b) {
  __shared__ float s_tab[4][256];
  __shared__ uint32_t s_stash[4][kSingleWords * 64];
  __shared__ uint32_t s_rng[4][kRngSlots * 64];
  __shared__ uint32_t s_emit[4][kEmitWords * 64];
  __shared__ float4 s_log[kLogEntries];
  stage_log_rows(s_log);
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u;
  float* tab = s_tab[threadIdx.x >> 6];
  uint64_t res_next = 0, res_end = 0;  // the wavefront's pair-buffer block, kept across chunks
  const TransportParams* last = nullptr;
  // The next slice (converged call): its request and histories in ch;
  // false once the cursor has passed the end.  Positions only grow for one
  // wavefront, so the chunk it falls in is found by walking forward from
  // the last one (ci, starting at position cstart).
  uint32_t ci = 0;
  uint64_t cstart = 0;
  // The list and the requests' parameters are read through the constant
  // address space (they are written before the launch, by the host or by an
  // earlier kernel on the stream) with wave-uniform indices, so that their
  // loads are scalar loads the compiler may keep or repeat; through generic
  // pointers they would be vector loads inside the transport loop.
  const ConstChunk* chunks = (const ConstChunk*)(b.chunks);
  const ConstParams* items = (const ConstParams*)(b.items);
  auto claim = [&](WorkChunk& ch) -> bool {
    uint32_t pos = 0;
    if (lane == 0) {
      // A fill launch stops claiming once the buffer holds what every
      // resident wavefront may still add to it, or once the end flag is set:
      // in the empty launches that follow a fill run, every wavefront's
      // atomic add on the one cursor would serialise.  (The flag is read
      // rather than the cursor, whose line the atomic adds keep busy; both
      // words are read at device scope, past this CU's cache.)
      bool stop = false;
      if (b.done) {  // a fill launch (both words are loaded before either is tested)
        const uint32_t done = __hip_atomic_load(b.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t count = __hip_atomic_load(b.pair_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        stop = done != 0u || static_cast<uint64_t>(count) > b.stop_at;
      }
      pos = stop ? 0xffffffffu : atomicAdd(b.counter, kBatchSlice);
      if (b.done && !stop && pos >= b.n_positions)
        __hip_atomic_store(b.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    pos = __builtin_amdgcn_readfirstlane(__shfl(pos, 0, 64));
    if (pos >= b.n_positions) return false;
    for (;;) {
      if (ci >= b.n_chunks) return false;  // only if n_positions overstates the list
      const uint64_t len = (static_cast<uint64_t>(chunks[ci].n) + kBatchSlice - 1) / kBatchSlice * kBatchSlice;
      if (pos < cstart + len) break;
      cstart += len;
      ++ci;
    }
    const WorkChunk c = {chunks[ci].h0, chunks[ci].n, chunks[ci].item};
    const uint64_t off = pos - cstart;  // a multiple of kBatchSlice below c.n
    ch.item = c.item;
    ch.h0 = c.h0 + off;
    ch.n = static_cast<uint32_t>(c.n - off < kBatchSlice ? c.n - off : kBatchSlice);
    return true;
  };
  WorkChunk cur;
  bool have = claim(cur);
  while (have) {
    const TransportParams& p = *(const TransportParams*)(items + __builtin_amdgcn_readfirstlane(cur.item));
    if (p.mu8) {
      for (uint32_t i = lane; i < 256u; i += 64u) tab[i] = p.mu_table[i];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    WorkChunk held;
    bool holding = false, used_up = false;
    auto more = [&](uint64_t& next, uint64_t& end) {
      if (holding || used_up) return;
      WorkChunk ch;
      if (!claim(ch)) {
        used_up = true;
      } else if (ch.item == cur.item) {
        next = ch.h0;
        end = ch.h0 + ch.n;
      } else {
        held = ch;
        holding = true;
      }
    };
    run_histories<false, true>(p, cur.h0, cur.h0 + cur.n, nullptr, (LdsFloat*)(tab),
                               (LdsWord*)(s_stash[threadIdx.x >> 6]), (LdsWord*)(s_rng[threadIdx.x >> 6]),
                               (LdsWord*)(s_emit[threadIdx.x >> 6]), (LdsLogRow*)(s_log), res_next, res_end, more);
    last = &p;
    __builtin_amdgcn_wave_barrier();
    have = holding;
    if (holding) cur = held;
  }
  if (last) pad_pairs(*last, res_next, res_end);
}

// The records the last transport launch reserved, one per thread (padding
// records are skipped).
template <bool kInstr, bool kGaps>
__global__ void __launch_bounds__(256) coincidence_kernel(TransportParams p) {
  __shared__ unsigned long long s_stats[kStatCount];
  if (kInstr && threadIdx.x < kStatCount) s_stats[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t count = *p.pair_count;
  const uint64_t n = count < p.pair_cap ? count : p.pair_cap;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    evaluate_pair<kInstr, kGaps>(p, p.pairs, i, s_stats);
  if (kInstr) {
    __syncthreads();
    if (p.stats && threadIdx.x < kStatCount && s_stats[threadIdx.x])
      atomicAdd(p.stats + threadIdx.x, s_stats[threadIdx.x]);
  }
}

// Work-list form: each pair carries its request slot.
template <bool kGaps>
__global__ void __launch_bounds__(256) coincidence_batch_kernel(BatchParams b) {
  const uint64_t count = *b.pair_count;
  const uint64_t n = count < b.pair_cap ? count : b.pair_cap;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t flags = b.pairs[i * kPairWords + kPFlags];
    if (flags == kEmptyPair) continue;
    evaluate_pair<false, kGaps>(b.items[flags >> 16], b.pairs, i, nullptr);
  }
}

__global__ void reset_counter_kernel(uint32_t* c) { *c = 0u; }

// One request's parameters and one chunk, stored where the work-list
// kernels read them by a single thread, so that the store is ordered on the
// stream with the launches that read it (and with earlier ones still
// reading the previous values).
__global__ void store_item_kernel(TransportParams p, WorkChunk c, TransportParams* item, WorkChunk* chunk) {
  *item = p;
  *chunk = c;
}

// Check of DevDiv against the IEEE operator: the refined reciprocal of every
// significand in [1, 2) (counts[0]: differences from 1 / b), then n quotients
// of operands with hashed significands and exponents in [-20, 20]
// (counts[1]: differences from a / b).
__device__ __forceinline__ uint32_t check_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ void __launch_bounds__(256) check_division_kernel(uint64_t n, uint32_t seed,
                                                             unsigned long long* counts) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  const uint64_t t0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  unsigned long long bad_r = 0, bad_q = 0;
  for (uint64_t m = t0; m < (1ull << 23); m += stride) {
    const float b = __uint_as_float(0x3f800000u | static_cast<uint32_t>(m));
    const float y0 = __builtin_amdgcn_rcpf(b);
    const float y = __builtin_fmaf(__builtin_fmaf(-b, y0, 1.0f), y0, y0);
    bad_r += __float_as_uint(y) != __float_as_uint(1.0f / b) ? 1u : 0u;
  }
  for (uint64_t i = t0; i < n; i += stride) {
    const uint32_t h1 = check_hash(static_cast<uint32_t>(i) ^ check_hash(static_cast<uint32_t>(i >> 32) + seed));
    const uint32_t h2 = check_hash(h1 ^ 0x85ebca6bu);
    const uint32_t h3 = check_hash(h2 ^ 0xc2b2ae35u);
    const int ea = static_cast<int>(h3 % 41u) - 20;
    const int eb = static_cast<int>((h3 >> 16) % 41u) - 20;
    const float a = ldexpf(__uint_as_float(0x3f800000u | (h1 >> 9)), ea);
    const float b = ldexpf(__uint_as_float(0x3f800000u | (h2 >> 9)), eb);
    bad_q += __float_as_uint(DevDiv::div(a, b)) != __float_as_uint(a / b) ? 1u : 0u;
  }
  if (bad_r) atomicAdd(counts, bad_r);
  if (bad_q) atomicAdd(counts + 1, bad_q);
}

hipError_t device_info(int& cus) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return e;
}

// Blocks for a grid-stride pass over at most `items` items.
int stride_grid(uint64_t items, int cus) {
  const uint64_t want = (items + 255) / 256;
  const uint64_t most = static_cast<uint64_t>(cus) * 8u;
  return static_cast<int>(want < most ? (want > 0 ? want : 1) : most);
}

constexpr int kBlock = 256;

// Resident blocks of a transport kernel on the whole device.
template <class K>
uint64_t resident_blocks(K kernel) {
  int cus = 0, per_cu = 0;
  if (device_info(cus) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess) return 0;
  return static_cast<uint64_t>(cus) * static_cast<uint64_t>(per_cu > 0 ? per_cu : 1);
}

uint64_t transport_resident_waves() {
  const uint64_t a = resident_blocks(transport_kernel<true>), b = resident_blocks(transport_kernel<false>);
  return (a > b ? a : b) * (kBlock / 64);
}

// Wavefronts a launch of n histories runs with.
uint64_t waves_for(uint64_t n, uint64_t resident_waves) {
  const uint64_t want = ((n + kBlock - 1) / kBlock) * (kBlock / 64);
  return want < resident_waves ? want : resident_waves;
}

// Largest n with pair_records_needed(n, waves(n)) <= cap.
template <class W>
uint64_t max_histories(uint64_t cap, W waves) {
  uint64_t lo = 0, hi = cap;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (pair_records_needed(mid, waves(mid)) <= cap) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <bool kInstr>
hipError_t launch(const TransportParams& p, hipStream_t stream) {
  int cus = 0;
  hipError_t e = device_info(cus);
  if (e != hipSuccess) return e;
  const uint64_t resident = resident_blocks(transport_kernel<kInstr>);
  if (resident == 0) return hipErrorInvalidDeviceFunction;
  // one resident wave per 64 histories at most: small runs use fewer blocks
  const uint64_t want = (p.n + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(want < resident ? want : resident);
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, p.pair_count);
  hipLaunchKernelGGL(transport_kernel<kInstr>, dim3(grid), dim3(kBlock), 0, stream, p);
  const dim3 cgrid(stride_grid(pair_records_needed(p.n, 4ull * grid), cus));
  if (p.gap_on)
    hipLaunchKernelGGL((coincidence_kernel<kInstr, true>), cgrid, dim3(kBlock), 0, stream, p);
  else
    hipLaunchKernelGGL((coincidence_kernel<kInstr, false>), cgrid, dim3(kBlock), 0, stream, p);
  return hipGetLastError();
}

}  // namespace

uint64_t transport_pairs_needed(uint64_t n) {
  return pair_records_needed(n, waves_for(n, transport_resident_waves()));
}

uint64_t transport_max_histories(uint64_t cap) {
  const uint64_t rw = transport_resident_waves();
  return max_histories(cap, [rw](uint64_t n) { return waves_for(n, rw); });
}

uint64_t transport_batch_pairs_needed(uint64_t n) {
  return pair_records_needed(n, resident_blocks(transport_batch_kernel) * (kBlock / 64));
}

uint64_t transport_batch_max_histories(uint64_t cap) {
  const uint64_t rw = resident_blocks(transport_batch_kernel) * (kBlock / 64);
  return max_histories(cap, [rw](uint64_t) { return rw; });  // chunks go to every resident wave
}

hipError_t launch_transport(const TransportParams& p, hipStream_t stream) {
  if (!p.pairs || !p.pair_count || p.pair_cap == 0 || p.pair_cap > kMaxPairCap) return hipErrorInvalidValue;
  const uint64_t most = transport_max_histories(p.pair_cap);
  if (most == 0) return hipErrorInvalidValue;
  for (uint64_t done = 0; done < p.n;) {
    TransportParams q = p;
    q.h0 = p.h0 + done;
    q.n = p.n - done < most ? p.n - done : most;
    const hipError_t e = (p.stats || p.rec) ? launch<true>(q, stream) : launch<false>(q, stream);
    if (e != hipSuccess) return e;
    done += q.n;
  }
  return hipSuccess;
}

namespace {
hipError_t launch_batch_pass(const BatchParams& b, hipStream_t stream, KernelTiming* kt, bool reset_cursor);
// Histories of one fill run: its claim positions fit 32 bits.
constexpr uint64_t kFillRun = 1ull << 31;
}  // namespace

hipError_t launch_transport_item(const TransportParams& p, TransportParams* d_item, WorkChunk* d_chunk,
                                 uint32_t* d_cursor, hipStream_t stream, KernelTiming* kt) {
  if (!p.pairs || !p.pair_count || p.pair_cap == 0 || p.pair_cap > kMaxPairCap || !d_item || !d_chunk || !d_cursor)
    return hipErrorInvalidValue;
  TransportParams q = p;
  q.item = 0;
  // Fill launches: the work list spans the whole run (up to kFillRun
  // histories) and each launch takes slices from the common cursor until
  // the pair buffer holds stop_at records -- in practice one launch, as a
  // pair is queued for a few per cent of histories -- and as many launches
  // are queued as the worst case (a pair for every history) needs; those
  // that find the cursor at the end exit at once.  After its last claim a
  // wavefront adds at most the pairs of its slice and of its lanes still in
  // flight (kBatchSlice + 64), with the padding of the blocks it leaves:
  // three blocks.
  const uint64_t rw = resident_blocks(transport_batch_kernel) * (kBlock / 64);
  const uint64_t headroom = rw * 3u * kPairBlock;
  const uint64_t stop_at = p.pair_cap > headroom ? p.pair_cap - headroom : 0;
  // Histories a launch takes at least before it stops: it stops with more
  // than stop_at records reserved, of which every block gave at most 63 to
  // padding and every wavefront at most a block to its unused tail, and a
  // history queues at most one pair.
  const uint64_t records_min = stop_at / kPairBlock * (kPairBlock - 63);
  const uint64_t per_launch = records_min > 2u * rw * kPairBlock ? records_min - rw * kPairBlock : 0;
  if (rw > 0 && per_launch > 0) {
    for (uint64_t done = 0; done < p.n;) {
      const uint64_t n = p.n - done < kFillRun ? p.n - done : kFillRun;
      const WorkChunk ch{p.h0 + done, static_cast<uint32_t>(n), 0u};
      hipLaunchKernelGGL(store_item_kernel, dim3(1), dim3(1), 0, stream, q, ch, d_item, d_chunk);
      hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, d_cursor);
      hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, d_cursor + kDoneOffsetWords);
      const uint64_t positions = (n + kBatchSlice - 1) / kBatchSlice * kBatchSlice;
      BatchParams b{d_item, d_chunk, 1u, static_cast<uint32_t>(positions), d_cursor, n,
                    p.pairs, p.pair_count, p.pair_cap, p.gap_on};
      b.stop_at = stop_at;
      b.done = d_cursor + kDoneOffsetWords;
      const uint64_t launches = (n + per_launch - 1) / per_launch;
      for (uint64_t k = 0; k < launches; ++k) {
        const hipError_t e = launch_batch_pass(b, stream, kt, false);
        if (e != hipSuccess) return e;
      }
      done += n;
    }
    return hipSuccess;
  }
  // a small buffer: launches sized for the worst case
  const uint64_t most = transport_batch_max_histories(p.pair_cap);
  if (most == 0) return hipErrorInvalidValue;
  for (uint64_t done = 0; done < p.n;) {
    const uint64_t n = p.n - done < most ? p.n - done : most;
    const WorkChunk ch{p.h0 + done, static_cast<uint32_t>(n), 0u};
    hipLaunchKernelGGL(store_item_kernel, dim3(1), dim3(1), 0, stream, q, ch, d_item, d_chunk);
    const uint64_t positions = (n + kBatchSlice - 1) / kBatchSlice * kBatchSlice;
    const BatchParams b{d_item, d_chunk, 1u, static_cast<uint32_t>(positions), d_cursor, n,
                        p.pairs, p.pair_count, p.pair_cap, p.gap_on};
    const hipError_t e = launch_transport_batch(b, stream, kt);
    if (e != hipSuccess) return e;
    done += n;
  }
  return hipSuccess;
}

hipError_t upload_log_table() {
  float4 rows[kLogEntries];
  for (int i = 0; i < kLogEntries; ++i) {
    float a, b;
    const uint32_t ba = kLogBase + (static_cast<uint32_t>(i) << 16), bb = kLogBase + (static_cast<uint32_t>(i + 1) << 16);
    std::memcpy(&a, &ba, sizeof a);
    std::memcpy(&b, &bb, sizeof b);
    const float c = (i >= 73 && i <= 77) ? 1.0f : static_cast<float>(1.0 / (0.5 * (static_cast<double>(a) + b)));
    const double t = -std::log(static_cast<double>(c));
    const double hi = std::nearbyint(t * 65536.0) / 65536.0;
    rows[i] = make_float4(c, static_cast<float>(hi), static_cast<float>(t - hi), 0.0f);
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(c_log_rows), rows, sizeof rows);
}

hipError_t launch_check_division(uint64_t n, uint32_t seed, unsigned long long* counts, hipStream_t stream) {
  int cus = 0;
  hipError_t e = device_info(cus);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(check_division_kernel, dim3(static_cast<unsigned>(cus) * 16u), dim3(kBlock), 0, stream, n,
                     seed, counts);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// allocation-free simulate
// ---------------------------------------------------------------------------
// The device scratch of sse_simulate_noalloc: one parameter set, one chunk,
// the claim cursor and the pair counter (each at a multiple of 256 bytes),
// then the pair buffer.  Each GPU the library runs on holds its own copy until the process
// ends; calls that use it on one GPU at the same time race (the library
// orders the calls of one context; calls of different contexts on one GPU
// are the caller's to order).
constexpr uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }
constexpr uint64_t kNoAllocChunkAt = align256(sizeof(TransportParams));
constexpr uint64_t kNoAllocCursorAt = kNoAllocChunkAt + align256(sizeof(WorkChunk));
constexpr uint64_t kNoAllocCountAt = kNoAllocCursorAt + 256;
static_assert(kNoAllocCountAt - kNoAllocCursorAt >= kCursorWords * sizeof(uint32_t), "cursor slot too small");
constexpr uint64_t kNoAllocHeader = kNoAllocCountAt + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

uint64_t noalloc_max_histories() {
  return transport_batch_max_histories((kNoAllocScratchBytes - kNoAllocHeader) / (kPairWords * sizeof(uint32_t)));
}

hipError_t launch_transport_noalloc(int device, const TransportParams& p0, hipStream_t stream) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (device >= 0 && device < kMaxDevices) base = g_scratch_ptr[device];
  }
  if (!base) return hipErrorNotInitialized;
  unsigned char* b = static_cast<unsigned char*>(base);
  TransportParams p = p0;
  TransportParams* d_item = reinterpret_cast<TransportParams*>(b);
  WorkChunk* d_chunk = reinterpret_cast<WorkChunk*>(b + kNoAllocChunkAt);
  uint32_t* d_cursor = reinterpret_cast<uint32_t*>(b + kNoAllocCursorAt);
  p.pair_count = reinterpret_cast<uint32_t*>(b + kNoAllocCountAt);
  p.pairs = reinterpret_cast<uint32_t*>(b + kNoAllocHeader);
  p.pair_cap = (kNoAllocScratchBytes - kNoAllocHeader) / (kPairWords * sizeof(uint32_t));
  return launch_transport_item(p, d_item, d_chunk, d_cursor, stream);
}

hipError_t launch_transport_batch(const BatchParams& b, hipStream_t stream, KernelTiming* kt) {
  if (b.n_chunks == 0) return hipSuccess;
  if (!b.pairs || !b.pair_count || b.pair_cap > kMaxPairCap || b.stop_at != ~0ull || b.done ||
      b.n_histories > transport_batch_max_histories(b.pair_cap))
    return hipErrorInvalidValue;
  return launch_batch_pass(b, stream, kt, true);
}

namespace {
// One pass of a work list: the claim cursor reset (reset_cursor) or left
// where the last pass stopped, the pair counter reset, the transport kernel,
// then the coincidence kernel over the records it queued.
hipError_t launch_batch_pass(const BatchParams& b, hipStream_t stream, KernelTiming* kt, bool reset_cursor) {
  if (b.n_positions < b.n_histories ||
      b.n_positions > b.n_histories + static_cast<uint64_t>(b.n_chunks) * kBatchSlice)
    return hipErrorInvalidValue;
  int cus = 0;
  hipError_t e = device_info(cus);
  if (e != hipSuccess) return e;
  const uint64_t resident = resident_blocks(transport_batch_kernel);
  if (resident == 0) return hipErrorInvalidDeviceFunction;
  const uint64_t want = (static_cast<uint64_t>(b.n_positions) / kBatchSlice + 3) / 4;  // a slice per wave at least
  const int grid = static_cast<int>(want < resident ? want : resident);
  hipEvent_t* ev = nullptr;
  if (kt && kt->ev) {
    if (kt->n < kt->cap) ev = kt->ev + 4u * kt->n++;
    else ++kt->dropped;
  }
  if (reset_cursor) hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, b.counter);
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, b.pair_count);
  if (ev) (void)hipEventRecord(ev[0], stream);
  hipLaunchKernelGGL(transport_batch_kernel, dim3(grid), dim3(kBlock), 0, stream, b);
  if (ev) (void)hipEventRecord(ev[1], stream);
  const uint64_t most_records = pair_records_needed(b.n_histories, 4ull * grid);
  const dim3 cgrid(stride_grid(most_records < b.pair_cap ? most_records : b.pair_cap, cus));
  if (ev) (void)hipEventRecord(ev[2], stream);
  if (b.gap_on)
    hipLaunchKernelGGL(coincidence_batch_kernel<true>, cgrid, dim3(kBlock), 0, stream, b);
  else
    hipLaunchKernelGGL(coincidence_batch_kernel<false>, cgrid, dim3(kBlock), 0, stream, b);
  if (ev) (void)hipEventRecord(ev[3], stream);
  return hipGetLastError();
}
}  // namespace

}  // namespace sse
