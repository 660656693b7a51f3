// Monte Carlo pair transport, detection, LUT weighting and TOF sinogram
// accumulation on gfx950.
//
// One launch simulates histories h0 .. h0+n-1.  Each history: emission from
// the activity alias table, two photons tracked with Woodcock steps through
// the attenuation map (Compton by Kahn's method, Rayleigh with an analytic
// form factor, photoabsorption), crossing of the detection cylinder, crystal /
// ring / 5D-LUT indexing of each single, and one atomic update of the TOF
// sinogram bin with count 1 and weight p_A p_B (Methods, "Scatter simulator
// description" and "Photon detection probability LUT").
//
// Numerics: binary32 transport with IEEE-rounded + - * / sqrt (no
// contraction); ln, atan2 and the cross-section formula in binary64, rounded
// once where they feed binary32 values.  Random numbers are Philox4x32-10
// streams keyed by (seed), countered by (block, history, substream), so a
// history's result does not depend on the launch geometry.
#include "internal.h"

namespace sse {
namespace {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;
constexpr double kHalfPi = 1.5707963267948966;

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

// A random stream of 32-bit words: the words of blocks 0, 1, 2, ... with
// counter (block, h_lo, h_hi, substream).  The four words of the current
// block are shifted out in order (no dynamically indexed registers).
struct Stream {
  uint32_t k0, k1, hlo, hhi, sub, blk;
  uint32_t w0, w1, w2, w3;
  uint32_t left;

  __device__ __forceinline__ void init(uint64_t seed, uint64_t h, uint32_t s) {
    k0 = static_cast<uint32_t>(seed);
    k1 = static_cast<uint32_t>(seed >> 32);
    hlo = static_cast<uint32_t>(h);
    hhi = static_cast<uint32_t>(h >> 32);
    sub = s;
    blk = 0;
    left = 0;
  }
  __device__ __forceinline__ uint32_t next() {
    if (left == 0) {
      philox(blk, hlo, hhi, sub, k0, k1, w0, w1, w2, w3);
      ++blk;
      left = 4;
    }
    const uint32_t r = w0;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    --left;
    return r;
  }
  // uniform in (0, 1): 24 bits with the last forced odd, times 2^-24
  __device__ __forceinline__ float uniform() {
    return static_cast<float>((next() >> 8) | 1u) * 5.9604644775390625e-08f;
  }
};

__device__ __forceinline__ float neg_log(float u) { return static_cast<float>(-log(static_cast<double>(u))); }

__device__ float normal_polar(Stream& r) {
  for (int i = 0; i < kMaxTries; ++i) {
    const float a = 2.0f * r.uniform() - 1.0f;
    const float b = 2.0f * r.uniform() - 1.0f;
    const float s = a * a + b * b;
    if (s < 1.0f)
      return a * static_cast<float>(sqrt(-2.0 * log(static_cast<double>(s)) / static_cast<double>(s)));
  }
  return 0.0f;
}

// ---------------------------------------------------------------------------
// physics
// ---------------------------------------------------------------------------
__device__ void energy_coefficients(ECoef& c, float E, const TransportParams& p) {
  c.E = E;
  c.alpha = E / kMec2;
  const double a = static_cast<double>(c.alpha);
  const double fc = p.f_c * (kn_total(a) / p.kn511);
  const double fr = p.f_r * (1.0 / (a * a));
  const double fp = p.f_p * (1.0 / (a * a * a));
  c.g = static_cast<float>(fc + fr + fp);
  c.cC = static_cast<float>(fc);
  c.cCR = static_cast<float>(fc + fr);
  c.inv_maj = 1.0f / (p.mu_maj * c.g);
}

// Kahn (1954) rejection sampling of x = E/E' for Klein-Nishina scattering.
__device__ bool sample_compton(Stream& r, float alpha, float& x_out) {
  const float twoa = 2.0f * alpha;
  const float b1 = 1.0f + twoa;
  const float b2 = 9.0f + twoa;
  for (int i = 0; i < kMaxTries; ++i) {
    const float r1 = r.uniform();
    const float r2 = r.uniform();
    const float r3 = r.uniform();
    if (r1 * b2 <= b1) {
      const float x = 1.0f + twoa * r2;
      if (r3 * (x * x) <= 4.0f * (x - 1.0f)) { x_out = x; return true; }
    } else {
      const float x = b1 / (1.0f + twoa * r2);
      const float c = 1.0f + (1.0f - x) / alpha;
      if (2.0f * r3 <= c * c + 1.0f / x) { x_out = x; return true; }
    }
  }
  return false;
}

// Rayleigh polar angle: (1 + beta' t)^-2 by inversion in t = 1 - cos, then
// the Thomson factor (1 + cos^2)/2 by rejection.
__device__ bool sample_rayleigh(Stream& r, float alpha, float beta, float& cos_out) {
  const float bp = beta * (alpha * alpha);
  const float cc = (2.0f * bp) / (1.0f + 2.0f * bp);
  for (int i = 0; i < kMaxTries; ++i) {
    const float r1 = r.uniform();
    const float r2 = r.uniform();
    const float q = r1 * cc;
    const float t = q / ((1.0f - q) * bp);
    float c = 1.0f - t;
    if (c < -1.0f) c = -1.0f;
    if (2.0f * r2 <= 1.0f + c * c) { cos_out = c; return true; }
  }
  return false;
}

// (cos phi, sin phi) of a uniform azimuth from a point in the unit disk.
__device__ void sample_azimuth(Stream& r, float& cp, float& sp) {
  for (int i = 0; i < kMaxTries; ++i) {
    const float a = 2.0f * r.uniform() - 1.0f;
    const float b = 2.0f * r.uniform() - 1.0f;
    const float s = a * a + b * b;
    if (s < 1.0f) {
      cp = (a * a - b * b) / s;
      sp = (2.0f * a * b) / s;
      return;
    }
  }
  cp = 1.0f;
  sp = 0.0f;
}

__device__ __forceinline__ void rotate(float& dx, float& dy, float& dz, float ct, float cp, float sp) {
  const float st = sqrtf((1.0f - ct) * (1.0f + ct));
  const float ux = dx, uy = dy, uz = dz;
  if (fabsf(uz) > 0.99999f) {
    const float sg = uz > 0.0f ? 1.0f : -1.0f;
    dx = st * cp;
    dy = st * sp;
    dz = sg * ct;
  } else {
    const float tmp = sqrtf((1.0f - uz) * (1.0f + uz));
    dx = ux * ct + st * (ux * uz * cp - uy * sp) / tmp;
    dy = uy * ct + st * (uy * uz * cp + ux * sp) / tmp;
    dz = uz * ct - tmp * st * cp;
  }
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
__device__ __forceinline__ float box_exit(const TransportParams& p, float px, float py, float pz, float dx,
                                          float dy, float dz) {
  float t = __builtin_huge_valf();
  if (dx > 0.0f) t = fminf(t, (p.hix - px) / dx);
  else if (dx < 0.0f) t = fminf(t, (p.lox - px) / dx);
  if (dy > 0.0f) t = fminf(t, (p.hiy - py) / dy);
  else if (dy < 0.0f) t = fminf(t, (p.loy - py) / dy);
  if (dz > 0.0f) t = fminf(t, (p.hiz - pz) / dz);
  else if (dz < 0.0f) t = fminf(t, (p.loz - pz) / dz);
  return t;
}

__device__ __forceinline__ int clamp_floor(float f, int n) {
  f = floorf(f);
  if (!(f >= 0.0f)) return 0;
  if (f >= static_cast<float>(n)) return n - 1;
  return static_cast<int>(f);
}

__device__ __forceinline__ uint32_t voxel_at(const TransportParams& p, float x, float y, float z) {
  const int ix = clamp_floor((x - p.lox) * p.ivx, p.nx);
  const int iy = clamp_floor((y - p.loy) * p.ivy, p.ny);
  const int iz = clamp_floor((z - p.loz) * p.ivz, p.nz);
  return (static_cast<uint32_t>(iz) * static_cast<uint32_t>(p.ny) + static_cast<uint32_t>(iy)) *
             static_cast<uint32_t>(p.nx) + static_cast<uint32_t>(ix);
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

enum Fate { kDetected = 0, kAbsorbed = 1, kKilled = 2, kCapped = 3, kAxial = 4 };

struct Counters {
  uint32_t v[kStatCount];
};

struct Single {
  float hx, hy, hz, dx, dy, dz, E, Edet, path;
  int fate, nC, nR;
  uint32_t steps;
};

// Track one photon from (px,py,pz) along (dx,dy,dz) at 511 keV to the cylinder.
__device__ void track(const TransportParams& p, Stream& r, float px, float py, float pz, float dx, float dy,
                      float dz, Single& o, Counters& cnt) {
  ECoef ec = p.e511;
  float len = 0.0f;
  float t = 0.0f;
  float texit = box_exit(p, px, py, pz, dx, dy, dz);
  int nC = 0, nR = 0, nint = 0;
  uint32_t steps = 0;
  int fate = -1;
  for (;;) {
    if (steps >= static_cast<uint32_t>(kMaxSteps)) { fate = kCapped; break; }
    ++steps;
    const float s = neg_log(r.uniform()) * ec.inv_maj;
    t = t + s;
    if (!(t < texit)) break;
    const float qx = px + t * dx;
    const float qy = py + t * dy;
    const float qz = pz + t * dz;
    const float mu = p.mu[voxel_at(p, qx, qy, qz)];
    if (!(r.uniform() * p.mu_maj < mu)) continue;  // null collision
    ++cnt.v[2];
    px = qx; py = qy; pz = qz;
    len = len + t;
    t = 0.0f;
    if (++nint > p.max_int) { fate = kCapped; break; }
    const float ug = r.uniform() * ec.g;
    float ct;
    if (ug < ec.cC) {
      float x;
      if (!sample_compton(r, ec.alpha, x)) { fate = kAbsorbed; break; }
      const float e2 = ec.E / x;
      ct = 1.0f - (x - 1.0f) / ec.alpha;
      ct = fminf(fmaxf(ct, -1.0f), 1.0f);
      ++nC;
      ++cnt.v[3];
      if (e2 < p.e_kill) { fate = kKilled; break; }
      energy_coefficients(ec, e2, p);
    } else if (ug < ec.cCR) {
      if (!sample_rayleigh(r, ec.alpha, p.rayleigh_beta, ct)) { fate = kAbsorbed; break; }
      ++nR;
      ++cnt.v[4];
    } else {
      fate = kAbsorbed;
      break;
    }
    float cp, sp;
    sample_azimuth(r, cp, sp);
    rotate(dx, dy, dz, ct, cp, sp);
    texit = box_exit(p, px, py, pz, dx, dy, dz);
  }
  cnt.v[1] += steps;
  o.steps = steps;
  o.nC = nC;
  o.nR = nR;
  o.E = ec.E;
  o.Edet = ec.E;
  o.path = 0.0f;
  o.hx = o.hy = o.hz = 0.0f;
  o.dx = dx; o.dy = dy; o.dz = dz;
  if (fate >= 0) {
    o.fate = fate;
    if (fate == kAbsorbed) ++cnt.v[5];
    else if (fate == kKilled) ++cnt.v[6];
    else ++cnt.v[7];
    return;
  }
  ++cnt.v[8];
  // crossing of x^2 + y^2 = R^2 ahead of the last point
  const float a = dx * dx + dy * dy;
  if (!(a > 0.0f)) { o.fate = kAxial; return; }
  const float b = px * dx + py * dy;
  const float c = px * px + py * py - p.rr;
  const float disc = b * b - a * c;
  const float sq = sqrtf(disc);
  const float tc = (b > 0.0f) ? (-c) / (b + sq) : (sq - b) / a;
  const float hz = pz + tc * dz;
  if (!(hz >= -p.half_len && hz < p.half_len)) { o.fate = kAxial; return; }
  o.fate = kDetected;
  o.hx = px + tc * dx;
  o.hy = py + tc * dy;
  o.hz = hz;
  o.path = len + tc;
  ++cnt.v[9];
  if (p.e_fwhm > 0.0f) {
    const float nrm = normal_polar(r);
    const float sig = (p.e_fwhm / 2.35482f) * sqrtf(kMec2 / ec.E);
    o.Edet = ec.E * (1.0f + sig * nrm);
  }
}

// Crystal, ring and flat LUT index of a detected single.
__device__ void index_single(const TransportParams& p, const Single& o, int& crystal, int& ring, uint32_t& lut) {
  double phi = atan2(static_cast<double>(o.hy), static_cast<double>(o.hx));
  if (phi < 0.0) phi += kTwoPi;
  const double fc = floor(phi * static_cast<double>(p.n_crystals) / kTwoPi);
  const int c = fc >= static_cast<double>(p.n_crystals) ? p.n_crystals - 1 : (fc < 0.0 ? 0 : static_cast<int>(fc));
  const int rg = clamp_floor((o.hz + p.half_len) / p.pitch, p.n_rings);
  crystal = c;
  ring = rg;
  const int ie = clamp_floor((o.E - p.e_min) * p.e_scale, p.d0);
  const double hx = static_cast<double>(o.hx), hy = static_cast<double>(o.hy);
  const double rho = sqrt(hx * hx + hy * hy);
  const double dr = (hx * static_cast<double>(o.dx) + hy * static_cast<double>(o.dy)) / rho;
  const double tt = (hx * static_cast<double>(o.dy) - hy * static_cast<double>(o.dx)) / rho;
  const int it = angle_bin(atan2(tt, dr), p.d1);
  const int ia = angle_bin(atan2(static_cast<double>(o.dz), dr), p.d2);
  const int ct = ((c % p.cmod) * p.d3) / p.cmod;
  const int ca = ((rg % p.rblk) * p.d4) / p.rblk;
  lut = static_cast<uint32_t>((((ie * p.d1 + it) * p.d2 + ia) * p.d3 + ct) * p.d4 + ca);
}

__device__ void write_single(uint32_t* w, const Single& o, bool inwin, int c, int rg, uint32_t lut) {
  w[0] = __float_as_uint(o.hx);
  w[1] = __float_as_uint(o.hy);
  w[2] = __float_as_uint(o.hz);
  w[3] = __float_as_uint(o.dx);
  w[4] = __float_as_uint(o.dy);
  w[5] = __float_as_uint(o.dz);
  w[6] = __float_as_uint(o.E);
  w[7] = __float_as_uint(o.Edet);
  w[8] = __float_as_uint(o.path);
  w[9] = inwin ? (static_cast<uint32_t>(c) | (static_cast<uint32_t>(rg) << 16)) : 0xffffffffu;
  w[10] = inwin ? lut : 0xffffffffu;
  w[11] = static_cast<uint32_t>(o.nC) | (static_cast<uint32_t>(o.nR) << 8) | (static_cast<uint32_t>(o.fate) << 16);
}

__device__ void simulate_history(const TransportParams& p, uint64_t h, Counters& cnt) {
  Stream rs;
  rs.init(p.seed, h, 0);
  // emission voxel: 64-bit multiply-shift column, 32-bit alias decision
  const uint64_t lo = rs.next();
  const uint64_t hi = rs.next();
  const uint64_t col = __umul64hi((hi << 32) | lo, p.nvox);
  const uint32_t x1 = rs.next();
  const uint2 al = p.alias[col];
  const uint32_t v = (x1 < al.x) ? static_cast<uint32_t>(col) : al.y;
  const uint32_t nx = static_cast<uint32_t>(p.nx), ny = static_cast<uint32_t>(p.ny);
  const uint32_t ix = v % nx, iy = (v / nx) % ny, iz = v / (nx * ny);
  const float ux = rs.uniform();
  const float uy = rs.uniform();
  const float uz = rs.uniform();
  const float px = p.lox + (static_cast<float>(ix) + ux) * p.vx;
  const float py = p.loy + (static_cast<float>(iy) + uy) * p.vy;
  const float pz = p.loz + (static_cast<float>(iz) + uz) * p.vz;
  // isotropic direction (Marsaglia 1972)
  float dx = 0.0f, dy = 0.0f, dz = 1.0f;
  for (int i = 0; i < kMaxTries; ++i) {
    const float a = 2.0f * rs.uniform() - 1.0f;
    const float b = 2.0f * rs.uniform() - 1.0f;
    const float s = a * a + b * b;
    if (s < 1.0f) {
      const float q = 2.0f * sqrtf(1.0f - s);
      dx = a * q;
      dy = b * q;
      dz = 1.0f - 2.0f * s;
      break;
    }
  }
  Single A, B;
  Stream r1;
  r1.init(p.seed, h, 1);
  track(p, r1, px, py, pz, dx, dy, dz, A, cnt);
  Stream r2;
  r2.init(p.seed, h, 2);
  track(p, r2, px, py, pz, -dx, -dy, -dz, B, cnt);
  ++cnt.v[0];

  const bool winA = A.fate == kDetected && A.Edet >= p.e_lo && A.Edet <= p.e_hi;
  const bool winB = B.fate == kDetected && B.Edet >= p.e_lo && B.Edet <= p.e_hi;
  int cA = -1, rA = -1, cB = -1, rB = -1;
  uint32_t lA = 0xffffffffu, lB = 0xffffffffu;
  if (winA) { index_single(p, A, cA, rA, lA); ++cnt.v[10]; }
  if (winB) { index_single(p, B, cB, rB, lB); ++cnt.v[10]; }
  const bool scattered = (A.nC + A.nR + B.nC + B.nR) > 0;
  uint32_t outcome;
  uint64_t bin = ~0ull;
  float w = 0.0f, tau = 0.0f;
  Stream r3;
  r3.init(p.seed, h, 3);
  if (A.fate != kDetected || B.fate != kDetected) {
    outcome = 2;
  } else if (!winA || !winB) {
    outcome = 3;
    ++cnt.v[13];
  } else if (cA == cB) {
    outcome = 4;
    ++cnt.v[14];
  } else if (p.max_ring_diff >= 0 && abs(rA - rB) > p.max_ring_diff) {
    outcome = 5;
    ++cnt.v[15];
  } else {
    const int n = p.n_crystals;
    int k = cA + cB + 1;
    int rho = n / 2 - abs(cA - cB);
    if (k >= n) { k -= n; rho = -rho; }
    const int view = k >> 1;
    int m = (2 * cA + 1 - k) % (2 * n);
    if (m < 0) m += 2 * n;
    const bool a_pos = m > 0 && m < n;
    const int half = (p.n_rad - 1) / 2;
    if (abs(rho) > half) {
      outcome = 6;
      ++cnt.v[16];
    } else {
      tau = a_pos ? (B.path - A.path) * 0.5f : (A.path - B.path) * 0.5f;
      if (p.tof_sigma > 0.0f) tau = tau + p.tof_sigma * normal_polar(r3);
      const float xt = tau / p.tof_bin + static_cast<float>(p.n_tof) * 0.5f;
      if (!(xt >= 0.0f) || !(xt < static_cast<float>(p.n_tof))) {
        outcome = 7;
        ++cnt.v[17];
      } else {
        const uint64_t tof = static_cast<uint64_t>(floorf(xt));
        const uint64_t plane = static_cast<uint64_t>(rA + rB);
        bin = ((tof * static_cast<uint64_t>(p.n_plane) + plane) * static_cast<uint64_t>(p.n_view) +
               static_cast<uint64_t>(view)) * static_cast<uint64_t>(p.n_rad) + static_cast<uint64_t>(rho + half);
        w = lut_value(p, lA) * lut_value(p, lB);
        if (scattered) {
          outcome = 0;
          ++cnt.v[11];
          atomicAdd(p.sc_n + bin, 1u);
          unsafeAtomicAdd(p.sc_w + bin, static_cast<double>(w));
        } else {
          outcome = 1;
          ++cnt.v[12];
          if (p.tr_n) atomicAdd(p.tr_n + bin, 1u);
          if (p.tr_w) unsafeAtomicAdd(p.tr_w + bin, static_cast<double>(w));
        }
      }
    }
  }
  cnt.v[18] += rs.blk + r1.blk + r2.blk + r3.blk;
  if (p.rec) {
    const uint64_t off = h - p.h0;
    if (off % p.rec_stride == 0) {
      uint32_t* wr = p.rec + (off / p.rec_stride) * kRecordWords;
      wr[0] = outcome | (scattered ? 0x100u : 0u);
      wr[1] = static_cast<uint32_t>(bin);
      wr[2] = static_cast<uint32_t>(bin >> 32);
      wr[3] = v;
      wr[4] = __float_as_uint(w);
      wr[5] = __float_as_uint(tau);
      wr[6] = A.steps + B.steps;
      wr[7] = 0u;
      write_single(wr + 8, A, winA, cA, rA, lA);
      write_single(wr + 20, B, winB, cB, rB, lB);
    }
  }
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ void __launch_bounds__(256) transport_kernel(TransportParams p) {
  Counters cnt;
#pragma unroll
  for (int i = 0; i < kStatCount; ++i) cnt.v[i] = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < p.n; i += stride)
    simulate_history(p, p.h0 + i, cnt);
  if (p.stats) {
    const bool leader = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < kStatCount; ++i) {
      const uint64_t s = wave_sum(cnt.v[i]);
      if (leader && s) atomicAdd(p.stats + i, static_cast<unsigned long long>(s));
    }
  }
}

}  // namespace

hipError_t launch_transport(const TransportParams& p, hipStream_t stream) {
  if (p.n == 0) return hipSuccess;
  const int block = 256;
  const uint64_t want = (p.n + block - 1) / block;
  const int grid = static_cast<int>(want < 16384 ? want : 16384);
  hipLaunchKernelGGL(transport_kernel, dim3(grid), dim3(block), 0, stream, p);
  return hipGetLastError();
}

}  // namespace sse
