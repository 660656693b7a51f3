// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sse {

constexpr float kMec2 = 510.99895f;          // electron rest energy, keV (CODATA 2018)
constexpr int kMaxSteps = 100000;            // tentative Woodcock steps per photon
constexpr int kMaxTries = 1000;              // rejection-loop guard (never reached)
constexpr int kRecordWords = 32;
constexpr int kStatCount = 19;

enum LutType { kLutF32 = 0, kLutF16 = 1, kLutBF16 = 2 };

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
  float mu_maj;             // Woodcock majorant at 511 keV
  // scanner and sinogram
  int n_crystals, n_rings, cmod, rblk, max_ring_diff;
  float rr, half_len, pitch;
  int n_rad, n_view, n_plane, n_tof;
  float tof_bin, tof_sigma;
  // physics
  float e_lo, e_hi, e_kill, e_fwhm, rayleigh_beta;
  double f_c, f_r, f_p, kn511;
  int max_int;
  ECoef e511;               // coefficients at 511 keV (host-evaluated)
  // LUT
  const void* lut;
  int lut_type;
  int d0, d1, d2, d3, d4;
  float e_min, e_scale;
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
};

// Total Klein-Nishina cross section in units of 2 pi r_e^2, a = E / m_e c^2.
__host__ __device__ inline double kn_total(double a) {
  double L = log(1.0 + 2.0 * a);
  double t1 = (1.0 + a) / (a * a) * (2.0 * (1.0 + a) / (1.0 + 2.0 * a) - L / a);
  double t2 = L / (2.0 * a);
  double t3 = (1.0 + 3.0 * a) / ((1.0 + 2.0 * a) * (1.0 + 2.0 * a));
  return t1 + t2 - t3;
}

hipError_t launch_transport(const TransportParams& p, hipStream_t stream);

// One sub-chunk of a request: histories [h0, h0 + n) of items[item].
struct WorkChunk {
  uint64_t h0;
  uint32_t n;
  uint32_t item;
};

// A list of sub-chunks over several requests, simulated by one launch.
struct BatchParams {
  const TransportParams* items;  // device array, one per request slot
  const WorkChunk* chunks;       // device array
  uint32_t n_chunks;
  uint32_t* counter;             // device, reset by the launcher
};

hipError_t launch_transport_batch(const BatchParams& b, hipStream_t stream);

struct PostParams {
  int n_rad, n_view, n_plane, n_tof;
};

hipError_t launch_apply_sensitivity(const PostParams& g, const double* W, double scale, const float* sens,
                                    int sens_tof, float* out, hipStream_t stream);
hipError_t launch_scale_to_float(const PostParams& g, const double* W, double scale, float* out,
                                 hipStream_t stream);
hipError_t launch_multiply_sens(const PostParams& g, const float* in, const float* sens, int sens_tof,
                                float* out, hipStream_t stream);
constexpr int kMaxSmoothRadius = 63;
// Normalised Gaussian taps w[0 .. 2*radius], passed by value to the kernel.
struct Taps {
  float w[2 * kMaxSmoothRadius + 1];
  int radius;
};
// One separable pass along axis (0 radial, 1 view, 2 plane).  The input is
// binary32, or binary64 weights scaled by `scale` and rounded on load
// (in_is_f64); if sens is not NULL the output is multiplied by it.
hipError_t launch_smooth_axis(const PostParams& g, int axis, const void* in, bool in_is_f64, double scale,
                              float* out, const Taps& taps, const float* sens, int sens_tof, hipStream_t stream);

}  // namespace sse
