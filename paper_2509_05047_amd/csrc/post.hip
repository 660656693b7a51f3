// Sinogram post-processing on gfx950: sensitivity multiply and separable
// Gaussian smoothing.  All of it is HBM-bandwidth bound streaming over
// [tof][plane][view][rad] float / double arrays.
//
// The final scatter estimate is the LUT-weighted simulator sinogram times the
// scatter-sensitivity sinogram (Methods, "Scatter sensitivity sinogram"); the
// smoothing runs along the radial, angular and planar axes (Methods, "Known
// activity distribution, very limited simulation time"), here as one pass per
// axis over a 3D grid: x covers the radial index, y the view, z the
// (tof, plane) pair, so no thread divides 64-bit indices.  In the fused
// finalize the first pass reads the binary64 weights (scaled and rounded to
// binary32 on load) and the last pass multiplies by the sensitivity.
#include "internal.h"

namespace sse {
namespace {

constexpr int kRadBlock = 128;

// out[t][inner] = (float)((scale * W) * sens[t][inner] or sens[inner])
__global__ void __launch_bounds__(256) apply_sens_kernel(const double* __restrict__ W, double scale,
                                                          const float* __restrict__ sens, uint64_t inner,
                                                          int sens_tof, float* __restrict__ out) {
  const uint64_t t = blockIdx.y;
  const uint64_t base = t * inner;
  const uint64_t sbase = sens_tof ? base : 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < inner; j += stride)
    out[base + j] = static_cast<float>((scale * W[base + j]) * static_cast<double>(sens[sbase + j]));
}

__device__ __forceinline__ int reflect(int i, int n) {
  const int period = 2 * n;
  int m = i % period;
  if (m < 0) m += period;
  return m < n ? m : period - 1 - m;
}

template <bool kFromF64>
__device__ __forceinline__ float load_in(const void* in, uint64_t i, double scale) {
  if (kFromF64) return static_cast<float>(scale * static_cast<const double*>(in)[i]);
  return static_cast<const float*>(in)[i];
}

// One separable pass along `axis` (0 radial, 1 view, 2 plane).
template <int kAxis, bool kFromF64, bool kMulSens>
__global__ void __launch_bounds__(kRadBlock) smooth_pass(PostParams g, const void* __restrict__ in,
                                                          float* __restrict__ out, Taps taps, double scale,
                                                          const float* __restrict__ sens, int sens_tof) {
  const int r = blockIdx.x * kRadBlock + threadIdx.x;
  if (r >= g.n_rad) return;
  const int v = blockIdx.y;
  const int t = blockIdx.z / g.n_plane;
  const int pl = blockIdx.z - t * g.n_plane;
  const uint64_t row = static_cast<uint64_t>(g.n_rad);
  const uint64_t vstride = row;
  const uint64_t pstride = row * g.n_view;
  const uint64_t tstride = pstride * g.n_plane;
  const uint64_t o = static_cast<uint64_t>(t) * tstride + static_cast<uint64_t>(pl) * pstride +
                     static_cast<uint64_t>(v) * vstride + static_cast<uint64_t>(r);
  const int radius = taps.radius;
  float acc = 0.0f;
  if (kAxis == 0) {
    const uint64_t base = o - r;
    for (int k = -radius; k <= radius; ++k) acc += taps.w[k + radius] * load_in<kFromF64>(in, base + reflect(r + k, g.n_rad), scale);
  } else if (kAxis == 2) {
    const uint64_t base = o - static_cast<uint64_t>(pl) * pstride;
    for (int k = -radius; k <= radius; ++k)
      acc += taps.w[k + radius] * load_in<kFromF64>(in, base + static_cast<uint64_t>(reflect(pl + k, g.n_plane)) * pstride, scale);
  } else {
    // views are periodic over 180 degrees; past the seam the same LOR is
    // seen from the other end (radial and TOF indices reversed)
    const int period = 2 * g.n_view;
    const uint64_t plane_off = static_cast<uint64_t>(pl) * pstride;
    const uint64_t direct = static_cast<uint64_t>(t) * tstride + plane_off + static_cast<uint64_t>(r);
    const uint64_t flipped = static_cast<uint64_t>(g.n_tof - 1 - t) * tstride + plane_off +
                             static_cast<uint64_t>(g.n_rad - 1 - r);
    for (int k = -radius; k <= radius; ++k) {
      int m = (v + k) % period;
      if (m < 0) m += period;
      const uint64_t idx = m < g.n_view ? direct + static_cast<uint64_t>(m) * vstride
                                        : flipped + static_cast<uint64_t>(m - g.n_view) * vstride;
      acc += taps.w[k + radius] * load_in<kFromF64>(in, idx, scale);
    }
  }
  if (kMulSens) {
    const uint64_t inner = tstride;
    acc = acc * sens[sens_tof ? o : o - static_cast<uint64_t>(t) * inner];
  }
  out[o] = acc;
}

// scale * W -> float (with optional sensitivity), used when no axis is smoothed
__global__ void __launch_bounds__(256) scale_kernel(const double* __restrict__ W, double scale, uint64_t n,
                                                     float* __restrict__ out) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = static_cast<float>(scale * W[i]);
}

__global__ void __launch_bounds__(256) mul_sens_kernel(const float* __restrict__ in, const float* __restrict__ sens,
                                                        uint64_t inner, int sens_tof, float* __restrict__ out) {
  const uint64_t base = static_cast<uint64_t>(blockIdx.y) * inner;
  const uint64_t sbase = sens_tof ? base : 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < inner; j += stride)
    out[base + j] = in[base + j] * sens[sbase + j];
}

uint64_t inner_bins(const PostParams& g) { return static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane; }

int blocks_for(uint64_t inner) {
  const uint64_t b = (inner + 255) / 256;
  return static_cast<int>(b < 4096 ? (b ? b : 1) : 4096);
}

template <int kAxis>
hipError_t pass(const PostParams& g, const void* in, bool from_f64, float* out, const Taps& taps, double scale,
                const float* sens, int sens_tof, hipStream_t s) {
  const dim3 grid((g.n_rad + kRadBlock - 1) / kRadBlock, g.n_view, g.n_plane * g.n_tof);
  if (from_f64 && sens)
    hipLaunchKernelGGL((smooth_pass<kAxis, true, true>), grid, dim3(kRadBlock), 0, s, g, in, out, taps, scale, sens, sens_tof);
  else if (from_f64)
    hipLaunchKernelGGL((smooth_pass<kAxis, true, false>), grid, dim3(kRadBlock), 0, s, g, in, out, taps, scale, sens, sens_tof);
  else if (sens)
    hipLaunchKernelGGL((smooth_pass<kAxis, false, true>), grid, dim3(kRadBlock), 0, s, g, in, out, taps, scale, sens, sens_tof);
  else
    hipLaunchKernelGGL((smooth_pass<kAxis, false, false>), grid, dim3(kRadBlock), 0, s, g, in, out, taps, scale, sens, sens_tof);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_sensitivity(const PostParams& g, const double* W, double scale, const float* sens,
                                    int sens_tof, float* out, hipStream_t stream) {
  const uint64_t inner = inner_bins(g);
  hipLaunchKernelGGL(apply_sens_kernel, dim3(blocks_for(inner), g.n_tof), dim3(256), 0, stream, W, scale, sens, inner,
                     sens_tof, out);
  return hipGetLastError();
}

hipError_t launch_scale_to_float(const PostParams& g, const double* W, double scale, float* out,
                                 hipStream_t stream) {
  const uint64_t n = inner_bins(g) * g.n_tof;
  hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, W, scale, n, out);
  return hipGetLastError();
}

hipError_t launch_multiply_sens(const PostParams& g, const float* in, const float* sens, int sens_tof,
                                float* out, hipStream_t stream) {
  const uint64_t inner = inner_bins(g);
  hipLaunchKernelGGL(mul_sens_kernel, dim3(blocks_for(inner), g.n_tof), dim3(256), 0, stream, in, sens, inner,
                     sens_tof, out);
  return hipGetLastError();
}

hipError_t launch_smooth_axis(const PostParams& g, int axis, const void* in, bool in_is_f64, double scale,
                              float* out, const Taps& taps, const float* sens, int sens_tof, hipStream_t stream) {
  if (axis == 0) return pass<0>(g, in, in_is_f64, out, taps, scale, sens, sens_tof, stream);
  if (axis == 1) return pass<1>(g, in, in_is_f64, out, taps, scale, sens, sens_tof, stream);
  return pass<2>(g, in, in_is_f64, out, taps, scale, sens, sens_tof, stream);
}

}  // namespace sse
