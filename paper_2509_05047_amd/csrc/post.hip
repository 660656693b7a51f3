// Sinogram post-processing on gfx950: sensitivity multiply and separable
// Gaussian smoothing.  All of it is HBM-bandwidth bound streaming over
// [tof][plane][view][rad] float / double arrays.
//
// The final scatter estimate is the LUT-weighted simulator sinogram times the
// scatter-sensitivity sinogram (Methods, "Scatter sensitivity sinogram"); the
// smoothing runs along the radial, angular and planar axes (Methods, "Known
// activity distribution, very limited simulation time").
#include "internal.h"

namespace sse {
namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) apply_sens_kernel(const double* __restrict__ W, double scale,
                                                             const float* __restrict__ sens, uint64_t n,
                                                             uint64_t sens_period, float* __restrict__ out) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t j = sens_period ? i % sens_period : i;
    out[i] = static_cast<float>((scale * W[i]) * static_cast<double>(sens[j]));
  }
}

__global__ void __launch_bounds__(kBlock) scale_kernel(const double* __restrict__ W, double scale, uint64_t n,
                                                        float* __restrict__ out) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = static_cast<float>(scale * W[i]);
}

__global__ void __launch_bounds__(kBlock) mul_sens_kernel(const float* __restrict__ in,
                                                           const float* __restrict__ sens, uint64_t n,
                                                           uint64_t sens_period, float* __restrict__ out) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t j = sens_period ? i % sens_period : i;
    out[i] = in[i] * sens[j];
  }
}

__device__ __forceinline__ int reflect(int i, int n) {
  const int period = 2 * n;
  int m = i % period;
  if (m < 0) m += period;
  return m < n ? m : period - 1 - m;
}

// One output bin per thread; taps read through L2.
__global__ void __launch_bounds__(kBlock) smooth_kernel(PostParams g, int axis, const float* __restrict__ in,
                                                         float* __restrict__ out, Taps taps, uint64_t n) {
  const int radius = taps.radius;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int r = static_cast<int>(i % g.n_rad);
    uint64_t rest = i / g.n_rad;
    const int v = static_cast<int>(rest % g.n_view);
    rest /= g.n_view;
    const int pl = static_cast<int>(rest % g.n_plane);
    const int t = static_cast<int>(rest / g.n_plane);
    float acc = 0.0f;
    if (axis == 0) {
      const uint64_t base = i - r;
      for (int k = -radius; k <= radius; ++k) acc += taps.w[k + radius] * in[base + reflect(r + k, g.n_rad)];
    } else if (axis == 2) {
      for (int k = -radius; k <= radius; ++k) {
        const int q = reflect(pl + k, g.n_plane);
        acc += taps.w[k + radius] *
               in[((static_cast<uint64_t>(t) * g.n_plane + q) * g.n_view + v) * g.n_rad + r];
      }
    } else {
      const int period = 2 * g.n_view;
      for (int k = -radius; k <= radius; ++k) {
        int m = (v + k) % period;
        if (m < 0) m += period;
        int tt = t, rr = r, vv = m;
        if (m >= g.n_view) {  // past 180 degrees: same LOR from the other end
          vv = m - g.n_view;
          tt = g.n_tof - 1 - t;
          rr = g.n_rad - 1 - r;
        }
        acc += taps.w[k + radius] *
               in[((static_cast<uint64_t>(tt) * g.n_plane + pl) * g.n_view + vv) * g.n_rad + rr];
      }
    }
    out[i] = acc;
  }
}

int grid_for(uint64_t n) {
  const uint64_t b = (n + kBlock - 1) / kBlock;
  return static_cast<int>(b < 65536 ? (b ? b : 1) : 65536);
}

uint64_t nbins(const PostParams& g) {
  return static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane * g.n_tof;
}

}  // namespace

hipError_t launch_apply_sensitivity(const PostParams& g, const double* W, double scale, const float* sens,
                                    int sens_tof, float* out, hipStream_t stream) {
  const uint64_t n = nbins(g);
  const uint64_t period = sens_tof ? 0 : static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane;
  hipLaunchKernelGGL(apply_sens_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, W, scale, sens, n, period, out);
  return hipGetLastError();
}

hipError_t launch_scale_to_float(const PostParams& g, const double* W, double scale, float* out,
                                 hipStream_t stream) {
  const uint64_t n = nbins(g);
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, W, scale, n, out);
  return hipGetLastError();
}

hipError_t launch_multiply_sens(const PostParams& g, const float* in, const float* sens, int sens_tof,
                                float* out, hipStream_t stream) {
  const uint64_t n = nbins(g);
  const uint64_t period = sens_tof ? 0 : static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane;
  hipLaunchKernelGGL(mul_sens_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, in, sens, n, period, out);
  return hipGetLastError();
}

hipError_t launch_smooth_axis(const PostParams& g, int axis, const float* in, float* out, const Taps& taps,
                              hipStream_t stream) {
  const uint64_t n = nbins(g);
  hipLaunchKernelGGL(smooth_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, g, axis, in, out, taps, n);
  return hipGetLastError();
}

}  // namespace sse
