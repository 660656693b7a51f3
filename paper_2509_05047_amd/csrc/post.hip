// Sinogram post-processing on gfx950: sensitivity multiply and separable
// Gaussian smoothing.  All of it is HBM-bandwidth bound streaming over
// [tof][plane][view][rad] float / double arrays.
//
// The final scatter estimate is the LUT-weighted simulator sinogram times the
// scatter-sensitivity sinogram (Methods, "Scatter sensitivity sinogram"); the
// smoothing runs along the radial, angular and planar axes (Methods, "Known
// activity distribution, very limited simulation time"), one pass per axis,
// each staging its input through LDS so that HBM sees every element read
// and written once per pass.  In the fused finalize the first pass reads the
// binary64 weights (scaled and rounded to binary32 on load) and the last
// pass multiplies by the sensitivity; with a smoothing normalisation
// sinogram the first pass also multiplies by it and the last divides by it
// (Discussion / Methods: the simulator output is normalised before smoothing
// and the structures re-applied after).
#include "post.h"

namespace sse {
namespace {

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

// Arguments of one smoothing pass.
struct SmoothArgs {
  PostParams g;
  const void* in;         // binary32, or binary64 weights times `scale` (rounded on load)
  double scale;
  const float* norm_in;   // multiplies the input on load (or NULL)
  float* out;
  const float* norm_out;  // divides the output (entries <= 0 count as 1; or NULL)
  const float* sens;      // multiplies the output (or NULL)
  int sens_tof;
  Taps taps;
};

template <bool kFromF64>
__device__ __forceinline__ float load_in(const SmoothArgs& a, uint64_t i) {
  float v;
  if (kFromF64) v = static_cast<float>(a.scale * static_cast<const double*>(a.in)[i]);
  else v = static_cast<const float*>(a.in)[i];
  if (a.norm_in) v = v * a.norm_in[i];
  return v;
}

__device__ __forceinline__ float finish_out(const SmoothArgs& a, float acc, uint64_t o, uint64_t inner) {
  if (a.norm_out) {
    const float nrm = a.norm_out[o];
    acc = nrm > 0.0f ? acc / nrm : acc;
  }
  if (a.sens) acc = acc * a.sens[a.sens_tof ? o : o % inner];
  return acc;
}

// Passes along the view (kAxis 1) or plane (kAxis 2) axis.  A block stages
// a tile of kTL positions along the axis (plus the kernel's halo) by kTC
// consecutive radial columns in LDS -- every input read once, in 128-byte
// rows -- and computes the tile's outputs from LDS.  Views are periodic over
// 180 degrees, and past the seam the same LOR is seen from the other end
// (radial and TOF indices reversed); planes reflect at the ends.
constexpr int kTC = 32;
constexpr int kTL = 128;

template <int kAxis, bool kFromF64>
__global__ void __launch_bounds__(256) smooth_cols(SmoothArgs a) {
  __shared__ float tile[(kTL + 2 * kMaxSmoothRadius) * kTC];
  const PostParams& g = a.g;
  const int R = a.taps.radius;
  const int n = kAxis == 1 ? g.n_view : g.n_plane;
  const int n_other = kAxis == 1 ? g.n_plane : g.n_view;
  const int r0 = blockIdx.x * kTC;
  const int p0 = blockIdx.y * kTL;
  const int tl = n - p0 < kTL ? n - p0 : kTL;
  const int t = blockIdx.z / n_other;
  const int other = blockIdx.z - t * n_other;
  const uint64_t vs = static_cast<uint64_t>(g.n_rad);
  const uint64_t ps = vs * g.n_view;
  const uint64_t ts = ps * g.n_plane;
  const int col = threadIdx.x & (kTC - 1);
  const int sub = threadIdx.x / kTC;
  constexpr int kRowsPerSweep = 256 / kTC;
  const int r = r0 + col;
  const int rows = tl + 2 * R;
  for (int i = sub; i < rows; i += kRowsPerSweep) {
    const int pos = p0 - R + i;
    float v = 0.0f;
    if (r < g.n_rad) {
      uint64_t idx;
      if (kAxis == 2) {
        idx = static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(reflect(pos, g.n_plane)) * ps +
              static_cast<uint64_t>(other) * vs + static_cast<uint64_t>(r);
      } else {
        const int period = 2 * g.n_view;
        int m = pos % period;
        if (m < 0) m += period;
        idx = m < g.n_view ? static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(other) * ps +
                                 static_cast<uint64_t>(m) * vs + static_cast<uint64_t>(r)
                           : static_cast<uint64_t>(g.n_tof - 1 - t) * ts + static_cast<uint64_t>(other) * ps +
                                 static_cast<uint64_t>(m - g.n_view) * vs + static_cast<uint64_t>(g.n_rad - 1 - r);
      }
      v = load_in<kFromF64>(a, idx);
    }
    tile[i * kTC + col] = v;
  }
  __syncthreads();
  if (r >= g.n_rad) return;
  for (int i = sub; i < tl; i += kRowsPerSweep) {
    float acc = 0.0f;
    for (int k = 0; k <= 2 * R; ++k) acc += a.taps.w[k] * tile[(i + k) * kTC + col];
    const int pos = p0 + i;
    const uint64_t o = kAxis == 2 ? static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(pos) * ps +
                                        static_cast<uint64_t>(other) * vs + static_cast<uint64_t>(r)
                                  : static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(other) * ps +
                                        static_cast<uint64_t>(pos) * vs + static_cast<uint64_t>(r);
    a.out[o] = finish_out(a, acc, o, ts);
  }
}

// Pass along the radial axis (contiguous rows, reflected at both ends): each
// wavefront stages a segment of kSeg outputs of one row plus the halo in LDS.
constexpr int kSeg = 256;

template <bool kFromF64>
__global__ void __launch_bounds__(256) smooth_rows(SmoothArgs a, uint64_t n_rows) {
  __shared__ float seg[4][kSeg + 2 * kMaxSmoothRadius];
  const PostParams& g = a.g;
  const int R = a.taps.radius;
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const int segs = (g.n_rad + kSeg - 1) / kSeg;
  const uint64_t job = static_cast<uint64_t>(blockIdx.x) * 4u + w;  // (row, segment)
  const uint64_t row = job / static_cast<uint64_t>(segs);
  if (row >= n_rows) return;
  const int s0 = static_cast<int>(job - row * static_cast<uint64_t>(segs)) * kSeg;
  const int len = g.n_rad - s0 < kSeg ? g.n_rad - s0 : kSeg;
  const uint64_t base = row * static_cast<uint64_t>(g.n_rad);
  float* buf = seg[w];
  for (int i = static_cast<int>(lane); i < len + 2 * R; i += 64)
    buf[i] = load_in<kFromF64>(a, base + static_cast<uint64_t>(reflect(s0 - R + i, g.n_rad)));
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint64_t inner = static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane;
  for (int i = static_cast<int>(lane); i < len; i += 64) {
    float acc = 0.0f;
    for (int k = 0; k <= 2 * R; ++k) acc += a.taps.w[k] * buf[i + k];
    const uint64_t o = base + static_cast<uint64_t>(s0 + i);
    a.out[o] = finish_out(a, acc, o, inner);
  }
}

// No axis smoothed: out = ((float)(scale W) or in) * norm_in / norm_out * sens.
template <bool kFromF64>
__global__ void __launch_bounds__(256) pointwise_kernel(SmoothArgs a, uint64_t n) {
  const uint64_t inner = static_cast<uint64_t>(a.g.n_rad) * a.g.n_view * a.g.n_plane;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    a.out[i] = finish_out(a, load_in<kFromF64>(a, i), i, inner);
}

// norm = G / S (S = float(scale W)), 1 where S or G is not positive.
__global__ void __launch_bounds__(256) norm_ratio_kernel(const double* __restrict__ W, double scale,
                                                          float* __restrict__ norm, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float s = static_cast<float>(scale * W[i]);
    const float gs = norm[i];
    norm[i] = (s > 0.0f && gs > 0.0f) ? gs / s : 1.0f;
  }
}

uint64_t inner_bins(const PostParams& g) { return static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane; }

int blocks_for(uint64_t inner) {
  const uint64_t b = (inner + 255) / 256;
  return static_cast<int>(b < 4096 ? (b ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_apply_sensitivity(const PostParams& g, const double* W, double scale, const float* sens,
                                    int sens_tof, float* out, hipStream_t stream) {
  const uint64_t inner = inner_bins(g);
  hipLaunchKernelGGL(apply_sens_kernel, dim3(blocks_for(inner), g.n_tof), dim3(256), 0, stream, W, scale, sens, inner,
                     sens_tof, out);
  return hipGetLastError();
}

hipError_t launch_norm_ratio(const PostParams& g, const double* W, double scale, float* norm, hipStream_t stream) {
  const uint64_t n = inner_bins(g) * static_cast<uint64_t>(g.n_tof);
  hipLaunchKernelGGL(norm_ratio_kernel, dim3(blocks_for(n)), dim3(256), 0, stream, W, scale, norm, n);
  return hipGetLastError();
}

hipError_t launch_smooth_axis(const PostParams& g, int axis, const void* in, bool in_is_f64, double scale,
                              const float* norm_in, float* out, const Taps& taps, const float* norm_out,
                              const float* sens, int sens_tof, hipStream_t stream) {
  SmoothArgs a{g, in, scale, norm_in, out, norm_out, sens, sens_tof, taps};
  const uint64_t n_bins = inner_bins(g) * static_cast<uint64_t>(g.n_tof);
  if (axis < 0) {
    if (in_is_f64) hipLaunchKernelGGL(pointwise_kernel<true>, dim3(blocks_for(n_bins)), dim3(256), 0, stream, a, n_bins);
    else hipLaunchKernelGGL(pointwise_kernel<false>, dim3(blocks_for(n_bins)), dim3(256), 0, stream, a, n_bins);
    return hipGetLastError();
  }
  if (axis == 0) {
    const uint64_t rows = static_cast<uint64_t>(g.n_view) * g.n_plane * g.n_tof;
    const uint64_t jobs = rows * static_cast<uint64_t>((g.n_rad + kSeg - 1) / kSeg);
    const dim3 grid(static_cast<unsigned>((jobs + 3) / 4));
    if (in_is_f64) hipLaunchKernelGGL(smooth_rows<true>, grid, dim3(256), 0, stream, a, rows);
    else hipLaunchKernelGGL(smooth_rows<false>, grid, dim3(256), 0, stream, a, rows);
    return hipGetLastError();
  }
  const int n = axis == 1 ? g.n_view : g.n_plane;
  const int n_other = axis == 1 ? g.n_plane : g.n_view;
  const dim3 grid((g.n_rad + kTC - 1) / kTC, (n + kTL - 1) / kTL, static_cast<unsigned>(n_other * g.n_tof));
  if (axis == 1) {
    if (in_is_f64) hipLaunchKernelGGL((smooth_cols<1, true>), grid, dim3(256), 0, stream, a);
    else hipLaunchKernelGGL((smooth_cols<1, false>), grid, dim3(256), 0, stream, a);
  } else {
    if (in_is_f64) hipLaunchKernelGGL((smooth_cols<2, true>), grid, dim3(256), 0, stream, a);
    else hipLaunchKernelGGL((smooth_cols<2, false>), grid, dim3(256), 0, stream, a);
  }
  return hipGetLastError();
}

}  // namespace sse
