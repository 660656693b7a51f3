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

// Total of the estimate scale * W * sens in binary64 (sens broadcast over
// TOF when it has no TOF axis), in a fixed order: block b sums the bins of
// its contiguous chunk, thread k those at offsets k, k + 256, ... in turn,
// then a tree over the block's threads; total_final sums the kTotalBlocks
// partial sums by the same tree.  The order depends only on n, so the
// result is the same bits on every run.
constexpr int kTotalBlocks = 1024;

__device__ __forceinline__ double block_tree_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (unsigned w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(256) total_partial_kernel(const double* __restrict__ W, double scale,
                                                             const float* __restrict__ sens, uint64_t n,
                                                             uint64_t inner, int sens_tof,
                                                             double* __restrict__ partial) {
  __shared__ double sh[256];
  const uint64_t chunk = (n + kTotalBlocks - 1) / kTotalBlocks;
  const uint64_t lo = static_cast<uint64_t>(blockIdx.x) * chunk;
  const uint64_t hi = lo + chunk < n ? lo + chunk : n;
  double acc = 0.0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double sv = static_cast<double>(sens[sens_tof ? i : i % inner]);
    acc += (scale * W[i]) * sv;
  }
  const double t = block_tree_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(1024) total_final_kernel(const double* __restrict__ partial,
                                                           double* __restrict__ total) {
  __shared__ double sh[kTotalBlocks];
  const double t = block_tree_sum(partial[threadIdx.x], sh);
  if (threadIdx.x == 0) *total = t;
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
  int tile_len;           // positions per tile of the view and plane passes
};

template <bool kFromF64>
__device__ __forceinline__ float load_raw(const SmoothArgs& a, uint64_t i) {
  if (kFromF64) return static_cast<float>(a.scale * static_cast<const double*>(a.in)[i]);
  return static_cast<const float*>(a.in)[i];
}

template <bool kFromF64>
__device__ __forceinline__ float load_in(const SmoothArgs& a, uint64_t i) {
  float v = load_raw<kFromF64>(a, i);
  if (a.norm_in) v = v * a.norm_in[i];
  return v;
}

// n inputs of one thread, read at idx[b] (an index that is in range even
// where ok[b] is false) and set to 0 where ok[b] is false: all input loads
// are issued unconditionally, then all normalisation loads, then the
// products and selects, so that no wait falls between two loads.
template <bool kFromF64, int n>
__device__ __forceinline__ void load_batch(const SmoothArgs& a, const uint64_t* idx, const bool* ok, float* v) {
#pragma unroll
  for (int b = 0; b < n; ++b) v[b] = load_raw<kFromF64>(a, idx[b]);
  if (a.norm_in) {
    float f[n];
#pragma unroll
    for (int b = 0; b < n; ++b) f[b] = a.norm_in[idx[b]];
#pragma unroll
    for (int b = 0; b < n; ++b) v[b] = v[b] * f[b];
  }
#pragma unroll
  for (int b = 0; b < n; ++b) v[b] = ok[b] ? v[b] : 0.0f;
}

__device__ __forceinline__ float finish_out(const SmoothArgs& a, float acc, uint64_t o, uint64_t inner) {
  if (a.norm_out) {
    const float nrm = a.norm_out[o];
    acc = nrm > 0.0f ? acc / nrm : acc;
  }
  if (a.sens) acc = acc * a.sens[a.sens_tof ? o : o % inner];
  return acc;
}

// The output factors of bin o, read before the taps are summed so that the
// loads are in flight meanwhile; finish() then applies them as finish_out.
struct OutFactors {
  float nrm, sv;
  __device__ __forceinline__ void load(const SmoothArgs& a, uint64_t o, uint64_t inner) {
    nrm = a.norm_out ? a.norm_out[o] : 1.0f;
    sv = a.sens ? a.sens[a.sens_tof ? o : o % inner] : 1.0f;
  }
  __device__ __forceinline__ float finish(const SmoothArgs& a, float acc) const {
    if (a.norm_out) acc = nrm > 0.0f ? acc / nrm : acc;
    if (a.sens) acc = acc * sv;
    return acc;
  }
};

// Outputs per thread in the sums: each tap (a scalar load) and, along the
// view and plane axes, each staged value then serves four outputs.  The sums
// are fused multiply-adds (each product enters unrounded): one instruction
// per tap and output, and no less accurate than a product and a sum.
constexpr int kOuts = 4;
static_assert(kOuts == 4, "the sliding window of the column passes holds four values");

// Loads issued back to back before their LDS stores in the view and plane
// passes, so that each thread has this many in flight instead of one (a
// clinical tile takes two or three such rounds).
constexpr int kLoadBatch = 16;

// Passes along the view (kAxis 1) or plane (kAxis 2) axis.  A block stages
// a tile of a.tile_len positions along the axis (plus the kernel's halo) by
// kTC consecutive radial columns in LDS -- every input read once, in
// 256-byte rows, one wavefront per row -- and computes the tile's outputs
// from LDS.  The tile (dynamic LDS) is sized by the radius: the launch
// picks the longest tile_len <= 128 whose tile fits kColTileBytes (three
// blocks per CU at least; four or more for the finalize's radii).  Views
// are periodic over 180 degrees, and past the seam the same LOR is seen
// from the other end (radial and TOF indices reversed); planes reflect at
// the ends.
constexpr int kTC = 64;
constexpr int kMaxTileLen = 128;
constexpr size_t kColTileBytes = 48 * 1024;

// LDS bytes of a column-pass tile: tile_len positions (at most n), the halo,
// and kOuts - 1 rows read (unused) by the last thread's block of outputs.
size_t col_tile_bytes(int tile_len, int n, int radius) {
  const int len = tile_len < n ? tile_len : n;
  return static_cast<size_t>(len + 2 * radius + kOuts - 1) * kTC * sizeof(float);
}

template <int kAxis, bool kFromF64>
__global__ void __launch_bounds__(256) smooth_cols(SmoothArgs a) {
  extern __shared__ float tile[];
  const PostParams& g = a.g;
  const int R = a.taps.radius;
  const int n = kAxis == 1 ? g.n_view : g.n_plane;
  const int n_other = kAxis == 1 ? g.n_plane : g.n_view;
  const int r0 = blockIdx.x * kTC;
  const int p0 = blockIdx.y * a.tile_len;
  const int tl = n - p0 < a.tile_len ? n - p0 : a.tile_len;
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
  // input index of tile row i (row p0 - R + i along the axis)
  auto in_index = [&](int i) -> uint64_t {
    const int pos = p0 - R + i;
    if (kAxis == 2)
      return static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(reflect(pos, g.n_plane)) * ps +
             static_cast<uint64_t>(other) * vs + static_cast<uint64_t>(r);
    const int period = 2 * g.n_view;
    int m = pos % period;
    if (m < 0) m += period;
    return m < g.n_view ? static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(other) * ps +
                              static_cast<uint64_t>(m) * vs + static_cast<uint64_t>(r)
                        : static_cast<uint64_t>(g.n_tof - 1 - t) * ts + static_cast<uint64_t>(other) * ps +
                              static_cast<uint64_t>(m - g.n_view) * vs + static_cast<uint64_t>(g.n_rad - 1 - r);
  };
  for (int i0 = sub; i0 < rows; i0 += kLoadBatch * kRowsPerSweep) {
    uint64_t idx[kLoadBatch];
    bool ok[kLoadBatch];
    float v[kLoadBatch];
#pragma unroll
    for (int b = 0; b < kLoadBatch; ++b) {
      const int i = i0 + b * kRowsPerSweep;
      ok[b] = i < rows && r < g.n_rad;
      idx[b] = ok[b] ? in_index(i) : 0;
    }
    load_batch<kFromF64, kLoadBatch>(a, idx, ok, v);
#pragma unroll
    for (int b = 0; b < kLoadBatch; ++b) {
      const int i = i0 + b * kRowsPerSweep;
      if (i < rows) tile[i * kTC + col] = v[b];
    }
  }
  __syncthreads();
  if (r >= g.n_rad) return;
  // outputs i0 .. i0 + kOuts - 1 (those below tl are stored): a window of
  // kOuts staged values slides down the tile, each output summing its taps
  // in order k = 0 .. 2R as a one-output loop would
  for (int i0 = kOuts * sub; i0 < tl; i0 += kOuts * kRowsPerSweep) {
    uint64_t o[kOuts];
    OutFactors f[kOuts];
#pragma unroll
    for (int j = 0; j < kOuts; ++j) {
      const int pos = p0 + (i0 + j < tl ? i0 + j : i0);
      o[j] = kAxis == 2 ? static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(pos) * ps +
                              static_cast<uint64_t>(other) * vs + static_cast<uint64_t>(r)
                        : static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(other) * ps +
                              static_cast<uint64_t>(pos) * vs + static_cast<uint64_t>(r);
      f[j].load(a, o[j], ts);
    }
    float acc[kOuts] = {};
    float x0 = tile[i0 * kTC + col], x1 = tile[(i0 + 1) * kTC + col], x2 = tile[(i0 + 2) * kTC + col];
    for (int k = 0; k <= 2 * R; ++k) {
      const float w = a.taps.w[k];
      const float x3 = tile[(i0 + k + 3) * kTC + col];
      acc[0] = __builtin_fmaf(w, x0, acc[0]);
      acc[1] = __builtin_fmaf(w, x1, acc[1]);
      acc[2] = __builtin_fmaf(w, x2, acc[2]);
      acc[3] = __builtin_fmaf(w, x3, acc[3]);
      x0 = x1;
      x1 = x2;
      x2 = x3;
    }
#pragma unroll
    for (int j = 0; j < kOuts; ++j)
      if (i0 + j < tl) a.out[o[j]] = f[j].finish(a, acc[j]);
  }
}

// Pass along the radial axis (contiguous rows, reflected at both ends): each
// wavefront stages a segment of kSeg outputs of one row plus the halo in LDS.
constexpr int kSeg = 256;
static_assert(kSeg == 64 * kOuts, "one block of outputs per lane covers a segment");

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
  const int n_in = len + 2 * R;
  // every load of the segment at once (at most six per lane)
  constexpr int kRowLoads = (kSeg + 2 * kMaxSmoothRadius + 63) / 64;
  uint64_t idx[kRowLoads];
  bool ok[kRowLoads];
  float v[kRowLoads];
#pragma unroll
  for (int b = 0; b < kRowLoads; ++b) {
    const int i = static_cast<int>(lane) + 64 * b;
    ok[b] = i < n_in;
    idx[b] = ok[b] ? base + static_cast<uint64_t>(reflect(s0 - R + i, g.n_rad)) : 0;
  }
  load_batch<kFromF64, kRowLoads>(a, idx, ok, v);
#pragma unroll
  for (int b = 0; b < kRowLoads; ++b) {
    const int i = static_cast<int>(lane) + 64 * b;
    if (i < n_in) buf[i] = v[b];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint64_t inner = static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane;
  // outputs lane + 64 j (kSeg = 64 kOuts: the whole segment), each tap
  // read once for all of them; reads for outputs past len stay inside buf
  const int i = static_cast<int>(lane);
  uint64_t o[kOuts];
  OutFactors f[kOuts];
#pragma unroll
  for (int j = 0; j < kOuts; ++j) {
    o[j] = base + static_cast<uint64_t>(s0 + (i + 64 * j < len ? i + 64 * j : 0));
    f[j].load(a, o[j], inner);
  }
  float acc[kOuts] = {};
  for (int k = 0; k <= 2 * R; ++k) {
    const float w = a.taps.w[k];
#pragma unroll
    for (int j = 0; j < kOuts; ++j) acc[j] = __builtin_fmaf(w, buf[i + 64 * j + k], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < kOuts; ++j)
    if (i + 64 * j < len) a.out[o[j]] = f[j].finish(a, acc[j]);
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

hipError_t launch_total_scatter(const PostParams& g, const double* W, double scale, const float* sens, int sens_tof,
                                double* partial, double* total, hipStream_t stream) {
  const uint64_t inner = static_cast<uint64_t>(g.n_rad) * g.n_view * g.n_plane;
  const uint64_t n = inner * static_cast<uint64_t>(g.n_tof);
  hipLaunchKernelGGL(total_partial_kernel, dim3(kTotalBlocks), dim3(256), 0, stream, W, scale, sens, n, inner,
                     sens_tof, partial);
  hipLaunchKernelGGL(total_final_kernel, dim3(1), dim3(kTotalBlocks), 0, stream, partial, total);
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
  SmoothArgs a{g, in, scale, norm_in, out, norm_out, sens, sens_tof, taps, 0};
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
  int tile_len = kMaxTileLen;
  while (tile_len > 16 && col_tile_bytes(tile_len, n, taps.radius) > kColTileBytes) tile_len /= 2;
  a.tile_len = tile_len;
  const size_t lds = col_tile_bytes(tile_len, n, taps.radius);  // <= kColTileBytes up to radius 63
  const dim3 grid((g.n_rad + kTC - 1) / kTC, (n + tile_len - 1) / tile_len, static_cast<unsigned>(n_other * g.n_tof));
  if (axis == 1) {
    if (in_is_f64) hipLaunchKernelGGL((smooth_cols<1, true>), grid, dim3(256), lds, stream, a);
    else hipLaunchKernelGGL((smooth_cols<1, false>), grid, dim3(256), lds, stream, a);
  } else {
    if (in_is_f64) hipLaunchKernelGGL((smooth_cols<2, true>), grid, dim3(256), lds, stream, a);
    else hipLaunchKernelGGL((smooth_cols<2, false>), grid, dim3(256), lds, stream, a);
  }
  return hipGetLastError();
}

}  // namespace sse
