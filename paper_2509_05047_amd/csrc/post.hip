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

#include <type_traits>

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
  const double* ratio_w;  // the output becomes out / float(scale ratio_w), 1 where
                          // either is not positive (or NULL: no ratio)
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

// The ratio G / S of a smoothed value G and S = float(scale w), or 1 where
// either is not positive.
__device__ __forceinline__ float smoothing_ratio(float g, float s) { return (s > 0.0f && g > 0.0f) ? g / s : 1.0f; }

__device__ __forceinline__ float finish_out(const SmoothArgs& a, float acc, uint64_t o, uint64_t inner) {
  if (a.norm_out) {
    const float nrm = a.norm_out[o];
    acc = nrm > 0.0f ? acc / nrm : acc;
  }
  if (a.sens) acc = acc * a.sens[a.sens_tof ? o : o % inner];
  if (a.ratio_w) acc = smoothing_ratio(acc, static_cast<float>(a.scale * a.ratio_w[o]));
  return acc;
}

// What a pass does to its outputs (a template argument, so that each kernel
// holds only the factors it applies): nothing, the normalisation and
// sensitivity factors, or the ratio to float(scale ratio_w).
constexpr int kOutPlain = 0, kOutFinish = 1, kOutRatio = 2;

// The output factors of bin o, read before the taps are summed so that the
// loads are in flight meanwhile; finish() then applies them as finish_out.
template <int kOut>
struct OutFactors {
  __device__ __forceinline__ void load(const SmoothArgs&, uint64_t, uint64_t) {}
  __device__ __forceinline__ float finish(const SmoothArgs&, float acc) const { return acc; }
};
template <>
struct OutFactors<kOutFinish> {
  float nrm, sv;
  // o: the bin; o_inner: the same bin without its TOF offset
  __device__ __forceinline__ void load(const SmoothArgs& a, uint64_t o, uint64_t o_inner) {
    nrm = a.norm_out ? a.norm_out[o] : 1.0f;
    sv = a.sens ? a.sens[a.sens_tof ? o : o_inner] : 1.0f;
  }
  __device__ __forceinline__ float finish(const SmoothArgs& a, float acc) const {
    if (a.norm_out) acc = nrm > 0.0f ? acc / nrm : acc;
    if (a.sens) acc = acc * sv;
    return acc;
  }
};
template <>
struct OutFactors<kOutRatio> {
  double rw;
  __device__ __forceinline__ void load(const SmoothArgs& a, uint64_t o, uint64_t) { rw = a.ratio_w[o]; }
  __device__ __forceinline__ float finish(const SmoothArgs& a, float acc) const {
    return smoothing_ratio(acc, static_cast<float>(a.scale * rw));
  }
};

// Outputs per lane in the radial pass of the one-axis route (each tap, a
// scalar load, serves four).  All sums are fused multiply-adds (each product
// enters unrounded): one instruction per tap and output, and no less accurate
// than a product and a sum.
constexpr int kOuts = 4;

// Loads issued back to back before their LDS stores in the view and plane
// passes, so that each thread has this many in flight instead of one (a
// clinical tile takes two or three such rounds).
constexpr int kLoadBatch = 16;

// Outputs per thread and item in the view, plane and fused passes.  Along
// the sum each staged value serves kWin outputs and each block of four taps
// (one 16-byte LDS read) 4 kWin fused multiply-adds, which keeps the LDS
// traffic well under its bandwidth.
constexpr int kWin = 8;

// s[j] += sum over k = 0 .. n - 1 (in that order) of w[k] x[(j + k) stride],
// j < kO: a window of staged values slides along the sum, four taps per
// step.  w (the taps, 16-byte aligned) and x are in LDS, so the loop waits
// only on LDS reads, which return in order.
template <int kO>
__device__ __forceinline__ void window_sums(const float* x, int stride, const float* w, int n, float (&s)[kO]) {
  float win[kO + 3];  // x[k .. k + kO + 2]
#pragma unroll
  for (int i = 0; i < kO - 1; ++i) win[i] = x[i * stride];
  int k = 0;
#pragma unroll 2
  for (; k + 4 <= n; k += 4) {
    const float4 w4 = *reinterpret_cast<const float4*>(w + k);
#pragma unroll
    for (int i = 0; i < 4; ++i) win[kO - 1 + i] = x[(k + kO - 1 + i) * stride];
    const float wt[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < kO; ++j) s[j] = __builtin_fmaf(wt[t], win[j + t], s[j]);
#pragma unroll
    for (int i = 0; i < kO - 1; ++i) win[i] = win[i + 4];
  }
  for (; k < n; ++k) {
    const float wk = w[k];
    win[kO - 1] = x[(k + kO - 1) * stride];
#pragma unroll
    for (int j = 0; j < kO; ++j) s[j] = __builtin_fmaf(wk, win[j], s[j]);
#pragma unroll
    for (int i = 0; i < kO - 1; ++i) win[i] = win[i + 1];
  }
}

// The taps of a pass copied into LDS (block-wide; a barrier must follow
// before they are read).
__device__ __forceinline__ void stage_taps(const Taps& t, float* dst) {
  for (int k = static_cast<int>(threadIdx.x); k < 2 * t.radius + 1; k += static_cast<int>(blockDim.x)) dst[k] = t.w[k];
}

// Passes along the view (kAxis 1) or plane (kAxis 2) axis.  A block stages
// a tile of a.tile_len positions along the axis (plus the kernel's halo) by
// kTC consecutive radial columns in LDS -- every input read once, in
// 256-byte rows, one wavefront per row -- and computes the tile's outputs
// from LDS.  The tile (dynamic LDS) is sized by the radius: the launch
// picks the longest tile_len <= 128 whose tile fits col_tile_limit() (two
// 512-thread blocks per CU, the register budget's limit, or one tile of
// kColTileBytesSmall on a device with less LDS).  Views
// are periodic over 180 degrees, and past the seam the same LOR is seen
// from the other end (radial and TOF indices reversed); planes reflect at
// the ends.
//
// Block b serves tile (b / 8) % T of slab 8 (b / 8T) + b % 8 (a slab: one
// TOF bin and one position on the other axis; T tiles: column tiles times
// axis tiles): workgroups go round-robin over the eight XCDs, so the tiles
// of one slab run on one XCD one after another, and a tile's halo rows and
// the cache lines it shares with the neighbouring column tiles (rows are not
// line-aligned) are the neighbours' data in that L2.  With output factors
// (the last pass) every thread reads the factors of all its outputs before
// it stages the tile, so that their latency overlaps the staging loads
// instead of stalling each block of outputs.  (A persistent,
// pipelined form of this pass, like the fused radial and plane pass, measured
// no faster: its tiles are short sums over few taps.)
constexpr int kTC = 64;
constexpr int kMaxTileLen = 128;
constexpr size_t kColTileBytes = 78 * 1024;
constexpr size_t kColTileBytesSmall = 48 * 1024;
constexpr int kColThreads = 512;
constexpr int kColMinBlocks = 3;  // minimum waves per SIMD the register budget allows for
constexpr int kColRowsPerSweep = kColThreads / kTC;
constexpr int kColGroups = kMaxTileLen / (kWin * kColRowsPerSweep);  // output blocks per thread

// LDS bytes of a column-pass tile: tile_len positions (at most n), the halo,
// and kWin - 1 rows read (unused) by the last thread's block of outputs.
size_t col_tile_bytes(int tile_len, int n, int radius) {
  const int len = tile_len < n ? tile_len : n;
  return static_cast<size_t>(len + 2 * radius + kWin - 1) * kTC * sizeof(float);
}

__device__ __forceinline__ bool xcd_tile(uint32_t b, uint32_t T, uint32_t n_groups, uint32_t& group, uint32_t& tile) {
  group = (b / (8u * T)) * 8u + (b & 7u);
  tile = (b >> 3) % T;
  return group < n_groups;
}

// Position i (any integer) folded into [0, 2n) by whole periods: the halos
// reach at most kMaxSmoothRadius past an end, so this takes one step or
// none unless the axis is shorter than the radius.
__device__ __forceinline__ int fold(int i, int n) {
  const int period = 2 * n;
  while (i < 0) i += period;
  while (i >= period) i -= period;
  return i;
}

// Binary32 input value at element offset o of a row that starts at element
// `row` (the scaled and rounded binary64 weight, or the binary32 input).
template <bool kFromF64>
__device__ __forceinline__ float raw_at(const SmoothArgs& a, uint64_t row, uint32_t o) {
  if (kFromF64) return static_cast<float>(a.scale * (static_cast<const double*>(a.in) + row)[o]);
  return (static_cast<const float*>(a.in) + row)[o];
}

template <int kAxis, bool kFromF64, int kOut>
__global__ void __launch_bounds__(kColThreads, kColMinBlocks) smooth_cols(SmoothArgs a, int n_col_tiles, int n_axis_tiles) {
  extern __shared__ float tile[];
  __shared__ __align__(16) float tw[2 * kMaxSmoothRadius + 4];
  const PostParams& g = a.g;
  const int R = a.taps.radius;
  const int n = kAxis == 1 ? g.n_view : g.n_plane;
  const int n_other = kAxis == 1 ? g.n_plane : g.n_view;
  uint32_t group, tile_id;
  if (!xcd_tile(blockIdx.x, static_cast<uint32_t>(n_col_tiles * n_axis_tiles),
                static_cast<uint32_t>(n_other * g.n_tof), group, tile_id))
    return;
  // block-uniform geometry
  const int xt = static_cast<int>(tile_id % static_cast<uint32_t>(n_col_tiles));
  const uint32_t ytile = tile_id / static_cast<uint32_t>(n_col_tiles);
  const int z = static_cast<int>(group);
  const int r0 = xt * kTC;
  const int p0 = static_cast<int>(ytile) * a.tile_len;
  const int tl = n - p0 < a.tile_len ? n - p0 : a.tile_len;
  const int t = z / n_other;
  const int other = z - t * n_other;
  const uint64_t vs = static_cast<uint64_t>(g.n_rad);
  const uint64_t ps = vs * g.n_view;
  const uint64_t ts = ps * g.n_plane;
  const uint64_t ax = kAxis == 1 ? vs : ps;                     // stride along the axis
  const uint64_t other_off = kAxis == 1 ? other * ps : other * vs;
  const uint64_t out0 = static_cast<uint64_t>(t) * ts + other_off + static_cast<uint64_t>(p0) * ax;
  // per lane: the radial column (clamped into the row for lanes past its end)
  const int col = static_cast<int>(threadIdx.x & (kTC - 1));
  const int sub = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kTC));  // the wave
  const int r = r0 + col;
  const bool live = r < g.n_rad;
  const uint32_t rc = static_cast<uint32_t>(live ? r : g.n_rad - 1);
  const uint32_t rflip = static_cast<uint32_t>(g.n_rad - 1) - rc;
  const int rows = tl + 2 * R;
  stage_taps(a.taps, tw);
  // outputs i0 .. i0 + kWin - 1 of block q: i0 = kWin (sub + kColRowsPerSweep q)
  OutFactors<kOut> f[kOut ? kColGroups : 1][kWin];
  if (kOut && live) {
#pragma unroll
    for (int q = 0; q < kColGroups; ++q) {
      const int i0 = kWin * (sub + kColRowsPerSweep * q);
      if (i0 < tl) {
#pragma unroll
        for (int j = 0; j < kWin; ++j) {
          const uint64_t o = out0 + static_cast<uint64_t>(i0 + j < tl ? i0 + j : i0) * ax + rc;
          f[q][j].load(a, o, o - static_cast<uint64_t>(t) * ts);
        }
      }
    }
  }
  // Stage: the wave's rows i = sub + 4 k (tile row i is position p0 - R + i
  // along the axis); row offsets are wave-uniform, only the column varies.
  for (int i0 = sub; i0 < rows; i0 += kLoadBatch * kColRowsPerSweep) {
    uint64_t roff[kLoadBatch];
    uint32_t c[kLoadBatch];
#pragma unroll
    for (int b = 0; b < kLoadBatch; ++b) {
      const int i = i0 + b * kColRowsPerSweep;
      const int pos = p0 - R + (i < rows ? i : rows - 1);
      if (kAxis == 2) {
        const int m = fold(pos, g.n_plane);
        const int pl = m < g.n_plane ? m : 2 * g.n_plane - 1 - m;
        roff[b] = static_cast<uint64_t>(t) * ts + static_cast<uint64_t>(pl) * ps + other_off;
        c[b] = rc;
      } else {
        const int m = fold(pos, g.n_view);  // past the seam: the other end of the LOR
        const bool flip = m >= g.n_view;
        roff[b] = static_cast<uint64_t>(flip ? g.n_tof - 1 - t : t) * ts + other_off +
                  static_cast<uint64_t>(flip ? m - g.n_view : m) * vs;
        c[b] = flip ? rflip : rc;
      }
    }
    float v[kLoadBatch];
#pragma unroll
    for (int b = 0; b < kLoadBatch; ++b)
      if (i0 + b * kColRowsPerSweep < rows) v[b] = raw_at<kFromF64>(a, roff[b], c[b]);
    if (a.norm_in) {
      float nv[kLoadBatch];
#pragma unroll
      for (int b = 0; b < kLoadBatch; ++b)
        if (i0 + b * kColRowsPerSweep < rows) nv[b] = (a.norm_in + roff[b])[c[b]];
#pragma unroll
      for (int b = 0; b < kLoadBatch; ++b) v[b] = v[b] * nv[b];
    }
#pragma unroll
    for (int b = 0; b < kLoadBatch; ++b) {
      const int i = i0 + b * kColRowsPerSweep;
      if (i < rows) tile[i * kTC + col] = v[b];
    }
  }
  __syncthreads();
  if (!live) return;
  // a window of staged values slides down the tile, each output summing its
  // taps in order k = 0 .. 2R as a one-output loop would
#pragma unroll
  for (int q = 0; q < kColGroups; ++q) {
    const int i0 = kWin * (sub + kColRowsPerSweep * q);
    if (i0 >= tl) break;
    float acc[kWin] = {};
    window_sums<kWin>(tile + i0 * kTC + col, kTC, tw, 2 * R + 1, acc);
#pragma unroll
    for (int j = 0; j < kWin; ++j)
      if (i0 + j < tl)
        (a.out + out0 + static_cast<uint64_t>(i0 + j) * ax)[rc] =
            f[kOut ? q : 0][j].finish(a, acc[j]);
  }
}

// Pass along the radial axis (contiguous rows, reflected at both ends): each
// wavefront stages a segment of kSeg outputs of one row plus the halo in LDS.
constexpr int kSeg = 256;
static_assert(kSeg == 64 * kOuts, "one block of outputs per lane covers a segment");

template <bool kFromF64, int kOut>
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
  const uint64_t tof_off = row / (static_cast<uint64_t>(g.n_view) * g.n_plane) * inner;
  // outputs lane + 64 j (kSeg = 64 kOuts: the whole segment), each tap
  // read once for all of them; reads for outputs past len stay inside buf
  const int i = static_cast<int>(lane);
  uint64_t o[kOuts];
  OutFactors<kOut> f[kOuts];
#pragma unroll
  for (int j = 0; j < kOuts; ++j) {
    o[j] = base + static_cast<uint64_t>(s0 + (i + 64 * j < len ? i + 64 * j : 0));
    f[j].load(a, o[j], o[j] - tof_off);
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

// Radial and plane passes fused over one (TOF, view) row: a tile of f.tl
// radial positions by every plane, plus the radial halo (reflected at the
// row ends), is staged in LDS; the rows are smoothed radially and stored in
// a second LDS region, each plane also into the slots of the plane halo
// that reflect it, and the columns are smoothed along the planes from
// there.  HBM sees the input once (plus the radial halo, which the tile's
// neighbours on the same XCD read at about the same time) and the output
// once: the intermediate never leaves the CU.
//
// The kernel is persistent, one 1024-thread block per CU, and pipelined:
// while a block smooths one tile, the loads of its next tile are in flight
// into registers, so the CU's memory traffic overlaps its arithmetic instead
// of alternating with it.  With the two regions apart a tile takes two
// barriers: the next staging writes only the first region, so it does not
// wait for the plane sums, and no radial sum is held across a barrier.
//
// Radial outputs come in blocks of kFusedWin per thread (sliding window,
// lanes on consecutive planes: the row stride is odd, so the lanes hit
// distinct banks); plane outputs likewise, lanes on consecutive radial
// positions, from the radially smoothed values stored one radial position's
// planes after another, so that both sums read LDS at unit stride and the
// window loads take immediate offsets.  Both sums run their taps in the
// order k = 0 .. 2R as the one-axis passes do.
struct FusedArgs {
  SmoothArgs a;   // a.taps: the radial taps
  Taps plane;     // the plane taps
  int tl;         // radial outputs per tile (<= kFusedMaxTile)
  int n_tiles;    // tiles per (TOF, view) row
  int sx;         // LDS row stride of the staged input (odd, >= tl + 2 R + kFusedWin - 1)
  int sy;         // LDS stride between radial positions of the radially smoothed columns (odd, >= np + 2 Rp + kFusedWin - 1)
  int y0;         // LDS float offset of the smoothed columns (after the np sx staged floats)
  uint32_t n_units;  // tile slots of the XCD mapping (8 ceil(rows / 8) n_tiles)
};
constexpr int kFusedThreads = 1024;
constexpr int kFusedWaves = kFusedThreads / 64;
constexpr int kFusedPrefetch = 16;                          // staged elements per thread
constexpr int kFusedStage = kFusedThreads * kFusedPrefetch;  // staged elements per tile
constexpr int kFusedWin = kWin;  // outputs per thread and item
constexpr int kFusedItems = 2;   // radial output blocks per thread
constexpr int kFusedMaxTile = 128;

// One tile's geometry.
struct FusedTile {
  int t, r0, tl, wx;
  uint64_t row0;  // element offset of (t, plane 0, view, column 0)
};

__device__ __forceinline__ bool fused_tile(const FusedArgs& f, uint32_t u, FusedTile& ft) {
  const PostParams& g = f.a.g;
  uint32_t row, tile;
  if (!xcd_tile(u, static_cast<uint32_t>(f.n_tiles), static_cast<uint32_t>(g.n_view) * static_cast<uint32_t>(g.n_tof),
                row, tile))
    return false;
  ft.t = static_cast<int>(row / static_cast<uint32_t>(g.n_view));
  const int v = static_cast<int>(row) - ft.t * g.n_view;
  ft.r0 = static_cast<int>(tile) * f.tl;
  ft.tl = g.n_rad - ft.r0 < f.tl ? g.n_rad - ft.r0 : f.tl;
  ft.wx = ft.tl + 2 * f.a.taps.radius;
  const uint64_t vs = static_cast<uint64_t>(g.n_rad);
  ft.row0 = static_cast<uint64_t>(ft.t) * vs * g.n_view * g.n_plane + static_cast<uint64_t>(v) * vs;
  return true;
}

// The next unit of this block at or after u that holds a tile (n_units if none).
__device__ __forceinline__ uint32_t fused_next(const FusedArgs& f, uint32_t u, FusedTile& ft) {
  for (; u < f.n_units; u += gridDim.x)
    if (fused_tile(f, u, ft)) return u;
  return f.n_units;
}

// The value of type T at element offset o past base, the byte offset taken
// in 32 bits (the planner keeps every offset within a (TOF, view) row's
// planes below 2^32 bytes), so that the address is a uniform base plus a
// 32-bit lane offset.
template <class T>
__device__ __forceinline__ T load_at(const T* base, uint32_t o) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + o * static_cast<uint32_t>(sizeof(T)));
}

// Prefetch registers of one staged tile: element e = threadIdx.x + 1024 i
// is plane e / wx, staged column e % wx (stepped without division).  Every
// element slot is loaded (slots past the tile from a clamped, valid index,
// never stored), so that the loads are straight-line code and nothing waits
// between them.
template <bool kFromF64, bool kNormIn>
struct FusedPrefetch {
  using Raw = typename std::conditional<kFromF64, double, float>::type;
  Raw w[kFusedPrefetch];
  float nrm[kNormIn ? kFusedPrefetch : 1];

  // ps: the plane stride in elements (below 2^24, by the planner)
  __device__ __forceinline__ void issue(const SmoothArgs& a, const FusedTile& ft, int np, uint32_t ps) {
    const int dp = kFusedThreads / ft.wx, dc = kFusedThreads % ft.wx;
    int p = static_cast<int>(threadIdx.x) / ft.wx, c = static_cast<int>(threadIdx.x) % ft.wx;
    const Raw* in = static_cast<const Raw*>(a.in) + ft.row0;
    const float* nin = a.norm_in + ft.row0;
    const int n_rad = a.g.n_rad;
    const int c0 = ft.r0 - a.taps.radius;
#pragma unroll
    for (int i = 0; i < kFusedPrefetch; ++i) {
      // one reflection at most: the planner keeps the radius <= n_rad
      int col = c0 + c;
      col = col < 0 ? -col - 1 : col;
      col = col >= n_rad ? 2 * n_rad - 1 - col : col;
      const int pc = p < np ? p : np - 1;
      const uint32_t o = __umul24(static_cast<uint32_t>(pc), ps) + static_cast<uint32_t>(col);
      w[i] = load_at(in, o);
      if (kNormIn) nrm[kNormIn ? i : 0] = load_at(nin, o);
      p += dp;
      c += dc;
      if (c >= ft.wx) {
        c -= ft.wx;
        ++p;
      }
    }
  }

  __device__ __forceinline__ void store(const SmoothArgs& a, const FusedTile& ft, int np, int sx, float* lds) const {
    const int n = np * ft.wx;
    const int dp = kFusedThreads / ft.wx, dc = kFusedThreads % ft.wx;
    int p = static_cast<int>(threadIdx.x) / ft.wx, c = static_cast<int>(threadIdx.x) % ft.wx;
#pragma unroll
    for (int i = 0; i < kFusedPrefetch; ++i) {
      const int e = static_cast<int>(threadIdx.x) + kFusedThreads * i;
      float x = kFromF64 ? static_cast<float>(a.scale * static_cast<double>(w[i])) : static_cast<float>(w[i]);
      if (kNormIn) x = x * nrm[kNormIn ? i : 0];
      if (e < n) lds[p * sx + c] = x;
      p += dp;
      c += dc;
      if (c >= ft.wx) {
        c -= ft.wx;
        ++p;
      }
    }
  }
};

template <bool kFromF64, bool kNormIn, int kOut>
__global__ void __launch_bounds__(kFusedThreads, 1) smooth_rad_plane(FusedArgs f) {
  extern __shared__ float lds[];
  __shared__ __align__(16) float tw_r[2 * kMaxSmoothRadius + 4];
  __shared__ __align__(16) float tw_p[2 * kMaxSmoothRadius + 4];
  const SmoothArgs& a = f.a;
  const PostParams& g = a.g;
  const int Rr = a.taps.radius, Rp = f.plane.radius;
  const int np = g.n_plane;
  stage_taps(a.taps, tw_r);  // read after the first barrier below
  stage_taps(f.plane, tw_p);
  const uint32_t ps = static_cast<uint32_t>(g.n_rad) * static_cast<uint32_t>(g.n_view);
  const uint64_t ts = static_cast<uint64_t>(ps) * g.n_plane;
  const int lane = static_cast<int>(threadIdx.x & 63u);
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int y_rows = np + 2 * Rp + kFusedWin - 1;  // smoothed planes and plane halo
  // the halo rows are written with the planes they reflect when one
  // reflection reaches them all, else copied in a pass of their own
  const bool direct_halo = Rp + kFusedWin - 1 <= np;

  FusedTile cur, nxt;
  uint32_t u = fused_next(f, blockIdx.x, cur);
  if (u >= f.n_units) return;
  FusedPrefetch<kFromF64, kNormIn> pre;
  pre.issue(a, cur, np, ps);
  float* const ys = lds + f.y0;  // the radially smoothed values, after the staged input
  while (true) {
    // The staged input was last read by the previous tile's radial sums,
    // before the barrier that preceded its plane sums: it may be
    // overwritten while other waves still sum planes.
    pre.store(a, cur, np, f.sx, lds);
    __syncthreads();  // staged; and the previous tile's plane sums are done with ys
    const uint32_t un = fused_next(f, u + gridDim.x, nxt);
    if (un < f.n_units) pre.issue(a, nxt, np, ps);  // in flight while this tile is smoothed
    const int tl = cur.tl;

    // Radial sums: item i = threadIdx.x + 1024 m is plane i % np, outputs
    // kFusedWin (i / np) .. + kFusedWin - 1 of the tile, stored as soon as
    // they are summed.  The radially smoothed values are kept by radial
    // position: column c holds y_rows consecutive floats, plane p at Rp + p
    // and, with direct_halo, also at the halo slots that reflect it:
    // Rp - 1 - p (p < Rp) and Rp + 2 np - 1 - p (when below y_rows; the last
    // kFusedWin - 1 halo slots are read only by outputs past the final
    // plane).  Lanes on consecutive planes write consecutive floats.
    const int n_ch = (tl + kFusedWin - 1) / kFusedWin;
    const int dp = kFusedThreads % np, dch = kFusedThreads / np;
    {
      int p = static_cast<int>(threadIdx.x) % np, ch = static_cast<int>(threadIdx.x) / np;
#pragma unroll
      for (int m = 0; m < kFusedItems; ++m) {
        if (ch < n_ch) {
          float acc[kFusedWin] = {};
          window_sums<kFusedWin>(lds + p * f.sx + kFusedWin * ch, 1, tw_r, 2 * Rr + 1, acc);
          const int c0 = kFusedWin * ch;
          // The store addresses do not change from tile to tile; computed
          // here (the empty asm hides that) rather than hoisted out of the
          // tile loop, where 48 of them would take registers the prefetch
          // needs and spill.
          int col = c0 * f.sy;
          asm volatile("" : "+v"(col));
          float* yr = ys + col + (Rp + p);
          float* ytop = ys + col + (Rp - 1 - p);
          float* ybot = ys + col + (Rp + 2 * np - 1 - p);
          const bool top = direct_halo && p < Rp;
          const bool bot = direct_halo && Rp + 2 * np - 1 - p < y_rows;
#pragma unroll
          for (int j = 0; j < kFusedWin; ++j)
            if (c0 + j < tl) {
              yr[j * f.sy] = acc[j];
              if (top) ytop[j * f.sy] = acc[j];
              if (bot) ybot[j * f.sy] = acc[j];
            }
        }
        p += dp;
        ch += dch;
        if (p >= np) {
          p -= np;
          ++ch;
        }
      }
    }
    __syncthreads();  // the staged input is read: the next staging may overwrite it
    if (!direct_halo) {  // halo slots by folding (radius near the plane count)
      for (int h = wave; h < 2 * Rp + kFusedWin - 1; h += kFusedWaves) {
        const int e = h < Rp ? h : np + h;
        const int m = fold(e - Rp, np);
        const int src = Rp + (m < np ? m : 2 * np - 1 - m);
        for (int c = lane; c < tl; c += 64) ys[c * f.sy + e] = ys[c * f.sy + src];
      }
      __syncthreads();
    }

    // Plane sums: item i is radial position i % tl, planes kFusedWin (i / tl)
    // .. + kFusedWin - 1, summed along its column (unit stride, as the radial
    // sums; the lanes' columns lie an odd stride apart, in distinct banks).
    const int n_pg = (np + kFusedWin - 1) / kFusedWin;
    float* out_row = a.out + cur.row0 + static_cast<uint64_t>(cur.r0);  // plane 0 of the tile
    const int dc = kFusedThreads % tl, dpg = kFusedThreads / tl;
    int c = static_cast<int>(threadIdx.x) % tl, pg = static_cast<int>(threadIdx.x) / tl;
    while (pg < n_pg) {
      OutFactors<kOut> fo[kOut ? kFusedWin : 1];
      if (kOut) {
#pragma unroll
        for (int j = 0; j < kFusedWin; ++j) {
          const int p = kFusedWin * pg + j < np ? kFusedWin * pg + j : kFusedWin * pg;
          const uint64_t o = cur.row0 + static_cast<uint64_t>(p) * ps + static_cast<uint64_t>(cur.r0 + c);
          fo[kOut ? j : 0].load(a, o, o - static_cast<uint64_t>(cur.t) * ts);
        }
      }
      float sm[kFusedWin] = {};
      window_sums<kFusedWin>(ys + c * f.sy + kFusedWin * pg, 1, tw_p, 2 * Rp + 1, sm);
#pragma unroll
      for (int j = 0; j < kFusedWin; ++j)
        if (kFusedWin * pg + j < np)
          *reinterpret_cast<float*>(reinterpret_cast<char*>(out_row) +
                                    (__umul24(static_cast<uint32_t>(kFusedWin * pg + j), ps) +
                                     static_cast<uint32_t>(c)) * 4u) = fo[kOut ? j : 0].finish(a, sm[j]);
      c += dc;
      pg += dpg;
      if (c >= tl) {
        c -= tl;
        ++pg;
      }
    }
    if (un >= f.n_units) break;
    u = un;
    cur = nxt;
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

namespace {
// Compute units and LDS bytes per block of the current device (the
// persistent kernels run one block per CU), cached per device.
struct DeviceShape {
  int cus;
  size_t lds;
};
DeviceShape device_shape() {
  static DeviceShape cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DeviceShape{256, 64 * 1024};
  if (!cached[dev].cus) {
    int cus = 0, lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0)
      lds = 64 * 1024;
    cached[dev] = DeviceShape{cus, static_cast<size_t>(lds)};
  }
  return cached[dev];
}
int device_cus() { return device_shape().cus; }
}  // namespace

namespace {
// LDS bytes of one column-pass tile: two tiles of kColTileBytes per CU when
// the device's LDS holds them, else kColTileBytesSmall.
size_t col_tile_limit() {
  const size_t dev = device_shape().lds;
  const size_t static_lds = (2 * kMaxSmoothRadius + 4) * sizeof(float);  // the tap array
  return dev >= 2 * (kColTileBytes + static_lds) ? kColTileBytes : kColTileBytesSmall;
}
}  // namespace

size_t fused_lds_limit() {
  const size_t dev = device_shape().lds;
  const size_t static_lds = 2 * (2 * kMaxSmoothRadius + 4) * sizeof(float);  // the two tap arrays
  const size_t avail = dev > static_lds ? dev - static_lds : 0;
  return avail < kFusedLdsBytes ? avail : kFusedLdsBytes;
}

FusedPlan plan_rad_plane(const PostParams& g, int radial_radius, int plane_radius) {
  FusedPlan pl{};
  if (g.n_plane <= 0 || g.n_rad <= 0 || radial_radius > g.n_rad) return pl;
  // offsets within a (TOF, view) row's planes: 24-bit plane strides and
  // 32-bit byte offsets of binary64 elements
  const uint64_t plane_stride = static_cast<uint64_t>(g.n_rad) * static_cast<uint64_t>(g.n_view);
  if (plane_stride >= (1ull << 24) || plane_stride * static_cast<uint64_t>(g.n_plane) * sizeof(double) >= (1ull << 32))
    return pl;
  const size_t lds_max = fused_lds_limit();
  for (int k = (g.n_rad + kFusedMaxTile - 1) / kFusedMaxTile;; ++k) {  // k tiles of about equal length
    const int tl = (g.n_rad + k - 1) / k;
    const int n_tiles = (g.n_rad + tl - 1) / tl;
    if (tl < 16 && tl < g.n_rad) break;  // halo-dominated: the one-axis passes do better
    const int64_t radial_items = static_cast<int64_t>(g.n_plane) * ((tl + kFusedWin - 1) / kFusedWin);
    if (radial_items > static_cast<int64_t>(kFusedThreads) * kFusedItems) continue;
    if (static_cast<int64_t>(g.n_plane) * (tl + 2 * radial_radius) > kFusedStage) continue;
    const int sx = (tl + 2 * radial_radius + kFusedWin - 1) | 1;
    const int sy = (g.n_plane + 2 * plane_radius + kFusedWin - 1) | 1;
    const size_t x_floats = static_cast<size_t>(g.n_plane) * sx;
    const size_t y_floats = static_cast<size_t>(tl) * sy;
    const size_t lds = (x_floats + y_floats) * sizeof(float);
    if (lds <= lds_max) {
      pl.tl = tl;
      pl.n_tiles = n_tiles;
      pl.sx = sx;
      pl.sy = sy;
      pl.lds_bytes = lds;
      return pl;
    }
    if (tl == 1) break;
  }
  return pl;
}

namespace {
// The output mode of a pass (kOut*), or -1 for a ratio combined with the
// other factors, which no caller needs.
int out_mode(const float* norm_out, const float* sens, const double* ratio_w) {
  if (ratio_w) return (norm_out || sens) ? -1 : kOutRatio;
  return (norm_out || sens) ? kOutFinish : kOutPlain;
}

template <bool kF64, bool kNin>
void launch_fused(int mode, dim3 grid, size_t lds, hipStream_t stream, const FusedArgs& f) {
  if (mode == kOutRatio)
    hipLaunchKernelGGL((smooth_rad_plane<kF64, kNin, kOutRatio>), grid, dim3(kFusedThreads), lds, stream, f);
  else if (mode == kOutFinish)
    hipLaunchKernelGGL((smooth_rad_plane<kF64, kNin, kOutFinish>), grid, dim3(kFusedThreads), lds, stream, f);
  else
    hipLaunchKernelGGL((smooth_rad_plane<kF64, kNin, kOutPlain>), grid, dim3(kFusedThreads), lds, stream, f);
}

template <int kAxis, bool kF64>
void launch_cols(int mode, dim3 grid, size_t lds, hipStream_t stream, const SmoothArgs& a, int n_col_tiles,
                 int n_axis_tiles) {
  if (mode == kOutRatio)
    hipLaunchKernelGGL((smooth_cols<kAxis, kF64, kOutRatio>), grid, dim3(kColThreads), lds, stream, a, n_col_tiles,
                       n_axis_tiles);
  else if (mode == kOutFinish)
    hipLaunchKernelGGL((smooth_cols<kAxis, kF64, kOutFinish>), grid, dim3(kColThreads), lds, stream, a, n_col_tiles,
                       n_axis_tiles);
  else
    hipLaunchKernelGGL((smooth_cols<kAxis, kF64, kOutPlain>), grid, dim3(kColThreads), lds, stream, a, n_col_tiles,
                       n_axis_tiles);
}

template <bool kF64>
void launch_rows(int mode, dim3 grid, hipStream_t stream, const SmoothArgs& a, uint64_t rows) {
  if (mode == kOutRatio) hipLaunchKernelGGL((smooth_rows<kF64, kOutRatio>), grid, dim3(256), 0, stream, a, rows);
  else if (mode == kOutFinish) hipLaunchKernelGGL((smooth_rows<kF64, kOutFinish>), grid, dim3(256), 0, stream, a, rows);
  else hipLaunchKernelGGL((smooth_rows<kF64, kOutPlain>), grid, dim3(256), 0, stream, a, rows);
}
}  // namespace

hipError_t launch_smooth_rad_plane(const PostParams& g, const FusedPlan& pl, const void* in, bool in_is_f64,
                                   double scale, const float* norm_in, float* out, const Taps& radial,
                                   const Taps& plane, const float* norm_out, const float* sens, int sens_tof,
                                   const double* ratio_w, hipStream_t stream) {
  const int mode = out_mode(norm_out, sens, ratio_w);
  if (pl.tl <= 0 || mode < 0) return hipErrorInvalidValue;
  const uint64_t rows = static_cast<uint64_t>(g.n_view) * g.n_tof;
  const uint64_t units = (rows + 7) / 8 * 8 * static_cast<uint64_t>(pl.n_tiles);
  if (units == 0) return hipSuccess;
  if (units > 0xffffffffull) return hipErrorInvalidValue;
  FusedArgs f{SmoothArgs{g, in, scale, norm_in, out, norm_out, sens, sens_tof, radial, 0, ratio_w}, plane, pl.tl,
              pl.n_tiles, pl.sx, pl.sy, g.n_plane * pl.sx, static_cast<uint32_t>(units)};
  // one block per CU (a multiple of 8: a block's units stay on its XCD)
  uint64_t blocks = static_cast<uint64_t>(device_cus() + 7) / 8 * 8;
  if (blocks > units) blocks = (units + 7) / 8 * 8;
  const bool nin = norm_in != nullptr;
  const dim3 grid(static_cast<unsigned>(blocks));
  if (in_is_f64) {
    if (nin) launch_fused<true, true>(mode, grid, pl.lds_bytes, stream, f);
    else launch_fused<true, false>(mode, grid, pl.lds_bytes, stream, f);
  } else {
    if (nin) launch_fused<false, true>(mode, grid, pl.lds_bytes, stream, f);
    else launch_fused<false, false>(mode, grid, pl.lds_bytes, stream, f);
  }
  return hipGetLastError();
}

hipError_t launch_smooth_axis(const PostParams& g, int axis, const void* in, bool in_is_f64, double scale,
                              const float* norm_in, float* out, const Taps& taps, const float* norm_out,
                              const float* sens, int sens_tof, const double* ratio_w, hipStream_t stream) {
  SmoothArgs a{g, in, scale, norm_in, out, norm_out, sens, sens_tof, taps, 0, ratio_w};
  const int mode = out_mode(norm_out, sens, ratio_w);
  if (mode < 0) return hipErrorInvalidValue;
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
    if (in_is_f64) launch_rows<true>(mode, grid, stream, a, rows);
    else launch_rows<false>(mode, grid, stream, a, rows);
    return hipGetLastError();
  }
  const int n = axis == 1 ? g.n_view : g.n_plane;
  const int n_other = axis == 1 ? g.n_plane : g.n_view;
  const size_t limit = col_tile_limit();
  int tile_len = kMaxTileLen;
  while (tile_len > 16 && col_tile_bytes(tile_len, n, taps.radius) > limit) tile_len /= 2;
  a.tile_len = tile_len;
  const size_t lds = col_tile_bytes(tile_len, n, taps.radius);  // <= 38 KB at tile_len 16 and radius 63
  const int n_col_tiles = (g.n_rad + kTC - 1) / kTC;
  const int n_axis_tiles = (n + tile_len - 1) / tile_len;
  const uint64_t groups = static_cast<uint64_t>(n_other) * g.n_tof;
  const dim3 grid(static_cast<unsigned>((groups + 7) / 8 * 8 * static_cast<uint64_t>(n_col_tiles * n_axis_tiles)));
  if (axis == 1) {
    if (in_is_f64) launch_cols<1, true>(mode, grid, lds, stream, a, n_col_tiles, n_axis_tiles);
    else launch_cols<1, false>(mode, grid, lds, stream, a, n_col_tiles, n_axis_tiles);
  } else {
    if (in_is_f64) launch_cols<2, true>(mode, grid, lds, stream, a, n_col_tiles, n_axis_tiles);
    else launch_cols<2, false>(mode, grid, lds, stream, a, n_col_tiles, n_axis_tiles);
  }
  return hipGetLastError();
}

}  // namespace sse
