// Throughput microbenchmarks of the units the scatter simulation is bound by
// (vector ALU instruction kinds, random gathers through the cache levels,
// random atomic adds, a plain copy).  Declarations: include/sse_peaks.h.
//
// Every loop keeps 8 independent chains per lane so that one instruction's
// latency is hidden by the next chain's, and launches 8 blocks of 256
// threads per compute unit so that every SIMD holds several waves.  The
// instruction under test is written as inline assembly on registers only, so
// the compiler can neither fold a chain nor change the instruction count;
// the chains' results are stored so that nothing is dead.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "sse_peaks.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBlocksPerCu = 8;
constexpr int kChains = 8;
constexpr int kUnroll = 16;

enum Op { kAdd = 0, kXor, kFma, kMad64, kCnd, kLog };

template <int OP>
__global__ void __launch_bounds__(kThreads) valu_loop(uint32_t iters, uint32_t* sink, unsigned long long* clocks) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t a[kChains];
  float f[kChains];
  uint64_t m[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    a[k] = t * 2654435761u + static_cast<uint32_t>(k);
    f[k] = 1.0f + static_cast<float>(k) * 1e-3f;
    m[k] = static_cast<uint64_t>(a[k]) | (static_cast<uint64_t>(t) << 32);
  }
  const uint32_t c = t | 1u;
  const uint64_t sel = __ballot(t & 1u);  // a lane mask in scalar registers
  const float x = 0.999f, y = 1e-7f;
  uint64_t c0 = 0, r0 = 0;
  if (threadIdx.x == 0) {
    c0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        if (OP == kAdd) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(c));
        if (OP == kXor) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[k]) : "v"(c));
        if (OP == kFma) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(f[k]) : "v"(x), "v"(y));
        // (in C: the compiler's own form of the instruction, without the
        // scalar carry register that the assembly form must name)
        if (OP == kMad64) m[k] = static_cast<uint64_t>(static_cast<uint32_t>(m[k] >> 32)) * c + m[k];
        if (OP == kCnd) asm volatile("v_cndmask_b32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(c), "s"(sel));
        if (OP == kLog) asm volatile("v_log_f32 %0, %0" : "+v"(f[k]));
      }
    }
  }
  if (threadIdx.x == 0) {
    const uint64_t c1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
    if (blockIdx.x == 0) {
      clocks[0] = c1 - c0;
      clocks[1] = r1 - r0;
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    acc ^= a[k] ^ __float_as_uint(f[k]) ^ static_cast<uint32_t>(m[k] >> 7);
  }
  sink[t] = acc;
}

__device__ __forceinline__ uint32_t mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Random independent 4-byte loads, kChains in flight per lane per round.
__global__ void __launch_bounds__(kThreads) gather_loop(const uint32_t* __restrict__ buf, uint32_t mask,
                                                        uint32_t rounds, uint32_t* sink) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t h = mix(t * 0x9E3779B9u + 1u), acc = 0;
  for (uint32_t i = 0; i < rounds; ++i) {
    uint32_t v[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) {
      h = h * 1664525u + 1013904223u;
      v[k] = buf[(h ^ (h >> 13)) & mask];
    }
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc += v[k];
  }
  sink[t] = acc;
}

// Random atomic adds without return: n per lane.
template <bool kF64>
__global__ void __launch_bounds__(kThreads) atomic_loop(void* buf, uint64_t bins, uint32_t n) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t h = static_cast<uint64_t>(mix(t + 7u)) * 0x9E3779B97F4A7C15ull + t;
  for (uint32_t i = 0; i < n; ++i) {
    h = h * 6364136223846793005ull + 1442695040888963407ull;
    const uint64_t b = __umul64hi(h, bins);
    if (kF64) unsafeAtomicAdd(static_cast<double*>(buf) + b, 1.0);
    else atomicAdd(static_cast<uint32_t*>(buf) + b, 1u);
  }
}

__global__ void __launch_bounds__(kThreads) copy_loop(const uint4* __restrict__ in, uint4* __restrict__ out,
                                                      uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Timer() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  void start() { (void)hipEventRecord(a, 0); }
  double stop_s() {
    (void)hipEventRecord(b, 0);
    (void)hipEventSynchronize(b);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    return 1e-3 * static_cast<double>(ms);
  }
};

template <int OP>
hipError_t run_valu(int blocks, uint32_t iters, uint32_t* sink, unsigned long long* clocks, double& rate,
                    double& mhz) {
  Timer tm;
  hipLaunchKernelGGL(valu_loop<OP>, dim3(blocks), dim3(kThreads), 0, 0, iters / 8, sink, clocks);  // warm-up
  tm.start();
  hipLaunchKernelGGL(valu_loop<OP>, dim3(blocks), dim3(kThreads), 0, 0, iters, sink, clocks);
  const double s = tm.stop_s();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  unsigned long long ck[2] = {0, 0};
  e = hipMemcpy(ck, clocks, sizeof ck, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  const double ops = static_cast<double>(blocks) * kThreads * static_cast<double>(iters) * kUnroll * kChains;
  rate = ops / s;
  if (ck[1] > 0) mhz = 100.0 * static_cast<double>(ck[0]) / static_cast<double>(ck[1]);
  return hipSuccess;
}

hipError_t run_gather(int blocks, const uint32_t* buf, uint64_t bytes, uint32_t rounds, uint32_t* sink,
                      double& rate) {
  const uint32_t mask = static_cast<uint32_t>(bytes / 4 - 1);
  Timer tm;
  hipLaunchKernelGGL(gather_loop, dim3(blocks), dim3(kThreads), 0, 0, buf, mask, rounds / 4 + 1, sink);
  tm.start();
  hipLaunchKernelGGL(gather_loop, dim3(blocks), dim3(kThreads), 0, 0, buf, mask, rounds, sink);
  const double s = tm.stop_s();
  rate = static_cast<double>(blocks) * kThreads * static_cast<double>(rounds) * kChains / s;
  return hipGetLastError();
}

template <bool kF64>
hipError_t run_atomic(int blocks, void* buf, uint64_t bins, uint32_t n, double& rate) {
  Timer tm;
  hipLaunchKernelGGL(atomic_loop<kF64>, dim3(blocks), dim3(kThreads), 0, 0, buf, bins, n / 4 + 1);
  tm.start();
  hipLaunchKernelGGL(atomic_loop<kF64>, dim3(blocks), dim3(kThreads), 0, 0, buf, bins, n);
  const double s = tm.stop_s();
  rate = static_cast<double>(blocks) * kThreads * static_cast<double>(n) / s;
  return hipGetLastError();
}

}  // namespace

extern "C" int sse_measure_peaks(int device, uint64_t atomic_bins, sse_peaks* out) {
  if (!out) return -static_cast<int>(hipErrorInvalidValue);
  std::memset(out, 0, sizeof *out);
  if (!atomic_bins) atomic_bins = 206397408ull;
  hipError_t e = hipSetDevice(device);
  int cus = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return -static_cast<int>(e);
  out->cus = static_cast<uint64_t>(cus);
  out->atomic_bins = atomic_bins;
  const int blocks = cus * kBlocksPerCu;
  const uint64_t threads = static_cast<uint64_t>(blocks) * kThreads;
  constexpr uint64_t kGatherMax = 2ull << 30;
  uint32_t* sink = nullptr;
  unsigned long long* clocks = nullptr;
  uint32_t* gbuf = nullptr;
  void* abuf = nullptr;
  e = hipMalloc(&sink, threads * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&clocks, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&gbuf, kGatherMax);
  if (e == hipSuccess) e = hipMemset(gbuf, 1, kGatherMax);
  if (e == hipSuccess) e = hipMalloc(&abuf, atomic_bins * sizeof(double));
  if (e == hipSuccess) e = hipMemset(abuf, 0, atomic_bins * sizeof(double));
  double mhz = 0.0, mhz_x = 0.0;
  constexpr uint32_t kIters = 2048;  // x 16 x 8 instructions per lane
  if (e == hipSuccess) e = run_valu<kAdd>(blocks, kIters, sink, clocks, out->valu_add, mhz);
  if (e == hipSuccess) e = run_valu<kXor>(blocks, kIters, sink, clocks, out->valu_xor, mhz_x);
  if (e == hipSuccess) e = run_valu<kFma>(blocks, kIters, sink, clocks, out->valu_fma, mhz_x);
  if (e == hipSuccess) e = run_valu<kMad64>(blocks, kIters / 4, sink, clocks, out->valu_mad64, mhz_x);
  if (e == hipSuccess) e = run_valu<kCnd>(blocks, kIters, sink, clocks, out->valu_cndmask, mhz_x);
  if (e == hipSuccess) e = run_valu<kLog>(blocks, kIters / 4, sink, clocks, out->valu_log, mhz_x);
  out->sclk_mhz = mhz;
  if (e == hipSuccess) e = run_gather(blocks, gbuf, 2ull << 20, 256, sink, out->gather_l2);
  if (e == hipSuccess) e = run_gather(blocks, gbuf, 32ull << 20, 128, sink, out->gather_llc);
  if (e == hipSuccess) e = run_gather(blocks, gbuf, kGatherMax, 64, sink, out->gather_hbm);
  if (e == hipSuccess) e = run_atomic<false>(blocks, abuf, atomic_bins, 64, out->atomic_u32);
  if (e == hipSuccess) e = run_atomic<true>(blocks, abuf, atomic_bins, 64, out->atomic_f64);
  if (e == hipSuccess) {
    const uint64_t n16 = (kGatherMax / 2) / 16;
    const uint4* in = reinterpret_cast<const uint4*>(gbuf);
    uint4* dst = reinterpret_cast<uint4*>(gbuf) + n16;
    Timer tm;
    hipLaunchKernelGGL(copy_loop, dim3(blocks), dim3(kThreads), 0, 0, in, dst, n16);
    tm.start();
    hipLaunchKernelGGL(copy_loop, dim3(blocks), dim3(kThreads), 0, 0, in, dst, n16);
    const double s = tm.stop_s();
    out->copy_bytes_per_s = 2.0 * static_cast<double>(n16 * 16) / s;
    e = hipGetLastError();
  }
  if (sink) (void)hipFree(sink);
  if (clocks) (void)hipFree(clocks);
  if (gbuf) (void)hipFree(gbuf);
  if (abuf) (void)hipFree(abuf);
  return e == hipSuccess ? 0 : -static_cast<int>(e);
}
