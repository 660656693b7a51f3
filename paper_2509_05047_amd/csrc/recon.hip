// Reconstruction of the joint activity / scatter estimation loop on gfx950:
// a TOF Joseph forward projector, its exact transpose as a pixel-driven back
// projector, and the OSEM update kernels.  The paper reconstructs with
// TOF-OSEM, 1 iteration of 28 subsets per loop iteration, between the short
// scatter simulations (Methods, "Unknown activity distribution, very limited
// simulation time"; "Evaluation metrics").
//
// Geometry (readings; the paper does not specify its projector): the LOR of
// sinogram bin (view, rad) joins the centres of the crystal pair the
// simulator bins there, on the detection cylinder; plane p is the transaxial
// plane at the mean of its two rings, and the image has one slice per plane
// on the phantom's transaxial grid, so a plane's LORs read one slice.  Along
// the LOR's major axis one sample per pixel column (row), linear
// interpolation between the two pixels next to the crossing along the minor
// axis, weight = pixel size / |major direction component|.  The major axis
// comes from the crystal indices (the LOR of crystals a, b runs at angle
// pi q / (2 n), q = (2 k + n) mod 2n, k = (a + b + 1) mod n: x when 2q <= n
// or 2q >= 3n), so that rounding of the direction never decides it.  TOF: the sample's
// signed distance s from the LOR midpoint towards the simulator's
// TOF-positive crystal, and bin j gets Phi((hi_j - s)/sigma) -
// Phi((lo_j - s)/sigma) for the bins within 5 sigma of s (the bin holding s
// with sigma = 0).
//
// Forward: four threads per LOR of the requested views, each over a share
// of its samples, their TOF bins accumulated in private LDS columns and
// added in a fixed order.  Back: one thread per pixel and group of planes,
// which finds the LORs of each view whose samples read the pixel (a window
// of radial indices around the pixel's distance from the view's centre LOR)
// and takes exactly the weights the forward sample computes, so the pair is
// a transpose up to the order of binary32 sums.  Binary32 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "recon.h"

namespace sse {
namespace {

constexpr int kReconThreads = 256;

struct Sample {
  int i0;       // minor-axis index of the first pixel read (i0 + 1 the second)
  float w1;     // weight of pixel i0 + 1 (pixel i0 gets 1 - w1)
  float s;      // TOF coordinate
  float dl;     // path length
};

// Sample k of the LOR with midpoint (mx, my) along its major axis (x if
// xmaj); ux, uy hold the table's (1 / u_x, u_y) for an x-major LOR and
// (u_x, 1 / u_y) for a y-major one.
__device__ __forceinline__ Sample lor_sample(const ReconGeom& g, float mx, float my, float ux, float uy, bool xmaj,
                                             int k) {
  Sample o;
  float f;
  // (quotients as products with the reciprocals of the LOR table and the
  // geometry: forward and back projector take the same binary32 values)
  if (xmaj) {
    const float xc = g.lox + (static_cast<float>(k) + 0.5f) * g.vx;
    o.s = (xc - mx) * ux;
    const float y = my + o.s * uy;
    f = (y - g.loy) * g.ivy - 0.5f;
    o.dl = g.vx * fabsf(ux);
  } else {
    const float yc = g.loy + (static_cast<float>(k) + 0.5f) * g.vy;
    o.s = (yc - my) * uy;
    const float x = mx + o.s * ux;
    f = (x - g.lox) * g.ivx - 0.5f;
    o.dl = g.vy * fabsf(uy);
  }
  const float fl = floorf(f);
  o.i0 = static_cast<int>(fl);
  o.w1 = f - fl;
  return o;
}

// TOF bins a sample at s adds to: [jlo, jhi] (empty if jlo > jhi).
__device__ __forceinline__ void tof_range(const ReconGeom& g, float s, int& jlo, int& jhi) {
  const float half = 0.5f * static_cast<float>(g.n_tof);
  if (g.tof_sigma <= 0.0f) {
    const float fj = floorf(s / g.tof_bin + half);
    jlo = jhi = static_cast<int>(fmaxf(fminf(fj, 1e6f), -1e6f));
    if (!(fj >= 0.0f && fj < static_cast<float>(g.n_tof))) jlo = 1, jhi = 0;
    return;
  }
  const float r = 5.0f * g.tof_sigma;
  jlo = static_cast<int>(ceilf((s - r) / g.tof_bin + half)) - 1;
  jhi = static_cast<int>(floorf((s + r) / g.tof_bin + half));
  jlo = jlo < 0 ? 0 : jlo;
  jhi = jhi > g.n_tof - 1 ? g.n_tof - 1 : jhi;
}

// Phi((e_j - s) / sigma) = Q((s - e_j) / sigma) for the lower edge e_j of
// bin j, from the interpolation table (three multiply-adds and one 16-byte
// read instead of an erfc).
__device__ __forceinline__ float edge_cdf(const ReconGeom& g, int j, float s) {
  const float e = (static_cast<float>(j) - 0.5f * static_cast<float>(g.n_tof)) * g.tof_bin;
  // w = v / h counts intervals from v = 0, so that the fraction f keeps its
  // precision where Q varies fastest (the table's origin is interval
  // kQIntervals / 2)
  const float w = (s - e) * g.q_scale;
  const float fl = floorf(w);
  const float kf = fl + static_cast<float>(kQIntervals / 2);
  const bool below = !(kf >= 0.0f), above = kf > static_cast<float>(kQIntervals - 1);
  const int k = below ? 0 : (above ? kQIntervals - 1 : static_cast<int>(kf));
  const float f = below ? 0.0f : (above ? 1.0f : w - fl);
  const float4 c = g.q_tab[k];
  return __builtin_fmaf(f, __builtin_fmaf(f, __builtin_fmaf(f, c.w, c.z), c.y), c.x);
}

__device__ __forceinline__ float4 lor_at(const ReconGeom& g, int view, int rad) {
  return g.lor[static_cast<uint64_t>(view) * g.n_rad + rad];
}

// Forward projection: kProjSplit threads per (plane, sv, rad) LOR (views
// subset + sv n_subsets), each over an equal share of the LOR's samples: a
// block takes 64 LORs, wavefront w the w-th share of each, so the launch
// has four times as many wavefronts as LORs need and its long sample loops
// overlap.  Each thread accumulates its TOF bins in its own LDS column; the
// shares are then added in share order (deterministic) and written.
constexpr int kProjSplit = kReconThreads / 64;
__global__ void __launch_bounds__(kReconThreads) project_kernel(ReconGeom g, const float* __restrict__ img,
                                                                SinoOut out, int tof) {
  extern __shared__ float acc_lds[];  // [nt][kReconThreads]
  const int lane = static_cast<int>(threadIdx.x & 63u);
  const int share = static_cast<int>(threadIdx.x >> 6);
  const uint64_t id = static_cast<uint64_t>(blockIdx.x) * 64u + lane;
  const uint64_t n_lor = static_cast<uint64_t>(g.n_plane) * g.n_sv * g.n_rad;
  const bool live = id < n_lor;
  const uint64_t idc = live ? id : 0;
  const int rad = static_cast<int>(idc % g.n_rad);
  const int sv = static_cast<int>((idc / g.n_rad) % g.n_sv);
  const int plane = static_cast<int>(idc / (static_cast<uint64_t>(g.n_rad) * g.n_sv));
  const int view = g.subset + sv * g.n_subsets;
  const int nt = tof ? g.n_tof : 1;
  float* acc = acc_lds + threadIdx.x;
  for (int j = 0; j < nt; ++j) acc[j * kReconThreads] = 0.0f;
  const float4 l = lor_at(g, view, rad);
  if (live && (l.z != 0.0f || l.w != 0.0f)) {
    const float* im = img + static_cast<uint64_t>(plane) * g.nx * g.ny;
    const bool mx = g.major[static_cast<uint64_t>(view) * g.n_rad + rad] != 0;
    const int ns = mx ? g.nx : g.ny, n_minor = mx ? g.ny : g.nx;
    const int k0 = ns * share / kProjSplit, k1 = ns * (share + 1) / kProjSplit;
    for (int k = k0; k < k1; ++k) {
      const Sample o = lor_sample(g, l.x, l.y, l.z, l.w, mx, k);
      if (o.i0 < -1 || o.i0 >= n_minor) continue;
      const float v0 = o.i0 >= 0 ? im[mx ? o.i0 * g.nx + k : k * g.nx + o.i0] : 0.0f;
      const float v1 = o.i0 + 1 < n_minor ? im[mx ? (o.i0 + 1) * g.nx + k : k * g.nx + o.i0 + 1] : 0.0f;
      const float val = (1.0f - o.w1) * v0 + o.w1 * v1;
      if (val == 0.0f) continue;
      const float c = o.dl * val;
      if (!tof) {
        acc[0] += c;
        continue;
      }
      int jlo, jhi;
      tof_range(g, o.s, jlo, jhi);
      if (g.tof_sigma <= 0.0f) {
        if (jlo <= jhi) acc[jlo * kReconThreads] += c;
        continue;
      }
      float lo = edge_cdf(g, jlo, o.s);
      for (int j = jlo; j <= jhi; ++j) {
        const float hi = edge_cdf(g, j + 1, o.s);
        acc[j * kReconThreads] += (hi - lo) * c;
        lo = hi;
      }
    }
  }
  __syncthreads();
  if (!live) return;
  // bins j = share, share + kProjSplit, ... of the block's LOR `lane`
  const uint64_t base = static_cast<uint64_t>(plane) * out.ps + static_cast<uint64_t>(sv) * out.vs + rad;
  const float* col = acc_lds + lane;
  for (int j = share; j < nt; j += kProjSplit) {
    float v = col[j * kReconThreads];
#pragma unroll
    for (int q = 1; q < kProjSplit; ++q) v += col[j * kReconThreads + 64 * q];
    out.p[base + static_cast<uint64_t>(j) * (tof ? out.ts : 0)] = v;
  }
}

// Back projection: thread per (iy, ix) pixel and group of kBackPlanes
// planes.  A plane's LORs read only its own slice and the geometry is the
// same in every plane, so the window, the Joseph weights and the TOF
// weights of a (pixel, LOR) pair are computed once for the group and
// applied to each of its planes' sinogram values, each plane summing in
// the order a thread per pixel would.
constexpr int kBackPlanes = 4;
constexpr int kTofBlock = 4;  // TOF bins whose reads are issued together
__global__ void __launch_bounds__(kReconThreads) backproject_kernel(ReconGeom g, SinoIn in, float* __restrict__ img,
                                                                    int tof) {
  const uint64_t id = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t npix = static_cast<uint64_t>(g.nx) * g.ny;
  const int n_groups = (g.n_plane + kBackPlanes - 1) / kBackPlanes;
  if (id >= npix * n_groups) return;
  const int ix = static_cast<int>(id % g.nx);
  const int iy = static_cast<int>((id / g.nx) % g.ny);
  const int p0 = static_cast<int>(id / npix) * kBackPlanes;
  const int np = g.n_plane - p0 < kBackPlanes ? g.n_plane - p0 : kBackPlanes;  // planes of the group
  const float px = g.lox + (static_cast<float>(ix) + 0.5f) * g.vx;
  const float py = g.loy + (static_cast<float>(iy) + 0.5f) * g.vy;
  const int half = (g.n_rad - 1) / 2;
  float total[kBackPlanes] = {};
  for (int sv = 0; sv < g.n_sv; ++sv) {
    const int view = g.subset + sv * g.n_subsets;
    // the pixel's distance from the view's centre LOR (normal and sign of
    // the radial direction from the view table), and the radial window
    // around it that holds every LOR whose samples can read the pixel
    const float4 vt = g.view_tab[view];  // (nx, ny, d of rad half+1 minus rad half sign, unused)
    const float d = vt.x * px + vt.y * py;
    const float q = fminf(fmaxf(d / g.radius, -1.0f), 1.0f);
    const float rho_est = vt.z * asinf(q) * g.rho_scale;
    // half-width: the distance bound win_num (in radial steps at the centre)
    // over the slope cos(pi rho / n_crystals) at the window's far end
    const float c0 = cosf(fminf(fabsf(rho_est) + g.win_extra, g.rho_max) / g.rho_scale);
    const int w0 = static_cast<int>(ceilf(g.win_num / fmaxf(c0, 1e-3f))) + 1;
    const float c1 = cosf(fminf(fabsf(rho_est) + static_cast<float>(w0), g.rho_max) / g.rho_scale);
    const int w = static_cast<int>(ceilf(g.win_num / fmaxf(c1, 1e-3f))) + 1;
    const int rc = static_cast<int>(rintf(rho_est)) + half;
    const int r0 = rc - w < 0 ? 0 : rc - w, r1 = rc + w > g.n_rad - 1 ? g.n_rad - 1 : rc + w;
    // each candidate's LOR entry is read one candidate ahead (the first
    // read clamped into the row: the window is empty, r0 > r1, for pixels
    // outside the field of view, where r0 may pass the last radial index)
    const int rp = r0 < g.n_rad - 1 ? r0 : g.n_rad - 1;
    float4 ln = lor_at(g, view, rp);
    bool mn = g.major[static_cast<uint64_t>(view) * g.n_rad + rp] != 0;
    for (int rad = r0; rad <= r1; ++rad) {
      const float4 l = ln;
      const bool mx = mn;
      {
        const int rn = rad < r1 ? rad + 1 : rad;
        ln = lor_at(g, view, rn);
        mn = g.major[static_cast<uint64_t>(view) * g.n_rad + rn] != 0;
      }
      if (l.z == 0.0f && l.w == 0.0f) continue;
      const Sample o = lor_sample(g, l.x, l.y, l.z, l.w, mx, mx ? ix : iy);
      const int minor = mx ? iy : ix;
      float wt;
      if (o.i0 == minor) wt = 1.0f - o.w1;
      else if (o.i0 + 1 == minor) wt = o.w1;
      else continue;
      const float* src = in.p + static_cast<uint64_t>(p0) * in.ps + static_cast<uint64_t>(sv) * in.vs + rad;
      float a[kBackPlanes] = {};
      if (!tof) {
#pragma unroll
        for (int k = 0; k < kBackPlanes; ++k)
          if (k < np) a[k] = src[static_cast<uint64_t>(k) * in.ps];
      } else if (g.tof_sigma <= 0.0f) {
        int jlo, jhi;
        tof_range(g, o.s, jlo, jhi);
        if (jlo <= jhi) {
#pragma unroll
          for (int k = 0; k < kBackPlanes; ++k)
            if (k < np) a[k] = src[static_cast<uint64_t>(k) * in.ps + static_cast<uint64_t>(jlo) * in.ts];
        }
      } else {
        // the bins in blocks of kTofBlock, every table and sinogram read of
        // a block issued before any is used (indices clamped into range,
        // values past the last bin or plane unused), so that a block costs
        // one memory latency rather than one per bin
        int jlo, jhi;
        tof_range(g, o.s, jlo, jhi);
        float lo = edge_cdf(g, jlo, o.s);
        for (int j0 = jlo; j0 <= jhi; j0 += kTofBlock) {
          float ed[kTofBlock];
          float v[kTofBlock][kBackPlanes];
#pragma unroll
          for (int i = 0; i < kTofBlock; ++i) {
            const int j = j0 + i <= jhi ? j0 + i : jhi;
            ed[i] = edge_cdf(g, j + 1, o.s);
            const float* sj = src + static_cast<uint64_t>(j) * in.ts;
#pragma unroll
            for (int k = 0; k < kBackPlanes; ++k) v[i][k] = sj[static_cast<uint64_t>(k < np ? k : np - 1) * in.ps];
          }
#pragma unroll
          for (int i = 0; i < kTofBlock; ++i) {
            if (j0 + i > jhi) break;
            const float wj = ed[i] - lo;
#pragma unroll
            for (int k = 0; k < kBackPlanes; ++k) a[k] += wj * v[i][k];
            lo = ed[i];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kBackPlanes; ++k) total[k] += wt * o.dl * a[k];
    }
  }
  float* dst = img + static_cast<uint64_t>(p0) * npix + static_cast<uint64_t>(iy) * g.nx + ix;
#pragma unroll
  for (int k = 0; k < kBackPlanes; ++k)
    if (k < np) dst[static_cast<uint64_t>(k) * npix] = total[k];
}

// ratio[b] = m y / (m fp + a) over a subset's bins (compact layout of fp and
// ratio; prompts and additive in the full layout; m without TOF axis): 0 for
// a non-positive denominator, which counts as 1e-20 when smaller than that.
__global__ void __launch_bounds__(256) ratio_kernel(ReconGeom g, const float* __restrict__ prompts,
                                                    const float* __restrict__ mult, const float* __restrict__ add,
                                                    float* __restrict__ fp_ratio) {
  const uint64_t n = static_cast<uint64_t>(g.n_tof) * g.n_plane * g.n_sv * g.n_rad;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int rad = static_cast<int>(i % g.n_rad);
    const int sv = static_cast<int>((i / g.n_rad) % g.n_sv);
    const uint64_t tp = i / (static_cast<uint64_t>(g.n_rad) * g.n_sv);  // t * n_plane + plane
    const int plane = static_cast<int>(tp % g.n_plane);
    const uint64_t t = tp / g.n_plane;
    const int view = g.subset + sv * g.n_subsets;
    const uint64_t inner = (static_cast<uint64_t>(plane) * g.n_view + view) * g.n_rad + rad;
    const uint64_t full = t * static_cast<uint64_t>(g.n_plane) * g.n_view * g.n_rad + inner;
    const float m = mult[inner];
    const float den = m * fp_ratio[i] + add[full];
    fp_ratio[i] = den > 0.0f ? m * prompts[full] / fmaxf(den, 1e-20f) : 0.0f;
  }
}

// the subset's multiplicative sinogram broadcast over TOF (compact layout)
__global__ void __launch_bounds__(256) mult_tof_kernel(ReconGeom g, const float* __restrict__ mult,
                                                       float* __restrict__ out) {
  const uint64_t n = static_cast<uint64_t>(g.n_tof) * g.n_plane * g.n_sv * g.n_rad;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int rad = static_cast<int>(i % g.n_rad);
    const int sv = static_cast<int>((i / g.n_rad) % g.n_sv);
    const int plane = static_cast<int>((i / (static_cast<uint64_t>(g.n_rad) * g.n_sv)) % g.n_plane);
    const int view = g.subset + sv * g.n_subsets;
    out[i] = mult[(static_cast<uint64_t>(plane) * g.n_view + view) * g.n_rad + rad];
  }
}

// x <- x back / sens where sens > 0
__global__ void __launch_bounds__(256) update_kernel(float* __restrict__ x, const float* __restrict__ back,
                                                     const float* __restrict__ sens, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float s = sens[i];
    if (s > 0.0f) x[i] = x[i] * back[i] / s;
  }
}

// image slice p = volume slice iz_of[p] (nearest voxel slice to plane p)
__global__ void __launch_bounds__(256) plane_slices_kernel(const float* __restrict__ vol,
                                                           const int* __restrict__ iz_of, uint64_t slice,
                                                           uint64_t n_plane, float* __restrict__ img) {
  const uint64_t n = slice * n_plane;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    img[i] = vol[static_cast<uint64_t>(iz_of[i / slice]) * slice + i % slice];
}

__global__ void __launch_bounds__(256) exp_neg_kernel(float* __restrict__ x, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    x[i] = expf(-x[i]);
}

int grid_for(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return static_cast<int>(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_project(const ReconGeom& g, const float* img, const SinoOut& out, int tof, hipStream_t s) {
  const uint64_t n = static_cast<uint64_t>(g.n_plane) * g.n_sv * g.n_rad;
  const size_t lds = static_cast<size_t>(tof ? g.n_tof : 1) * kReconThreads * sizeof(float);
  hipLaunchKernelGGL(project_kernel, dim3(static_cast<unsigned>((n + 63) / 64)), dim3(kReconThreads), lds, s, g, img,
                     out, tof);
  return hipGetLastError();
}

hipError_t launch_backproject(const ReconGeom& g, const SinoIn& in, float* img, int tof, hipStream_t s) {
  const uint64_t n = static_cast<uint64_t>(g.nx) * g.ny * ((g.n_plane + kBackPlanes - 1) / kBackPlanes);
  hipLaunchKernelGGL(backproject_kernel, dim3(static_cast<unsigned>((n + kReconThreads - 1) / kReconThreads)),
                     dim3(kReconThreads), 0, s, g, in, img, tof);
  return hipGetLastError();
}

hipError_t launch_attenuation_factors(const ReconGeom& g, const float* mu, const int* iz_of, float* mu_img,
                                      float* out, hipStream_t s) {
  const uint64_t slice = static_cast<uint64_t>(g.nx) * g.ny;
  hipLaunchKernelGGL(plane_slices_kernel, dim3(grid_for(slice * g.n_plane)), dim3(256), 0, s, mu, iz_of, slice,
                     static_cast<uint64_t>(g.n_plane), mu_img);
  const uint64_t plane_bins = static_cast<uint64_t>(g.n_view) * g.n_rad;
  const SinoOut o{out, 0, plane_bins, static_cast<uint64_t>(g.n_rad)};
  hipError_t e = launch_project(g, mu_img, o, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(exp_neg_kernel, dim3(grid_for(plane_bins * g.n_plane)), dim3(256), 0, s, out,
                     plane_bins * g.n_plane);
  return hipGetLastError();
}

hipError_t launch_subset_sensitivity(const ReconGeom& g, const float* mult, float* fp, float* sens, hipStream_t s) {
  const uint64_t tb = static_cast<uint64_t>(g.n_plane) * g.n_sv * g.n_rad;
  const SinoIn in{fp, tb, static_cast<uint64_t>(g.n_sv) * g.n_rad, static_cast<uint64_t>(g.n_rad)};
  hipLaunchKernelGGL(mult_tof_kernel, dim3(grid_for(tb * g.n_tof)), dim3(256), 0, s, g, mult, fp);
  return launch_backproject(g, in, sens, 1, s);
}

hipError_t launch_osem_subset(const ReconGeom& g, const float* prompts, const float* mult, const float* add,
                              float* img, float* fp, float* back, float* sens, bool sens_ready, hipStream_t s) {
  const uint64_t tb = static_cast<uint64_t>(g.n_plane) * g.n_sv * g.n_rad;  // compact bins per TOF bin
  const SinoOut out{fp, tb, static_cast<uint64_t>(g.n_sv) * g.n_rad, static_cast<uint64_t>(g.n_rad)};
  const SinoIn in{fp, tb, static_cast<uint64_t>(g.n_sv) * g.n_rad, static_cast<uint64_t>(g.n_rad)};
  const uint64_t nb = tb * g.n_tof, ni = static_cast<uint64_t>(g.nx) * g.ny * g.n_plane;
  hipError_t e = launch_project(g, img, out, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ratio_kernel, dim3(grid_for(nb)), dim3(256), 0, s, g, prompts, mult, add, fp);
  e = launch_backproject(g, in, back, 1, s);
  if (e != hipSuccess) return e;
  if (!sens_ready) {
    e = launch_subset_sensitivity(g, mult, fp, sens, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(ni)), dim3(256), 0, s, img, back, sens, ni);
  return hipGetLastError();
}

}  // namespace sse
