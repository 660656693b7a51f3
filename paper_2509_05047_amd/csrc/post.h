// Declarations of the sinogram post-processing kernels (sensitivity
// multiply, smoothing, smoothing normalisation) shared by the library's
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sse {

struct PostParams {
  int n_rad, n_view, n_plane, n_tof;
};

hipError_t launch_apply_sensitivity(const PostParams& g, const double* W, double scale, const float* sens,
                                    int sens_tof, float* out, hipStream_t stream);
constexpr int kMaxSmoothRadius = 63;
// Normalised Gaussian taps w[0 .. 2*radius], passed by value to the kernel.
struct Taps {
  float w[2 * kMaxSmoothRadius + 1];
  int radius;
};
// One separable pass along axis (0 radial, 1 view, 2 plane; -1: no
// smoothing, pointwise only).  The input is binary32, or binary64 weights
// scaled by `scale` and rounded on load (in_is_f64); norm_in (if not NULL)
// multiplies the input on load; norm_out (if not NULL) divides the output
// (entries <= 0 count as 1) and sens (if not NULL) multiplies it; ratio_w
// (if not NULL) then replaces the output G by G / S, S = float(scale ratio_w),
// or by 1 where S or G is not positive.
hipError_t launch_smooth_axis(const PostParams& g, int axis, const void* in, bool in_is_f64, double scale,
                              const float* norm_in, float* out, const Taps& taps, const float* norm_out,
                              const float* sens, int sens_tof, const double* ratio_w, hipStream_t stream);
// The radial and plane passes in one launch (both axes smoothed): tiles of
// tl radial positions by all planes of one (TOF, view) row, staged in LDS by
// a persistent block per CU.  plan_rad_plane picks the tile for the radii
// (tl == 0: the tile does not fit in fused_lds_limit() bytes of LDS -- the
// device's per-block LDS, at most kFusedLdsBytes -- or its staging slots, or
// would be mostly halo; use the one-axis passes).  Same input and output
// treatment as launch_smooth_axis.
constexpr size_t kFusedLdsBytes = 160 * 1024;
size_t fused_lds_limit();
struct FusedPlan {
  int tl, n_tiles, sx, sy;
  size_t lds_bytes;
};
FusedPlan plan_rad_plane(const PostParams& g, int radial_radius, int plane_radius);
hipError_t launch_smooth_rad_plane(const PostParams& g, const FusedPlan& plan, const void* in, bool in_is_f64,
                                   double scale, const float* norm_in, float* out, const Taps& radial,
                                   const Taps& plane, const float* norm_out, const float* sens, int sens_tof,
                                   const double* ratio_w, hipStream_t stream);
// total[0] = sum over bins of (scale * W) * sens in binary64, in a fixed
// order (partial: device scratch of kTotalPartials doubles).
constexpr int kTotalPartials = 1024;
hipError_t launch_total_scatter(const PostParams& g, const double* W, double scale, const float* sens, int sens_tof,
                                double* partial, double* total, hipStream_t stream);

}  // namespace sse
