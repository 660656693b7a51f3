// Declarations of the reconstruction kernels of the estimation loop (TOF
// Joseph projector, its transpose, OSEM update), shared by the library's
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sse {

// Geometry of one projection: the image grid (nx x ny pixels of vx x vy mm
// from (lox, loy), one slice per sinogram plane), the sinogram, the LOR table
// lor[view * n_rad + rad] = (midpoint x, y, and the unit direction towards
// the TOF-positive crystal stored as (1 / u_x, u_y) for an x-major LOR, (u_x,
// 1 / u_y) for a y-major one; zero where no crystal pair maps) with its
// major axis decided from the crystal indices (see recon.hip), and the
// views taken: subset + sv * n_subsets for sv in [0, n_sv).  view_tab[view]
// = (normal x, y of the view's centre LOR, +-1 so that the radial index
// grows with the signed distance along that normal, 0) and the window
// parameters of the back projector's search (see recon.hip).
struct ReconGeom {
  int n_rad, n_view, n_plane, n_tof;
  float tof_bin, tof_sigma;
  float q_scale;        // 1 / (sigma h): TOF distance to table intervals
  const float4* q_tab;  // the normal tail Q by intervals (see kQIntervals)
  int nx, ny;
  float vx, vy, lox, loy, ivx, ivy;
  const float4* lor;
  const uint8_t* major;        // per (view, rad): 1 if x is the LOR's major axis
  const float4* view_tab;
  int subset, n_subsets, n_sv;
  float radius, rho_scale, rho_max, win_num, win_extra;
};

// The TOF weights' normal tail Q(v) = erfc(v / sqrt 2) / 2 by cubic
// Hermite interpolation on kQIntervals intervals of [-kQRange, kQRange]:
// q_tab[k] holds the binary64 coefficients, rounded, of Q(v_k + f h) =
// a0 + f (a1 + f (a2 + f a3)), f in [0, 1], h = 2 kQRange / kQIntervals
// (interpolation error below 1e-10; Q is held at its end values outside).
constexpr int kQIntervals = 1024;
constexpr double kQRange = 6.5;

// A sinogram as the kernels address it: bin (t, plane, sv, rad) at
// p[t ts + plane ps + sv vs + rad].
struct SinoOut {
  float* p;
  uint64_t ts, ps, vs;
};
struct SinoIn {
  const float* p;
  uint64_t ts, ps, vs;
};

hipError_t launch_project(const ReconGeom& g, const float* img, const SinoOut& out, int tof, hipStream_t s);
hipError_t launch_backproject(const ReconGeom& g, const SinoIn& in, float* img, int tof, hipStream_t s);
// Attenuation factors exp(-line integral) of all views ([plane][view][rad])
// from the phantom's attenuation volume mu: image slice p is volume slice
// iz_of[p] (device table), staged in mu_img (image-sized scratch).
hipError_t launch_attenuation_factors(const ReconGeom& g, const float* mu, const int* iz_of, float* mu_img,
                                      float* out, hipStream_t s);
// The subset's sensitivity image P_s^T m (m broadcast over TOF) into sens;
// fp: scratch of n_tof n_plane n_sv n_rad floats.
hipError_t launch_subset_sensitivity(const ReconGeom& g, const float* mult, float* fp, float* sens, hipStream_t s);
// One OSEM subset update of img in place; fp: scratch as above; back:
// scratch image; sens: the subset's sensitivity image, computed here unless
// sens_ready.
hipError_t launch_osem_subset(const ReconGeom& g, const float* prompts, const float* mult, const float* add,
                              float* img, float* fp, float* back, float* sens, bool sens_ready, hipStream_t s);

}  // namespace sse
