// C ABI of the reconstruction step of the joint estimation loop: projector,
// back projector, TOF-OSEM, and the update of a phantom's activity from a
// reconstructed image.  Declarations and documentation: include/sse.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <vector>

#include "context.h"
#include "recon.h"

using namespace sse_detail;

namespace {

constexpr double kPiD = 3.141592653589793;

// The crystal pair of each (view, rad) as the simulator bins coincidences
// (the sinogram mapping of the coincidence evaluation), TOF-positive end
// first, and from it the LOR table and the view table of the projector.
sse_status ensure_lor_tables(sse_ctx* c) {
  if (c->d_lor && c->d_view && c->d_major && c->d_qtab) return SSE_OK;
  for (void** t : {&c->d_lor, &c->d_view, &c->d_major, &c->d_qtab}) {  // after a failed build
    release(*t);
    *t = nullptr;
  }
  const int n = c->sc.n_crystals, n_rad = c->sn.n_rad, n_view = c->sn.n_view, half = (n_rad - 1) / 2;
  const double R = c->sc.radius_mm;
  std::vector<float4> lor(static_cast<size_t>(n_view) * n_rad, make_float4(0.0f, 0.0f, 0.0f, 0.0f));
  std::vector<double> ux(lor.size(), 0.0), uy(lor.size(), 0.0), mxs(lor.size(), 0.0), mys(lor.size(), 0.0);
  std::vector<uint8_t> major(static_cast<size_t>(n_view) * n_rad, 1);
  for (int c1 = 0; c1 < n; ++c1)
    for (int c2 = c1 + 1; c2 < n; ++c2) {
      int k = c1 + c2 + 1, rho = n / 2 - std::abs(c1 - c2);
      if (k >= n) {
        k -= n;
        rho = -rho;
      }
      if (std::abs(rho) > half) continue;
      int m = (2 * c1 + 1 - k) % (2 * n);
      if (m < 0) m += 2 * n;
      const bool c1_pos = m > 0 && m < n;
      const int a = c1_pos ? c1 : c2, b = c1_pos ? c2 : c1;
      const double pa = 2.0 * kPiD * (a + 0.5) / n, pb = 2.0 * kPiD * (b + 0.5) / n;
      const double ax = R * std::cos(pa), ay = R * std::sin(pa), bx = R * std::cos(pb), by = R * std::sin(pb);
      const double dx = ax - bx, dy = ay - by, len = std::sqrt(dx * dx + dy * dy);
      const size_t idx = static_cast<size_t>(k >> 1) * n_rad + (rho + half);
      // direction angle pi q / (2 n): x is the major axis within 45 degrees of it
      const int q = (2 * k + n) % (2 * n);
      major[idx] = (2 * q <= n || 2 * q >= 3 * n) ? 1 : 0;
      ux[idx] = dx / len;
      uy[idx] = dy / len;
      mxs[idx] = 0.5 * (ax + bx);
      mys[idx] = 0.5 * (ay + by);
      // the sample divides by the major component: stored as its reciprocal
      lor[idx] = make_float4(static_cast<float>(mxs[idx]), static_cast<float>(mys[idx]),
                             static_cast<float>(major[idx] ? len / dx : dx / len),
                             static_cast<float>(major[idx] ? dy / len : len / dy));
    }
  // view table: the centre LOR's normal, and the sign that makes the signed
  // distance along it grow with the radial index
  std::vector<float4> view(n_view);
  for (int v = 0; v < n_view; ++v) {
    const size_t i0 = static_cast<size_t>(v) * n_rad + half;
    const double nx = -uy[i0], ny = ux[i0];
    double sg = 1.0;
    if (n_rad > 1) sg = (nx * mxs[i0 + 1] + ny * mys[i0 + 1]) >= (nx * mxs[i0] + ny * mys[i0]) ? 1.0 : -1.0;
    view[v] = make_float4(static_cast<float>(nx), static_cast<float>(ny), static_cast<float>(sg), 0.0f);
  }
  HIP_TRY(hipMalloc(&c->d_lor, lor.size() * sizeof(float4)), "allocate LOR table");
  HIP_TRY(hipMalloc(&c->d_view, view.size() * sizeof(float4)), "allocate view table");
  HIP_TRY(hipMalloc(&c->d_major, major.size()), "allocate major-axis table");
  HIP_TRY(hipMemcpy(c->d_major, major.data(), major.size(), hipMemcpyHostToDevice), "upload major-axis table");
  HIP_TRY(hipMemcpy(c->d_lor, lor.data(), lor.size() * sizeof(float4), hipMemcpyHostToDevice), "upload LOR table");
  HIP_TRY(hipMemcpy(c->d_view, view.data(), view.size() * sizeof(float4), hipMemcpyHostToDevice),
          "upload view table");
  // the TOF weights' normal tail Q(v) = erfc(v / sqrt 2) / 2, cubic Hermite
  // coefficients (values and slopes -phi at the interval ends) per interval
  std::vector<float4> q(sse::kQIntervals);
  const double h = 2.0 * sse::kQRange / sse::kQIntervals;
  auto tail = [](double v) { return 0.5 * std::erfc(v / std::sqrt(2.0)); };
  auto slope = [h](double v) { return -h * std::exp(-0.5 * v * v) / std::sqrt(2.0 * kPiD); };
  for (int k = 0; k < sse::kQIntervals; ++k) {
    const double v0 = -sse::kQRange + k * h, v1 = v0 + h;
    const double q0 = tail(v0), q1 = tail(v1), d0 = slope(v0), d1 = slope(v1);
    q[k] = make_float4(static_cast<float>(q0), static_cast<float>(d0), static_cast<float>(3.0 * (q1 - q0) - 2.0 * d0 - d1),
                       static_cast<float>(2.0 * (q0 - q1) + d0 + d1));
  }
  HIP_TRY(hipMalloc(&c->d_qtab, q.size() * sizeof(float4)), "allocate TOF weight table");
  HIP_TRY(hipMemcpy(c->d_qtab, q.data(), q.size() * sizeof(float4), hipMemcpyHostToDevice),
          "upload TOF weight table");
  return SSE_OK;
}

sse::ReconGeom geom_of(const sse_ctx* c, const Phantom* ph, int subset, int n_subsets) {
  sse::ReconGeom g{};
  g.n_rad = c->sn.n_rad;
  g.n_view = c->sn.n_view;
  g.n_plane = c->sn.n_plane;
  g.n_tof = c->sn.n_tof;
  g.tof_bin = c->sn.tof_bin_mm;
  g.tof_sigma = c->sn.tof_sigma_mm;
  g.q_scale = g.tof_sigma > 0.0f ? static_cast<float>(sse::kQIntervals / (2.0 * sse::kQRange * g.tof_sigma)) : 0.0f;
  g.q_tab = static_cast<const float4*>(c->d_qtab);
  g.nx = ph->desc.nx;
  g.ny = ph->desc.ny;
  g.vx = ph->desc.voxel_mm[0];
  g.vy = ph->desc.voxel_mm[1];
  g.lox = ph->desc.lo_mm[0];
  g.loy = ph->desc.lo_mm[1];
  g.ivx = static_cast<float>(1.0 / ph->desc.voxel_mm[0]);
  g.ivy = static_cast<float>(1.0 / ph->desc.voxel_mm[1]);
  g.lor = static_cast<const float4*>(c->d_lor);
  g.major = static_cast<const uint8_t*>(c->d_major);
  g.view_tab = static_cast<const float4*>(c->d_view);
  g.subset = n_subsets <= 1 ? 0 : subset;
  g.n_subsets = n_subsets <= 1 ? 1 : n_subsets;
  g.n_sv = (g.n_view - g.subset + g.n_subsets - 1) / g.n_subsets;
  const double R = c->sc.radius_mm, n = c->sc.n_crystals;
  g.radius = static_cast<float>(R);
  g.rho_scale = static_cast<float>(n / kPiD);
  g.rho_max = static_cast<float>((g.n_rad - 1) / 2);
  // a LOR whose samples read a pixel passes within one pixel of its centre;
  // the two LOR families of a view differ by pi / n in angle, which moves
  // signed distances by at most R pi / n each against the centre LOR's
  // normal: the window covers (pixel + 3 R pi / n + 1 mm) in distance, in
  // radial steps of R pi / n cos(pi rho / n)
  const double vmax = std::max(g.vx, g.vy);
  g.win_num = static_cast<float>((vmax + 3.0 * kPiD * R / n + 1.0) * n / (kPiD * R));
  g.win_extra = 0.0f;
  return g;
}

sse_status check_grid(sse_ctx* c, sse_phantom_id grid, Phantom*& ph) {
  ph = get_phantom(c, grid);
  if (!ph) return fail(SSE_EINVAL, "unknown phantom id (the image grid)");
  // the transaxial grid must lie inside the detection cylinder (it does for
  // every loaded phantom) and every plane needs a slice
  return SSE_OK;
}

sse_status ensure_recon_scratch(sse_ctx* c, uint64_t fp_floats, uint64_t img_floats) {
  if (fp_floats && c->recon_fp_cap < fp_floats) {
    release(c->d_recon_fp);
    c->d_recon_fp = nullptr;
    c->recon_fp_cap = 0;
    HIP_TRY(hipMalloc(&c->d_recon_fp, fp_floats * sizeof(float)), "allocate projection scratch");
    c->recon_fp_cap = fp_floats;
  }
  if (c->recon_img_cap < img_floats) {
    release(c->d_recon_img[0]);
    release(c->d_recon_img[1]);
    c->d_recon_img[0] = c->d_recon_img[1] = nullptr;
    c->recon_img_cap = 0;
    HIP_TRY(hipMalloc(&c->d_recon_img[0], img_floats * sizeof(float)), "allocate image scratch");
    HIP_TRY(hipMalloc(&c->d_recon_img[1], img_floats * sizeof(float)), "allocate image scratch");
    c->recon_img_cap = img_floats;
  }
  return SSE_OK;
}

// The forward projector keeps a thread's TOF bins in LDS (n_tof x 256
// floats per block).
constexpr int kMaxReconTof = 48;

sse_status check_tof(const sse_ctx* c, int tof) {
  if (tof != 0 && tof != 1) return fail(SSE_EINVAL, "tof must be 0 or 1");
  if (tof && c->sn.n_tof > kMaxReconTof) return fail(SSE_EINVAL, "the TOF projector takes at most 48 TOF bins");
  return SSE_OK;
}

sse_status check_subsets(int subset, int n_subsets, int n_view) {
  if (n_subsets < 1 || n_subsets > n_view) return fail(SSE_EINVAL, "n_subsets must be 1 .. n_view");
  if (subset < 0 || subset >= n_subsets) return fail(SSE_EINVAL, "subset must be 0 .. n_subsets - 1");
  return SSE_OK;
}

}  // namespace

extern "C" {

sse_status sse_project(sse_ctx* c, sse_phantom_id grid, const float* image, float* sino, int tof, int subset,
                       int n_subsets, void* stream) {
  if (!c || !image || !sino) return fail(SSE_EINVAL, "null argument");
  if (sse_status st = check_tof(c, tof); st != SSE_OK) return st;
  Phantom* ph = nullptr;
  if (sse_status st = check_grid(c, grid, ph); st != SSE_OK) return st;
  if (sse_status st = check_subsets(subset, n_subsets, c->sn.n_view); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (sse_status st = ensure_lor_tables(c); st != SSE_OK) return st;
  const sse::ReconGeom g = geom_of(c, ph, subset, n_subsets);
  const uint64_t nr = g.n_rad, plane_bins = static_cast<uint64_t>(g.n_view) * nr;
  const sse::SinoOut out{sino + static_cast<uint64_t>(g.subset) * nr, plane_bins * g.n_plane, plane_bins,
                         static_cast<uint64_t>(g.n_subsets) * nr};
  HIP_TRY(sse::launch_project(g, image, out, tof, static_cast<hipStream_t>(stream)), "projector");
  return SSE_OK;
}

sse_status sse_backproject(sse_ctx* c, sse_phantom_id grid, const float* sino, float* image, int tof, int subset,
                           int n_subsets, void* stream) {
  if (!c || !image || !sino) return fail(SSE_EINVAL, "null argument");
  if (sse_status st = check_tof(c, tof); st != SSE_OK) return st;
  Phantom* ph = nullptr;
  if (sse_status st = check_grid(c, grid, ph); st != SSE_OK) return st;
  if (sse_status st = check_subsets(subset, n_subsets, c->sn.n_view); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (sse_status st = ensure_lor_tables(c); st != SSE_OK) return st;
  const sse::ReconGeom g = geom_of(c, ph, subset, n_subsets);
  const uint64_t nr = g.n_rad, plane_bins = static_cast<uint64_t>(g.n_view) * nr;
  const sse::SinoIn in{sino + static_cast<uint64_t>(g.subset) * nr, plane_bins * g.n_plane, plane_bins,
                       static_cast<uint64_t>(g.n_subsets) * nr};
  HIP_TRY(sse::launch_backproject(g, in, image, tof, static_cast<hipStream_t>(stream)), "back projector");
  return SSE_OK;
}

sse_status sse_osem_sensitivity(sse_ctx* c, sse_phantom_id grid, const float* mult, int n_subsets, float* sens,
                                void* stream) {
  if (!c || !mult || !sens) return fail(SSE_EINVAL, "null argument");
  Phantom* ph = nullptr;
  if (sse_status st = check_grid(c, grid, ph); st != SSE_OK) return st;
  if (sse_status st = check_subsets(0, n_subsets, c->sn.n_view); st != SSE_OK) return st;
  if (sse_status st = check_tof(c, 1); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (sse_status st = ensure_lor_tables(c); st != SSE_OK) return st;
  const uint64_t n_sv_max = (static_cast<uint64_t>(c->sn.n_view) + n_subsets - 1) / n_subsets;
  const uint64_t fp = static_cast<uint64_t>(c->sn.n_tof) * c->sn.n_plane * n_sv_max * c->sn.n_rad;
  const uint64_t img = static_cast<uint64_t>(ph->desc.nx) * ph->desc.ny * c->sn.n_plane;
  if (sse_status st = ensure_recon_scratch(c, fp, img); st != SSE_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  for (int sub = 0; sub < n_subsets; ++sub) {
    const sse::ReconGeom g = geom_of(c, ph, sub, n_subsets);
    HIP_TRY(sse::launch_subset_sensitivity(g, mult, c->d_recon_fp, sens + static_cast<uint64_t>(sub) * img, s),
            "subset sensitivity");
  }
  return SSE_OK;
}

sse_status sse_osem(sse_ctx* c, sse_phantom_id grid, const float* prompts, const float* mult, const float* additive,
                    const float* sens, float* image, int n_iter, int n_subsets, void* stream) {
  if (!c || !prompts || !mult || !additive || !image) return fail(SSE_EINVAL, "null argument");
  if (n_iter < 0) return fail(SSE_EINVAL, "n_iter must be >= 0");
  if (sse_status st = check_tof(c, 1); st != SSE_OK) return st;
  Phantom* ph = nullptr;
  if (sse_status st = check_grid(c, grid, ph); st != SSE_OK) return st;
  if (sse_status st = check_subsets(0, n_subsets, c->sn.n_view); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (sse_status st = ensure_lor_tables(c); st != SSE_OK) return st;
  const uint64_t n_sv_max = (static_cast<uint64_t>(c->sn.n_view) + n_subsets - 1) / n_subsets;
  const uint64_t fp = static_cast<uint64_t>(c->sn.n_tof) * c->sn.n_plane * n_sv_max * c->sn.n_rad;
  const uint64_t img = static_cast<uint64_t>(ph->desc.nx) * ph->desc.ny * c->sn.n_plane;
  if (sse_status st = ensure_recon_scratch(c, fp, img); st != SSE_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  for (int it = 0; it < n_iter; ++it)
    for (int sub = 0; sub < n_subsets; ++sub) {
      const sse::ReconGeom g = geom_of(c, ph, sub, n_subsets);
      float* sub_sens = sens ? const_cast<float*>(sens) + static_cast<uint64_t>(sub) * img : c->d_recon_img[1];
      HIP_TRY(sse::launch_osem_subset(g, prompts, mult, additive, image, c->d_recon_fp, c->d_recon_img[0], sub_sens,
                                      sens != nullptr, s),
              "OSEM subset");
    }
  return SSE_OK;
}

sse_status sse_attenuation_factors(sse_ctx* c, sse_phantom_id id, float* out, void* stream) {
  if (!c || !out) return fail(SSE_EINVAL, "null argument");
  Phantom* ph = get_phantom(c, id);
  if (!ph) return fail(SSE_EINVAL, "unknown phantom id");
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (sse_status st = ensure_lor_tables(c); st != SSE_OK) return st;
  const sse_phantom_desc& d = ph->desc;
  const int np = c->sn.n_plane;
  const uint64_t img = static_cast<uint64_t>(d.nx) * d.ny * np;
  if (sse_status st = ensure_recon_scratch(c, 0, img); st != SSE_OK) return st;
  // plane p reads the voxel slice nearest its z
  const double half_pitch = 0.5 * static_cast<double>(c->sc.length_mm) / c->sc.n_rings;
  std::vector<int> iz_of(np);
  for (int p = 0; p < np; ++p) {
    const double z = -0.5 * c->sc.length_mm + (p + 1) * half_pitch;
    double iz = std::floor((z - d.lo_mm[2]) / d.voxel_mm[2]);
    iz = iz < 0.0 ? 0.0 : (iz > d.nz - 1 ? static_cast<double>(d.nz - 1) : iz);
    iz_of[p] = static_cast<int>(iz);
  }
  int* d_iz = nullptr;
  HIP_TRY(hipMalloc(&d_iz, np * sizeof(int)), "allocate plane table");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(d_iz, iz_of.data(), np * sizeof(int), hipMemcpyHostToDevice, s);
  const sse::ReconGeom g = geom_of(c, ph, 0, 1);
  if (e == hipSuccess) e = sse::launch_attenuation_factors(g, ph->d_mu, d_iz, c->d_recon_img[0], out, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release(d_iz);
  if (e != hipSuccess) return hip_fail(e, "attenuation factors");
  return SSE_OK;
}

sse_status sse_image_to_activity(sse_ctx* c, sse_phantom_id id, const float* image, void* stream) {
  if (!c || !image) return fail(SSE_EINVAL, "null argument");
  Phantom* ph = get_phantom(c, id);
  if (!ph) return fail(SSE_EINVAL, "unknown phantom id");
  if (sse_status st = refuse_while_serving(c, "cannot update an activity"); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  const sse_phantom_desc& d = ph->desc;
  const uint64_t slice = static_cast<uint64_t>(d.nx) * d.ny, np = c->sn.n_plane;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // the image copy (pinned) and the activity are kept with the phantom's
  // alias-table workspace, so that repeated updates reuse their pages
  if (!ph->alias_work) ph->alias_work = std::make_shared<AliasWork>();
  AliasWork& w = *ph->alias_work;
  if (w.image_cap < slice * np) {
    if (w.image) (void)hipHostFree(w.image);
    w.image = nullptr;
    w.image_cap = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.image), slice * np * sizeof(float), hipHostMallocDefault),
            "allocate pinned image copy");
    w.image_cap = slice * np;
  }
  const float* im = w.image;
  HIP_TRY(hipMemcpyAsync(w.image, image, slice * np * sizeof(float), hipMemcpyDeviceToHost, s), "copy image");
  HIP_TRY(hipStreamSynchronize(s), "synchronise image copy");
  // phantom slice iz takes the image slice of the plane nearest its centre
  const double half_pitch = 0.5 * static_cast<double>(c->sc.length_mm) / c->sc.n_rings;
  std::vector<float>& act = w.act;
  act.resize(slice * static_cast<uint64_t>(d.nz));
  for (int iz = 0; iz < d.nz; ++iz) {
    const double z = d.lo_mm[2] + (iz + 0.5) * static_cast<double>(d.voxel_mm[2]);
    double fp = std::nearbyint((z + 0.5 * c->sc.length_mm) / half_pitch - 1.0);
    fp = fp < 0.0 ? 0.0 : (fp > static_cast<double>(np - 1) ? static_cast<double>(np - 1) : fp);
    const float* src = im + static_cast<uint64_t>(fp) * slice;
    float* dst = act.data() + static_cast<uint64_t>(iz) * slice;
    for (uint64_t i = 0; i < slice; ++i) dst[i] = src[i] > 0.0f && std::isfinite(src[i]) ? src[i] : 0.0f;
  }
  return sse_update_activity(c, id, act.data(), SSE_MEM_HOST, stream);
}

}  // extern "C"
