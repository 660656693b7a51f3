// C ABI of libsse.so: context and resource management, argument validation,
// emission alias tables, and launches of the transport and post-processing
// kernels.  Declarations and documentation: include/sse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "context.h"
#include "post.h"

namespace sse_detail {

constexpr double kTwoPiD = 6.283185307179586;

thread_local std::string g_error;

sse_status fail(sse_status st, const std::string& msg) {
  g_error = msg;
  return st;
}

sse_status hip_fail(hipError_t e, const char* what) {
  g_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? SSE_ENOMEM : SSE_EDEVICE;
}

void release(void* p) {
  if (p) (void)hipFree(p);
}

sse_status refuse_while_serving(const sse_ctx* c, const char* what) {
  if (c->servers.load() > 0)
    return fail(SSE_EBUSY, std::string(what) + " while a server runs on the context (stop it first)");
  return SSE_OK;
}

// With gaps, the LUT's crystal axes carry the virtual gap indices (or are
// ignored with size 1).
bool lut_fits_gaps(const sse_scanner_desc& sc, const sse_lut_desc& d) {
  const int cm = sc.crystals_per_module, rb = sc.rings_per_block, nb = sc.n_rings / rb;
  return (d.dims[3] == 1 || d.dims[3] == cm + 2) && (d.dims[4] == 1 || d.dims[4] == nb * (rb + 2));
}

Phantom* get_phantom(sse_ctx* c, sse_phantom_id id) {
  if (!c) return nullptr;
  std::lock_guard<std::mutex> lk(c->phantoms_mu);
  if (id == 0 || id > c->phantoms.size() || !c->phantoms[id - 1]->used) return nullptr;
  return c->phantoms[id - 1].get();
}

void build_transport_params(const sse_ctx* c, const Phantom* ph, uint64_t seed, uint64_t h0, uint64_t n,
                            sse::TransportParams& p) {
  p = sse::TransportParams{};
  const sse_phantom_desc& d = ph->desc;
  p.mu = ph->d_mu;
  p.mu8 = ph->d_mu8;
  p.mu_table = ph->d_mu_table;
  p.alias = ph->d_alias;
  p.nvox = ph->nvox;
  p.nx = d.nx; p.ny = d.ny; p.nz = d.nz;
  p.inv_nx = 1.0f / static_cast<float>(d.nx);
  p.inv_nxy = 1.0f / static_cast<float>(d.nx * d.ny);
  p.vx = d.voxel_mm[0]; p.vy = d.voxel_mm[1]; p.vz = d.voxel_mm[2];
  p.lox = d.lo_mm[0]; p.loy = d.lo_mm[1]; p.loz = d.lo_mm[2];
  p.hix = p.lox + static_cast<float>(d.nx) * p.vx;
  p.hiy = p.loy + static_cast<float>(d.ny) * p.vy;
  p.hiz = p.loz + static_cast<float>(d.nz) * p.vz;
  p.ivx = 1.0f / p.vx; p.ivy = 1.0f / p.vy; p.ivz = 1.0f / p.vz;
  p.fx_max = static_cast<float>(d.nx - 1);
  p.fy_max = static_cast<float>(d.ny - 1);
  p.fz_max = static_cast<float>(d.nz - 1);
  // (iz ny + iy) < ny nz and each factor below 2^24: exact 24-bit products
  p.vox24 = static_cast<uint64_t>(d.ny) * static_cast<uint64_t>(d.nz) <= (1ull << 24) && d.nx < (1 << 24);
  // every index below 2^24: the binary32 sums iz nx ny + iy nx + ix are exact
  p.voxf = static_cast<uint64_t>(d.nx) * static_cast<uint64_t>(d.ny) * static_cast<uint64_t>(d.nz) <= (1ull << 24);
  p.fnx = static_cast<float>(d.nx);
  p.fnxy = static_cast<float>(static_cast<uint64_t>(d.nx) * static_cast<uint64_t>(d.ny));
  p.mu_maj = c->ph.mu_majorant > 0.0f ? c->ph.mu_majorant : ph->mu_max;
  p.n_crystals = c->sc.n_crystals;
  p.n_rings = c->sc.n_rings;
  p.cmod = c->sc.crystals_per_module;
  p.rblk = c->sc.rings_per_block;
  p.max_ring_diff = c->sc.max_ring_diff;
  p.rr = c->sc.radius_mm * c->sc.radius_mm;
  p.half_len = 0.5f * c->sc.length_mm;
  p.pitch = c->sc.length_mm / static_cast<float>(c->sc.n_rings);
  p.n_rad = c->sn.n_rad; p.n_view = c->sn.n_view; p.n_plane = c->sn.n_plane; p.n_tof = c->sn.n_tof;
  p.tof_bin = c->sn.tof_bin_mm;
  p.tof_sigma = c->sn.tof_sigma_mm;
  p.e_lo = c->ph.e_lo_kev; p.e_hi = c->ph.e_hi_kev; p.e_kill = c->ph.e_kill_kev; p.e_fwhm = c->ph.e_fwhm_frac;
  p.rayleigh_beta = c->ph.rayleigh_beta;
  p.kc = c->ph.f_compton / sse::kn_total32(1.0f);
  p.f_r = c->ph.f_rayleigh;
  p.f_p = c->ph.f_photo;
  p.max_int = c->ph.max_interactions;
  // coefficients at 511 keV, evaluated once on the host (same binary32 model)
  sse::energy_coefficients(p.e511, sse::kMec2, p.kc, p.f_r, p.f_p, p.mu_maj);
  p.lut = c->d_lut;
  p.lut_type = c->lut_type;
  p.d0 = c->lut.dims[0]; p.d1 = c->lut.dims[1]; p.d2 = c->lut.dims[2]; p.d3 = c->lut.dims[3]; p.d4 = c->lut.dims[4];
  p.e_min = c->lut.e_min_kev;
  p.e_scale = static_cast<float>(c->lut.dims[0]) / (c->lut.e_max_kev - c->lut.e_min_kev);
  p.gap_on = c->gaps_on;
  if (c->gaps_on) {
    const int rb = c->sc.rings_per_block;
    p.n_mod = c->sc.n_crystals / c->sc.crystals_per_module;
    p.n_blk = c->sc.n_rings / rb;
    p.gap_policy = c->gaps.policy;
    p.gap_t = static_cast<double>(c->gaps.transaxial_gap_rad);
    p.mod_d = kTwoPiD / static_cast<double>(p.n_mod);
    const double L = static_cast<double>(c->sc.length_mm), w = static_cast<double>(c->gaps.axial_gap_mm);
    p.half_len_d = 0.5 * L;
    p.gap_a = w;
    p.pitch_a = (L - static_cast<double>(p.n_blk - 1) * w) / static_cast<double>(c->sc.n_rings);
    p.block_span = static_cast<double>(rb) * p.pitch_a;
    p.block_period = p.block_span + w;
    p.edge_t = c->d_edge[0];
    p.edge_a = c->d_edge[1];
    p.edge_na = c->gaps.edge_n_angle;
    p.edge_np = c->gaps.edge_n_pos;
  }
  p.prune_b = c->prune_b;
  p.seed = seed;
  p.h0 = h0;
  p.rec_h0 = h0;
  p.n = n;
}

}  // namespace sse_detail

using namespace sse_detail;

namespace {

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

// Path lengths of a ray in the lower (x <= -w/2) and upper (x >= w/2) block
// of the slab 0 <= depth <= D: the ray crosses depth doi at lateral position
// x with angle theta to the depth axis, so its lateral coordinate runs
// linearly from xf at the front face to xb at the back face over a path of
// D / cos(theta).
void edge_ray_paths(const sse_edge_geom& g, double theta, double x, double& lo, double& hi, bool& lower_first) {
  const double D = static_cast<double>(g.depth_mm), hw = 0.5 * static_cast<double>(g.gap_mm);
  const double doi = static_cast<double>(g.doi_mm);
  const double t = std::tan(theta);
  const double xf = x - doi * t, xb = x + (D - doi) * t;
  const double len = D / std::cos(theta);
  lower_first = xb >= xf;
  if (xf == xb) {
    lo = xf <= -hw ? len : 0.0;
    hi = xf >= hw ? len : 0.0;
    return;
  }
  // share of the path before the lateral coordinate passes xc
  auto share = [&](double xc) { return std::min(1.0, std::max(0.0, (xc - xf) / (xb - xf))); };
  if (xb > xf) {
    lo = len * share(-hw);
    hi = len * (1.0 - share(hw));
  } else {
    lo = len * (1.0 - share(-hw));
    hi = len * share(hw);
  }
}

sse_status check_descs(const sse_scanner_desc* s, const sse_sino_desc* n, const sse_physics_desc* p) {
  if (!s || !n || !p) return fail(SSE_EINVAL, "null descriptor");
  if (s->n_crystals <= 0 || s->n_crystals % 2) return fail(SSE_EINVAL, "n_crystals must be even and positive");
  if (s->n_rings <= 0) return fail(SSE_EINVAL, "n_rings must be positive");
  if (!finite_pos(s->radius_mm) || !finite_pos(s->length_mm)) return fail(SSE_EINVAL, "radius and length must be positive");
  if (s->crystals_per_module <= 0 || s->rings_per_block <= 0)
    return fail(SSE_EINVAL, "crystals_per_module and rings_per_block must be positive");
  if (n->n_view != s->n_crystals / 2) return fail(SSE_EINVAL, "n_view must equal n_crystals / 2");
  if (n->n_plane != 2 * s->n_rings - 1) return fail(SSE_EINVAL, "n_plane must equal 2 n_rings - 1");
  if (n->n_rad <= 0 || n->n_rad % 2 == 0 || n->n_rad > s->n_crystals - 1)
    return fail(SSE_EINVAL, "n_rad must be odd and at most n_crystals - 1");
  if (n->n_tof <= 0) return fail(SSE_EINVAL, "n_tof must be positive");
  if (!finite_pos(n->tof_bin_mm) || !(n->tof_sigma_mm >= 0.0f) || !std::isfinite(n->tof_sigma_mm))
    return fail(SSE_EINVAL, "bad TOF bin width or jitter");
  if (!(p->e_lo_kev <= p->e_hi_kev) || !std::isfinite(p->e_lo_kev) || !std::isfinite(p->e_hi_kev))
    return fail(SSE_EINVAL, "bad energy window");
  if (!(p->e_kill_kev >= 100.0f) || !std::isfinite(p->e_kill_kev))
    return fail(SSE_EINVAL, "kill energy must be >= 100 keV (range of the binary32 energy model)");
  if (!(p->e_fwhm_frac >= 0.0f) || !std::isfinite(p->e_fwhm_frac)) return fail(SSE_EINVAL, "bad energy blur");
  if (!(p->f_compton >= 0.0f) || !(p->f_rayleigh >= 0.0f) || !(p->f_photo >= 0.0f) ||
      !(p->f_compton + p->f_rayleigh + p->f_photo > 0.0f) || !std::isfinite(p->f_compton + p->f_rayleigh + p->f_photo))
    return fail(SSE_EINVAL, "bad interaction fractions");
  if (!finite_pos(p->rayleigh_beta)) return fail(SSE_EINVAL, "rayleigh_beta must be positive");
  if (!(p->mu_majorant >= 0.0f) || !std::isfinite(p->mu_majorant)) return fail(SSE_EINVAL, "bad majorant");
  if (p->max_interactions < 1) return fail(SSE_EINVAL, "max_interactions must be >= 1");
  const uint64_t bins = static_cast<uint64_t>(n->n_rad) * n->n_view * n->n_plane * n->n_tof;
  if (bins >= (static_cast<uint64_t>(1) << 62)) return fail(SSE_EINVAL, "sinogram too large");
  return SSE_OK;
}

// Copy n floats of host or device memory to a host vector.
sse_status fetch_floats(const float* src, uint64_t n, int mem, hipStream_t s, std::vector<float>& dst) {
  dst.resize(n);
  if (mem == SSE_MEM_HOST) {
    std::memcpy(dst.data(), src, n * sizeof(float));
    return SSE_OK;
  }
  if (mem != SSE_MEM_DEVICE) return fail(SSE_EINVAL, "mem must be SSE_MEM_HOST or SSE_MEM_DEVICE");
  HIP_TRY(hipMemcpyAsync(dst.data(), src, n * sizeof(float), hipMemcpyDeviceToHost, s), "copy input to host");
  HIP_TRY(hipStreamSynchronize(s), "synchronise input copy");
  return SSE_OK;
}

// Integer alias table (see sse_build_alias_table), packed as (threshold,
// alias) pairs into out; returns false on bad input.  The sum runs in index
// order (its rounding is part of the definition); each voxel's mass depends
// only on its activity and the sum, so the masses are computed in parallel,
// the remainder going to the first largest; Vose's pairing is sequential by
// definition and runs on the two stacks of the workspace.
bool build_alias(const float* act, uint64_t n, AliasWork& w, uint2* out, double* sum_out) {
  if (n == 0 || n > 0xffffffffull) return false;
  double sum = 0.0;
  bool bad = false;
  for (uint64_t i = 0; i < n; ++i) {
    const double a = static_cast<double>(act[i]);
    bad |= !(a >= 0.0) || std::isinf(a);
    sum += a;
  }
  if (bad || !(sum > 0.0) || std::isinf(sum)) return false;
  constexpr uint64_t T = static_cast<uint64_t>(1) << 32;
  if (w.mass.size() < n) {
    w.mass.resize(n);
    w.small.resize(n);
    w.large.resize(n);
  }
  uint64_t* mass = w.mass.data();
  const double scale = static_cast<double>(n) * 4294967296.0 / sum;
  const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const unsigned nt = n >= (1u << 20) ? hw : 1u;
  std::vector<uint64_t> part_total(nt, 0), part_max(nt, 0);
  auto quantise = [&](unsigned t) {
    const uint64_t a = n * t / nt, b = n * (t + 1) / nt;
    uint64_t tot = 0, m = a;
    for (uint64_t i = a; i < b; ++i) {
      const uint64_t v = static_cast<uint64_t>(std::floor(static_cast<double>(act[i]) * scale));
      mass[i] = v;
      tot += v;
      if (v > mass[m]) m = i;
    }
    part_total[t] = tot;
    part_max[t] = m;
  };
  if (nt == 1) {
    quantise(0);
  } else {
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t) pool.emplace_back(quantise, t);
    for (auto& th : pool) th.join();
  }
  uint64_t total = 0, imax = part_max[0];
  for (unsigned t = 0; t < nt; ++t) {
    total += part_total[t];
    if (mass[part_max[t]] > mass[imax]) imax = part_max[t];
  }
  mass[imax] += n * T - total;
  uint32_t* small = w.small.data();
  uint32_t* large = w.large.data();
  uint64_t ns = 0, nl = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (mass[i] < T) small[ns++] = static_cast<uint32_t>(i);
    else large[nl++] = static_cast<uint32_t>(i);
  }
  // Vose's pairing, one pop of each stack per column: g, on top of the large
  // stack, pairs with the small columns popped one by one and keeps its
  // remaining mass in a register until it falls below 2^32 (pushed on the
  // small stack, so that it is the next small column) or the small stack
  // runs out (pushed back on the large one) -- the same pops and pushes as
  // popping both stacks for every column.
  while (ns && nl) {
    const uint32_t g = large[--nl];
    uint64_t mg = mass[g];
    for (;;) {
      const uint32_t l = small[--ns];
      const uint64_t ml = mass[l];
      out[l] = make_uint2(static_cast<uint32_t>(ml), g);
      mg -= T - ml;
      if (mg < T) {
        mass[g] = mg;
        small[ns++] = g;
        break;
      }
      if (ns == 0) {
        mass[g] = mg;
        large[nl++] = g;
        break;
      }
    }
  }
  while (nl) {
    const uint32_t g = large[--nl];
    out[g] = make_uint2(0xffffffffu, g);
  }
  while (ns) {
    const uint32_t l = small[--ns];
    out[l] = make_uint2(0xffffffffu, l);
  }
  if (sum_out) *sum_out = sum;
  return true;
}

// Build a phantom's alias table from host activity into its pinned staging
// buffer and upload it on stream s (synchronous: the table is in place for
// work on any stream when this returns).
sse_status upload_alias(const float* act_host, hipStream_t s, Phantom& p) {
  if (!p.alias_work) p.alias_work = std::make_shared<AliasWork>();
  AliasWork& w = *p.alias_work;
  const uint64_t n = p.nvox;
  if (w.staging_cap < n) {
    if (w.staging) (void)hipHostFree(w.staging);
    w.staging = nullptr;
    w.staging_cap = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&w.staging), n * sizeof(uint2), hipHostMallocDefault),
            "allocate alias staging buffer");
    w.staging_cap = n;
  }
  double sum = 0.0;
  if (!build_alias(act_host, n, w, w.staging, &sum))
    return fail(SSE_EINVAL, "activity must be finite, non-negative and not all zero");
  HIP_TRY(hipMemcpyAsync(p.d_alias, w.staging, n * sizeof(uint2), hipMemcpyHostToDevice, s), "upload alias table");
  HIP_TRY(hipStreamSynchronize(s), "synchronise alias upload");
  p.activity_sum = sum;
  return SSE_OK;
}

// Attenuation maps with at most 256 distinct values (segmented phantoms)
// are also stored as one-byte indices into a table of the exact values: the
// kernel reads the same binary32 numbers from a map a quarter of the size,
// which stays resident in each XCD's L2.
sse_status upload_palette(const std::vector<float>& mu, hipStream_t s, Phantom& p) {
  std::map<uint32_t, uint32_t> index;
  for (float m : mu) {
    uint32_t bits;
    std::memcpy(&bits, &m, 4);
    if (index.emplace(bits, 0u).second && index.size() > 256) return SSE_OK;  // no palette
  }
  std::vector<float> table(256, 0.0f);
  uint32_t k = 0;
  for (auto& kv : index) {
    kv.second = k;
    std::memcpy(&table[k], &kv.first, 4);
    ++k;
  }
  std::vector<uint8_t> idx(mu.size());
  for (size_t i = 0; i < mu.size(); ++i) {
    uint32_t bits;
    std::memcpy(&bits, &mu[i], 4);
    idx[i] = static_cast<uint8_t>(index[bits]);
  }
  HIP_TRY(hipMalloc(&p.d_mu8, mu.size()), "allocate palette map");
  HIP_TRY(hipMalloc(&p.d_mu_table, 256 * sizeof(float)), "allocate palette");
  HIP_TRY(hipMemcpyAsync(p.d_mu8, idx.data(), mu.size(), hipMemcpyHostToDevice, s), "upload palette map");
  HIP_TRY(hipMemcpyAsync(p.d_mu_table, table.data(), 256 * sizeof(float), hipMemcpyHostToDevice, s), "upload palette");
  HIP_TRY(hipStreamSynchronize(s), "synchronise palette upload");
  return SSE_OK;
}

sse::PostParams post_params(const sse_ctx* c) {
  return sse::PostParams{c->sn.n_rad, c->sn.n_view, c->sn.n_plane, c->sn.n_tof};
}

// Pair buffer for runs of n histories: the records one launch of n needs in
// the worst case (in either launch form), at most pair_cap_max (2^27 = 10.7
// GB unless set: a run beyond it goes through fill launches, which end when
// the buffer is nearly full), rounded up to 2^16 and grown when needed
// (halved down to 2^22 while allocation fails); and the work-list scratch of
// the production path.
constexpr uint64_t kMinPairCap = 1ull << 22;
sse_status ensure_pairs(sse_ctx* c, uint64_t n) {
  const uint64_t kDefaultCap = c->pair_cap_max;
  constexpr uint64_t kMinCap = kMinPairCap;
  if (!c->d_item) HIP_TRY(hipMalloc(&c->d_item, sizeof(sse::TransportParams)), "allocate work-list scratch");
  if (!c->d_chunk) HIP_TRY(hipMalloc(&c->d_chunk, sizeof(sse::WorkChunk)), "allocate work-list scratch");
  if (!c->d_cursor)
    HIP_TRY(hipMalloc(&c->d_cursor, sse::kCursorWords * sizeof(uint32_t)), "allocate work-list scratch");
  const uint64_t want = std::max(sse::transport_pairs_needed(n), sse::transport_batch_pairs_needed(n));
  uint64_t cap = want < kDefaultCap ? want : kDefaultCap;
  cap = (cap + 0xffffull) & ~0xffffull;
  if (c->d_pairs && c->pair_cap >= cap) return SSE_OK;
  if (!c->d_pair_count) HIP_TRY(hipMalloc(&c->d_pair_count, sizeof(uint32_t)), "allocate pair counter");
  if (c->d_pairs) {  // the freeing waits for the device
    release(c->d_pairs);
    c->d_pairs = nullptr;
    c->pair_cap = 0;
  }
  for (;;) {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, static_cast<size_t>(sse::kPairWords) * cap * sizeof(uint32_t)) == hipSuccess) {
      c->d_pairs = static_cast<uint32_t*>(ptr);
      break;
    }
    (void)hipGetLastError();
    if (cap <= kMinCap) return fail(SSE_ENOMEM, "cannot allocate the pair buffer");
    cap /= 2;
  }
  c->pair_cap = cap;
  return SSE_OK;
}

sse_status ensure_scratch(sse_ctx* c) {
  for (int i = 0; i < 2; ++i)
    if (!c->d_scratch[i]) HIP_TRY(hipMalloc(&c->d_scratch[i], c->n_bins * sizeof(float)), "allocate smoothing scratch");
  return SSE_OK;
}

// Separable smoothing of `in` (binary32, or binary64 weights times `scale`
// rounded on load) into `out`, optionally multiplied by the sensitivity;
// with ratio_w the last pass writes G / float(scale ratio_w) instead of the
// smoothed G (1 where either is not positive).
sse_status smooth(sse_ctx* c, const void* in, bool in_is_f64, double scale, float* out, const float* sigma,
                  float truncate, const float* sens, hipStream_t s, const float* norm = nullptr,
                  const double* ratio_w = nullptr) {
  if (!sigma) return fail(SSE_EINVAL, "null sigma");
  if (!in || !out) return fail(SSE_EINVAL, "null buffer");
  if (!(truncate > 0.0f) || !std::isfinite(truncate)) return fail(SSE_EINVAL, "truncate must be positive");
  sse::Taps taps[3] = {};  // by axis
  bool on[3] = {};
  for (int a = 0; a < 3; ++a) {
    const float sg = sigma[a];
    if (!(sg >= 0.0f) || !std::isfinite(sg)) return fail(SSE_EINVAL, "sigma must be finite and >= 0");
    if (sg == 0.0f) continue;
    const double sd = sg;
    const int radius = static_cast<int>(static_cast<double>(truncate) * sd + 0.5);
    if (radius > sse::kMaxSmoothRadius) return fail(SSE_EINVAL, "smoothing kernel wider than 127 taps");
    double w[2 * sse::kMaxSmoothRadius + 1], tot = 0.0;
    for (int k = -radius; k <= radius; ++k) {
      w[k + radius] = std::exp(-0.5 * k * k / (sd * sd));
      tot += w[k + radius];
    }
    taps[a].radius = radius;
    for (int k = 0; k <= 2 * radius; ++k) taps[a].w[k] = static_cast<float>(w[k] / tot);
    on[a] = true;
  }
  const sse::PostParams g = post_params(c);
  if (!on[0] && !on[1] && !on[2]) {  // elementwise (in place allowed)
    HIP_TRY(sse::launch_smooth_axis(g, -1, in, in_is_f64, scale, norm, out, taps[0], norm, sens, c->sens_tof, ratio_w,
                                    s),
            "pointwise kernel");
    return SSE_OK;
  }
  // The passes: radial and plane in one launch when both are smoothed and
  // the tile fits in LDS, then the view pass; otherwise one pass per axis.
  // The axes commute (each pass is linear along its own axis, and the view
  // seam's reversal of the radial and TOF indices commutes with the radial
  // sum, whose taps and reflection are symmetric).
  constexpr int kFused = 3;
  sse::FusedPlan plan{};
  if (on[0] && on[2]) plan = sse::plan_rad_plane(g, taps[0].radius, taps[2].radius);
  int passes[3], np = 0;
  if (plan.tl > 0) {
    passes[np++] = kFused;
    if (on[1]) passes[np++] = 1;
  } else {
    for (int a = 0; a < 3; ++a)
      if (on[a]) passes[np++] = a;
  }
  sse_status st = ensure_scratch(c);
  if (st != SSE_OK) return st;
  // A pass never reads and writes the same buffer: with in == out and one
  // pass the result goes through scratch.
  const void* src = in;
  bool src_f64 = in_is_f64;
  float* dst = nullptr;
  for (int i = 0; i < np; ++i) {
    const bool last = i == np - 1;
    dst = (last && !(np == 1 && in == out)) ? out : c->d_scratch[i % 2];
    const float* n_in = i == 0 ? norm : nullptr;
    const float* n_out = last ? norm : nullptr;
    const float* sv = last ? sens : nullptr;
    const double* rw = last ? ratio_w : nullptr;
    if (passes[i] == kFused)
      HIP_TRY(sse::launch_smooth_rad_plane(g, plan, src, src_f64, scale, n_in, dst, taps[0], taps[2], n_out, sv,
                                           c->sens_tof, rw, s),
              "smoothing kernel (radial and plane)");
    else
      HIP_TRY(sse::launch_smooth_axis(g, passes[i], src, src_f64, scale, n_in, dst, taps[passes[i]], n_out, sv,
                                      c->sens_tof, rw, s),
              "smoothing kernel");
    src = dst;
    src_f64 = false;
  }
  if (dst != out)
    HIP_TRY(hipMemcpyAsync(out, dst, c->n_bins * sizeof(float), hipMemcpyDeviceToDevice, s), "copy smoothed");
  return SSE_OK;
}

}  // namespace

extern "C" {

int sse_abi_version(void) { return SSE_ABI_VERSION; }

const char* sse_last_error(void) { return g_error.c_str(); }

sse_status sse_build_alias_table(const float* activity, uint64_t n, uint32_t* thresh, uint32_t* alias) {
  if (!activity || !thresh || !alias) return fail(SSE_EINVAL, "null pointer");
  if (n == 0 || n > 0xffffffffull) return fail(SSE_EINVAL, "activity must have 1 .. 2^32 - 1 entries");
  AliasWork w;
  std::vector<uint2> packed(n);
  if (!build_alias(activity, n, w, packed.data(), nullptr))
    return fail(SSE_EINVAL, "activity must be finite, non-negative and not all zero");
  for (uint64_t i = 0; i < n; ++i) {
    thresh[i] = packed[i].x;
    alias[i] = packed[i].y;
  }
  return SSE_OK;
}

sse_status sse_create(sse_ctx** out, int device, const sse_scanner_desc* scanner, const sse_sino_desc* sino,
                      const sse_physics_desc* physics) {
  if (!out) return fail(SSE_EINVAL, "null output pointer");
  *out = nullptr;
  sse_status st = check_descs(scanner, sino, physics);
  if (st != SSE_OK) return st;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count), "count devices");
  if (device < 0 || device >= count) return fail(SSE_EINVAL, "no such HIP device");
  HIP_TRY(hipSetDevice(device), "set device");
  HIP_TRY(sse::upload_log_table(), "upload the free-path logarithm's table");
  // the device's allocation-free scratch (looked up once per device)
  HIP_TRY(sse::noalloc_scratch_init(device), "find the allocation-free scratch");
  hipEvent_t ev = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "create event");
  sse_ctx* c = new (std::nothrow) sse_ctx();
  if (!c) {
    (void)hipEventDestroy(ev);
    return fail(SSE_ENOMEM, "host allocation");
  }
  c->pair_done = ev;
  c->device = device;
  c->sc = *scanner;
  c->sn = *sino;
  c->ph = *physics;
  c->n_bins = static_cast<uint64_t>(sino->n_rad) * sino->n_view * sino->n_plane * sino->n_tof;
  *out = c;
  return SSE_OK;
}

sse_status sse_destroy(sse_ctx* c) {
  if (!c) return SSE_OK;
  if (sse_status st = refuse_while_serving(c, "cannot destroy the context"); st != SSE_OK) return st;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& p : c->phantoms) {
    release(p->d_mu);
    release(p->d_alias);
    release(p->d_mu8);
    release(p->d_mu_table);
  }
  if (c->d_lut) release(c->d_lut);
  if (c->d_sens) release(c->d_sens);
  for (float* e : c->d_edge) release(e);
  for (auto* s : c->d_scratch)
    if (s) release(s);
  if (c->d_partials) release(c->d_partials);
  release(c->d_lor);
  release(c->d_view);
  release(c->d_qtab);
  release(c->d_major);
  release(c->d_recon_fp);
  release(c->d_recon_img[0]);
  release(c->d_recon_img[1]);
  if (c->d_pairs) release(c->d_pairs);
  if (c->d_item) release(c->d_item);
  if (c->d_chunk) release(c->d_chunk);
  if (c->d_cursor) release(c->d_cursor);
  if (c->d_pair_count) release(c->d_pair_count);
  if (c->pair_done) (void)hipEventDestroy(c->pair_done);
  for (hipEvent_t e : c->timing_ev) (void)hipEventDestroy(e);
  delete c;
  return SSE_OK;
}

sse_status sse_load_phantom(sse_ctx* c, const sse_phantom_desc* d, const float* mu, const float* activity, int mem,
                            void* stream, sse_phantom_id* out) {
  if (!c || !d || !mu || !activity || !out) return fail(SSE_EINVAL, "null argument");
  if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0) return fail(SSE_EINVAL, "phantom dimensions must be positive");
  for (int i = 0; i < 3; ++i)
    if (!finite_pos(d->voxel_mm[i]) || !std::isfinite(d->lo_mm[i])) return fail(SSE_EINVAL, "bad voxel size or origin");
  const uint64_t n = static_cast<uint64_t>(d->nx) * d->ny * d->nz;
  if (n > 0xffffffffull) return fail(SSE_EINVAL, "too many voxels");
  // the voxel box must lie inside the detection cylinder transaxially
  const double R = c->sc.radius_mm;
  for (int cx = 0; cx < 2; ++cx)
    for (int cy = 0; cy < 2; ++cy) {
      const double x = d->lo_mm[0] + cx * static_cast<double>(d->nx) * d->voxel_mm[0];
      const double y = d->lo_mm[1] + cy * static_cast<double>(d->ny) * d->voxel_mm[1];
      if (!(x * x + y * y < R * R)) return fail(SSE_EINVAL, "phantom box reaches outside the detection cylinder");
    }
  HIP_TRY(hipSetDevice(c->device), "set device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> hmu, hact;
  sse_status st = fetch_floats(mu, n, mem, s, hmu);
  if (st != SSE_OK) return st;
  st = fetch_floats(activity, n, mem, s, hact);
  if (st != SSE_OK) return st;
  float mmax = 0.0f;
  for (float m : hmu) {
    if (!(m >= 0.0f) || !std::isfinite(m)) return fail(SSE_EINVAL, "attenuation must be finite and >= 0");
    mmax = m > mmax ? m : mmax;
  }
  if (c->ph.mu_majorant > 0.0f && c->ph.mu_majorant < mmax)
    return fail(SSE_EINVAL, "physics mu_majorant is below the phantom's maximum attenuation");
  Phantom p;
  p.used = true;
  p.desc = *d;
  p.nvox = n;
  p.mu_max = mmax;
  HIP_TRY(hipMalloc(&p.d_mu, n * sizeof(float)), "allocate attenuation map");
  hipError_t e = hipMalloc(&p.d_alias, n * sizeof(uint2));
  if (e != hipSuccess) {
    release(p.d_mu);
    return hip_fail(e, "allocate alias table");
  }
  st = upload_alias(hact.data(), s, p);
  if (st == SSE_OK) {
    e = hipMemcpyAsync(p.d_mu, hmu.data(), n * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "upload attenuation map");
  }
  if (st == SSE_OK) st = upload_palette(hmu, s, p);
  if (st != SSE_OK) {
    release(p.d_mu);
    release(p.d_alias);
    release(p.d_mu8);
    release(p.d_mu_table);
    return st;
  }
  p.device_bytes = n * (sizeof(float) + sizeof(uint2)) + (p.d_mu8 ? n + 256 * sizeof(float) : 0);
  std::lock_guard<std::mutex> lk(c->phantoms_mu);
  c->phantom_bytes += p.device_bytes;
  for (size_t i = 0; i < c->phantoms.size(); ++i)
    if (!c->phantoms[i]->used) {
      *c->phantoms[i] = p;
      *out = static_cast<sse_phantom_id>(i + 1);
      return SSE_OK;
    }
  c->phantoms.push_back(std::make_unique<Phantom>(p));
  *out = static_cast<sse_phantom_id>(c->phantoms.size());
  return SSE_OK;
}

sse_status sse_update_activity(sse_ctx* c, sse_phantom_id id, const float* activity, int mem, void* stream) {
  Phantom* p = get_phantom(c, id);
  if (!p) return fail(SSE_EINVAL, "unknown phantom id");
  if (sse_status st = refuse_while_serving(c, "cannot update an activity"); st != SSE_OK) return st;
  if (!activity) return fail(SSE_EINVAL, "null activity");
  HIP_TRY(hipSetDevice(c->device), "set device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!p->alias_work) p->alias_work = std::make_shared<AliasWork>();
  const float* host_act = activity;
  if (mem != SSE_MEM_HOST) {
    sse_status st = fetch_floats(activity, p->nvox, mem, s, p->alias_work->act);
    if (st != SSE_OK) return st;
    host_act = p->alias_work->act.data();
  }
  // Simulations queued before this call, on any stream, may still read the
  // table: every simulate records pair_done when it is enqueued, and each one
  // waits for the previous record, so the last record covers them all.
  if (c->pair_done) HIP_TRY(hipEventSynchronize(c->pair_done), "wait for simulations reading the phantom");
  return upload_alias(host_act, s, *p);
}

sse_status sse_unload_phantom(sse_ctx* c, sse_phantom_id id) {
  Phantom* p = get_phantom(c, id);
  if (!p) return fail(SSE_EINVAL, "unknown phantom id");
  if (sse_status st = refuse_while_serving(c, "cannot unload a phantom"); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(hipDeviceSynchronize(), "wait for pending work");
  release(p->d_mu);
  release(p->d_alias);
  release(p->d_mu8);
  release(p->d_mu_table);
  std::lock_guard<std::mutex> lk(c->phantoms_mu);
  c->phantom_bytes -= p->device_bytes;
  *p = Phantom();
  return SSE_OK;
}

sse_status sse_load_lut(sse_ctx* c, const sse_lut_desc* d, const void* values, int dtype, int mem, void* stream) {
  if (!c || !d || !values) return fail(SSE_EINVAL, "null argument");
  if (sse_status st = refuse_while_serving(c, "cannot replace the LUT"); st != SSE_OK) return st;
  uint64_t n = 1;
  for (int i = 0; i < 5; ++i) {
    if (d->dims[i] <= 0) return fail(SSE_EINVAL, "LUT dimensions must be positive");
    n *= static_cast<uint64_t>(d->dims[i]);
  }
  if (c->gaps_on && !lut_fits_gaps(c->sc, *d))
    return fail(SSE_EINVAL, "with gaps the LUT's crystal axes must be crystals_per_module + 2 and "
                            "n_blocks (rings_per_block + 2) long, or 1");
  if (n >= 0xffffffffull) return fail(SSE_EINVAL, "LUT too large");
  if (!(d->e_max_kev > d->e_min_kev) || !std::isfinite(d->e_min_kev) || !std::isfinite(d->e_max_kev))
    return fail(SSE_EINVAL, "LUT energy range must be increasing");
  size_t esz;
  if (dtype == SSE_F32) esz = 4;
  else if (dtype == SSE_F16 || dtype == SSE_BF16) esz = 2;
  else return fail(SSE_EINVAL, "LUT dtype must be SSE_F32, SSE_F16 or SSE_BF16");
  if (mem != SSE_MEM_HOST && mem != SSE_MEM_DEVICE) return fail(SSE_EINVAL, "bad mem kind");
  HIP_TRY(hipSetDevice(c->device), "set device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<unsigned char> host(n * esz);
  if (mem == SSE_MEM_HOST) {
    std::memcpy(host.data(), values, n * esz);
  } else {
    HIP_TRY(hipMemcpyAsync(host.data(), values, n * esz, hipMemcpyDeviceToHost, s), "copy LUT to host");
    HIP_TRY(hipStreamSynchronize(s), "synchronise LUT copy");
  }
  for (uint64_t i = 0; i < n; ++i) {
    float v;
    if (dtype == SSE_F32) {
      std::memcpy(&v, &host[i * 4], 4);
    } else {
      uint16_t b;
      std::memcpy(&b, &host[i * 2], 2);
      if (dtype == SSE_BF16) {
        const uint32_t u = static_cast<uint32_t>(b) << 16;
        std::memcpy(&v, &u, 4);
      } else {
        v = static_cast<float>(__builtin_bit_cast(_Float16, b));
      }
    }
    if (!(v >= 0.0f && v <= 1.0f)) return fail(SSE_EINVAL, "LUT values must lie in [0, 1]");
  }
  void* dptr = nullptr;
  HIP_TRY(hipMalloc(&dptr, n * esz), "allocate LUT");
  hipError_t e = hipMemcpyAsync(dptr, host.data(), n * esz, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release(dptr);
    return hip_fail(e, "upload LUT");
  }
  if (c->d_lut) {
    HIP_TRY(hipDeviceSynchronize(), "wait for pending work");
    release(c->d_lut);
  }
  c->d_lut = dptr;
  c->lut_type = dtype;
  c->lut = *d;
  return SSE_OK;
}

sse_status sse_load_sensitivity(sse_ctx* c, const float* sens, int has_tof_axis, int mem, void* stream) {
  if (!c || !sens) return fail(SSE_EINVAL, "null argument");
  const uint64_t n = has_tof_axis ? c->n_bins : c->n_bins / static_cast<uint64_t>(c->sn.n_tof);
  HIP_TRY(hipSetDevice(c->device), "set device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<float> h;
  sse_status st = fetch_floats(sens, n, mem, s, h);
  if (st != SSE_OK) return st;
  for (float v : h)
    if (!(v >= 0.0f) || !std::isfinite(v)) return fail(SSE_EINVAL, "sensitivity must be finite and >= 0");
  float* d = nullptr;
  HIP_TRY(hipMalloc(&d, n * sizeof(float)), "allocate sensitivity");
  hipError_t e = hipMemcpyAsync(d, h.data(), n * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release(d);
    return hip_fail(e, "upload sensitivity");
  }
  if (c->d_sens) {
    HIP_TRY(hipDeviceSynchronize(), "wait for pending work");
    release(c->d_sens);
  }
  c->d_sens = d;
  c->sens_tof = has_tof_axis ? 1 : 0;
  return SSE_OK;
}

sse_status sse_set_pair_buffer(sse_ctx* c, uint64_t max_records) {
  if (!c) return fail(SSE_EINVAL, "null context");
  if (max_records < kMinPairCap || max_records > sse::kMaxPairCap)
    return fail(SSE_EINVAL, "max_records must be 2^22 .. 2^31");
  if (sse_status st = refuse_while_serving(c, "cannot change the pair buffer"); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (c->d_pairs) {  // the freeing waits for the device; the next simulate allocates anew
    release(c->d_pairs);
    c->d_pairs = nullptr;
    c->pair_cap = 0;
  }
  c->pair_cap_max = max_records;
  return SSE_OK;
}

sse_status sse_set_pair_pruning(sse_ctx* c, int enable) {
  if (!c) return fail(SSE_EINVAL, "null context");
  if (enable != 0 && enable != 1) return fail(SSE_EINVAL, "enable must be 0 or 1");
  if (sse_status st = refuse_while_serving(c, "cannot change pair pruning"); st != SSE_OK) return st;
  c->prune_b = enable;
  return SSE_OK;
}

sse_status sse_set_gaps(sse_ctx* c, const sse_gap_desc* d, const float* edge_t, const float* edge_a, int mem,
                        void* stream) {
  if (!c) return fail(SSE_EINVAL, "null context");
  if (sse_status st = refuse_while_serving(c, "cannot change the gap model"); st != SSE_OK) return st;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (!d) {
    HIP_TRY(hipDeviceSynchronize(), "wait for pending work");
    for (float*& e : c->d_edge) {
      release(e);
      e = nullptr;
    }
    c->gaps_on = 0;
    c->gaps = sse_gap_desc{};
    return SSE_OK;
  }
  const int cm = c->sc.crystals_per_module, rb = c->sc.rings_per_block;
  if (c->sc.n_crystals % cm || c->sc.n_rings % rb)
    return fail(SSE_EINVAL, "gaps need whole modules and blocks: n_crystals a multiple of crystals_per_module, "
                            "n_rings of rings_per_block");
  const int nm = c->sc.n_crystals / cm, nb = c->sc.n_rings / rb;
  if (!(d->transaxial_gap_rad >= 0.0f) || !(static_cast<double>(d->transaxial_gap_rad) < kTwoPiD / nm))
    return fail(SSE_EINVAL, "transaxial gap angle must lie in [0, 2 pi / n_modules)");
  if (!(d->axial_gap_mm >= 0.0f) ||
      !(static_cast<double>(nb - 1) * static_cast<double>(d->axial_gap_mm) < static_cast<double>(c->sc.length_mm)))
    return fail(SSE_EINVAL, "axial gaps must be >= 0 and leave room for the rings");
  if (d->policy != SSE_GAP_DISCARD && d->policy != SSE_GAP_NEAREST && d->policy != SSE_GAP_EDGE_LUT)
    return fail(SSE_EINVAL, "unknown gap policy");
  if (c->d_lut && !lut_fits_gaps(c->sc, c->lut))
    return fail(SSE_EINVAL, "the loaded LUT lacks the gap layout on its crystal axes");
  float* fresh[2] = {nullptr, nullptr};
  if (d->policy == SSE_GAP_EDGE_LUT) {
    if (d->edge_n_angle < 1 || d->edge_n_pos < 1 || d->edge_n_angle > 65536 || d->edge_n_pos > 65536)
      return fail(SSE_EINVAL, "edge LUT sizes must lie in [1, 65536]");
    if (!edge_t || !edge_a) return fail(SSE_EINVAL, "the edge-LUT policy needs both edge LUTs");
    const uint64_t n = static_cast<uint64_t>(d->edge_n_angle) * static_cast<uint64_t>(d->edge_n_pos);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const float* src[2] = {edge_t, edge_a};
    for (int k = 0; k < 2; ++k) {
      std::vector<float> h;
      sse_status st = fetch_floats(src[k], n, mem, s, h);
      for (uint64_t i = 0; st == SSE_OK && i < n; ++i)
        if (!(h[i] >= 0.0f && h[i] <= 1.0f)) st = fail(SSE_EINVAL, "edge LUT values must lie in [0, 1]");
      hipError_t e = hipSuccess;
      if (st == SSE_OK) e = hipMalloc(&fresh[k], n * sizeof(float));
      if (st == SSE_OK && e == hipSuccess) e = hipMemcpy(fresh[k], h.data(), n * sizeof(float), hipMemcpyHostToDevice);
      if (st == SSE_OK && e != hipSuccess) st = hip_fail(e, "upload edge LUT");
      if (st != SSE_OK) {
        release(fresh[0]);
        release(fresh[1]);
        return st;
      }
    }
  }
  HIP_TRY(hipDeviceSynchronize(), "wait for pending work");
  for (int k = 0; k < 2; ++k) {
    release(c->d_edge[k]);
    c->d_edge[k] = fresh[k];
  }
  c->gaps = *d;
  c->gaps_on = 1;
  return SSE_OK;
}

sse_status sse_check_division(sse_ctx* c, uint64_t n_random, uint32_t seed, uint64_t* reciprocal_mismatches,
                              uint64_t* quotient_mismatches) {
  if (!c || !reciprocal_mismatches || !quotient_mismatches) return fail(SSE_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(c->device), "set device");
  unsigned long long* d = nullptr;
  HIP_TRY(hipMalloc(&d, 2 * sizeof(unsigned long long)), "allocate counters");
  unsigned long long h[2] = {0, 0};
  hipError_t e = hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sse::launch_check_division(n_random, seed, d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost);
  release(d);
  if (e != hipSuccess) return hip_fail(e, "division check");
  *reciprocal_mismatches = h[0];
  *quotient_mismatches = h[1];
  return SSE_OK;
}

sse_status sse_build_edge_lut(const sse_edge_geom* g, float* out) {
  if (!g || !out) return fail(SSE_EINVAL, "null argument");
  if (g->n_angle < 1 || g->n_pos < 1 || g->n_angle > 65536 || g->n_pos > 65536)
    return fail(SSE_EINVAL, "bin counts must lie in [1, 65536]");
  if (!finite_pos(g->gap_mm) || !finite_pos(g->depth_mm) || !(g->doi_mm >= 0.0f) || !(g->doi_mm <= g->depth_mm) ||
      !finite_pos(g->mu_per_mm))
    return fail(SSE_EINVAL, "gap, depth and attenuation must be positive, 0 <= doi <= depth");
  const double mu = static_cast<double>(g->mu_per_mm), w = static_cast<double>(g->gap_mm);
  for (int a = 0; a < g->n_angle; ++a) {
    const double deg = -90.0 + (static_cast<double>(a) + 0.5) * 180.0 / static_cast<double>(g->n_angle);
    const double theta = deg * (kTwoPiD / 360.0);
    for (int j = 0; j < g->n_pos; ++j) {
      const double x = -0.5 * w + (static_cast<double>(j) + 0.5) * w / static_cast<double>(g->n_pos);
      double lo, hi;
      bool lower_first;
      edge_ray_paths(*g, theta, x, lo, hi, lower_first);
      // absorption in the block met first, then in the other one
      const double a_lo = -std::expm1(-mu * lo), a_hi = -std::expm1(-mu * hi);
      const double p_lo = lower_first ? a_lo : std::exp(-mu * hi) * a_lo;
      const double p_hi = lower_first ? std::exp(-mu * lo) * a_hi : a_hi;
      double v;
      if (p_lo + p_hi > 0.0) v = p_lo / (p_lo + p_hi);
      else v = x < 0.0 ? 1.0 : (x > 0.0 ? 0.0 : 0.5);
      out[a * g->n_pos + j] = static_cast<float>(v);
    }
  }
  return SSE_OK;
}

sse_status sse_simulate(sse_ctx* c, sse_phantom_id id, uint64_t n_histories, uint64_t seed, uint64_t h_offset,
                        const sse_outputs* out, void* stream) {
  if (!c) return fail(SSE_EINVAL, "null context");
  Phantom* ph = get_phantom(c, id);
  if (!ph) return fail(SSE_EINVAL, "unknown phantom id");
  if (!c->d_lut) return fail(SSE_ESTATE, "no LUT loaded");
  if (c->gaps_on && !lut_fits_gaps(c->sc, c->lut)) return fail(SSE_ESTATE, "the loaded LUT lacks the gap layout");
  if (!out || !out->scatter_counts || !out->scatter_weights) return fail(SSE_EINVAL, "scatter outputs are required");
  if (reinterpret_cast<uintptr_t>(out->scatter_counts) % 4 || reinterpret_cast<uintptr_t>(out->scatter_weights) % 8 ||
      reinterpret_cast<uintptr_t>(out->true_counts) % 4 || reinterpret_cast<uintptr_t>(out->true_weights) % 8 ||
      reinterpret_cast<uintptr_t>(out->stats) % 8 || reinterpret_cast<uintptr_t>(out->records) % 4)
    return fail(SSE_EINVAL, "misaligned output buffer");
  if (out->records && out->record_stride == 0) return fail(SSE_EINVAL, "record_stride must be >= 1");
  if (n_histories > ~static_cast<uint64_t>(0) - h_offset) return fail(SSE_EINVAL, "history range overflows");
  if (n_histories == 0) return SSE_OK;
  HIP_TRY(hipSetDevice(c->device), "set device");
  sse::TransportParams p;
  build_transport_params(c, ph, seed, h_offset, n_histories, p);
  p.sc_n = out->scatter_counts;
  p.sc_w = out->scatter_weights;
  p.tr_n = out->true_counts;
  p.tr_w = out->true_weights;
  p.stats = out->stats;
  p.rec = reinterpret_cast<uint32_t*>(out->records);
  p.rec_stride = out->record_stride;
  sse_status st = ensure_pairs(c, n_histories);
  if (st != SSE_OK) return st;
  p.pairs = c->d_pairs;
  p.pair_count = c->d_pair_count;
  p.pair_cap = c->pair_cap;
  p.item = 0;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipStreamWaitEvent(s, c->pair_done, 0), "order the pair buffer");
  if (p.stats || p.rec)
    HIP_TRY(sse::launch_transport(p, s), "transport kernel launch");
  else
    HIP_TRY(sse::launch_transport_item(p, c->d_item, c->d_chunk, c->d_cursor, s,
                                       c->timing.ev ? &c->timing : nullptr),
            "transport kernel launch");
  HIP_TRY(hipEventRecord(c->pair_done, s), "record pair-buffer use");
  return SSE_OK;
}

sse_status sse_simulate_noalloc(sse_ctx* c, sse_phantom_id id, uint64_t n_histories, uint64_t seed,
                                uint64_t h_offset, const sse_outputs* out, void* stream) {
  if (!c) return fail(SSE_EINVAL, "null context");
  Phantom* ph = get_phantom(c, id);
  if (!ph) return fail(SSE_EINVAL, "unknown phantom id");
  if (!c->d_lut) return fail(SSE_ESTATE, "no LUT loaded");
  if (c->gaps_on && !lut_fits_gaps(c->sc, c->lut)) return fail(SSE_ESTATE, "the loaded LUT lacks the gap layout");
  if (!out || !out->scatter_counts || !out->scatter_weights) return fail(SSE_EINVAL, "scatter outputs are required");
  if (out->stats || out->records)
    return fail(SSE_EINVAL, "statistics and records need sse_simulate (the allocation-free call has neither)");
  if (reinterpret_cast<uintptr_t>(out->scatter_counts) % 4 || reinterpret_cast<uintptr_t>(out->scatter_weights) % 8 ||
      reinterpret_cast<uintptr_t>(out->true_counts) % 4 || reinterpret_cast<uintptr_t>(out->true_weights) % 8)
    return fail(SSE_EINVAL, "misaligned output buffer");
  if (n_histories > ~static_cast<uint64_t>(0) - h_offset) return fail(SSE_EINVAL, "history range overflows");
  if (n_histories == 0) return SSE_OK;
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (sse::noalloc_max_histories() == 0)
    return fail(SSE_EINVAL, "the device's resident transport grid needs more pair records than the " +
                                std::to_string(sse::kNoAllocScratchBytes >> 20) + " MiB allocation-free scratch holds");
  sse::TransportParams p;
  build_transport_params(c, ph, seed, h_offset, n_histories, p);
  p.sc_n = out->scatter_counts;
  p.sc_w = out->scatter_weights;
  p.tr_n = out->true_counts;
  p.tr_w = out->true_weights;
  p.item = 0;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // ordered after the context's earlier simulations, like sse_simulate (the
  // chain lets sse_update_activity wait for all of them)
  HIP_TRY(hipStreamWaitEvent(s, c->pair_done, 0), "order after earlier simulations");
  HIP_TRY(sse::launch_transport_noalloc(c->device, p, s), "transport kernel launch");
  HIP_TRY(hipEventRecord(c->pair_done, s), "record the simulation");
  return SSE_OK;
}

sse_status sse_set_kernel_timing(sse_ctx* c, int enable, uint32_t max_launches) {
  if (!c) return fail(SSE_EINVAL, "null context");
  if (enable != 0 && enable != 1) return fail(SSE_EINVAL, "enable must be 0 or 1");
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (c->pair_done) HIP_TRY(hipEventSynchronize(c->pair_done), "wait for timed launches");
  for (hipEvent_t e : c->timing_ev) (void)hipEventDestroy(e);
  c->timing_ev.clear();
  c->timing = sse::KernelTiming{};
  if (!enable) return SSE_OK;
  if (max_launches == 0 || max_launches > (1u << 20)) return fail(SSE_EINVAL, "max_launches must be 1 .. 2^20");
  c->timing_ev.resize(4ull * max_launches, nullptr);
  for (auto& e : c->timing_ev) {
    const hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      for (hipEvent_t x : c->timing_ev)
        if (x) (void)hipEventDestroy(x);
      c->timing_ev.clear();
      return hip_fail(err, "create timing events");
    }
  }
  c->timing.ev = c->timing_ev.data();
  c->timing.cap = max_launches;
  return SSE_OK;
}

sse_status sse_read_kernel_timing(sse_ctx* c, sse_kernel_timing* out) {
  if (!c || !out) return fail(SSE_EINVAL, "null argument");
  if (!c->timing.ev) return fail(SSE_ESTATE, "kernel timing is off");
  HIP_TRY(hipSetDevice(c->device), "set device");
  *out = sse_kernel_timing{};
  for (uint32_t i = 0; i < c->timing.n; ++i) {
    hipEvent_t* e = c->timing.ev + 4ull * i;
    HIP_TRY(hipEventSynchronize(e[3]), "wait for a timed launch");
    float t = 0.0f, q = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, e[0], e[1]), "transport kernel time");
    HIP_TRY(hipEventElapsedTime(&q, e[2], e[3]), "coincidence kernel time");
    out->transport_ms += t;
    out->coincidence_ms += q;
  }
  out->launches = c->timing.n;
  out->dropped = c->timing.dropped;
  c->timing.n = 0;
  c->timing.dropped = 0;
  return SSE_OK;
}

sse_status sse_emission_scale(sse_ctx* c, sse_phantom_id id, uint64_t n_histories, double acq_seconds, double factor,
                              double* scale) {
  Phantom* p = get_phantom(c, id);
  if (!p) return fail(SSE_EINVAL, "unknown phantom id");
  if (!scale || n_histories == 0 || !std::isfinite(acq_seconds) || !std::isfinite(factor))
    return fail(SSE_EINVAL, "bad arguments");
  const double vol_ml = static_cast<double>(p->desc.voxel_mm[0]) * static_cast<double>(p->desc.voxel_mm[1]) *
                        static_cast<double>(p->desc.voxel_mm[2]) * 1e-3;
  *scale = p->activity_sum * vol_ml * acq_seconds / static_cast<double>(n_histories) * factor;
  return SSE_OK;
}

sse_status sse_apply_sensitivity(sse_ctx* c, const double* W, double scale, float* out, void* stream) {
  if (!c || !W || !out) return fail(SSE_EINVAL, "null argument");
  if (!c->d_sens) return fail(SSE_ESTATE, "no sensitivity sinogram loaded");
  if (!std::isfinite(scale)) return fail(SSE_EINVAL, "scale must be finite");
  HIP_TRY(hipSetDevice(c->device), "set device");
  HIP_TRY(sse::launch_apply_sensitivity(post_params(c), W, scale, c->d_sens, c->sens_tof, out,
                                        static_cast<hipStream_t>(stream)),
          "sensitivity kernel");
  return SSE_OK;
}

sse_status sse_total_scatter(sse_ctx* c, const double* W, double scale, double* total, void* stream) {
  if (!c || !W || !total) return fail(SSE_EINVAL, "null argument");
  if (!c->d_sens) return fail(SSE_ESTATE, "no sensitivity sinogram loaded");
  if (!std::isfinite(scale)) return fail(SSE_EINVAL, "scale must be finite");
  if (reinterpret_cast<uintptr_t>(W) % 8 || reinterpret_cast<uintptr_t>(total) % 8)
    return fail(SSE_EINVAL, "misaligned buffer");
  HIP_TRY(hipSetDevice(c->device), "set device");
  if (!c->d_partials)
    HIP_TRY(hipMalloc(&c->d_partials, sse::kTotalPartials * sizeof(double)), "allocate reduction scratch");
  HIP_TRY(sse::launch_total_scatter(post_params(c), W, scale, c->d_sens, c->sens_tof, c->d_partials, total,
                                    static_cast<hipStream_t>(stream)),
          "total-scatter kernels");
  return SSE_OK;
}

sse_status sse_gaussian_smooth(sse_ctx* c, const float* in, float* out, const float sigma_bins[3], float truncate,
                               void* stream) {
  if (!c) return fail(SSE_EINVAL, "null context");
  HIP_TRY(hipSetDevice(c->device), "set device");
  return smooth(c, in, false, 1.0, out, sigma_bins, truncate, nullptr, static_cast<hipStream_t>(stream));
}

sse_status sse_finalize(sse_ctx* c, const double* W, double scale, const float* sigma_bins, float truncate,
                        float* out, void* stream) {
  if (!c || !W || !out) return fail(SSE_EINVAL, "null argument");
  if (!sigma_bins) return sse_apply_sensitivity(c, W, scale, out, stream);
  if (!c->d_sens) return fail(SSE_ESTATE, "no sensitivity sinogram loaded");
  if (!std::isfinite(scale)) return fail(SSE_EINVAL, "scale must be finite");
  HIP_TRY(hipSetDevice(c->device), "set device");
  return smooth(c, W, true, scale, out, sigma_bins, truncate, c->d_sens, static_cast<hipStream_t>(stream));
}

sse_status sse_smoothing_normalisation(sse_ctx* c, const double* W, double scale, const float sigma_bins[3],
                                       float truncate, float* norm_out, void* stream) {
  if (!c || !W || !norm_out || !sigma_bins) return fail(SSE_EINVAL, "null argument");
  if (!std::isfinite(scale)) return fail(SSE_EINVAL, "scale must be finite");
  HIP_TRY(hipSetDevice(c->device), "set device");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // the ratio to the unsmoothed estimate is taken in the last pass
  return smooth(c, W, true, scale, norm_out, sigma_bins, truncate, nullptr, s, nullptr, W);
}

sse_status sse_finalize_normalised(sse_ctx* c, const double* W, double scale, const float* norm,
                                   const float sigma_bins[3], float truncate, float* out, void* stream) {
  if (!c || !W || !norm || !out || !sigma_bins) return fail(SSE_EINVAL, "null argument");
  if (!c->d_sens) return fail(SSE_ESTATE, "no sensitivity sinogram loaded");
  if (!std::isfinite(scale)) return fail(SSE_EINVAL, "scale must be finite");
  if (static_cast<const void*>(out) == static_cast<const void*>(norm)) return fail(SSE_EINVAL, "out overlaps norm");
  HIP_TRY(hipSetDevice(c->device), "set device");
  return smooth(c, W, true, scale, out, sigma_bins, truncate, c->d_sens, static_cast<hipStream_t>(stream), norm);
}

}  // extern "C"
