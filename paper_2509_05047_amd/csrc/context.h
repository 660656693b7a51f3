// Library-internal state shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "sse.h"

// Host workspace of a phantom's alias-table builds, kept between activity
// updates so that a rebuild touches no fresh pages: the integer masses, the
// two index stacks of the pairing, a host copy of device-resident activity,
// and a pinned staging copy of the packed table for the upload.
struct AliasWork {
  std::vector<uint64_t> mass;
  std::vector<uint32_t> small, large;
  std::vector<float> act;
  uint2* staging = nullptr;
  uint64_t staging_cap = 0;
  float* image = nullptr;  // pinned copy of a reconstructed image (image to activity)
  uint64_t image_cap = 0;
  AliasWork() = default;
  AliasWork(const AliasWork&) = delete;
  AliasWork& operator=(const AliasWork&) = delete;
  ~AliasWork() {
    if (staging) (void)hipHostFree(staging);
    if (image) (void)hipHostFree(image);
  }
};

struct Phantom {
  bool used = false;
  sse_phantom_desc desc{};
  uint64_t nvox = 0;
  float mu_max = 0.0f;
  double activity_sum = 0.0;
  float* d_mu = nullptr;
  uint2* d_alias = nullptr;
  uint8_t* d_mu8 = nullptr;      // palette indices when the map has <= 256 distinct values
  float* d_mu_table = nullptr;   // the 256-entry palette (exact values)
  uint64_t device_bytes = 0;     // of the four device arrays above
  std::shared_ptr<AliasWork> alias_work;
};

struct sse_ctx {
  int device = 0;
  sse_scanner_desc sc{};
  sse_sino_desc sn{};
  sse_physics_desc ph{};
  uint64_t n_bins = 0;
  // phantom slots (id = index + 1); each phantom has a fixed address, and
  // the list is changed and searched under phantoms_mu, since a server's
  // scheduler thread looks phantoms up while the caller may load more;
  // phantom_bytes is the device memory of the loaded ones
  std::vector<std::unique_ptr<Phantom>> phantoms;
  std::mutex phantoms_mu;
  std::atomic<uint64_t> phantom_bytes{0};
  void* d_lut = nullptr;
  int lut_type = -1;
  sse_lut_desc lut{};
  float* d_sens = nullptr;
  // gap model (gaps_on = 0: plain cylinder) and the device copies of the edge LUTs
  int gaps_on = 0;
  sse_gap_desc gaps{};
  float* d_edge[2] = {nullptr, nullptr};
  int sens_tof = 0;
  // photon B is not tracked when photon A ended outside the energy window
  // (the sinograms do not change; calls that collect statistics or records
  // always track both photons)
  int prune_b = 0;
  float* d_scratch[2] = {nullptr, nullptr};
  double* d_partials = nullptr;  // the total-scatter reduction's partial sums
  // reconstruction: LOR and view tables of the projector, OSEM scratch
  void* d_lor = nullptr;
  void* d_view = nullptr;
  void* d_qtab = nullptr;
  void* d_major = nullptr;
  float* d_recon_fp = nullptr;
  uint64_t recon_fp_cap = 0;
  float* d_recon_img[2] = {nullptr, nullptr};
  uint64_t recon_img_cap = 0;
  // pair buffer of the transport -> coincidence hand-over (kPairWords words
  // per pair), its counter, and an event after its last use so that a call
  // on another stream waits for it
  uint32_t* d_pairs = nullptr;
  uint32_t* d_pair_count = nullptr;
  uint64_t pair_cap = 0;
  uint64_t pair_cap_max = 1ull << 27;  // most records the buffer may hold (sse_set_pair_buffer)
  // the production simulate's work-list scratch: one parameter set, one
  // chunk and the claim cursor (ordered like the pair buffer)
  sse::TransportParams* d_item = nullptr;
  sse::WorkChunk* d_chunk = nullptr;
  uint32_t* d_cursor = nullptr;
  hipEvent_t pair_done = nullptr;
  // per-kernel timing of production launches (sse_set_kernel_timing)
  std::vector<hipEvent_t> timing_ev;
  sse::KernelTiming timing{};
  // servers running on this context: their requests hold its device tables,
  // so calls that replace or free them are refused meanwhile
  std::atomic<int> servers{0};
};

namespace sse_detail {

extern thread_local std::string g_error;
sse_status fail(sse_status st, const std::string& msg);
sse_status hip_fail(hipError_t e, const char* what);
void release(void* p);
Phantom* get_phantom(sse_ctx* c, sse_phantom_id id);
// SSE_EBUSY if a server runs on the context.
sse_status refuse_while_serving(const sse_ctx* c, const char* what);
// With gaps on, whether a LUT's crystal axes have the gap layout.
bool lut_fits_gaps(const sse_scanner_desc& sc, const sse_lut_desc& d);
// Kernel parameters of histories [h0, h0 + n) of a phantom (outputs unset).
void build_transport_params(const sse_ctx* c, const Phantom* ph, uint64_t seed, uint64_t h0, uint64_t n,
                            sse::TransportParams& p);

}  // namespace sse_detail

#define HIP_TRY(expr, what)                                       \
  do {                                                            \
    hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return sse_detail::hip_fail(e_, what);  \
  } while (0)
