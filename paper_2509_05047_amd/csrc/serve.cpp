// Request server of libsse.so: a host scheduler thread that admits
// scatter-estimate requests by HBM footprint and, every tick, launches one
// work-list transport kernel over history sub-chunks of all active requests.
// Declarations and documentation: include/sse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "context.h"

using namespace sse_detail;

namespace {

constexpr uint64_t kDefaultTick = 32ull << 20;
// Default sub-chunk size: about this many sub-chunks per tick.  The kernel
// balances a launch by claiming kBatchSlice histories at a time, so
// sub-chunks only split requests to fit launches.
constexpr uint64_t kChunksPerTick = 16;
constexpr int kInFlight = 2;  // ticks queued on the device at once

struct Buffer {
  uint32_t* counts = nullptr;
  double* weights = nullptr;
};

struct Req {
  uint64_t id = 0;
  sse_request r{};
  double t_submit = 0.0, t_admit = 0.0;
  bool owned = false;      // outputs come from the pool
  bool cancelled = false;
  uint64_t next = 0;       // histories handed out so far
  uint64_t inflight = 0;   // ticks in flight holding its chunks
  Buffer out;
};

struct Tick {
  hipEvent_t ev = nullptr;
  std::vector<int> slots;  // slots with chunks in this tick
};

}  // namespace

struct sse_server {
  sse_ctx* ctx = nullptr;
  sse_server_cfg cfg{};
  hipStream_t stream = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::mutex m;
  std::condition_variable wake;   // scheduler: submit, cancel, release, stop
  std::condition_variable done;   // pollers
  std::deque<Req> pending;
  std::vector<Req> slots;
  std::vector<bool> used;
  std::deque<sse_completion> completions;
  std::vector<Buffer> pool;                 // free library-allocated outputs
  std::map<uint64_t, Buffer> held;          // completed, not yet released
  std::set<uint64_t> finished_ids;          // every completed request
  bool alloc_blocked = false;               // an output allocation failed; none until a release
  uint64_t next_id = 1;
  bool stopping = false;
  sse_server_stats st{};
  uint64_t footprint = 0;                   // bytes of one output pair
  uint64_t phantom_bytes0 = 0;              // the context's phantom memory when the budget was taken
  sse::TransportParams* d_items = nullptr;  // one per slot
  sse::TransportParams* h_items = nullptr;  // pinned staging
  sse::WorkChunk* d_chunks[2] = {nullptr, nullptr};
  sse::WorkChunk* h_chunks[2] = {nullptr, nullptr};
  uint32_t max_chunks = 0;
  uint32_t* d_counter = nullptr;
  // pair buffer of the transport -> coincidence hand-over, shared by the
  // ticks (they run in stream order); a tick is launched in segments of at
  // most pair_cap histories
  uint32_t* d_pairs = nullptr;
  uint32_t* d_pair_count = nullptr;
  uint64_t pair_cap = 0;
  uint64_t segment_histories = 0;           // most histories of one segment
  std::deque<Tick> ticks;
  int parity = 0;
  std::thread thread;
  std::string async_error;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void complete(sse_server* s, int slot) {
  Req& q = s->slots[slot];
  sse_completion c{};
  c.id = q.id;
  c.status = q.cancelled ? SSE_REQ_CANCELLED : SSE_REQ_DONE;
  c.t_submit = q.t_submit;
  c.t_admit = q.t_admit;
  c.t_complete = s->now();
  c.histories = q.next;
  c.scatter_counts = q.out.counts;
  c.scatter_weights = q.out.weights;
  if (q.owned) s->held[q.id] = q.out;
  s->finished_ids.insert(q.id);
  s->completions.push_back(c);
  if (q.cancelled) ++s->st.cancelled; else ++s->st.completed;
  s->used[slot] = false;
  s->slots[slot] = Req();
  s->done.notify_all();
}

void complete_finished(sse_server* s) {
  for (size_t i = 0; i < s->slots.size(); ++i) {
    if (!s->used[i]) continue;
    const Req& q = s->slots[i];
    if (q.inflight == 0 && (q.cancelled || q.next >= q.r.n_histories)) complete(s, static_cast<int>(i));
  }
}

void note_error(sse_server* s, hipError_t e, const char* what) {
  if (s->async_error.empty()) s->async_error = std::string(what) + ": " + hipGetErrorString(e);
  s->done.notify_all();
}

// The front request needs library-allocated outputs that neither the pool
// nor a new allocation can give it.  If no buffer can come back either (none
// held by completed requests, none in use by active ones), waiting is futile:
// it completes as failed and true is returned.  Called with the lock held.
bool fail_if_starved(sse_server* s) {
  if (!s->held.empty()) return false;
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (s->used[i] && s->slots[i].owned) return false;
  Req& q = s->pending.front();
  sse_completion c{};
  c.id = q.id;
  c.status = SSE_REQ_FAILED;
  c.t_submit = q.t_submit;
  c.t_admit = c.t_complete = s->now();
  s->completions.push_back(c);
  ++s->st.failed;
  s->finished_ids.insert(q.id);
  s->pending.pop_front();
  s->done.notify_all();
  return true;
}

// Device memory of phantoms loaded since the budget was taken: it counts
// against the budget as the outputs do (phantoms cannot be unloaded while
// the server runs, so it only grows).
uint64_t phantom_growth(const sse_server* s) {
  const uint64_t now = s->ctx->phantom_bytes.load();
  return now > s->phantom_bytes0 ? now - s->phantom_bytes0 : 0;
}

// Admit queued requests first-in first-out while a slot is free and their
// output buffers, with the phantoms loaded since the start, fit the budget.
// Called with the lock held.
void admit(sse_server* s) {
  while (!s->pending.empty()) {
    Req& q = s->pending.front();
    if (q.cancelled) {  // never started: complete without output
      sse_completion c{};
      c.id = q.id;
      c.status = SSE_REQ_CANCELLED;
      c.t_submit = q.t_submit;
      c.t_admit = c.t_complete = s->now();
      s->completions.push_back(c);
      ++s->st.cancelled;
      s->finished_ids.insert(q.id);
      s->pending.pop_front();
      s->done.notify_all();
      continue;
    }
    int slot = -1;
    for (size_t i = 0; i < s->used.size(); ++i)
      if (!s->used[i]) { slot = static_cast<int>(i); break; }
    if (slot < 0) return;
    Buffer b{q.r.scatter_counts, q.r.scatter_weights};
    const bool owned = b.counts == nullptr;
    if (owned) {
      if (!s->pool.empty()) {
        b = s->pool.back();
        s->pool.pop_back();
      } else if (s->st.bytes_allocated + s->footprint + phantom_growth(s) <= s->st.budget_bytes &&
                 !s->alloc_blocked) {
        const uint64_t nb = s->ctx->n_bins;
        hipError_t ea = hipMalloc(&b.counts, nb * sizeof(uint32_t));
        if (ea == hipSuccess) {
          ea = hipMalloc(&b.weights, nb * sizeof(double));
          if (ea != hipSuccess) {
            release(b.counts);
            b.counts = nullptr;
          }
        }
        if (ea != hipSuccess) {
          // The device is fuller than the budget assumed (memory allocated
          // outside the server).  Clear the error so that it does not
          // surface at the next launch, and allocate nothing more until a
          // release; the request waits for buffers to come back, or fails
          // if none can.
          (void)hipGetLastError();
          s->alloc_blocked = true;
          if (!fail_if_starved(s)) return;
          continue;
        }
        s->st.bytes_allocated += s->footprint;
      } else {
        if (!fail_if_starved(s)) return;  // wait for a release
        continue;
      }
    }
    const uint64_t nb = s->ctx->n_bins;
    hipError_t e = hipMemsetAsync(b.counts, 0, nb * sizeof(uint32_t), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.weights, 0, nb * sizeof(double), s->stream);
    Phantom* ph = get_phantom(s->ctx, q.r.phantom);
    sse::TransportParams& p = s->h_items[slot];
    build_transport_params(s->ctx, ph, q.r.seed, q.r.h_offset, q.r.n_histories, p);
    p.sc_n = b.counts;
    p.sc_w = b.weights;
    p.pairs = s->d_pairs;
    p.pair_count = s->d_pair_count;
    p.pair_cap = s->pair_cap;
    p.item = static_cast<uint32_t>(slot);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_items + slot, &p, sizeof(p), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) note_error(s, e, "admit request");
    q.owned = owned;
    q.out = b;
    q.t_admit = s->now();
    s->slots[slot] = q;
    s->used[slot] = true;
    s->pending.pop_front();
  }
}

// Wait for the oldest tick in flight (lock released meanwhile) and complete
// the requests it finished.
void retire_oldest(sse_server* s, std::unique_lock<std::mutex>& lk) {
  Tick t = s->ticks.front();
  s->ticks.pop_front();
  lk.unlock();
  const hipError_t e = hipEventSynchronize(t.ev);
  (void)hipEventDestroy(t.ev);
  lk.lock();
  if (e != hipSuccess) note_error(s, e, "tick");
  for (int slot : t.slots) --s->slots[slot].inflight;
  complete_finished(s);
}

void scheduler(sse_server* s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->m);
  const uint64_t chunk = s->cfg.chunk_histories;
  for (;;) {
    admit(s);
    // requests with work left
    std::vector<int> act;
    const size_t ns = s->slots.size();
    for (size_t i = 0; i < ns; ++i)
      if (s->used[i] && !s->slots[i].cancelled && s->slots[i].next < s->slots[i].r.n_histories)
        act.push_back(static_cast<int>(i));
    if (act.empty()) {
      if (!s->ticks.empty()) {
        retire_oldest(s, lk);
        continue;
      }
      complete_finished(s);
      bool any_active = false;
      for (bool u : s->used) any_active = any_active || u;
      if (s->stopping && s->pending.empty() && !any_active) break;
      s->wake.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    // Shortest remaining work first: the tick goes to the requests closest to
    // completion (small requests finish within one tick), the rest of the
    // tick to the next ones; ties keep admission order.  The request that
    // was submitted first gets the first quarter of every tick, so a large
    // request cannot be starved by a stream of smaller arrivals.
    std::stable_sort(act.begin(), act.end(), [s](int a, int b) {
      return s->slots[a].r.n_histories - s->slots[a].next < s->slots[b].r.n_histories - s->slots[b].next;
    });
    int oldest = act[0];
    for (int slot : act)
      if (s->slots[slot].t_submit < s->slots[oldest].t_submit) oldest = slot;
    sse::WorkChunk* list = s->h_chunks[s->parity];
    uint32_t nc = 0;
    uint64_t room = s->cfg.tick_histories;
    std::vector<int> in_tick;
    auto give = [&](int slot, uint64_t want) {
      Req& q = s->slots[slot];
      uint64_t take = std::min<uint64_t>(want, q.r.n_histories - q.next);
      bool added = false;
      while (take > 0 && nc < s->max_chunks) {
        const uint64_t len = std::min<uint64_t>(take, chunk);
        list[nc].h0 = q.r.h_offset + q.next;
        list[nc].n = static_cast<uint32_t>(len);
        list[nc].item = static_cast<uint32_t>(slot);
        ++nc;
        q.next += len;
        take -= len;
        room -= len;
        s->st.histories += len;
        added = true;
      }
      if (added && std::find(in_tick.begin(), in_tick.end(), slot) == in_tick.end()) {
        ++q.inflight;
        in_tick.push_back(slot);
      }
    };
    give(oldest, room / 4);
    for (int slot : act) {
      if (room == 0 || nc >= s->max_chunks) break;
      give(slot, room);
    }
    s->st.max_active_seen = std::max<uint64_t>(s->st.max_active_seen, in_tick.size());
    ++s->st.ticks;
    Tick t;
    t.slots = in_tick;
    hipError_t e = hipEventCreateWithFlags(&t.ev, hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_chunks[s->parity], list, nc * sizeof(sse::WorkChunk), hipMemcpyHostToDevice, s->stream);
    // segments of whole chunks of at most pair_cap histories
    for (uint32_t c0 = 0; c0 < nc && e == hipSuccess;) {
      uint32_t c1 = c0;
      uint64_t hist = 0, positions = 0;
      while (c1 < nc && hist + list[c1].n <= s->segment_histories) {
        hist += list[c1].n;
        positions += (list[c1].n + sse::kBatchSlice - 1) / sse::kBatchSlice * sse::kBatchSlice;
        ++c1;
      }
      if (c1 == c0) {  // a chunk larger than the buffer: excluded at start-up
        e = hipErrorInvalidValue;
        break;
      }
      sse::BatchParams b{s->d_items, s->d_chunks[s->parity] + c0, c1 - c0, static_cast<uint32_t>(positions),
                         s->d_counter, hist, s->d_pairs, s->d_pair_count, s->pair_cap, s->ctx->gaps_on};
      e = sse::launch_transport_batch(b, s->stream);
      c0 = c1;
    }
    if (e == hipSuccess) e = hipEventRecord(t.ev, s->stream);
    if (e != hipSuccess) note_error(s, e, "tick launch");
    s->ticks.push_back(t);
    s->parity ^= 1;
    while (static_cast<int>(s->ticks.size()) >= kInFlight) retire_oldest(s, lk);
  }
  while (!s->ticks.empty()) retire_oldest(s, lk);
}

void free_server(sse_server* s) {
  for (auto& b : s->pool) { release(b.counts); release(b.weights); }
  for (auto& kv : s->held) { release(kv.second.counts); release(kv.second.weights); }
  release(s->d_items);
  release(s->d_chunks[0]);
  release(s->d_chunks[1]);
  release(s->d_counter);
  release(s->d_pairs);
  release(s->d_pair_count);
  if (s->h_items) (void)hipHostFree(s->h_items);
  if (s->h_chunks[0]) (void)hipHostFree(s->h_chunks[0]);
  if (s->h_chunks[1]) (void)hipHostFree(s->h_chunks[1]);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

sse_status sse_server_start(sse_ctx* c, const sse_server_cfg* cfg, sse_server** out) {
  if (!c || !cfg || !out) return fail(SSE_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->max_active < 1 || cfg->max_active > 256) return fail(SSE_EINVAL, "max_active must be 1..256");
  if (!c->d_lut) return fail(SSE_ESTATE, "no LUT loaded");
  if (c->gaps_on && !lut_fits_gaps(c->sc, c->lut)) return fail(SSE_ESTATE, "the loaded LUT lacks the gap layout");
  HIP_TRY(hipSetDevice(c->device), "set device");
  sse_server* s = new (std::nothrow) sse_server();
  if (!s) return fail(SSE_ENOMEM, "host allocation");
  s->ctx = c;
  s->cfg = *cfg;
  if (!s->cfg.tick_histories) s->cfg.tick_histories = kDefaultTick;
  if (!s->cfg.chunk_histories) {
    uint64_t chunk = s->cfg.tick_histories / kChunksPerTick;
    chunk = std::max<uint64_t>(256, chunk / 64 * 64);
    s->cfg.chunk_histories = chunk;
  }
  if (s->cfg.chunk_histories > (1ull << 31)) {
    delete s;
    return fail(SSE_EINVAL, "chunk_histories too large");
  }
  s->footprint = c->n_bins * (sizeof(uint32_t) + sizeof(double));
  const int na = cfg->max_active;
  s->slots.assign(na, Req());
  s->used.assign(na, false);
  s->max_chunks = static_cast<uint32_t>(s->cfg.tick_histories / s->cfg.chunk_histories + na + 1);
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&s->d_items, na * sizeof(sse::TransportParams));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s->h_items), na * sizeof(sse::TransportParams), hipHostMallocDefault);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipMalloc(&s->d_chunks[i], s->max_chunks * sizeof(sse::WorkChunk));
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&s->h_chunks[i]), s->max_chunks * sizeof(sse::WorkChunk), hipHostMallocDefault);
  }
  if (e == hipSuccess) e = hipMalloc(&s->d_counter, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&s->d_pair_count, sizeof(uint32_t));
  if (e == hipSuccess) {
    // the records a tick needs (one pair per history at most), up to 2^27
    // (10.7 GB; longer ticks run in segments, and each segment ends with a
    // drain), and room for one chunk at least
    uint64_t cap = std::min<uint64_t>(sse::transport_batch_pairs_needed(s->cfg.tick_histories), 1ull << 27);
    cap = std::max<uint64_t>(cap, sse::transport_batch_pairs_needed(s->cfg.chunk_histories));
    s->pair_cap = (cap + 0xffffull) & ~0xffffull;
    s->segment_histories = sse::transport_batch_max_histories(s->pair_cap);
    e = hipMalloc(&s->d_pairs, static_cast<size_t>(sse::kPairWords) * s->pair_cap * sizeof(uint32_t));
  }
  if (e != hipSuccess) {
    free_server(s);
    return hip_fail(e, "server resources");
  }
  // the default budget: what is free once the server's own buffers exist
  s->phantom_bytes0 = c->phantom_bytes.load();
  if (cfg->hbm_budget_bytes) {
    s->st.budget_bytes = cfg->hbm_budget_bytes;
  } else {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      free_server(s);
      return fail(SSE_EDEVICE, "query free memory");
    }
    s->st.budget_bytes = static_cast<uint64_t>(0.9 * static_cast<double>(free_b));
  }
  s->t0 = std::chrono::steady_clock::now();
  try {
    s->thread = std::thread(scheduler, s);
  } catch (...) {
    free_server(s);
    return fail(SSE_ENOMEM, "scheduler thread");
  }
  c->servers.fetch_add(1);
  *out = s;
  return SSE_OK;
}

sse_status sse_server_submit(sse_server* s, const sse_request* req, uint64_t* id) {
  if (!s || !req || !id) return fail(SSE_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->m);
  if (s->stopping) return fail(SSE_ESTATE, "server is stopping");
  if (!get_phantom(s->ctx, req->phantom)) return fail(SSE_EINVAL, "unknown phantom id");
  if (req->n_histories == 0) return fail(SSE_EINVAL, "n_histories must be >= 1");
  if (req->n_histories > ~static_cast<uint64_t>(0) - req->h_offset) return fail(SSE_EINVAL, "history range overflows");
  if ((req->scatter_counts == nullptr) != (req->scatter_weights == nullptr))
    return fail(SSE_EINVAL, "give both output buffers or neither");
  if (reinterpret_cast<uintptr_t>(req->scatter_counts) % 4 || reinterpret_cast<uintptr_t>(req->scatter_weights) % 8)
    return fail(SSE_EINVAL, "misaligned output buffer");
  if (!req->scatter_counts && s->footprint + phantom_growth(s) > s->st.budget_bytes)
    return fail(SSE_EBUSY, "one request's outputs (with the phantoms loaded since the start) exceed the HBM budget");
  Req q;
  q.id = s->next_id++;
  q.r = *req;
  q.t_submit = s->now();
  s->pending.push_back(q);
  ++s->st.submitted;
  *id = q.id;
  s->wake.notify_one();
  return SSE_OK;
}

sse_status sse_server_poll(sse_server* s, sse_completion* out, int32_t max, int32_t* n, int32_t wait_ms) {
  if (!s || !n || (max > 0 && !out)) return fail(SSE_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(s->m);
  if (wait_ms > 0 && s->completions.empty())
    s->done.wait_for(lk, std::chrono::milliseconds(wait_ms),
                     [s] { return !s->completions.empty() || !s->async_error.empty(); });
  int32_t k = 0;
  while (k < max && !s->completions.empty()) {
    out[k++] = s->completions.front();
    s->completions.pop_front();
  }
  *n = k;
  if (!s->async_error.empty()) return fail(SSE_EDEVICE, s->async_error);
  return SSE_OK;
}

sse_status sse_server_cancel(sse_server* s, uint64_t id) {
  if (!s) return fail(SSE_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->m);
  for (auto& q : s->pending)
    if (q.id == id) { q.cancelled = true; s->wake.notify_one(); return SSE_OK; }
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (s->used[i] && s->slots[i].id == id) { s->slots[i].cancelled = true; s->wake.notify_one(); return SSE_OK; }
  return fail(SSE_EINVAL, "no queued or active request with this id");
}

sse_status sse_server_release(sse_server* s, uint64_t id) {
  if (!s) return fail(SSE_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->held.find(id);
  if (it == s->held.end()) {
    // a completed request with caller-owned outputs (or released before):
    // nothing to do; an id never issued, queued or still active: an error
    if (s->finished_ids.count(id)) return SSE_OK;
    return fail(SSE_EINVAL, "no completed request with this id");
  }
  s->pool.push_back(it->second);
  s->held.erase(it);
  s->alloc_blocked = false;
  s->wake.notify_one();
  return SSE_OK;
}

sse_status sse_server_stats_get(sse_server* s, sse_server_stats* out) {
  if (!s || !out) return fail(SSE_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->m);
  *out = s->st;
  return SSE_OK;
}

sse_status sse_server_stop(sse_server* s) {
  if (!s) return SSE_OK;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stopping = true;
    s->wake.notify_one();
  }
  if (s->thread.joinable()) s->thread.join();
  (void)hipStreamSynchronize(s->stream);
  const std::string err = s->async_error;
  sse_ctx* c = s->ctx;
  free_server(s);
  c->servers.fetch_sub(1);
  if (!err.empty()) return fail(SSE_EDEVICE, err);
  return SSE_OK;
}

}  // extern "C"
