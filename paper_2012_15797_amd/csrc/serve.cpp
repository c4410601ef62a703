// Serving (gfc_server_*): continuous batching of render requests on the
// device.  The policy is the scheduling core of sched_core.hpp, run by its
// threaded loop; this file supplies the HIP executor (pinned staging, one
// launch per batch on the batch's stream, completion events, batch memory
// from an arena reserved at creation) and the server's PSF tables.
//
// PSFs: the first request naming a PSF at a stamp size enters the PSF's
// cached spectrum for that size (filled then if needed) and its Gaussian in
// the server's device tables, on the submitting thread; each galaxy of a
// batch carries the index of its request's PSF, so requests with different
// PSFs share a launch and the launch thread never fills a cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gfc_internal.hpp"
#include "gfc_launch.hpp"
#include "gfc_trace.hpp"
#include "sched_core.hpp"

namespace gfc {
namespace serve {

// Per-batch state of the HIP executor.
struct HipBatch : BatchState {
  void* mem = nullptr;
  hipEvent_t event = nullptr;
  std::vector<hipEvent_t> reads;         // copies out of `mem` on callers' streams (gfc_server_copy)
  size_t arena_off = 0, arena_size = 0;  // `mem` is arena_size bytes of the arena (0: its own allocation)
  std::chrono::steady_clock::time_point t_launch;
};

static HipBatch& hb(Batch& b) {
  if (!b.state) b.state = std::make_unique<HipBatch>();
  return static_cast<HipBatch&>(*b.state);
}

// ---------------------------------------------------------------- device executor
class HipExecutor : public Executor {
 public:
  HipExecutor(gfc_ctx* ctx, int n_streams, size_t budget) : ctx_(ctx) {
    DeviceGuard g(ctx_->device);
    // Resident PSF tables: per stamp size, kPsfSlots spectrum pointers (main
    // columns, Nyquist column), then kPsfSlots Gaussians [6].
    const size_t ptrs = (size_t)kSizes * 2 * kPsfSlots;
    void* t = nullptr;
    if (hipMalloc(&t, ptrs * sizeof(void*) + (size_t)kPsfSlots * 6 * sizeof(float)) == hipSuccess) {
      tables_ = t;
      auto** base = static_cast<const float2**>(t);
      for (int i = 0; i < kSizes; ++i) {
        d_main_[i] = base + (size_t)(2 * i) * kPsfSlots;
        d_nyq_[i] = base + (size_t)(2 * i + 1) * kPsfSlots;
      }
      d_pg_ = reinterpret_cast<float*>(base + ptrs);
    }
    hipStreamCreateWithFlags(&reg_stream_, hipStreamNonBlocking);
    streams_.resize(std::max(1, n_streams), nullptr);
    events_.resize(streams_.size(), nullptr);
    staging_.resize(streams_.size(), nullptr);
    staging_bytes_.resize(streams_.size(), 0);
    for (auto& s : streams_) hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    // one completion event per stream: a stream holds at most one batch in flight
    for (auto& e : events_) hipEventCreateWithFlags(&e, hipEventDisableTiming);
    // Batch memory comes from one device arena the size of the budget (at
    // most 80% of the free memory): a stream-ordered allocation per batch
    // cost up to several milliseconds of host time each under load.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
      const size_t want = std::min(budget, free_b / 10 * 8) & ~(size_t)(kAlign - 1);
      void* p = nullptr;
      if (want >= ((size_t)1 << 20) && hipMalloc(&p, want) == hipSuccess) {
        arena_ = static_cast<char*>(p);
        arena_bytes_ = want;
        free_[0] = want;
      }
    }
  }
  ~HipExecutor() override {
    DeviceGuard g(ctx_->device);
    for (auto s : streams_) {
      hipStreamSynchronize(s);
      hipStreamDestroy(s);
    }
    for (auto& pd : pending_)
      for (hipEvent_t ev : pd.reads) {
        hipEventSynchronize(ev);
        hipEventDestroy(ev);
      }
    if (arena_) hipFree(arena_);
    if (tables_) hipFree(tables_);
    if (reg_stream_) hipStreamDestroy(reg_stream_);
    for (auto p : staging_)
      if (p) hipHostFree(p);
    for (auto e : events_)
      if (e) hipEventDestroy(e);
  }
  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  }
  // The PSF's slot in the resident tables, entering it (and its spectrum for
  // W) on first use.  Called on submitting threads, never under the server
  // lock: filling a spectrum runs the PSF's DFT and waits for it.
  gfc_status psf_slot(gfc_psf* psf, int W, int* slot_out) {
    if (!tables_) return fail(GFC_ENOMEM, "the server's PSF tables could not be allocated");
    std::lock_guard<std::mutex> lock(reg_mu_);
    DeviceGuard g(ctx_->device);
    int slot;
    const auto it = slot_of_.find(psf->uid);
    if (it == slot_of_.end()) {
      slot = n_slots_.load();
      if (slot >= kPsfSlots) return fail(GFC_EINVAL, "a server holds at most 65536 PSFs");
      float pg[6];
      for (int i = 0; i < 6; ++i) pg[i] = (float)psf->gauss[i];
      hipError_t e = hipMemcpyAsync(d_pg_ + 6 * (size_t)slot, pg, sizeof(pg), hipMemcpyHostToDevice, reg_stream_);
      if (e == hipSuccess) e = hipStreamSynchronize(reg_stream_);
      if (e != hipSuccess) return hip_fail(e, "PSF table entry");
      slot_of_[psf->uid] = slot;
      filled_.push_back(0);
      n_slots_.store(slot + 1);
    } else {
      slot = it->second;
    }
    const int wi = size_index(W);
    if (!((filled_[(size_t)slot] >> wi) & 1u)) {
      const PsfSpectrum* spec = nullptr;
      const gfc_status st = psf_cache(psf, W, reg_stream_, &spec);
      if (st != GFC_OK) return st;
      hipError_t e = hipMemcpyAsync(d_main_[wi] + slot, &spec->main_cols, sizeof(void*), hipMemcpyHostToDevice,
                                    reg_stream_);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d_nyq_[wi] + slot, &spec->nyq_col, sizeof(void*), hipMemcpyHostToDevice, reg_stream_);
      if (e == hipSuccess) e = hipStreamSynchronize(reg_stream_);  // the pointers are pageable stack values
      if (e != hipSuccess) return hip_fail(e, "PSF table entry");
      filled_[(size_t)slot] |= 1u << wi;
    }
    *slot_out = slot;
    return GFC_OK;
  }
  int launch(Batch& b) override {
    TraceScope trace("gfc batch launch");
    DeviceGuard g(ctx_->device);
    Req* r0 = b.reqs.front();
    const int W = r0->W;
    const int64_t n = b.n;
    const size_t out_bytes = (size_t)n * W * W * sizeof(float);
    const size_t par_bytes = (size_t)n * (6 * sizeof(float) + 2 * sizeof(int32_t));  // params, mix_id, psf_id
    hipStream_t s = streams_[b.stream];
    // pinned staging for this stream (its previous batch has completed)
    if (staging_bytes_[b.stream] < par_bytes) {
      if (staging_[b.stream]) hipHostFree(staging_[b.stream]);
      staging_[b.stream] = nullptr;
      staging_bytes_[b.stream] = 0;
      if (hipHostMalloc(&staging_[b.stream], par_bytes * 2, hipHostMallocDefault) != hipSuccess) return -1;
      staging_bytes_[b.stream] = par_bytes * 2;
    }
    float* hp = static_cast<float*>(staging_[b.stream]);
    int32_t* hm = reinterpret_cast<int32_t*>(hp + 6 * n);
    int32_t* hs = hm + n;
    for (Req* r : b.reqs) {
      for (int f = 0; f < 6; ++f)
        std::memcpy(hp + f * n + r->offset, r->params.data() + f * r->n, r->n * sizeof(float));
      if (r->mix_id.empty())
        std::memset(hm + r->offset, 0, r->n * sizeof(int32_t));
      else
        std::memcpy(hm + r->offset, r->mix_id.data(), r->n * sizeof(int32_t));
      std::fill(hs + r->offset, hs + r->offset + r->n, (int32_t)r->psf_slot);
    }
    HipBatch& h = hb(b);
    h.arena_size = 0;
    if (void* m = arena_alloc(out_bytes + par_bytes, &h.arena_off)) {
      h.mem = m;
      h.arena_size = align(out_bytes + par_bytes);
    } else if (hipMallocAsync(&h.mem, out_bytes + par_bytes, s) != hipSuccess) {  // arena full or fragmented
      h.mem = nullptr;
      for (Req* r : b.reqs) r->status = GFC_ENOMEM;
      return -1;
    }
    float* dout = static_cast<float*>(h.mem);
    float* dpar = reinterpret_cast<float*>(static_cast<char*>(h.mem) + out_bytes);
    if (hipMemcpyAsync(dpar, hp, par_bytes, hipMemcpyHostToDevice, s) != hipSuccess) return fail_batch(b);
    gfc_galaxies gal{};
    gal.x = dpar;
    gal.y = dpar + n;
    gal.flux = dpar + 2 * n;
    gal.r_e = dpar + 3 * n;
    gal.e1 = dpar + 4 * n;
    gal.e2 = dpar + 5 * n;
    gal.mix_id = reinterpret_cast<const int32_t*>(dpar + 6 * n);
    gal.cd = nullptr;
    RenderArgs a;
    if (fill_render_args(ctx_, r0->psf, r0->mix, &gal, n, W, r0->flags, &a) != GFC_OK) return fail_batch(b);
    // each galaxy's PSF from the resident tables (its request's slot)
    const int wi = size_index(W);
    a.psf_id = reinterpret_cast<const int32_t*>(dpar + 7 * n);
    a.psf_main_tab = d_main_[wi];
    a.psf_nyq_tab = d_nyq_[wi];
    a.pg_tab = d_pg_;
    a.n_psf = n_slots_.load();
    a.out = dout;
    if (render_launch(a, W, s) != GFC_OK) return fail_batch(b);
    h.event = events_[b.stream];
    if (hipEventRecord(h.event, s) != hipSuccess) return fail_batch(b);
    for (Req* r : b.reqs) r->out_ptr = dout + r->offset * (int64_t)W * W;
    h.t_launch = std::chrono::steady_clock::now();
    if (log_enabled())
      log_event("batch_launch", "\"batch\": " + std::to_string(b.id) + ", \"requests\": " +
                                    std::to_string(b.reqs.size()) + ", \"stamps\": " + std::to_string(n) +
                                    ", \"W\": " + std::to_string(W) + ", \"stream\": " + std::to_string(b.stream));
    return 0;
  }
  int poll(Batch& b) override {
    HipBatch& h = hb(b);
    if (!h.event) return -1;
    const hipError_t e = hipEventQuery(h.event);
    if (e == hipSuccess) {
      trace_mark("gfc batch complete");
      if (log_enabled())
        log_event("batch_complete", "\"batch\": " + std::to_string(b.id) + ", \"ms\": " +
                                        std::to_string(std::chrono::duration<double, std::milli>(
                                                           std::chrono::steady_clock::now() - h.t_launch).count()));
      return 1;
    }
    if (e == hipErrorNotReady) return 0;
    return -1;
  }
  size_t release(Batch& b) override {
    DeviceGuard g(ctx_->device);
    HipBatch& h = hb(b);
    size_t held = 0;
    if (h.arena_size) {
      // The batch has finished, so only callers' copies can still read the
      // block: it is free now, or once those copies have completed (until
      // then the scheduler keeps it charged to the budget).
      if (h.reads.empty()) {
        arena_free(h.arena_off, h.arena_size);
      } else {
        pending_.push_back(Pending{h.arena_off, h.arena_size, std::move(h.reads)});
        held = h.arena_size;
      }
      h.reads.clear();
      h.arena_size = 0;
      h.mem = nullptr;
    }
    // stream-ordered allocation: reused in this stream's order, so first wait
    // for the copies callers made from it on their own streams
    for (hipEvent_t ev : h.reads) {
      hipStreamWaitEvent(streams_[b.stream], ev, 0);
      hipEventDestroy(ev);
    }
    h.reads.clear();
    if (h.mem) hipFreeAsync(h.mem, streams_[b.stream]);
    h.mem = nullptr;
    h.event = nullptr;
    return held;
  }
  size_t reclaimed() override {
    reclaim();
    const size_t r = reclaimed_;
    reclaimed_ = 0;
    return r;
  }
  // Records a caller's copy out of the batch's memory (gfc_server_copy).
  void add_read(Batch& b, hipEvent_t ev) { hb(b).reads.push_back(ev); }

 private:
  int fail_batch(Batch& b) {
    // wait for anything already enqueued on this stream before its memory is reused
    hipStreamSynchronize(streams_[b.stream]);
    return -1;
  }
  gfc_ctx* ctx_;
  // ---- resident PSFs (entries written on submitting threads under reg_mu_;
  // the launch thread reads only n_slots_ and the device tables)
  static constexpr int kPsfSlots = 65536;
  static constexpr int kSizes = 5;  // W = 16, 32, 64, 128, 256
  static int size_index(int W) { return __builtin_ctz((unsigned)W) - 4; }
  void* tables_ = nullptr;
  const float2** d_main_[kSizes] = {};
  const float2** d_nyq_[kSizes] = {};
  float* d_pg_ = nullptr;
  hipStream_t reg_stream_ = nullptr;
  std::mutex reg_mu_;
  std::unordered_map<uint64_t, int> slot_of_;  // PSF uid -> slot
  std::vector<uint8_t> filled_;                // per slot: bit i set once its spectrum for W = 16 << i is entered
  std::atomic<int> n_slots_{0};
  std::vector<hipStream_t> streams_;
  std::vector<hipEvent_t> events_;
  std::vector<void*> staging_;
  std::vector<size_t> staging_bytes_;

  // ---- batch memory arena (guarded by the server lock, like every executor call)
  static constexpr size_t kAlign = 256;
  struct Pending {
    size_t off, size;
    std::vector<hipEvent_t> reads;  // the block is free once these have completed
  };
  static size_t align(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }
  // First fit over the free blocks (offset -> size); nullptr if nothing fits.
  void* arena_alloc(size_t bytes, size_t* off) {
    if (!arena_) return nullptr;
    reclaim();
    bytes = align(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      *off = o;
      return arena_ + o;
    }
    return nullptr;
  }
  // Returns a block, merging it with free neighbours.
  void arena_free(size_t off, size_t bytes) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  // Frees the pending blocks whose callers' copies have completed.
  void reclaim() {
    for (size_t i = 0; i < pending_.size();) {
      bool done = true;
      for (hipEvent_t ev : pending_[i].reads) done = done && hipEventQuery(ev) != hipErrorNotReady;
      if (!done) {
        ++i;
        continue;
      }
      for (hipEvent_t ev : pending_[i].reads) hipEventDestroy(ev);
      arena_free(pending_[i].off, pending_[i].size);
      reclaimed_ += pending_[i].size;
      pending_[i] = std::move(pending_.back());
      pending_.pop_back();
    }
  }
  char* arena_ = nullptr;
  size_t arena_bytes_ = 0;
  std::map<size_t, size_t> free_;
  std::vector<Pending> pending_;
  size_t reclaimed_ = 0;  // bytes of pending blocks freed since the scheduler last asked
};

}  // namespace serve
}  // namespace gfc

using namespace gfc;
using namespace gfc::serve;

struct gfc_server {
  gfc_ctx* ctx = nullptr;
  std::unique_ptr<HipExecutor> ex;
  std::unique_ptr<Loop> loop;
};

extern "C" {

gfc_status gfc_server_create(gfc_ctx* ctx, size_t mem_budget_bytes, int n_streams, int64_t max_batch_stamps,
                             gfc_server** out) {
  if (!ctx || !out) return fail(GFC_EINVAL, "null argument");
  if (n_streams < 1 || n_streams > 8) return fail(GFC_EINVAL, "n_streams must be 1..8");
  if (mem_budget_bytes == 0) return fail(GFC_EINVAL, "zero memory budget");
  auto* s = new (std::nothrow) gfc_server();
  if (!s) return fail(GFC_ENOMEM, "server allocation failed");
  s->ctx = ctx;
  s->ex = std::make_unique<HipExecutor>(ctx, n_streams, mem_budget_bytes);
  s->loop = std::make_unique<Loop>(s->ex.get(), mem_budget_bytes, n_streams, max_batch_stamps);
  ctx->n_objects++;
  *out = s;
  return GFC_OK;
}

gfc_status gfc_server_submit(gfc_server* s, const gfc_request* q, uint64_t* ticket) {
  TraceScope trace("gfc server submit");
  if (!s || !q || !ticket) return fail(GFC_EINVAL, "null argument");
  if (!q->psf || !q->mix || q->psf->ctx != s->ctx || q->mix->ctx != s->ctx)
    return fail(GFC_EINVAL, "request PSF or mixture missing or from another context");
  if (!stamp_size_ok(q->W)) return fail(GFC_EINVAL, "unsupported stamp size");
  if (q->psf->J > 0) return fail(GFC_EUNSUPPORTED, "requests take constant PSFs (no per-galaxy PSF positions)");
  if (q->n < 1) return fail(GFC_EINVAL, "request needs at least one galaxy");
  if ((q->flags & ~15u) || ((q->flags & GFC_FORCE_FOURIER) && (q->flags & GFC_FORCE_REAL)))  // no GFC_ACCUMULATE
    return fail(GFC_EINVAL, "bad flags");
  if (!q->x || !q->y || !q->flux || !q->r_e || !q->e1 || !q->e2) return fail(GFC_EINVAL, "null parameter array");
  auto r = std::make_unique<Req>();
  r->n = q->n;
  r->W = q->W;
  r->psf = q->psf;
  r->mix = q->mix;
  r->flags = q->flags;
  // outputs and parameters (6 floats, mix_id, psf_id per galaxy), rounded up
  // to the arena's 256-byte blocks so that a batch's block never exceeds the
  // sum of its requests' charges
  r->bytes = ((size_t)q->n * ((size_t)q->W * q->W * sizeof(float) + 6 * sizeof(float) + 2 * sizeof(int32_t)) +
              255) & ~(size_t)255;
  // batching key: mixture, stamp size, flags (PSFs mix within a batch)
  r->key.a = reinterpret_cast<uintptr_t>(q->mix);
  r->key.b = (uint64_t)q->W << 32 | q->flags;
  const gfc_status pst = s->ex->psf_slot(q->psf, q->W, &r->psf_slot);
  if (pst != GFC_OK) return pst;
  r->params.resize((size_t)6 * q->n);
  const float* src[6] = {q->x, q->y, q->flux, q->r_e, q->e1, q->e2};
  for (int f = 0; f < 6; ++f) std::memcpy(r->params.data() + (size_t)f * q->n, src[f], q->n * sizeof(float));
  if (q->mix_id) r->mix_id.assign(q->mix_id, q->mix_id + q->n);
  const int slot = r->psf_slot;
  const gfc_status st = s->loop->submit(std::move(r), ticket);
  if (st == GFC_OK && log_enabled())
    log_event("server_submit", "\"ticket\": " + std::to_string(*ticket) + ", \"stamps\": " + std::to_string(q->n) +
                                   ", \"W\": " + std::to_string(q->W) + ", \"psf_slot\": " + std::to_string(slot));
  return st;
}

gfc_status gfc_server_poll(gfc_server* s, uint64_t ticket, int* done, const float** out_dev,
                           gfc_status* status_out) {
  if (!s) return fail(GFC_EINVAL, "null server");
  return s->loop->poll(ticket, done, out_dev, status_out);
}

gfc_status gfc_server_wait(gfc_server* s, uint64_t ticket, int timeout_ms, const float** out_dev) {
  if (!s) return fail(GFC_EINVAL, "null server");
  return s->loop->wait(ticket, timeout_ms, out_dev);
}

gfc_status gfc_server_copy(gfc_server* s, uint64_t ticket, float* dst, void* hip_stream) {
  if (!s || !dst) return fail(GFC_EINVAL, "null argument");
  return s->loop->locked([&](Core& core) -> gfc_status {
    Req* r = core.find(ticket);
    if (!r) return fail(GFC_EINVAL, "unknown ticket");
    if (r->state != GFC_REQ_DONE)
      return fail(r->state == GFC_REQ_FAILED ? r->status : GFC_EBUSY, "request not done");
    DeviceGuard g(s->ctx->device);
    hipError_t e = hipMemcpyAsync(dst, r->out_ptr, (size_t)r->n * r->W * r->W * sizeof(float),
                                  hipMemcpyDeviceToDevice, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "copy of request stamps");
    // the batch's memory is reused only after this copy (see HipExecutor::release)
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
      if (ev) hipEventDestroy(ev);
      hipStreamSynchronize((hipStream_t)hip_stream);  // no event: finish the copy here instead
      return GFC_OK;
    }
    Batch* b = core.batch(r->batch);
    if (b) s->ex->add_read(*b, ev);
    else hipEventDestroy(ev);
    return GFC_OK;
  });
}

gfc_status gfc_server_release(gfc_server* s, uint64_t ticket) {
  if (!s) return fail(GFC_EINVAL, "null server");
  return s->loop->release(ticket);
}

gfc_status gfc_server_stats(gfc_server* s, double* p50_ms, double* p99_ms, double* max_ms, double* stamps_per_s,
                            uint64_t* n_launches, uint64_t* n_done) {
  if (!s) return fail(GFC_EINVAL, "null server");
  s->loop->stats(p50_ms, p99_ms, max_ms, stamps_per_s, n_launches, n_done);
  return GFC_OK;
}

gfc_status gfc_server_replay(gfc_server* s, const gfc_request* reqs, const double* t_arrive, int64_t n,
                             float* const* keep, double* lag, double* span_s) {
  if (!s || n < 0 || (n > 0 && (!reqs || !t_arrive))) return fail(GFC_EINVAL, "null argument or negative count");
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(t_arrive[i]) || t_arrive[i] < 0.0 || (i > 0 && t_arrive[i] < t_arrive[i - 1]))
      return fail(GFC_EINVAL, "arrival times must be finite, non-negative and non-decreasing");
  using clock = std::chrono::steady_clock;
  std::vector<uint64_t> tickets((size_t)n);
  hipStream_t keep_stream = nullptr;  // copies of the kept requests' stamps
  if (keep) {
    DeviceGuard g(s->ctx->device);
    const hipError_t e = hipStreamCreateWithFlags(&keep_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "replay copy stream");
  }
  gfc_status keep_st = GFC_OK;
  std::mutex m;
  std::condition_variable cv;
  int64_t submitted = 0;  // guarded by m
  bool stopped = false;   // guarded by m: no further submissions
  gfc_status wait_st = GFC_OK;
  double t_last = 0.0;
  const clock::time_point t0 = clock::now();
  // Completions in submission order: wait, then release at once.
  std::thread waiter([&] {
    for (int64_t i = 0; i < n; ++i) {
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return submitted > i || stopped; });
        if (submitted <= i) return;
      }
      const gfc_status st = gfc_server_wait(s, tickets[(size_t)i], -1, nullptr);
      if (st != GFC_OK && wait_st == GFC_OK) wait_st = st;
      t_last = std::chrono::duration<double>(clock::now() - t0).count();
      if (st == GFC_OK && keep && keep[i]) {  // ordered before the block's reuse by the server
        const gfc_status cs = gfc_server_copy(s, tickets[(size_t)i], keep[i], keep_stream);
        if (cs != GFC_OK && keep_st == GFC_OK) keep_st = cs;
      }
      gfc_server_release(s, tickets[(size_t)i]);
    }
  });
  gfc_status sub_st = GFC_OK;
  for (int64_t i = 0; i < n; ++i) {
    const clock::time_point target =
        t0 + std::chrono::duration_cast<clock::duration>(std::chrono::duration<double>(t_arrive[i]));
    for (;;) {  // sleep to within 0.3 ms of the arrival, then spin
      const clock::time_point now = clock::now();
      if (now >= target) break;
      if (target - now > std::chrono::microseconds(500))
        std::this_thread::sleep_for(target - now - std::chrono::microseconds(300));
    }
    if (lag) lag[i] = std::chrono::duration<double>(clock::now() - target).count();
    uint64_t tk = 0;
    sub_st = gfc_server_submit(s, &reqs[i], &tk);
    if (sub_st != GFC_OK) break;
    {
      std::lock_guard<std::mutex> lk(m);
      tickets[(size_t)i] = tk;
      submitted = i + 1;
    }
    cv.notify_one();
  }
  {
    std::lock_guard<std::mutex> lk(m);
    stopped = true;
  }
  cv.notify_one();
  waiter.join();
  if (keep_stream) {
    DeviceGuard g(s->ctx->device);
    const hipError_t e = hipStreamSynchronize(keep_stream);
    hipStreamDestroy(keep_stream);
    if (e != hipSuccess && keep_st == GFC_OK) keep_st = hip_fail(e, "replay copies");
  }
  if (span_s) *span_s = t_last;
  if (sub_st != GFC_OK) return fail(sub_st, "a replayed request was not accepted");
  if (wait_st != GFC_OK) return fail(wait_st, "a replayed request failed");
  if (keep_st != GFC_OK) return fail(keep_st, "a kept request's stamps could not be copied");
  return GFC_OK;
}

gfc_status gfc_server_destroy(gfc_server* s) {
  if (!s) return fail(GFC_EINVAL, "null server");
  s->loop->shutdown();  // drains, joins the loop's thread, frees the batches
  s->loop.reset();
  s->ex.reset();
  s->ctx->n_objects--;
  delete s;
  return GFC_OK;
}

}  // extern "C"
