// Serving: continuous batching of render requests (gfc_server_*), and the same
// scheduling core driven through caller callbacks (gfc_sched_*).
//
// Policy, identical for both front ends:
//   admission  strict FIFO: the oldest pending request is admitted when its
//              bytes fit in what the budget has left; nothing behind it
//              overtakes it (no starvation of large requests).
//   batching   among admitted requests, the oldest one picks the key
//              (mixture, stamp size, flags), compared as that whole tuple;
//              later admitted requests with the same key join in arrival
//              order up to max_batch_stamps, whatever their PSFs: each galaxy
//              of a batch carries the index of its request's PSF into the
//              server's device tables of resident PSF spectra and Gaussians.
//              max_batch_stamps <= 0 launches every request alone (plain).
//   PSFs       the first request naming a PSF at a stamp size enters the
//              PSF's cached spectrum for that size (filled then if needed)
//              and its Gaussian in those tables, on the submitting thread:
//              the launch thread never fills a cache.
//   streams    at most one batch in flight per stream; requests arriving
//              while every stream is busy are admitted and wait for the next
//              free stream, where they are fused with whatever else arrived.
//   memory     a request is charged its bytes from admission to release.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gfc_internal.hpp"
#include "gfc_launch.hpp"

namespace gfc {
namespace serve {

// Batching key, compared as a whole: (mixture, stamp size << 32 | flags) for
// the server; (caller's key, 0) for the callback scheduler.
struct BatchKey {
  uint64_t a = 0, b = 0;
  bool operator==(const BatchKey& o) const { return a == o.a && b == o.b; }
};

struct Req {
  uint64_t ticket = 0;
  BatchKey key;
  int64_t n = 0;
  size_t bytes = 0;
  int state = GFC_REQ_PENDING;
  gfc_status status = GFC_OK;
  bool charged = false;
  double t_submit = 0.0, t_done = 0.0;
  uint64_t batch = 0;
  int64_t offset = 0;  // first stamp of this request within its batch
  const float* out_ptr = nullptr;  // device stamps once launched
  // payload used by the device executor
  gfc_psf* psf = nullptr;
  int psf_slot = 0;               // index of the PSF in the server's device tables
  const gfc_mix* mix = nullptr;
  int W = 0;
  unsigned flags = 0;
  std::vector<float> params;      // SoA [6][n]
  std::vector<int32_t> mix_id;    // [n] or empty
};

struct Batch {
  uint64_t id = 0;
  BatchKey key;
  int stream = -1;
  std::vector<Req*> reqs;
  int64_t n = 0;
  bool finished = false;
  int live = 0;  // requests not yet released
  // device executor state
  void* mem = nullptr;
  hipEvent_t event = nullptr;
  std::vector<hipEvent_t> reads;  // copies out of `mem` on callers' streams (gfc_server_copy)
  size_t arena_off = 0, arena_size = 0;  // `mem` is arena_size bytes of the server's arena (0: its own allocation)
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual double now() = 0;
  virtual int launch(Batch& b) = 0;     // 0 = ok
  virtual int poll(Batch& b) = 0;       // 1 done, 0 running, <0 failed
  virtual void release(Batch& b) = 0;   // after completion and after every request is released
};

class Core {
 public:
  Core(Executor* ex, size_t budget, int n_streams, int64_t max_batch)
      : ex_(ex), budget_(budget), max_batch_(max_batch), slots_(std::max(1, n_streams), 0) {
    t0_ = ex_->now();
  }

  gfc_status submit(std::unique_ptr<Req> r, uint64_t* ticket) {
    if (r->bytes > budget_) return fail(GFC_EREJECTED, "request exceeds the memory budget");
    r->ticket = next_ticket_++;
    r->t_submit = ex_->now();
    r->state = GFC_REQ_PENDING;
    pending_.push_back(r.get());
    *ticket = r->ticket;
    reqs_[r->ticket] = std::move(r);
    return GFC_OK;
  }

  // One pass: reap finished batches, admit, launch.  Returns true if any
  // request changed state.
  bool step() {
    bool changed = false;
    for (size_t s = 0; s < slots_.size(); ++s) {
      if (!slots_[s]) continue;
      Batch& b = *batches_[slots_[s]];
      const int st = ex_->poll(b);
      if (st == 0) continue;
      const double t = ex_->now();
      for (Req* r : b.reqs) {
        r->t_done = t;
        if (st > 0) {
          r->state = GFC_REQ_DONE;
          latencies_ms_.push_back((t - r->t_submit) * 1e3);
          stamps_done_ += r->n;
          t_last_ = t;
        } else {
          r->state = GFC_REQ_FAILED;
          r->status = GFC_EDEVICE;
        }
      }
      b.finished = true;
      slots_[s] = 0;
      changed = true;
      maybe_free(b);
    }
    while (!pending_.empty()) {
      Req* r = pending_.front();
      if (used_ + r->bytes > budget_) break;
      used_ += r->bytes;
      r->charged = true;
      r->state = GFC_REQ_ADMITTED;
      admitted_.push_back(r);
      pending_.pop_front();
      changed = true;
    }
    for (size_t s = 0; s < slots_.size() && !admitted_.empty(); ++s) {
      if (slots_[s]) continue;
      auto b = std::make_unique<Batch>();
      b->id = next_batch_++;
      b->stream = (int)s;
      b->key = admitted_.front()->key;
      for (auto it = admitted_.begin(); it != admitted_.end();) {
        Req* r = *it;
        const bool first = b->reqs.empty();
        if (!(r->key == b->key)) { ++it; continue; }
        if (!first && (max_batch_ <= 0 || b->n + r->n > max_batch_)) break;
        r->offset = b->n;
        r->batch = b->id;
        r->state = GFC_REQ_LAUNCHED;
        b->n += r->n;
        b->reqs.push_back(r);
        it = admitted_.erase(it);
        if (max_batch_ <= 0) break;
      }
      b->live = (int)b->reqs.size();
      Batch& ref = *b;
      batches_[b->id] = std::move(b);
      ++launches_;
      if (ex_->launch(ref) != 0) {
        for (Req* r : ref.reqs) {
          r->state = GFC_REQ_FAILED;
          if (r->status == GFC_OK) r->status = GFC_EDEVICE;
          r->t_done = ex_->now();
        }
        ref.finished = true;
        maybe_free(ref);
      } else {
        slots_[s] = ref.id;
      }
      changed = true;
    }
    return changed;
  }

  Req* find(uint64_t t) {
    auto it = reqs_.find(t);
    return it == reqs_.end() ? nullptr : it->second.get();
  }
  Batch* batch(uint64_t id) {
    auto it = batches_.find(id);
    return it == batches_.end() ? nullptr : it->second.get();
  }

  gfc_status release(uint64_t t) {
    Req* r = find(t);
    if (!r) return fail(GFC_EINVAL, "unknown ticket");
    if (r->state != GFC_REQ_DONE && r->state != GFC_REQ_FAILED) return fail(GFC_EBUSY, "request still in flight");
    if (r->charged) used_ -= r->bytes;
    if (r->batch) {
      auto it = batches_.find(r->batch);
      if (it != batches_.end()) {
        it->second->live--;
        maybe_free(*it->second);
      }
    }
    reqs_.erase(t);
    return GFC_OK;
  }

  bool busy() const {
    if (!pending_.empty() || !admitted_.empty()) return true;
    for (uint64_t s : slots_)
      if (s) return true;
    return false;
  }
  bool any_in_flight() const {
    for (uint64_t s : slots_)
      if (s) return true;
    return false;
  }

  void stats(double* p50, double* p99, double* mx, double* sps, uint64_t* nl, uint64_t* nd) const {
    std::vector<double> v = latencies_ms_;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {  // nearest rank
      if (v.empty()) return 0.0;
      const double rank = std::ceil(f * (double)v.size());
      const size_t i = rank < 1.0 ? 0 : std::min(v.size() - 1, (size_t)rank - 1);
      return v[i];
    };
    if (p50) *p50 = q(0.5);
    if (p99) *p99 = q(0.99);
    if (mx) *mx = v.empty() ? 0.0 : v.back();
    if (sps) *sps = (t_last_ > t0_) ? (double)stamps_done_ / (t_last_ - t0_) : 0.0;
    if (nl) *nl = launches_;
    if (nd) *nd = v.size();
  }

  // Fails every request that has not been admitted yet (server shutdown).
  void cancel_pending() {
    const double t = ex_->now();
    for (Req* r : pending_) {
      r->state = GFC_REQ_FAILED;
      r->status = GFC_EBUSY;
      r->t_done = t;
    }
    pending_.clear();
  }

  size_t used() const { return used_; }
  uint64_t n_pending() const { return pending_.size(); }
  // Frees every batch (used by the destructors after draining).
  void free_all() {
    for (auto& kv : batches_)
      if (kv.second->finished) ex_->release(*kv.second);
    batches_.clear();
  }

 private:
  void maybe_free(Batch& b) {
    if (b.finished && b.live <= 0) {
      ex_->release(b);
      batches_.erase(b.id);
    }
  }

  Executor* ex_;
  size_t budget_, used_ = 0;
  int64_t max_batch_;
  std::vector<uint64_t> slots_;  // batch id in flight per stream (0 = free)
  std::deque<Req*> pending_, admitted_;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs_;
  std::map<uint64_t, std::unique_ptr<Batch>> batches_;
  uint64_t next_ticket_ = 1, next_batch_ = 1, launches_ = 0;
  std::vector<double> latencies_ms_;
  uint64_t stamps_done_ = 0;
  double t0_ = 0.0, t_last_ = 0.0;
};

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
    b.arena_size = 0;
    if (void* m = arena_alloc(out_bytes + par_bytes, &b.arena_off)) {
      b.mem = m;
      b.arena_size = align(out_bytes + par_bytes);
    } else if (hipMallocAsync(&b.mem, out_bytes + par_bytes, s) != hipSuccess) {  // arena full or fragmented
      b.mem = nullptr;
      for (Req* r : b.reqs) r->status = GFC_ENOMEM;
      return -1;
    }
    float* dout = static_cast<float*>(b.mem);
    float* dpar = reinterpret_cast<float*>(static_cast<char*>(b.mem) + out_bytes);
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
    b.event = events_[b.stream];
    if (hipEventRecord(b.event, s) != hipSuccess) return fail_batch(b);
    for (Req* r : b.reqs) r->out_ptr = dout + r->offset * (int64_t)W * W;
    return 0;
  }
  int poll(Batch& b) override {
    if (!b.event) return -1;
    const hipError_t e = hipEventQuery(b.event);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return -1;
  }
  void release(Batch& b) override {
    DeviceGuard g(ctx_->device);
    if (b.arena_size) {
      // The batch has finished, so only callers' copies can still read the
      // block: it is free now, or once those copies have completed.
      if (b.reads.empty()) arena_free(b.arena_off, b.arena_size);
      else pending_.push_back(Pending{b.arena_off, b.arena_size, std::move(b.reads)});
      b.reads.clear();
      b.arena_size = 0;
      b.mem = nullptr;
    }
    // stream-ordered allocation: reused in this stream's order, so first wait
    // for the copies callers made from it on their own streams
    for (hipEvent_t ev : b.reads) {
      hipStreamWaitEvent(streams_[b.stream], ev, 0);
      hipEventDestroy(ev);
    }
    b.reads.clear();
    if (b.mem) hipFreeAsync(b.mem, streams_[b.stream]);
    b.mem = nullptr;
    b.event = nullptr;
  }
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
      pending_[i] = std::move(pending_.back());
      pending_.pop_back();
    }
  }
  char* arena_ = nullptr;
  size_t arena_bytes_ = 0;
  std::map<size_t, size_t> free_;
  std::vector<Pending> pending_;
};

// ---------------------------------------------------------------- callback executor
class CallbackExecutor : public Executor {
 public:
  explicit CallbackExecutor(const gfc_sched_executor& cb) : cb_(cb) {}
  double now() override { return cb_.now(cb_.user); }
  int launch(Batch& b) override {
    std::vector<uint64_t> t;
    for (Req* r : b.reqs) t.push_back(r->ticket);
    return cb_.launch(cb_.user, b.id, b.stream, (int)t.size(), t.data(), b.n);
  }
  int poll(Batch& b) override { return cb_.poll(cb_.user, b.id); }
  void release(Batch& b) override {
    if (cb_.release) cb_.release(cb_.user, b.id);
  }

 private:
  gfc_sched_executor cb_;
};

}  // namespace serve
}  // namespace gfc

using namespace gfc;
using namespace gfc::serve;

struct gfc_server {
  gfc_ctx* ctx = nullptr;
  std::unique_ptr<HipExecutor> ex;
  std::unique_ptr<Core> core;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
};

struct gfc_sched {
  std::unique_ptr<CallbackExecutor> ex;
  std::unique_ptr<Core> core;
};

static void server_loop(gfc_server* s) {
  std::unique_lock<std::mutex> lock(s->mu);
  while (true) {
    if (s->stop) s->core->cancel_pending();  // never admitted: fail rather than wait for budget
    const bool changed = s->core->step();
    if (changed || s->stop) s->cv_done.notify_all();
    if (s->stop && !s->core->busy()) break;
    if (!s->core->busy()) {
      s->cv_work.wait(lock, [&] { return s->stop || s->core->busy(); });
      continue;
    }
    if (!changed) {
      // launches in flight: poll again shortly without holding the lock
      lock.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lock.lock();
    }
  }
}

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
  s->core = std::make_unique<Core>(s->ex.get(), mem_budget_bytes, n_streams, max_batch_stamps);
  s->worker = std::thread(server_loop, s);
  ctx->n_objects++;
  *out = s;
  return GFC_OK;
}

gfc_status gfc_server_submit(gfc_server* s, const gfc_request* q, uint64_t* ticket) {
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
  std::lock_guard<std::mutex> lock(s->mu);
  gfc_status st = s->core->submit(std::move(r), ticket);
  if (st == GFC_OK) s->cv_work.notify_one();
  return st;
}

gfc_status gfc_server_poll(gfc_server* s, uint64_t ticket, int* done, const float** out_dev,
                           gfc_status* status_out) {
  if (!s) return fail(GFC_EINVAL, "null server");
  std::lock_guard<std::mutex> lock(s->mu);
  Req* r = s->core->find(ticket);
  if (!r) return fail(GFC_EINVAL, "unknown ticket");
  const bool fin = r->state == GFC_REQ_DONE || r->state == GFC_REQ_FAILED;
  if (done) *done = fin ? 1 : 0;
  if (status_out) *status_out = r->status;
  if (out_dev) *out_dev = (r->state == GFC_REQ_DONE) ? r->out_ptr : nullptr;
  return GFC_OK;
}

gfc_status gfc_server_wait(gfc_server* s, uint64_t ticket, int timeout_ms, const float** out_dev) {
  if (!s) return fail(GFC_EINVAL, "null server");
  std::unique_lock<std::mutex> lock(s->mu);
  Req* r = s->core->find(ticket);
  if (!r) return fail(GFC_EINVAL, "unknown ticket");
  auto fin = [&] { return r->state == GFC_REQ_DONE || r->state == GFC_REQ_FAILED; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lock, fin);
  } else if (!s->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), fin)) {
    return fail(GFC_ETIMEOUT, "request not finished within the timeout");
  }
  if (out_dev) *out_dev = (r->state == GFC_REQ_DONE) ? r->out_ptr : nullptr;
  if (r->state == GFC_REQ_FAILED) return fail(r->status, "request failed");
  return GFC_OK;
}

gfc_status gfc_server_copy(gfc_server* s, uint64_t ticket, float* dst, void* hip_stream) {
  if (!s || !dst) return fail(GFC_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(s->mu);
  Req* r = s->core->find(ticket);
  if (!r) return fail(GFC_EINVAL, "unknown ticket");
  if (r->state != GFC_REQ_DONE) return fail(r->state == GFC_REQ_FAILED ? r->status : GFC_EBUSY, "request not done");
  DeviceGuard g(s->ctx->device);
  hipError_t e = hipMemcpyAsync(dst, r->out_ptr, (size_t)r->n * r->W * r->W * sizeof(float),
                                hipMemcpyDeviceToDevice, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "copy of request stamps");
  // the batch's memory is freed only after this copy (see HipExecutor::release)
  hipEvent_t ev = nullptr;
  e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    if (ev) hipEventDestroy(ev);
    hipStreamSynchronize((hipStream_t)hip_stream);  // no event: finish the copy here instead
    return GFC_OK;
  }
  Batch* b = s->core->batch(r->batch);
  if (b) b->reads.push_back(ev);
  else hipEventDestroy(ev);
  return GFC_OK;
}

gfc_status gfc_server_release(gfc_server* s, uint64_t ticket) {
  if (!s) return fail(GFC_EINVAL, "null server");
  std::lock_guard<std::mutex> lock(s->mu);
  gfc_status st = s->core->release(ticket);
  if (st == GFC_OK) s->cv_work.notify_one();  // budget freed: admission may proceed
  return st;
}

gfc_status gfc_server_stats(gfc_server* s, double* p50_ms, double* p99_ms, double* max_ms, double* stamps_per_s,
                            uint64_t* n_launches, uint64_t* n_done) {
  if (!s) return fail(GFC_EINVAL, "null server");
  std::lock_guard<std::mutex> lock(s->mu);
  s->core->stats(p50_ms, p99_ms, max_ms, stamps_per_s, n_launches, n_done);
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
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->worker.join();
  s->core->free_all();
  s->core.reset();
  s->ex.reset();
  s->ctx->n_objects--;
  delete s;
  return GFC_OK;
}

// ---------------------------------------------------------------- callback front end
gfc_status gfc_sched_create(const gfc_sched_executor* ex, size_t mem_budget_bytes, int n_streams,
                            int64_t max_batch_stamps, gfc_sched** out) {
  if (!ex || !out || !ex->now || !ex->launch || !ex->poll) return fail(GFC_EINVAL, "null argument");
  if (n_streams < 1 || n_streams > 64) return fail(GFC_EINVAL, "n_streams must be 1..64");
  auto* s = new (std::nothrow) gfc_sched();
  if (!s) return fail(GFC_ENOMEM, "allocation failed");
  s->ex = std::make_unique<CallbackExecutor>(*ex);
  s->core = std::make_unique<Core>(s->ex.get(), mem_budget_bytes, n_streams, max_batch_stamps);
  *out = s;
  return GFC_OK;
}

gfc_status gfc_sched_submit(gfc_sched* s, uint64_t key, int64_t n_stamps, size_t bytes, uint64_t* ticket) {
  if (!s || !ticket || n_stamps < 1) return fail(GFC_EINVAL, "bad argument");
  auto r = std::make_unique<Req>();
  r->key.a = key;
  r->n = n_stamps;
  r->bytes = bytes;
  return s->core->submit(std::move(r), ticket);
}

gfc_status gfc_sched_step(gfc_sched* s) {
  if (!s) return fail(GFC_EINVAL, "null scheduler");
  s->core->step();
  return GFC_OK;
}

gfc_status gfc_sched_query(gfc_sched* s, uint64_t ticket, int* state, uint64_t* batch) {
  if (!s) return fail(GFC_EINVAL, "null scheduler");
  Req* r = s->core->find(ticket);
  if (!r) return fail(GFC_EINVAL, "unknown ticket");
  if (state) *state = r->state;
  if (batch) *batch = r->batch;
  return GFC_OK;
}

gfc_status gfc_sched_release(gfc_sched* s, uint64_t ticket) {
  if (!s) return fail(GFC_EINVAL, "null scheduler");
  return s->core->release(ticket);
}

gfc_status gfc_sched_usage(gfc_sched* s, size_t* bytes_in_use, uint64_t* n_pending) {
  if (!s) return fail(GFC_EINVAL, "null scheduler");
  if (bytes_in_use) *bytes_in_use = s->core->used();
  if (n_pending) *n_pending = s->core->n_pending();
  return GFC_OK;
}

gfc_status gfc_sched_stats(gfc_sched* s, double* p50_ms, double* p99_ms, double* max_ms, double* stamps_per_s,
                           uint64_t* n_launches, uint64_t* n_done) {
  if (!s) return fail(GFC_EINVAL, "null scheduler");
  s->core->stats(p50_ms, p99_ms, max_ms, stamps_per_s, n_launches, n_done);
  return GFC_OK;
}

gfc_status gfc_sched_destroy(gfc_sched* s) {
  if (!s) return fail(GFC_EINVAL, "null scheduler");
  s->core->free_all();
  delete s;
  return GFC_OK;
}

}  // extern "C"

