// The serving scheduler (no HIP): requests, batches, the policy core and the
// threaded loop that runs it.  The device server (serve.cpp) drives it with
// a HIP executor; gfc_sched_* (sched.cpp) with caller callbacks; the CPU
// sanitizer tests with a simulated device.
//
// Policy:
//   admission  strict FIFO: the oldest pending request is admitted when its
//              bytes fit in what the budget has left; nothing behind it
//              overtakes it (no starvation of large requests).
//   batching   among admitted requests, the oldest one picks the key,
//              compared as a whole; later admitted requests with the same
//              key join in arrival order up to max_batch_stamps.
//              max_batch_stamps <= 0 launches every request alone (plain).
//   streams    at most one batch in flight per stream; requests arriving
//              while every stream is busy are admitted and wait for the next
//              free stream, where they are fused with whatever else arrived.
//   memory     a request is charged its bytes from admission to release; a
//              batch's memory that the executor still holds after its last
//              request is released (callers' copies in flight) stays charged
//              until the executor reports it reclaimed.
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gfc.h"
#include "gfc_error.hpp"

namespace gfc {
namespace serve {

// Batching key, compared as a whole.  The device server uses (mixture,
// stamp size << 32 | flags); the callback scheduler (caller's key, 0).
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
  int64_t offset = 0;              // first stamp of this request within its batch
  const float* out_ptr = nullptr;  // device stamps once launched
  // payload read by the device executor
  gfc_psf* psf = nullptr;
  int psf_slot = 0;                // index of the PSF in the server's device tables
  const gfc_mix* mix = nullptr;
  int W = 0;
  unsigned flags = 0;
  std::vector<float> params;       // SoA [6][n]
  std::vector<int32_t> mix_id;     // [n] or empty
};

// Whatever an executor keeps per batch (device memory, events).
struct BatchState {
  virtual ~BatchState() = default;
};

struct Batch {
  uint64_t id = 0;
  BatchKey key;
  int stream = -1;
  std::vector<Req*> reqs;
  int64_t n = 0;
  bool finished = false;
  int live = 0;  // requests not yet released
  std::unique_ptr<BatchState> state;
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual double now() = 0;
  virtual int launch(Batch& b) = 0;    // 0 = ok
  virtual int poll(Batch& b) = 0;      // 1 done, 0 running, < 0 failed
  // after completion and after every request is released; returns the bytes
  // of the batch's memory it still holds (freed later, see reclaimed())
  virtual size_t release(Batch& b) = 0;
  // bytes of memory held past release() that have been freed since the last call
  virtual size_t reclaimed() { return 0; }
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
    used_ -= std::min(used_, ex_->reclaimed());
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

  // Fails every request that has not been admitted yet (shutdown).
  void cancel_pending() {
    const double t = ex_->now();
    for (Req* r : pending_) {
      r->state = GFC_REQ_FAILED;
      r->status = GFC_EBUSY;
      r->t_done = t;
    }
    pending_.clear();
  }

  // Bytes charged to admitted, unreleased requests and to batch memory the
  // executor still holds.
  size_t used() const { return used_; }
  size_t budget() const { return budget_; }
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
      used_ += ex_->release(b);  // still held (callers' copies in flight): stays charged
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

// The core run by a background thread: submissions, waits and releases come
// from any thread; the loop reaps, admits and launches, polling while
// batches are in flight.  Every call into the core and the executor holds
// one lock.
class Loop {
 public:
  Loop(Executor* ex, size_t budget, int n_streams, int64_t max_batch)
      : core_(ex, budget, n_streams, max_batch) {
    worker_ = std::thread([this] { run(); });
  }
  ~Loop() { shutdown(); }
  Loop(const Loop&) = delete;
  Loop& operator=(const Loop&) = delete;

  gfc_status submit(std::unique_ptr<Req> r, uint64_t* ticket) {
    std::lock_guard<std::mutex> lock(mu_);
    const gfc_status st = core_.submit(std::move(r), ticket);
    if (st == GFC_OK) cv_work_.notify_one();
    return st;
  }

  gfc_status poll(uint64_t ticket, int* done, const float** out_dev, gfc_status* status_out) {
    std::lock_guard<std::mutex> lock(mu_);
    Req* r = core_.find(ticket);
    if (!r) return fail(GFC_EINVAL, "unknown ticket");
    const bool fin = r->state == GFC_REQ_DONE || r->state == GFC_REQ_FAILED;
    if (done) *done = fin ? 1 : 0;
    if (status_out) *status_out = r->status;
    if (out_dev) *out_dev = (r->state == GFC_REQ_DONE) ? r->out_ptr : nullptr;
    return GFC_OK;
  }

  gfc_status wait(uint64_t ticket, int timeout_ms, const float** out_dev) {
    std::unique_lock<std::mutex> lock(mu_);
    Req* r = core_.find(ticket);
    if (!r) return fail(GFC_EINVAL, "unknown ticket");
    auto fin = [&] { return r->state == GFC_REQ_DONE || r->state == GFC_REQ_FAILED; };
    if (timeout_ms < 0) {
      cv_done_.wait(lock, fin);
    } else if (!cv_done_.wait_for(lock, std::chrono::milliseconds(timeout_ms), fin)) {
      return fail(GFC_ETIMEOUT, "request not finished within the timeout");
    }
    if (out_dev) *out_dev = (r->state == GFC_REQ_DONE) ? r->out_ptr : nullptr;
    if (r->state == GFC_REQ_FAILED) return fail(r->status, "request failed");
    return GFC_OK;
  }

  gfc_status release(uint64_t ticket) {
    std::lock_guard<std::mutex> lock(mu_);
    const gfc_status st = core_.release(ticket);
    if (st == GFC_OK) cv_work_.notify_one();  // budget freed: admission may proceed
    return st;
  }

  void stats(double* p50, double* p99, double* mx, double* sps, uint64_t* nl, uint64_t* nd) {
    std::lock_guard<std::mutex> lock(mu_);
    core_.stats(p50, p99, mx, sps, nl, nd);
  }

  // Runs f(core) under the lock (for executor-specific calls on a request).
  template <class F>
  auto locked(F&& f) {
    std::lock_guard<std::mutex> lock(mu_);
    return f(core_);
  }

  // Fails what was never admitted, drains the rest, joins the thread and
  // frees every batch.  Idempotent.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lock(mu_);
      if (joined_) return;
      stop_ = true;
    }
    cv_work_.notify_all();
    worker_.join();
    std::lock_guard<std::mutex> lock(mu_);
    joined_ = true;
    core_.free_all();
  }

 private:
  void run() {
    std::unique_lock<std::mutex> lock(mu_);
    while (true) {
      if (stop_) core_.cancel_pending();  // never admitted: fail rather than wait for budget
      const bool changed = core_.step();
      if (changed || stop_) cv_done_.notify_all();
      if (stop_ && !core_.busy()) break;
      if (!core_.busy()) {
        cv_work_.wait(lock, [&] { return stop_ || core_.busy(); });
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

  Core core_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::thread worker_;
  bool stop_ = false;
  bool joined_ = false;
};

}  // namespace serve
}  // namespace gfc
