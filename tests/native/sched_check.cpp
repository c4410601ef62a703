// CPU check of the serving scheduler (the library's sched_core.hpp, sched.cpp
// and gfc_error.cpp, no HIP), built by tests/test_sanitizers_cpu.py with
// AddressSanitizer + UndefinedBehaviorSanitizer and with ThreadSanitizer:
//   1. the policy through the C ABI (gfc_sched_*) on a simulated clock:
//      strict-FIFO admission, batching by key, the plain mode, rejection,
//      failure isolation, release rules;
//   2. memory the executor still holds after a batch's last release stays
//      charged to the budget until it is reclaimed;
//   3. the threaded loop the device server runs (Loop) with a simulated
//      device: submitter, waiter/releaser and monitor threads at once; every
//      request completes and the charged bytes never exceed the budget.
// Prints "sched_check ok" and exits 0, or names the failed check and exits 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <thread>
#include <vector>

#include "gfc.h"
#include "sched_core.hpp"

#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::fprintf(stderr, "sched_check: %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                    \
    }                                                                  \
  } while (0)

using namespace gfc::serve;

// ------------------------------------------------------------ 1. policy via the C ABI
namespace sim {
double t = 0.0;
std::map<uint64_t, std::pair<double, bool>> batches;  // id -> (finish time, fails)
std::vector<uint64_t> released;
uint64_t fail_ticket = 0;
double now(void*) { return t; }
int launch(void*, uint64_t b, int, int n_req, const uint64_t* tickets, int64_t n) {
  bool fails = false;
  for (int i = 0; i < n_req; ++i) fails = fails || tickets[i] == fail_ticket;
  batches[b] = {t + 1e-3 + 1e-6 * (double)n, fails};
  return 0;
}
int poll(void*, uint64_t b) {
  const auto& e = batches.at(b);
  if (t < e.first) return 0;
  return e.second ? -1 : 1;
}
void release(void*, uint64_t b) { released.push_back(b); }
}  // namespace sim

static int state_of(gfc_sched* s, uint64_t t, uint64_t* batch = nullptr) {
  int st = -1;
  uint64_t b = 0;
  CHECK(gfc_sched_query(s, t, &st, &b) == GFC_OK);
  if (batch) *batch = b;
  return st;
}

static void policy_checks() {
  gfc_sched_executor ex{nullptr, sim::now, sim::launch, sim::poll, sim::release};
  gfc_sched* s = nullptr;
  CHECK(gfc_sched_create(&ex, 100, 1, 1 << 20, &s) == GFC_OK);
  uint64_t t[6];
  // one stream: the first request launches alone, the rest queue and are
  // admitted in order while the budget lasts
  CHECK(gfc_sched_submit(s, 7, 10, 40, &t[0]) == GFC_OK);
  CHECK(gfc_sched_step(s) == GFC_OK);
  CHECK(state_of(s, t[0]) == GFC_REQ_LAUNCHED);
  CHECK(gfc_sched_submit(s, 7, 10, 30, &t[1]) == GFC_OK);
  CHECK(gfc_sched_submit(s, 9, 10, 20, &t[2]) == GFC_OK);   // other key
  CHECK(gfc_sched_submit(s, 7, 10, 20, &t[3]) == GFC_OK);   // does not fit: waits (strict FIFO)
  CHECK(gfc_sched_step(s) == GFC_OK);
  CHECK(state_of(s, t[1]) == GFC_REQ_ADMITTED && state_of(s, t[2]) == GFC_REQ_ADMITTED);
  CHECK(state_of(s, t[3]) == GFC_REQ_PENDING);
  size_t used = 0;
  uint64_t pending = 0;
  CHECK(gfc_sched_usage(s, &used, &pending) == GFC_OK && used == 90 && pending == 1);
  CHECK(gfc_sched_release(s, t[0]) == GFC_EBUSY);           // still in flight
  CHECK(gfc_sched_submit(s, 7, 1, 101, &t[4]) == GFC_EREJECTED);
  sim::t = 1.0;
  CHECK(gfc_sched_step(s) == GFC_OK);                       // t0 done; t1 launches (t2 has another key)
  CHECK(state_of(s, t[0]) == GFC_REQ_DONE);
  uint64_t b1 = 0, b2 = 0;
  CHECK(state_of(s, t[1], &b1) == GFC_REQ_LAUNCHED && state_of(s, t[2]) == GFC_REQ_ADMITTED);
  CHECK(gfc_sched_release(s, t[0]) == GFC_OK);
  CHECK(gfc_sched_step(s) == GFC_OK);                       // t3 admitted now
  sim::t = 2.0;
  CHECK(gfc_sched_step(s) == GFC_OK);
  CHECK(state_of(s, t[1]) == GFC_REQ_DONE);
  CHECK(state_of(s, t[2], &b2) == GFC_REQ_LAUNCHED && b2 != b1);
  CHECK(gfc_sched_release(s, t[1]) == GFC_OK);
  sim::t = 3.0;
  CHECK(gfc_sched_step(s) == GFC_OK);
  sim::t = 4.0;
  CHECK(gfc_sched_step(s) == GFC_OK);
  CHECK(state_of(s, t[2]) == GFC_REQ_DONE && state_of(s, t[3]) == GFC_REQ_DONE);
  CHECK(gfc_sched_release(s, t[2]) == GFC_OK && gfc_sched_release(s, t[3]) == GFC_OK);
  CHECK(gfc_sched_usage(s, &used, &pending) == GFC_OK && used == 0 && pending == 0);
  CHECK(gfc_sched_release(s, t[3]) == GFC_EINVAL);          // unknown now
  // a failing batch fails its own requests only
  CHECK(gfc_sched_submit(s, 3, 5, 10, &t[4]) == GFC_OK);
  sim::fail_ticket = t[4];
  CHECK(gfc_sched_submit(s, 4, 5, 10, &t[5]) == GFC_OK);
  for (int i = 0; i < 4; ++i) {
    sim::t += 1.0;
    CHECK(gfc_sched_step(s) == GFC_OK);
  }
  CHECK(state_of(s, t[4]) == GFC_REQ_FAILED && state_of(s, t[5]) == GFC_REQ_DONE);
  CHECK(gfc_sched_release(s, t[4]) == GFC_OK && gfc_sched_release(s, t[5]) == GFC_OK);
  double p50 = 0, p99 = 0, mx = 0, sps = 0;
  uint64_t nl = 0, nd = 0;
  CHECK(gfc_sched_stats(s, &p50, &p99, &mx, &sps, &nl, &nd) == GFC_OK && nd == 5 && nl == 6);
  CHECK(gfc_sched_destroy(s) == GFC_OK);

  // batching: four admitted requests with one key fuse (max 25 stamps per batch)
  sim::batches.clear();
  sim::t = 0.0;
  CHECK(gfc_sched_create(&ex, 1000, 1, 25, &s) == GFC_OK);
  uint64_t u[5];
  CHECK(gfc_sched_submit(s, 1, 10, 1, &u[0]) == GFC_OK);
  CHECK(gfc_sched_step(s) == GFC_OK);                       // u0 alone on the stream
  for (int i = 1; i < 5; ++i) CHECK(gfc_sched_submit(s, 1, 10, 1, &u[i]) == GFC_OK);
  sim::t = 1.0;
  CHECK(gfc_sched_step(s) == GFC_OK);
  uint64_t bb[5];
  for (int i = 0; i < 5; ++i) state_of(s, u[i], &bb[i]);
  CHECK(bb[1] == bb[2] && bb[3] == 0 && bb[1] != bb[0]);    // 10 + 10 <= 25, a third would not fit
  CHECK(gfc_sched_destroy(s) == GFC_OK);
}

// ------------------------------------------------------------ 2. held memory stays charged
struct HoldingExecutor : Executor {
  double t = 0.0;
  std::map<uint64_t, double> done_at;
  size_t hold = 0, to_reclaim = 0;
  double now() override { return t; }
  int launch(Batch& b) override {
    done_at[b.id] = t + 1.0;
    return 0;
  }
  int poll(Batch& b) override { return t >= done_at[b.id] ? 1 : 0; }
  size_t release(Batch&) override { return hold; }  // a caller's copy still reads it
  size_t reclaimed() override {
    const size_t r = to_reclaim;
    to_reclaim = 0;
    return r;
  }
};

static void held_memory_checks() {
  HoldingExecutor ex;
  Core core(&ex, 100, 1, 1 << 20);
  auto req = [](size_t bytes) {
    auto r = std::make_unique<Req>();
    r->n = 1;
    r->bytes = bytes;
    return r;
  };
  uint64_t a = 0, b = 0;
  CHECK(core.submit(req(80), &a) == GFC_OK);
  core.step();
  ex.t = 2.0;
  core.step();
  ex.hold = 80;                       // the block outlives the release
  CHECK(core.release(a) == GFC_OK);
  CHECK(core.used() == 80);
  CHECK(core.submit(req(60), &b) == GFC_OK);
  core.step();
  CHECK(core.find(b)->state == GFC_REQ_PENDING);   // 80 held + 60 > 100: waits
  ex.to_reclaim = 80;
  core.step();
  CHECK(core.used() == 60 && core.find(b)->state == GFC_REQ_LAUNCHED);
}

// ------------------------------------------------------------ 3. the threaded loop
struct SimDevice : Executor {
  std::mutex mu;  // the loop calls under its own lock; the device's clock is real time
  std::map<uint64_t, std::chrono::steady_clock::time_point> done_at;
  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  }
  int launch(Batch& b) override {
    std::lock_guard<std::mutex> lk(mu);
    done_at[b.id] = std::chrono::steady_clock::now() + std::chrono::microseconds(50 + 2 * b.n);
    return 0;
  }
  int poll(Batch& b) override {
    std::lock_guard<std::mutex> lk(mu);
    return std::chrono::steady_clock::now() >= done_at[b.id] ? 1 : 0;
  }
  size_t release(Batch& b) override {
    std::lock_guard<std::mutex> lk(mu);
    done_at.erase(b.id);
    return 0;
  }
};

static void threaded_checks() {
  SimDevice dev;
  const size_t budget = 4000;
  Loop loop(&dev, budget, 2, 64);
  constexpr int kThreads = 4, kPerThread = 300;
  std::atomic<int> released{0};
  std::atomic<bool> over{false}, stop_monitor{false};
  std::thread monitor([&] {
    while (!stop_monitor.load()) {
      loop.locked([&](Core& c) {
        if (c.used() > c.budget()) over = true;
        return 0;
      });
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
  });
  std::vector<std::thread> workers;
  for (int w = 0; w < kThreads; ++w) {
    workers.emplace_back([&, w] {
      std::mt19937 rng(1234 + w);
      std::vector<uint64_t> mine;
      for (int i = 0; i < kPerThread; ++i) {
        auto r = std::make_unique<Req>();
        r->key.a = rng() % 3;
        r->n = 1 + rng() % 32;
        r->bytes = 10 * (size_t)r->n;
        uint64_t t = 0;
        CHECK(loop.submit(std::move(r), &t) == GFC_OK);
        mine.push_back(t);
        if (mine.size() > 8) {  // keep a few in flight per thread, release the oldest
          CHECK(loop.wait(mine.front(), 10000, nullptr) == GFC_OK);
          int done = 0;
          gfc_status st = GFC_EINVAL;
          CHECK(loop.poll(mine.front(), &done, nullptr, &st) == GFC_OK && done == 1 && st == GFC_OK);
          CHECK(loop.release(mine.front()) == GFC_OK);
          mine.erase(mine.begin());
          released++;
        }
      }
      for (uint64_t t : mine) {
        CHECK(loop.wait(t, 10000, nullptr) == GFC_OK);
        CHECK(loop.release(t) == GFC_OK);
        released++;
      }
    });
  }
  for (auto& th : workers) th.join();
  stop_monitor = true;
  monitor.join();
  CHECK(released.load() == kThreads * kPerThread);
  CHECK(!over.load());
  double p50 = 0, p99 = 0, mx = 0, sps = 0;
  uint64_t nl = 0, nd = 0;
  loop.stats(&p50, &p99, &mx, &sps, &nl, &nd);
  CHECK(nd == (uint64_t)(kThreads * kPerThread) && nl >= 1 && nl <= nd && p99 >= p50);
  loop.shutdown();
}

int main() {
  policy_checks();
  held_memory_checks();
  threaded_checks();
  std::printf("sched_check ok\n");
  return 0;
}
