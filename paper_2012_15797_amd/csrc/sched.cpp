// gfc_sched_*: the serving scheduler's core with the device replaced by
// caller callbacks (include/gfc.h), stepped explicitly by the caller.
#include <memory>
#include <vector>

#include "sched_core.hpp"

namespace gfc {
namespace serve {

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
  size_t release(Batch& b) override {
    if (cb_.release) cb_.release(cb_.user, b.id);
    return 0;
  }

 private:
  gfc_sched_executor cb_;
};

}  // namespace serve
}  // namespace gfc

using namespace gfc;
using namespace gfc::serve;

struct gfc_sched {
  std::unique_ptr<CallbackExecutor> ex;
  std::unique_ptr<Core> core;
};

extern "C" {

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
