// Request loop for serving encrypted queries against resident models.
//
// Clients submit query groups (already encrypted) from any thread; the device work is driven by the
// threads that wait for results (the library starts no thread of its own).  A waiter that finds no
// leader becomes the leader and pumps the loop until its own ticket is done:
//   * a finished batch is retired as soon as its completion event has fired (its tickets complete);
//   * while a lane is free and requests are queued, it takes every queued request of one model (up to
//     max_batch, oldest model first) and enqueues their evaluation on that lane without waiting;
//   * otherwise it waits for the oldest batch on the device.
// Each lane has its own HIP stream (default priority) and its own memory pool, so two batches - of the
// same forest or of different forests - run on the device at once, and the requests that arrive while a
// batch is on the GPU form the next batch, which starts on the other lane right away (continuous
// batching with overlapping device work).  Temporaries of a lane are reused only by that lane's later
// work, in its stream's order.
// A request is admitted only while the device memory it needs fits the budget left after resident
// models and keys: its own ciphertexts plus the working set of one query group of its model, which is
// the peak the lane pools measured on that model's batches so far (before the first one, a bound of 64
// top-level ciphertexts).  Each group's result is computed by the same deterministic schedule whether it
// runs alone, in a batch or beside another batch, so its bits do not depend on the mix.
#include <chrono>
#include <condition_variable>
#include <deque>

#include "compiled.hpp"

using namespace copse;

namespace {
using Clock = std::chrono::steady_clock;
constexpr int kLanes = 2;          // device lanes (HIP streams); the process has 4 hardware queues
constexpr size_t kKeepLatency = 1 << 16;

struct Req {
  uint64_t ticket;
  int model;
  std::unique_ptr<copse_cts> q;
  size_t bytes;
  Clock::time_point t_submit, t_done;
  bool done = false;
  int rc = COPSE_OK;
  std::string err;
  std::unique_ptr<copse_cts> result;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::shared_ptr<Pool> pool;
  std::vector<Req*> batch;      // on the device (empty: free)
  std::vector<CtPtr> results;
  uint64_t seq = 0;             // launch order
};
}  // namespace

struct copse_server {
  Context* c = nullptr;
  size_t budget = 0;
  size_t resident = 0;
  int max_batch = 1;
  struct ModelEntry {
    const Model* m;
    const Keys* k;
    size_t per_group = 0;       // measured working set of one query group (0: not measured yet)
  };
  std::vector<ModelEntry> models;
  std::mutex mu;
  std::condition_variable cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;            // submitted, not yet collected
  std::map<uint64_t, double> latency;                       // collected tickets (the newest kKeepLatency)
  size_t in_flight = 0;
  uint64_t next_ticket = 1, next_seq = 1;
  bool leader = false;          // a thread is pumping the loop
  Lane lanes[kLanes];

  size_t request_bytes(const copse_cts& q, const ModelEntry& e) const {
    size_t b = 0;
    for (auto& ct : q.v) b += ct->words() * 8;
    const size_t fallback = 64 * (2 * (size_t)(c->L + 1) * c->N * 8);
    return b + (e.per_group ? e.per_group : fallback);
  }

  bool busy() const {
    for (const Lane& l : lanes)
      if (!l.batch.empty()) return true;
    return false;
  }

  // mu held: the batch on `l` has finished on the device (or failed to launch); its tickets complete
  void retire(Lane& l, int rc, const std::string& err) {
    const auto now = Clock::now();
    for (size_t i = 0; i < l.batch.size(); ++i) {
      Req* r = l.batch[i];
      r->rc = rc;
      r->err = err;
      if (rc == COPSE_OK) {
        r->result = std::make_unique<copse_cts>();
        r->result->v.push_back(std::move(l.results[i]));
      }
      r->q.reset();               // the device no longer reads the query planes
      in_flight -= r->bytes;
      r->t_done = now;
      r->done = true;
    }
    l.batch.clear();
    l.results.clear();
    cv_done.notify_all();
  }

  // mu held on entry and exit: takes one batch and enqueues it on the free lane `l` (unlocked meanwhile)
  void launch(Lane& l, std::unique_lock<std::mutex>& lk) {
    std::vector<Req*> batch;
    const int model = queue.front()->model;
    for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < max_batch;) {
      if ((*it)->model == model) {
        batch.push_back(*it);
        it = queue.erase(it);
      } else {
        ++it;
      }
    }
    l.batch = batch;
    l.seq = next_seq++;
    const ModelEntry e = models[model];
    lk.unlock();
    std::vector<std::vector<const Ct*>> groups;
    for (Req* r : batch) {
      std::vector<const Ct*> planes;
      for (auto& p : r->q->v) planes.push_back(p.get());
      groups.push_back(planes);
    }
    std::vector<CtPtr> res;
    int rc = COPSE_OK;
    std::string err;
    size_t per_group = 0;
    {
      // the context enqueues on this lane's stream and allocates from its pool while the batch is issued
      const hipStream_t saved_stream = c->stream;
      const std::shared_ptr<Pool> saved_pool = c->pool;
      c->stream = l.stream;
      c->pool = l.pool;
      try {
        COPSE_HIP(hipSetDevice(c->device));
        const size_t base = l.pool->live_bytes();
        l.pool->reset_peak();
        res = evaluate_groups(*c, *e.m, *e.k, groups);
        COPSE_HIP(hipEventRecord(l.done, l.stream));
        per_group = (l.pool->peak_bytes() - base + batch.size() - 1) / batch.size();
      } catch (const Error& ex) {
        rc = ex.code;
        err = ex.msg;
      }
      c->stream = saved_stream;
      c->pool = saved_pool;
    }
    lk.lock();
    models[model].per_group = std::max(models[model].per_group, per_group);
    if (rc != COPSE_OK) {
      // nothing of the failed batch may still be running when its tickets complete
      (void)hipStreamSynchronize(l.stream);
      retire(l, rc, err);
      return;
    }
    l.results = std::move(res);
  }

  // mu held on entry and exit: one turn of the loop (see the file comment)
  void pump(std::unique_lock<std::mutex>& lk) {
    for (Lane& l : lanes)
      if (!l.batch.empty() && hipEventQuery(l.done) == hipSuccess) retire(l, COPSE_OK, "");
    if (!queue.empty()) {
      for (Lane& l : lanes)
        if (l.batch.empty()) {
          launch(l, lk);
          return;
        }
    }
    Lane* oldest = nullptr;
    for (Lane& l : lanes)
      if (!l.batch.empty() && (!oldest || l.seq < oldest->seq)) oldest = &l;
    if (!oldest) return;
    const uint64_t seq = oldest->seq;
    const hipEvent_t ev = oldest->done;
    lk.unlock();
    const hipError_t e = hipEventSynchronize(ev);
    lk.lock();
    // still the same batch (only the leader launches or retires)
    if (!oldest->batch.empty() && oldest->seq == seq)
      retire(*oldest, e == hipSuccess ? COPSE_OK : COPSE_EDEVICE,
             e == hipSuccess ? "" : std::string("batch failed on the device: ") + hipGetErrorString(e));
  }

  // Pump until `stop_when` holds or nothing is queued or on the device; mu held on entry and exit.
  template <typename P>
  void lead(std::unique_lock<std::mutex>& lk, P stop_when) {
    leader = true;
    while (!stop_when() && (!queue.empty() || busy())) pump(lk);
    leader = false;
    cv_done.notify_all();
  }
};

extern "C" {

int copse_server_create(copse_ctx* ctx, size_t hbm_budget_bytes, int max_batch, copse_server** out) {
  if (!ctx || !out || max_batch < 1) return COPSE_EINVAL;
  auto s = std::make_unique<copse_server>();
  s->c = ctx->c.get();
  s->budget = hbm_budget_bytes;
  s->max_batch = max_batch;
  if (hipSetDevice(s->c->device) != hipSuccess) return COPSE_EDEVICE;
  for (Lane& l : s->lanes) {
    if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess)
      return COPSE_EDEVICE;
    l.pool = std::make_shared<Pool>(s->c->device);
  }
  *out = s.release();
  return COPSE_OK;
}

void copse_server_destroy(copse_server* s) {
  if (!s) return;
  {
    // finish every admitted request before releasing the server
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->queue.empty() || s->busy() || s->leader) {
      if (!s->leader) s->lead(lk, [] { return false; });
      else s->cv_done.wait(lk);
    }
  }
  s->reqs.clear();
  for (Lane& l : s->lanes) {
    if (l.stream) (void)hipStreamSynchronize(l.stream);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.stream) (void)hipStreamDestroy(l.stream);
  }
  delete s;
}

int copse_server_add_model(copse_server* s, const copse_model* m, const copse_keys* eval_keys, int* model_id) {
  if (!s || !m || !eval_keys || !model_id) return COPSE_EINVAL;
  if (m->m->primes != s->c->primes || eval_keys->k->primes != s->c->primes) return COPSE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  size_t add = m->m->bytes + eval_keys->k->bytes;
  if (s->resident + add > s->budget) return COPSE_ENOMEM;
  s->resident += add;
  s->models.push_back({m->m.get(), eval_keys->k.get(), 0});
  *model_id = (int)s->models.size() - 1;
  return COPSE_OK;
}

int copse_server_submit(copse_server* s, int model_id, copse_cts* q, uint64_t* ticket) {
  if (!s || !q || !ticket) return COPSE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (model_id < 0 || model_id >= (int)s->models.size()) return COPSE_EINVAL;
  if (q->v.size() != s->models[model_id].m->meta.precision) return COPSE_EINVAL;
  for (auto& ct : q->v)
    if (!ct || ct->n != s->c->N || ct->npolys != 2 || ct->level != s->c->L) return COPSE_EINVAL;
  size_t need = s->request_bytes(*q, s->models[model_id]);
  if (s->resident + s->in_flight + need > s->budget) return COPSE_ENOMEM;
  auto r = std::make_unique<Req>();
  r->ticket = s->next_ticket++;
  r->model = model_id;
  r->q.reset(q);
  r->bytes = need;
  r->t_submit = Clock::now();
  s->in_flight += need;
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  return COPSE_OK;
}

int copse_server_wait(copse_server* s, uint64_t ticket, int timeout_ms, copse_cts** result) {
  if (!s || !result) return COPSE_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return COPSE_EINVAL;
  Req* r = it->second.get();
  auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
  while (!r->done) {
    if (!s->leader && (!s->queue.empty() || s->busy())) {
      // pump until this ticket is done (its batch has finished on the device)
      s->lead(lk, [&] { return r->done; });
      continue;
    }
    if (timeout_ms < 0) {
      s->cv_done.wait(lk);
    } else if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->done) {
      return COPSE_ETIMEOUT;
    }
  }
  const int rc = r->rc;
  if (rc == COPSE_OK) *result = r->result.release();
  // collected: keep only the latency
  s->latency[ticket] = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  while (s->latency.size() > kKeepLatency) s->latency.erase(s->latency.begin());
  s->reqs.erase(it);
  return rc;
}

int copse_server_latency(copse_server* s, uint64_t ticket, double* ms) {
  if (!s || !ms) return COPSE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->latency.find(ticket);
  if (it != s->latency.end()) {
    *ms = it->second;
    return COPSE_OK;
  }
  auto r = s->reqs.find(ticket);
  if (r == s->reqs.end() || !r->second->done) return COPSE_EINVAL;
  *ms = std::chrono::duration<double, std::milli>(r->second->t_done - r->second->t_submit).count();
  return COPSE_OK;
}

}  // extern "C"
