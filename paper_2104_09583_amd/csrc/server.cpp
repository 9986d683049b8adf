// Request loop for serving encrypted queries against resident models.
//
// Clients submit query groups (already encrypted) from any thread; the
// device work is driven by the threads that wait for results: the first
// waiter that finds no batch running becomes the leader and repeatedly takes
// every queued request of one model (up to max_batch) and evaluates them
// together, until the queue is empty.  Requests submitted while a batch is on
// the GPU join the next batch (continuous batching); other waiters sleep
// until their ticket completes.  The library starts no thread of its own.
// A request is admitted only while the device memory it needs (its
// ciphertexts plus the evaluation working set, estimated from the ring and
// level sizes) fits the budget left after resident models and keys;
// otherwise submit returns COPSE_ENOMEM.  Each group's result is computed by
// the same deterministic schedule whether it runs alone or in a batch, so its
// bits do not depend on the mix.
#include <chrono>
#include <condition_variable>
#include <deque>

#include "compiled.hpp"

using namespace copse;

namespace {
using Clock = std::chrono::steady_clock;
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
}  // namespace

struct copse_server {
  Context* c = nullptr;
  size_t budget = 0;
  size_t resident = 0;
  int max_batch = 1;
  std::vector<std::pair<const Model*, const Keys*>> models;
  std::mutex mu;
  std::condition_variable cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  size_t in_flight = 0;
  uint64_t next_ticket = 1;
  bool leader = false;     // a thread is running batches

  size_t request_bytes(const copse_cts& q) const {
    size_t b = 0;
    for (auto& ct : q.v) b += ct->words() * 8;
    // working set of one group: baby rotations and key-switch buffers, bounded by
    // a fixed number of top-level ciphertexts
    size_t ct_top = 2 * (size_t)(c->L + 1) * c->N * 8;
    return b + 64 * ct_top;
  }

  // Called with mu held by the leader: takes one batch, runs it unlocked, publishes results.
  void run_one_batch(std::unique_lock<std::mutex>& lk) {
    std::vector<Req*> batch;
    int model = queue.front()->model;
    for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < max_batch;) {
      if ((*it)->model == model) {
        batch.push_back(*it);
        it = queue.erase(it);
      } else {
        ++it;
      }
    }
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
    try {
      COPSE_HIP(hipSetDevice(c->device));
      res = evaluate_groups(*c, *models[model].first, *models[model].second, groups);
      COPSE_HIP(hipStreamSynchronize(c->stream));
    } catch (const Error& e) {
      rc = e.code;
      err = e.msg;
    }
    auto now = Clock::now();
    std::vector<std::unique_ptr<copse_cts>> spent;
    lk.lock();
    for (size_t i = 0; i < batch.size(); ++i) {
      Req* r = batch[i];
      r->rc = rc;
      r->err = err;
      if (rc == COPSE_OK) {
        r->result = std::make_unique<copse_cts>();
        r->result->v.push_back(std::move(res[i]));
      }
      spent.push_back(std::move(r->q));
      in_flight -= r->bytes;
      r->t_done = now;
      r->done = true;
    }
    cv_done.notify_all();
  }

  // Lead until the queue is empty (or until `stop_when` holds); mu held on entry and exit.
  template <typename P>
  void lead(std::unique_lock<std::mutex>& lk, P stop_when) {
    leader = true;
    while (!queue.empty() && !stop_when()) run_one_batch(lk);
    leader = false;
    cv_done.notify_all();
  }
};

extern "C" {

int copse_server_create(copse_ctx* ctx, size_t hbm_budget_bytes, int max_batch, copse_server** out) {
  if (!ctx || !out || max_batch < 1) return COPSE_EINVAL;
  auto s = new copse_server();
  s->c = ctx->c.get();
  s->budget = hbm_budget_bytes;
  s->max_batch = max_batch;
  *out = s;
  return COPSE_OK;
}

void copse_server_destroy(copse_server* s) {
  if (!s) return;
  {
    // finish every admitted request before releasing the server
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->queue.empty() || s->leader) {
      if (!s->leader) s->lead(lk, [] { return false; });
      else s->cv_done.wait(lk);
    }
  }
  delete s;
}

int copse_server_add_model(copse_server* s, const copse_model* m, const copse_keys* eval_keys, int* model_id) {
  if (!s || !m || !eval_keys || !model_id) return COPSE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  size_t add = m->m->bytes + eval_keys->k->bytes;
  if (s->resident + add > s->budget) return COPSE_ENOMEM;
  s->resident += add;
  s->models.push_back({m->m.get(), eval_keys->k.get()});
  *model_id = (int)s->models.size() - 1;
  return COPSE_OK;
}

int copse_server_submit(copse_server* s, int model_id, copse_cts* q, uint64_t* ticket) {
  if (!s || !q || !ticket) return COPSE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (model_id < 0 || model_id >= (int)s->models.size()) return COPSE_EINVAL;
  if (q->v.size() != s->models[model_id].first->meta.precision) return COPSE_EINVAL;
  size_t need = s->request_bytes(*q);
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
    if (!s->leader && !s->queue.empty()) {
      // lead until this ticket is done (the batch holding it completes)
      s->lead(lk, [&] { return r->done; });
      continue;
    }
    if (timeout_ms < 0) {
      s->cv_done.wait(lk);
    } else if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->done) {
      return COPSE_ETIMEOUT;
    }
  }
  if (r->rc != COPSE_OK) return r->rc;
  if (!r->result) return COPSE_EINVAL;   // already collected
  *result = r->result.release();
  return COPSE_OK;
}

int copse_server_latency(copse_server* s, uint64_t ticket, double* ms) {
  if (!s || !ms) return COPSE_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || !it->second->done) return COPSE_EINVAL;
  *ms = std::chrono::duration<double, std::milli>(it->second->t_done - it->second->t_submit).count();
  return COPSE_OK;
}

}  // extern "C"
