// Captured evaluation: the whole batched schedule of one model over a fixed number of query groups
// recorded once as a HIP graph and replayed per call, so that a single query's hundreds of small
// launches cost one graph launch on the host.
//
// The graph addresses fixed device buffers: its inputs (the query planes), every temporary of the
// schedule and its outputs.  They come from an arena owned by the executor and never shared: a warm-up
// evaluation on the arena leaves every block the schedule needs in its cache, and the capture, which
// asks for the same sizes in the same order, is served from that cache without device allocation.
// The arena never releases cached blocks while the executor lives.  A run copies the caller's planes
// into the input buffers with copy kernels, launches the graph and copies each result into a fresh
// ciphertext; all of it is ordered on the context's stream, so consecutive runs cannot overlap.
// Results are bit-identical to copse_evaluate_batch: the same kernels run with the same arguments.
#include "compiled.hpp"

using namespace copse;

namespace {
// while alive, the context allocates from `arena` and records no profiling events
struct ArenaScope {
  Context& c;
  std::shared_ptr<Pool> saved;
  bool prof;
  ArenaScope(Context& c_, std::shared_ptr<Pool> arena) : c(c_), saved(c_.pool), prof(c_.profiling) {
    c.pool = std::move(arena);
    c.profiling = false;
  }
  ~ArenaScope() {
    c.pool = saved;
    c.profiling = prof;
  }
};

std::vector<std::vector<const Ct*>> plane_ptrs(const std::vector<std::vector<CtPtr>>& in) {
  std::vector<std::vector<const Ct*>> g;
  for (auto& planes : in) {
    g.emplace_back();
    for (auto& p : planes) g.back().push_back(p.get());
  }
  return g;
}
}  // namespace

namespace copse {

std::unique_ptr<copse_exec> exec_create(Context& c, const Model& model, const Keys& keys, int n_groups) {
  if (n_groups <= 0 || n_groups > 4096) fail(COPSE_EINVAL, "group count out of range");
  auto e = std::make_unique<copse_exec>();
  e->c = &c;
  e->model = &model;
  e->keys = &keys;
  e->groups = n_groups;
  e->arena = std::make_shared<Pool>(c.device, true);
  ArenaScope scope(c, e->arena);
  const int p = (int)model.meta.precision;
  // all input planes in one block, so that a run fills them with one gather launch
  const size_t words = (size_t)2 * (c.L + 1) * c.N;
  auto store = std::make_shared<DBuf>(&c, words * n_groups * p);
  COPSE_HIP(hipMemsetAsync(store->get(), 0, words * n_groups * p * sizeof(double), c.stream));
  for (int g = 0; g < n_groups; ++g) {
    e->inputs.emplace_back();
    for (int k = 0; k < p; ++k) {
      auto ct = std::make_unique<Ct>();
      ct->level = c.L;
      ct->npolys = 2;
      ct->n = c.N;
      ct->store = store;
      ct->ptr = store->get() + words * ((size_t)g * p + k);
      e->inputs.back().push_back(std::move(ct));
    }
  }
  e->input_base = store->get();
  const auto planes = plane_ptrs(e->inputs);
  // warm-up: fills the arena's cache and every lookup table the schedule uses
  { auto warm = evaluate_groups(c, model, keys, planes); }
  COPSE_HIP(hipStreamSynchronize(c.stream));
  COPSE_HIP(hipStreamBeginCapture(c.stream, hipStreamCaptureModeRelaxed));
  try {
    e->outputs = evaluate_groups(c, model, keys, planes);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(c.stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  COPSE_HIP(hipStreamEndCapture(c.stream, &e->graph));
  COPSE_HIP(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
  return e;
}

std::vector<CtPtr> exec_run(copse_exec& e, const std::vector<std::vector<const Ct*>>& queries) {
  Context& c = *e.c;
  if (queries.size() != (size_t)e.groups) fail(COPSE_EINVAL, "group count differs from the capture");
  for (size_t g = 0; g < queries.size(); ++g) {
    if (queries[g].size() != e.inputs[g].size()) fail(COPSE_EINVAL, "wrong number of bit planes");
    for (const Ct* q : queries[g])
      if (!q || q->level != c.L || q->npolys != 2 || q->n != c.N)
        fail(COPSE_EINVAL, "query planes must be fresh encryptions at the top level");
  }
  std::vector<const double*> src;
  for (size_t g = 0; g < queries.size(); ++g)
    for (const Ct* q : queries[g]) src.push_back(q->data());
  launch_gather(c, e.input_base, src, 2 * (c.L + 1));
  COPSE_HIP(hipGraphLaunch(e.exec, c.stream));
  // results: one block, filled by one gather launch
  const Ct& o0 = *e.outputs[0];
  const size_t words = o0.words();
  auto store = std::make_shared<DBuf>(&c, words * e.groups);
  std::vector<const double*> res;
  std::vector<CtPtr> out;
  for (int g = 0; g < e.groups; ++g) {
    const Ct& o = *e.outputs[g];
    if (o.level != o0.level || o.npolys != o0.npolys) fail(COPSE_EINVAL, "internal: results differ in shape");
    res.push_back(o.data());
    auto ct = std::make_unique<Ct>();
    ct->level = o.level;
    ct->npolys = o.npolys;
    ct->n = c.N;
    ct->store = store;
    ct->ptr = store->get() + words * g;
    out.push_back(std::move(ct));
  }
  launch_gather(c, store->get(), res, o0.npolys * (o0.level + 1));
  return out;
}

}  // namespace copse

copse_exec::~copse_exec() {
  if (c) (void)hipStreamSynchronize(c->stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  outputs.clear();
  inputs.clear();
}
