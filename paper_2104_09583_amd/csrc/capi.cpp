// extern "C" boundary of the library (declared in include/copse.h).
#include <algorithm>
#include <chrono>

#include "compiled.hpp"

using namespace copse;

static thread_local std::string g_last_error;


template <typename F>
static int guarded(F f) {
  try {
    f();
    return COPSE_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return COPSE_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return COPSE_EINVAL;
  }
}

#define NEED(x)                                                      \
  do {                                                               \
    if (!(x)) fail(COPSE_EINVAL, "invalid argument: " #x);           \
  } while (0)

// handles made by another context would make the kernels read past their buffers: refuse them
static const Keys& keys_of(const Context& c, const copse_keys* k) {
  if (k->k->primes != c.primes) fail(COPSE_EINVAL, "keys belong to another context");
  return *k->k;
}
static const Ct& ct_of(const Context& c, const copse_cts* x, size_t i) {
  if (!x || i >= x->v.size() || !x->v[i]) fail(COPSE_EINVAL, "invalid argument: ciphertext index");
  const Ct& ct = *x->v[i];
  if (ct.n != c.N || ct.level < 0 || ct.level > c.L || ct.npolys < 2 || ct.npolys > 3)
    fail(COPSE_EINVAL, "ciphertext of another ring or chain");
  return ct;
}

namespace {
std::vector<uint64_t> primes_below(uint64_t bound, uint64_t modulus, int count, const std::vector<uint64_t>& taken) {
  std::vector<uint64_t> out;
  if (bound < 2) fail(COPSE_EINVAL, "prime bound too small");
  uint64_t k = (bound - 2) / modulus;
  while ((int)out.size() < count) {
    if (k == 0) fail(COPSE_EINVAL, "not enough primes = 1 mod 2Nt below the bound");
    uint64_t cand = k * modulus + 1;
    if (cand < bound && std::find(taken.begin(), taken.end(), cand) == taken.end() && is_prime(cand))
      out.push_back(cand);
    --k;
  }
  return out;
}
void check_params(const copse_params* p) {
  if (p->log_n < 4 || p->log_n > 17) fail(COPSE_EINVAL, "log_n must be in [4, 17]");
  const uint64_t N = 1ULL << p->log_n;
  if (p->t < 3 || (p->t - 1) % (2 * N)) fail(COPSE_EINVAL, "t must be 1 mod 2N");
  if (!is_prime(p->t)) fail(COPSE_EINVAL, "t must be prime");
  if (p->alpha == 0 || p->n_data_primes == 0) fail(COPSE_EINVAL, "need at least one data and one special prime");
  if (p->n_data_primes + p->alpha > (uint32_t)kMaxPrimes) fail(COPSE_EINVAL, "too many primes");
  const uint64_t lim = 1ULL << 49;
  if (p->q0_max > lim || p->data_max > lim || p->special_max > lim)
    fail(COPSE_EINVAL, "prime bounds must not exceed 2^49");
}

// q_0, q_1..q_L, p_0..p_{alpha-1} (see copse_params)
std::vector<uint64_t> make_chain(const copse_params& p) {
  check_params(&p);
  const uint64_t modulus = 2 * (1ULL << p.log_n) * p.t;
  std::vector<uint64_t> taken;
  auto special = primes_below(p.special_max, modulus, (int)p.alpha, taken);
  taken.insert(taken.end(), special.begin(), special.end());
  auto mids = primes_below(p.data_max, modulus, (int)p.n_data_primes - 1, taken);
  taken.insert(taken.end(), mids.begin(), mids.end());
  auto q0 = primes_below(p.q0_max, modulus, 1, taken);
  std::vector<uint64_t> out{q0[0]};
  out.insert(out.end(), mids.begin(), mids.end());
  out.insert(out.end(), special.begin(), special.end());
  return out;
}

// slot (r, j) holds m(zeta^e), e = 5^j (r = 0) or -5^j (r = 1) mod 2N; in the bit-reversed
// evaluation order position bitrev((e-1)/2) holds m(zeta^e)
void setup_slots(Context& c) {
  const uint64_t N = c.N;
  c.zeta = powmod(3, (c.t - 1) / (2 * N), c.t);
  if (powmod(c.zeta, N, c.t) != c.t - 1) fail(COPSE_EINVAL, "3 does not give a primitive 2N-th root mod t");
  c.slot_pos.resize(N);
  uint64_t e = 1;
  for (uint64_t j = 0; j < N / 2; ++j) {
    uint64_t e1 = (2 * N - e) % (2 * N);
    c.slot_pos[j] = bitrev((uint32_t)((e - 1) / 2), (int)c.log_n);
    c.slot_pos[N / 2 + j] = bitrev((uint32_t)((e1 - 1) / 2), (int)c.log_n);
    e = (e * 5) % (2 * N);
  }
}
}  // namespace

extern "C" {

const char* copse_last_error(void) { return g_last_error.c_str(); }

int copse_ctx_create(const copse_params* p, copse_ctx** out) {
  return guarded([&] {
    NEED(p && out);
    *out = nullptr;
    check_params(p);
    const uint64_t N = 1ULL << p->log_n;
    auto ctx = std::make_unique<copse_ctx>();
    auto c = std::make_unique<Context>();
    c->device = p->device;
    COPSE_HIP(hipSetDevice(p->device));
    COPSE_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    c->stream = c->own_stream;
    c->log_n = p->log_n;
    c->N = N;
    c->t = p->t;
    c->alpha = (int)p->alpha;
    c->L = (int)p->n_data_primes - 1;
    c->pool = std::make_shared<Pool>(p->device);
    c->primes = make_chain(*p);
    // transform tables
    std::vector<DevPrime> dp;
    for (uint64_t q : c->primes) {
      uint64_t psi = root_of_unity(2 * N, q);
      uint64_t psi_inv = invmod(psi, q);
      c->psi.push_back(psi);
      std::vector<double> fw(N), iv(N);
      for (uint64_t k = 0; k < N; ++k) {
        uint32_t br = bitrev((uint32_t)k, (int)p->log_n);
        fw[k] = (double)powmod(psi, br, q);
        iv[k] = (double)powmod(psi_inv, br, q);
      }
      double *dfw, *div;
      COPSE_HIP(hipMalloc(&dfw, N * 8));
      COPSE_HIP(hipMalloc(&div, N * 8));
      c->tables.push_back(dfw);
      c->tables.push_back(div);
      COPSE_HIP(hipMemcpy(dfw, fw.data(), N * 8, hipMemcpyHostToDevice));
      COPSE_HIP(hipMemcpy(div, iv.data(), N * 8, hipMemcpyHostToDevice));
      DevPrime d;
      d.q = (double)q;
      d.qinv = 1.0 / (double)q;
      d.fwd = dfw;
      d.inv = div;
      d.ninv = (double)invmod(N % q, q);
      dp.push_back(d);
    }
    COPSE_HIP(hipMalloc(&c->d_primes, dp.size() * sizeof(DevPrime)));
    COPSE_HIP(hipMemcpy(c->d_primes, dp.data(), dp.size() * sizeof(DevPrime), hipMemcpyHostToDevice));
    setup_slots(*c);
    // every level's key-switching and modulus-switching tables now, and the scratch array's address on this
    // device: an evaluation without allocation (copse_evaluate_noalloc) then finds everything it reads
    c->build_level_tables();
    scratch_acquire(p->device);
    ctx->c = std::move(c);
    *out = ctx.release();
  });
}

void copse_ctx_destroy(copse_ctx* ctx) {
  if (!ctx) return;
  try { hipStreamSynchronize(ctx->c->stream); } catch (...) {}
  delete ctx;
}

int copse_ctx_primes(const copse_ctx* ctx, uint64_t* out, size_t cap, size_t* n) {
  return guarded([&] {
    NEED(ctx && n);
    *n = ctx->c->primes.size();
    if (out) {
      if (cap < ctx->c->primes.size()) fail(COPSE_EINVAL, "buffer too small");
      std::copy(ctx->c->primes.begin(), ctx->c->primes.end(), out);
    }
  });
}

void* copse_ctx_stream(copse_ctx* ctx) { return ctx ? (void*)ctx->c->stream : nullptr; }

int copse_ctx_set_stream(copse_ctx* ctx, void* stream) {
  return guarded([&] {
    NEED(ctx);
    COPSE_HIP(hipStreamSynchronize(ctx->c->stream));
    ctx->c->stream = stream ? (hipStream_t)stream : ctx->c->own_stream;
  });
}

int copse_ctx_sync(copse_ctx* ctx) {
  return guarded([&] {
    NEED(ctx);
    COPSE_HIP(hipStreamSynchronize(ctx->c->stream));
  });
}

size_t copse_ctx_device_bytes(const copse_ctx* ctx) { return ctx ? ctx->c->pool->held() : 0; }

// ---------------------------------------------------------------- compile
int copse_forest_compile(const char* text, size_t len, uint32_t n_features, uint32_t precision, uint32_t log_n,
                         int fold, uint32_t n1_R, uint32_t n1_L, copse_compiled** out, copse_public_meta* meta) {
  return guarded([&] {
    NEED(text && out);
    *out = nullptr;
    if (log_n < 4 || log_n > 17) fail(COPSE_EINVAL, "log_n must be in [4, 17]");
    auto cc = std::make_unique<copse_compiled>();
    cc->c = compile_forest(text, len, n_features, precision, log_n, fold, n1_R, n1_L);
    if (meta) *meta = cc->c->meta;
    *out = cc.release();
  });
}

int copse_forest_compile_ex(const char* text, size_t len, uint32_t n_features, uint32_t precision, uint32_t log_n,
                            const copse_compile_options* opts, copse_compiled** out, copse_public_meta* meta) {
  return guarded([&] {
    NEED(text && out && opts);
    *out = nullptr;
    if (log_n < 4 || log_n > 17) fail(COPSE_EINVAL, "log_n must be in [4, 17]");
    auto cc = std::make_unique<copse_compiled>();
    cc->c = compile_forest(text, len, n_features, precision, log_n, opts->fold, opts->n1_R, opts->n1_L);
    if (opts->result_privacy) privatize(*cc->c, opts->privacy_seed, opts->n_pad);
    if (opts->server_replication) server_replicate(*cc->c, opts->n1_F);
    if (meta) *meta = cc->c->meta;
    *out = cc.release();
  });
}

int copse_forest_compile_private(const char* text, size_t len, uint32_t n_features, uint32_t precision,
                                 uint32_t log_n, int fold, uint32_t n1_R, uint32_t n1_L, const uint8_t seed[32],
                                 uint32_t n_pad, copse_compiled** out, copse_public_meta* meta) {
  return guarded([&] {
    NEED(text && out && seed);
    *out = nullptr;
    if (log_n < 4 || log_n > 17) fail(COPSE_EINVAL, "log_n must be in [4, 17]");
    auto cc = std::make_unique<copse_compiled>();
    cc->c = compile_forest(text, len, n_features, precision, log_n, fold, n1_R, n1_L);
    privatize(*cc->c, seed, n_pad);
    if (meta) *meta = cc->c->meta;
    *out = cc.release();
  });
}

int copse_compiled_codebook(const copse_compiled* compiled, uint32_t* out, size_t cap, size_t* n) {
  return guarded([&] {
    NEED(compiled && n);
    const auto& book = compiled->c->codebook;
    *n = book.size();
    if (out) {
      if (cap < book.size()) fail(COPSE_EINVAL, "buffer too small");
      for (size_t i = 0; i < book.size(); ++i) out[i] = (uint32_t)book[i];
    }
  });
}

void copse_compiled_destroy(copse_compiled* c) { delete c; }

int copse_compiled_rotations(const copse_public_meta* meta, int32_t* out, size_t cap, size_t* n) {
  return guarded([&] {
    NEED(meta && n);
    auto r = needed_rotations(*meta);
    *n = r.size();
    if (out) {
      if (cap < r.size()) fail(COPSE_EINVAL, "buffer too small");
      std::copy(r.begin(), r.end(), out);
    }
  });
}

// ---------------------------------------------------------------- keys
int copse_keygen(copse_ctx* ctx, const uint8_t seed[32], const int32_t* rots, size_t n_rots, int relin,
                 copse_keys** out) {
  return guarded([&] {
    NEED(ctx && seed && out && (rots || n_rots == 0));
    *out = nullptr;
    std::vector<int32_t> r(rots, rots + n_rots);
    for (int32_t x : r)
      if (x <= 0 || (size_t)x >= ctx->c->N / 2) fail(COPSE_EINVAL, "rotation offsets must be in (0, N/2)");
    auto k = std::make_unique<copse_keys>();
    k->k = keygen(*ctx->c, seed, r, relin != 0);
    *out = k.release();
  });
}

void copse_keys_destroy(copse_keys* k) { delete k; }

int copse_keys_export_eval(copse_ctx* ctx, const copse_keys* k, copse_keys** out) {
  return guarded([&] {
    NEED(ctx && k && out);
    Context& c = *ctx->c;
    auto copy = [&](const DBuf& src) {
      DBuf d(&c, src.size());
      if (src.size())
        COPSE_HIP(hipMemcpyAsync(d.get(), src.get(), src.size() * 8, hipMemcpyDeviceToDevice, c.stream));
      return d;
    };
    if (k->k->primes != c.primes) fail(COPSE_EINVAL, "keys belong to another context");
    auto e = std::make_unique<Keys>();
    e->primes = c.primes;
    e->has_secret = false;
    e->pk_a = copy(k->k->pk_a);
    e->pk_b = copy(k->k->pk_b);
    if (k->k->relin) {
      e->relin = std::make_unique<Keys::KSK>();
      e->relin->a = copy(k->k->relin->a);
      e->relin->b = copy(k->k->relin->b);
    }
    for (auto& kv : k->k->rot) {
      auto r = std::make_unique<Keys::KSK>();
      r->a = copy(kv.second->a);
      r->b = copy(kv.second->b);
      e->rot[kv.first] = std::move(r);
    }
    e->bytes = k->k->bytes;
    COPSE_HIP(hipStreamSynchronize(c.stream));
    auto h = std::make_unique<copse_keys>();
    h->k = std::move(e);
    *out = h.release();
  });
}

size_t copse_keys_bytes(const copse_keys* k) { return k ? k->k->bytes : 0; }

// ---------------------------------------------------------------- model
int copse_model_encode(copse_ctx* ctx, const copse_compiled* c, const copse_keys* keys, int encrypt_model,
                       const uint8_t seed[32], copse_model** out) {
  return guarded([&] {
    NEED(ctx && c && out);
    if (encrypt_model) NEED(keys && seed);
    *out = nullptr;
    uint8_t zero[32] = {0};
    auto m = std::make_unique<copse_model>();
    m->m = build_model(*ctx->c, *c->c, keys ? keys->k.get() : nullptr, encrypt_model != 0, seed ? seed : zero);
    *out = m.release();
  });
}

void copse_model_destroy(copse_model* m) { delete m; }
size_t copse_model_bytes(const copse_model* m) { return m ? m->m->bytes : 0; }

// ---------------------------------------------------------------- queries
int copse_query_encrypt(copse_ctx* ctx, const copse_keys* keys, const copse_public_meta* meta,
                        const uint32_t* features, size_t n_queries, const uint8_t seed[32], uint32_t group,
                        copse_cts** out) {
  return guarded([&] {
    NEED(ctx && keys && meta && features && seed && out);
    *out = nullptr;
    Context& c = *ctx->c;
    if ((1ULL << meta->log_n) != c.N) fail(COPSE_EINVAL, "layout made for another ring size");
    if (n_queries == 0 || n_queries > meta->queries_per_ct) fail(COPSE_EINVAL, "query count must be 1..N/W");
    const uint64_t lim = meta->precision >= 32 ? ~0ULL : (1ULL << meta->precision);
    for (size_t i = 0; i < n_queries * meta->n_features; ++i)
      if (features[i] >= lim) fail(COPSE_EINVAL, "feature value exceeds the precision");
    auto cts = std::make_unique<copse_cts>();
    std::vector<uint64_t> slots;
    for (uint32_t k = 0; k < meta->precision; ++k) {
      query_plane_slots(*meta, c.N, features, n_queries, k, slots);
      std::vector<int64_t> poly;
      encode_slots(c, slots.data(), poly);
      cts->v.push_back(encrypt(c, keys_of(c, keys), poly, c.L, seed, (1ULL << 56) | ((uint64_t)group << 32) | k));
    }
    *out = cts.release();
  });
}

void copse_cts_destroy(copse_cts* c) { delete c; }
size_t copse_cts_count(const copse_cts* c) { return c ? c->v.size() : 0; }
int copse_cts_level(const copse_cts* c, size_t i) { return (c && i < c->v.size()) ? c->v[i]->level : -1; }

// ---------------------------------------------------------------- evaluate
int copse_evaluate(copse_ctx* ctx, const copse_model* model, const copse_keys* keys, const copse_cts* query,
                   copse_cts** result) {
  return guarded([&] {
    NEED(ctx && model && keys && query && result);
    *result = nullptr;
    std::vector<const Ct*> planes;
    for (auto& p : query->v) planes.push_back(p.get());
    auto r = std::make_unique<copse_cts>();
    r->v.push_back(evaluate_group(*ctx->c, *model->m, *keys->k, planes));
    *result = r.release();
  });
}

int copse_ctx_set_tuning(copse_ctx* ctx, const copse_tune_entry* entries, size_t n) {
  return guarded([&] {
    NEED(ctx && (entries || n == 0));
    std::vector<TuneEntry> table;
    for (size_t i = 0; i < n; ++i) {
      const copse_tune_entry& e = entries[i];
      auto in = [](int v, int lo, int hi) { return v == 0 || (v >= lo && v <= hi); };
      if (!in(e.mm_cap, 4, 32) || !(e.mm_waves == 0 || e.mm_waves == 4 || e.mm_waves == 8) || !in(e.ks_jobs, 1, 32) ||
          !in(e.bridge_wgs, 64, 8192) || !(e.gsum_b == 0 || e.gsum_b == 4 || e.gsum_b == 8) || e.batch_lo > e.batch_hi ||
          e.model < -1 || e.model > 1)
        fail(COPSE_EINVAL, "tuning entry " + std::to_string(i) + " out of range");
      table.push_back(TuneEntry{e.log_n, e.top_level, e.batch_lo, e.batch_hi, e.model,
                                Tuning{e.mm_cap, e.mm_waves, e.ks_jobs, e.bridge_wgs, e.gsum_b}});
    }
    ctx->c->tune_table = std::move(table);
  });
}

int copse_evaluate_noalloc(copse_ctx* ctx, const copse_model* model, const copse_keys* keys, const copse_cts* query,
                           copse_cts* result) {
  return guarded([&] {
    NEED(ctx && model && keys && query && result && result->v.size() == 1 && result->v[0]);
    std::vector<const Ct*> planes;
    for (auto& p : query->v) planes.push_back(p.get());
    evaluate_group_noalloc(*ctx->c, *model->m, *keys->k, planes, *result->v[0]);
  });
}

int copse_exec_create(copse_ctx* ctx, const copse_model* model, const copse_keys* eval_keys, size_t n_groups,
                      copse_exec** out) {
  return guarded([&] {
    NEED(ctx && model && eval_keys && out && n_groups > 0);
    *out = nullptr;
    *out = exec_create(*ctx->c, *model->m, *eval_keys->k, (int)std::min<size_t>(n_groups, 1u << 20)).release();
  });
}

int copse_exec_run(copse_exec* exec, const copse_cts* const* queries, size_t n_groups, copse_cts** results) {
  return guarded([&] {
    NEED(exec && queries && results);
    std::vector<std::vector<const Ct*>> groups;
    for (size_t g = 0; g < n_groups; ++g) {
      NEED(queries[g]);
      groups.emplace_back();
      for (auto& p : queries[g]->v) groups.back().push_back(p.get());
    }
    auto r = exec_run(*exec, groups);
    for (size_t g = 0; g < r.size(); ++g) {
      auto c = std::make_unique<copse_cts>();
      c->v.push_back(std::move(r[g]));
      results[g] = c.release();
    }
  });
}

void copse_exec_destroy(copse_exec* exec) { delete exec; }

int copse_evaluate_plain(copse_ctx* ctx, const copse_model* model, const copse_keys* keys, const copse_cts* query,
                         copse_cts** result) {
  return guarded([&] {
    NEED(ctx && model && keys && query && result);
    *result = nullptr;
    std::vector<const Ct*> planes;
    for (auto& p : query->v) planes.push_back(p.get());
    auto r = std::make_unique<copse_cts>();
    r->v.push_back(evaluate_group_plain(*ctx->c, *model->m, *keys->k, planes));
    *result = r.release();
  });
}

int copse_evaluate_batch(copse_ctx* ctx, const copse_model* model, const copse_keys* keys,
                         const copse_cts* const* queries, size_t n_groups, copse_cts** results) {
  return guarded([&] {
    NEED(ctx && model && keys && queries && results);
    std::vector<std::vector<const Ct*>> groups;
    for (size_t g = 0; g < n_groups; ++g) {
      NEED(queries[g]);
      std::vector<const Ct*> planes;
      for (auto& p : queries[g]->v) planes.push_back(p.get());
      groups.push_back(planes);
    }
    auto rs = evaluate_groups(*ctx->c, *model->m, *keys->k, groups);
    for (size_t g = 0; g < n_groups; ++g) {
      auto r = new copse_cts();
      r->v.push_back(std::move(rs[g]));
      results[g] = r;
    }
  });
}

// ---------------------------------------------------------------- decrypt
int copse_decrypt_labels(copse_ctx* ctx, const copse_keys* keys, const copse_public_meta* meta,
                         const copse_cts* result, size_t n_queries, uint8_t* bits, size_t cap) {
  return guarded([&] {
    NEED(ctx && keys && meta && result && bits && result->v.size() == 1);
    Context& c = *ctx->c;
    const Ct& ct = ct_of(c, result, 0);
    keys_of(c, keys);
    if (ct.level != 0 || ct.npolys != 2) fail(COPSE_EINVAL, "result must be at level 0");
    if ((1ULL << meta->log_n) != c.N || meta->block_w == 0 || meta->block_w > c.N / 2 || meta->m > meta->block_w)
      fail(COPSE_EINVAL, "layout made for another ring size");
    if (n_queries > meta->queries_per_ct) fail(COPSE_EINVAL, "more queries than blocks");
    if (cap < n_queries * meta->m) fail(COPSE_EINVAL, "bits buffer too small");
    std::vector<uint64_t> ph;
    phase_coef(c, *keys->k, ct, ph);
    const uint64_t q0 = c.primes[0];
    std::vector<uint64_t> coef(c.N);
    uint64_t worst = 0;
    for (size_t i = 0; i < c.N; ++i) {
      uint64_t v = ph[i];
      bool neg = v > q0 / 2;
      uint64_t mag = neg ? q0 - v : v;
      worst = std::max(worst, mag);
      uint64_t r = mag % c.t;
      coef[i] = neg ? (r ? c.t - r : 0) : r;
    }
    if (worst >= (q0 >> 11)) fail(COPSE_ENOISE, "decryption noise above q_0 / 2^11");
    std::vector<uint64_t> slots(c.N);
    decode_poly(c, coef, slots.data());
    size_t bpr = (c.N / 2) / meta->block_w;
    for (size_t k = 0; k < n_queries; ++k) {
      size_t row = k / bpr, col0 = (k % bpr) * meta->block_w;
      uint32_t ones = 0;
      for (uint32_t j = 0; j < meta->m; ++j) {
        uint64_t v = slots[row * (c.N / 2) + col0 + j];
        if (v > 1) fail(COPSE_ENOISE, "decrypted label slot is not a bit");
        bits[k * meta->m + j] = (uint8_t)v;
        ones += (uint32_t)v;
      }
      // the result is N-hot: exactly one label per tree (Section 4.1, "Classification Result")
      if (ones != meta->n_trees)
        fail(COPSE_ENOISE, "query " + std::to_string(k) + " decrypts to " + std::to_string(ones) + " labels for " +
                               std::to_string(meta->n_trees) + " trees");
    }
  });
}

// ---------------------------------------------------------------- raw ciphertext ops
int copse_encrypt_slots(copse_ctx* ctx, const copse_keys* keys, const uint64_t* slots, int level,
                        const uint8_t seed[32], uint64_t obj, copse_cts** out) {
  return guarded([&] {
    NEED(ctx && keys && slots && seed && out);
    Context& c = *ctx->c;
    if (level < 0 || level > c.L) fail(COPSE_EINVAL, "level out of range");
    std::vector<int64_t> poly;
    encode_slots(c, slots, poly);
    auto r = std::make_unique<copse_cts>();
    r->v.push_back(encrypt(c, keys_of(c, keys), poly, level, seed, obj));
    *out = r.release();
  });
}

int copse_decrypt_slots(copse_ctx* ctx, const copse_keys* keys, const copse_cts* cts, size_t i, uint64_t* slots) {
  return guarded([&] {
    NEED(ctx && keys && cts && slots && i < cts->v.size());
    Context& c = *ctx->c;
    const Ct& ct = ct_of(c, cts, i);
    std::vector<uint64_t> ph;
    phase_coef(c, keys_of(c, keys), ct, ph);
    // exact CRT of each coefficient over q_0..q_level, centered, mod t (Garner's mixed radix)
    const int nl = ct.level + 1;
    std::vector<uint64_t> coef(c.N);
    for (size_t j = 0; j < c.N; ++j) {
      // mixed-radix digits v_i so that x = v_0 + v_1 q_0 + v_2 q_0 q_1 + ...
      std::vector<uint64_t> v(nl);
      for (int a = 0; a < nl; ++a) {
        uint64_t qa = c.primes[a];
        uint64_t x = ph[(size_t)a * c.N + j] % qa;
        uint64_t acc = 0, prod = 1;
        for (int b2 = 0; b2 < a; ++b2) {
          acc = (acc + mulmod(v[b2] % qa, prod, qa)) % qa;
          prod = mulmod(prod, c.primes[b2] % qa, qa);
        }
        uint64_t diff = (x + qa - acc) % qa;
        v[a] = mulmod(diff, invmod(prod, qa), qa);
      }
      // centered: x > Q/2 iff the top digit comparison says so; evaluate x mod t and Q mod t
      // x in [0, Q): compare with Q/2 through the mixed-radix digits of (Q-1)/2
      // Q/2 digits: compute digits of Q - 1 - x (negative side) lazily by comparing digit strings
      std::vector<uint64_t> h(nl);   // mixed-radix digits of (Q-1)/2
      {
        // (Q-1)/2 has digits ((q_i - 1)/2 ... ) only when all q_i odd: Q-1 has digits q_i-1
        // and halving a mixed-radix number with odd radices carries the remainder downward.
        uint64_t carry = 0;
        for (int a = nl - 1; a >= 0; --a) {
          unsigned __int128 cur = (unsigned __int128)carry * c.primes[a] + (c.primes[a] - 1);
          h[a] = (uint64_t)(cur / 2);
          carry = (uint64_t)(cur % 2);
        }
      }
      bool neg = false;
      for (int a = nl - 1; a >= 0; --a) {
        if (v[a] != h[a]) { neg = v[a] > h[a]; break; }
      }
      // x mod t and Q mod t
      uint64_t xm = 0, prod = 1, Qm = 1;
      for (int a = 0; a < nl; ++a) {
        xm = (xm + mulmod(v[a] % c.t, prod, c.t)) % c.t;
        prod = mulmod(prod, c.primes[a] % c.t, c.t);
      }
      Qm = prod;
      coef[j] = neg ? (xm + c.t - Qm) % c.t : xm;
    }
    decode_poly(c, coef, slots);
  });
}

int copse_cts_export(copse_ctx* ctx, const copse_cts* cts, uint64_t* buf, size_t cap, size_t* need) {
  return guarded([&] {
    NEED(ctx && cts && need);
    Context& c = *ctx->c;
    size_t total = 0;
    for (auto& ct : cts->v) total += 4 + ct->words();
    *need = total;
    if (!buf) return;
    if (cap < total) fail(COPSE_EINVAL, "export buffer too small");
    size_t off = 0;
    for (auto& ct : cts->v) {
      std::vector<uint64_t> co;
      to_coef_u64(c, *ct, co);
      buf[off++] = (uint64_t)ct->npolys;
      buf[off++] = (uint64_t)ct->level;
      buf[off++] = (uint64_t)c.N;
      buf[off++] = 0;
      std::copy(co.begin(), co.end(), buf + off);
      off += co.size();
    }
  });
}

int copse_cts_import(copse_ctx* ctx, const uint64_t* buf, size_t len, copse_cts** out) {
  return guarded([&] {
    NEED(ctx && buf && out);
    *out = nullptr;
    Context& c = *ctx->c;
    auto r = std::make_unique<copse_cts>();
    size_t off = 0;
    while (off < len) {
      if (len - off < 4) fail(COPSE_EINVAL, "truncated header");
      uint64_t np = buf[off], lv = buf[off + 1], n = buf[off + 2];
      if (np < 1 || np > 3 || lv > (uint64_t)c.L || n != c.N) fail(COPSE_EINVAL, "bad ciphertext header");
      off += 4;
      size_t words = (size_t)np * (lv + 1) * c.N;
      if (len - off < words) fail(COPSE_EINVAL, "truncated ciphertext");
      r->v.push_back(from_coef_u64(c, buf + off, (int)lv, (int)np));
      off += words;
    }
    *out = r.release();
  });
}

int copse_ct_op(copse_ctx* ctx, const copse_keys* keys, int op, const copse_cts* a, size_t ia, const copse_cts* b,
                size_t ib, int32_t arg, const uint64_t* slots, copse_cts** out) {
  return guarded([&] {
    NEED(ctx && a && ia < a->v.size() && out);
    *out = nullptr;
    Context& c = *ctx->c;
    const Ct& x = ct_of(c, a, ia);
    auto needb = [&]() -> const Ct& {
      NEED(b);
      return ct_of(c, b, ib);
    };
    auto needk = [&]() -> const Keys& {
      NEED(keys);
      return keys_of(c, keys);
    };
    CtPtr r;
    switch (op) {
      case COPSE_OP_ADD: r = op_add(c, x, needb()); break;
      case COPSE_OP_SUB: r = op_sub(c, x, needb()); break;
      case COPSE_OP_TENSOR: r = op_tensor(c, x, needb()); break;
      case COPSE_OP_RELIN: r = op_relin(c, needk(), x); break;
      case COPSE_OP_MODSWITCH: r = op_modswitch(c, x); break;
      case COPSE_OP_MUL: r = op_mul(c, needk(), x, needb()); break;
      case COPSE_OP_ROTATE: r = op_rotate(c, needk(), x, arg); break;
      case COPSE_OP_MUL_PLAIN: {
        NEED(slots);
        auto p = make_plain_slots(c, slots, x.level);
        r = op_mul_plain(c, x, *p);
        break;
      }
      case COPSE_OP_ADD_PLAIN: {
        NEED(slots);
        auto p = make_plain_slots(c, slots, x.level);
        r = op_add_plain(c, x, *p);
        break;
      }
      default: fail(COPSE_EINVAL, "unknown op");
    }
    COPSE_HIP(hipStreamSynchronize(c.stream));
    auto res = std::make_unique<copse_cts>();
    res->v.push_back(std::move(r));
    *out = res.release();
  });
}

int copse_ct_rotate_many(copse_ctx* ctx, const copse_keys* keys, const copse_cts* a, size_t ia, const int32_t* rots,
                         size_t n, copse_cts** out) {
  return guarded([&] {
    NEED(ctx && keys && a && ia < a->v.size() && rots && out);
    std::vector<int32_t> r(rots, rots + n);
    auto v = op_rotate_hoisted(*ctx->c, keys_of(*ctx->c, keys), ct_of(*ctx->c, a, ia), r);
    auto res = std::make_unique<copse_cts>();
    for (auto& x : v) res->v.push_back(std::move(x));
    COPSE_HIP(hipStreamSynchronize(ctx->c->stream));
    *out = res.release();
  });
}

int copse_poly_mul(copse_ctx* ctx, int prime, const uint64_t* a, const uint64_t* b, uint64_t* out) {
  return guarded([&] {
    NEED(ctx && a && b && out);
    Context& c = *ctx->c;
    if (prime < 0 || prime >= c.n_primes()) fail(COPSE_EINVAL, "prime index out of range");
    const size_t N = c.N;
    std::vector<double> h(2 * N);
    for (size_t i = 0; i < N; ++i) {
      if (a[i] >= c.primes[prime] || b[i] >= c.primes[prime]) fail(COPSE_EINVAL, "residue out of range");
      h[i] = (double)a[i];
      h[N + i] = (double)b[i];
    }
    DBuf d(&c, 2 * N);
    COPSE_HIP(hipMemcpyAsync(d.get(), h.data(), 2 * N * 8, hipMemcpyHostToDevice, c.stream));
    std::vector<int2> rows = {make_int2(0, prime), make_int2(1, prime)};
    const int2* r2 = c.rows("pm2:" + std::to_string(prime), rows);
    launch_ntt_fwd(c, d.get(), r2, 2);
    launch_mul(c, d.get(), d.get(), d.get() + N, r2, 1);
    launch_ntt_inv(c, d.get(), r2, 1);
    COPSE_HIP(hipMemcpyAsync(h.data(), d.get(), N * 8, hipMemcpyDeviceToHost, c.stream));
    COPSE_HIP(hipStreamSynchronize(c.stream));
    for (size_t i = 0; i < N; ++i) out[i] = (uint64_t)h[i];
  });
}

int copse_profile_enable(copse_ctx* ctx, int on) {
  return guarded([&] {
    NEED(ctx);
    ctx->c->profiling = on != 0;
  });
}

int copse_profile_read(copse_ctx* ctx, int kind, uint64_t* launches, double* total_ms, double* bytes, int reset) {
  return guarded([&] {
    NEED(ctx && kind >= 0 && kind < kProfKinds);
    Context& c = *ctx->c;
    prof_collect(c);
    if (launches) *launches = c.prof[kind].launches;
    if (total_ms) *total_ms = c.prof[kind].ms;
    if (bytes) *bytes = c.prof[kind].bytes;
    if (reset) c.prof[kind] = ProfSlot();
  });
}

int copse_calib_copy(copse_ctx* ctx, size_t bytes) {
  return guarded([&] {
    NEED(ctx && bytes >= 8);
    Context& c = *ctx->c;
    size_t n = bytes / 8;
    DBuf a(&c, n), b(&c, n);
    COPSE_HIP(hipMemsetAsync(a.get(), 0, n * 8, c.stream));
    launch_calib_copy(c, b.get(), a.get(), n);
    COPSE_HIP(hipStreamSynchronize(c.stream));
  });
}

int copse_chain_primes(const copse_params* p, uint64_t* out, size_t cap, size_t* n) {
  return guarded([&] {
    NEED(p && n);
    auto v = make_chain(*p);
    *n = v.size();
    if (out) {
      if (cap < v.size()) fail(COPSE_EINVAL, "buffer too small");
      std::copy(v.begin(), v.end(), out);
    }
  });
}

int copse_test_encode(uint32_t log_n, uint64_t t, const uint64_t* slots, int64_t* coeffs) {
  return guarded([&] {
    NEED(slots && coeffs && log_n >= 1 && log_n <= 17);
    Context c;
    c.log_n = log_n;
    c.N = 1ULL << log_n;
    c.t = t;
    if ((t - 1) % (2 * c.N)) fail(COPSE_EINVAL, "t must be 1 mod 2N");
    setup_slots(c);
    std::vector<int64_t> out;
    encode_slots(c, slots, out);
    std::copy(out.begin(), out.end(), coeffs);
  });
}

int copse_test_shake256(const uint8_t* msg, size_t len, uint8_t* out, size_t outlen) {
  return guarded([&] {
    NEED((msg || len == 0) && out);
    shake256(msg, len, out, outlen);
  });
}

int copse_test_sample(const uint8_t seed[32], const char* domain, uint64_t obj, uint32_t limb, int kind, uint64_t q,
                      size_t n, int64_t* out) {
  return guarded([&] {
    NEED(seed && domain && out);
    if (kind == 0) {
      std::vector<double> v(n);
      sample_uniform(seed, domain, obj, limb, q, n, v.data());
      for (size_t i = 0; i < n; ++i) out[i] = (int64_t)v[i];
    } else if (kind == 1) {
      sample_ternary(seed, domain, obj, n, out);
    } else {
      sample_cbd21(seed, domain, obj, n, out);
    }
  });
}

}  // extern "C"
