// BGV over the RNS chain on the device: context tables, encoding, keys,
// encryption and the homomorphic operations (tensor, relinearization,
// hoisted rotations with hybrid key switching, modulus switching).
//
// Ciphertexts are kept in the evaluation (NTT) domain; the coefficient
// domain is visited only where an operation is defined on coefficients:
// the base conversions of key switching and the division by the dropped
// prime of a modulus switch.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace copse {

// ------------------------------------------------------------------ DBuf
DBuf::DBuf(Context* c, size_t doubles) : pool_(c->pool), n_(doubles) {
  p_ = doubles ? (double*)pool_->alloc(doubles * sizeof(double)) : nullptr;
}
DBuf& DBuf::operator=(DBuf&& o) noexcept {
  if (this != &o) {
    reset();
    pool_ = std::move(o.pool_); p_ = o.p_; n_ = o.n_;
    o.p_ = nullptr; o.n_ = 0;
  }
  return *this;
}
void DBuf::reset() {
  if (p_ && pool_) pool_->free(p_);
  p_ = nullptr; n_ = 0;
  pool_.reset();
}

// ------------------------------------------------------------------ profiling
void prof_begin(Context& c, int kind, hipEvent_t* ev) {
  *ev = nullptr;
  if (!c.profiling) return;
  hipEvent_t e;
  if (!c.event_cache.empty()) { e = c.event_cache.back(); c.event_cache.pop_back(); }
  else COPSE_HIP(hipEventCreate(&e));
  COPSE_HIP(hipEventRecord(e, c.stream));
  *ev = e;
  (void)kind;
}
void prof_end(Context& c, int kind, hipEvent_t ev, double bytes) {
  if (!c.profiling || !ev) return;
  hipEvent_t e;
  if (!c.event_cache.empty()) { e = c.event_cache.back(); c.event_cache.pop_back(); }
  else COPSE_HIP(hipEventCreate(&e));
  COPSE_HIP(hipEventRecord(e, c.stream));
  c.pending[kind].push_back({ev, e});
  c.prof[kind].launches += 1;
  c.prof[kind].bytes += bytes;
  if (c.pending[kind].size() > 4096) prof_collect(c);
}
void prof_collect(Context& c) {
  for (int k = 0; k < kProfKinds; ++k) {
    for (auto& pr : c.pending[k]) {
      COPSE_HIP(hipEventSynchronize(pr.second));
      float ms = 0;
      COPSE_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      c.prof[k].ms += ms;
      c.event_cache.push_back(pr.first);
      c.event_cache.push_back(pr.second);
    }
    c.pending[k].clear();
  }
}

// ------------------------------------------------------------------ context helpers
Context::~Context() {
  if (!d_primes && !own_stream && tables.empty()) return;   // host-only context
  hipSetDevice(device);
  for (auto& ev : event_cache) (void)hipEventDestroy(ev);
  for (int k = 0; k < kProfKinds; ++k)
    for (auto& pr : pending[k]) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
  for (auto& kv : ks)
    for (double* p : kv.second->owned) (void)hipFree(p);
  for (auto& kv : row_tables) (void)hipFree(kv.second);
  for (double* p : tables) (void)hipFree(p);
  if (d_primes) (void)hipFree(d_primes);
  pool.reset();
  if (own_stream) (void)hipStreamDestroy(own_stream);
}

const int2* Context::rows(const std::string& key, const std::vector<int2>& host) {
  auto it = row_tables.find(key);
  if (it != row_tables.end()) return it->second;
  if (no_alloc) {
    // built in the scratch pool for this call only; the host copy lives until the call has synchronized
    auto ic = call_rows.find(key);
    if (ic != call_rows.end()) return ic->second;
    call_row_bufs.emplace_back(this, (std::max<size_t>(1, host.size()) * sizeof(int2) + 7) / 8);
    call_rows_host.push_back(host);
    int2* d = reinterpret_cast<int2*>(call_row_bufs.back().get());
    COPSE_HIP(hipMemcpyAsync(d, call_rows_host.back().data(), host.size() * sizeof(int2), hipMemcpyHostToDevice,
                             stream));
    call_rows[key] = d;
    return d;
  }
  int2* d = nullptr;
  COPSE_HIP(hipMalloc(&d, std::max<size_t>(1, host.size()) * sizeof(int2)));
  COPSE_HIP(hipMemcpy(d, host.data(), host.size() * sizeof(int2), hipMemcpyHostToDevice));
  row_tables[key] = d;
  return d;
}

// rows of an [np][nl][N] block with primes 0..nl-1
static const int2* ct_rows(Context& c, int np, int nl) {
  std::string key = "ct:" + std::to_string(np) + ":" + std::to_string(nl);
  std::vector<int2> h;
  for (int k = 0; k < np; ++k)
    for (int i = 0; i < nl; ++i) h.push_back(make_int2(k * nl + i, i));
  return c.rows(key, h);
}

static double* upload(std::vector<double*>& owner, const std::vector<double>& v) {
  double* d = nullptr;
  COPSE_HIP(hipMalloc(&d, std::max<size_t>(1, v.size()) * sizeof(double)));
  COPSE_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  owner.push_back(d);
  return d;
}

KSTables& Context::kstab(int level) {
  auto it = ks.find(level);
  if (it != ks.end()) return *it->second;
  if (no_alloc) fail(COPSE_EINVAL, "internal: level tables missing in an evaluation without allocation");
  auto T = std::make_unique<KSTables>();
  const int nl = level + 1, nE = nl + alpha;
  auto prime_of_ext = [&](int o) { return o < nl ? o : L + 1 + (o - nl); };
  for (int j = 0; j < n_digits(level); ++j) {
    KSTables::Digit dg;
    dg.first = j * alpha;
    dg.count = std::min(alpha, nl - dg.first);
    for (int o = 0; o < nE; ++o)
      if (o < dg.first || o >= dg.first + dg.count) dg.targets.push_back(o);
    std::vector<double> mult, mat;
    for (int k = 0; k < dg.count; ++k) {
      uint64_t qi = primes[dg.first + k];
      // (Q_j / q_i)^-1 mod q_i
      uint64_t hat = 1;
      for (int k2 = 0; k2 < dg.count; ++k2)
        if (k2 != k) hat = mulmod(hat, primes[dg.first + k2] % qi, qi);
      mult.push_back((double)invmod(hat, qi));
    }
    for (int k = 0; k < dg.count; ++k) {
      for (int o : dg.targets) {
        uint64_t p = primes[prime_of_ext(o)];
        uint64_t hat = 1;
        for (int k2 = 0; k2 < dg.count; ++k2)
          if (k2 != k) hat = mulmod(hat, primes[dg.first + k2] % p, p);
        mat.push_back((double)hat);
      }
    }
    dg.d_mult = upload(T->owned, mult);
    dg.d_mat = upload(T->owned, mat);
    std::vector<int2> outr, inr;
    for (int o : dg.targets) outr.push_back(make_int2(j * nE + o, prime_of_ext(o)));
    for (int k = 0; k < dg.count; ++k) inr.push_back(make_int2(dg.first + k, dg.first + k));
    dg.d_out_rows = const_cast<int2*>(rows("ksout:" + std::to_string(level) + ":" + std::to_string(j), outr));
    dg.d_in_rows = const_cast<int2*>(rows("ksin:" + std::to_string(level) + ":" + std::to_string(j), inr));
    T->digits.push_back(std::move(dg));
  }
  // ModDown constants
  std::vector<double> mdm, mdmat, pinv, tpinv;
  for (int r = 0; r < alpha; ++r) {
    uint64_t p = primes[L + 1 + r];
    uint64_t hat = 1;
    for (int r2 = 0; r2 < alpha; ++r2)
      if (r2 != r) hat = mulmod(hat, primes[L + 1 + r2] % p, p);
    mdm.push_back((double)mulmod(invmod(t % p, p), invmod(hat, p), p));
  }
  for (int r = 0; r < alpha; ++r)
    for (int i = 0; i < nl; ++i) {
      uint64_t q = primes[i];
      uint64_t hat = 1;
      for (int r2 = 0; r2 < alpha; ++r2)
        if (r2 != r) hat = mulmod(hat, primes[L + 1 + r2] % q, q);
      mdmat.push_back((double)hat);
    }
  for (int i = 0; i < nl; ++i) {
    uint64_t q = primes[i];
    uint64_t P = 1;
    for (int r = 0; r < alpha; ++r) P = mulmod(P, primes[L + 1 + r] % q, q);
    uint64_t pi = invmod(P, q);
    pinv.push_back((double)pi);
    tpinv.push_back((double)mulmod(t % q, pi, q));
  }
  T->d_md_mult = upload(T->owned, mdm);
  T->d_md_mat = upload(T->owned, mdmat);
  T->d_md_pinv = upload(T->owned, pinv);
  T->d_md_tpinv = upload(T->owned, tpinv);
  if (level >= 1) {
    uint64_t ql = primes[level];
    std::vector<double> ms = {(double)level, (double)invmod(t % ql, ql)};
    for (int i = 0; i < level; ++i) {
      uint64_t q = primes[i];
      uint64_t inv = invmod(ql % q, q);
      ms.push_back((double)inv);
      ms.push_back((double)mulmod(t % q, inv, q));
    }
    T->d_ms = upload(T->owned, ms);
    // ModDown merged with the switch to level - 1 (see launch_ntt_fwd_rows_mdms_finish)
    std::vector<double> mm_mult, mm_mat, m1, m2, m3;
    for (int r = 0; r < alpha; ++r) mm_mult.push_back(mdm[r]);
    uint64_t Pl = 1;
    for (int r = 0; r < alpha; ++r) Pl = mulmod(Pl, primes[L + 1 + r] % ql, ql);
    mm_mult.push_back((double)invmod(mulmod(t % ql, Pl, ql), ql));
    for (int r = 0; r < alpha; ++r)
      for (int i = 0; i <= level; ++i) {
        uint64_t q = primes[i];
        mm_mat.push_back((double)invmod(primes[L + 1 + r] % q, q));
      }
    bool ok = true;
    for (int i = 0; i < level; ++i) {
      uint64_t q = primes[i];
      uint64_t P = 1;
      for (int r = 0; r < alpha; ++r) P = mulmod(P, primes[L + 1 + r] % q, q);
      uint64_t qlinv = invmod(ql % q, q);
      m1.push_back((double)mulmod(invmod(P, q), qlinv, q));
      m2.push_back((double)mulmod(t % q, qlinv, q));
      m3.push_back((double)qlinv);
      ok = ok && ql < 4 * q;
    }
    T->d_mm_mult = upload(T->owned, mm_mult);
    T->d_mm_mat = upload(T->owned, mm_mat);
    T->d_mm_m1 = upload(T->owned, m1);
    T->d_mm_m2 = upload(T->owned, m2);
    T->d_mm_m3 = upload(T->owned, m3);
    T->mm_ptop = (double)Pl;
    T->mm_ok = ok;
  }
  auto& ref = *T;
  ks[level] = std::move(T);
  return ref;
}

const MsMulti& Context::ms_multi(int level, int k) {
  if (k < 1 || k > 4 || k > level) fail(COPSE_EINVAL, "internal: switch by an unsupported prime count");
  KSTables& T = kstab(level);
  auto it = T.multi.find(k);
  if (it != T.multi.end()) return it->second;
  if (no_alloc) fail(COPSE_EINVAL, "internal: switch tables missing in an evaluation without allocation");
  MsMulti M;
  const int n_out = level - k + 1;
  std::vector<uint64_t> pm;   // p_m = q_{level - m}
  for (int m = 0; m < k; ++m) pm.push_back(primes[level - m]);
  // D_u mod x for u <= k
  auto Dmod = [&](int u, uint64_t x) {
    uint64_t d = 1;
    for (int v = 0; v < u; ++v) d = mulmod(d, pm[v] % x, x);
    return d;
  };
  std::vector<double> mult, mat((size_t)k * n_out + 4 * k, 0.0), tab(2 + 2 * (size_t)n_out, 0.0);
  for (int m = 0; m < k; ++m) mult.push_back((double)invmod(mulmod(t % pm[m], Dmod(m, pm[m]), pm[m]), pm[m]));
  for (int u = 0; u < k; ++u)
    for (int o = 0; o < n_out; ++o) mat[(size_t)u * n_out + o] = (double)Dmod(u, primes[o]);
  for (int m = 1; m < k; ++m) {
    const uint64_t dinv = invmod(Dmod(m, pm[m]), pm[m]);
    for (int u = 0; u < m; ++u) mat[(size_t)k * n_out + 4 * m + u] = (double)mulmod(Dmod(u, pm[m]), dinv, pm[m]);
  }
  tab[0] = (double)level;
  for (int o = 0; o < n_out; ++o) {
    const uint64_t q = primes[o];
    const uint64_t dinv = invmod(Dmod(k, q), q);
    tab[2 + 2 * o] = (double)dinv;
    tab[3 + 2 * o] = (double)mulmod(t % q, dinv, q);
  }
  M.mult = upload(T.owned, mult);
  M.mat = upload(T.owned, mat);
  M.tab = upload(T.owned, tab);
  std::vector<int2> ir, orr;
  for (int m = 0; m < k; ++m) ir.push_back(make_int2(m, level - m));
  for (int o = 0; o < n_out; ++o) orr.push_back(make_int2(o, o));
  M.in_rows = rows("mskin:" + std::to_string(level) + ":" + std::to_string(k), ir);
  M.out_rows = rows("mskout:" + std::to_string(level) + ":" + std::to_string(k), orr);
  return T.multi.emplace(k, M).first->second;
}

void Context::select_tuning(int batch, bool encrypted_model) {
  tune = Tuning{};
  for (const TuneEntry& e : tune_table)
    if (e.log_n == log_n && e.top_level == (uint32_t)L && (uint32_t)batch >= e.batch_lo &&
        (uint32_t)batch <= e.batch_hi && (e.model < 0 || e.model == (encrypted_model ? 1 : 0))) {
      tune = e.t;
      return;
    }
}

void Context::build_level_tables() {
  for (int l = 0; l <= L; ++l) {
    kstab(l);
    for (int k = 1; k <= std::min(4, l); ++k) ms_multi(l, k);
  }
}

uint64_t galois_of(const Context& c, int64_t r) {
  int64_t half = (int64_t)c.N / 2;
  int64_t rr = ((r % half) + half) % half;
  return powmod(5, (uint64_t)rr, 2 * c.N);
}

// ------------------------------------------------------------------ ciphertext helpers
CtPtr ct_alloc(Context& c, int level, int npolys) {
  auto ct = std::make_unique<Ct>();
  ct->level = level;
  ct->npolys = npolys;
  ct->n = c.N;
  ct->store = std::make_shared<DBuf>(&c, (size_t)npolys * (level + 1) * c.N);
  ct->ptr = ct->store->get();
  return ct;
}

CtPtr ct_copy(Context& c, const Ct& a) {
  auto o = ct_alloc(c, a.level, a.npolys);
  COPSE_HIP(hipMemcpyAsync(o->data(), a.data(), a.words() * sizeof(double), hipMemcpyDeviceToDevice,
                           c.stream));
  return o;
}

// Drop limbs above `level` (no rescaling): used to read a key or plaintext at a lower level.
static CtPtr ct_truncate_copy(Context& c, const Ct& a, int level) {
  auto o = ct_alloc(c, level, a.npolys);
  for (int k = 0; k < a.npolys; ++k)
    COPSE_HIP(hipMemcpyAsync(o->poly(k, c.N), a.poly(k, c.N), (size_t)(level + 1) * c.N * sizeof(double),
                             hipMemcpyDeviceToDevice, c.stream));
  return o;
}

// ------------------------------------------------------------------ encoding (host, mod t)
// Host transform mod t: the same bit-reversed Cooley-Tukey / Gentleman-Sande pair as the device
// kernels, with the slot root zeta in place of psi.  Evaluation slot k holds m(zeta^(2 bitrev(k)+1)).
static void host_ntt_t(const Context& c, std::vector<uint64_t>& a, bool inverse) {
  const uint64_t t = c.t;
  const size_t N = c.N;
  const int logN = (int)c.log_n;
  static thread_local std::vector<uint64_t> fw, iv;
  static thread_local uint64_t cached_zeta = 0, cached_n = 0;
  if (cached_zeta != c.zeta || cached_n != N) {
    fw.assign(N, 0); iv.assign(N, 0);
    uint64_t zinv = invmod(c.zeta, t);
    for (size_t k = 0; k < N; ++k) {
      uint32_t br = bitrev((uint32_t)k, logN);
      fw[k] = powmod(c.zeta, br, t);
      iv[k] = powmod(zinv, br, t);
    }
    cached_zeta = c.zeta; cached_n = N;
  }
  if (!inverse) {
    for (int s = 0; s < logN; ++s) {
      size_t half = N >> (s + 1), m = (size_t)1 << s;
      for (size_t i = 0; i < m; ++i) {
        uint64_t w = fw[m + i];
        for (size_t j = 2 * i * half; j < 2 * i * half + half; ++j) {
          uint64_t x = a[j], y = mulmod(a[j + half], w, t);
          a[j] = (x + y) % t;
          a[j + half] = (x + t - y) % t;
        }
      }
    }
  } else {
    for (int s = logN - 1; s >= 0; --s) {
      size_t half = N >> (s + 1), m = (size_t)1 << s;
      for (size_t i = 0; i < m; ++i) {
        uint64_t w = iv[m + i];
        for (size_t j = 2 * i * half; j < 2 * i * half + half; ++j) {
          uint64_t x = a[j], y = a[j + half];
          a[j] = (x + y) % t;
          a[j + half] = mulmod((x + t - y) % t, w, t);
        }
      }
    }
    uint64_t ninv = invmod(N % t, t);
    for (size_t j = 0; j < N; ++j) a[j] = mulmod(a[j], ninv, t);
  }
}

void encode_slots(const Context& c, const uint64_t* slots, std::vector<int64_t>& out) {
  std::vector<uint64_t> ev(c.N);
  for (size_t s = 0; s < c.N; ++s) ev[c.slot_pos[s]] = slots[s] % c.t;
  host_ntt_t(c, ev, true);
  out.resize(c.N);
  const int64_t half = (int64_t)(c.t - 1) / 2;
  for (size_t j = 0; j < c.N; ++j) {
    int64_t v = (int64_t)ev[j];
    out[j] = v > half ? v - (int64_t)c.t : v;
  }
}

void decode_poly(const Context& c, const std::vector<uint64_t>& coeffs, uint64_t* slots) {
  std::vector<uint64_t> ev(coeffs);
  for (auto& v : ev) v %= c.t;
  host_ntt_t(c, ev, false);
  for (size_t s = 0; s < c.N; ++s) slots[s] = ev[c.slot_pos[s]];
}

// Upload small signed integers and reduce them modulo primes 0..level (NTT form on return).
static void lift_to(Context& c, double* dst, const std::vector<int64_t>& v, int nrows_level, bool ntt,
                    const int2* rows_override = nullptr, int nrows_override = 0) {
  std::vector<double> hv(v.size());
  for (size_t i = 0; i < v.size(); ++i) hv[i] = (double)v[i];
  DBuf tmp(&c, c.N);
  COPSE_HIP(hipMemcpyAsync(tmp.get(), hv.data(), c.N * sizeof(double), hipMemcpyHostToDevice, c.stream));
  const int2* rows = rows_override ? rows_override : ct_rows(c, 1, nrows_level + 1);
  int nrows = rows_override ? nrows_override : nrows_level + 1;
  launch_lift(c, dst, tmp.get(), rows, nrows);
  if (ntt) launch_ntt_fwd(c, dst, rows, nrows);
  COPSE_HIP(hipStreamSynchronize(c.stream));   // hv is pageable host memory
}

std::unique_ptr<Plain> make_plain(Context& c, const std::vector<int64_t>& centered, int level) {
  auto p = std::make_unique<Plain>();
  p->level = level;
  p->buf = DBuf(&c, (size_t)(level + 1) * c.N);
  lift_to(c, p->buf.get(), centered, level, true);
  return p;
}

std::unique_ptr<Plain> make_plain_slots(Context& c, const uint64_t* slots, int level) {
  std::vector<int64_t> m;
  encode_slots(c, slots, m);
  return make_plain(c, m, level);
}

// ------------------------------------------------------------------ keys
static const int2* all_rows(Context& c, int count_polys) {
  // [count][Ltot] rows, primes 0..Ltot-1
  int Lt = c.n_primes();
  return ct_rows(c, count_polys, Lt);
}

std::unique_ptr<Keys> keygen(Context& c, const uint8_t seed[32], const std::vector<int32_t>& rots, bool relin) {
  const size_t N = c.N;
  const int Lt = c.n_primes();
  auto K = std::make_unique<Keys>();
  K->primes = c.primes;
  K->has_secret = true;
  K->s_host.resize(N);
  sample_ternary(seed, "sk.s", 0, N, K->s_host.data());
  K->s = DBuf(&c, (size_t)Lt * N);
  lift_to(c, K->s.get(), K->s_host, 0, true, all_rows(c, 1), Lt);
  // pk over data primes
  const int nd = c.L + 1;
  const int2* drows = ct_rows(c, 1, nd);
  K->pk_a = DBuf(&c, (size_t)nd * N);
  K->pk_b = DBuf(&c, (size_t)nd * N);
  {
    std::vector<double> ha((size_t)nd * N);
    for (int i = 0; i < nd; ++i) sample_uniform(seed, "pk.a", 0, (uint32_t)i, c.primes[i], N, ha.data() + (size_t)i * N);
    COPSE_HIP(hipMemcpyAsync(K->pk_a.get(), ha.data(), ha.size() * 8, hipMemcpyHostToDevice, c.stream));
    launch_ntt_fwd(c, K->pk_a.get(), drows, nd);
    std::vector<int64_t> e(N);
    sample_cbd21(seed, "pk.e", 0, N, e.data());
    for (auto& v : e) v *= (int64_t)c.t;
    DBuf te(&c, (size_t)nd * N);
    lift_to(c, te.get(), e, c.L, true);
    DBuf as(&c, (size_t)nd * N);
    launch_mul(c, as.get(), K->pk_a.get(), K->s.get(), drows, nd);
    launch_sub(c, K->pk_b.get(), te.get(), as.get(), drows, nd);
    COPSE_HIP(hipStreamSynchronize(c.stream));
  }
  const int D = c.n_digits(c.L);
  const int2* arows = all_rows(c, 1);
  auto make_ksk = [&](const DBuf& snew, uint64_t key_id) {
    auto k = std::make_unique<Keys::KSK>();
    k->a = DBuf(&c, (size_t)D * Lt * N);
    k->b = DBuf(&c, (size_t)D * Lt * N);
    std::vector<double> ha((size_t)Lt * N);
    std::vector<int64_t> e(N);
    DBuf te(&c, (size_t)Lt * N), as(&c, (size_t)Lt * N);
    for (int j = 0; j < D; ++j) {
      uint64_t obj = key_id * 256 + (uint64_t)j;
      for (int i = 0; i < Lt; ++i)
        sample_uniform(seed, "ksk.a", obj, (uint32_t)i, c.primes[i], N, ha.data() + (size_t)i * N);
      double* aj = k->a.get() + (size_t)j * Lt * N;
      double* bj = k->b.get() + (size_t)j * Lt * N;
      COPSE_HIP(hipMemcpyAsync(aj, ha.data(), ha.size() * 8, hipMemcpyHostToDevice, c.stream));
      launch_ntt_fwd(c, aj, arows, Lt);
      sample_cbd21(seed, "ksk.e", obj, N, e.data());
      for (auto& v : e) v *= (int64_t)c.t;
      lift_to(c, te.get(), e, 0, true, arows, Lt);
      launch_mul(c, as.get(), aj, K->s.get(), arows, Lt);
      launch_sub(c, bj, te.get(), as.get(), arows, Lt);
      // gadget: + (P mod q_i) s' on the limbs of digit j
      int first = j * c.alpha, cnt = std::min(c.alpha, c.L + 1 - first);
      std::vector<double> pmod(Lt, 0.0);
      for (int i = first; i < first + cnt; ++i) {
        uint64_t P = 1;
        for (int r = 0; r < c.alpha; ++r) P = mulmod(P, c.primes[c.L + 1 + r] % c.primes[i], c.primes[i]);
        pmod[i] = (double)P;
      }
      DBuf dp(&c, Lt);
      COPSE_HIP(hipMemcpyAsync(dp.get(), pmod.data(), Lt * 8, hipMemcpyHostToDevice, c.stream));
      std::vector<int2> gr;
      for (int i = first; i < first + cnt; ++i) gr.push_back(make_int2(i, i));
      const int2* grow = c.rows("gad:" + std::to_string(first) + ":" + std::to_string(cnt), gr);
      DBuf gs(&c, (size_t)Lt * N);
      launch_mul_scalar(c, gs.get(), snew.get(), dp.get(), grow, cnt);
      launch_add(c, bj, bj, gs.get(), grow, cnt);
      COPSE_HIP(hipStreamSynchronize(c.stream));
    }
    K->bytes += 2 * (size_t)D * Lt * N * 8;
    return k;
  };
  if (relin) {
    DBuf s2(&c, (size_t)Lt * N);
    launch_mul(c, s2.get(), K->s.get(), K->s.get(), arows, Lt);
    K->relin = make_ksk(s2, 0);
  }
  for (int32_t r : rots) {
    uint64_t g = galois_of(c, r);
    if (g == 1 || K->rot.count(g)) continue;
    DBuf sg(&c, (size_t)Lt * N);
    launch_automorphism(c, sg.get(), K->s.get(), g, Lt, 1);
    K->rot[g] = make_ksk(sg, g);
  }
  K->bytes += (size_t)(Lt + 2 * nd) * N * 8;
  return K;
}

CtPtr encrypt(Context& c, const Keys& k, const std::vector<int64_t>& m, int level, const uint8_t seed[32],
              uint64_t obj) {
  const size_t N = c.N;
  const int nl = level + 1;
  const int2* rows1 = ct_rows(c, 1, nl);
  std::vector<int64_t> u(N), e0(N), e1(N);
  sample_ternary(seed, "enc.u", obj, N, u.data());
  sample_cbd21(seed, "enc.e0", obj, N, e0.data());
  sample_cbd21(seed, "enc.e1", obj, N, e1.data());
  for (size_t i = 0; i < N; ++i) {
    e0[i] = e0[i] * (int64_t)c.t + m[i];
    e1[i] = e1[i] * (int64_t)c.t;
  }
  DBuf du(&c, (size_t)nl * N), d0(&c, (size_t)nl * N), d1(&c, (size_t)nl * N);
  lift_to(c, du.get(), u, level, true);
  lift_to(c, d0.get(), e0, level, true);
  lift_to(c, d1.get(), e1, level, true);
  auto ct = ct_alloc(c, level, 2);
  launch_mul(c, ct->poly(0, N), k.pk_b.get(), du.get(), rows1, nl);
  launch_add(c, ct->poly(0, N), ct->poly(0, N), d0.get(), rows1, nl);
  launch_mul(c, ct->poly(1, N), k.pk_a.get(), du.get(), rows1, nl);
  launch_add(c, ct->poly(1, N), ct->poly(1, N), d1.get(), rows1, nl);
  COPSE_HIP(hipStreamSynchronize(c.stream));
  return ct;
}

// [c0 + c1 s (+ c2 s^2)] in coefficient form, per limb, as u64 residues.
void phase_coef(Context& c, const Keys& k, const Ct& a, std::vector<uint64_t>& out) {
  if (!k.has_secret) fail(COPSE_EKEY, "secret key absent");
  const size_t N = c.N;
  const int nl = a.level + 1;
  const int2* rows1 = ct_rows(c, 1, nl);
  DBuf acc(&c, (size_t)nl * N), sp(&c, (size_t)nl * N), tmp(&c, (size_t)nl * N);
  COPSE_HIP(hipMemcpyAsync(acc.get(), a.poly(0, N), (size_t)nl * N * 8, hipMemcpyDeviceToDevice, c.stream));
  COPSE_HIP(hipMemcpyAsync(sp.get(), k.s.get(), (size_t)nl * N * 8, hipMemcpyDeviceToDevice, c.stream));
  for (int p = 1; p < a.npolys; ++p) {
    launch_mac(c, acc.get(), a.poly(p, N), sp.get(), rows1, nl);
    if (p + 1 < a.npolys) {
      launch_mul(c, tmp.get(), sp.get(), k.s.get(), rows1, nl);
      std::swap(tmp, sp);
    }
  }
  launch_ntt_inv(c, acc.get(), rows1, nl);
  std::vector<double> h((size_t)nl * N);
  COPSE_HIP(hipMemcpyAsync(h.data(), acc.get(), h.size() * 8, hipMemcpyDeviceToHost, c.stream));
  COPSE_HIP(hipStreamSynchronize(c.stream));
  out.resize(h.size());
  for (size_t i = 0; i < h.size(); ++i) out[i] = (uint64_t)h[i];
}

void to_coef_u64(Context& c, const Ct& a, std::vector<uint64_t>& out) {
  const size_t N = c.N;
  const int nl = a.level + 1;
  DBuf tmp(&c, a.words());
  COPSE_HIP(hipMemcpyAsync(tmp.get(), a.data(), a.words() * 8, hipMemcpyDeviceToDevice, c.stream));
  launch_ntt_inv(c, tmp.get(), ct_rows(c, a.npolys, nl), a.npolys * nl);
  std::vector<double> h(a.words());
  COPSE_HIP(hipMemcpyAsync(h.data(), tmp.get(), h.size() * 8, hipMemcpyDeviceToHost, c.stream));
  COPSE_HIP(hipStreamSynchronize(c.stream));
  out.resize(h.size());
  for (size_t i = 0; i < h.size(); ++i) out[i] = (uint64_t)h[i];
  (void)N;
}

CtPtr from_coef_u64(Context& c, const uint64_t* data, int level, int npolys) {
  const size_t N = c.N;
  const int nl = level + 1;
  auto ct = ct_alloc(c, level, npolys);
  std::vector<double> h((size_t)npolys * nl * N);
  for (int k = 0; k < npolys; ++k)
    for (int i = 0; i < nl; ++i)
      for (size_t j = 0; j < N; ++j) {
        uint64_t v = data[((size_t)k * nl + i) * N + j];
        if (v >= c.primes[i]) fail(COPSE_EINVAL, "residue out of range in import");
        h[((size_t)k * nl + i) * N + j] = (double)v;
      }
  COPSE_HIP(hipMemcpyAsync(ct->data(), h.data(), h.size() * 8, hipMemcpyHostToDevice, c.stream));
  launch_ntt_fwd(c, ct->data(), ct_rows(c, npolys, nl), npolys * nl);
  COPSE_HIP(hipStreamSynchronize(c.stream));
  return ct;
}

// ------------------------------------------------------------------ exact operations
static void check_same(const Ct& a, const Ct& b) {
  if (a.level != b.level) fail(COPSE_EINVAL, "operand levels differ");
}

CtPtr op_modswitch_to(Context& c, const Ct& a, int level) {
  if (level > a.level) fail(COPSE_EINVAL, "cannot raise a ciphertext's level");
  CtPtr cur;
  const Ct* src = &a;
  while (src->level > level) {
    cur = op_modswitch(c, *src);
    src = cur.get();
  }
  if (!cur) cur = ct_copy(c, a);
  return cur;
}

// binary op with level equalization: the higher operand is switched down first
template <typename F>
static CtPtr equalized(Context& c, const Ct& a, const Ct& b, F f) {
  if (a.level == b.level) return f(a, b);
  if (a.level > b.level) {
    auto a2 = op_modswitch_to(c, a, b.level);
    return f(*a2, b);
  }
  auto b2 = op_modswitch_to(c, b, a.level);
  return f(a, *b2);
}

CtPtr op_add(Context& c, const Ct& a, const Ct& b) {
  return equalized(c, a, b, [&](const Ct& x, const Ct& y) {
    int np = std::max(x.npolys, y.npolys), nl = x.level + 1;
    auto o = ct_alloc(c, x.level, np);
    int common = std::min(x.npolys, y.npolys);
    launch_add(c, o->data(), x.data(), y.data(), ct_rows(c, common, nl), common * nl);
    const Ct& longer = x.npolys > y.npolys ? x : y;
    for (int k = common; k < np; ++k)
      COPSE_HIP(hipMemcpyAsync(o->poly(k, c.N), longer.poly(k, c.N), (size_t)nl * c.N * 8,
                               hipMemcpyDeviceToDevice, c.stream));
    return o;
  });
}

CtPtr op_neg(Context& c, const Ct& a) {
  auto o = ct_alloc(c, a.level, a.npolys);
  launch_neg(c, o->data(), a.data(), ct_rows(c, a.npolys, a.level + 1), a.npolys * (a.level + 1));
  return o;
}

CtPtr op_sub(Context& c, const Ct& a, const Ct& b) {
  auto nb = op_neg(c, b);
  return op_add(c, a, *nb);
}

CtPtr op_mul_int(Context& c, const Ct& a, uint64_t k) {
  const int nl = a.level + 1;
  std::vector<double> sc(c.n_primes());
  for (int i = 0; i < c.n_primes(); ++i) sc[i] = (double)(k % c.primes[i]);
  DBuf ds(&c, sc.size());
  COPSE_HIP(hipMemcpyAsync(ds.get(), sc.data(), sc.size() * 8, hipMemcpyHostToDevice, c.stream));
  auto o = ct_alloc(c, a.level, a.npolys);
  launch_mul_scalar(c, o->data(), a.data(), ds.get(), ct_rows(c, a.npolys, nl), a.npolys * nl);
  COPSE_HIP(hipStreamSynchronize(c.stream));
  return o;
}

CtPtr op_add_plain(Context& c, const Ct& a, const Plain& p) {
  if (p.level < a.level) fail(COPSE_EINVAL, "plaintext encoded below the ciphertext level");
  auto o = ct_copy(c, a);
  const int nl = a.level + 1;
  launch_add(c, o->poly(0, c.N), a.poly(0, c.N), p.buf.get(), ct_rows(c, 1, nl), nl);
  return o;
}

CtPtr op_add_const(Context& c, const Ct& a, uint64_t v) {
  // the constant polynomial v: every evaluation equals v
  auto o = ct_copy(c, a);
  launch_add_const(c, o->poly(0, c.N), a.level + 1, (double)v);
  return o;
}

CtPtr op_mul_plain(Context& c, const Ct& a, const Plain& p) {
  if (p.level < a.level) fail(COPSE_EINVAL, "plaintext encoded below the ciphertext level");
  auto o = ct_alloc(c, a.level, a.npolys);
  launch_mul_plain(c, o->data(), a.data(), p.buf.get(), a.npolys, a.level + 1);
  return o;
}

CtPtr op_tensor(Context& c, const Ct& a, const Ct& b) {
  return equalized(c, a, b, [&](const Ct& x, const Ct& y) {
    if (x.npolys != 2 || y.npolys != 2) fail(COPSE_EINVAL, "tensor needs 2-component ciphertexts");
    auto o = ct_alloc(c, x.level, 3);
    launch_tensor(c, o->data(), x.data(), y.data(), x.level + 1, false);
    return o;
  });
}

// ------------------------------------------------------------------ modulus switch
CtPtr op_modswitch(Context& c, const Ct& a) {
  const int l = a.level;
  if (l == 0) fail(COPSE_ECAPACITY, "modulus chain exhausted");
  const size_t N = c.N;
  KSTables& T = c.kstab(l);
  const int np = a.npolys;
  // coefficient form of the dropped limb of every poly
  DBuf top(&c, (size_t)np * N);
  for (int k = 0; k < np; ++k)
    COPSE_HIP(hipMemcpyAsync(top.get() + (size_t)k * N, a.poly(k, N) + (size_t)l * N, N * 8,
                             hipMemcpyDeviceToDevice, c.stream));
  std::vector<int2> tr;
  for (int k = 0; k < np; ++k) tr.push_back(make_int2(k, l));
  const int2* trows = c.rows("top:" + std::to_string(np) + ":" + std::to_string(l), tr);
  DBuf w(&c, (size_t)np * l * N);
  if (bridge_supported(c, 1)) {
    std::vector<int2> ir{make_int2(0, l)}, orr;
    for (int i = 0; i < l; ++i) orr.push_back(make_int2(i, i));
    launch_ntt_inv_rows(c, top.get(), trows, np);
    launch_bridge(c, 1, w.get(), c.rows("msout:" + std::to_string(l), orr), l, top.get(),
                  c.rows("msin:" + std::to_string(l), ir), 1, T.d_ms + 1, nullptr, np, N, (size_t)l * N);
    launch_ntt_fwd_rows(c, w.get(), ct_rows(c, np, l), np * l);
  } else {
    launch_ntt_inv(c, top.get(), trows, np);
    launch_ms_prep(c, w.get(), top.get(), np, l, T.d_ms);
    launch_ntt_fwd(c, w.get(), ct_rows(c, np, l), np * l);
  }
  auto o = ct_alloc(c, l - 1, np);
  launch_ms_finish(c, o->data(), a.data(), w.get(), np, l, T.d_ms);
  return o;
}

// ------------------------------------------------------------------ key switching
// ModUp of one NTT-form poly at `level`: D digits, each extended to P Q_l, NTT form, [D][nE][N].
static DBuf modup(Context& c, const double* d, int level) {
  const size_t N = c.N;
  const int nl = level + 1, nE = nl + c.alpha, D = c.n_digits(level);
  KSTables& T = c.kstab(level);
  DBuf coef(&c, (size_t)nl * N);
  COPSE_HIP(hipMemcpyAsync(coef.get(), d, (size_t)nl * N * 8, hipMemcpyDeviceToDevice, c.stream));
  const bool fused = bridge_supported(c, c.alpha);
  if (fused) launch_ntt_inv_rows(c, coef.get(), ct_rows(c, 1, nl), nl);
  else launch_ntt_inv(c, coef.get(), ct_rows(c, 1, nl), nl);
  DBuf ext(&c, (size_t)D * nE * N);
  std::vector<int2> nttrows;
  for (int j = 0; j < D; ++j) {
    auto& dg = T.digits[j];
    if (fused)
      launch_bridge(c, 0, ext.get(), dg.d_out_rows, (int)dg.targets.size(), coef.get(), dg.d_in_rows, dg.count,
                    dg.d_mult, dg.d_mat, 1, 0, 0);
    else
      launch_bconv(c, ext.get(), dg.d_out_rows, (int)dg.targets.size(), coef.get(), dg.d_in_rows, dg.count,
                   dg.d_mult, dg.d_mat, 1, 0, 0);
    COPSE_HIP(hipMemcpyAsync(ext.get() + ((size_t)j * nE + dg.first) * N, d + (size_t)dg.first * N,
                             (size_t)dg.count * N * 8, hipMemcpyDeviceToDevice, c.stream));
    for (int o : dg.targets) nttrows.push_back(make_int2(j * nE + o, o < nl ? o : c.L + 1 + (o - nl)));
  }
  const int2* nr = c.rows("modup:" + std::to_string(level), nttrows);
  if (fused) launch_ntt_fwd_rows(c, ext.get(), nr, (int)nttrows.size());
  else launch_ntt_fwd(c, ext.get(), nr, (int)nttrows.size());
  return ext;
}

// ModDown of `count` accumulators acc[k] = [nE][N] (k < count, stride nE*N) into out [count][nl][N].
static void moddown(Context& c, double* acc, int count, int level, double* out, const double* add, size_t adds,
                    int add_mode) {
  const size_t N = c.N;
  const int nl = level + 1, nE = nl + c.alpha;
  KSTables& T = c.kstab(level);
  std::vector<int2> sr;
  for (int k = 0; k < count; ++k)
    for (int r = 0; r < c.alpha; ++r) sr.push_back(make_int2(k * nE + nl + r, c.L + 1 + r));
  const int2* srows = c.rows("mdspec:" + std::to_string(level) + ":" + std::to_string(count), sr);
  const bool fused = bridge_supported(c, c.alpha);
  if (fused) launch_ntt_inv_rows(c, acc, srows, count * c.alpha);
  else launch_ntt_inv(c, acc, srows, count * c.alpha);
  DBuf zh(&c, (size_t)count * nl * N);
  std::vector<int2> inr, outr;
  for (int r = 0; r < c.alpha; ++r) inr.push_back(make_int2(nl + r, c.L + 1 + r));
  for (int i = 0; i < nl; ++i) outr.push_back(make_int2(i, i));
  const int2* in_rows = c.rows("mdin:" + std::to_string(level), inr);
  const int2* out_rows = c.rows("mdout:" + std::to_string(level), outr);
  if (fused) {
    launch_bridge(c, 0, zh.get(), out_rows, nl, acc, in_rows, c.alpha, T.d_md_mult, T.d_md_mat, count,
                  (size_t)nE * N, (size_t)nl * N);
    launch_ntt_fwd_rows(c, zh.get(), ct_rows(c, count, nl), count * nl);
  } else {
    launch_bconv(c, zh.get(), out_rows, nl, acc, in_rows, c.alpha, T.d_md_mult, T.d_md_mat, count, (size_t)nE * N,
                 (size_t)nl * N);
    launch_ntt_fwd(c, zh.get(), ct_rows(c, count, nl), count * nl);
  }
  launch_moddown_finish(c, out, acc, (size_t)nE * N, zh.get(), count, nl, T.d_md_pinv, T.d_md_tpinv, add, adds,
                        add_mode);
}

CtPtr op_relin(Context& c, const Keys& k, const Ct& a) {
  if (a.npolys != 3) fail(COPSE_EINVAL, "relinearization needs a 3-component ciphertext");
  if (!k.relin) fail(COPSE_EKEY, "relinearization key absent");
  const size_t N = c.N;
  const int l = a.level, nl = l + 1, nE = nl + c.alpha, D = c.n_digits(l);
  const int Lt = c.n_primes();
  DBuf ext = modup(c, a.poly(2, N), l);
  DBuf acc(&c, (size_t)2 * nE * N);
  KsJob job{ext.get(), k.relin->b.get(), k.relin->a.get(), acc.get(), 1};
  launch_ks_inner(c, &job, 1, D, nE, l, (size_t)Lt * N);
  auto o = ct_alloc(c, l, 2);
  moddown(c, acc.get(), 2, l, o->data(), a.data(), (size_t)nl * N, 1);
  return o;
}

CtPtr op_mul(Context& c, const Keys& k, const Ct& a, const Ct& b) {
  auto t3 = op_tensor(c, a, b);
  auto r = op_relin(c, k, *t3);
  return op_modswitch(c, *r);
}

std::vector<CtPtr> op_rotate_hoisted(Context& c, const Keys& k, const Ct& a, const std::vector<int32_t>& rs) {
  if (a.npolys != 2) fail(COPSE_EINVAL, "rotation needs a 2-component ciphertext");
  const size_t N = c.N;
  const int l = a.level, nl = l + 1, nE = nl + c.alpha, D = c.n_digits(l);
  const int Lt = c.n_primes();
  std::vector<CtPtr> out(rs.size());
  std::vector<size_t> todo;
  for (size_t i = 0; i < rs.size(); ++i) {
    uint64_t g = galois_of(c, rs[i]);
    if (g == 1) out[i] = ct_copy(c, a);
    else {
      if (!k.rot.count(g)) fail(COPSE_EKEY, "rotation key for offset " + std::to_string(rs[i]) + " absent");
      todo.push_back(i);
    }
  }
  if (todo.empty()) return out;
  DBuf ext = modup(c, a.poly(1, N), l);
  const size_t chunk = 16;
  for (size_t first = 0; first < todo.size(); first += chunk) {
    size_t cnt = std::min(chunk, todo.size() - first);
    DBuf acc(&c, cnt * 2 * nE * N);
    DBuf c0r(&c, cnt * nl * N);
    std::vector<KsJob> jobs;
    for (size_t u = 0; u < cnt; ++u) {
      uint64_t g = galois_of(c, rs[todo[first + u]]);
      const auto& key = *k.rot.at(g);
      jobs.push_back(KsJob{ext.get(), key.b.get(), key.a.get(), acc.get() + u * 2 * nE * N, g});
      launch_automorphism(c, c0r.get() + u * nl * N, a.poly(0, N), g, nl, 1);
    }
    launch_ks_inner(c, jobs.data(), (int)cnt, D, nE, l, (size_t)Lt * N);
    DBuf res(&c, cnt * 2 * nl * N);
    moddown(c, acc.get(), (int)(2 * cnt), l, res.get(), c0r.get(), (size_t)nl * N, 2);
    for (size_t u = 0; u < cnt; ++u) {
      auto o = ct_alloc(c, l, 2);
      COPSE_HIP(hipMemcpyAsync(o->data(), res.get() + u * 2 * nl * N, 2 * (size_t)nl * N * 8,
                               hipMemcpyDeviceToDevice, c.stream));
      out[todo[first + u]] = std::move(o);
    }
  }
  return out;
}

CtPtr op_rotate(Context& c, const Keys& k, const Ct& a, int32_t r) {
  auto v = op_rotate_hoisted(c, k, a, {r});
  return std::move(v[0]);
}

// sum_u rot(x_u, r_u) with one ModDown: the rotated terms' key-switch inner products are added in the
// extended basis and brought down once; sigma(c0) parts and unrotated terms are added in Q_l
CtPtr op_rotate_sum(Context& c, const Keys& k, const std::vector<std::pair<const Ct*, int32_t>>& items) {
  if (items.empty()) fail(COPSE_EINVAL, "empty rotation sum");
  const size_t N = c.N;
  const int l = items[0].first->level, nl = l + 1, nE = nl + c.alpha, D = c.n_digits(l);
  const int Lt = c.n_primes();
  for (auto& it : items)
    if (it.first->level != l || it.first->npolys != 2) fail(COPSE_EINVAL, "rotation sum terms must share one level");
  std::vector<int2> er;
  for (int kk = 0; kk < 2; ++kk)
    for (int o = 0; o < nE; ++o) er.push_back(make_int2(kk * nE + o, o < nl ? o : c.L + 1 + (o - nl)));
  const int2* extrows = c.rows("extrows:" + std::to_string(l), er);
  CtPtr unrot;               // sum of the unrotated terms
  DBuf c0s(&c, (size_t)nl * N), acc(&c, (size_t)2 * nE * N), one(&c, (size_t)2 * nE * N);
  bool have = false;
  for (auto& it : items) {
    const Ct& x = *it.first;
    const uint64_t g = galois_of(c, it.second);
    if (g == 1) {
      unrot = unrot ? op_add(c, *unrot, x) : ct_copy(c, x);
      continue;
    }
    auto kit = k.rot.find(g);
    if (kit == k.rot.end()) fail(COPSE_EKEY, "rotation key for offset " + std::to_string(it.second) + " absent");
    DBuf ext = modup(c, x.poly(1, N), l);
    KsJob job{ext.get(), kit->second->b.get(), kit->second->a.get(), have ? one.get() : acc.get(), g};
    launch_ks_inner(c, &job, 1, D, nE, l, (size_t)Lt * N);
    if (have) {
      launch_add(c, acc.get(), acc.get(), one.get(), extrows, 2 * nE);
      DBuf t(&c, (size_t)nl * N);
      launch_automorphism(c, t.get(), x.poly(0, N), g, nl, 1);
      launch_add(c, c0s.get(), c0s.get(), t.get(), ct_rows(c, 1, nl), nl);
    } else {
      launch_automorphism(c, c0s.get(), x.poly(0, N), g, nl, 1);
    }
    have = true;
  }
  if (!have) return unrot;
  auto o = ct_alloc(c, l, 2);
  moddown(c, acc.get(), 2, l, o->data(), c0s.get(), 0, 2);   // the sigma(c0) sum joins poly 0
  if (unrot) return op_add(c, *o, *unrot);
  return o;
}

}  // namespace copse
