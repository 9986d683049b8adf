// Batched evaluation engine: the canonical schedule of Algorithm 1 run on
// many ciphertexts at once.  Every operation below takes a list of
// ciphertexts and issues one launch per step for all of them (per level
// group), so the query groups of a batch, the bit planes of a comparison, the
// products of a prefix-scan round and the baby/giant rotations of a matrix
// product all travel through the same kernels together.  Each output is the
// same deterministic function of its inputs as the one-at-a-time operations,
// so results are bit-identical whatever the batch.
#include <algorithm>
#include <map>
#include <set>

#include "compiled.hpp"

namespace copse {

using SCt = std::shared_ptr<Ct>;

static std::vector<SCt> alloc_batch(Context& c, int count, int level, int npolys) {
  const size_t words = (size_t)npolys * (level + 1) * c.N;
  auto store = std::make_shared<DBuf>(&c, words * count);
  std::vector<SCt> out;
  for (int i = 0; i < count; ++i) {
    auto ct = std::make_shared<Ct>();
    ct->level = level;
    ct->npolys = npolys;
    ct->n = c.N;
    ct->store = store;
    ct->ptr = store->get() + words * i;
    out.push_back(ct);
  }
  return out;
}

static const int2* rows_cached(Context& c, const std::string& key, const std::vector<int2>& h) { return c.rows(key, h); }

static const int2* block_rows(Context& c, int np, int nl) {
  std::string key = "ct:" + std::to_string(np) + ":" + std::to_string(nl);
  auto it = c.row_tables.find(key);
  if (it != c.row_tables.end()) return it->second;
  std::vector<int2> h;
  for (int k = 0; k < np; ++k)
    for (int i = 0; i < nl; ++i) h.push_back(make_int2(k * nl + i, i));
  return c.rows(key, h);
}

// ------------------------------------------------------------------ modulus switch (batched)
// adds (optional, one per input, may be null): added after the switch to the first add_np polys
std::vector<SCt> b_modswitch(Context& c, const std::vector<const Ct*>& in,
                             const std::vector<const double*>* adds = nullptr, int add_np = 0) {
  std::vector<SCt> out(in.size());
  const size_t N = c.N;
  for (const Ct* x : in)
    if (x->level == 0) fail(COPSE_ECAPACITY, "modulus chain exhausted");
  if (bridge_supported(c, 1)) {
    // one set of launches per level and polynomial count (the kernels also take mixed levels, which
    // measured no faster: the small switches are latency-bound either way)
    std::map<std::pair<int, int>, std::vector<size_t>> by_np;
    for (size_t i = 0; i < in.size(); ++i) by_np[{-in[i]->level, in[i]->npolys}].push_back(i);
    for (auto& kv : by_np) {
      const int np = kv.first.second;
      std::vector<size_t> idx = kv.second;
      const int J = (int)idx.size();
      size_t wrows = 0;
      for (size_t j : idx) wrows += (size_t)np * in[j]->level;
      DBuf top(&c, (size_t)J * np * N);
      DBuf w(&c, wrows * N);
      std::vector<double*> po;
      std::vector<const double*> pi, pa, pw, tabs;
      std::vector<int> lv;
      std::vector<BridgeDesc> ds;
      size_t woff = 0;
      for (int j0 = 0; j0 < J;) {
        const int l = in[idx[j0]]->level;
        int j1 = j0;
        while (j1 < J && in[idx[j1]]->level == l) ++j1;
        KSTables& T = c.kstab(l);
        auto outs = alloc_batch(c, j1 - j0, l - 1, np);
        std::vector<int2> ir{make_int2(0, l)}, orr;
        for (int i = 0; i < l; ++i) orr.push_back(make_int2(i, i));
        BridgeDesc d{rows_cached(c, "msout:" + std::to_string(l), orr), rows_cached(c, "msin:" + std::to_string(l), ir),
                     T.d_ms + 1, nullptr, l, 1, 0, 0};
        d.in = top.get() + (size_t)j0 * np * N;
        d.out = w.get() + woff * N;
        d.in_bs = N;
        d.out_bs = (size_t)l * N;
        d.nz = (j1 - j0) * np;
        ds.push_back(d);
        for (int j = j0; j < j1; ++j) {
          const size_t g = idx[j];
          po.push_back(outs[j - j0]->data());
          pi.push_back(in[g]->data());
          if (adds) pa.push_back((*adds)[g]);
          pw.push_back(w.get() + woff * N);
          tabs.push_back(T.d_ms);
          lv.push_back(l);
          out[g] = outs[j - j0];
          woff += (size_t)np * l;
        }
        j0 = j1;
      }
      // top rows read in place by the inverse row pass; the forward row pass ends the switch
      launch_ntt_inv_rows_gather(c, top.get(), pi, np, 0, 0, -2, &lv);
      launch_bridge_set(c, 1, nullptr, nullptr, ds, 0, 0, 0);
      launch_ntt_fwd_rows_ms_finish(c, po, pi, pw, lv, tabs, np, adds ? &pa : nullptr, add_np);
    }
    return out;
  }
  std::map<std::pair<int, int>, std::vector<size_t>> groups;
  for (size_t i = 0; i < in.size(); ++i) groups[{in[i]->level, in[i]->npolys}].push_back(i);
  for (auto& kv : groups) {
    const int l = kv.first.first, np = kv.first.second;
    const auto& idx = kv.second;
    const int J = (int)idx.size();
    KSTables& T = c.kstab(l);
    DBuf top(&c, (size_t)J * np * N);
    DBuf w(&c, (size_t)J * np * l * N);
    auto outs = alloc_batch(c, J, l - 1, np);
    std::vector<double*> po;
    std::vector<const double*> pi, pa;
    for (int j = 0; j < J; ++j) {
      po.push_back(outs[j]->data());
      pi.push_back(in[idx[j]]->data());
      if (adds) pa.push_back((*adds)[idx[j]]);
      out[idx[j]] = outs[j];
    }
    std::vector<const double*> src;
    for (size_t j : idx)
      for (int k = 0; k < np; ++k) src.push_back(in[j]->poly(k, N) + (size_t)l * N);
    launch_gather(c, top.get(), src, 1);
    std::vector<int2> tr;
    for (int z = 0; z < J * np; ++z) tr.push_back(make_int2(z, l));
    const int2* trows = rows_cached(c, "top:" + std::to_string(J * np) + ":" + std::to_string(l), tr);
    launch_ntt_inv(c, top.get(), trows, J * np);
    launch_ms_prep(c, w.get(), top.get(), J * np, l, T.d_ms);
    launch_ntt_fwd(c, w.get(), block_rows(c, J * np, l), J * np * l);
    launch_ms_finish_multi(c, po, pi, w.get(), np, l, T.d_ms, adds ? &pa : nullptr, add_np);
  }
  return out;
}

// switch in[i] down by k[i] primes at once (1 <= k[i] <= 4): bit-identical to k[i] single switches.  Per
// polynomial count: one inverse row pass over the dropped limbs of every job, fused column passes per
// (level, k) (mode 3: the single switches' lifts one after the other), one forward row pass with the finish.
static std::vector<SCt> b_switch_by(Context& c, const std::vector<const Ct*>& in, const std::vector<int>& kk) {
  std::vector<SCt> out(in.size());
  const size_t N = c.N;
  std::map<int, std::vector<size_t>> by_np;
  for (size_t i = 0; i < in.size(); ++i) {
    if (kk[i] < 1 || kk[i] > 4 || kk[i] > in[i]->level) fail(COPSE_EINVAL, "internal: switch count");
    by_np[in[i]->npolys].push_back(i);
  }
  for (auto& kv : by_np) {
    const int np = kv.first;
    std::vector<size_t> idx = kv.second;
    // jobs of one (level, k) next to each other
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
      return std::make_pair(-in[a]->level, kk[a]) < std::make_pair(-in[b]->level, kk[b]);
    });
    const int J = (int)idx.size();
    int kmax = 0;
    size_t wrows = 0;
    for (size_t j : idx) {
      kmax = std::max(kmax, kk[j]);
      wrows += (size_t)np * (in[j]->level - kk[j] + 1);
    }
    const int rpj = np * kmax;
    DBuf top(&c, (size_t)J * rpj * N);
    DBuf w(&c, wrows * N);
    std::vector<double*> po;
    std::vector<const double*> pi, pw, tabs;
    std::vector<int> glv, flv;
    std::vector<BridgeDesc> ds;
    size_t woff = 0;
    for (int j0 = 0; j0 < J;) {
      const int l = in[idx[j0]]->level, k = kk[idx[j0]];
      int j1 = j0;
      while (j1 < J && in[idx[j1]]->level == l && kk[idx[j1]] == k) ++j1;
      const MsMulti& M = c.ms_multi(l, k);
      const int n_out = l - k + 1;
      auto outs = alloc_batch(c, j1 - j0, l - k, np);
      BridgeDesc d{M.out_rows, M.in_rows, M.mult, M.mat, n_out, k, 0, 0};
      d.in = top.get() + (size_t)j0 * rpj * N;
      d.out = w.get() + woff * N;
      d.in_bs = (size_t)kmax * N;
      d.out_bs = (size_t)n_out * N;
      d.nz = (j1 - j0) * np;
      ds.push_back(d);
      for (int j = j0; j < j1; ++j) {
        const size_t g = idx[j];
        po.push_back(outs[j - j0]->data());
        pi.push_back(in[g]->data());
        pw.push_back(w.get() + woff * N);
        tabs.push_back(M.tab);
        glv.push_back(l | (k << 16));
        flv.push_back(n_out | ((l + 1) << 16));
        out[g] = outs[j - j0];
        woff += (size_t)np * n_out;
      }
      j0 = j1;
    }
    launch_ntt_inv_rows_gather(c, top.get(), pi, rpj, (size_t)kmax, 0, -3, &glv);
    launch_bridge_set(c, 3, nullptr, nullptr, ds, 0, 0, 0);
    launch_ntt_fwd_rows_ms_finish(c, po, pi, pw, flv, tabs, np, nullptr, 0);
  }
  return out;
}

// the plaintext layer out_j = (x_j * mul_j + add_j on polynomial 0, x_j * mul_j on polynomial 1) at level l,
// switched to l - 1, without writing the layer: the switch's inverse row pass and finish compute it
static std::vector<SCt> b_ptlayer_switch(Context& c, const std::vector<const double*>& x,
                                         const std::vector<const double*>& mul, const std::vector<const double*>& add,
                                         int l) {
  const size_t N = c.N;
  const int J = (int)x.size(), np = 2;
  KSTables& T = c.kstab(l);
  auto outs = alloc_batch(c, J, l - 1, np);
  DBuf top(&c, (size_t)J * np * N);
  DBuf w(&c, (size_t)J * np * l * N);
  std::vector<double*> po;
  std::vector<const double*> pw, tabs;
  std::vector<int> lv(J, l);
  for (int j = 0; j < J; ++j) {
    po.push_back(outs[j]->data());
    pw.push_back(w.get() + (size_t)j * np * l * N);
    tabs.push_back(T.d_ms);
  }
  std::vector<int2> ir{make_int2(0, l)}, orr;
  for (int i = 0; i < l; ++i) orr.push_back(make_int2(i, i));
  BridgeDesc d{rows_cached(c, "msout:" + std::to_string(l), orr), rows_cached(c, "msin:" + std::to_string(l), ir),
               T.d_ms + 1, nullptr, l, 1, 0, 0};
  d.in = top.get();
  d.out = w.get();
  d.in_bs = N;
  d.out_bs = (size_t)l * N;
  d.nz = J * np;
  launch_ntt_inv_rows_gather(c, top.get(), x, np, 0, 0, -4, &lv, &mul, &add);
  launch_bridge_set(c, 1, nullptr, nullptr, {d}, 0, 0, 0);
  launch_ntt_fwd_rows_ms_finish(c, po, x, pw, lv, tabs, np, &add, 0, &mul);
  return outs;
}

// switch each ciphertext down to its target level (several primes per step where the fused passes run)
static std::vector<SCt> b_down(Context& c, std::vector<SCt> v, const std::vector<int>& target) {
  if (bridge_supported(c, 4)) {
    while (true) {
      std::vector<size_t> todo;
      std::vector<int> kk;
      for (size_t i = 0; i < v.size(); ++i)
        if (v[i]->level > target[i]) {
          todo.push_back(i);
          kk.push_back(std::min(4, v[i]->level - target[i]));
        }
      if (todo.empty()) return v;
      std::vector<const Ct*> in;
      for (size_t i : todo) in.push_back(v[i].get());
      bool single = true;
      for (int k : kk) single = single && k == 1;
      // switches by one prime keep the single-switch path (its own lift kernel)
      auto r = single ? b_modswitch(c, in) : b_switch_by(c, in, kk);
      for (size_t k = 0; k < todo.size(); ++k) v[todo[k]] = r[k];
    }
  }
  while (true) {
    std::vector<size_t> todo;
    for (size_t i = 0; i < v.size(); ++i)
      if (v[i]->level > target[i]) todo.push_back(i);
    if (todo.empty()) return v;
    std::vector<const Ct*> in;
    for (size_t i : todo) in.push_back(v[i].get());
    auto r = b_modswitch(c, in);
    for (size_t k = 0; k < todo.size(); ++k) v[todo[k]] = r[k];
  }
}

// ------------------------------------------------------------------ key switching (batched)
// ModUp of every input (NTT form, `level`): coefficient form, base conversion per digit, transform of the
// new rows; out [I][D][nE][N] (the digits' own limbs are not copied: readers take them from the input)
// row_pass false (fused path only): the new rows are left after the column stages, for a consumer that
// runs the forward row pass itself (launch_ks_inner_rows)
// inputs_b (optional): input i is the product inputs[i] (.) inputs_b[i] (a product's third polynomial,
// not written)
static DBuf modup_batch(Context& c, int level, const std::vector<const double*>& inputs, bool row_pass = true,
                        const std::vector<const double*>* inputs_b = nullptr) {
  const size_t N = c.N;
  const int nl = level + 1, nE = nl + c.alpha, D = c.n_digits(level);
  const int I = (int)inputs.size();
  KSTables& T = c.kstab(level);
  DBuf cf(&c, (size_t)I * nl * N);
  DBuf ext(&c, (size_t)I * D * nE * N);
  const bool fused = bridge_supported(c, c.alpha);
  if (inputs_b && !fused) fail(COPSE_EINVAL, "internal: product inputs need the fused column pass");
  if (!fused) launch_gather(c, cf.get(), inputs, nl);
  if (fused) {
    // inverse row pass read straight from the inputs, then per digit the fused column passes with the
    // base conversion, then the forward row pass of every new row
    launch_ntt_inv_rows_gather(c, cf.get(), inputs, nl, N, 0, -1, nullptr, inputs_b);
    // all digits in one launch (up to four per launch)
    std::vector<BridgeDesc> ds;
    for (int j = 0; j < D; ++j) {
      auto& dg = T.digits[j];
      ds.push_back(BridgeDesc{dg.d_out_rows, dg.d_in_rows, dg.d_mult, dg.d_mat, (int)dg.targets.size(), dg.count, 0, 0});
      if ((int)ds.size() == BridgeSet::kMax || j == D - 1) {
        launch_bridge_set(c, 0, ext.get(), cf.get(), ds, I, (size_t)nl * N, (size_t)D * nE * N);
        ds.clear();
      }
    }
  } else {
    launch_ntt_inv(c, cf.get(), block_rows(c, I, nl), I * nl);
    for (int j = 0; j < D; ++j) {
      auto& dg = T.digits[j];
      launch_bconv(c, ext.get(), dg.d_out_rows, (int)dg.targets.size(), cf.get(), dg.d_in_rows, dg.count, dg.d_mult,
                   dg.d_mat, I, (size_t)nl * N, (size_t)D * nE * N);
    }
  }
  if (fused && !row_pass) return ext;
  {
    std::string key = "ksntt:" + std::to_string(level) + ":" + std::to_string(I);
    auto it = c.row_tables.find(key);
    const int2* r;
    int cnt = 0;
    for (int j = 0; j < D; ++j) cnt += (int)T.digits[j].targets.size();
    cnt *= I;
    if (it != c.row_tables.end()) {
      r = it->second;
    } else {
      std::vector<int2> h;
      for (int i = 0; i < I; ++i)
        for (int j = 0; j < D; ++j)
          for (int o : T.digits[j].targets) h.push_back(make_int2((i * D + j) * nE + o, o < nl ? o : c.L + 1 + (o - nl)));
      r = c.rows(key, h);
    }
    if (fused) launch_ntt_fwd_rows(c, ext.get(), r, cnt);
    else launch_ntt_fwd(c, ext.get(), r, cnt);
  }
  return ext;
}

struct KsReq {
  int input;
  const Keys::KSK* key;
  uint64_t g;
  double* out;          // 2 polys at the level
  const double* add;    // mode 1: (d0, d1) to add; mode 2: c0 to permute and add
  const double* add_b = nullptr;   // merged mode 1 only: (d0, d1) is the product of the ciphertexts add and add_b
};

// merge (add_mode 1 only): the ModDown also switches to level - 1, as a relinearization followed by a
// modulus switch would; each request's out then holds 2 polys of `level` limbs
// inputs_b (merge only): a product's relinearization with its tensor not written: input i is
// inputs[i] (.) inputs_b[i] (a1 b1), and each request's addend is the product of add and add_b
static void ks_batch(Context& c, int level, const std::vector<const double*>& inputs, const std::vector<KsReq>& reqs,
                     int add_mode, bool merge = false, const std::vector<const double*>* inputs_b = nullptr) {
  if (reqs.empty()) return;
  const size_t N = c.N;
  const int nl = level + 1, nE = nl + c.alpha, D = c.n_digits(level);
  const int R = (int)reqs.size();
  const int Lt = c.n_primes();
  KSTables& T = c.kstab(level);
  const bool fused = bridge_supported(c, c.alpha);
  if (merge && !(fused && add_mode == 1 && level >= 1 && T.mm_ok))
    fail(COPSE_EINVAL, "internal: merged switch not available here");
  if (inputs_b && (!merge || inputs_b->size() != inputs.size()))
    fail(COPSE_EINVAL, "internal: product inputs only for the merged relinearization");
  // relinearizations (no automorphism) fold the ModUp's forward row pass and the ModDown's inverse row
  // pass into the inner products (two launches fewer, the extended rows never written in NTT form)
  bool no_auto = fused;
  for (const KsReq& rq : reqs) no_auto = no_auto && rq.g == 1;
  DBuf ext = modup_batch(c, level, inputs, !no_auto, inputs_b);
  // inner products
  DBuf acc(&c, (size_t)R * 2 * nE * N);
  std::vector<KsJob2> jobs;
  for (int q = 0; q < R; ++q) {
    const KsReq& rq = reqs[q];
    jobs.push_back(KsJob2{inputs[rq.input], ext.get() + (size_t)rq.input * D * nE * N, rq.key->b.get(),
                          rq.key->a.get(), acc.get() + (size_t)q * 2 * nE * N, rq.g, merge ? rq.add : nullptr,
                          inputs_b ? (*inputs_b)[rq.input] : nullptr, inputs_b ? rq.add_b : nullptr});
  }
  // the fused inner product also runs the ModDown's inverse row pass on the rows that need it
  if (no_auto) launch_ks_inner_rows(c, jobs, D, nE, level, (size_t)Lt * N, merge ? T.mm_ptop : 0.0, merge ? nl - 1 : nl);
  else launch_ks_inner2(c, jobs, D, nE, level, (size_t)Lt * N, merge ? T.mm_ptop : 0.0);
  if (merge) {
    // ModDown by P and switch by q_l in one pass: the top data row (now y_l + P a_l) joins the special rows
    // in the inverse transform, the fused column pass lifts the switched top limb, and the finish writes
    // the result at level - 1
    const int l = level;
    const int2* r = rows_cached(c, "mdmsrows:" + std::to_string(level) + ":" + std::to_string(2 * R), [&] {
      std::vector<int2> h;
      for (int k = 0; k < 2 * R; ++k) {
        for (int s2 = 0; s2 < c.alpha; ++s2) h.push_back(make_int2(k * nE + nl + s2, c.L + 1 + s2));
        h.push_back(make_int2(k * nE + l, l));
      }
      return h;
    }());
    if (!no_auto) launch_ntt_inv_rows(c, acc.get(), r, 2 * R * (c.alpha + 1));
    std::vector<int2> inr, outr;
    for (int s2 = 0; s2 < c.alpha; ++s2) inr.push_back(make_int2(nl + s2, c.L + 1 + s2));
    inr.push_back(make_int2(l, l));
    for (int i = 0; i < l; ++i) outr.push_back(make_int2(i, i));
    DBuf w(&c, (size_t)2 * R * l * N);
    launch_bridge(c, 2, w.get(), rows_cached(c, "mdmsout:" + std::to_string(level), outr), l, acc.get(),
                  rows_cached(c, "mdmsin:" + std::to_string(level), inr), c.alpha + 1, T.d_mm_mult, T.d_mm_mat,
                  2 * R, (size_t)nE * N, (size_t)l * N);
    std::vector<double*> outs;
    std::vector<const double*> adds, adds_b;
    for (auto& rq : reqs) {
      outs.push_back(rq.out);
      adds.push_back(rq.add);
      adds_b.push_back(rq.add_b);
    }
    launch_ntt_fwd_rows_mdms_finish(c, outs, adds, acc.get(), w.get(), nE, l, T.d_mm_m1, T.d_mm_m2, T.d_mm_m3,
                                    nullptr, 0, inputs_b ? &adds_b : nullptr);
    return;
  }
  // ModDown of all accumulators
  {
    std::string key = "mdspec:" + std::to_string(level) + ":" + std::to_string(2 * R);
    auto it = c.row_tables.find(key);
    const int2* r;
    if (it != c.row_tables.end()) {
      r = it->second;
    } else {
      std::vector<int2> h;
      for (int k = 0; k < 2 * R; ++k)
        for (int s = 0; s < c.alpha; ++s) h.push_back(make_int2(k * nE + nl + s, c.L + 1 + s));
      r = c.rows(key, h);
    }
    if (no_auto) {
      // done by the fused inner product
    } else if (fused) {
      launch_ntt_inv_rows(c, acc.get(), r, 2 * R * c.alpha);
    } else {
      launch_ntt_inv(c, acc.get(), r, 2 * R * c.alpha);
    }
  }
  DBuf zh(&c, (size_t)2 * R * nl * N);
  std::vector<int2> inr, outr;
  for (int s = 0; s < c.alpha; ++s) inr.push_back(make_int2(nl + s, c.L + 1 + s));
  for (int i = 0; i < nl; ++i) outr.push_back(make_int2(i, i));
  std::vector<double*> outs;
  std::vector<const double*> adds;
  std::vector<uint64_t> gal;
  for (auto& rq : reqs) {
    outs.push_back(rq.out);
    adds.push_back(rq.add);
    gal.push_back(rq.g);
  }
  if (fused) {
    launch_bridge(c, 0, zh.get(), rows_cached(c, "mdout:" + std::to_string(level), outr), nl, acc.get(),
                  rows_cached(c, "mdin:" + std::to_string(level), inr), c.alpha, T.d_md_mult, T.d_md_mat, 2 * R,
                  (size_t)nE * N, (size_t)nl * N);
    launch_ntt_fwd_rows_md_finish(c, outs, adds, gal, acc.get(), zh.get(), nE, nl, T.d_md_pinv, T.d_md_tpinv,
                                  add_mode);
    return;
  } else {
    launch_bconv(c, zh.get(), rows_cached(c, "mdout:" + std::to_string(level), outr), nl, acc.get(),
                 rows_cached(c, "mdin:" + std::to_string(level), inr), c.alpha, T.d_md_mult, T.d_md_mat, 2 * R,
                 (size_t)nE * N, (size_t)nl * N);
    launch_ntt_fwd(c, zh.get(), block_rows(c, 2 * R, nl), 2 * R * nl);
  }
  launch_md_finish2(c, outs, adds, gal, acc.get(), zh.get(), nE, nl, T.d_md_pinv, T.d_md_tpinv, add_mode);
}

// relinearize 3-component ciphertexts (any mix of levels)
static std::vector<SCt> b_relin(Context& c, const Keys& k, const std::vector<const Ct*>& in3) {
  if (!k.relin) fail(COPSE_EKEY, "relinearization key absent");
  std::vector<SCt> out(in3.size());
  std::map<int, std::vector<size_t>> groups;
  for (size_t i = 0; i < in3.size(); ++i) groups[in3[i]->level].push_back(i);
  for (auto& kv : groups) {
    const int l = kv.first;
    auto outs = alloc_batch(c, (int)kv.second.size(), l, 2);
    std::vector<const double*> inputs;
    std::vector<KsReq> reqs;
    for (size_t q = 0; q < kv.second.size(); ++q) {
      const Ct* x = in3[kv.second[q]];
      inputs.push_back(x->poly(2, c.N));
      reqs.push_back(KsReq{(int)q, k.relin.get(), 1, outs[q]->data(), x->data()});
      out[kv.second[q]] = outs[q];
    }
    ks_batch(c, l, inputs, reqs, 1);
  }
  return out;
}

// whether a product at level l can relinearize and switch in one key switch
static bool merged_switch_ok(Context& c, int l) {
  return l >= 1 && bridge_supported(c, c.alpha) && c.kstab(l).mm_ok;
}

// products of pairs: equalize, tensor, relinearize, switch
std::vector<SCt> b_mul(Context& c, const Keys& k, const std::vector<std::pair<SCt, SCt>>& pairs) {
  std::vector<SCt> ops;
  std::vector<int> tgt;
  for (auto& pr : pairs) {
    int lv = std::min(pr.first->level, pr.second->level);
    ops.push_back(pr.first);
    ops.push_back(pr.second);
    tgt.push_back(lv);
    tgt.push_back(lv);
  }
  ops = b_down(c, ops, tgt);
  std::vector<SCt> out(pairs.size());
  std::map<int, std::vector<size_t>> groups;
  for (size_t i = 0; i < pairs.size(); ++i) groups[tgt[2 * i]].push_back(i);
  for (auto& kv : groups) {
    const int l = kv.first;
    std::vector<const double*> a, b;
    for (size_t q = 0; q < kv.second.size(); ++q) {
      size_t i = kv.second[q];
      if (ops[2 * i]->npolys != 2 || ops[2 * i + 1]->npolys != 2) fail(COPSE_EINVAL, "product of non-linear ciphertexts");
      a.push_back(ops[2 * i]->data());
      b.push_back(ops[2 * i + 1]->data());
    }
    if (merged_switch_ok(c, l)) {
      // relinearization and switch to l - 1 in one key switch, bit-identical to b_modswitch of the
      // relinearized tensor; the tensor (a0 b0, a0 b1 + a1 b0, a1 b1) is never written: the ModUp's
      // inverse row pass and the inner products form a1 b1 from the operands, the finish the other two
      if (!k.relin) fail(COPSE_EKEY, "relinearization key absent");
      auto outs = alloc_batch(c, (int)kv.second.size(), l - 1, 2);
      const size_t ps = (size_t)(l + 1) * c.N;
      std::vector<const double*> in1, in1b;
      std::vector<KsReq> reqs;
      for (size_t q = 0; q < kv.second.size(); ++q) {
        in1.push_back(a[q] + ps);
        in1b.push_back(b[q] + ps);
        KsReq rq{(int)q, k.relin.get(), 1, outs[q]->data(), a[q]};
        rq.add_b = b[q];
        reqs.push_back(rq);
        out[kv.second[q]] = outs[q];
      }
      ks_batch(c, l, in1, reqs, 1, true, &in1b);
      continue;
    }
    auto t3 = alloc_batch(c, (int)kv.second.size(), l, 3);
    std::vector<double*> d;
    for (auto& x : t3) d.push_back(x->data());
    launch_tensor_multi(c, d, a, b, l + 1);
    std::vector<const Ct*> in3;
    for (auto& x : t3) in3.push_back(x.get());
    auto rel = b_relin(c, k, in3);
    std::vector<const Ct*> rin;
    for (auto& x : rel) rin.push_back(x.get());
    auto ms = b_modswitch(c, rin);
    for (size_t q = 0; q < kv.second.size(); ++q) out[kv.second[q]] = ms[q];
  }
  return out;
}

// hoisted rotations of each of v (same level) by every offset in rots, into B[u][b]; returns the slot u of
// the rotation by zero when it is left empty (the inner sums then read v in place), else -1
static int b_rotate_into(Context& c, const Keys& k, const std::vector<const Ct*>& v, const std::vector<int32_t>& rots,
                         double* B) {
  const size_t N = c.N;
  const int l = v[0]->level, nl = l + 1, G = (int)v.size();
  const size_t ps = (size_t)2 * nl * N;
  std::vector<const double*> inputs;
  for (auto* x : v) {
    if (x->level != l || x->npolys != 2) fail(COPSE_EINVAL, "rotation batch must share one level");
    inputs.push_back(x->poly(1, N));
  }
  std::vector<KsReq> reqs;
  int u0 = -1;
  for (size_t u = 0; u < rots.size(); ++u) {
    uint64_t g = galois_of(c, rots[u]);
    if (g == 1 && u0 < 0 && G <= kPack) {
      u0 = (int)u;
      continue;
    }
    for (int b = 0; b < G; ++b) {
      double* dst = B + ((size_t)u * G + b) * ps;
      if (g == 1) {
        launch_copy(c, dst, v[b]->data(), ps);
        continue;
      }
      auto it = k.rot.find(g);
      if (it == k.rot.end()) fail(COPSE_EKEY, "rotation key for offset " + std::to_string(rots[u]) + " absent");
      reqs.push_back(KsReq{b, it->second.get(), g, dst, v[b]->data()});
    }
  }
  ks_batch(c, l, inputs, reqs, 2);
  return u0;
}

// ------------------------------------------------------------------ MatMul (baby-step / giant-step)
// Several products that share one baby-step buffer B[u][b] (the same rotation slots): one launch of the
// inner sums over the giant groups of all of them (tab is their concatenated [u][group] diagonal table),
// one batch of giant rotations, a sum per product and batch element, one switch for all.  adds[i * G + b]
// (optional) is added to the first add_np polys of result (i, b) after the switch.
// u0 / v0: the baby slot of the rotation by zero left empty by b_rotate_into and the unrotated inputs
static std::vector<std::vector<SCt>> b_matmul_many(Context& c, const Keys& k, const std::vector<const MatPlan*>& plans,
                                                   const double* const* tab, int n_u, const double* B, int G,
                                                   int level, int u0, const std::vector<const Ct*>& v0,
                                                   const std::vector<const double*>* adds = nullptr,
                                                   int add_np = 0) {
  const size_t N = c.N;
  const int nl = level + 1;
  const size_t ps2 = (size_t)2 * nl * N, ps3 = (size_t)3 * nl * N;
  const bool enc = plans[0]->enc;
  std::vector<int> off;
  int ngs = 0;
  for (auto* P : plans) {
    if (P->enc != enc || P->n1 != plans[0]->n1) fail(COPSE_EINVAL, "internal: products of one batch differ");
    if (P->groups.empty()) fail(COPSE_EINVAL, "internal: product without a nonzero diagonal");
    off.push_back(ngs);
    ngs += (int)P->groups.size();
  }
  DBuf inner(&c, (size_t)ngs * G * (enc ? ps3 : ps2));
  size_t nnz = 0;
  for (auto* P : plans)
    for (auto* d : P->tab) nnz += d != nullptr;
  std::vector<const double*> b0;
  for (auto* x : v0) b0.push_back(x->data());
  launch_mm_inner(c, inner.get(), B, tab, n_u, ngs, G, nl, (size_t)G * ps2, ps2, enc, nnz, u0, &b0);
  std::vector<SCt> in2;   // encrypted model: per (group, b) relinearized inner sums
  if (enc) {
    std::vector<SCt> t3;
    for (int z = 0; z < ngs * G; ++z) {
      auto ct = std::make_shared<Ct>();
      ct->level = level; ct->npolys = 3; ct->n = N; ct->ptr = inner.get() + (size_t)z * ps3;
      t3.push_back(ct);
    }
    std::vector<const Ct*> in3;
    for (auto& x : t3) in3.push_back(x.get());
    in2 = b_relin(c, k, in3);
  }
  auto ptr2 = [&](int z) -> const double* { return enc ? in2[z]->data() : inner.get() + (size_t)z * ps2; };
  const int np = (int)plans.size();
  std::vector<std::vector<SCt>> out(np, std::vector<SCt>(G));
  // Giant steps: per output (product i, batch element b), sum_s rot(inner_s, g_s n1) with one ModDown of
  // the summed key-switch inner products (BGV rotation sum), then one switch and the mask.
  if (merged_switch_ok(c, level)) {
    // one batched pass: ModUp of every rotated inner sum; the sigma(c0) parts and the unrotated inner sum
    // gathered per output (the addend); the inner products summed per output, with P times the addend's
    // top limb on the top data row; the ModDown merged with the switch, whose finish adds the mask
    KSTables& T = c.kstab(level);
    const int nE = nl + c.alpha, D = c.n_digits(level);
    std::vector<const double*> inputs;
    std::vector<GsumStep> steps;
    std::vector<GsumProd> prods;
    std::vector<AutoTerm> terms;
    std::vector<AutoOut> aouts;
    std::vector<double*> outs;
    std::vector<const double*> addp, maskp;
    DBuf addend(&c, (size_t)np * G * ps2);
    DBuf acc(&c, (size_t)np * G * 2 * nE * N);
    auto res = alloc_batch(c, np * G, level - 1, 2);
    for (int i = 0; i < np; ++i) {
      const MatPlan& P = *plans[i];
      // per output: the sigma(c0) parts and the unrotated inner sum (the addend)
      for (int b = 0; b < G; ++b) {
        const int u = i * G + b;
        AutoOut ao{addend.get() + (size_t)u * ps2, nullptr, nullptr, (int)terms.size(), 0};
        for (size_t s2 = 0; s2 < P.groups.size(); ++s2) {
          const uint32_t g = P.groups[s2];
          const int z = (off[i] + (int)s2) * G + b;
          if (g == 0) {
            ao.f0 = ptr2(z);
            ao.f1 = ptr2(z) + (size_t)nl * N;
            continue;
          }
          terms.push_back(AutoTerm{ptr2(z), galois_of(c, (int64_t)g * P.n1)});
          ++ao.count;
        }
        aouts.push_back(ao);
        outs.push_back(res[u]->data());
        addp.push_back(addend.get() + (size_t)u * ps2);
        maskp.push_back(adds ? (*adds)[u] : nullptr);
        out[i][b] = res[u];
      }
      // per giant step: one key for every batch element; the ModUp inputs in (step, batch element) order, so
      // that element b of a step sits b ModUp outputs after element 0 (the inner sums are ps2 apart)
      GsumProd pd{(int)steps.size(), 0, acc.get() + (size_t)i * G * 2 * nE * N, addend.get() + (size_t)i * G * ps2, 0};
      for (size_t s2 = 0; s2 < P.groups.size(); ++s2) {
        const uint32_t g = P.groups[s2];
        if (g == 0) continue;
        const uint64_t gal = galois_of(c, (int64_t)g * P.n1);
        auto it = k.rot.find(gal);
        if (it == k.rot.end()) fail(COPSE_EKEY, "giant-step key absent");
        const int z0 = (off[i] + (int)s2) * G;
        steps.push_back(GsumStep{gal, it->second->b.get(), it->second->a.get(), ptr2(z0) + (size_t)nl * N, nullptr});
        for (int b = 0; b < G; ++b) inputs.push_back(ptr2(z0 + b) + (size_t)nl * N);
        ++pd.count;
      }
      prods.push_back(pd);
    }
    DBuf ext = inputs.empty() ? DBuf(&c, 1) : modup_batch(c, level, inputs);
    const size_t ext_bs = (size_t)D * nE * N;
    for (size_t t = 0; t < steps.size(); ++t) steps[t].ext = ext.get() + t * G * ext_bs;
    launch_auto_sum(c, terms, aouts, nl);
    launch_ks_inner_gsum(c, steps, prods, G, ps2, ext_bs, (size_t)2 * nE * N, ps2, D, nE, level,
                         (size_t)c.n_primes() * N, T.mm_ptop);
    const int l = level, R = np * G;
    const int2* r = rows_cached(c, "mdmsrows:" + std::to_string(level) + ":" + std::to_string(2 * R), [&] {
      std::vector<int2> h;
      for (int kk = 0; kk < 2 * R; ++kk) {
        for (int s2 = 0; s2 < c.alpha; ++s2) h.push_back(make_int2(kk * nE + nl + s2, c.L + 1 + s2));
        h.push_back(make_int2(kk * nE + l, l));
      }
      return h;
    }());
    launch_ntt_inv_rows(c, acc.get(), r, 2 * R * (c.alpha + 1));
    std::vector<int2> inr, outr;
    for (int s2 = 0; s2 < c.alpha; ++s2) inr.push_back(make_int2(nl + s2, c.L + 1 + s2));
    inr.push_back(make_int2(l, l));
    for (int i = 0; i < l; ++i) outr.push_back(make_int2(i, i));
    DBuf w(&c, (size_t)2 * R * l * N);
    launch_bridge(c, 2, w.get(), rows_cached(c, "mdmsout:" + std::to_string(level), outr), l, acc.get(),
                  rows_cached(c, "mdmsin:" + std::to_string(level), inr), c.alpha + 1, T.d_mm_mult, T.d_mm_mat,
                  2 * R, (size_t)nE * N, (size_t)l * N);
    launch_ntt_fwd_rows_mdms_finish(c, outs, addp, acc.get(), w.get(), nE, l, T.d_mm_m1, T.d_mm_m2, T.d_mm_m3,
                                    adds ? &maskp : nullptr, add_np);
    return out;
  }
  // otherwise (small rings): the rotation sum per output, then one batched switch with the masks
  std::vector<SCt> sums;
  std::vector<std::shared_ptr<Ct>> views;
  for (int i = 0; i < np; ++i) {
    const MatPlan& P = *plans[i];
    for (int b = 0; b < G; ++b) {
      std::vector<std::pair<const Ct*, int32_t>> items;
      for (size_t s2 = 0; s2 < P.groups.size(); ++s2) {
        const int z = (off[i] + (int)s2) * G + b;
        auto v = std::make_shared<Ct>();
        v->level = level; v->npolys = 2; v->n = N; v->ptr = const_cast<double*>(ptr2(z));
        views.push_back(v);
        items.push_back({v.get(), (int32_t)(P.groups[s2] * P.n1)});
      }
      sums.push_back(SCt(op_rotate_sum(c, k, items).release()));
    }
  }
  std::vector<const Ct*> sin;
  for (auto& x : sums) sin.push_back(x.get());
  auto sw = b_modswitch(c, sin, adds, add_np);
  for (int i = 0; i < np; ++i) out[i].assign(sw.begin() + (size_t)i * G, sw.begin() + (size_t)(i + 1) * G);
  return out;
}

// ------------------------------------------------------------------ sums and masks
static std::vector<SCt> b_sum_all(Context& c, const std::vector<std::vector<SCt>>& terms_per_b) {
  // per b: switch every term to the lowest level, then add
  std::vector<SCt> flat;
  std::vector<int> tgt;
  std::vector<size_t> start;
  for (auto& terms : terms_per_b) {
    int lv = terms[0]->level;
    for (auto& t : terms) lv = std::min(lv, t->level);
    start.push_back(flat.size());
    for (auto& t : terms) {
      flat.push_back(t);
      tgt.push_back(lv);
    }
  }
  flat = b_down(c, flat, tgt);
  const int G = (int)terms_per_b.size();
  std::vector<SCt> out(G);
  // accumulate term by term, all b at once (terms of one b share a level; levels may differ across b)
  std::map<int, std::vector<int>> by_level;
  for (int b = 0; b < G; ++b) by_level[flat[start[b]]->level].push_back(b);
  for (auto& kv : by_level) {
    const int l = kv.first, nl = l + 1;
    auto acc = alloc_batch(c, (int)kv.second.size(), l, 2);
    size_t T = terms_per_b[kv.second[0]].size();
    for (int b : kv.second)
      if (terms_per_b[b].size() != T) fail(COPSE_EINVAL, "internal: ragged sums");
    if (T > 1) {
      std::vector<double*> o;
      std::vector<const double*> terms;
      for (size_t q = 0; q < kv.second.size(); ++q) {
        const int b = kv.second[q];
        o.push_back(acc[q]->data());
        for (size_t t = 0; t < T; ++t) terms.push_back(flat[start[b] + t]->data());
      }
      launch_sum_terms(c, o, terms, (int)T, nl, 2 * nl);
    }
    for (size_t q = 0; q < kv.second.size(); ++q) out[kv.second[q]] = T == 1 ? flat[start[kv.second[q]]] : acc[q];
  }
  return out;
}

// ------------------------------------------------------------------ the evaluation
void check_evaluation(const Context& c, const Model& M, const Keys& k,
                      const std::vector<std::vector<const Ct*>>& groups) {
  if (M.primes != c.primes || (1ULL << M.meta.log_n) != c.N || M.top_level > c.L)
    fail(COPSE_EINVAL, "model encoded for another context");
  if (k.primes != c.primes) fail(COPSE_EINVAL, "keys belong to another context");
  const size_t p = M.meta.precision;
  for (auto& g : groups) {
    if (g.size() != p) fail(COPSE_EINVAL, "query group must hold one ciphertext per bit plane");
    for (auto* x : g) {
      if (!x || x->n != c.N) fail(COPSE_EINVAL, "query ciphertext of another ring");
      if (x->npolys != 2 || x->level != c.L) fail(COPSE_EINVAL, "query ciphertexts must be fresh (top level)");
    }
  }
}

std::vector<CtPtr> evaluate_groups(Context& c, const Model& M, const Keys& k,
                                   const std::vector<std::vector<const Ct*>>& groups) {
  const int G = (int)groups.size();
  const int p = (int)M.meta.precision;
  const size_t N = c.N;
  check_evaluation(c, M, k, groups);
  c.select_tuning(G, M.encrypted);
  auto view = [](const Ct* x) { return SCt(const_cast<Ct*>(x), [](Ct*) {}); };
  // stage timings for the profiler (comparison, reshuffle, levels, aggregation; Section 8's breakdown)
  hipEvent_t stage_ev = nullptr;
  int stage = -1;
  auto next_stage = [&](int s) {
    if (stage >= 0) prof_end(c, kProfStage0 + stage, stage_ev, 0.0);
    stage = s;
    if (s >= 0) prof_begin(c, kProfStage0 + s, &stage_ev);
  };
  // 1. comparison
  next_stage(0);
  // server-side replication: every plane of every group through the replication product first
  std::vector<std::vector<SCt>> rep_planes;
  std::vector<std::vector<const Ct*>> planes_in = groups;
  if (M.meta.server_rep) {
    std::vector<const Ct*> all;
    for (auto& g : groups)
      for (auto* x : g) all.push_back(x);
    const MatPlan& P = M.plan_F;
    const int GP = (int)all.size();
    DBuf B(&c, P.rots.size() * GP * 2 * (size_t)(c.L + 1) * N);
    const int u0 = b_rotate_into(c, k, all, P.rots, B.get());
    auto r = b_matmul_many(c, k, {&P}, P.d_tab, (int)P.rots.size(), B.get(), GP, c.L, u0, all)[0];
    for (int b = 0; b < G; ++b) {
      rep_planes.emplace_back(r.begin() + (size_t)b * p, r.begin() + (size_t)(b + 1) * p);
      for (int kb = 0; kb < p; ++kb) planes_in[b][kb] = rep_planes[b][kb].get();
    }
  }
  std::vector<std::vector<SCt>> eq(p, std::vector<SCt>(G)), lt(p, std::vector<SCt>(G));
  if (!M.encrypted) {
    const int L = M.top_level, nl = L + 1;
    const int J = (2 * p - 1) * G;
    std::vector<const double*> a, mul, add;
    for (int kb = 0; kb < p; ++kb)
      for (int e = (kb >= 1 ? 1 : 0); e >= 0; --e)
        for (int b = 0; b < G; ++b) {
          a.push_back(planes_in[b][kb]->data());
          mul.push_back(e ? M.E[kb].pt->buf.get() : M.G[kb].pt->buf.get());
          add.push_back(e ? M.C[kb].pt->buf.get() : M.TH[kb].pt->buf.get());
        }
    std::vector<SCt> sw;
    if (bridge_supported(c, 1) && L >= 1) {
      // the layer is computed inside its switch
      sw = b_ptlayer_switch(c, a, mul, add, L);
    } else {
      auto raw = alloc_batch(c, J, L, 2);
      std::vector<double*> out;
      for (auto& x : raw) out.push_back(x->data());
      launch_ptlayer(c, out, a, mul, add, nl);
      std::vector<const Ct*> rin;
      for (auto& x : raw) rin.push_back(x.get());
      sw = b_modswitch(c, rin);
    }
    int z = 0;
    for (int kb = 0; kb < p; ++kb)
      for (int e = (kb >= 1 ? 1 : 0); e >= 0; --e)
        for (int b = 0; b < G; ++b) (e ? eq : lt)[kb][b] = sw[z++];
  } else {
    std::vector<std::pair<SCt, SCt>> pairs;
    for (int kb = 0; kb < p; ++kb)
      for (int b = 0; b < G; ++b) pairs.push_back({view(planes_in[b][kb]), view(M.TH[kb].ct.get())});
    auto u = b_mul(c, k, pairs);
    std::vector<const Ct*> xin, tin;
    for (int kb = 0; kb < p; ++kb) {
      tin.push_back(M.TH[kb].ct.get());
      for (int b = 0; b < G; ++b) xin.push_back(planes_in[b][kb]);
    }
    auto xs = b_modswitch(c, xin);
    auto ts = b_modswitch(c, tin);
    const int l = c.L - 1, nl = l + 1;
    auto eqb = alloc_batch(c, p * G, l, 2), ltb = alloc_batch(c, p * G, l, 2);
    std::vector<double*> pe, pl;
    std::vector<const double*> pu, px, pt;
    for (int kb = 0; kb < p; ++kb)
      for (int b = 0; b < G; ++b) {
        int z = kb * G + b;
        pe.push_back(kb >= 1 ? eqb[z]->data() : nullptr);
        pl.push_back(ltb[z]->data());
        pu.push_back(u[z]->data());
        px.push_back(xs[z]->data());
        pt.push_back(ts[kb]->data());
        if (kb >= 1) eq[kb][b] = eqb[z];
        lt[kb][b] = ltb[z];
      }
    launch_seccomp_combine(c, pe, pl, pu, px, pt, nl);
  }
  // the terms lt_k prod_{j > k} eq_j in ceil(log2 p) rounds of products; each round first switches all
  // its operands to the lowest level among them (one key-switch batch per round)
  const int n = p - 1;
  const SeccompPlan plan = seccomp_plan(n);
  std::vector<std::vector<SCt>> val(plan.n_values, std::vector<SCt>(G));
  for (int m = 0; m < n; ++m)
    for (int b = 0; b < G; ++b) {
      val[m][b] = eq[p - 1 - m][b];
      val[n + m][b] = lt[p - 2 - m][b];
    }
  for (const auto& rnd : plan.rounds) {
    int lv = c.L;
    for (const auto& pr : rnd)
      for (int b = 0; b < G; ++b) lv = std::min({lv, val[pr.a][b]->level, val[pr.b][b]->level});
    std::vector<SCt> ops;
    for (const auto& pr : rnd)
      for (int b = 0; b < G; ++b) {
        ops.push_back(val[pr.a][b]);
        ops.push_back(val[pr.b][b]);
      }
    ops = b_down(c, ops, std::vector<int>(ops.size(), lv));
    std::vector<std::pair<SCt, SCt>> pairs;
    for (size_t i = 0; i + 1 < ops.size(); i += 2) pairs.push_back({ops[i], ops[i + 1]});
    auto r = b_mul(c, k, pairs);
    size_t z = 0;
    for (const auto& pr : rnd)
      for (int b = 0; b < G; ++b) val[pr.out][b] = r[z++];
  }
  std::vector<std::vector<SCt>> terms(G);
  for (int b = 0; b < G; ++b) {
    terms[b].push_back(lt[p - 1][b]);
    for (int i = 0; i < n; ++i) terms[b].push_back(val[plan.terms[i]][b]);
  }
  std::vector<SCt> dec = b_sum_all(c, terms);
  for (auto& x : dec)
    if (x->level != M.dec_level) fail(COPSE_EINVAL, "internal: comparison ended at an unexpected level");
  // 2. reshuffle
  next_stage(1);
  std::vector<SCt> src = dec;
  if (!M.meta.fold) {
    const MatPlan& P = M.plan_R;
    const int l = dec[0]->level;
    DBuf B(&c, P.rots.size() * G * 2 * (size_t)(l + 1) * N);
    std::vector<const Ct*> v;
    for (auto& x : dec) v.push_back(x.get());
    const int u0 = b_rotate_into(c, k, v, P.rots, B.get());
    src = b_matmul_many(c, k, {&P}, P.d_tab, (int)P.rots.size(), B.get(), G, l, u0, v)[0];
  }
  // 3. levels: one set of hoisted baby rotations shared by every level
  next_stage(2);
  std::vector<std::vector<SCt>> lv(M.meta.d);
  {
    const int l = src[0]->level;
    DBuf B(&c, M.lvl_rots.size() * G * 2 * (size_t)(l + 1) * N);
    std::vector<const Ct*> v;
    for (auto& x : src) v.push_back(x.get());
    const int u0 = b_rotate_into(c, k, v, M.lvl_rots, B.get());
    // all level products at once; the mask is added by the switch that ends each product
    std::vector<const MatPlan*> plans;
    std::vector<const double*> madd;
    const int ml = l - 1;
    for (uint32_t L_ = 0; L_ < M.meta.d; ++L_) {
      plans.push_back(&M.plan_L[L_]);
      const Operand& mk = M.masks[L_];
      if (mk.ct && mk.ct->level != ml) fail(COPSE_EINVAL, "internal: mask level");
      if (!mk.ct && mk.pt->level != ml) fail(COPSE_EINVAL, "internal: mask level");
      for (int b = 0; b < G; ++b) madd.push_back(mk.ct ? mk.ct->data() : mk.pt->buf.get());
    }
    lv = b_matmul_many(c, k, plans, M.d_lcat, (int)M.lvl_rots.size(), B.get(), G, l, u0, v, &madd,
                       M.masks[0].ct ? 2 : 1);
  }
  // 4. product tree
  next_stage(3);
  while (lv.size() > 1) {
    std::vector<std::pair<SCt, SCt>> pairs;
    for (size_t i = 0; i + 1 < lv.size(); i += 2)
      for (int b = 0; b < G; ++b) pairs.push_back({lv[i][b], lv[i + 1][b]});
    auto r = b_mul(c, k, pairs);
    std::vector<std::vector<SCt>> nxt;
    size_t z = 0;
    for (size_t i = 0; i + 1 < lv.size(); i += 2) {
      nxt.emplace_back();
      for (int b = 0; b < G; ++b) nxt.back().push_back(r[z++]);
    }
    if (lv.size() % 2) nxt.push_back(lv.back());
    lv = std::move(nxt);
  }
  std::vector<SCt> res = b_down(c, lv[0], std::vector<int>(G, 0));
  next_stage(-1);
  std::vector<CtPtr> out;
  for (int b = 0; b < G; ++b) out.push_back(std::make_unique<Ct>(*res[b]));   // shares the storage
  return out;
}

CtPtr evaluate_group(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes) {
  auto r = evaluate_groups(c, M, k, {planes});
  return std::move(r[0]);
}

}  // namespace copse
