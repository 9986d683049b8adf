// The unbatched reference path: one query group per call and one homomorphic
// operation at a time (every rotation is its own key switch, every product
// its own tensor / relinearization / switch, every plaintext product its own
// launch), with the same canonical schedule and hence the same bits as the
// batched engine.  It exists to measure what batching buys.
#include <algorithm>
#include <map>
#include <set>

#include "compiled.hpp"

namespace copse {
namespace {
using SCt = std::shared_ptr<Ct>;
SCt share(CtPtr p) { return SCt(p.release()); }

struct Plain1 {
  Context& c;
  const Model& M;
  const Keys& k;

  SCt mul(const SCt& a, const SCt& b) { return share(op_mul(c, k, *a, *b)); }

  SCt sum_all(std::vector<SCt> terms) {
    int lv = terms[0]->level;
    for (auto& t : terms) lv = std::min(lv, t->level);
    for (auto& t : terms)
      if (t->level > lv) t = share(op_modswitch_to(c, *t, lv));
    SCt out = terms[0];
    for (size_t i = 1; i < terms.size(); ++i) out = share(op_add(c, *out, *terms[i]));
    return out;
  }

  SCt seccomp(const std::vector<const Ct*>& X) {
    const int p = (int)X.size();
    std::vector<SCt> eq(p), lt(p);
    for (int kb = 0; kb < p; ++kb) {
      if (!M.encrypted) {
        if (kb >= 1) {
          auto t1 = op_mul_plain(c, *X[kb], *M.E[kb].pt);
          auto t2 = op_add_plain(c, *t1, *M.C[kb].pt);
          eq[kb] = share(op_modswitch(c, *t2));
        }
        auto t1 = op_mul_plain(c, *X[kb], *M.G[kb].pt);
        auto t2 = op_add_plain(c, *t1, *M.TH[kb].pt);
        lt[kb] = share(op_modswitch(c, *t2));
      } else {
        const Ct& th = *M.TH[kb].ct;
        auto u = share(op_mul(c, k, *X[kb], th));
        auto xs = op_modswitch(c, *X[kb]);
        auto ts = op_modswitch(c, th);
        if (kb >= 1) {
          auto u2 = op_mul_int(c, *u, 2);
          auto a1 = op_sub(c, *u2, *xs);
          auto a2 = op_sub(c, *a1, *ts);
          eq[kb] = share(op_add_const(c, *a2, 1));
        }
        lt[kb] = share(op_sub(c, *ts, *u));
      }
    }
    // the terms lt_k prod_{j > k} eq_j in ceil(log2 p) rounds; each round at the lowest level of its
    // operands
    const int n = p - 1;
    const SeccompPlan plan = seccomp_plan(n);
    std::vector<SCt> val(plan.n_values);
    for (int m = 0; m < n; ++m) {
      val[m] = eq[p - 1 - m];
      val[n + m] = lt[p - 2 - m];
    }
    for (const auto& rnd : plan.rounds) {
      int lv = c.L;
      for (const auto& pr : rnd) lv = std::min({lv, val[pr.a]->level, val[pr.b]->level});
      auto down = [&](const SCt& x) { return x->level > lv ? share(op_modswitch_to(c, *x, lv)) : x; };
      for (const auto& pr : rnd) val[pr.out] = mul(down(val[pr.a]), down(val[pr.b]));
    }
    std::vector<SCt> terms{lt[p - 1]};
    for (int i = 0; i < n; ++i) terms.push_back(val[plan.terms[i]]);
    return sum_all(terms);
  }

  SCt matmul(const SCt& v, const std::vector<Operand>& diags, uint32_t n1) {
    const uint32_t n = (uint32_t)diags.size();
    const uint32_t n2 = (n + n1 - 1) / n1;
    std::set<int32_t> used;
    for (uint32_t kd = 0; kd < n; ++kd)
      if (!diags[kd].zero()) used.insert((int32_t)(kd % n1));
    std::map<int32_t, SCt> baby;
    for (int32_t r : used) baby[r] = share(op_rotate(c, k, *v, r));   // one key switch per rotation
    const int nl = v->level + 1;
    std::vector<SCt> parts;
    std::vector<int32_t> shifts;
    for (uint32_t g = 0; g < n2; ++g) {
      std::vector<std::pair<uint32_t, const Operand*>> terms;
      for (uint32_t j = 0; j < n1; ++j) {
        uint32_t kd = g * n1 + j;
        if (kd < n && !diags[kd].zero()) terms.push_back({j, &diags[kd]});
      }
      if (terms.empty()) continue;
      CtPtr inner;
      if (!M.encrypted) {
        inner = ct_alloc(c, v->level, 2);
        bool first = true;
        for (auto& tj : terms) {
          const Ct& bj = *baby[(int32_t)tj.first];
          if (first) launch_mul_plain(c, inner->data(), bj.data(), tj.second->pt->buf.get(), 2, nl);
          else launch_mac_plain(c, inner->data(), bj.data(), tj.second->pt->buf.get(), 2, nl);
          first = false;
        }
      } else {
        auto acc = ct_alloc(c, v->level, 3);
        bool first = true;
        for (auto& tj : terms) {
          const Ct& bj = *baby[(int32_t)tj.first];
          const Ct& dj = *tj.second->ct;
          launch_tensor(c, acc->data(), bj.data(), dj.data(), nl, !first);
          first = false;
        }
        inner = op_relin(c, k, *acc);
      }
      parts.push_back(share(std::move(inner)));
      shifts.push_back((int32_t)(g * n1));
    }
    // giant steps: the rotated inner sums added with one ModDown, then one switch
    std::vector<std::pair<const Ct*, int32_t>> items;
    for (size_t i = 0; i < parts.size(); ++i) items.push_back({parts[i].get(), shifts[i]});
    auto sum = op_rotate_sum(c, k, items);
    return share(op_modswitch(c, *sum));
  }

  SCt add_mask(const SCt& a, const Operand& mk) {
    if (mk.ct) return share(op_add(c, *a, *mk.ct));
    return share(op_add_plain(c, *a, *mk.pt));
  }

  CtPtr run(const std::vector<const Ct*>& X) {
    check_evaluation(c, M, k, {X});
    c.select_tuning(1, M.encrypted);
    std::vector<SCt> rep;
    std::vector<const Ct*> planes = X;
    if (M.meta.server_rep) {
      // server-side replication: each plane through the replication product first
      for (auto* x : X) rep.push_back(matmul(SCt(const_cast<Ct*>(x), [](Ct*) {}), M.fdiag, M.meta.n1_F));
      for (size_t i = 0; i < X.size(); ++i) planes[i] = rep[i].get();
    }
    SCt dec = seccomp(planes);
    std::vector<SCt> lv;
    SCt src = M.meta.fold ? dec : matmul(dec, M.rdiag, M.meta.n1_R);
    for (uint32_t l = 0; l < M.meta.d; ++l) lv.push_back(add_mask(matmul(src, M.ldiag[l], M.meta.n1_L), M.masks[l]));
    while (lv.size() > 1) {
      std::vector<SCt> nxt;
      for (size_t i = 0; i + 1 < lv.size(); i += 2) nxt.push_back(mul(lv[i], lv[i + 1]));
      if (lv.size() % 2) nxt.push_back(lv.back());
      lv = std::move(nxt);
    }
    return op_modswitch_to(c, *lv[0], 0);
  }
};
}  // namespace

CtPtr evaluate_group_plain(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes) {
  Plain1 e{c, M, k};
  return e.run(planes);
}

}  // namespace copse
