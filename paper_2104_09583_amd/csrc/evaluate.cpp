// Model encoding and the encrypted evaluation of Algorithm 1 (Section 4.3):
// SecComp -> reshuffle MatMul -> per-level MatMul with the mask -> MultAll.
//
// The schedule that fixes every ciphertext bit:
//   * binary operations switch the higher operand down one prime at a time;
//   * a sum of several terms switches each term to the lowest level, then adds;
//   * ciphertext product = tensor, relinearize, one modulus switch;
//   * a plaintext-product layer is followed by one modulus switch;
//   * MatMul (diagonal method, baby-step/giant-step): hoisted baby rotations,
//     per giant group the sum of products with pre-rotated diagonals
//     (ciphertext diagonals: tensor sum relinearized once per group), the
//     giant rotation, the sum over groups, one modulus switch; zero
//     plaintext diagonals and unused baby steps are skipped (no bit changes);
//   * the level mask is added after the MatMul's modulus switch;
//   * MultAll pairs (0,1), (2,3), ... and carries an odd last element up;
//   * the result is switched down to q_0.
// Comparison (the paper cites SecComp without restating it; this is the
// most-significant-bit-first circuit): with plaintext thresholds
//   eq_k = x_k (2 th_k - 1) + (1 - th_k),  lt_k = x_k (-th_k) + th_k;
// with encrypted thresholds u_k = x_k Th_k, eq_k = 2u_k - x_k - Th_k + 1,
// lt_k = Th_k - u_k; then S_k = prod_{j>k} eq_j by a Kogge-Stone prefix
// product over (eq_{p-1}, ..., eq_1) and dec = lt_{p-1} + sum_k lt_k S_k.
#include <algorithm>
#include <cmath>
#include <set>

#include "compiled.hpp"

namespace copse {

using SCt = std::shared_ptr<Ct>;

static SCt share(CtPtr p) { return SCt(p.release()); }

static int seccomp_depth(uint32_t p) {
  if (p <= 2) return (int)p;
  int r = 0;
  while ((1u << r) < p - 1) ++r;
  return 2 + r;
}

static uint64_t obj_id(uint64_t kind, uint64_t a, uint64_t b) { return (kind << 56) | (a << 32) | b; }

std::unique_ptr<Model> build_model(Context& c, const Compiled& C, const Keys* k, bool encrypt_model,
                                   const uint8_t seed[32]) {
  const copse_public_meta& meta = C.meta;
  if ((1ULL << meta.log_n) != c.N) fail(COPSE_EINVAL, "forest compiled for another ring size");
  if (encrypt_model && (!k || !k->pk_b.get())) fail(COPSE_EKEY, "public key needed to encrypt the model");
  auto M = std::make_unique<Model>();
  M->meta = meta;
  M->encrypted = encrypt_model;
  const int L = c.L;
  M->dec_level = L - seccomp_depth(meta.precision);
  M->br_level = meta.fold ? M->dec_level : M->dec_level - 1;
  M->lvl_level = M->br_level - 1;
  int tree = 0;
  while ((1u << tree) < meta.d) ++tree;
  if (M->lvl_level - tree < 0)
    fail(COPSE_ECAPACITY, "circuit needs " + std::to_string(meta.depth) + " levels, chain has " + std::to_string(L));
  const size_t N = c.N;
  const uint64_t t = c.t;
  const uint32_t q = meta.q, b = meta.b, m = meta.m, K = meta.K;
  const uint32_t B_in = m + b + q - 2;
  auto enc_slots = [&](const std::vector<uint64_t>& slots, int level, uint64_t obj) {
    std::vector<int64_t> poly;
    encode_slots(c, slots.data(), poly);
    return encrypt(c, *k, poly, level, seed, obj);
  };
  auto make_operand = [&](const std::vector<uint64_t>& slots, int level, uint64_t obj, bool skip_zero) {
    Operand o;
    bool nz = std::any_of(slots.begin(), slots.end(), [](uint64_t v) { return v != 0; });
    if (encrypt_model) {
      o.ct = enc_slots(slots, level, obj);
      M->bytes += o.ct->buf.size() * 8;
    } else if (nz || !skip_zero) {
      o.pt = make_plain_slots(c, slots.data(), level);
      M->bytes += o.pt->buf.size() * 8;
    }
    return o;
  };
  // thresholds over the cyclically extended padded layout
  std::vector<int64_t> thr_ext(B_in);
  for (uint32_t s = 0; s < B_in; ++s) {
    int bi = C.padded[s % q];
    thr_ext[s] = bi < 0 ? 0 : (int64_t)C.nodes[C.branch_nodes[bi]].threshold;
  }
  (void)K;
  std::vector<uint64_t> slots;
  for (uint32_t kb = 0; kb < meta.precision; ++kb) {
    std::vector<int64_t> th(B_in);
    for (uint32_t s = 0; s < B_in; ++s) th[s] = (thr_ext[s] >> kb) & 1;
    if (encrypt_model) {
      replicate_blocks(meta, N, th, slots, t);
      M->TH.push_back(make_operand(slots, L, obj_id(2, 0, kb), false));
      M->E.emplace_back(); M->C.emplace_back(); M->G.emplace_back();
    } else {
      // slots outside B_in have th = 0: E = -1, C = 1 there, as the formula gives
      std::vector<uint64_t> sE(N, t - 1), sC(N, 1), sG(N, 0), sT(N, 0);
      std::vector<uint64_t> thslots;
      replicate_blocks(meta, N, th, thslots, t);
      for (size_t i = 0; i < N; ++i) {
        uint64_t v = thslots[i];
        sE[i] = v ? 1 : t - 1;
        sC[i] = v ? 0 : 1;
        sG[i] = v ? t - 1 : 0;
        sT[i] = v;
      }
      M->E.push_back(make_operand(sE, L, 0, false));
      M->C.push_back(make_operand(sC, L, 0, false));
      M->G.push_back(make_operand(sG, L, 0, false));
      M->TH.push_back(make_operand(sT, L, 0, false));
    }
  }
  // column of each branch in the padded vector
  std::vector<int> col(b, -1);
  for (uint32_t j = 0; j < q; ++j)
    if (C.padded[j] >= 0) col[C.padded[j]] = (int)j;
  auto add_diags = [&](const std::vector<std::vector<int64_t>>& A, uint32_t n1, int level, uint64_t kind,
                       uint64_t lidx, std::vector<Operand>& out) {
    const uint32_t n = (uint32_t)A[0].size();
    for (uint32_t kd = 0; kd < n; ++kd) {
      bool nz;
      diagonal_slots(meta, N, A, kd, n1, slots, t, &nz);
      if (!encrypt_model && !nz) { out.emplace_back(); continue; }
      out.push_back(make_operand(slots, level, obj_id(kind, lidx, kd), true));
    }
  };
  if (!meta.fold) {
    std::vector<std::vector<int64_t>> Rext(m + b - 1, std::vector<int64_t>(q, 0));
    for (uint32_t j = 0; j < m + b - 1; ++j) Rext[j][col[j % b]] = 1;
    add_diags(Rext, meta.n1_R, M->dec_level, 3, 0, M->rdiag);
  }
  M->ldiag.resize(meta.d);
  for (uint32_t l = 0; l < meta.d; ++l) {
    const uint32_t n = meta.fold ? q : b;
    std::vector<std::vector<int64_t>> A(m, std::vector<int64_t>(n, 0));
    for (uint32_t i = 0; i < m; ++i) {
      int s = C.sel[l][i];
      if (s < 0) continue;
      int64_t v = 1 - 2 * (int64_t)C.mask[l][i];
      A[i][meta.fold ? col[s] : s] = v;
    }
    add_diags(A, meta.n1_L, meta.fold ? M->dec_level : M->br_level, 4, l, M->ldiag[l]);
  }
  for (uint32_t l = 0; l < meta.d; ++l) {
    std::vector<int64_t> mk(m);
    for (uint32_t i = 0; i < m; ++i) mk[i] = C.mask[l][i];
    replicate_blocks(meta, N, mk, slots, t);
    M->masks.push_back(make_operand(slots, M->lvl_level, obj_id(5, 0, l), false));
  }
  COPSE_HIP(hipStreamSynchronize(c.stream));
  return M;
}

// ------------------------------------------------------------------ evaluation of one group
namespace {
struct Eval {
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
    std::vector<SCt> cur;
    for (int i = 0; i < p - 1; ++i) cur.push_back(eq[p - 1 - i]);
    for (size_t s = 1; s < cur.size(); s *= 2) {
      std::vector<SCt> nxt = cur;
      for (size_t i = s; i < cur.size(); ++i) nxt[i] = mul(cur[i], cur[i - s]);
      cur = std::move(nxt);
    }
    std::vector<SCt> terms{lt[p - 1]};
    for (int kb = 0; kb < p - 1; ++kb) terms.push_back(mul(lt[kb], cur[p - 2 - kb]));
    return sum_all(terms);
  }

  SCt matmul(const SCt& v, const std::vector<Operand>& diags, uint32_t n1) {
    const uint32_t n = (uint32_t)diags.size();
    const uint32_t n2 = (n + n1 - 1) / n1;
    std::set<int32_t> used;
    for (uint32_t kd = 0; kd < n; ++kd)
      if (!diags[kd].zero()) used.insert((int32_t)(kd % n1));
    std::vector<int32_t> rs(used.begin(), used.end());
    auto baby_v = op_rotate_hoisted(c, k, *v, rs);
    std::map<int32_t, size_t> at;
    for (size_t i = 0; i < rs.size(); ++i) at[rs[i]] = i;
    const size_t N = c.N;
    const int nl = v->level + 1;
    std::vector<SCt> parts;
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
          const Ct& bj = *baby_v[at[(int32_t)tj.first]];
          if (first) launch_mul_plain(c, inner->buf.get(), bj.buf.get(), tj.second->pt->buf.get(), 2, nl);
          else launch_mac_plain(c, inner->buf.get(), bj.buf.get(), tj.second->pt->buf.get(), 2, nl);
          first = false;
        }
      } else {
        auto acc = ct_alloc(c, v->level, 3);
        bool first = true;
        for (auto& tj : terms) {
          const Ct& bj = *baby_v[at[(int32_t)tj.first]];
          const Ct& dj = *tj.second->ct;
          if (dj.level != v->level) fail(COPSE_EINVAL, "encrypted diagonal at the wrong level");
          launch_tensor(c, acc->buf.get(), bj.buf.get(), dj.buf.get(), nl, !first);
          first = false;
        }
        inner = op_relin(c, k, *acc);
      }
      (void)N;
      if (g > 0) inner = op_rotate(c, k, *inner, (int32_t)(g * n1));
      parts.push_back(share(std::move(inner)));
    }
    SCt out = parts[0];
    for (size_t i = 1; i < parts.size(); ++i) out = share(op_add(c, *out, *parts[i]));
    return share(op_modswitch(c, *out));
  }

  SCt add_mask(const SCt& a, const Operand& mk) {
    if (mk.ct) return share(op_add(c, *a, *mk.ct));
    return share(op_add_plain(c, *a, *mk.pt));
  }

  CtPtr run(const std::vector<const Ct*>& X) {
    if (X.size() != M.meta.precision) fail(COPSE_EINVAL, "query group must hold one ciphertext per bit plane");
    for (auto* x : X)
      if (x->npolys != 2 || x->level != c.L) fail(COPSE_EINVAL, "query ciphertexts must be fresh (top level)");
    SCt dec = seccomp(X);
    if (dec->level != M.dec_level) fail(COPSE_EINVAL, "internal: comparison ended at an unexpected level");
    std::vector<SCt> lv;
    if (M.meta.fold) {
      for (uint32_t l = 0; l < M.meta.d; ++l) lv.push_back(add_mask(matmul(dec, M.ldiag[l], M.meta.n1_L), M.masks[l]));
    } else {
      SCt br = matmul(dec, M.rdiag, M.meta.n1_R);
      for (uint32_t l = 0; l < M.meta.d; ++l) lv.push_back(add_mask(matmul(br, M.ldiag[l], M.meta.n1_L), M.masks[l]));
    }
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

CtPtr evaluate_group(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes) {
  Eval e{c, M, k};
  return e.run(planes);
}

std::vector<CtPtr> evaluate_groups(Context& c, const Model& M, const Keys& k,
                                   const std::vector<std::vector<const Ct*>>& groups) {
  std::vector<CtPtr> out;
  for (auto& g : groups) out.push_back(evaluate_group(c, M, k, g));
  return out;
}

}  // namespace copse
