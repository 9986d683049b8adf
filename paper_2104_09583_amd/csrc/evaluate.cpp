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

static uint64_t obj_id(uint64_t kind, uint64_t a, uint64_t b) { return (kind << 56) | (a << 32) | b; }

std::unique_ptr<Model> build_model(Context& c, const Compiled& C, const Keys* k, bool encrypt_model,
                                   const uint8_t seed[32]) {
  const copse_public_meta& meta = C.meta;
  if ((1ULL << meta.log_n) != c.N) fail(COPSE_EINVAL, "forest compiled for another ring size");
  if (encrypt_model && (!k || !k->pk_b.get())) fail(COPSE_EKEY, "public key needed to encrypt the model");
  if (k && k->primes != c.primes) fail(COPSE_EINVAL, "keys belong to another context");
  auto M = std::make_unique<Model>();
  M->primes = c.primes;
  M->meta = meta;
  M->encrypted = encrypt_model;
  if (meta.server_rep && encrypt_model) fail(COPSE_EINVAL, "server-side replication is for a server-held model");
  const int L = c.L;
  // with server-side replication the comparison reads the replicated planes one level down
  const int top = meta.server_rep ? L - 1 : L;
  M->top_level = top;
  M->dec_level = top - seccomp_depth(meta.precision);
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
      M->bytes += o.ct->words() * 8;
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
      M->TH.push_back(make_operand(slots, top, obj_id(2, 0, kb), false));
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
      M->E.push_back(make_operand(sE, top, 0, false));
      M->C.push_back(make_operand(sC, top, 0, false));
      M->G.push_back(make_operand(sG, top, 0, false));
      M->TH.push_back(make_operand(sT, top, 0, false));
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
  if (meta.server_rep) {
    // Rep (B_in x F): padded slot s mod q holds feature (s mod q) / K
    const uint32_t F = meta.n_features;
    std::vector<std::vector<int64_t>> Rep(B_in, std::vector<int64_t>(F, 0));
    for (uint32_t s = 0; s < B_in; ++s) Rep[s][(s % q) / meta.K] = 1;
    add_diags(Rep, meta.n1_F, L, 6, 0, M->fdiag);
  }
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
  // matrix-product plans; the level products share one set of baby rotations
  if (!meta.fold) build_plan(c, M->plan_R, M->rdiag, meta.n1_R, encrypt_model, nullptr);
  if (meta.server_rep) build_plan(c, M->plan_F, M->fdiag, meta.n1_F, false, nullptr);
  {
    std::set<int32_t> used;
    for (auto& dl : M->ldiag)
      for (size_t kd = 0; kd < dl.size(); ++kd)
        if (!dl[kd].zero()) used.insert((int32_t)(kd % meta.n1_L));
    M->lvl_rots.assign(used.begin(), used.end());
  }
  M->plan_L.resize(meta.d);
  for (uint32_t l = 0; l < meta.d; ++l) build_plan(c, M->plan_L[l], M->ldiag[l], meta.n1_L, encrypt_model, &M->lvl_rots);
  {
    // all level products run as one launch over their concatenated giant groups
    size_t ngs = 0;
    for (auto& P : M->plan_L) ngs += P.groups.size();
    const size_t nu = M->lvl_rots.size();
    std::vector<const double*> cat(nu * ngs + kMmTabPad, nullptr);
    size_t off = 0;
    for (auto& P : M->plan_L) {
      const size_t ng = P.groups.size();
      for (size_t u = 0; u < nu; ++u)
        for (size_t s = 0; s < ng; ++s) cat[u * ngs + off + s] = P.tab[u * ng + s];
      off += ng;
    }
    M->lcat_buf = DBuf(&c, cat.size());
    COPSE_HIP(hipMemcpyAsync(M->lcat_buf.get(), cat.data(), cat.size() * sizeof(const double*), hipMemcpyHostToDevice,
                             c.stream));
    COPSE_HIP(hipStreamSynchronize(c.stream));   // cat is a host temporary
    M->d_lcat = reinterpret_cast<const double* const*>(M->lcat_buf.get());
  }
  COPSE_HIP(hipStreamSynchronize(c.stream));
  return M;
}

// ------------------------------------------------------------------ matrix-product plans
void build_plan(Context& c, MatPlan& P, const std::vector<Operand>& diags, uint32_t n1, bool enc,
                const std::vector<int32_t>* shared_rots) {
  const uint32_t n = (uint32_t)diags.size();
  P.n1 = n1;
  P.enc = enc;
  if (shared_rots) {
    P.rots = *shared_rots;
  } else {
    std::set<int32_t> used;
    for (uint32_t kd = 0; kd < n; ++kd)
      if (!diags[kd].zero()) used.insert((int32_t)(kd % n1));
    P.rots.assign(used.begin(), used.end());
  }
  std::map<int32_t, int> slot;
  for (size_t u = 0; u < P.rots.size(); ++u) slot[P.rots[u]] = (int)u;
  const uint32_t n2 = (n + n1 - 1) / n1;
  std::vector<std::vector<std::pair<int, const double*>>> per_group;
  for (uint32_t g = 0; g < n2; ++g) {
    std::vector<std::pair<int, const double*>> terms;
    for (uint32_t j = 0; j < n1; ++j) {
      uint32_t kd = g * n1 + j;
      if (kd >= n || diags[kd].zero()) continue;
      const double* dp = enc ? diags[kd].ct->data() : diags[kd].pt->buf.get();
      terms.emplace_back(slot.at((int32_t)j), dp);
    }
    if (!terms.empty()) {
      P.groups.push_back(g);
      per_group.push_back(std::move(terms));
    }
  }
  const size_t nu = P.rots.size(), ng = P.groups.size();
  std::vector<const double*>& tab = P.tab;
  tab.assign(nu * ng, nullptr);
  for (size_t s = 0; s < ng; ++s)
    for (auto& t : per_group[s]) tab[(size_t)t.first * ng + s] = t.second;
  std::vector<const double*> padded(tab);
  padded.resize(tab.size() + kMmTabPad, nullptr);
  P.tab_buf = DBuf(&c, padded.size());
  COPSE_HIP(hipMemcpyAsync(P.tab_buf.get(), padded.data(), padded.size() * sizeof(const double*),
                           hipMemcpyHostToDevice, c.stream));
  COPSE_HIP(hipStreamSynchronize(c.stream));
  P.d_tab = reinterpret_cast<const double* const*>(P.tab_buf.get());
}

}  // namespace copse
