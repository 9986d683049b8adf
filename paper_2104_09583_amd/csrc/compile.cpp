// Forest compiler (model owner): serialized forest -> padded thresholds,
// reshuffle matrix, level matrices and masks, slot layout and baby-step
// counts.  Definitions follow Section 4.1 ("Properties of nodes", "Properties
// of models", generalized diagonals) and Section 4.2 (padded threshold
// vector, reshuffling matrix, level matrices, level masks).
#include <algorithm>
#include <cmath>
#include <sstream>

#include <functional>
#include <map>

#include "compiled.hpp"

namespace copse {

namespace {
struct Parser {
  std::vector<std::string> toks;
  size_t pos = 0;
  int n_labels_names = 0;
  int parse(std::vector<Node>& nodes) {
    if (pos >= toks.size()) fail(COPSE_EINVAL, "truncated tree");
    const std::string& tag = toks[pos];
    if (tag == "L") {
      if (pos + 1 >= toks.size()) fail(COPSE_EINVAL, "truncated leaf");
      long lab = std::stol(toks[pos + 1]);
      pos += 2;
      if (lab < 0 || lab >= n_labels_names) fail(COPSE_EINVAL, "label index out of range");
      nodes.push_back(Node{true, 0, 0, (int)lab, -1, -1, -1});
      return (int)nodes.size() - 1;
    }
    if (tag == "B") {
      if (pos + 2 >= toks.size()) fail(COPSE_EINVAL, "truncated branch");
      long f = std::stol(toks[pos + 1]);
      long long thr = std::stoll(toks[pos + 2]);
      if (f < 0 || thr < 0) fail(COPSE_EINVAL, "negative feature or threshold");
      pos += 3;
      int me = (int)nodes.size();
      nodes.push_back(Node{false, (int)f, (uint64_t)thr, 0, -1, -1, -1});
      int l = parse(nodes);
      int r = parse(nodes);
      nodes[me].left = l;
      nodes[me].right = r;
      return me;
    }
    fail(COPSE_EINVAL, "bad token '" + tag + "'");
  }
};

int level_of(std::vector<Node>& nodes, int n) {
  Node& x = nodes[n];
  if (x.leaf) return 0;
  if (x.level >= 0) return x.level;
  x.level = 1 + std::max(level_of(nodes, x.left), level_of(nodes, x.right));
  return x.level;
}
}  // namespace

uint32_t pow2_ceil(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint32_t baby_steps(uint32_t n) {
  if (n <= 1) return 1;
  // 2^ceil(log2 sqrt(n)): smallest power of two p with p*p >= n
  uint32_t p = 1;
  while ((uint64_t)p * p < n) p <<= 1;
  return p;
}

std::unique_ptr<Compiled> compile_forest(const char* text, size_t len, uint32_t F, uint32_t prec, uint32_t log_n,
                                         int fold, uint32_t n1R, uint32_t n1L) {
  if (!text) fail(COPSE_EINVAL, "null forest text");
  if (F == 0 || prec == 0 || prec > 32) fail(COPSE_EINVAL, "bad feature count or precision");
  std::string s(text, len);
  std::istringstream in(s);
  std::string line;
  std::vector<std::string> lines;
  while (std::getline(in, line)) {
    bool blank = line.find_first_not_of(" \t\r") == std::string::npos;
    if (!blank) lines.push_back(line);
  }
  if (lines.empty()) fail(COPSE_EINVAL, "empty forest text");
  auto C = std::make_unique<Compiled>();
  {
    std::istringstream ls(lines[0]);
    std::string nm;
    while (ls >> nm) C->label_names.push_back(nm);
  }
  if (lines.size() < 2) fail(COPSE_EINVAL, "forest has no trees");
  for (size_t li = 1; li < lines.size(); ++li) {
    Parser p;
    std::istringstream ls(lines[li]);
    std::string tk;
    while (ls >> tk) p.toks.push_back(tk);
    p.n_labels_names = (int)C->label_names.size();
    int root;
    try {
      root = p.parse(C->nodes);
    } catch (const std::invalid_argument&) {
      fail(COPSE_EINVAL, "non-numeric token");
    } catch (const std::out_of_range&) {
      fail(COPSE_EINVAL, "numeric token out of range");
    }
    if (p.pos != p.toks.size()) fail(COPSE_EINVAL, "trailing tokens on a tree line");
    C->roots.push_back(root);
  }
  auto& nodes = C->nodes;
  // preorder indices, ancestors and sides of labels
  struct Frame { int n; std::vector<int> anc; std::vector<int> side; };
  for (int root : C->roots) {
    std::vector<Frame> st;
    st.push_back({root, {}, {}});
    while (!st.empty()) {
      Frame f = std::move(st.back());
      st.pop_back();
      Node& x = nodes[f.n];
      if (x.leaf) {
        x.index = (int)C->label_nodes.size();
        C->label_nodes.push_back(f.n);
        C->anc.push_back(f.anc);
        C->side.push_back(f.side);
        continue;
      }
      x.index = (int)C->branch_nodes.size();
      C->branch_nodes.push_back(f.n);
      auto al = f.anc, ar = f.anc;
      al.push_back(f.n); ar.push_back(f.n);
      auto sl = f.side, sr = f.side;
      sl.push_back(0); sr.push_back(1);
      st.push_back({x.right, ar, sr});   // pushed first, visited second
      st.push_back({x.left, al, sl});
    }
  }
  const uint32_t b = (uint32_t)C->branch_nodes.size();
  const uint32_t m = (uint32_t)C->label_nodes.size();
  if (b == 0) fail(COPSE_EINVAL, "forest has no branches");
  for (int bn : C->branch_nodes) {
    if ((uint32_t)nodes[bn].feature >= F) fail(COPSE_EINVAL, "feature index out of range");
    if (prec < 64 && nodes[bn].threshold >= (1ULL << prec)) fail(COPSE_EINVAL, "threshold exceeds precision");
  }
  uint32_t d = 0;
  for (int r : C->roots) d = std::max<uint32_t>(d, (uint32_t)level_of(nodes, r));
  std::vector<uint32_t> kappa(F, 0);
  for (int bn : C->branch_nodes) kappa[nodes[bn].feature]++;
  uint32_t K = *std::max_element(kappa.begin(), kappa.end());
  uint32_t q = K * F;
  // padded threshold vector: per feature, its branches in ascending preorder, then sentinels
  C->padded.assign(q, -1);
  for (uint32_t f = 0; f < F; ++f) {
    uint32_t k = 0;
    for (uint32_t bi = 0; bi < b; ++bi)
      if ((uint32_t)nodes[C->branch_nodes[bi]].feature == f) C->padded[f * K + k++] = (int)bi;
  }
  // level selections and masks
  C->sel.assign(d, std::vector<int>(m, -1));
  C->mask.assign(d, std::vector<int>(m, 1));
  for (uint32_t l = 1; l <= d; ++l) {
    for (uint32_t i = 0; i < m; ++i) {
      const auto& A = C->anc[i];
      if (A.empty()) { C->sel[l - 1][i] = -1; C->mask[l - 1][i] = 1; continue; }
      int choice = -1;
      for (size_t a = 0; a < A.size(); ++a)
        if ((uint32_t)nodes[A[a]].level == l) choice = (int)a;
      if (choice < 0) {
        int best = -1;
        for (size_t a = 0; a < A.size(); ++a)
          if ((uint32_t)nodes[A[a]].level < l && (best < 0 || nodes[A[a]].level > nodes[A[best]].level))
            best = (int)a;
        choice = best >= 0 ? best : (int)A.size() - 1;
      }
      C->sel[l - 1][i] = nodes[A[choice]].index;
      C->mask[l - 1][i] = C->side[i][choice] == 1 ? 0 : 1;
    }
  }
  auto& M = C->meta;
  std::memset(&M, 0, sizeof(M));
  M.n_features = F; M.precision = prec; M.K = K; M.q = q; M.b = b; M.m = m; M.d = d;
  M.n_trees = (uint32_t)C->roots.size();
  uint32_t B_in = m + b + q - 2;
  M.block_w = pow2_ceil(std::max<uint32_t>(B_in, 1));
  M.log_n = log_n;
  uint64_t N = 1ULL << log_n;
  if (M.block_w > N / 2) fail(COPSE_ECAPACITY, "query block of " + std::to_string(M.block_w) +
                                                  " slots exceeds a slot row of " + std::to_string(N / 2));
  M.queries_per_ct = (uint32_t)(N / M.block_w);
  M.fold = fold ? 1 : 0;
  M.n1_R = n1R ? n1R : baby_steps(q);
  M.n1_L = n1L ? n1L : baby_steps(fold ? q : b);
  // depth: comparison, reshuffle (unless folded), level product, product tree
  const uint32_t seccomp = (uint32_t)seccomp_depth(prec);
  uint32_t tree = 0;
  while ((1u << tree) < d) ++tree;
  M.depth = seccomp + (fold ? 1 : 2) + tree;
  M.server_rep = 0;
  M.n1_F = baby_steps(F);
  C->B_in = B_in;
  for (int ln : C->label_nodes) C->codebook.push_back(nodes[ln].label);
  for (uint32_t i = 0; i < m; ++i) C->perm.push_back((int)i);
  return C;
}

// Result privacy (Section 7.2.2, "Returning classification bitvectors"): the server shuffles the result
// bitvector and the codebook by one random permutation and pads both with n_pad labels that are never
// selected; here the shuffle is folded into the level products by permuting the rows of every level
// matrix and mask (a padding row is all zero with mask 0, so its level results and its product are 0),
// at no extra homomorphic cost.  Slot s takes original row arr[s]: arr starts as the identity on
// m + n_pad rows and is shuffled by Fisher-Yates (i from m + n_pad - 1 down to 1: swap arr[i] with
// arr[j], j drawn below i + 1); then one class is drawn per padding row (increasing row order) below
// the number of label names.  Draws: 8-byte little-endian words of the SHAKE-256 stream of domain
// "res.perm" (object 0, limb 0), masked to the bound's bit length and rejected at or above it.
void privatize(Compiled& C, const uint8_t seed[32], uint32_t n_pad) {
  auto& M = C.meta;
  const uint32_t m = M.m, mp = m + n_pad;
  if ((uint64_t)mp + M.b + M.q > (1ULL << 31)) fail(COPSE_EINVAL, "padding too large");
  ShakeStream st(seed, "res.perm", 0, 0);
  auto below = [&](uint64_t bound) -> uint64_t {
    int bits = 64 - __builtin_clzll(bound);
    const uint64_t mask = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
    while (true) {
      uint8_t b[8];
      st.read(b, 8);
      uint64_t w = 0;
      for (int k = 0; k < 8; ++k) w |= (uint64_t)b[k] << (8 * k);
      w &= mask;
      if (w < bound) return w;
    }
  };
  std::vector<int> arr(mp);
  for (uint32_t i = 0; i < mp; ++i) arr[i] = (int)i;
  for (uint32_t i = mp - 1; i >= 1 && mp > 1; --i) std::swap(arr[i], arr[below(i + 1)]);
  const uint64_t classes = std::max<size_t>(1, C.label_names.size());
  std::vector<int> pad_label(n_pad);
  for (uint32_t r = 0; r < n_pad; ++r) pad_label[r] = (int)below(classes);
  std::vector<std::vector<int>> sel(C.sel.size(), std::vector<int>(mp)), mask(C.mask.size(), std::vector<int>(mp));
  std::vector<int> book(mp), perm(mp);
  for (uint32_t s = 0; s < mp; ++s) {
    const int r = arr[s];
    for (size_t l = 0; l < C.sel.size(); ++l) {
      sel[l][s] = r < (int)m ? C.sel[l][r] : -1;
      mask[l][s] = r < (int)m ? C.mask[l][r] : 0;
    }
    book[s] = r < (int)m ? C.codebook[r] : pad_label[r - m];
    perm[s] = r < (int)m ? C.perm[r] : r;
  }
  C.sel = std::move(sel);
  C.mask = std::move(mask);
  C.codebook = std::move(book);
  C.perm = std::move(perm);
  M.m = mp;
  C.B_in = mp + M.b + M.q - 2;
  set_block(C);
}

// Server-side feature replication (Section 7.2.1, "Feature padding"): the query holds feature s mod F in block slot s for
// s < B_in + F - 1; the server multiplies by Rep (B_in x F, Rep[s][f] = 1 iff padded slot s mod q
// belongs to feature f) with the diagonal method before the comparison: one more level.
void server_replicate(Compiled& C, uint32_t n1F) {
  auto& M = C.meta;
  M.server_rep = 1;
  M.n1_F = n1F ? n1F : baby_steps(M.n_features);
  M.depth += 1;
  set_block(C);
}

void set_block(Compiled& C) {
  auto& M = C.meta;
  const uint32_t span = C.B_in + (M.server_rep ? M.n_features - 1 : 0);
  M.block_w = pow2_ceil(std::max<uint32_t>(span, 1));
  const uint64_t N = 1ULL << M.log_n;
  if (M.block_w > N / 2) fail(COPSE_ECAPACITY, "query block of " + std::to_string(M.block_w) +
                                                  " slots exceeds a slot row of " + std::to_string(N / 2));
  M.queries_per_ct = (uint32_t)(N / M.block_w);
}

std::vector<int32_t> needed_rotations(const copse_public_meta& M) {
  std::vector<int32_t> r;
  auto add = [&](uint32_t n, uint32_t n1) {
    for (uint32_t j = 1; j < n1; ++j) r.push_back((int32_t)j);
    for (uint32_t g = 1; g * n1 < n; ++g) r.push_back((int32_t)(g * n1));
  };
  if (!M.fold) add(M.q, M.n1_R);
  add(M.fold ? M.q : M.b, M.n1_L);
  if (M.server_rep) add(M.n_features, M.n1_F);
  std::sort(r.begin(), r.end());
  r.erase(std::unique(r.begin(), r.end()), r.end());
  return r;
}

// ---------------------------------------------------------------- slot vectors of the layout
// slot index of block k, offset s: row k / bpr, column (k % bpr) * W + s; rows of N/2 slots.
static size_t slot_index(const copse_public_meta& M, size_t N, uint32_t k, uint32_t s) {
  size_t bpr = (N / 2) / M.block_w;
  size_t row = k / bpr, col = (k % bpr) * M.block_w + s;
  return row * (N / 2) + col;
}

void replicate_blocks(const copse_public_meta& M, size_t N, const std::vector<int64_t>& vec,
                      std::vector<uint64_t>& slots, uint64_t t) {
  slots.assign(N, 0);
  for (uint32_t k = 0; k < M.queries_per_ct; ++k)
    for (size_t s = 0; s < vec.size(); ++s) {
      int64_t v = vec[s] % (int64_t)t;
      if (v < 0) v += (int64_t)t;
      slots[slot_index(M, N, k, (uint32_t)s)] = (uint64_t)v;
    }
}

void query_plane_slots(const copse_public_meta& M, size_t N, const uint32_t* feats, size_t nq, uint32_t plane,
                       std::vector<uint64_t>& slots) {
  slots.assign(N, 0);
  uint32_t B_in = M.m + M.b + M.q - 2;
  for (size_t k = 0; k < nq; ++k) {
    if (M.server_rep) {
      // each feature once, extended with period F over B_in + F - 1 slots
      for (uint32_t s = 0; s < B_in + M.n_features - 1; ++s)
        slots[slot_index(M, N, (uint32_t)k, s)] = (feats[k * M.n_features + s % M.n_features] >> plane) & 1u;
      continue;
    }
    for (uint32_t s = 0; s < B_in; ++s) {
      uint32_t pos = s % M.q;
      uint32_t f = pos / M.K;
      slots[slot_index(M, N, (uint32_t)k, s)] = (feats[k * M.n_features + f] >> plane) & 1u;
    }
  }
}

// Generalized diagonal k of A (rows x n), pre-rotated to block offset g*n1, replicated per block.
void diagonal_slots(const copse_public_meta& M, size_t N, const std::vector<std::vector<int64_t>>& A, uint32_t k,
                    uint32_t n1, std::vector<uint64_t>& slots, uint64_t t, bool* nonzero) {
  const size_t rows = A.size(), n = A[0].size();
  const uint32_t g = k / n1;
  std::vector<int64_t> vec((size_t)g * n1 + rows, 0);
  bool nz = false;
  for (size_t j = 0; j < rows; ++j) {
    int64_t v = A[j][(j + k) % n];
    vec[(size_t)g * n1 + j] = v;
    if (v % (int64_t)t) nz = true;
  }
  *nonzero = nz;
  replicate_blocks(M, N, vec, slots, t);
}

// Every value is named by the set of leaves it multiplies (bit m: e_m, bit 32 + i: l_i), so a product
// is made once.  The e's are combined in aligned blocks [j 2^s, (j + 1) 2^s) (block s from two blocks
// s - 1, depth s); t_i multiplies the aligned blocks that tile [0, i] (left to right, sizes falling)
// and l_i, from the right end (the last two into one) until one value is left.  As the block sizes
// are distinct powers of two, t_i ends at depth ceil(log2(i + 2)).
SeccompPlan seccomp_plan(int n) {
  if (n < 0 || n > 31) fail(COPSE_EINVAL, "comparison of more than 32 bits");
  SeccompPlan P;
  P.n = n;
  std::vector<uint64_t> mask;
  std::vector<int> depth;
  std::map<uint64_t, int> id_of;
  for (int m = 0; m < n; ++m) {
    mask.push_back(1ULL << m);
    depth.push_back(0);
  }
  for (int i = 0; i < n; ++i) {
    mask.push_back(1ULL << (32 + i));
    depth.push_back(0);
  }
  std::vector<SeccompPlan::Prod> order;
  auto prod = [&](int a, int b) {
    const uint64_t k = mask[a] | mask[b];
    auto it = id_of.find(k);
    if (it != id_of.end()) return it->second;
    const int id = (int)mask.size();
    mask.push_back(k);
    depth.push_back(std::max(depth[a], depth[b]) + 1);
    id_of[k] = id;
    order.push_back({id, a, b});
    return id;
  };
  std::function<int(int, int)> block = [&](int s, int j) -> int {
    if (s == 0) return j;
    const int a = block(s - 1, 2 * j);
    const int b = block(s - 1, 2 * j + 1);
    return prod(a, b);
  };
  for (int i = 0; i < n; ++i) {
    std::vector<int> f;
    for (int start = 0; start <= i;) {
      int size = 1, s = 0;
      while (start % (2 * size) == 0 && start + 2 * size <= i + 1) {
        size *= 2;
        ++s;
      }
      f.push_back(block(s, start / size));
      start += size;
    }
    f.push_back(n + i);
    while (f.size() > 1) {
      const int b = f.back();
      f.pop_back();
      const int a = f.back();
      f.pop_back();
      f.push_back(prod(a, b));
    }
    P.terms.push_back(f[0]);
  }
  int rounds = 0;
  for (int t : P.terms) rounds = std::max(rounds, depth[t]);
  P.rounds.resize(rounds);
  for (auto& pr : order) P.rounds[depth[pr.out] - 1].push_back(pr);
  P.n_values = (int)mask.size();
  return P;
}

int seccomp_depth(uint32_t p) {
  int r = 0;
  while ((1u << r) < p) ++r;
  return 1 + r;
}

}  // namespace copse
