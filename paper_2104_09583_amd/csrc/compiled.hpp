// Compiled forest, model and evaluation structures (host side).
#pragma once

#include "internal.hpp"

namespace copse {

struct Node {
  bool leaf;
  int feature;
  uint64_t threshold;
  int label;
  int left, right;
  int level;   // -1 until computed; branch level (leaf 0)
  int index = -1;   // preorder index among branches or among labels
};

struct Compiled {
  copse_public_meta meta;
  std::vector<std::string> label_names;
  std::vector<Node> nodes;
  std::vector<int> roots;
  std::vector<int> branch_nodes;            // node id by branch preorder index
  std::vector<int> label_nodes;             // node id by label preorder index
  std::vector<std::vector<int>> anc;        // per label: ancestor node ids, root..parent
  std::vector<std::vector<int>> side;       // per label: 1 if in the right (true) subtree
  std::vector<int> padded;                  // padded slot -> branch index or -1
  std::vector<std::vector<int>> sel;        // [level-1][label] -> branch index or -1
  std::vector<std::vector<int>> mask;       // [level-1][label]
  std::vector<int> codebook;                // class of each result slot
  std::vector<int> perm;                    // result slot -> original label row (>= labels: padding)
  uint32_t B_in = 0;
};

uint32_t pow2_ceil(uint32_t x);
uint32_t baby_steps(uint32_t n);
std::unique_ptr<Compiled> compile_forest(const char* text, size_t len, uint32_t F, uint32_t prec, uint32_t log_n,
                                         int fold, uint32_t n1R, uint32_t n1L);
// result privacy: shuffle the result slots and pad them with never-selected labels (see compile.cpp)
void privatize(Compiled& C, const uint8_t seed[32], uint32_t n_pad);
// server-side feature replication (queries hold each feature once; see compile.cpp)
void server_replicate(Compiled& C, uint32_t n1F);
// block width and queries per ciphertext from B_in (and the replication input span)
void set_block(Compiled& C);
std::vector<int32_t> needed_rotations(const copse_public_meta& M);
// The comparison's products: with e_m = eq_{p-1-m} and l_i = lt_{p-2-i} (n = p - 1), the terms
// t_i = l_i e_0 ... e_i = lt_k prod_{j > k} eq_j (k = p - 2 - i) in ceil(log2(n + 1)) rounds.  Value
// ids: e_m = m, l_i = n + i, products from 2 n on; rounds[d] holds the products of depth d + 1.
struct SeccompPlan {
  struct Prod {
    int out, a, b;
  };
  std::vector<std::vector<Prod>> rounds;
  std::vector<int> terms;   // id of t_i
  int n = 0, n_values = 0;
};
SeccompPlan seccomp_plan(int n);
// levels the comparison takes: the plaintext layer's switch and the product rounds
int seccomp_depth(uint32_t p);
void replicate_blocks(const copse_public_meta& M, size_t N, const std::vector<int64_t>& vec,
                      std::vector<uint64_t>& slots, uint64_t t);
void query_plane_slots(const copse_public_meta& M, size_t N, const uint32_t* feats, size_t nq, uint32_t plane,
                       std::vector<uint64_t>& slots);
void diagonal_slots(const copse_public_meta& M, size_t N, const std::vector<std::vector<int64_t>>& A, uint32_t k,
                    uint32_t n1, std::vector<uint64_t>& slots, uint64_t t, bool* nonzero);

// Either a plaintext (NTT form) or a ciphertext operand of the model.
struct Operand {
  std::unique_ptr<Plain> pt;
  CtPtr ct;
  bool zero() const { return !pt && !ct; }
};

// Static description of one matrix product of the model: the baby-step offsets (slot order of the
// baby buffer), the giant groups that have terms, and per group its terms (baby slot, diagonal).
struct MatPlan {
  uint32_t n1 = 1;
  bool enc = false;
  std::vector<int32_t> rots;
  std::vector<uint32_t> groups;   // giant groups with at least one nonzero diagonal
  std::vector<const double*> tab;   // [rots][groups] diagonal pointers (null = zero diagonal)
  DBuf tab_buf;                      // device copy of tab
  const double* const* d_tab = nullptr;
};

struct Model {
  std::vector<uint64_t> primes;                 // chain of the context the model was encoded for
  copse_public_meta meta;
  MatPlan plan_R;
  std::vector<MatPlan> plan_L;
  std::vector<int32_t> lvl_rots;
  DBuf lcat_buf;                                // the level plans' tables side by side: [lvl_rots][sum of groups]
  const double* const* d_lcat = nullptr;
  bool encrypted = false;
  int top_level = 0;                            // level of the query planes the comparison reads
  int dec_level = 0, br_level = 0, lvl_level = 0;
  MatPlan plan_F;                               // server-side replication product (meta.server_rep)
  std::vector<Operand> fdiag;
  // comparison operands: plaintext thresholds -> E, C, G, TH plaintexts; encrypted -> TH ciphertexts
  std::vector<Operand> E, C, G, TH;
  std::vector<Operand> rdiag;                   // q diagonals of R_ext (empty when folded)
  std::vector<std::vector<Operand>> ldiag;      // d x (b or q) diagonals of the level matrices
  std::vector<Operand> masks;
  size_t bytes = 0;
  // evaluations without allocation (noalloc.hip): the largest scratch working set seen, and whether one
  // did not fit the scratch array (later calls are then refused before anything is enqueued)
  mutable size_t noalloc_peak = 0;
  mutable bool noalloc_too_big = false;
};

std::unique_ptr<Model> build_model(Context& c, const Compiled& C, const Keys* k, bool encrypt_model,
                                   const uint8_t seed[32]);
// query group (p ciphertexts) -> result ciphertext at level 0
void build_plan(Context& c, MatPlan& P, const std::vector<Operand>& diags, uint32_t n1, bool enc,
                const std::vector<int32_t>* shared_rots);
CtPtr evaluate_group(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes);
CtPtr evaluate_group_plain(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes);
std::vector<CtPtr> evaluate_groups(Context& c, const Model& M, const Keys& k,
                                   const std::vector<std::vector<const Ct*>>& groups);
// EINVAL unless the model, the keys and every query plane belong to this context and fit its chain
void check_evaluation(const Context& c, const Model& M, const Keys& k,
                      const std::vector<std::vector<const Ct*>>& groups);
// evaluate_group with every temporary in the scratch array; the result is written to `out` (level 0,
// 2 polys); returns after the device has finished
void evaluate_group_noalloc(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes,
                            Ct& out);

}  // namespace copse

// Opaque handles of the C ABI.
struct copse_ctx {
  std::unique_ptr<copse::Context> c;
};
struct copse_keys {
  std::unique_ptr<copse::Keys> k;
};
struct copse_compiled {
  std::unique_ptr<copse::Compiled> c;
};
struct copse_model {
  std::unique_ptr<copse::Model> m;
};
struct copse_cts {
  std::vector<copse::CtPtr> v;
};
// captured evaluation (graph.cpp)
struct copse_exec {
  copse::Context* c = nullptr;
  const copse::Model* model = nullptr;
  const copse::Keys* keys = nullptr;
  int groups = 0;
  std::shared_ptr<copse::Pool> arena;
  std::vector<std::vector<copse::CtPtr>> inputs;   // [group][plane] at the top level, one block
  double* input_base = nullptr;
  std::vector<copse::CtPtr> outputs;               // the captured results (level 0)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~copse_exec();
};
namespace copse {
std::unique_ptr<copse_exec> exec_create(Context& c, const Model& model, const Keys& keys, int n_groups);
std::vector<CtPtr> exec_run(copse_exec& e, const std::vector<std::vector<const Ct*>>& queries);
}  // namespace copse
