// Internal declarations of the COPSE gfx950 library.
//
// Residues modulo every prime are held as IEEE doubles with exact integer
// values in [0, q), q < 2^49.  A product a*b mod q is computed exactly with
// the fused multiply-add: h = a*b (rounded), l = fma(a, b, -h) (the exact
// rounding error, so a*b = h + l), k = floor(h * (1/q)) is the quotient up
// to +-1 (|error| < 0.4 because a*b/q < 2^50 and three roundings of 2^-53),
// r = fma(-k, q, h) + l is then an exact integer in [-q, 2q) and one
// conditional add or subtract brings it to [0, q).  On CDNA the fp64 FMA
// issues at full rate while 32-bit integer multiplies do not, which makes
// this the fastest exact 50-bit modular product on the chip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/copse.h"

namespace copse {

constexpr int kMaxPrimes = 48;

struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);

#define COPSE_HIP(x)                                                                  \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      ::copse::fail(COPSE_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ------------------------------------------------------------------ host number theory
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t m);
uint64_t invmod(uint64_t a, uint64_t m);
bool is_prime(uint64_t n);
uint64_t root_of_unity(uint64_t order, uint64_t q);
uint32_t bitrev(uint32_t x, int bits);

// ------------------------------------------------------------------ SHAKE-256 samplers
void shake256(const uint8_t* msg, size_t len, uint8_t* out, size_t outlen);
class ShakeStream {
 public:
  ShakeStream(const uint8_t seed[32], const char* domain, uint64_t obj, uint32_t limb);
  void read(uint8_t* out, size_t n);

 private:
  void permute_block();
  uint64_t st_[25];
  uint8_t buf_[136];
  size_t pos_;
};
void sample_uniform(const uint8_t seed[32], const char* dom, uint64_t obj, uint32_t limb, uint64_t q,
                    size_t n, double* out);
void sample_ternary(const uint8_t seed[32], const char* dom, uint64_t obj, size_t n, int64_t* out);
void sample_cbd21(const uint8_t seed[32], const char* dom, uint64_t obj, size_t n, int64_t* out);

// ------------------------------------------------------------------ device-side descriptors
struct DevPrime {
  double q;
  double qinv;         // fl(1/q)
  const double* fwd;   // psi^bitrev(k), k < N
  const double* inv;   // psi^-bitrev(k), k < N
  double ninv;         // N^-1 mod q
};

// A batched launch works on rows of N values; row r lives at base + rows[r].x * N and is
// reduced modulo prime rows[r].y.
using RowDesc = int2;

// ------------------------------------------------------------------ memory pool
class Pool {
 public:
  // keep_cached: never release cached blocks (a captured graph may still address them)
  explicit Pool(int device, bool keep_cached = false) : device_(device), keep_cached_(keep_cached) {}
  virtual ~Pool();
  virtual void* alloc(size_t bytes);
  virtual void free(void* p);
  size_t held() const { return held_; }
  void trim();
  // bytes handed out and not yet freed, and the most that has been since the last reset_peak
  size_t live_bytes();
  size_t peak_bytes();
  void reset_peak();

 private:
  int device_;
  bool keep_cached_;
  std::map<size_t, std::vector<void*>> cache_;
  std::map<void*, size_t> live_;
  size_t held_ = 0, live_bytes_ = 0, peak_bytes_ = 0;
  std::mutex mu_;
};

struct Context;

// Device buffer owned through the context pool.
class DBuf {
 public:
  DBuf() = default;
  DBuf(Context* c, size_t doubles);
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept;
  ~DBuf() { reset(); }
  void reset();
  double* get() const { return p_; }
  size_t size() const { return n_; }

 private:
  std::shared_ptr<Pool> pool_;   // keeps the pool alive while the buffer lives
  double* p_ = nullptr;
  size_t n_ = 0;
};

// A ciphertext (or a 3-component tensor) in NTT form: [npolys][level+1][N] starting at ptr.
// The storage may be shared by several ciphertexts produced by one batched launch.
struct Ct {
  int level = 0;
  int npolys = 0;
  std::shared_ptr<DBuf> store;
  double* ptr = nullptr;
  size_t n = 0;   // ring dimension
  double* data() const { return ptr; }
  double* poly(int k, size_t N) const { return ptr + (size_t)k * (level + 1) * N; }
  size_t limbs() const { return (size_t)level + 1; }
  size_t words() const { return (size_t)npolys * (level + 1) * n; }
};
using CtPtr = std::unique_ptr<Ct>;

// Profiling counters per kernel class: 0 forward NTT (row pass), 1 forward NTT (column pass),
// 2 inverse NTT (row pass), 3 inverse NTT (column pass), 4 key-switch inner product,
// 5 base conversion, 6 elementwise.
// kernel classes 0..10; 11..14: the evaluation's stages (comparison, reshuffle, levels, aggregation)
// 15: relinearization inner products with the fused row passes, 16: giant-step sums of inner products
constexpr int kProfStage0 = 11;
constexpr int kProfKinds = 17;
struct ProfSlot {
  uint64_t launches = 0;
  double ms = 0;
  double bytes = 0;   // algorithmic bytes
};

struct KSTables;  // per-level base-conversion constants (device)

// Launch-shape knobs that change no result bit (how exact sums are split across launches, workgroups and
// registers); 0 means the built-in choice.  The active values are picked per evaluation from the context's
// table by (log N, top data level, query groups per call) (copse_ctx_set_tuning).
struct Tuning {
  int mm_cap = 0;       // giant groups per register tile of the MatMul inner sums (4..32)
  int mm_waves = 0;     // batch elements per MatMul workgroup when the batch is a multiple of 8 (4 or 8)
  int ks_jobs = 0;      // key-switch inner products per launch (1..32)
  int bridge_wgs = 0;   // workgroup count under which the fused column pass splits its outputs (64..8192)
  int gsum_b = 0;       // batch elements per thread of the giant-step sums (4 or 8)
};
struct TuneEntry {
  uint32_t log_n, top_level, batch_lo, batch_hi;
  int model;   // -1 any, 0 plaintext, 1 encrypted
  Tuning t;
};

struct Context {
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  uint32_t log_n = 0;
  size_t N = 0;
  uint64_t t = 0;
  int L = 0;          // top data level (L+1 data primes)
  int alpha = 0;      // special primes = digit size
  std::vector<uint64_t> primes;   // q_0..q_L, p_0..p_{alpha-1}
  std::vector<uint64_t> psi;      // the device transform's 2N-th roots
  DevPrime* d_primes = nullptr;
  std::vector<double*> tables;
  std::shared_ptr<Pool> pool;
  uint64_t zeta = 0;              // slot root mod t
  std::vector<uint32_t> slot_pos; // slot (r,j) -> natural evaluation index (host encode)
  std::map<int, std::unique_ptr<KSTables>> ks;   // by level
  std::map<std::string, int2*> row_tables;       // cached device row lists
  // set while an evaluation runs without device allocation (noalloc.hip): every buffer comes from `pool`
  // (the scratch array), a row list missing from row_tables is built in the pool for that call only (its
  // host copy kept until the call has synchronized), and the per-level tables must already exist
  bool no_alloc = false;
  std::map<std::string, int2*> call_rows;
  std::vector<std::vector<int2>> call_rows_host;
  std::vector<DBuf> call_row_bufs;
  Tuning tune;                    // active for the evaluation being issued
  std::vector<TuneEntry> tune_table;
  // the table's entry for an evaluation of `batch` query groups of a plaintext or encrypted model (defaults
  // when none matches)
  void select_tuning(int batch, bool encrypted_model);
  bool profiling = false;
  ProfSlot prof[kProfKinds];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kProfKinds];
  std::vector<hipEvent_t> event_cache;

  int n_primes() const { return (int)primes.size(); }
  int special(int r) const { return L + 1 + r; }
  int n_digits(int level) const { return (level + 1 + alpha - 1) / alpha; }
  const int2* rows(const std::string& key, const std::vector<int2>& host);
  KSTables& kstab(int level);
  // constants of the switch from `level` by k primes at once (1 <= k <= min(4, level))
  const struct MsMulti& ms_multi(int level, int k);
  // builds the tables of every level up front (so that no later call has to allocate them)
  void build_level_tables();
  ~Context();
};

struct KSTables {
  // ModUp: per digit j, bconv from the digit's primes to all other primes of P Q_l.
  struct Digit {
    int first, count;                  // data prime range of the digit
    std::vector<int> targets;          // ext-row index (0..nl-1 data, nl.. special) of outputs
    double* d_mult = nullptr;          // [count]  (Q_j/q_i)^-1 mod q_i
    double* d_mat = nullptr;           // [count][targets] (Q_j/q_i) mod p_o
    int2* d_out_rows = nullptr;        // output row descriptors in the ext buffer
    int2* d_in_rows = nullptr;
  };
  std::vector<Digit> digits;
  // ModDown: special primes -> data primes 0..level
  double* d_md_mult = nullptr;   // [alpha] t^-1 (P/p_r)^-1 mod p_r
  double* d_md_mat = nullptr;    // [alpha][nl] (P/p_r) mod q_i
  double* d_md_pinv = nullptr;   // [nl] P^-1 mod q_i
  double* d_md_tpinv = nullptr;  // [nl] t P^-1 mod q_i
  // Modulus switch from this level to level-1
  double* d_ms = nullptr;        // [4 + 2*level]: q_l, t^-1 mod q_l, then per i<l: q_l^-1, t q_l^-1
  // ModDown merged with the switch to level-1 (level >= 1): conversion multipliers of the special rows
  // and (t P)^-1 mod q_l for the top row, [alpha][level + 1] p_r^-1 mod q_i, and the finish factors
  // (P q_l)^-1, t q_l^-1, q_l^-1 mod q_i for i < level; ptop = P mod q_l
  double* d_mm_mult = nullptr;
  double* d_mm_mat = nullptr;
  double* d_mm_m1 = nullptr;
  double* d_mm_m2 = nullptr;
  double* d_mm_m3 = nullptr;
  double mm_ptop = 0.0;
  bool mm_ok = false;            // the merged step's bounds hold for this chain (q_l < 4 q_i for i < l)
  std::map<int, MsMulti> multi;  // switches by k > 1 primes from this level
  std::vector<double*> owned;
};

// Switch from level l by k primes p_m = q_{l-m} (m < k) at once (fused column pass mode 3 and the
// switch finish): mult[k], mat = [k][n_out] D_m mod q_o then the chain constants at k n_out + 4 m + u,
// tab in the single switch's layout with D_k^-1 and t D_k^-1 per output limb; row descriptors of the k
// input rows (m, q_{l-m}) and the n_out = l - k + 1 output rows (o, q_o).
struct MsMulti {
  double* mult = nullptr;
  double* mat = nullptr;
  double* tab = nullptr;
  const int2* in_rows = nullptr;
  const int2* out_rows = nullptr;
};

// ------------------------------------------------------------------ kernel launchers (kernels.hip)
void launch_ntt_fwd(Context& c, double* base, const int2* rows, int nrows);
void launch_ntt_inv(Context& c, double* base, const int2* rows, int nrows);
// split transform for the fused base changes (N = 2^13 .. 2^16, at most 4 input rows)
bool bridge_supported(const Context& c, int n_in);
void launch_ntt_inv_rows(Context& c, double* base, const int2* rows, int nrows);
void launch_ntt_fwd_rows(Context& c, double* base, const int2* rows, int nrows);
// inverse row pass reading row r of job j from src[j] + r * src_stride + src_off (r < rpj), writing the
// jobs' rows contiguously to dst; prime r, or prime_fixed when >= 0; prime_fixed -2: row r is the top
// limb (levels[j]) of polynomial r of job j
// prime_fixed -4: as -2 for the plaintext layer src * mulp (+ addp on polynomial 0)
void launch_ntt_inv_rows_gather(Context& c, double* dst, const std::vector<const double*>& src, int rpj,
                                size_t src_stride, size_t src_off, int prime_fixed,
                                const std::vector<int>* levels = nullptr,
                                const std::vector<const double*>* mulp = nullptr,
                                const std::vector<const double*>* addp = nullptr);
// forward row pass of the ModDown rows w fused with the ModDown finish (as launch_md_finish2)
void launch_ntt_fwd_rows_md_finish(Context& c, const std::vector<double*>& out, const std::vector<const double*>& add,
                                   const std::vector<uint64_t>& gal, const double* acc, const double* w, int nE,
                                   int nl, const double* pinv, const double* tpinv, int add_mode);
// forward row pass of the merged ModDown + switch rows w (l = level of the inputs, l output limbs) fused
// with its finish: out_j[k][i] = acc[2j+k][i] m1_i + add_j[k][i] m3_i - w[2j+k][i] m2_i  (i < l)
// masks (optional): masks[j] (l limbs per poly) is added to the first mask_np polys of out[j]
// add_b (optional): add_j is the product of the ciphertexts add_j and add_b_j (l + 1 limbs each), computed here
void launch_ntt_fwd_rows_mdms_finish(Context& c, const std::vector<double*>& out,
                                     const std::vector<const double*>& add, const double* acc, const double* w,
                                     int nE, int l, const double* m1, const double* m2, const double* m3,
                                     const std::vector<const double*>* masks = nullptr, int mask_np = 0,
                                     const std::vector<const double*>* add_b = nullptr);
// forward row pass of the modulus-switch rows fused with the switch's finish; job j switches from
// levels[j], its rows w[j] = [np][levels[j]][N], its table tabs[j] (as launch_ms_finish_multi)
// mulp (optional): the switch of the plaintext layer in * mulp (+ add on polynomial 0): `add` then holds
// the layer's addends and nothing is added after the switch
void launch_ntt_fwd_rows_ms_finish(Context& c, const std::vector<double*>& out, const std::vector<const double*>& in,
                                   const std::vector<const double*>& w, const std::vector<int>& levels,
                                   const std::vector<const double*>& tabs, int np,
                                   const std::vector<const double*>* add, int add_np,
                                   const std::vector<const double*>* mulp = nullptr);
// One coefficient map of the fused column pass: rows of the input block (index, prime), rows of the
// output block, per-input multipliers and the [n_in][n_out] matrix (mode 0).  chunk0 / ochunk are set by
// the launcher.  Several maps over the same input and output blocks (the digits of a ModUp) run as one
// launch.
struct BridgeDesc {
  const int2* out_rows;
  const int2* in_rows;
  const double* mult;
  const double* mat;
  int n_out, n_in;
  int chunk0, ochunk;
  // set by launch_bridge_set when left empty: the blocks and batch of this map
  const double* in = nullptr;
  double* out = nullptr;
  size_t in_bs = 0, out_bs = 0;
  int nz = -1;
};
struct BridgeSet {
  static constexpr int kMax = 4;
  BridgeDesc d[kMax];
  int n;
};
void launch_bridge_set(Context& c, int mode, double* out_base, const double* in_base, std::vector<BridgeDesc> descs,
                       int batch, size_t in_bs, size_t out_bs);
// mode 0: fast base conversion (as launch_bconv); mode 1: modulus-switch lift of one row (mult = t^-1);
// mode 2: ModDown merged with the modulus switch: n_in = alpha special rows and the top row, mat is
// [alpha][n_out + 1] (the last column for the top prime), see ntt_bridge_kernel
void launch_bridge(Context& c, int mode, double* out_base, const int2* out_rows, int n_out, const double* in_base,
                   const int2* in_rows, int n_in, const double* mult, const double* mat, int batch, size_t in_bs,
                   size_t out_bs);
// out = a op b over rows (same row layout for out, a, b)
void launch_add(Context& c, double* out, const double* a, const double* b, const int2* rows, int nrows);
void launch_sub(Context& c, double* out, const double* a, const double* b, const int2* rows, int nrows);
void launch_neg(Context& c, double* out, const double* a, const int2* rows, int nrows);
void launch_mul(Context& c, double* out, const double* a, const double* b, const int2* rows, int nrows);
void launch_mac(Context& c, double* acc, const double* a, const double* b, const int2* rows, int nrows);
// out[r] = a[r] * s where s = scal[prime of r]
void launch_mul_scalar(Context& c, double* out, const double* a, const double* scal_by_prime,
                       const int2* rows, int nrows);
// ciphertext x plaintext: out_k = a_k * pt for k < npolys (pt rows = limbs), nl limbs
void launch_mul_plain(Context& c, double* out, const double* a, const double* pt, int npolys, int nl);
// acc_k += a_k * pt
void launch_mac_plain(Context& c, double* acc, const double* a, const double* pt, int npolys, int nl);
void launch_tensor(Context& c, double* d, const double* a, const double* b, int nl, bool accumulate);
// out[r] = in[r] after sigma_g in the transform's bit-reversed evaluation order
void launch_automorphism(Context& c, double* out, const double* in, uint64_t g, int nl, int npolys);
// signed small integers (as doubles) -> residues for each prime row
void launch_lift(Context& c, double* out, const double* v, const int2* rows, int nrows);
// base conversion: out rows o < n_out (row desc out_rows) from in rows i < n_in
void launch_bconv(Context& c, double* out_base, const int2* out_rows, int n_out, const double* in_base,
                  const int2* in_rows, int n_in, const double* mult, const double* mat, int batch,
                  size_t in_batch_stride, size_t out_batch_stride);
// key-switch inner product with optional automorphism of the digits
struct KsJob {
  const double* ext;     // [D][nE][N]
  const double* kb;      // key b rows base [D][Ltot][N]
  const double* ka;
  double* acc;           // [2][nE][N]
  uint64_t g;            // Galois element (1 = none)
};
struct KsJobs {
  static constexpr int kMax = 24;
  KsJob j[kMax];
};
void launch_ks_inner(Context& c, const KsJob* jobs, int njobs, int D, int nE, int level,
                     size_t key_digit_stride);
// modulus switch helpers
void launch_ms_prep(Context& c, double* out, const double* top_coef, int npolys, int level,
                    const double* ms_tab);
void launch_ms_finish(Context& c, double* out, const double* in, const double* w, int npolys, int level,
                      const double* ms_tab);
// ModDown finish: out_k[i] = y_k[i] * pinv_i - w_k[i] * tpinv_i (+ an addend, see add_mode)
void launch_moddown_finish(Context& c, double* out, const double* y, size_t y_poly_stride, const double* w,
                           int npolys, int nl, const double* pinv, const double* tpinv,
                           const double* add, size_t add_poly_stride, int add_mode);
void launch_add_const(Context& c, double* a, int nl, double v);

// ------------------------------------------------------------------ batched launchers
constexpr int kPack = 64;
struct Pack { const double* p[kPack]; };
struct MPack { double* p[kPack]; };
struct GPack { uint64_t g[kPack]; };
struct IPack { int v[kPack]; };
struct KsJob2 {
  const double* in;      // input poly (NTT form, nl limbs): the digit's own limbs
  const double* ext;     // [D][nE][N] ModUp output (target rows only)
  const double* kb;
  const double* ka;
  double* acc;           // [2][nE][N]
  uint64_t g;
  // optional (relinearization merged with the switch): the 2 polys of the addend (NTT form, nl limbs);
  // P times their top limb is added to the top data row of acc
  const double* top = nullptr;
  // optional (a product's relinearization without its tensor written): in holds a1 and in_b b1, so the
  // digit rows are a1 (.) b1; top holds a and top_b b, so the addend is (a0 b0, a0 b1 + a1 b0)
  const double* in_b = nullptr;
  const double* top_b = nullptr;
};
struct KsPack {
  static constexpr int kMax = 32;   // 32 x 72 B of kernel arguments
  KsJob2 j[kMax];
};
void launch_gather(Context& c, double* dst, const std::vector<const double*>& src, int rows);
void launch_ptlayer(Context& c, const std::vector<double*>& out, const std::vector<const double*>& a,
                    const std::vector<const double*>& mul, const std::vector<const double*>& add, int nl);
void launch_tensor_multi(Context& c, const std::vector<double*>& d, const std::vector<const double*>& a,
                         const std::vector<const double*>& b, int nl);
void launch_ms_finish_multi(Context& c, const std::vector<double*>& out, const std::vector<const double*>& in,
                            const double* w, int np, int level, const double* tab,
                            const std::vector<const double*>* add = nullptr, int add_np = 0);
// ptop: P mod q_level, the factor of the jobs' top addends
void launch_ks_inner2(Context& c, const std::vector<KsJob2>& jobs, int D, int nE, int level, size_t key_ds,
                      double ptop = 0.0);
// the same for jobs without automorphism (g = 1) whose ext holds the ModUp rows after the column stages
// only: the forward row pass is done inside (relinearizations); extended rows inv_from.. nE - 1 of acc
// are written after the inverse row pass (the rows the ModDown transforms back; nE: none)
void launch_ks_inner_rows(Context& c, const std::vector<KsJob2>& jobs, int D, int nE, int level, size_t key_ds,
                          double ptop, int inv_from);
// Key-switch inner products summed per output (giant steps of a product, one ModDown for their sum).
// Product p has G outputs (batch elements) that share its key sequence: output (p, b) accumulates, over the
// product's steps s, sum_j digit_j(sigma_{g_s}(in_{s,b})) key_{s,j} in the extended basis, plus P times the
// top limb of its addend (2 polys, NTT form, nl limbs) on the top data row.  Batch element b's input,
// ModUp output, accumulator and addend sit at fixed strides from element 0's.
struct GsumStep {
  uint64_t g;           // Galois element
  const double* kb;     // its key [D][Ltot][N]
  const double* ka;
  const double* in;     // batch element 0's rotated input poly (NTT form, nl limbs): the digits' own limbs
  const double* ext;    // batch element 0's ModUp output [D][nE][N]
};
struct GsumProd {
  int first, count;     // its steps
  double* acc;          // batch element 0's accumulator [2][nE][N]
  const double* top;    // batch element 0's addend
  int accum = 0;        // set by the launcher: add to acc (a later chunk of a long product; no top term)
};
void launch_ks_inner_gsum(Context& c, const std::vector<GsumStep>& steps, const std::vector<GsumProd>& prods, int G,
                          size_t in_bs, size_t ext_bs, size_t acc_bs, size_t top_bs, int D, int nE, int level,
                          size_t key_ds, double ptop);
// Per output u: dst_u poly 0 = f0_u + sum_t sigma_{g_t}(c0_t), poly 1 = f1_u (null f: zero), nl limbs.
struct AutoTerm {
  const double* c0;
  uint64_t g;
};
struct AutoOut {
  double* dst;
  const double* f0;
  const double* f1;
  int first, count;
  int accum = 0;        // set by the launcher: add to dst (a later chunk of a long output; no f terms)
};
void launch_auto_sum(Context& c, const std::vector<AutoTerm>& terms, const std::vector<AutoOut>& outs, int nl);
void launch_md_finish2(Context& c, const std::vector<double*>& out, const std::vector<const double*>& add,
                       const std::vector<uint64_t>& gal, const double* acc, const double* w, int nE, int nl,
                       const double* pinv, const double* tpinv, int add_mode);
// MatMul inner sums.  The device table holds kMmTabPad null entries past its end (the kernel fetches
// whole chunks of a row); tab[u * n_groups + s] is the pre-rotated diagonal that multiplies baby step u in giant
// group s (plaintext [nl][N], or ciphertext [2][nl][N] when enc), null when that diagonal is zero.
constexpr int kMmTabPad = 32;
// u0 >= 0: baby step u0 of batch element b is read from b0[b] instead of the baby buffer
void launch_mm_inner(Context& c, double* out, const double* baby, const double* const* tab, int n_u, int n_groups,
                     int G, int nl, size_t baby_slot, size_t baby_b, bool enc, size_t nnz, int u0 = -1,
                     const std::vector<const double*>* b0 = nullptr);
// out_j = sum of terms[j * T .. j * T + T - 1] (canonical, exact)
void launch_sum_terms(Context& c, const std::vector<double*>& out, const std::vector<const double*>& terms, int T,
                      int nl, int rows_per_job);
void launch_seccomp_combine(Context& c, const std::vector<double*>& eq, const std::vector<double*>& lt,
                            const std::vector<const double*>& u, const std::vector<const double*>& xs,
                            const std::vector<const double*>& ts, int nl);

void launch_calib_copy(Context& c, double* dst, const double* src, size_t n);
// plain device copy of n doubles as a kernel (no copy-engine node when captured in a graph)
inline void launch_copy(Context& c, double* dst, const double* src, size_t n) { launch_calib_copy(c, dst, src, n); }

// profiling hooks: prof_end adds the launch's algorithmic bytes (each input and output row of the
// operation touched once; keys counted per job, twiddle tables not counted)
void prof_begin(Context& c, int kind, hipEvent_t* ev);
void prof_end(Context& c, int kind, hipEvent_t ev, double bytes);
void prof_collect(Context& c);

// ------------------------------------------------------------------ evaluation without allocation (noalloc.hip)
// Device address of the library's scratch array on `device` (looked up once per device; the device must be
// current).  Called when a context is created.
void scratch_acquire(int device);

// ------------------------------------------------------------------ BGV operations (bgv.cpp)
struct Keys {
  std::vector<uint64_t> primes;   // chain of the context the keys belong to
  bool has_secret = false;
  DBuf s;          // NTT form over all primes [Ltot][N]
  std::vector<int64_t> s_host;   // ternary coefficients
  DBuf pk_b, pk_a; // NTT form over data primes [L+1][N]
  struct KSK {
    DBuf b, a;     // [D][Ltot][N]
  };
  std::unique_ptr<KSK> relin;
  std::map<uint64_t, std::unique_ptr<KSK>> rot;   // by Galois element
  size_t bytes = 0;
};

struct Plain {
  int level = 0;
  DBuf buf;        // NTT form [level+1][N]
};

uint64_t galois_of(const Context& c, int64_t r);

CtPtr ct_alloc(Context& c, int level, int npolys);
CtPtr ct_copy(Context& c, const Ct& a);
void encode_slots(const Context& c, const uint64_t* slots, std::vector<int64_t>& coeffs_centered);
void decode_poly(const Context& c, const std::vector<uint64_t>& coeffs_mod_t, uint64_t* slots);
std::unique_ptr<Plain> make_plain(Context& c, const std::vector<int64_t>& centered, int level);
std::unique_ptr<Plain> make_plain_slots(Context& c, const uint64_t* slots, int level);

std::unique_ptr<Keys> keygen(Context& c, const uint8_t seed[32], const std::vector<int32_t>& rots, bool relin);
CtPtr encrypt(Context& c, const Keys& k, const std::vector<int64_t>& centered, int level,
              const uint8_t seed[32], uint64_t obj);
void phase_coef(Context& c, const Keys& k, const Ct& a, std::vector<uint64_t>& out);  // [level+1][N] u64

CtPtr op_add(Context& c, const Ct& a, const Ct& b);
CtPtr op_sub(Context& c, const Ct& a, const Ct& b);
CtPtr op_neg(Context& c, const Ct& a);
CtPtr op_mul_int(Context& c, const Ct& a, uint64_t k);
CtPtr op_add_plain(Context& c, const Ct& a, const Plain& p);
CtPtr op_mul_plain(Context& c, const Ct& a, const Plain& p);
CtPtr op_add_const(Context& c, const Ct& a, uint64_t v);
CtPtr op_tensor(Context& c, const Ct& a, const Ct& b);
CtPtr op_modswitch(Context& c, const Ct& a);
CtPtr op_modswitch_to(Context& c, const Ct& a, int level);
CtPtr op_relin(Context& c, const Keys& k, const Ct& a);
CtPtr op_mul(Context& c, const Keys& k, const Ct& a, const Ct& b);
std::vector<CtPtr> op_rotate_hoisted(Context& c, const Keys& k, const Ct& a, const std::vector<int32_t>& rs);
CtPtr op_rotate(Context& c, const Keys& k, const Ct& a, int32_t r);
// sum of rotations of same-level ciphertexts with one ModDown (see bgv.cpp)
CtPtr op_rotate_sum(Context& c, const Keys& k, const std::vector<std::pair<const Ct*, int32_t>>& items);

void to_coef_u64(Context& c, const Ct& a, std::vector<uint64_t>& out);
CtPtr from_coef_u64(Context& c, const uint64_t* data, int level, int npolys);

}  // namespace copse
