/*
 * copse.h -- C ABI of the MI355X (gfx950) library for vectorized secure
 * decision-forest inference (COPSE, Malik et al., PLDI'21).
 *
 * The operations follow the paper's statement of the problem (Section 3.1,
 * "The Players"; Section 3.2, "The Workflow"; Section 5, "COPSE Runtime"):
 * the model owner compiles a forest, the data owner generates keys and
 * encrypts feature vectors, the server evaluates Algorithm 1 (Section 4.3)
 * on ciphertexts, and the data owner decrypts the N-hot label vector
 * (Section 4.1, "Classification Result").  The encryption scheme is BGV over
 * Z_Q[X]/(X^N + 1) with an RNS prime chain (the paper uses HElib's BGV,
 * Section 5); every choice that decides ciphertext bits is fixed in the
 * comments below so an independent implementation reproduces them.
 *
 * Conventions shared by every entry point
 *   - Return value: COPSE_OK (0) or a negative COPSE_E* code; the message of
 *     the calling thread's last failure is returned by copse_last_error().
 *   - Handles are opaque, created by the library and released by the
 *     matching copse_*_destroy (NULL is accepted and ignored).
 *   - Array arguments are HOST pointers borrowed for the duration of the
 *     call unless stated otherwise; caller-sized output buffers are filled
 *     up to the stated size.
 *   - Ciphertexts, keys and encoded models live in device (HBM) memory of the
 *     context's GPU and stay resident until destroyed.
 *   - Work is enqueued on the context's HIP stream; entry points that return
 *     host data synchronize that stream before returning.
 *   - Not thread-safe per context: calls on one context must not overlap.
 *
 * Ciphertext export format (copse_cts_export / copse_cts_import): per
 * ciphertext, a header of 4 uint64 words {n_polys, level, N, reserved=0}
 * followed by n_polys x (level+1) x N coefficients, each the residue in
 * [0, q_i) of the coefficient-domain polynomial modulo prime q_i; polys
 * outermost, then limbs q_0..q_level, then coefficients 0..N-1.
 */
#ifndef COPSE_H
#define COPSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COPSE_OK 0
#define COPSE_EINVAL (-1)     /* malformed input, bad size, out-of-range value  */
#define COPSE_ECAPACITY (-2)  /* layout exceeds N/2 slots or circuit exceeds chain */
#define COPSE_ENOMEM (-3)     /* device or host allocation failed / HBM budget    */
#define COPSE_EDEVICE (-4)    /* HIP runtime error                               */
#define COPSE_ENOISE (-5)     /* decryption noise check failed                   */
#define COPSE_EKEY (-6)       /* a needed Galois or relinearization key is absent */
#define COPSE_ETIMEOUT (-7)   /* copse_server_wait timed out                     */

typedef struct copse_ctx copse_ctx;
typedef struct copse_keys copse_keys;
typedef struct copse_compiled copse_compiled;
typedef struct copse_model copse_model;
typedef struct copse_cts copse_cts;
typedef struct copse_server copse_server;

/*
 * Ring and prime chain.  Ring dimension N = 2^log_n, plaintext modulus t
 * (must satisfy t = 1 mod 2N so there are N slots).  Every prime q is
 * q = k (2 N t) + 1 (so dropping q in a modulus switch keeps the plaintext:
 * q^-1 = 1 mod t) and q < 2^49 (residues are held exactly in fp64, with
 * headroom for lazily reduced intermediates in the transforms).
 * Candidates k(2Nt)+1 are scanned downward in k below exclusive bounds:
 *   1. alpha special primes p_0 > p_1 > ... below special_max;
 *   2. data primes q_1 > ... > q_L (L = n_data_primes - 1) below data_max,
 *      skipping primes already taken;
 *   3. q_0 below q0_max, skipping primes already taken.
 * Primality: Miller-Rabin with witnesses 2..37 (exact for 64-bit inputs).
 * A key-switching digit is alpha consecutive data primes (q_0..q_{alpha-1},
 * ...); a modulus switch drops the highest-index data prime.
 */
typedef struct {
  uint32_t log_n;
  uint64_t t;
  uint32_t n_data_primes;
  uint64_t q0_max;
  uint64_t data_max;
  uint32_t alpha;
  uint64_t special_max;
  int device;            /* HIP device ordinal */
} copse_params;

/* Public facts about a compiled forest that the data owner and the server
 * may learn (Section 7.1, Tables 3-4): K is revealed so the query can be
 * laid out; q, b, m, d and the slot geometry fix the ciphertext shapes. */
typedef struct {
  uint32_t n_features;   /* F */
  uint32_t precision;    /* p, bits per value */
  uint32_t K;            /* maximum feature multiplicity */
  uint32_t q;            /* quantized branching K*F */
  uint32_t b;            /* branches */
  uint32_t m;            /* labels (output slots per query) */
  uint32_t d;            /* levels */
  uint32_t n_trees;
  uint32_t block_w;      /* W: slots per query block, next pow2 >= m+b+q-2 */
  uint32_t queries_per_ct;/* N / W */
  uint32_t n1_R;         /* baby steps of the reshuffle product */
  uint32_t n1_L;         /* baby steps of the level products */
  uint32_t fold;         /* 1: level matrices composed with R (one product less) */
  uint32_t depth;        /* modulus switches the evaluation consumes */
  uint32_t log_n;        /* ring the layout was made for */
  uint32_t server_rep;   /* 1: queries hold each feature once; the server replicates (Section 7.2.1) */
  uint32_t n1_F;         /* baby steps of the replication product */
} copse_public_meta;

/* ---------------------------------------------------------------- context */
/* Creates the prime chain and device tables: the encryption parameters of
 * Section 8.1 (Table 5: security level, modulus bits, key-switching columns),
 * reinterpreted as a ring, an RNS chain within the HE-standard bound and
 * digits of alpha primes.  Also builds every level's key-switching and
 * modulus-switching tables and looks up the scratch array of
 * copse_evaluate_noalloc on params->device.  Ownership: the context owns its
 * stream, tables and memory pool until copse_ctx_destroy.  Errors: EINVAL
 * (t not 1 mod 2N, bounds too small, alpha 0, more than 48 primes), EDEVICE. */
int copse_ctx_create(const copse_params* params, copse_ctx** out);
void copse_ctx_destroy(copse_ctx* ctx);
/* Writes the primes (q_0..q_L then p_0..p_{alpha-1}) to out[0..cap); *n gets
 * the total count.  EINVAL if cap is too small. */
int copse_ctx_primes(const copse_ctx* ctx, uint64_t* out, size_t cap, size_t* n);
/* The HIP stream (hipStream_t) the context enqueues on. */
void* copse_ctx_stream(copse_ctx* ctx);
/* Makes the context enqueue on `stream` (a hipStream_t, or NULL for the
 * context's own stream).  The caller keeps ownership of the stream. */
int copse_ctx_set_stream(copse_ctx* ctx, void* stream);
/* Blocks until all work enqueued on the context's stream has finished. */
int copse_ctx_sync(copse_ctx* ctx);
/* Device bytes currently held by the context's pool (in use + cached). */
size_t copse_ctx_device_bytes(const copse_ctx* ctx);

/* Launch-shape knobs of the evaluation (chosen by an autotuner; none of them
 * changes a result bit: they only split exact sums differently across
 * launches, workgroups and registers).  An evaluation of G query groups on a
 * context with ring 2^log_n and top data level L uses the first entry with
 * that log_n and top_level, batch_lo <= G <= batch_hi and a matching model
 * kind (model: -1 any, 0 plaintext, 1 encrypted); a knob of 0 (or no
 * matching entry) keeps the built-in choice.  Knobs: mm_cap, giant groups per
 * register tile of the MatMul inner sums (4..32; built in: 24 for several
 * groups of a plaintext model, else 12); mm_waves, batch elements per MatMul
 * workgroup when G is a multiple of 8 (4 or 8; built in 8); ks_jobs,
 * key-switch inner products per launch (1..32; built in 32); bridge_wgs, the
 * workgroup count under which the fused column pass of a base change splits
 * its outputs (built in 512); gsum_b, batch elements per thread of the
 * giant-step key-switch sums (4 or 8; built in 8). */
typedef struct {
  uint32_t log_n, top_level, batch_lo, batch_hi;
  int32_t model;
  int32_t mm_cap, mm_waves, ks_jobs, bridge_wgs, gsum_b;
} copse_tune_entry;
/* Replaces the context's table (entries copied; n = 0 clears it).  Errors:
 * EINVAL (null entries with n > 0, a knob out of its range). */
int copse_ctx_set_tuning(copse_ctx* ctx, const copse_tune_entry* entries, size_t n);

/* ---------------------------------------------------------------- compile */
/*
 * Forest compiler (model owner; Section 4.2 and Section 5, "Input
 * Representation").  text: first line label names, then one line per tree in
 * preorder tokens "B <feature> <threshold> <left> <right>" or "L <label>",
 * 0-based.  Branch i decides x[f_i] < t_i (true = right child).  Produces the
 * padded threshold vector (features in order, each group of K slots in
 * ascending branch preorder, sentinel 0), the reshuffle matrix R, the level
 * matrices and masks (label i, level l selects the ancestor at level l,
 * else the ancestor of greatest level below l, else the parent; mask 0 iff
 * the label lies under the selected branch's true child).
 * log_n fixes the slot geometry; n1_R / n1_L = 0 choose 2^ceil(log2 sqrt n).
 * Errors: EINVAL (grammar, feature >= n_features, threshold >= 2^precision,
 * no branches), ECAPACITY (W > N/2).
 */
int copse_forest_compile(const char* text, size_t len, uint32_t n_features, uint32_t precision,
                         uint32_t log_n, int fold, uint32_t n1_R, uint32_t n1_L,
                         copse_compiled** out, copse_public_meta* meta);
/* All compile options at once (the calls above and below are shorthands).
 * server_replication (Section 7.2.1, "Feature padding": the alternative to
 * replicated queries): queries
 * hold each feature once, extended with period F over B_in + F - 1 slots, so
 * the feature multiplicity K is not revealed; the server maps them onto the
 * padded layout with one plaintext matrix product before the comparison (one
 * more level; plaintext models only, W = next pow2 >= B_in + F - 1).
 * n1_F = 0 chooses 2^ceil(log2 sqrt F).  result_privacy: see
 * copse_forest_compile_private. */
typedef struct {
  int fold;
  uint32_t n1_R, n1_L, n1_F;
  int server_replication;
  int result_privacy;
  uint8_t privacy_seed[32];
  uint32_t n_pad;
} copse_compile_options;
int copse_forest_compile_ex(const char* text, size_t len, uint32_t n_features, uint32_t precision, uint32_t log_n,
                            const copse_compile_options* opts, copse_compiled** out, copse_public_meta* meta);
/* Result privacy (Section 7.2.2, "Returning classification bitvectors"): as
 * copse_forest_compile, then the result slots are shuffled by a permutation
 * drawn from `seed` (32 bytes, the model owner's) and padded with n_pad
 * labels that are never selected, folded into the level matrices and masks
 * (no extra homomorphic work, meta->m = labels + n_pad).  The client decodes
 * with copse_compiled_codebook, which the model owner hands over instead of
 * the forest's preorder label order.  Errors: as copse_forest_compile.
 */
int copse_forest_compile_private(const char* text, size_t len, uint32_t n_features, uint32_t precision,
                                 uint32_t log_n, int fold, uint32_t n1_R, uint32_t n1_L, const uint8_t seed[32],
                                 uint32_t n_pad, copse_compiled** out, copse_public_meta* meta);
/* Class index (position in the label-name line) of each of the meta.m result
 * slots, in slot order; *n receives meta.m; out may be null to query n.
 * Errors: EINVAL (null, cap < m). */
int copse_compiled_codebook(const copse_compiled* compiled, uint32_t* out, size_t cap, size_t* n);
void copse_compiled_destroy(copse_compiled* c);
/* Left rotations (slot offsets) whose Galois keys evaluation needs. */
int copse_compiled_rotations(const copse_public_meta* meta, int32_t* out, size_t cap, size_t* n);

/* ---------------------------------------------------------------- keys */
/*
 * Key generation (data owner; Section 3.2, "The Workflow": the data owner
 * holds the secret key, the server receives only what it needs to evaluate).  All randomness comes from SHAKE-256 streams
 * SHAKE256(seed[32] || domain || le64(object) || le32(limb)) read from the
 * start: uniform mod q = 8 bytes LE masked to bitlen(q), accepted if < q;
 * ternary = one byte, 255 rejected, b mod 3 -> {0, 1, -1}; error = centered
 * binomial eta=21 from 6 bytes LE (popcount of bits 0..20 minus bits
 * 21..41).  s: ternary, domain "sk.s".  pk = (-a s + t e, a) over Q_L with
 * a per limb "pk.a", e "pk.e".  A key-switching key from s' has, per digit
 * j, a_j uniform over P Q_L ("ksk.a", object key_id*256+j, limb = global
 * prime index), e_j ("ksk.e"), b_j = -a_j s + t e_j + g_j s' with
 * g_j = P mod q_i on the limbs of digit j, 0 elsewhere.  key_id 0 is the
 * relinearization key (s' = s^2); a rotation key has key_id = its Galois
 * element 5^r mod 2N (s' = s(X^g)).
 * rots: left rotations r (0 < r < N/2) that need keys; relin: nonzero to make
 * the relinearization key.
 */
int copse_keygen(copse_ctx* ctx, const uint8_t seed[32], const int32_t* rots, size_t n_rots,
                 int relin, copse_keys** out);
void copse_keys_destroy(copse_keys* k);
/* Copy without the secret key (what the server receives; Section 3.2, "The
 * Workflow").  Errors: EINVAL (keys of another context). */
int copse_keys_export_eval(copse_ctx* ctx, const copse_keys* k, copse_keys** out);
/* Device bytes held by the keys. */
size_t copse_keys_bytes(const copse_keys* k);

/* ---------------------------------------------------------------- model */
/*
 * Section 5, "COPSE Runtime" (encrypting a model) and Table 1e (the model
 * owner encrypts thresholds, reshuffle and level matrices and masks once).
 * Encodes the compiled model (server-held plaintext model, encrypt_model=0)
 * or encrypts it under `keys` (encrypt_model=1, seed for its randomness).
 * Plaintext slot vectors are encoded as m(X) with slot (r, j) = m(zeta^e),
 * e = 5^j (row 0) or -5^j (row 1) mod 2N, zeta = 3^((t-1)/2N) mod t, and
 * coefficients lifted centered into [-(t-1)/2, (t-1)/2].  The model stays
 * resident on the device.  Errors: ECAPACITY (circuit deeper than the
 * chain), EINVAL (layout made for another ring), EKEY.
 */
int copse_model_encode(copse_ctx* ctx, const copse_compiled* c, const copse_keys* keys,
                       int encrypt_model, const uint8_t seed[32], copse_model** out);
void copse_model_destroy(copse_model* m);
size_t copse_model_bytes(const copse_model* m);

/* ---------------------------------------------------------------- queries */
/*
 * Data owner (Section 3.3, "Step 0: Features": the feature vector is
 * replicated K times; Section 4.1.2, "Representing Non-integral Values":
 * fixed-point values sliced into p bit planes): replicates each feature K times (feature-major), slices the p
 * bit-planes (plane k = bit k), extends each block cyclically (slot s of a
 * block holds padded position s mod q for s < m+b+q-2, 0 beyond), puts
 * query i of the group in block i (row i / (N/2W), offset (i mod N/2W) W),
 * and encrypts each plane at the top level: (pk0 u + t e0 + m,
 * pk1 u + t e1), u ternary "enc.u", e0 "enc.e0", e1 "enc.e1", object
 * (1 << 56) | (group << 32) | plane.  features: [n_queries][n_features]
 * values < 2^p; n_queries <= queries_per_ct.  Result: p ciphertexts.
 */
int copse_query_encrypt(copse_ctx* ctx, const copse_keys* keys, const copse_public_meta* meta,
                        const uint32_t* features, size_t n_queries, const uint8_t seed[32],
                        uint32_t group, copse_cts** out);
void copse_cts_destroy(copse_cts* c);
size_t copse_cts_count(const copse_cts* c);
int copse_cts_level(const copse_cts* c, size_t i);

/* ---------------------------------------------------------------- evaluate */
/*
 * Server: Algorithm 1 on one query group: SecComp of the p planes with the
 * thresholds, the reshuffle product, d level products with the masks, and
 * the product tree; result switched to q_0 (one ciphertext).  Never takes
 * the secret key: `keys` may be an evaluation-only copy.  Schedule (fixes
 * every ciphertext bit): operands at different levels are switched down one
 * prime at a time; sums switch every term to the lowest level first; a
 * ciphertext product is tensor, relinearize, switch; a plaintext product
 * layer is followed by one switch; MatMul = hoisted baby rotations, per
 * giant group the sum of products with pre-rotated diagonals (relinearized
 * once per group when the diagonals are encrypted), a giant rotation, the
 * sum, one switch; the mask is added after that switch; MultAll pairs
 * (0,1),(2,3),... carrying an odd last one up.  Every rotation is in hoisted
 * form: ModUp(c1), the automorphism on each digit, inner product with the
 * key, ModDown, plus the automorphism of c0.  Errors: EKEY, EINVAL.
 */
int copse_evaluate(copse_ctx* ctx, const copse_model* model, const copse_keys* keys,
                   const copse_cts* query, copse_cts** result);
/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid hipMalloc):
 * copse_evaluate without any device allocation or release.  Every temporary of the evaluation lives in one
 * device array of the library, COPSE_NOALLOC_SCRATCH_BYTES (1 GiB) per GPU, held from the library's load
 * until the process ends; the result is written into `result`, an existing handle holding exactly one
 * ciphertext of this ring at level 0 with 2 polynomials (for instance the result of an earlier
 * copse_evaluate on the same model), whose previous contents are overwritten.  The bits equal
 * copse_evaluate's.  The call returns after the evaluation has finished on the device (it waits for the
 * context's stream), so it is not for use under stream capture.  Calls on one GPU share the array: the
 * library serializes them within a process (a call holds the array until its work has finished), and the
 * array keeps the last call's contents.  Requires a context created by copse_ctx_create (which builds the
 * per-level tables and looks up the array).  Errors: ENOMEM when the evaluation's working set exceeds the
 * array (found during the first such call, which then leaves `result` unchanged; later calls with that
 * model are refused before any work is enqueued), EINVAL (shapes, as copse_evaluate, or a wrong `result`),
 * EKEY, EDEVICE. */
#define COPSE_NOALLOC_SCRATCH_BYTES ((size_t)1 << 30)
int copse_evaluate_noalloc(copse_ctx* ctx, const copse_model* model, const copse_keys* keys,
                           const copse_cts* query, copse_cts* result);
/* The unbatched reference path: one homomorphic operation per call (every
 * rotation its own key switch, every product its own launches), same
 * schedule and the same result bits as copse_evaluate. */
int copse_evaluate_plain(copse_ctx* ctx, const copse_model* model, const copse_keys* keys,
                         const copse_cts* query, copse_cts** result);
/* Same for several query groups at once: the groups' ciphertexts travel
 * through every step together (one launch per step for all of them).
 * queries[i] and results[i] belong to group i.  Each result is bit-identical
 * to copse_evaluate on that group alone. */
int copse_evaluate_batch(copse_ctx* ctx, const copse_model* model, const copse_keys* keys,
                         const copse_cts* const* queries, size_t n_groups, copse_cts** results);

/* ---------------------------------------------------------------- captured evaluation
 * The batched evaluation (Algorithm 1, Section 4.3) of one model over a fixed
 * number of query groups, recorded once as a HIP graph on the context's stream
 * and replayed by each run, so that the hundreds of launches of one
 * evaluation cost the host one graph launch.
 *
 * copse_exec_create: runs the schedule once eagerly (on buffers of its own)
 *   and once under stream capture; the model and the evaluation keys must
 *   stay alive while the executor lives.  The executor owns device memory for
 *   the inputs, every temporary and the outputs of one evaluation (about one
 *   batched evaluation's working set) until it is destroyed.  Synchronizes the
 *   context's stream.  Errors: EINVAL (n_groups 0 or above 4096), ENOMEM,
 *   EKEY, EDEVICE.
 * copse_exec_run: queries[i] (n_groups of them, each p fresh encryptions at
 *   the top level as from copse_query_encrypt) are copied in, the graph is
 *   launched and results[i] receives a new ciphertext (level 0) owned by the
 *   caller, bit-identical to copse_evaluate_batch on the same queries.  Work
 *   is enqueued on the context's stream (no synchronization); runs of one
 *   executor are ordered by that stream.  Errors: EINVAL (group count, plane
 *   count or level differs from the capture).
 */
typedef struct copse_exec copse_exec;
int copse_exec_create(copse_ctx* ctx, const copse_model* model, const copse_keys* eval_keys, size_t n_groups,
                      copse_exec** out);
int copse_exec_run(copse_exec* exec, const copse_cts* const* queries, size_t n_groups, copse_cts** results);
void copse_exec_destroy(copse_exec* exec);

/* ---------------------------------------------------------------- decrypt */
/*
 * Data owner (Section 4.1, "Classification Result"; Section 3.2, "The
 * Workflow"): decrypts a level-0 result, checks the noise (the centered
 * phase must stay below q_0 / 2^11, else ENOISE), decodes the slots and
 * writes bits[i*m + j] = label j of query i (0/1; any other value -> ENOISE)
 * for i < n_queries, and checks that each query's vector is N-hot: exactly
 * meta->n_trees ones, one label per tree (else ENOISE; padding labels of a
 * private result are never set).  cap = size of bits.  Errors: EINVAL
 * (layout of another ring, too many queries, small buffer, keys or result of
 * another context), ENOISE.
 */
int copse_decrypt_labels(copse_ctx* ctx, const copse_keys* keys, const copse_public_meta* meta,
                         const copse_cts* result, size_t n_queries, uint8_t* bits, size_t cap);

/* ---------------------------------------------------------------- raw ciphertext ops
 * Used by the parity tests and the benchmark to check each step alone. */
/* Encrypts an arbitrary slot vector slots[2*(N/2)] (values mod t, row-major)
 * at `level` with encryption object `obj`. */
int copse_encrypt_slots(copse_ctx* ctx, const copse_keys* keys, const uint64_t* slots,
                        int level, const uint8_t seed[32], uint64_t obj, copse_cts** out);
/* Decrypts ciphertext i of c (any level) into slots[2*(N/2)] mod t. */
int copse_decrypt_slots(copse_ctx* ctx, const copse_keys* keys, const copse_cts* c, size_t i,
                        uint64_t* slots);
/* Needed size in words for export (NULL buf) and the export itself. */
int copse_cts_export(copse_ctx* ctx, const copse_cts* c, uint64_t* buf, size_t cap, size_t* need);
int copse_cts_import(copse_ctx* ctx, const uint64_t* buf, size_t len, copse_cts** out);

#define COPSE_OP_ADD 1        /* a + b */
#define COPSE_OP_SUB 2        /* a - b */
#define COPSE_OP_TENSOR 3     /* (a0 b0, a0 b1 + a1 b0, a1 b1) */
#define COPSE_OP_RELIN 4      /* 3-poly a -> 2 polys */
#define COPSE_OP_MODSWITCH 5  /* drop the highest prime */
#define COPSE_OP_MUL 6        /* tensor, relinearize, modulus switch */
#define COPSE_OP_ROTATE 7     /* left rotation by arg slots (hoisted form) */
#define COPSE_OP_MUL_PLAIN 8  /* a * encode(slots) */
#define COPSE_OP_ADD_PLAIN 9  /* a + encode(slots) */
/* out = op(a[ia], b[ib]).  b may be NULL for unary ops; slots (2*(N/2)
 * values mod t) is the plaintext operand of *_PLAIN ops. */
int copse_ct_op(copse_ctx* ctx, const copse_keys* keys, int op, const copse_cts* a, size_t ia,
                const copse_cts* b, size_t ib, int32_t arg, const uint64_t* slots, copse_cts** out);
/* Hoisted rotations of a[ia] by rots[0..n) (one ModUp shared): n results. */
int copse_ct_rotate_many(copse_ctx* ctx, const copse_keys* keys, const copse_cts* a, size_t ia,
                         const int32_t* rots, size_t n, copse_cts** out);
/* Negacyclic product of two coefficient vectors modulo the prime with global
 * index `prime` through the device transform: out = a * b mod (X^N+1, q). */
int copse_poly_mul(copse_ctx* ctx, int prime, const uint64_t* a, const uint64_t* b, uint64_t* out);

/* ---------------------------------------------------------------- profiling */
/* When on, the library brackets each launch of the named kernel class with
 * HIP events on the launching stream and accumulates the launch count, the
 * durations and the algorithmic bytes (every input and output row of the
 * operation read or written once; each distinct key's rows counted once per
 * launch; twiddle tables not counted).  kind: 0 = forward NTT row pass, 1 = forward
 * NTT column pass (unfused path), 2 = inverse NTT row pass, 3 = inverse NTT
 * column pass (unfused path), 4 = key-switch inner product, 5 = base
 * conversion (fused with the column passes where available), 6 = other
 * elementwise kernels, 7 = forward row pass with the ModDown finish,
 * 8 = forward row pass with the modulus-switch finish, 9 = MatMul inner sums,
 * 10 = inverse row pass reading ciphertext rows in place; 11..14 = the
 * stages of an evaluation (comparison, reshuffle product, level products with
 * masks, product tree with the final switch: the breakdown of Section 8),
 * bracketed on the evaluating stream, bytes 0; 15 = relinearization inner
 * products with the ModUp's forward and the ModDown's inverse row passes
 * inside, 16 = giant-step sums of key-switch inner products (kind 4 is then
 * the rotations' inner products).  reset clears the counters. */
int copse_profile_enable(copse_ctx* ctx, int on);
int copse_profile_read(copse_ctx* ctx, int kind, uint64_t* launches, double* total_ms,
                       double* bytes, int reset);

/* ---------------------------------------------------------------- serving */
/*
 * Request loop: resident models, encrypted queries admitted while device
 * memory is under hbm_budget_bytes, batched as they arrive (continuous
 * batching across query groups), results in arrival-independent bits.
 * The library starts no thread: a thread blocked in copse_server_wait runs
 * the queued batches (one leader at a time) until its ticket completes;
 * requests submitted meanwhile join the next batch.  Submission and waiting
 * may come from any threads.  copse_server_destroy first finishes every
 * admitted request.
 */
int copse_server_create(copse_ctx* ctx, size_t hbm_budget_bytes, int max_batch, copse_server** out);
void copse_server_destroy(copse_server* s);
/* Registers a model with the evaluation keys it needs (borrowed; both must
 * outlive the server). */
int copse_server_add_model(copse_server* s, const copse_model* m, const copse_keys* eval_keys,
                           int* model_id);
/* Takes ownership of q.  ENOMEM when the request does not fit the budget. */
int copse_server_submit(copse_server* s, int model_id, copse_cts* q, uint64_t* ticket);
/* Waits up to timeout_ms (-1 = forever) for the ticket's result; ETIMEOUT. */
int copse_server_wait(copse_server* s, uint64_t ticket, int timeout_ms, copse_cts** result);
/* Submission-to-completion latency of a finished ticket, in ms. */
int copse_server_latency(copse_server* s, uint64_t ticket, double* ms);

/* ---------------------------------------------------------------- self-test hooks
 * Expose the host samplers so their streams can be checked against an
 * independent SHAKE-256.  kind: 0 uniform mod q (limb = global prime
 * index), 1 ternary, 2 centered binomial. */
int copse_test_shake256(const uint8_t* msg, size_t len, uint8_t* out, size_t outlen);
/* Copies `bytes` bytes between two fresh device buffers with a plain copy
 * kernel: a known-size reference for hardware byte counters. */
int copse_calib_copy(copse_ctx* ctx, size_t bytes);
/* Prime chain of the parameters, computed on the host (no device needed). */
int copse_chain_primes(const copse_params* params, uint64_t* out, size_t cap, size_t* n);
/* Host encoder: slots[2*(N/2)] mod t -> centered coefficients[N]. */
int copse_test_encode(uint32_t log_n, uint64_t t, const uint64_t* slots, int64_t* coeffs);
int copse_test_sample(const uint8_t seed[32], const char* domain, uint64_t obj, uint32_t limb, int kind,
                      uint64_t q, size_t n, int64_t* out);

const char* copse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* COPSE_H */
