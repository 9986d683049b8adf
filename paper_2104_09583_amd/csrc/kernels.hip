// gfx950 kernels: negacyclic NTT / inverse NTT, elementwise modular
// arithmetic, ciphertext tensor, Galois automorphism in the evaluation
// domain, fast base conversion, key-switching inner product and the
// modulus-switch / ModDown finishing steps.
//
// Every kernel works on rows of N residues (fp64, exact integers in [0,q));
// a row descriptor {offset/N, prime index} gives each row's place and
// modulus, so one launch covers all limbs of all polynomials of an
// operation.  Rows are contiguous and each wavefront touches consecutive
// addresses.
#include <algorithm>

#include "internal.hpp"

namespace copse {

// ------------------------------------------------------------------ modular arithmetic in fp64
__device__ __forceinline__ double mod_mul(double a, double b, double q, double qinv) {
  double h = a * b;
  double l = __fma_rn(a, b, -h);
  double k = floor(h * qinv);
  double r = __fma_rn(-k, q, h) + l;
  r = (r < 0.0) ? r + q : r;
  r = (r >= q) ? r - q : r;
  return r;
}
__device__ __forceinline__ double mod_add(double a, double b, double q) {
  double s = a + b;
  return (s >= q) ? s - q : s;
}
__device__ __forceinline__ double mod_sub(double a, double b, double q) {
  double s = a - b;
  return (s < 0.0) ? s + q : s;
}
// reduce an exact integer |v| < 2^52 into [0, q)
__device__ __forceinline__ double mod_reduce(double v, double q, double qinv) {
  double k = floor(v * qinv);
  double r = __fma_rn(-k, q, v);
  r = (r < 0.0) ? r + q : r;
  r = (r >= q) ? r - q : r;
  return r;
}

// ------------------------------------------------------------------ NTT
// Forward transform: Cooley-Tukey butterflies, natural-order input,
// bit-reversed output.  Stage s (0-based, m = 2^s) pairs j and j + t with
// t = N / 2^(s+1); the pair of group i uses psi^bitrev(m + i).  After all
// stages slot k holds a(psi^(2 bitrev(k) + 1)).
// The log N stages run in two passes when N > TILE:
//   pass 1: stages 0..S1-1 on a tile of 2^S1 rows x CW columns of the
//           N = 2^S1 x C matrix view (C = N / 2^S1), columns contiguous;
//   pass 2: stages S1..logN-1 on contiguous blocks of C elements.
// The inverse runs the mirrored Gentleman-Sande butterflies
// (u, v) -> (u + v, (u - v) psi^-bitrev(m + i)) in reverse stage order and
// multiplies by N^-1 in its last pass.
constexpr int kTile = 2048;
constexpr int kThreads = 256;

__device__ __forceinline__ const DevPrime& prime_of(const DevPrime* P, int2 row) { return P[row.y]; }

// pass over columns: stages [0, S1)
template <bool kInverse>
__global__ __launch_bounds__(kThreads) void ntt_cols_kernel(double* __restrict__ base,
                                                            const int2* __restrict__ rows,
                                                            const DevPrime* __restrict__ P, int logN,
                                                            int S1, int scale) {
  __shared__ double sh[kTile];
  const int2 row = rows[blockIdx.y];
  const DevPrime pr = prime_of(P, row);
  const size_t N = (size_t)1 << logN;
  double* a = base + (size_t)row.x * N;
  const int R = 1 << S1;              // rows of the matrix view
  const int CW = kTile >> S1;         // columns per tile
  const size_t C = N >> S1;           // row length of the matrix view
  const size_t c0 = (size_t)blockIdx.x * CW;
  for (int p = threadIdx.x; p < kTile; p += kThreads) {
    int r = p / CW, cc = p % CW;
    sh[p] = a[(size_t)r * C + c0 + cc];
  }
  __syncthreads();
  const int pairs = kTile / 2;
  if (!kInverse) {
    for (int s = 0; s < S1; ++s) {
      const int half = R >> (s + 1);
      const int m = 1 << s;
      for (int u = threadIdx.x; u < pairs; u += kThreads) {
        int cc = u % CW, uu = u / CW;
        int blk = uu / half, off = uu % half;
        int r1 = blk * 2 * half + off, r2 = r1 + half;
        double w = pr.fwd[m + blk];
        double x = sh[r1 * CW + cc], y = sh[r2 * CW + cc];
        double v = mod_mul(y, w, pr.q, pr.qinv);
        sh[r1 * CW + cc] = mod_add(x, v, pr.q);
        sh[r2 * CW + cc] = mod_sub(x, v, pr.q);
      }
      __syncthreads();
    }
  } else {
    for (int s = S1 - 1; s >= 0; --s) {
      const int half = R >> (s + 1);
      const int m = 1 << s;
      for (int u = threadIdx.x; u < pairs; u += kThreads) {
        int cc = u % CW, uu = u / CW;
        int blk = uu / half, off = uu % half;
        int r1 = blk * 2 * half + off, r2 = r1 + half;
        double w = pr.inv[m + blk];
        double x = sh[r1 * CW + cc], y = sh[r2 * CW + cc];
        sh[r1 * CW + cc] = mod_add(x, y, pr.q);
        sh[r2 * CW + cc] = mod_mul(mod_sub(x, y, pr.q), w, pr.q, pr.qinv);
      }
      __syncthreads();
    }
  }
  for (int p = threadIdx.x; p < kTile; p += kThreads) {
    int r = p / CW, cc = p % CW;
    double v = sh[p];
    if (scale) v = mod_mul(v, pr.ninv, pr.q, pr.qinv);
    a[(size_t)r * C + c0 + cc] = v;
  }
}

// pass over contiguous blocks: stages [S1, logN); TILE/C blocks per workgroup
template <bool kInverse>
__global__ __launch_bounds__(kThreads) void ntt_rows_kernel(double* __restrict__ base,
                                                            const int2* __restrict__ rows,
                                                            const DevPrime* __restrict__ P, int logN,
                                                            int S1, int scale) {
  __shared__ double sh[kTile];
  const int2 row = rows[blockIdx.y];
  const DevPrime pr = prime_of(P, row);
  const size_t N = (size_t)1 << logN;
  double* a = base + (size_t)row.x * N;
  const int tile = (int)min((size_t)kTile, N);
  const size_t t0 = (size_t)blockIdx.x * tile;
  for (int p = threadIdx.x; p < tile; p += kThreads) sh[p] = a[t0 + p];
  __syncthreads();
  const int pairs = tile / 2;
  if (!kInverse) {
    for (int s = S1; s < logN; ++s) {
      const int half = (int)(N >> (s + 1));
      const size_t m = (size_t)1 << s;
      for (int u = threadIdx.x; u < pairs; u += kThreads) {
        int blk = u / half, off = u % half;
        int j1 = blk * 2 * half + off, j2 = j1 + half;
        size_t gi = (t0 + j1) / (2 * (size_t)half);
        double w = pr.fwd[m + gi];
        double x = sh[j1], y = sh[j2];
        double v = mod_mul(y, w, pr.q, pr.qinv);
        sh[j1] = mod_add(x, v, pr.q);
        sh[j2] = mod_sub(x, v, pr.q);
      }
      __syncthreads();
    }
  } else {
    for (int s = logN - 1; s >= S1; --s) {
      const int half = (int)(N >> (s + 1));
      const size_t m = (size_t)1 << s;
      for (int u = threadIdx.x; u < pairs; u += kThreads) {
        int blk = u / half, off = u % half;
        int j1 = blk * 2 * half + off, j2 = j1 + half;
        size_t gi = (t0 + j1) / (2 * (size_t)half);
        double w = pr.inv[m + gi];
        double x = sh[j1], y = sh[j2];
        sh[j1] = mod_add(x, y, pr.q);
        sh[j2] = mod_mul(mod_sub(x, y, pr.q), w, pr.q, pr.qinv);
      }
      __syncthreads();
    }
  }
  for (int p = threadIdx.x; p < tile; p += kThreads) {
    double v = sh[p];
    if (scale) v = mod_mul(v, pr.ninv, pr.q, pr.qinv);
    a[t0 + p] = v;
  }
}

static void split_stages(int logN, int& S1) {
  int S2 = logN < 11 ? logN : 11;   // 2^11 = kTile
  S1 = logN - S2;
}

void launch_ntt_fwd(Context& c, double* base, const int2* rows, int nrows) {
  if (nrows <= 0) return;
  hipEvent_t ev;
  prof_begin(c, 0, &ev);
  int logN = (int)c.log_n, S1;
  split_stages(logN, S1);
  size_t N = c.N;
  if (S1 > 0)
    hipLaunchKernelGGL(ntt_cols_kernel<false>, dim3((unsigned)((N >> S1) / (kTile >> S1)), nrows), dim3(kThreads),
                       0, c.stream, base, rows, c.d_primes, logN, S1, 0);
  unsigned tiles = (unsigned)(N > (size_t)kTile ? N / kTile : 1);
  hipLaunchKernelGGL(ntt_rows_kernel<false>, dim3(tiles, nrows), dim3(kThreads), 0, c.stream, base, rows,
                     c.d_primes, logN, S1, 0);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 0, ev, nrows);
}

void launch_ntt_inv(Context& c, double* base, const int2* rows, int nrows) {
  if (nrows <= 0) return;
  hipEvent_t ev;
  prof_begin(c, 1, &ev);
  int logN = (int)c.log_n, S1;
  split_stages(logN, S1);
  size_t N = c.N;
  unsigned tiles = (unsigned)(N > (size_t)kTile ? N / kTile : 1);
  hipLaunchKernelGGL(ntt_rows_kernel<true>, dim3(tiles, nrows), dim3(kThreads), 0, c.stream, base, rows,
                     c.d_primes, logN, S1, S1 == 0 ? 1 : 0);
  if (S1 > 0)
    hipLaunchKernelGGL(ntt_cols_kernel<true>, dim3((unsigned)((N >> S1) / (kTile >> S1)), nrows), dim3(kThreads),
                       0, c.stream, base, rows, c.d_primes, logN, S1, 1);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 1, ev, nrows);
}

// ------------------------------------------------------------------ elementwise
// grid: x over coefficients (256 threads, 1 element each), y over rows
#define EW_PROLOGUE                                          \
  const int2 row = rows[blockIdx.y];                         \
  const DevPrime& pr = P[row.y];                             \
  const size_t N = (size_t)1 << logN;                        \
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; \
  if (i >= N) return;                                        \
  const size_t o = (size_t)row.x * N + i;

__global__ void add_kernel(double* out, const double* a, const double* b, const int2* rows,
                           const DevPrime* P, int logN) {
  EW_PROLOGUE
  out[o] = mod_add(a[o], b[o], pr.q);
}
__global__ void sub_kernel(double* out, const double* a, const double* b, const int2* rows,
                           const DevPrime* P, int logN) {
  EW_PROLOGUE
  out[o] = mod_sub(a[o], b[o], pr.q);
}
__global__ void neg_kernel(double* out, const double* a, const int2* rows, const DevPrime* P, int logN) {
  EW_PROLOGUE
  double v = a[o];
  out[o] = v == 0.0 ? 0.0 : pr.q - v;
}
__global__ void mul_kernel(double* out, const double* a, const double* b, const int2* rows,
                           const DevPrime* P, int logN) {
  EW_PROLOGUE
  out[o] = mod_mul(a[o], b[o], pr.q, pr.qinv);
}
__global__ void mac_kernel(double* acc, const double* a, const double* b, const int2* rows,
                           const DevPrime* P, int logN) {
  EW_PROLOGUE
  acc[o] = mod_add(acc[o], mod_mul(a[o], b[o], pr.q, pr.qinv), pr.q);
}
__global__ void mul_scalar_kernel(double* out, const double* a, const double* scal, const int2* rows,
                                  const DevPrime* P, int logN) {
  EW_PROLOGUE
  out[o] = mod_mul(a[o], scal[row.y], pr.q, pr.qinv);
}
__global__ void lift_kernel(double* out, const double* v, const int2* rows, const DevPrime* P, int logN) {
  EW_PROLOGUE
  out[o] = mod_reduce(v[i], pr.q, pr.qinv);
}

static dim3 ew_grid(const Context& c, int nrows) { return dim3((unsigned)((c.N + 255) / 256), nrows); }

#define EW_LAUNCH(kern, ...)                                                                      \
  do {                                                                                            \
    if (nrows <= 0) return;                                                                       \
    hipEvent_t ev;                                                                                \
    prof_begin(c, 4, &ev);                                                                        \
    hipLaunchKernelGGL(kern, ew_grid(c, nrows), dim3(256), 0, c.stream, __VA_ARGS__, rows, c.d_primes, \
                       (int)c.log_n);                                                             \
    COPSE_HIP(hipGetLastError());                                                                 \
    prof_end(c, 4, ev, nrows);                                                                    \
  } while (0)

void launch_add(Context& c, double* out, const double* a, const double* b, const int2* rows, int nrows) {
  EW_LAUNCH(add_kernel, out, a, b);
}
void launch_sub(Context& c, double* out, const double* a, const double* b, const int2* rows, int nrows) {
  EW_LAUNCH(sub_kernel, out, a, b);
}
void launch_neg(Context& c, double* out, const double* a, const int2* rows, int nrows) {
  EW_LAUNCH(neg_kernel, out, a);
}
void launch_mul(Context& c, double* out, const double* a, const double* b, const int2* rows, int nrows) {
  EW_LAUNCH(mul_kernel, out, a, b);
}
void launch_mac(Context& c, double* acc, const double* a, const double* b, const int2* rows, int nrows) {
  EW_LAUNCH(mac_kernel, acc, a, b);
}
void launch_mul_scalar(Context& c, double* out, const double* a, const double* scal, const int2* rows,
                       int nrows) {
  EW_LAUNCH(mul_scalar_kernel, out, a, scal);
}
void launch_lift(Context& c, double* out, const double* v, const int2* rows, int nrows) {
  EW_LAUNCH(lift_kernel, out, v);
}

// ciphertext (npolys x nl limbs, primes 0..nl-1) times a plaintext (nl limbs)
__global__ void mul_plain_kernel(double* out, const double* a, const double* pt, int nl, int npolys,
                                 const DevPrime* P, int logN, int accumulate) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int limb = blockIdx.y;
  if (i >= N) return;
  const DevPrime& pr = P[limb];
  const double p = pt[(size_t)limb * N + i];
  for (int k = 0; k < npolys; ++k) {
    size_t o = ((size_t)k * nl + limb) * N + i;
    double v = mod_mul(a[o], p, pr.q, pr.qinv);
    out[o] = accumulate ? mod_add(out[o], v, pr.q) : v;
  }
}

void launch_mul_plain(Context& c, double* out, const double* a, const double* pt, int npolys, int nl) {
  hipEvent_t ev;
  prof_begin(c, 4, &ev);
  hipLaunchKernelGGL(mul_plain_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, out, a, pt, nl, npolys, c.d_primes,
                     (int)c.log_n, 0);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 4, ev, nl * npolys);
}
void launch_mac_plain(Context& c, double* acc, const double* a, const double* pt, int npolys, int nl) {
  hipEvent_t ev;
  prof_begin(c, 4, &ev);
  hipLaunchKernelGGL(mul_plain_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, acc, a, pt, nl, npolys, c.d_primes,
                     (int)c.log_n, 1);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 4, ev, nl * npolys);
}

// d = (a0 b0, a0 b1 + a1 b0, a1 b1), optionally accumulated into d
__global__ void tensor_kernel(double* d, const double* a, const double* b, int nl, const DevPrime* P, int logN,
                              int accumulate) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int limb = blockIdx.y;
  if (i >= N) return;
  const DevPrime& pr = P[limb];
  const size_t ps = (size_t)nl * N, o = (size_t)limb * N + i;
  double a0 = a[o], a1 = a[ps + o], b0 = b[o], b1 = b[ps + o];
  double d0 = mod_mul(a0, b0, pr.q, pr.qinv);
  double d1 = mod_add(mod_mul(a0, b1, pr.q, pr.qinv), mod_mul(a1, b0, pr.q, pr.qinv), pr.q);
  double d2 = mod_mul(a1, b1, pr.q, pr.qinv);
  if (accumulate) {
    d0 = mod_add(d[o], d0, pr.q);
    d1 = mod_add(d[ps + o], d1, pr.q);
    d2 = mod_add(d[2 * ps + o], d2, pr.q);
  }
  d[o] = d0;
  d[ps + o] = d1;
  d[2 * ps + o] = d2;
}

void launch_tensor(Context& c, double* d, const double* a, const double* b, int nl, bool accumulate) {
  hipEvent_t ev;
  prof_begin(c, 4, &ev);
  hipLaunchKernelGGL(tensor_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, d, a, b, nl, c.d_primes, (int)c.log_n,
                     accumulate ? 1 : 0);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 4, ev, 3 * nl);
}

__global__ void add_const_kernel(double* a, int nl, double v, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int limb = blockIdx.y;
  if (i >= N) return;
  const DevPrime& pr = P[limb];
  size_t o = (size_t)limb * N + i;
  a[o] = mod_add(a[o], mod_reduce(v, pr.q, pr.qinv), pr.q);
}
void launch_add_const(Context& c, double* a, int nl, double v) {
  hipLaunchKernelGGL(add_const_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, a, nl, v, c.d_primes, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ automorphism (evaluation domain)
// Slot k holds a(psi^e) with e = 2 bitrev(k) + 1.  sigma_g(a)(psi^e) = a(psi^(g e)), so the
// output slot k reads the input slot holding exponent g e mod 2N.
__device__ __forceinline__ uint32_t auto_src(uint32_t k, uint64_t g, int logN) {
  uint32_t e = 2 * (__builtin_bitreverse32(k) >> (32 - logN)) + 1;
  uint64_t ge = (g * e) & ((2ULL << logN) - 1);
  uint32_t idx = (uint32_t)((ge - 1) >> 1);
  return __builtin_bitreverse32(idx) >> (32 - logN);
}

__global__ void automorphism_kernel(double* out, const double* in, uint64_t g, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const size_t r = blockIdx.y;
  out[r * N + i] = in[r * N + auto_src((uint32_t)i, g, logN)];
}

void launch_automorphism(Context& c, double* out, const double* in, uint64_t g, int nl, int npolys) {
  hipLaunchKernelGGL(automorphism_kernel, ew_grid(c, nl * npolys), dim3(256), 0, c.stream, out, in, g, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ fast base conversion
// out_o[c] = sum_i [in_i[c] * mult_i]_{q_i} * mat[i][o]  mod p_o
// grid: x over coefficients, y over output rows, z over batch
__global__ void bconv_kernel(double* out_base, const int2* out_rows, int n_out, const double* in_base,
                             const int2* in_rows, int n_in, const double* mult, const double* mat,
                             const DevPrime* P, int logN, size_t in_bs, size_t out_bs) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int o = blockIdx.y;
  const double* in = in_base + (size_t)blockIdx.z * in_bs;
  double* out = out_base + (size_t)blockIdx.z * out_bs;
  const int2 orow = out_rows[o];
  const DevPrime& po = P[orow.y];
  double acc = 0.0;
  for (int k = 0; k < n_in; ++k) {
    const int2 irow = in_rows[k];
    const DevPrime& pk = P[irow.y];
    double y = mod_mul(in[(size_t)irow.x * N + i], mult[k], pk.q, pk.qinv);
    // y < q_k may exceed p_o: reduce before the product
    double yr = mod_reduce(y, po.q, po.qinv);
    acc = mod_add(acc, mod_mul(yr, mat[k * n_out + o], po.q, po.qinv), po.q);
  }
  out[(size_t)orow.x * N + i] = acc;
}

void launch_bconv(Context& c, double* out_base, const int2* out_rows, int n_out, const double* in_base,
                  const int2* in_rows, int n_in, const double* mult, const double* mat, int batch,
                  size_t in_bs, size_t out_bs) {
  if (n_out <= 0 || batch <= 0) return;
  hipEvent_t ev;
  prof_begin(c, 3, &ev);
  hipLaunchKernelGGL(bconv_kernel, dim3((unsigned)((c.N + 255) / 256), n_out, batch), dim3(256), 0, c.stream,
                     out_base, out_rows, n_out, in_base, in_rows, n_in, mult, mat, c.d_primes, (int)c.log_n, in_bs,
                     out_bs);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 3, ev, (double)n_out * batch);
}

// ------------------------------------------------------------------ key-switch inner product
// acc_0[o] = sum_j ext_j[o](sigma) * kb_j[o],  acc_1[o] = sum_j ext_j[o](sigma) * ka_j[o]
// ext rows o < nl are data primes 0..nl-1, rows nl.. are the special primes.
// grid: x over coefficients, y over ext rows, z over jobs
__global__ void ks_inner_kernel(const KsJobs jobs, int D, int nE, int nl, int L, int logN, size_t key_ds,
                                const DevPrime* P) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int o = blockIdx.y;
  const KsJob jb = jobs.j[blockIdx.z];
  const int prime = o < nl ? o : L + 1 + (o - nl);
  const DevPrime& pr = P[prime];
  const size_t src = jb.g == 1 ? i : auto_src((uint32_t)i, jb.g, logN);
  double a0 = 0.0, a1 = 0.0;
  for (int j = 0; j < D; ++j) {
    double e = jb.ext[((size_t)j * nE + o) * N + src];
    size_t ko = (size_t)j * key_ds + (size_t)prime * N + i;
    a0 = mod_add(a0, mod_mul(e, jb.kb[ko], pr.q, pr.qinv), pr.q);
    a1 = mod_add(a1, mod_mul(e, jb.ka[ko], pr.q, pr.qinv), pr.q);
  }
  jb.acc[(size_t)o * N + i] = a0;
  jb.acc[((size_t)nE + o) * N + i] = a1;
}

void launch_ks_inner(Context& c, const KsJob* jobs, int njobs, int D, int nE, int level, size_t key_ds) {
  for (int first = 0; first < njobs; first += KsJobs::kMax) {
    int cnt = std::min(KsJobs::kMax, njobs - first);
    KsJobs pack;
    for (int k = 0; k < cnt; ++k) pack.j[k] = jobs[first + k];
    hipEvent_t ev;
    prof_begin(c, 2, &ev);
    hipLaunchKernelGGL(ks_inner_kernel, dim3((unsigned)((c.N + 255) / 256), nE, cnt), dim3(256), 0, c.stream, pack,
                       D, nE, level + 1, c.L, (int)c.log_n, key_ds, c.d_primes);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 2, ev, (double)nE * cnt);
  }
}

// ------------------------------------------------------------------ modulus switch
// ms_tab: [0] = q_l (as prime index l), [1] = t^-1 mod q_l, then for i < l: [2+2i] = q_l^-1 mod q_i,
// [3+2i] = t q_l^-1 mod q_i.
// prep: top_coef = coefficient form of limb l of each poly; out[k][i] = (centered z) mod q_i, i < l
__global__ void ms_prep_kernel(double* out, const double* top, int npolys, int l, const double* tab,
                               const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = blockIdx.y;   // target limb
  const int k = blockIdx.z;   // poly
  const DevPrime& pl = P[l];
  const DevPrime& pi = P[i];
  double z = mod_mul(top[(size_t)k * N + c], tab[1], pl.q, pl.qinv);
  if (z > (pl.q - 1.0) * 0.5) z -= pl.q;    // centered in [-(q_l-1)/2, (q_l-1)/2]
  out[((size_t)k * l + i) * N + c] = mod_reduce(z, pi.q, pi.qinv);
}

// finish: out[k][i] = in[k][i] * q_l^-1 - w[k][i] * t q_l^-1  (w = NTT of the prep rows)
__global__ void ms_finish_kernel(double* out, const double* in, const double* w, int npolys, int l,
                                 const double* tab, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = blockIdx.y;
  const int k = blockIdx.z;
  const DevPrime& pi = P[i];
  double x = in[((size_t)k * (l + 1) + i) * N + c];
  double y = w[((size_t)k * l + i) * N + c];
  double v = mod_sub(mod_mul(x, tab[2 + 2 * i], pi.q, pi.qinv), mod_mul(y, tab[3 + 2 * i], pi.q, pi.qinv), pi.q);
  out[((size_t)k * l + i) * N + c] = v;
}

void launch_ms_prep(Context& c, double* out, const double* top, int npolys, int level, const double* tab) {
  hipLaunchKernelGGL(ms_prep_kernel, dim3((unsigned)((c.N + 255) / 256), level, npolys), dim3(256), 0, c.stream,
                     out, top, npolys, level, tab, c.d_primes, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
}
void launch_ms_finish(Context& c, double* out, const double* in, const double* w, int npolys, int level,
                      const double* tab) {
  hipEvent_t ev;
  prof_begin(c, 4, &ev);
  hipLaunchKernelGGL(ms_finish_kernel, dim3((unsigned)((c.N + 255) / 256), level, npolys), dim3(256), 0,
                     c.stream, out, in, w, npolys, level, tab, c.d_primes, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 4, ev, (double)level * npolys);
}

// ------------------------------------------------------------------ ModDown finish
// add_mode 0: nothing added; 1: add[k * adds] added to every poly k; 2: add[(k/2) * adds] added to
// the even polys only (the c0 of each rotation in a batch of (c0, c1) pairs).
__global__ void moddown_finish_kernel(double* out, const double* y, size_t ys, const double* w, int nl,
                                      const double* pinv, const double* tpinv, const double* add, size_t adds,
                                      int add_mode, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = blockIdx.y;
  const int k = blockIdx.z;
  const DevPrime& pi = P[i];
  double yv = y[(size_t)k * ys + (size_t)i * N + c];
  double wv = w[((size_t)k * nl + i) * N + c];
  double v = mod_sub(mod_mul(yv, pinv[i], pi.q, pi.qinv), mod_mul(wv, tpinv[i], pi.q, pi.qinv), pi.q);
  if (add_mode == 1) v = mod_add(v, add[(size_t)k * adds + (size_t)i * N + c], pi.q);
  if (add_mode == 2 && (k & 1) == 0) v = mod_add(v, add[(size_t)(k >> 1) * adds + (size_t)i * N + c], pi.q);
  out[((size_t)k * nl + i) * N + c] = v;
}

void launch_moddown_finish(Context& c, double* out, const double* y, size_t ys, const double* w, int npolys,
                           int nl, const double* pinv, const double* tpinv, const double* add, size_t adds,
                           int add_mode) {
  hipEvent_t ev;
  prof_begin(c, 4, &ev);
  hipLaunchKernelGGL(moddown_finish_kernel, dim3((unsigned)((c.N + 255) / 256), nl, npolys), dim3(256), 0,
                     c.stream, out, y, ys, w, nl, pinv, tpinv, add, adds, add_mode, c.d_primes, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 4, ev, (double)nl * npolys);
}

}  // namespace copse
