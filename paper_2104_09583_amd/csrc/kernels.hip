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
#include <type_traits>

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

// Lazy (signed) residues for the transforms.  With q < 2^49 and |a| < 4q, |b| < q:
//   mul_lazy: k = rint(a b / q) is within 0.5 + 2^-3 of the exact quotient, so
//   r = a b - k q = fma(-k, q, h) + l is an exact integer with |r| < 0.91 q;
//   reduce_sym: x - q rint(x / q) lies in [-q/2, q/2] for |x| < 8 q;
//   canon: maps [-q/2, q/2] to [0, q).
// A radix-8 round grows |x| from q/2 by at most 3 x 0.91 q (forward) or by a
// factor 8 (inverse sums), so one reduce_sym per element and round keeps every
// intermediate below 4 q and every product below 2^101 (exact in fp64).
__device__ __forceinline__ double mul_lazy(double a, double b, double q, double qinv) {
  double h = a * b;
  double l = __fma_rn(a, b, -h);
  double k = rint(h * qinv);
  return __fma_rn(-k, q, h) + l;
}
__device__ __forceinline__ double reduce_sym(double x, double q, double qinv) {
  return __fma_rn(-rint(x * qinv), q, x);
}
__device__ __forceinline__ double canon(double x, double q) { return x < 0.0 ? x + q : x; }

// A load known to be from global memory (not through a flat address).  Flat loads count on the same
// wait counter as LDS and scalar loads, so every LDS wait before a barrier would also wait for them;
// global loads count only on the vector-memory counter.
__device__ __forceinline__ double gload(const double* p) {
  return *(const __attribute__((address_space(1))) double*)(p);
}
// A load of a value that is uniform across the wave from a table no kernel writes (twiddles, row
// descriptors, primes, conversion constants): read through the constant address space, so it is a scalar
// load into scalar registers.
template <class T>
__device__ __forceinline__ T cload(const T* p) {
  static_assert(std::is_scalar<T>::value, "scalar loads take numbers and pointers");
  return *(const __attribute__((address_space(4))) T*)(p);
}
__device__ __forceinline__ int2 cload_row(const int2* p) {
  const int* w = reinterpret_cast<const int*>(p);
  return make_int2(cload(w), cload(w + 1));
}
// the fields of a prime the transforms use (q, 1/q, twiddle tables, N^-1)
__device__ __forceinline__ DevPrime cload_prime(const DevPrime* p) {
  DevPrime r;
  r.q = cload(&p->q);
  r.qinv = cload(&p->qinv);
  r.fwd = cload(&p->fwd);
  r.inv = cload(&p->inv);
  r.ninv = cload(&p->ninv);
  return r;
}
// Workgroup barrier for LDS exchanges: waits for this wave's LDS accesses only, so global loads issued
// before it (the next round's twiddles, an epilogue's operands) stay in flight across it.  The memory
// clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// An LDS exchange among the lanes of one wave: its writes are complete before its next reads are issued
// (no other wave takes part, so no workgroup barrier)
__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// ------------------------------------------------------------------ automorphism (evaluation domain)
// Slot k holds a(psi^e) with e = 2 bitrev(k) + 1.  sigma_g(a)(psi^e) = a(psi^(g e)), so the
// output slot k reads the input slot holding exponent g e mod 2N.
__device__ __forceinline__ uint32_t auto_src(uint32_t k, uint64_t g, int logN) {
  uint32_t e = 2 * (__builtin_bitreverse32(k) >> (32 - logN)) + 1;
  uint64_t ge = (g * e) & ((2ULL << logN) - 1);
  uint32_t idx = (uint32_t)((ge - 1) >> 1);
  return __builtin_bitreverse32(idx) >> (32 - logN);
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

// ------------------------------------------------------------------ register-radix NTT (log N >= 11)
// Column pass: stages 0..S1-1 touch only the 2^S1 elements r*C + c (r < 2^S1, C = N >> S1) of one
// column c, so one thread keeps a whole column in registers and needs no LDS.  Consecutive
// threads take consecutive columns: every load and store of a wavefront is one contiguous run.
__device__ __forceinline__ void bfly_ct(double& x, double& y, double w, double q, double qinv) {
  double v = mul_lazy(y, w, q, qinv);
  double u = x;
  x = u + v;
  y = u - v;
}
__device__ __forceinline__ void bfly_gs(double& x, double& y, double w, double q, double qinv) {
  double u = x, v = y;
  x = u + v;
  y = mul_lazy(u - v, w, q, qinv);
}

template <int S1, bool kInverse>
__global__ __launch_bounds__(64) void ntt_colreg_kernel(double* __restrict__ base, const int2* __restrict__ rows,
                                                       const DevPrime* __restrict__ P, int logN, int scale) {
  constexpr int R = 1 << S1;
  const int2 row = rows[blockIdx.y];
  const DevPrime pr = P[row.y];
  const size_t N = (size_t)1 << logN;
  const size_t C = N >> S1;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double* a = base + (size_t)row.x * N;
  double x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = a[r * C + c];
  if (!kInverse) {
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int half = R >> (s + 1);
#pragma unroll
      for (int g = 0; g < (1 << s); ++g) {
        const double w = pr.fwd[(1 << s) + g];
#pragma unroll
        for (int o = 0; o < half; ++o) bfly_ct(x[g * 2 * half + o], x[g * 2 * half + o + half], w, pr.q, pr.qinv);
      }
    }
  } else {
#pragma unroll
    for (int s = S1 - 1; s >= 0; --s) {
      const int half = R >> (s + 1);
#pragma unroll
      for (int g = 0; g < (1 << s); ++g) {
        const double w = pr.inv[(1 << s) + g];
#pragma unroll
        for (int o = 0; o < half; ++o) bfly_gs(x[g * 2 * half + o], x[g * 2 * half + o + half], w, pr.q, pr.qinv);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = x[r];
    if (scale) v = mul_lazy(v, pr.ninv, pr.q, pr.qinv);
    v = reduce_sym(v, pr.q, pr.qinv);
    // forward: the row pass follows and accepts signed values; inverse: final, canonical
    a[r * C + c] = kInverse ? canon(v, pr.q) : v;
  }
}

// Row pass over a tile of 2048 contiguous elements (stages S1..S1+10): 256 threads x 8 registers.
// Three radix-8 rounds (distances 1024/512/256, 128/64/32, 16/8/4) and one radix-4 round
// (2/1), with the tile exchanged through LDS between rounds.  A thread's 8 elements j0 + d k lie in
// one aligned block of 8d, so the three stages of a round need 1, 2 and 4 twiddles.
__device__ __forceinline__ int lds_idx(int j) { return j + (j >> 4); }
constexpr int kLdsTile = 2048 + 2048 / 16;

__device__ __forceinline__ void radix8_ct(double* x, size_t gb, size_t d, size_t m, const DevPrime& pr) {
  const size_t g0 = gb / (8 * d);
  const double w0 = pr.fwd[m + g0];
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_ct(x[k], x[k + 4], w0, pr.q, pr.qinv);
  const double w1a = pr.fwd[2 * m + 2 * g0], w1b = pr.fwd[2 * m + 2 * g0 + 1];
  bfly_ct(x[0], x[2], w1a, pr.q, pr.qinv);
  bfly_ct(x[1], x[3], w1a, pr.q, pr.qinv);
  bfly_ct(x[4], x[6], w1b, pr.q, pr.qinv);
  bfly_ct(x[5], x[7], w1b, pr.q, pr.qinv);
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_ct(x[2 * k], x[2 * k + 1], pr.fwd[4 * m + 4 * g0 + k], pr.q, pr.qinv);
}
__device__ __forceinline__ void radix8_gs(double* x, size_t gb, size_t d, size_t m, const DevPrime& pr) {
  const size_t g0 = gb / (8 * d);
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_gs(x[2 * k], x[2 * k + 1], pr.inv[4 * m + 4 * g0 + k], pr.q, pr.qinv);
  const double w1a = pr.inv[2 * m + 2 * g0], w1b = pr.inv[2 * m + 2 * g0 + 1];
  bfly_gs(x[0], x[2], w1a, pr.q, pr.qinv);
  bfly_gs(x[1], x[3], w1a, pr.q, pr.qinv);
  bfly_gs(x[4], x[6], w1b, pr.q, pr.qinv);
  bfly_gs(x[5], x[7], w1b, pr.q, pr.qinv);
  const double w0 = pr.inv[m + g0];
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_gs(x[k], x[k + 4], w0, pr.q, pr.qinv);
}

__device__ __forceinline__ void red8(double* x, const DevPrime& pr) {
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = reduce_sym(x[k], pr.q, pr.qinv);
}

template <bool kInverse>
__global__ __launch_bounds__(256) void ntt_rowreg_kernel(double* __restrict__ base, const int2* __restrict__ rows,
                                                        const DevPrime* __restrict__ P, int logN, int S1, int scale) {
  __shared__ double sh[kLdsTile];
  const int2 row = rows[blockIdx.y];
  const DevPrime pr = P[row.y];
  const size_t N = (size_t)1 << logN;
  double* a = base + (size_t)row.x * N;
  const int t = threadIdx.x;
  const size_t t0 = (size_t)blockIdx.x * 2048;
  const size_t mA = (size_t)1 << S1, mB = mA << 3, mC = mA << 6, mD = mA << 9;
  double x[8];
  // round geometry: A: j0 = t, d = 256; B: j0 = (t/32)*256 + t%32, d = 32; C: j0 = (t/4)*32 + t%4, d = 4;
  // D: two groups of 4 at 8t and 8t+4 (distances 2 and 1)
  const int jA = t, jB = (t >> 5) * 256 + (t & 31), jC = (t >> 2) * 32 + (t & 3), jD = 8 * t;
  if (!kInverse) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = a[t0 + jA + 256 * k];
    radix8_ct(x, t0 + jA, 256, mA, pr);
    red8(x, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[lds_idx(jA + 256 * k)] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jB + 32 * k)];
    radix8_ct(x, t0 + jB, 32, mB, pr);
    red8(x, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[lds_idx(jB + 32 * k)] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jC + 4 * k)];
    radix8_ct(x, t0 + jC, 4, mC, pr);
    red8(x, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[lds_idx(jC + 4 * k)] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jD + k)];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const size_t gb = t0 + jD + 4 * u;
      double* y = x + 4 * u;
      const double w = pr.fwd[mD + gb / 4];
      bfly_ct(y[0], y[2], w, pr.q, pr.qinv);
      bfly_ct(y[1], y[3], w, pr.q, pr.qinv);
      bfly_ct(y[0], y[1], pr.fwd[2 * mD + gb / 2], pr.q, pr.qinv);
      bfly_ct(y[2], y[3], pr.fwd[2 * mD + gb / 2 + 1], pr.q, pr.qinv);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) a[t0 + jD + k] = canon(reduce_sym(x[k], pr.q, pr.qinv), pr.q);
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = a[t0 + jD + k];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const size_t gb = t0 + jD + 4 * u;
      double* y = x + 4 * u;
      bfly_gs(y[0], y[1], pr.inv[2 * mD + gb / 2], pr.q, pr.qinv);
      bfly_gs(y[2], y[3], pr.inv[2 * mD + gb / 2 + 1], pr.q, pr.qinv);
      const double w = pr.inv[mD + gb / 4];
      bfly_gs(y[0], y[2], w, pr.q, pr.qinv);
      bfly_gs(y[1], y[3], w, pr.q, pr.qinv);
    }
    red8(x, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[lds_idx(jD + k)] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jC + 4 * k)];
    radix8_gs(x, t0 + jC, 4, mC, pr);
    red8(x, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[lds_idx(jC + 4 * k)] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jB + 32 * k)];
    radix8_gs(x, t0 + jB, 32, mB, pr);
    red8(x, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[lds_idx(jB + 32 * k)] = x[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jA + 256 * k)];
    radix8_gs(x, t0 + jA, 256, mA, pr);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double v = x[k];
      if (scale) v = mul_lazy(v, pr.ninv, pr.q, pr.qinv);
      v = reduce_sym(v, pr.q, pr.qinv);
      a[t0 + jA + 256 * k] = scale ? canon(v, pr.q) : v;
    }
  }
}

// Twiddles of one radix-8 round of a thread whose 8 elements gb + d k (k < 8) lie in one aligned block of
// 8 d at stage offset m (the round's three stages use 1, 2 and 4 of them).
struct Tw8 {
  double w0, w1a, w1b, w2[4];
};
__device__ __forceinline__ Tw8 tw8_load(const double* tab, size_t gb, size_t d, size_t m) {
  const size_t g0 = gb / (8 * d);
  Tw8 w;
  w.w0 = gload(tab + m + g0);
  w.w1a = gload(tab + 2 * m + 2 * g0);
  w.w1b = gload(tab + 2 * m + 2 * g0 + 1);
#pragma unroll
  for (int k = 0; k < 4; ++k) w.w2[k] = gload(tab + 4 * m + 4 * g0 + k);
  return w;
}
__device__ __forceinline__ void radix8_ct_w(double* x, const Tw8& w, const DevPrime& pr) {
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_ct(x[k], x[k + 4], w.w0, pr.q, pr.qinv);
  bfly_ct(x[0], x[2], w.w1a, pr.q, pr.qinv);
  bfly_ct(x[1], x[3], w.w1a, pr.q, pr.qinv);
  bfly_ct(x[4], x[6], w.w1b, pr.q, pr.qinv);
  bfly_ct(x[5], x[7], w.w1b, pr.q, pr.qinv);
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_ct(x[2 * k], x[2 * k + 1], w.w2[k], pr.q, pr.qinv);
}
__device__ __forceinline__ void radix8_gs_w(double* x, const Tw8& w, const DevPrime& pr) {
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_gs(x[2 * k], x[2 * k + 1], w.w2[k], pr.q, pr.qinv);
  bfly_gs(x[0], x[2], w.w1a, pr.q, pr.qinv);
  bfly_gs(x[1], x[3], w.w1a, pr.q, pr.qinv);
  bfly_gs(x[4], x[6], w.w1b, pr.q, pr.qinv);
  bfly_gs(x[5], x[7], w.w1b, pr.q, pr.qinv);
#pragma unroll
  for (int k = 0; k < 4; ++k) bfly_gs(x[k], x[k + 4], w.w0, pr.q, pr.qinv);
}

// Row pass over a tile of 4096 contiguous elements (stages S1..S1+11): 512 threads x 8 registers,
// four radix-8 rounds (distances 2048/1024/512, 256/128/64, 32/16/8, 4/2/1) with three LDS exchanges.
constexpr int kLdsTile4 = 4096 + 4096 / 16;

// One 4096-element tile of the row pass, 512 threads x 8 registers, four radix-8 rounds with LDS
// exchanges between them and one more so that global memory is always touched at t + 512 k (each
// load or store instruction covers 512 consecutive bytes per wave).  Both directions read src[t + 512 k]
// of the tile and leave the values of tile positions t + 512 k in x[k] (signed, not reduced).  gb0 is the
// tile's first index in the row (twiddle groups).  The twiddles of the first two rounds are loaded with
// the data and those of every later round one round ahead, so a small launch waits on memory once.
// With pre given, the forward tile also loads pre[t + 512 k] into y[k] during its third round (an
// epilogue's operand, so that its latency overlaps the transform).
__device__ __forceinline__ void row4_fwd_tile(const double* __restrict__ src, size_t gb0, int S1, const DevPrime& pr,
                                              double* sh, double x[8], const double* pre = nullptr,
                                              double* y = nullptr) {
  const int t = threadIdx.x;
  const size_t mA = (size_t)1 << S1, mB = mA << 3, mC = mA << 6, mD = mA << 9;
  const int jA = t, jB = (t >> 6) * 512 + (t & 63), jC = (t >> 3) * 64 + (t & 7), jD = 8 * t;
  const Tw8 wa = tw8_load(pr.fwd, gb0 + jA, 512, mA);
  const Tw8 wb = tw8_load(pr.fwd, gb0 + jB, 64, mB);
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = gload(src + jA + 512 * k);
  radix8_ct_w(x, wa, pr);
  const Tw8 wc = tw8_load(pr.fwd, gb0 + jC, 8, mC);
  red8(x, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jA + 512 * k)] = x[k];
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jB + 64 * k)];
  radix8_ct_w(x, wb, pr);
  const Tw8 wd = tw8_load(pr.fwd, gb0 + jD, 1, mD);
  red8(x, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jB + 64 * k)] = x[k];
  lds_wave_sync();   // rounds B and C touch the same 512 elements of this wave's block
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jC + 8 * k)];
  if (pre != nullptr) {
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = gload(pre + t + 512 * k);
  }
  radix8_ct_w(x, wc, pr);
  red8(x, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jC + 8 * k)] = x[k];
  lds_wave_sync();   // and so do rounds C and D
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jD + k)];
  radix8_ct_w(x, wd, pr);
  // each thread overwrites only the LDS words it just read
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jD + k)] = x[k];
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jA + 512 * k)];
}

// With vals given, the tile's values at t + 512 k are vals[k] instead of src[t + 512 k].
__device__ __forceinline__ void row4_inv_tile(const double* __restrict__ src, size_t gb0, int S1, const DevPrime& pr,
                                              double* sh, double x[8], const double* vals = nullptr) {
  const int t = threadIdx.x;
  const size_t mA = (size_t)1 << S1, mB = mA << 3, mC = mA << 6, mD = mA << 9;
  const int jA = t, jB = (t >> 6) * 512 + (t & 63), jC = (t >> 3) * 64 + (t & 7), jD = 8 * t;
  const Tw8 wd = tw8_load(pr.inv, gb0 + jD, 1, mD);
  const Tw8 wc = tw8_load(pr.inv, gb0 + jC, 8, mC);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jA + 512 * k)] = vals != nullptr ? vals[k] : gload(src + jA + 512 * k);
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jD + k)];
  radix8_gs_w(x, wd, pr);
  const Tw8 wb = tw8_load(pr.inv, gb0 + jB, 64, mB);
  red8(x, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jD + k)] = x[k];
  lds_wave_sync();   // rounds D and C touch the same 512 elements of this wave's block
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jC + 8 * k)];
  radix8_gs_w(x, wc, pr);
  const Tw8 wa = tw8_load(pr.inv, gb0 + jA, 512, mA);
  red8(x, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jC + 8 * k)] = x[k];
  lds_wave_sync();   // and so do rounds C and B
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jB + 64 * k)];
  radix8_gs_w(x, wb, pr);
  red8(x, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[lds_idx(jB + 64 * k)] = x[k];
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = sh[lds_idx(jA + 512 * k)];
  radix8_gs_w(x, wa, pr);
}

// Two tiles of one row pass at once (the same prime and tile position, so the same twiddles): the rounds of
// both run between the same exchanges, so a workgroup waits at half the barriers per tile and has twice the
// independent work between them.  sh and sh2: one tile buffer each.  The forward pair reads srcA[t + 512 k]
// and srcB[t + 512 k]; the inverse pair takes the tiles' values at t + 512 k in va and vb.  Results as for
// one tile, in x and y.
__device__ __forceinline__ void row4_fwd_tile2(const double* __restrict__ srcA, const double* __restrict__ srcB,
                                               size_t gb0, int S1, const DevPrime& pr, double* sh, double* sh2,
                                               double x[8], double y[8]) {
  const int t = threadIdx.x;
  const size_t mA = (size_t)1 << S1, mB = mA << 3, mC = mA << 6, mD = mA << 9;
  const int jA = t, jB = (t >> 6) * 512 + (t & 63), jC = (t >> 3) * 64 + (t & 7), jD = 8 * t;
  const Tw8 wa = tw8_load(pr.fwd, gb0 + jA, 512, mA);
  const Tw8 wb = tw8_load(pr.fwd, gb0 + jB, 64, mB);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = gload(srcA + jA + 512 * k);
    y[k] = gload(srcB + jA + 512 * k);
  }
  radix8_ct_w(x, wa, pr);
  radix8_ct_w(y, wa, pr);
  const Tw8 wc = tw8_load(pr.fwd, gb0 + jC, 8, mC);
  red8(x, pr);
  red8(y, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jA + 512 * k)] = x[k];
    sh2[lds_idx(jA + 512 * k)] = y[k];
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jB + 64 * k)];
    y[k] = sh2[lds_idx(jB + 64 * k)];
  }
  radix8_ct_w(x, wb, pr);
  radix8_ct_w(y, wb, pr);
  const Tw8 wd = tw8_load(pr.fwd, gb0 + jD, 1, mD);
  red8(x, pr);
  red8(y, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jB + 64 * k)] = x[k];
    sh2[lds_idx(jB + 64 * k)] = y[k];
  }
  lds_wave_sync();   // rounds B and C touch the same 512 elements of this wave's block
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jC + 8 * k)];
    y[k] = sh2[lds_idx(jC + 8 * k)];
  }
  radix8_ct_w(x, wc, pr);
  radix8_ct_w(y, wc, pr);
  red8(x, pr);
  red8(y, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jC + 8 * k)] = x[k];
    sh2[lds_idx(jC + 8 * k)] = y[k];
  }
  lds_wave_sync();   // and so do rounds C and D
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jD + k)];
    y[k] = sh2[lds_idx(jD + k)];
  }
  radix8_ct_w(x, wd, pr);
  radix8_ct_w(y, wd, pr);
  // each thread overwrites only the LDS words it just read
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jD + k)] = x[k];
    sh2[lds_idx(jD + k)] = y[k];
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jA + 512 * k)];
    y[k] = sh2[lds_idx(jA + 512 * k)];
  }
}

__device__ __forceinline__ void row4_inv_tile2(size_t gb0, int S1, const DevPrime& pr, double* sh, double* sh2,
                                               const double va[8], const double vb[8], double x[8], double y[8]) {
  const int t = threadIdx.x;
  const size_t mA = (size_t)1 << S1, mB = mA << 3, mC = mA << 6, mD = mA << 9;
  const int jA = t, jB = (t >> 6) * 512 + (t & 63), jC = (t >> 3) * 64 + (t & 7), jD = 8 * t;
  const Tw8 wd = tw8_load(pr.inv, gb0 + jD, 1, mD);
  const Tw8 wc = tw8_load(pr.inv, gb0 + jC, 8, mC);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jA + 512 * k)] = va[k];
    sh2[lds_idx(jA + 512 * k)] = vb[k];
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jD + k)];
    y[k] = sh2[lds_idx(jD + k)];
  }
  radix8_gs_w(x, wd, pr);
  radix8_gs_w(y, wd, pr);
  const Tw8 wb = tw8_load(pr.inv, gb0 + jB, 64, mB);
  red8(x, pr);
  red8(y, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jD + k)] = x[k];
    sh2[lds_idx(jD + k)] = y[k];
  }
  lds_wave_sync();   // rounds D and C touch the same 512 elements of this wave's block
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jC + 8 * k)];
    y[k] = sh2[lds_idx(jC + 8 * k)];
  }
  radix8_gs_w(x, wc, pr);
  radix8_gs_w(y, wc, pr);
  const Tw8 wa = tw8_load(pr.inv, gb0 + jA, 512, mA);
  red8(x, pr);
  red8(y, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jC + 8 * k)] = x[k];
    sh2[lds_idx(jC + 8 * k)] = y[k];
  }
  lds_wave_sync();   // and so do rounds C and B
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jB + 64 * k)];
    y[k] = sh2[lds_idx(jB + 64 * k)];
  }
  radix8_gs_w(x, wb, pr);
  radix8_gs_w(y, wb, pr);
  red8(x, pr);
  red8(y, pr);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sh[lds_idx(jB + 64 * k)] = x[k];
    sh2[lds_idx(jB + 64 * k)] = y[k];
  }
  lds_barrier();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = sh[lds_idx(jA + 512 * k)];
    y[k] = sh2[lds_idx(jA + 512 * k)];
  }
  radix8_gs_w(x, wa, pr);
  radix8_gs_w(y, wa, pr);
}

template <bool kInverse>
__global__ __launch_bounds__(512) void ntt_rowreg4_kernel(double* __restrict__ base, const int2* __restrict__ rows,
                                                         const DevPrime* __restrict__ P, int logN, int S1, int scale) {
  __shared__ double sh[kLdsTile4];
  const int2 row = rows[blockIdx.y];
  const DevPrime pr = P[row.y];
  const size_t N = (size_t)1 << logN;
  const size_t t0 = (size_t)blockIdx.x * 4096;
  double* a = base + (size_t)row.x * N + t0;
  const int t = threadIdx.x;
  double x[8];
  if (!kInverse) {
    row4_fwd_tile(a, t0, S1, pr, sh, x);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[t + 512 * k] = canon(reduce_sym(x[k], pr.q, pr.qinv), pr.q);
  } else {
    row4_inv_tile(a, t0, S1, pr, sh, x);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double v = x[k];
      if (scale) v = mul_lazy(v, pr.ninv, pr.q, pr.qinv);
      v = reduce_sym(v, pr.q, pr.qinv);
      a[t + 512 * k] = scale ? canon(v, pr.q) : v;
    }
  }
}

// Inverse row pass reading straight from ciphertexts (no gather copy): row r of the launch is row
// r % rpj of job r / rpj, read from src.p[job] + (r % rpj) * src_stride + src_off and written to
// dst + r * N; its prime is prime_fixed, or r % rpj when prime_fixed < 0.
__global__ __launch_bounds__(512) void ntt_rowinv_gather_kernel(double* __restrict__ dst, Pack src, IPack lv, int rpj,
                                                               size_t src_stride, size_t src_off, int prime_fixed,
                                                               const DevPrime* __restrict__ P, int logN, int S1,
                                                               Pack mulp, Pack addp) {
  __shared__ double sh[kLdsTile4];
  const int r = blockIdx.y;
  const int j = r / rpj, sub = r % rpj;
  const size_t N = (size_t)1 << logN;
  // prime_fixed -2: the top limb of job j's polynomial sub, job j at level lv[j];
  // prime_fixed -4: as -2 for the plaintext layer src * mulp (+ addp on polynomial 0), computed here;
  // prime_fixed -3: limb top - m of polynomial sub / src_stride with m = sub % src_stride, where lv[j] =
  //                 top | k << 16 and only m < k is transformed (job j at level top drops k limbs)
  const int top = prime_fixed == -3 ? (lv.v[j] & 0xffff) : lv.v[j];
  int prime, poly;
  if (prime_fixed == -3) {
    const int kmax = (int)src_stride, m = sub % kmax;
    if (m >= (lv.v[j] >> 16)) return;   // uniform per workgroup, before any barrier
    prime = top - m;
    poly = sub / kmax;
  } else {
    prime = prime_fixed <= -2 ? top : prime_fixed >= 0 ? prime_fixed : sub;
    poly = sub;
  }
  const size_t stride = prime_fixed <= -2 ? (size_t)(top + 1) * N : src_stride;
  const size_t off = prime_fixed <= -2 ? (size_t)prime * N : src_off;
  const DevPrime pr = P[prime];
  const size_t t0 = (size_t)blockIdx.x * 4096;
  const double* a = src.p[j] + (size_t)poly * stride + off + t0;
  double x[8];
  if (prime_fixed == -4) {
    const int t = threadIdx.x;
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t o2 = off + t0 + t + 512 * k;
      v[k] = mod_mul(gload(a + t + 512 * k), gload(mulp.p[j] + o2), pr.q, pr.qinv);
      if (poly == 0) v[k] = mod_add(v[k], gload(addp.p[j] + o2), pr.q);
    }
    row4_inv_tile(a, t0, S1, pr, sh, x, v);
  } else if (mulp.p[j] != nullptr) {
    // a product's third polynomial src (.) mulp, computed here (mulp in the layout of src)
    const double* bs = mulp.p[j] + (size_t)poly * stride + off + t0;
    const int t = threadIdx.x;
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = mod_mul(gload(a + t + 512 * k), gload(bs + t + 512 * k), pr.q, pr.qinv);
    row4_inv_tile(a, t0, S1, pr, sh, x, v);
  } else {
    row4_inv_tile(a, t0, S1, pr, sh, x);
  }
  double* o = dst + (size_t)r * N + t0;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[t + 512 * k] = reduce_sym(x[k], pr.q, pr.qinv);
}

// Forward row pass fused with the end of a ModDown (kMode 1) or of a modulus switch (kMode 2).
//   kMode 1: block (tile, i, z = job * 2 + k) transforms w row z * nl + i and writes
//            out_job[k][i] = acc[z][i] P^-1 - w t P^-1  (+ add_job[k][i] when add_mode 1,
//            + add_job[0][i] at the automorphism's source index when add_mode 2 and k = 0)
//   kMode 2: block (tile, i, z = job * np + k) transforms w row z * l + i and writes
//            out_job[k][i] = in_job[k][i] q_l^-1 - w t q_l^-1  (+ add_job[k][i] for k < add_np)
//   kMode 4: as kMode 2 for the switch of a plaintext layer: in_job[k] stands for in_job[k] * mulp_job
//            (+ add_job on k = 0), computed here (no post-switch add)
//   kMode 3: as kMode 1 for a ModDown merged with the switch by q_l (l = nl output limbs, the addend
//            add_job has l + 1 limbs): out_job[k][i] = acc[z][i] mul_i + add_job[k][i] amul_i - w tmul_i
//            with mul = (P q_l)^-1, tmul = t q_l^-1, amul = q_l^-1; when mulp_job is set the addend is
//            polynomial k of the product of the ciphertexts add_job and mulp_job, formed here
// mul/tmul are P^-1 and t P^-1 per limb (kMode 1) or the modulus-switch table (q_l^-1 at 2 + 2 i,
// t q_l^-1 at 3 + 2 i).  Outputs are canonical.
// at most 80 VGPRs: three workgroups per CU, as for the plain row pass
template <int kMode>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) void ntt_rowfwd_finish_kernel(MPack out, Pack in, Pack add, GPack gal, Pack ws,
                                                               Pack tabs, IPack lvs,
                                                               const double* __restrict__ acc,
                                                               const double* __restrict__ w, int nE, int nl_,
                                                               int np, int add_mode, int add_np,
                                                               const double* __restrict__ mul,
                                                               const double* __restrict__ tmul,
                                                               const DevPrime* __restrict__ P, int logN, int S1,
                                                               const double* __restrict__ amul, Pack mulp) {
  __shared__ double sh[kLdsTile4];
  const int i = blockIdx.y, z = blockIdx.z;
  constexpr bool kMd = kMode == 1 || kMode == 3;   // ModDown layout (2 polys per job, accumulator rows)
  const int j = kMd ? (z >> 1) : z / np, k = kMd ? (z & 1) : z % np;
  // kMode 2: job j writes nl = lv[j] & 0xffff limbs per poly from an input with lv[j] >> 16 limbs per poly
  // (nl + 1 when zero: a switch by one prime)
  const int nl = kMd ? nl_ : (lvs.v[j] & 0xffff);
  const int nin = kMd ? 0 : ((lvs.v[j] >> 16) != 0 ? (lvs.v[j] >> 16) : nl + 1);
  if (i >= nl) return;   // uniform per workgroup, before any barrier
  const DevPrime pr = P[i];
  const size_t N = (size_t)1 << logN;
  const size_t t0 = (size_t)blockIdx.x * 4096;
  const int t = threadIdx.x;
  double x[8];
  const double* wrow = kMd ? w + ((size_t)z * nl + i) * N : ws.p[j] + ((size_t)k * nl + i) * N;
  const double* tab = kMd ? nullptr : tabs.p[j];
  const double m1 = kMd ? mul[i] : tab[2 + 2 * i];
  const double m2 = kMd ? tmul[i] : tab[3 + 2 * i];
  const double m3 = kMode == 3 ? amul[i] : 0.0;
  const size_t orow = ((size_t)k * nl + i) * N;
  const double* yrow = kMd ? acc + ((size_t)z * nE + i) * N : in.p[j] + ((size_t)k * nin + i) * N;
  const uint64_t g = kMode == 1 ? gal.g[j] : 1;
  // the epilogue's main operand is loaded during the transform, so its latency overlaps it
  double yv[8];
  row4_fwd_tile(wrow + t0, t0, S1, pr, sh, x, yrow + t0, yv);
  if (kMode == 4) {
    // the plaintext layer's value of this limb (the input's limb i, the plaintexts' limb i)
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const size_t c = (size_t)i * N + t0 + t + 512 * kk;
      yv[kk] = mod_mul(yv[kk], gload(mulp.p[j] + c), pr.q, pr.qinv);
      if (k == 0) yv[kk] = mod_add(yv[kk], gload(add.p[j] + c), pr.q);
    }
  }
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    const size_t c = t0 + t + 512 * kk;
    const double wv = reduce_sym(x[kk], pr.q, pr.qinv);
    double v = mul_lazy(yv[kk], m1, pr.q, pr.qinv) - mul_lazy(wv, m2, pr.q, pr.qinv);
    if (kMode == 3) {
      double av;
      if (mulp.p[j] == nullptr) {
        av = add.p[j][((size_t)k * (nl + 1) + i) * N + c];
      } else {
        // the addend is the product of the ciphertexts add and mulp: its polynomial k (uniform)
        const size_t r0 = (size_t)i * N + c, r1 = ((size_t)(nl + 1) + i) * N + c;
        const double a0 = add.p[j][r0], b0 = mulp.p[j][r0];
        av = k == 0 ? mod_mul(a0, b0, pr.q, pr.qinv)
                    : mod_add(mod_mul(a0, mulp.p[j][r1], pr.q, pr.qinv),
                              mod_mul(add.p[j][r1], b0, pr.q, pr.qinv), pr.q);
      }
      v += mul_lazy(av, m3, pr.q, pr.qinv);
    }
    v = canon(reduce_sym(v, pr.q, pr.qinv), pr.q);
    // kMode 3: an optional mask (the `in` pack, l limbs per poly) on the first add_np polys
    if (kMode == 3 && k < add_np && in.p[j] != nullptr) v = mod_add(v, in.p[j][orow + c], pr.q);
    if (kMode == 1) {
      if (add_mode == 1) v = mod_add(v, add.p[j][orow + c], pr.q);
      if (add_mode == 2 && k == 0) {
        const size_t src = g == 1 ? c : auto_src((uint32_t)c, g, logN);
        v = mod_add(v, add.p[j][(size_t)i * N + src], pr.q);
      }
    } else if (kMode == 2 && k < add_np && add.p[j] != nullptr) {
      v = mod_add(v, add.p[j][orow + c], pr.q);
    }
    out.p[j][orow + c] = v;
  }
}

template <bool kInverse>
static void launch_colreg(Context& c, double* base, const int2* rows, int nrows, int S1, int scale) {
  const unsigned C = (unsigned)(c.N >> S1);
  dim3 grid((C + 63) / 64, nrows), blk(64);
  const int logN = (int)c.log_n;
  switch (S1) {
    case 1: hipLaunchKernelGGL((ntt_colreg_kernel<1, kInverse>), grid, blk, 0, c.stream, base, rows, c.d_primes, logN, scale); break;
    case 2: hipLaunchKernelGGL((ntt_colreg_kernel<2, kInverse>), grid, blk, 0, c.stream, base, rows, c.d_primes, logN, scale); break;
    case 3: hipLaunchKernelGGL((ntt_colreg_kernel<3, kInverse>), grid, blk, 0, c.stream, base, rows, c.d_primes, logN, scale); break;
    case 4: hipLaunchKernelGGL((ntt_colreg_kernel<4, kInverse>), grid, blk, 0, c.stream, base, rows, c.d_primes, logN, scale); break;
    case 5: hipLaunchKernelGGL((ntt_colreg_kernel<5, kInverse>), grid, blk, 0, c.stream, base, rows, c.d_primes, logN, scale); break;
    case 6: hipLaunchKernelGGL((ntt_colreg_kernel<6, kInverse>), grid, blk, 0, c.stream, base, rows, c.d_primes, logN, scale); break;
    default: fail(COPSE_EINVAL, "ring too large for the column pass");
  }
}

static void split_stages(int logN, int& S1) {
  int S2 = logN < 11 ? logN : 11;   // 2^11 = kTile
  S1 = logN - S2;
}

constexpr int kMaxGridY = 65535;

void launch_ntt_fwd(Context& c, double* base, const int2* rows, int nrows) {
  if (nrows <= 0) return;
  if (nrows > kMaxGridY) {
    for (int first = 0; first < nrows; first += kMaxGridY)
      launch_ntt_fwd(c, base, rows + first, std::min(kMaxGridY, nrows - first));
    return;
  }
  hipEvent_t ev;
  int logN = (int)c.log_n, S1;
  split_stages(logN, S1);
  size_t N = c.N;
  if (logN >= 12) {
    const int S1r = logN - 12;
    if (S1r > 0) {
      prof_begin(c, 1, &ev);
      launch_colreg<false>(c, base, rows, nrows, S1r, 0);
      prof_end(c, 1, ev, 2.0 * nrows * (double)c.N * 8.0);
    }
    prof_begin(c, 0, &ev);
    hipLaunchKernelGGL(ntt_rowreg4_kernel<false>, dim3((unsigned)(N / 4096), nrows), dim3(512), 0, c.stream, base,
                       rows, c.d_primes, logN, S1r, 0);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 0, ev, 2.0 * nrows * (double)c.N * 8.0);
    return;
  }
  if (logN == 11) {
    prof_begin(c, 0, &ev);
    hipLaunchKernelGGL(ntt_rowreg_kernel<false>, dim3(1, nrows), dim3(256), 0, c.stream, base, rows, c.d_primes,
                       logN, 0, 0);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 0, ev, 2.0 * nrows * (double)c.N * 8.0);
    return;
  }
  prof_begin(c, 0, &ev);
  if (S1 > 0)
    hipLaunchKernelGGL(ntt_cols_kernel<false>, dim3((unsigned)((N >> S1) / (kTile >> S1)), nrows), dim3(kThreads),
                       0, c.stream, base, rows, c.d_primes, logN, S1, 0);
  unsigned tiles = (unsigned)(N > (size_t)kTile ? N / kTile : 1);
  hipLaunchKernelGGL(ntt_rows_kernel<false>, dim3(tiles, nrows), dim3(kThreads), 0, c.stream, base, rows,
                     c.d_primes, logN, S1, 0);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 0, ev, 2.0 * nrows * (double)c.N * 8.0);
}

void launch_ntt_inv(Context& c, double* base, const int2* rows, int nrows) {
  if (nrows <= 0) return;
  if (nrows > kMaxGridY) {
    for (int first = 0; first < nrows; first += kMaxGridY)
      launch_ntt_inv(c, base, rows + first, std::min(kMaxGridY, nrows - first));
    return;
  }
  hipEvent_t ev;
  int logN = (int)c.log_n, S1;
  split_stages(logN, S1);
  size_t N = c.N;
  if (logN >= 12) {
    const int S1r = logN - 12;
    prof_begin(c, 2, &ev);
    hipLaunchKernelGGL(ntt_rowreg4_kernel<true>, dim3((unsigned)(N / 4096), nrows), dim3(512), 0, c.stream, base,
                       rows, c.d_primes, logN, S1r, S1r == 0 ? 1 : 0);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 2, ev, 2.0 * nrows * (double)c.N * 8.0);
    if (S1r > 0) {
      prof_begin(c, 3, &ev);
      launch_colreg<true>(c, base, rows, nrows, S1r, 1);
      prof_end(c, 3, ev, 2.0 * nrows * (double)c.N * 8.0);
    }
    return;
  }
  if (logN == 11) {
    prof_begin(c, 2, &ev);
    hipLaunchKernelGGL(ntt_rowreg_kernel<true>, dim3(1, nrows), dim3(256), 0, c.stream, base, rows, c.d_primes,
                       logN, 0, 1);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 2, ev, 2.0 * nrows * (double)c.N * 8.0);
    return;
  }
  prof_begin(c, 2, &ev);
  unsigned tiles = (unsigned)(N > (size_t)kTile ? N / kTile : 1);
  hipLaunchKernelGGL(ntt_rows_kernel<true>, dim3(tiles, nrows), dim3(kThreads), 0, c.stream, base, rows,
                     c.d_primes, logN, S1, S1 == 0 ? 1 : 0);
  if (S1 > 0)
    hipLaunchKernelGGL(ntt_cols_kernel<true>, dim3((unsigned)((N >> S1) / (kTile >> S1)), nrows), dim3(kThreads),
                       0, c.stream, base, rows, c.d_primes, logN, S1, 1);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 2, ev, 2.0 * nrows * (double)c.N * 8.0);
}

// ------------------------------------------------------------------ fused column passes + base change
// Every ModUp, ModDown and modulus switch is "inverse transform of some rows, a coefficient-wise map
// to rows of other primes, forward transform of those".  With the two-pass transform the inverse ends
// and the forward begins with the same column pass (stages 0..S1-1 on columns j + C k of the
// 2^S1 x C view), so one kernel runs, per column: the last inverse stages (and the N^-1 scaling) of the
// n_in input rows, the coefficient map, and the first forward stages of each output row.  The row
// passes stay separate (launch_ntt_inv_rows / launch_ntt_fwd_rows).  Maps:
//   kMode 0 (fast base conversion): out_o = sum_k [x_k mult_k]_{p_k} mat[k][o]  mod q_o
//   kMode 1 (modulus switch):       z = [x_0 mult_0]_{p_0} centered,  out_o = z mod q_o
//   kMode 2 (ModDown by P merged with the switch by q_l): inputs are the alpha special rows y_r and the
//            top data row y_l (which already holds P times the addend's top limb); with
//            z_r = [y_r mult_r]_{p_r} (mult_r = t^-1 (P/p_r)^-1) and s_o = sum_r z_r p_r^-1 mod q_o, the
//            ModDown result's top limb times t^-1 is [y_l (t P)^-1 - s_l]_{q_l}; v is its centered value
//            (the switch's lift) and out_o = s_o + v mod q_o for o < l.  mat is [alpha][n_out + 1]
//            (p_r^-1 mod q_o, the last column for q_l), mult[alpha] = (t P)^-1 mod q_l.
//   kMode 3 (switch by k primes at once, exactly as k single switches): inputs m < k are the limbs of
//            p_m = q_{l-m}; with D_m = p_0 ... p_{m-1}, mult_m = (t D_m)^-1 mod p_m, the single switches'
//            lifts are z_m = centered [x_m mult_m - sum_{u<m} z_u D_u D_m^-1]_{p_m} (mat[k n_out + 4 m + u]
//            holds D_u D_m^-1 mod p_m) and out_o = sum_m z_m D_m mod q_o (mat[m n_out + o] = D_m mod q_o);
//            the finish then computes (c - t out) D_k^-1.
// The values handed to the forward stages are any representatives of the residues (|v| <= q/2), so the
// transform's canonical output is the same as that of the unfused steps.
// grid: x over column groups of 64, y over chunks of ochunk outputs (small batches: more blocks, the
// inputs' stages recomputed per chunk), z over the batch (in_bs / out_bs apart).
constexpr int kBridgeIn = 4;
// A workgroup is 64 columns x 4 waves: wave k runs the inverse stages of input row k (k < n_in) and
// leaves [coef * mult_k] in LDS; then the four waves take the outputs of the block's chunk in turn.
// What a wave needs for one output row besides the LDS values: its place, prime and twiddles and its
// column of the conversion matrix.  All uniform (scalar registers); loaded one output ahead so that the
// chain row descriptor -> prime -> twiddles is off the critical path.
template <int S1>
struct BridgeOut {
  int2 row;
  double q, qinv;
  double w[1 << S1];   // fwd twiddles 1 .. 2^S1 - 1 of the first S1 stages
  double m[kBridgeIn];
};
template <int S1, int kMode>
__device__ __forceinline__ BridgeOut<S1> bridge_out_load(const BridgeDesc& d, const DevPrime* __restrict__ P, int o) {
  BridgeOut<S1> b;
  b.row = cload_row(d.out_rows + o);
  const DevPrime po = cload_prime(P + b.row.y);
  b.q = po.q;
  b.qinv = po.qinv;
#pragma unroll
  for (int k = 1; k < (1 << S1); ++k) b.w[k] = cload(po.fwd + k);
  // mode 2: the special rows' column of the [alpha][n_out + 1] matrix
  const int n_conv = kMode == 2 ? d.n_in - 1 : d.n_in;   // mode 3: the k lifts
  const int stride = kMode == 2 ? d.n_out + 1 : d.n_out;
#pragma unroll
  for (int k = 0; k < kBridgeIn; ++k) b.m[k] = (kMode != 1 && k < n_conv) ? cload(d.mat + k * stride + o) : 0.0;
  return b;
}

template <int S1, int kMode>
__global__ __launch_bounds__(256) void ntt_bridge_kernel(BridgeSet set, const DevPrime* __restrict__ P, int logN) {
  constexpr int R = 1 << S1;
  // mode 2 has one more input (the top row) than conversion rows
  constexpr int kSlots = kMode == 2 ? kBridgeIn + 1 : kBridgeIn;
  __shared__ double ys[kSlots][R][64];
  const size_t N = (size_t)1 << logN;
  const size_t C = N >> S1;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const size_t c = (size_t)blockIdx.x * 64 + lane;
  const bool active = c < C;
  // the conversion (digit) this block belongs to: set.d[k] owns grid rows [chunk0, next chunk0)
  int di = 0;
#pragma unroll
  for (int k = 1; k < BridgeSet::kMax; ++k)
    if (k < set.n && (int)blockIdx.y >= set.d[k].chunk0) di = k;
  const BridgeDesc& d = set.d[di];
  if ((int)blockIdx.z >= d.nz) return;   // uniform per workgroup, before the barrier
  const int n_in = d.n_in, n_out = d.n_out;
  const double* in = d.in + (size_t)blockIdx.z * d.in_bs;
  double* out = d.out + (size_t)blockIdx.z * d.out_bs;
  // this wave's outputs: o0 + wv, o0 + wv + 4, ... below o1; the first one's parameters are fetched now
  const int o0 = ((int)blockIdx.y - d.chunk0) * d.ochunk;
  const int o1 = min(n_out, o0 + d.ochunk);
  int o = o0 + wv;
  BridgeOut<S1> cur;
  if (o < o1) cur = bridge_out_load<S1, kMode>(d, P, o);
  // input k < n_in is run by wave k % 4
  for (int ik = wv; ik < n_in && active; ik += 4) {
    const int2 irow = cload_row(d.in_rows + ik);
    const DevPrime pk = cload_prime(P + irow.y);
    const double* a = in + (size_t)irow.x * N;
    double x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = gload(a + r * C + c);
    double wi[R];
#pragma unroll
    for (int k = 1; k < R; ++k) wi[k] = cload(pk.inv + k);
    // N^-1 mult_k mod p_k: one product per coefficient gives the canonical [coef * mult_k]_{p_k}
    const double nm = canon(reduce_sym(mul_lazy(pk.ninv, cload(d.mult + ik), pk.q, pk.qinv), pk.q, pk.qinv), pk.q);
#pragma unroll
    for (int s = S1 - 1; s >= 0; --s) {
      const int half = R >> (s + 1);
#pragma unroll
      for (int g = 0; g < (1 << s); ++g) {
        const double w = wi[(1 << s) + g];
#pragma unroll
        for (int oo = 0; oo < half; ++oo) bfly_gs(x[g * 2 * half + oo], x[g * 2 * half + oo + half], w, pk.q, pk.qinv);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // for S1 <= 3, |x| < 4 p_k, so the lazy product lies in (-p_k, p_k) and canon gives
      // [coef * mult_k]_{p_k}; four stages can reach 8 p_k, so the product is folded back first
      double v = mul_lazy(x[r], nm, pk.q, pk.qinv);
      if (S1 > 3) v = reduce_sym(v, pk.q, pk.qinv);
      v = canon(v, pk.q);
      if (kMode == 1 && v > (pk.q - 1.0) * 0.5) v -= pk.q;
      ys[ik][r][lane] = v;
    }
  }
  lds_barrier();
  if (kMode == 3) {
    // the k lifts of the single switches, one after the other per coefficient; wave w takes rows w, w + 4..
    for (int r = wv; r < R && active; r += 4) {
      double z[kBridgeIn];
#pragma unroll
      for (int m = 0; m < kBridgeIn; ++m) {
        if (m < n_in) {
          const int2 irow = cload_row(d.in_rows + m);
          const double pq = cload(&P[irow.y].q), pqinv = cload(&P[irow.y].qinv);
          double a = ys[m][r][lane];
#pragma unroll
          for (int u = 0; u < kBridgeIn; ++u)
            if (u < m) a -= mul_lazy(z[u], cload(d.mat + n_out * n_in + 4 * m + u), pq, pqinv);
          // |a| < 4 p_m: the symmetric reduction is the centered lift
          z[m] = reduce_sym(a, pq, pqinv);
          ys[m][r][lane] = z[m];
        }
      }
    }
    lds_barrier();
  }
  if (!active) return;
  // mode 2: the switch's centered lift v of the top limb, per coefficient of this thread's column
  double vt[kMode == 2 ? R : 1];
  if (kMode == 2 && o < o1) {
    const int nc = n_in - 1;
    const int2 trow = cload_row(d.in_rows + nc);
    const double ql = cload(&P[trow.y].q), qlinv = cload(&P[trow.y].qinv);
    double mt[kBridgeIn];
#pragma unroll
    for (int k = 0; k < kBridgeIn; ++k) mt[k] = k < nc ? cload(d.mat + k * (n_out + 1) + n_out) : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double sl = 0.0;
#pragma unroll
      for (int k = 0; k < kBridgeIn; ++k)
        if (k < nc) sl += mul_lazy(ys[k][r][lane], mt[k], ql, qlinv);
      // z_r < 2^49, so each lazy product is below 0.6 q_l and |ys_top - sl| < 4 q_l: the symmetric
      // reduction gives the centered representative
      vt[r] = reduce_sym(ys[nc][r][lane] - sl, ql, qlinv);
    }
  }
  for (; o < o1; o += 4) {
    BridgeOut<S1> nxt;
    if (o + 4 < o1) nxt = bridge_out_load<S1, kMode>(d, P, o + 4);
    const double q = cur.q, qinv = cur.qinv;
    double x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (kMode != 1) {
        const int nc = kMode == 2 ? n_in - 1 : n_in;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kBridgeIn; ++k)
          if (k < nc) acc += mul_lazy(ys[k][r][lane], cur.m[k], q, qinv);
        // mode 2: |v| <= q_l / 2 < 2 q_o, so the sum stays below 8 q_o
        if (kMode == 2) acc += vt[r];
        x[r] = reduce_sym(acc, q, qinv);
      } else {
        x[r] = reduce_sym(ys[0][r][lane], q, qinv);
      }
    }
#pragma unroll
    for (int s = 0; s < S1; ++s) {
      const int half = R >> (s + 1);
#pragma unroll
      for (int g = 0; g < (1 << s); ++g) {
        const double w = cur.w[(1 << s) + g];
#pragma unroll
        for (int oo = 0; oo < half; ++oo) bfly_ct(x[g * 2 * half + oo], x[g * 2 * half + oo + half], w, q, qinv);
      }
    }
    double* a = out + (size_t)cur.row.x * N;
#pragma unroll
    for (int r = 0; r < R; ++r) a[r * C + c] = reduce_sym(x[r], q, qinv);
    cur = nxt;
  }
}

bool bridge_supported(const Context& c, int n_in) { return c.log_n >= 13 && c.log_n <= 16 && n_in <= kBridgeIn; }

void launch_bridge_set(Context& c, int mode, double* out_base, const double* in_base, std::vector<BridgeDesc> descs,
                       int batch, size_t in_bs, size_t out_bs) {
  if (descs.empty()) return;
  const int S1 = (int)c.log_n - 12;
  const unsigned C = (unsigned)(c.N >> S1);
  const unsigned xb = (C + 63) / 64;
  for (size_t first = 0; first < descs.size(); first += BridgeSet::kMax) {
    BridgeSet set{};
    set.n = (int)std::min<size_t>(BridgeSet::kMax, descs.size() - first);
    int rows_y = 0, zmax = 0;
    double bytes = 0;
    for (int k = 0; k < set.n; ++k) {
      BridgeDesc d = descs[first + k];
      if (d.nz < 0) {
        d.in = in_base;
        d.out = out_base;
        d.in_bs = in_bs;
        d.out_bs = out_bs;
        d.nz = batch;
      }
      if (d.nz > kMaxGridY) fail(COPSE_EINVAL, "internal: batch too large for one fused column pass");
      if (!bridge_supported(c, mode == 2 ? d.n_in - 1 : d.n_in))
        fail(COPSE_EINVAL, "internal: fused column pass not available for this ring");
      if (mode == 1 && d.n_in != 1) fail(COPSE_EINVAL, "internal: modulus-switch map takes one row");
      if (mode == 2 && d.n_in < 2) fail(COPSE_EINVAL, "internal: merged switch needs special rows and the top row");
      if (mode == 3 && d.n_in < 1) fail(COPSE_EINVAL, "internal: switch by no prime");
      if (d.n_out <= 0) fail(COPSE_EINVAL, "internal: conversion without outputs");
      // at least ~512 workgroups (2048 waves) when the batch is small, by splitting the outputs into chunks
      // of at least 4 (one per wave)
      int chunks = 1;
      const size_t target = c.tune.bridge_wgs > 0 ? (size_t)c.tune.bridge_wgs : 512;
      while (chunks * 8 <= d.n_out && (size_t)xb * d.nz * chunks * set.n < target) chunks *= 2;
      d.ochunk = (d.n_out + chunks - 1) / chunks;
      chunks = (d.n_out + d.ochunk - 1) / d.ochunk;
      d.chunk0 = rows_y;
      rows_y += chunks;
      zmax = std::max(zmax, d.nz);
      set.d[k] = d;
      bytes += (double)(d.n_out + d.n_in) * d.nz * (double)c.N * 8.0;   // inputs counted once
    }
    if (zmax == 0) continue;
    hipEvent_t ev;
    prof_begin(c, 5, &ev);
    dim3 grid(xb, rows_y, zmax), blk(256);
#define COPSE_BRIDGE(S, M) hipLaunchKernelGGL((ntt_bridge_kernel<S, M>), grid, blk, 0, c.stream, set, c.d_primes, (int)c.log_n)
    if (mode == 0) {
      switch (S1) {
        case 1: COPSE_BRIDGE(1, 0); break;
        case 2: COPSE_BRIDGE(2, 0); break;
        case 3: COPSE_BRIDGE(3, 0); break;
        default: COPSE_BRIDGE(4, 0); break;
      }
    } else if (mode == 1) {
      switch (S1) {
        case 1: COPSE_BRIDGE(1, 1); break;
        case 2: COPSE_BRIDGE(2, 1); break;
        case 3: COPSE_BRIDGE(3, 1); break;
        default: COPSE_BRIDGE(4, 1); break;
      }
    } else if (mode == 2) {
      switch (S1) {
        case 1: COPSE_BRIDGE(1, 2); break;
        case 2: COPSE_BRIDGE(2, 2); break;
        case 3: COPSE_BRIDGE(3, 2); break;
        default: COPSE_BRIDGE(4, 2); break;
      }
    } else {
      switch (S1) {
        case 1: COPSE_BRIDGE(1, 3); break;
        case 2: COPSE_BRIDGE(2, 3); break;
        case 3: COPSE_BRIDGE(3, 3); break;
        default: COPSE_BRIDGE(4, 3); break;
      }
    }
#undef COPSE_BRIDGE
    COPSE_HIP(hipGetLastError());
    prof_end(c, 5, ev, bytes);
  }
}

void launch_bridge(Context& c, int mode, double* out_base, const int2* out_rows, int n_out, const double* in_base,
                   const int2* in_rows, int n_in, const double* mult, const double* mat, int batch, size_t in_bs,
                   size_t out_bs) {
  if (n_out <= 0 || batch <= 0) return;
  // batches beyond one launch's z range run in slices
  for (int first = 0; first < batch; first += kMaxGridY) {
    BridgeDesc d{out_rows, in_rows, mult, mat, n_out, n_in, 0, 0};
    d.in = in_base + (size_t)first * in_bs;
    d.out = out_base + (size_t)first * out_bs;
    d.in_bs = in_bs;
    d.out_bs = out_bs;
    d.nz = std::min(kMaxGridY, batch - first);
    launch_bridge_set(c, mode, out_base, in_base, {d}, batch, in_bs, out_bs);
  }
}

// row passes alone (the column passes are done by the bridge): inverse rows leave signed residues for
// the bridge, forward rows take the bridge's output and finish the transform (canonical)
void launch_ntt_inv_rows(Context& c, double* base, const int2* rows, int nrows) {
  if (nrows <= 0) return;
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  for (int first = 0; first < nrows; first += kMaxGridY) {
    const int cnt = std::min(kMaxGridY, nrows - first);
    hipEvent_t ev;
    prof_begin(c, 2, &ev);
    hipLaunchKernelGGL(ntt_rowreg4_kernel<true>, dim3((unsigned)(c.N / 4096), cnt), dim3(512), 0, c.stream, base,
                       rows + first, c.d_primes, (int)c.log_n, (int)c.log_n - 12, 0);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 2, ev, 2.0 * cnt * (double)c.N * 8.0);
  }
}

void launch_ntt_fwd_rows(Context& c, double* base, const int2* rows, int nrows) {
  if (nrows <= 0) return;
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  for (int first = 0; first < nrows; first += kMaxGridY) {
    const int cnt = std::min(kMaxGridY, nrows - first);
    hipEvent_t ev;
    prof_begin(c, 0, &ev);
    hipLaunchKernelGGL(ntt_rowreg4_kernel<false>, dim3((unsigned)(c.N / 4096), cnt), dim3(512), 0, c.stream, base,
                       rows + first, c.d_primes, (int)c.log_n, (int)c.log_n - 12, 0);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 0, ev, 2.0 * cnt * (double)c.N * 8.0);
  }
}

void launch_ntt_inv_rows_gather(Context& c, double* dst, const std::vector<const double*>& src, int rpj,
                                size_t src_stride, size_t src_off, int prime_fixed, const std::vector<int>* levels,
                                const std::vector<const double*>* mulp, const std::vector<const double*>* addp) {
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  if (prime_fixed <= -2 && (!levels || levels->size() != src.size())) fail(COPSE_EINVAL, "internal: levels");
  if (prime_fixed == -3 && (src_stride == 0 || rpj % (int)src_stride != 0)) fail(COPSE_EINVAL, "internal: limbs");
  if (prime_fixed == -4 && (!mulp || !addp || mulp->size() != src.size() || addp->size() != src.size()))
    fail(COPSE_EINVAL, "internal: plaintext layer operands");
  const int per = std::max(1, std::min(kPack, kMaxGridY / std::max(1, rpj)));
  for (size_t first = 0; first < src.size(); first += per) {
    const int cnt = (int)std::min<size_t>(per, src.size() - first);
    Pack pk, pm{}, pa{};
    IPack lv{};
    for (int k = 0; k < cnt; ++k) {
      pk.p[k] = src[first + k];
      lv.v[k] = levels ? (*levels)[first + k] : 0;
      if (mulp) pm.p[k] = (*mulp)[first + k];
      if (addp) pa.p[k] = (*addp)[first + k];
    }
    hipEvent_t ev;
    prof_begin(c, 10, &ev);
    hipLaunchKernelGGL(ntt_rowinv_gather_kernel, dim3((unsigned)(c.N / 4096), cnt * rpj), dim3(512), 0, c.stream,
                       dst + first * rpj * c.N, pk, lv, rpj, src_stride, src_off, prime_fixed, c.d_primes, (int)c.log_n,
                       (int)c.log_n - 12, pm, pa);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 10, ev, 2.0 * cnt * rpj * (double)c.N * 8.0);
  }
}

void launch_ntt_fwd_rows_md_finish(Context& c, const std::vector<double*>& out, const std::vector<const double*>& add,
                                   const std::vector<uint64_t>& gal, const double* acc, const double* w, int nE,
                                   int nl, const double* pinv, const double* tpinv, int add_mode) {
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  for (size_t first = 0; first < out.size(); first += kPack) {
    const int cnt = (int)std::min<size_t>(kPack, out.size() - first);
    MPack po;
    Pack pa, pin;
    GPack pg;
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k];
      pa.p[k] = add.empty() ? nullptr : add[first + k];
      pg.g[k] = gal.empty() ? 1 : gal[first + k];
      pin.p[k] = nullptr;
    }
    hipEvent_t ev;
    prof_begin(c, 7, &ev);
    Pack none{};
    IPack nolv{};
    hipLaunchKernelGGL(ntt_rowfwd_finish_kernel<1>, dim3((unsigned)(c.N / 4096), nl, 2 * cnt), dim3(512), 0,
                       c.stream, po, pin, pa, pg, none, none, nolv, acc + first * 2 * nE * c.N,
                       w + first * 2 * nl * c.N, nE, nl, 2, add_mode, 0, pinv, tpinv, c.d_primes, (int)c.log_n,
                       (int)c.log_n - 12, nullptr, none);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 7, ev, (6.0 + (add_mode == 1 ? 2.0 : add_mode == 2 ? 1.0 : 0.0)) * nl * cnt * (double)c.N * 8.0);
  }
}

void launch_ntt_fwd_rows_mdms_finish(Context& c, const std::vector<double*>& out,
                                     const std::vector<const double*>& add, const double* acc, const double* w,
                                     int nE, int l, const double* m1, const double* m2, const double* m3,
                                     const std::vector<const double*>* masks, int mask_np,
                                     const std::vector<const double*>* add_b) {
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  if (l < 1) fail(COPSE_EINVAL, "internal: no switch below level 0");
  if (add_b && add_b->size() != add.size()) fail(COPSE_EINVAL, "internal: product addends");
  for (size_t first = 0; first < out.size(); first += kPack) {
    const int cnt = (int)std::min<size_t>(kPack, out.size() - first);
    MPack po;
    Pack pa, pm, pb{}, none{};
    GPack pg;
    IPack nolv{};
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k];
      pa.p[k] = add[first + k];
      pm.p[k] = masks ? (*masks)[first + k] : nullptr;
      if (add_b) pb.p[k] = (*add_b)[first + k];
      pg.g[k] = 1;
    }
    hipEvent_t ev;
    prof_begin(c, 7, &ev);
    hipLaunchKernelGGL(ntt_rowfwd_finish_kernel<3>, dim3((unsigned)(c.N / 4096), l, 2 * cnt), dim3(512), 0,
                       c.stream, po, pm, pa, pg, none, none, nolv, acc + first * 2 * nE * c.N,
                       w + first * 2 * l * c.N, nE, l, 2, 0, masks ? mask_np : 0, m1, m2, c.d_primes,
                       (int)c.log_n, (int)c.log_n - 12, m3, pb);
    COPSE_HIP(hipGetLastError());
    // per output row: the bridge's row, the accumulator and addend rows read (a product's addend: its two
    // ciphertexts' rows, 2 for poly 0 and 4 for poly 1), the output written (+ mask)
    prof_end(c, 7, ev, ((add_b ? 3.0 * 2 + 6.0 : 4.0 * 2) + (masks ? mask_np : 0)) * l * cnt * (double)c.N * 8.0);
  }
}

void launch_ntt_fwd_rows_ms_finish(Context& c, const std::vector<double*>& out, const std::vector<const double*>& in,
                                   const std::vector<const double*>& w, const std::vector<int>& levels,
                                   const std::vector<const double*>& tabs, int np,
                                   const std::vector<const double*>* add, int add_np,
                                   const std::vector<const double*>* mulp) {
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  const int per = std::max(1, std::min(kPack, kMaxGridY / np));
  for (size_t first = 0; first < out.size(); first += per) {
    const int cnt = (int)std::min<size_t>(per, out.size() - first);
    MPack po;
    Pack pi, pa, pw, pt, pm{};
    GPack pg;
    IPack lv{};
    int lmax = 0;
    double bytes = 0;
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k];
      pi.p[k] = in[first + k];
      pa.p[k] = add ? (*add)[first + k] : nullptr;
      if (mulp) pm.p[k] = (*mulp)[first + k];
      pw.p[k] = w[first + k];
      pt.p[k] = tabs[first + k];
      pg.g[k] = 1;
      lv.v[k] = levels[first + k];
      const int nl = lv.v[k] & 0xffff;
      lmax = std::max(lmax, nl);
      bytes += (3.0 * np + (add ? add_np : 0)) * nl * (double)c.N * 8.0;
    }
    hipEvent_t ev;
    prof_begin(c, 8, &ev);
    if (mulp)   // the plaintext layer (`add` holds its addends, no post-switch add)
      hipLaunchKernelGGL(ntt_rowfwd_finish_kernel<4>, dim3((unsigned)(c.N / 4096), lmax, np * cnt), dim3(512), 0,
                         c.stream, po, pi, pa, pg, pw, pt, lv, nullptr, nullptr, 0, 0, np, 0, 0, nullptr, nullptr,
                         c.d_primes, (int)c.log_n, (int)c.log_n - 12, nullptr, pm);
    else
      hipLaunchKernelGGL(ntt_rowfwd_finish_kernel<2>, dim3((unsigned)(c.N / 4096), lmax, np * cnt), dim3(512), 0,
                         c.stream, po, pi, pa, pg, pw, pt, lv, nullptr, nullptr, 0, 0, np, 0, add ? add_np : 0,
                         nullptr, nullptr, c.d_primes, (int)c.log_n, (int)c.log_n - 12, nullptr, pm);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 8, ev, bytes);
  }
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
    if (nrows > 65535) fail(COPSE_EINVAL, "too many rows for one elementwise launch");            \
    hipEvent_t ev;                                                                                \
    prof_begin(c, 6, &ev);                                                                        \
    hipLaunchKernelGGL(kern, ew_grid(c, nrows), dim3(256), 0, c.stream, __VA_ARGS__, rows, c.d_primes, \
                       (int)c.log_n);                                                             \
    COPSE_HIP(hipGetLastError());                                                                 \
    prof_end(c, 6, ev, 3.0 * nrows * (double)c.N * 8.0);                                                                    \
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
  prof_begin(c, 6, &ev);
  hipLaunchKernelGGL(mul_plain_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, out, a, pt, nl, npolys, c.d_primes,
                     (int)c.log_n, 0);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 6, ev, (2.0 * npolys + 1) * nl * (double)c.N * 8.0);
}
void launch_mac_plain(Context& c, double* acc, const double* a, const double* pt, int npolys, int nl) {
  hipEvent_t ev;
  prof_begin(c, 6, &ev);
  hipLaunchKernelGGL(mul_plain_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, acc, a, pt, nl, npolys, c.d_primes,
                     (int)c.log_n, 1);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 6, ev, (3.0 * npolys + 1) * nl * (double)c.N * 8.0);
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
  prof_begin(c, 6, &ev);
  hipLaunchKernelGGL(tensor_kernel, ew_grid(c, nl), dim3(256), 0, c.stream, d, a, b, nl, c.d_primes, (int)c.log_n,
                     accumulate ? 1 : 0);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 6, ev, 7.0 * nl * (double)c.N * 8.0);
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

// out = sigma_g(in) on nl * npolys rows in the evaluation domain (index permutation auto_src)
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
// A thread converts one coefficient for up to kBcOut outputs: the n_in inputs are read once and
// their scaled residues y_i in [0, q_i) stay in registers.  For |a| < 2^49 and b in [0, p) the lazy
// product a b - p rint(a b / p) is exact with magnitude below 0.69 p (the quotient estimate is off by at
// most 2^-3 from the rounding of 1/p and 2^-4 from the dropped low product), so the n_in <= 8 terms sum
// below 5.6 p before a single symmetric reduction.  grid: x over coefficients, y over output chunks,
// z over the batch.
constexpr int kBcIn = 8;
constexpr int kBcOut = 16;
__global__ __launch_bounds__(256) void bconv_kernel(double* out_base, const int2* out_rows, int n_out,
                                                    const double* in_base, const int2* in_rows, int n_in,
                                                    const double* mult, const double* mat, const DevPrime* P,
                                                    int logN, size_t in_bs, size_t out_bs) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double* in = in_base + (size_t)blockIdx.z * in_bs;
  double* out = out_base + (size_t)blockIdx.z * out_bs;
  double y[kBcIn];
#pragma unroll
  for (int k = 0; k < kBcIn; ++k) {
    if (k < n_in) {
      const int2 irow = in_rows[k];
      const DevPrime& pk = P[irow.y];
      y[k] = canon(mul_lazy(in[(size_t)irow.x * N + i], mult[k], pk.q, pk.qinv), pk.q);
    }
  }
  const int o0 = blockIdx.y * kBcOut;
  const int no = min(n_out - o0, kBcOut);
  // unrolled so that the per-output constants are fetched together and the stores overlap
#pragma unroll
  for (int oo = 0; oo < kBcOut; ++oo) {
    if (oo < no) {
      const int o = o0 + oo;
      const int2 orow = out_rows[o];
      const DevPrime& po = P[orow.y];
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < kBcIn; ++k)
        if (k < n_in) acc += mul_lazy(y[k], mat[k * n_out + o], po.q, po.qinv);
      out[(size_t)orow.x * N + i] = canon(reduce_sym(acc, po.q, po.qinv), po.q);
    }
  }
}

void launch_bconv(Context& c, double* out_base, const int2* out_rows, int n_out, const double* in_base,
                  const int2* in_rows, int n_in, const double* mult, const double* mat, int batch,
                  size_t in_bs, size_t out_bs) {
  if (n_out <= 0 || batch <= 0) return;
  if (n_in > kBcIn) fail(COPSE_EINVAL, "base conversion supports at most 8 source primes");
  hipEvent_t ev;
  prof_begin(c, 5, &ev);
  hipLaunchKernelGGL(bconv_kernel, dim3((unsigned)((c.N + 255) / 256), (n_out + kBcOut - 1) / kBcOut, batch),
                     dim3(256), 0, c.stream, out_base, out_rows, n_out, in_base, in_rows, n_in, mult, mat,
                     c.d_primes, (int)c.log_n, in_bs, out_bs);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 5, ev, (double)(n_out + n_in) * batch * (double)c.N * 8.0);   // inputs counted once
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
    prof_begin(c, 4, &ev);
    hipLaunchKernelGGL(ks_inner_kernel, dim3((unsigned)((c.N + 255) / 256), nE, cnt), dim3(256), 0, c.stream, pack,
                       D, nE, level + 1, c.L, (int)c.log_n, key_ds, c.d_primes);
    COPSE_HIP(hipGetLastError());
    // per job and extended row: D digit rows and 2 D key rows read, 2 rows written
    prof_end(c, 4, ev, (3.0 * D + 2.0) * nE * cnt * (double)c.N * 8.0);
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
  prof_begin(c, 6, &ev);
  hipLaunchKernelGGL(ms_finish_kernel, dim3((unsigned)((c.N + 255) / 256), level, npolys), dim3(256), 0,
                     c.stream, out, in, w, npolys, level, tab, c.d_primes, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 6, ev, 3.0 * level * npolys * (double)c.N * 8.0);
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
  prof_begin(c, 6, &ev);
  hipLaunchKernelGGL(moddown_finish_kernel, dim3((unsigned)((c.N + 255) / 256), nl, npolys), dim3(256), 0,
                     c.stream, out, y, ys, w, nl, pinv, tpinv, add, adds, add_mode, c.d_primes, (int)c.log_n);
  COPSE_HIP(hipGetLastError());
  prof_end(c, 6, ev, 3.0 * nl * npolys * (double)c.N * 8.0);
}

}  // namespace copse

// ================================================================== batched kernels
// Operations over many ciphertexts at once take per-job pointers by value
// (Pack: up to kPack jobs per launch; longer lists are launched in chunks).
namespace copse {

// dst row (j * rows + r) <- src_j row r
// four consecutive values per thread, as two 16-byte loads and stores (rows hold N = 2^logN >= 16
// values, so every thread's quad is in range and 32-byte aligned)
__global__ void gather_kernel(double* dst, Pack src, int rows, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i >= N) return;
  const int r = blockIdx.y, j = blockIdx.z;
  typedef double dvec2 __attribute__((ext_vector_type(2)));
  const auto* s = (const __attribute__((address_space(1))) dvec2*)(src.p[j] + (size_t)r * N + i);
  auto* d = (__attribute__((address_space(1))) dvec2*)(dst + ((size_t)j * rows + r) * N + i);
  const dvec2 a = s[0], b = s[1];
  d[0] = a;
  d[1] = b;
}

void launch_gather(Context& c, double* dst, const std::vector<const double*>& src, int rows) {
  if (c.N % 4 != 0) fail(COPSE_EINVAL, "internal: gather needs N a multiple of 4");
  for (size_t first = 0; first < src.size(); first += kPack) {
    int cnt = (int)std::min<size_t>(kPack, src.size() - first);
    Pack pk;
    for (int k = 0; k < cnt; ++k) pk.p[k] = src[first + k];
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((c.N / 4 + 255) / 256), rows, cnt), dim3(256), 0, c.stream,
                       dst + first * rows * c.N, pk, rows, (int)c.log_n);
  }
  COPSE_HIP(hipGetLastError());
}


// plaintext layer: out_j = (a0 * m_j + p_j, a1 * m_j)  (2 polys, nl limbs)
__global__ void ptlayer_kernel(MPack out, Pack a, Pack mul, Pack add, int nl, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int l = blockIdx.y, j = blockIdx.z;
  const DevPrime& pr = P[l];
  const size_t o = (size_t)l * N + i, ps = (size_t)nl * N;
  const double m = mul.p[j][o];
  out.p[j][o] = mod_add(mod_mul(a.p[j][o], m, pr.q, pr.qinv), add.p[j][o], pr.q);
  out.p[j][ps + o] = mod_mul(a.p[j][ps + o], m, pr.q, pr.qinv);
}

void launch_ptlayer(Context& c, const std::vector<double*>& out, const std::vector<const double*>& a,
                    const std::vector<const double*>& mul, const std::vector<const double*>& add, int nl) {
  for (size_t first = 0; first < out.size(); first += kPack) {
    int cnt = (int)std::min<size_t>(kPack, out.size() - first);
    MPack po;
    Pack pa, pm, pd;
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k]; pa.p[k] = a[first + k]; pm.p[k] = mul[first + k]; pd.p[k] = add[first + k];
    }
    hipLaunchKernelGGL(ptlayer_kernel, dim3((unsigned)((c.N + 255) / 256), nl, cnt), dim3(256), 0, c.stream, po, pa,
                       pm, pd, nl, c.d_primes, (int)c.log_n);
  }
  COPSE_HIP(hipGetLastError());
}

// d_j = (a0 b0, a0 b1 + a1 b0, a1 b1)
__global__ void tensor_multi_kernel(MPack d, Pack a, Pack b, int nl, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int l = blockIdx.y, j = blockIdx.z;
  const DevPrime& pr = P[l];
  const size_t ps = (size_t)nl * N, o = (size_t)l * N + i;
  const double a0 = a.p[j][o], a1 = a.p[j][ps + o], b0 = b.p[j][o], b1 = b.p[j][ps + o];
  d.p[j][o] = mod_mul(a0, b0, pr.q, pr.qinv);
  d.p[j][ps + o] = mod_add(mod_mul(a0, b1, pr.q, pr.qinv), mod_mul(a1, b0, pr.q, pr.qinv), pr.q);
  d.p[j][2 * ps + o] = mod_mul(a1, b1, pr.q, pr.qinv);
}

void launch_tensor_multi(Context& c, const std::vector<double*>& d, const std::vector<const double*>& a,
                         const std::vector<const double*>& b, int nl) {
  for (size_t first = 0; first < d.size(); first += kPack) {
    int cnt = (int)std::min<size_t>(kPack, d.size() - first);
    MPack pd;
    Pack pa, pb;
    for (int k = 0; k < cnt; ++k) { pd.p[k] = d[first + k]; pa.p[k] = a[first + k]; pb.p[k] = b[first + k]; }
    hipEvent_t ev;
    prof_begin(c, 6, &ev);
    hipLaunchKernelGGL(tensor_multi_kernel, dim3((unsigned)((c.N + 255) / 256), nl, cnt), dim3(256), 0, c.stream,
                       pd, pa, pb, nl, c.d_primes, (int)c.log_n);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 6, ev, 6.0 * nl * cnt * (double)c.N * 8.0);
  }
}

// modulus switch finish over jobs: out_j[k][i] = in_j[k][i] q_l^-1 - w[(j np + k)][i] t q_l^-1
// out_j = (in_j - t z_j) q_l^-1 (+ add_j on the first add_np polys, when add_j is given)
__global__ void ms_finish_multi_kernel(MPack out, Pack in, Pack add, int add_np, const double* w, int np, int l,
                                       const double* tab, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = blockIdx.y;
  const int z = blockIdx.z;
  const int j = z / np, k = z % np;
  const DevPrime& pi = P[i];
  const double x = in.p[j][((size_t)k * (l + 1) + i) * N + c];
  const double y = w[((size_t)z * l + i) * N + c];
  const size_t oo = ((size_t)k * l + i) * N + c;
  double v = mod_sub(mod_mul(x, tab[2 + 2 * i], pi.q, pi.qinv), mod_mul(y, tab[3 + 2 * i], pi.q, pi.qinv), pi.q);
  if (k < add_np && add.p[j] != nullptr) v = mod_add(v, add.p[j][oo], pi.q);
  out.p[j][oo] = v;
}

void launch_ms_finish_multi(Context& c, const std::vector<double*>& out, const std::vector<const double*>& in,
                            const double* w, int np, int level, const double* tab,
                            const std::vector<const double*>* add, int add_np) {
  for (size_t first = 0; first < out.size(); first += kPack) {
    int cnt = (int)std::min<size_t>(kPack, out.size() - first);
    MPack po;
    Pack pi, pa;
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k];
      pi.p[k] = in[first + k];
      pa.p[k] = add ? (*add)[first + k] : nullptr;
    }
    hipEvent_t ev;
    prof_begin(c, 6, &ev);
    hipLaunchKernelGGL(ms_finish_multi_kernel, dim3((unsigned)((c.N + 255) / 256), level, cnt * np), dim3(256), 0,
                       c.stream, po, pi, pa, add ? add_np : 0, w + first * np * level * c.N, np, level, tab,
                       c.d_primes, (int)c.log_n);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 6, ev, (3.0 * np + (add ? add_np : 0)) * level * cnt * (double)c.N * 8.0);
  }
}

// (t0, t1) <- polynomials 0 and 1 of the product of ciphertexts (t0, t1) and (b0, b1) at one coefficient
__device__ __forceinline__ void ks_tensor_top(double& t0, double& t1, double b0, double b1, const DevPrime& pr) {
  const double a0 = t0;
  t0 = mod_mul(a0, b0, pr.q, pr.qinv);
  t1 = mod_add(mod_mul(a0, b1, pr.q, pr.qinv), mod_mul(t1, b0, pr.q, pr.qinv), pr.q);
}

// key-switch inner product over jobs; digit rows come straight from the job's input poly (a product's
// third polynomial in (.) in_b when in_b is set).  kD > 0: the digit count, known at compile time, so every
// digit's loads are issued before the first product (kD = 0: any count, one digit at a time).
template <int kD>
__global__ void ks_inner2_kernel(KsPack jobs, int D_, int nE, int nl, int L, int alpha, int logN, size_t key_ds,
                                 const DevPrime* P, double ptop) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int o = blockIdx.y;
  const KsJob2 jb = jobs.j[blockIdx.z];
  const int prime = o < nl ? o : L + 1 + (o - nl);
  const DevPrime& pr = P[prime];
  const size_t src = jb.g == 1 ? i : auto_src((uint32_t)i, jb.g, logN);
  const int own = o < nl ? o / alpha : -1;   // digit whose own limb this row is
  // digit j's row: the input's own limb, else the ModUp output; a product's own limb is a1 (.) b1, b1's
  // value (ob) loaded with the others and multiplied in after the loads
  auto row = [&](int j) -> const double* { return j == own ? jb.in + (size_t)o * N : jb.ext + ((size_t)j * nE + o) * N; };
  const bool prod = own >= 0 && jb.in_b != nullptr;   // uniform
  const double ob = prod ? jb.in_b[(size_t)o * N + src] : 0.0;
  // lazy sums: each product is in (-0.91 q, 0.91 q); D <= 8 digits stay far below 2^52
  double a0 = 0.0, a1 = 0.0;
  if (kD > 0) {
    // a known digit count: every digit's loads are issued before the first product
    double e[kD > 0 ? kD : 1], kb[kD > 0 ? kD : 1], ka[kD > 0 ? kD : 1];
#pragma unroll
    for (int j = 0; j < kD; ++j) {
      const size_t ko = (size_t)j * key_ds + (size_t)prime * N + i;
      e[j] = row(j)[src];
      kb[j] = jb.kb[ko];
      ka[j] = jb.ka[ko];
    }
#pragma unroll
    for (int j = 0; j < kD; ++j) {
      const double ej = prod && j == own ? mod_mul(e[j], ob, pr.q, pr.qinv) : e[j];
      a0 += mul_lazy(ej, kb[j], pr.q, pr.qinv);
      a1 += mul_lazy(ej, ka[j], pr.q, pr.qinv);
    }
  } else {
    for (int j = 0; j < D_; ++j) {
      double e = row(j)[src];
      if (prod && j == own) e = mod_mul(e, ob, pr.q, pr.qinv);
      const size_t ko = (size_t)j * key_ds + (size_t)prime * N + i;
      a0 += mul_lazy(e, jb.kb[ko], pr.q, pr.qinv);
      a1 += mul_lazy(e, jb.ka[ko], pr.q, pr.qinv);
    }
  }
  if (jb.top != nullptr && o == nl - 1) {   // uniform per workgroup
    double t0 = jb.top[(size_t)o * N + i], t1 = jb.top[((size_t)nl + o) * N + i];
    if (jb.top_b != nullptr) ks_tensor_top(t0, t1, jb.top_b[(size_t)o * N + i], jb.top_b[((size_t)nl + o) * N + i], pr);
    a0 += mul_lazy(t0, ptop, pr.q, pr.qinv);
    a1 += mul_lazy(t1, ptop, pr.q, pr.qinv);
  }
  jb.acc[(size_t)o * N + i] = canon(reduce_sym(a0, pr.q, pr.qinv), pr.q);
  jb.acc[((size_t)nE + o) * N + i] = canon(reduce_sym(a1, pr.q, pr.qinv), pr.q);
}

// algorithmic bytes of one pack: per job and extended row D digit rows read and 2 rows written; each
// distinct key's 2 D rows once; a product's own limbs read b1 too (nl rows); the addend's top limb 2 rows
// (4 for a product's, formed from both operands)
static double ks_pack_bytes(const Context& c, const KsPack& pk, int cnt, int D, int nE, int nl, int keys) {
  double rows = (double)(D + 2) * cnt * nE + 2.0 * D * keys * nE;
  for (int k = 0; k < cnt; ++k) {
    if (pk.j[k].in_b != nullptr) rows += nl;
    if (pk.j[k].top != nullptr) rows += pk.j[k].top_b != nullptr ? 4 : 2;
  }
  return rows * (double)c.N * 8.0;
}

void launch_ks_inner2(Context& c, const std::vector<KsJob2>& jobs, int D, int nE, int level, size_t key_ds,
                      double ptop) {
  const size_t per = c.tune.ks_jobs > 0 ? (size_t)std::min(c.tune.ks_jobs, KsPack::kMax) : KsPack::kMax;
  for (size_t first = 0; first < jobs.size(); first += per) {
    int cnt = (int)std::min<size_t>(per, jobs.size() - first);
    KsPack pk;
    for (int k = 0; k < cnt; ++k) pk.j[k] = jobs[first + k];
    hipEvent_t ev;
    prof_begin(c, 4, &ev);
    const dim3 grid((unsigned)((c.N + 255) / 256), nE, cnt);
#define COPSE_KS2(KD)                                                                                          \
  hipLaunchKernelGGL(ks_inner2_kernel<KD>, grid, dim3(256), 0, c.stream, pk, D, nE, level + 1, c.L, c.alpha, \
                     (int)c.log_n, key_ds, c.d_primes, ptop)
    switch (D) {
      case 1: COPSE_KS2(1); break;
      case 2: COPSE_KS2(2); break;
      case 3: COPSE_KS2(3); break;
      case 4: COPSE_KS2(4); break;
      default: COPSE_KS2(0); break;
    }
#undef COPSE_KS2
    COPSE_HIP(hipGetLastError());
    int keys = 0;
    for (int k = 0; k < cnt; ++k) {
      bool seen = false;
      for (int k2 = 0; k2 < k; ++k2) seen |= pk.j[k2].kb == pk.j[k].kb;
      keys += !seen;
    }
    prof_end(c, 4, ev, ks_pack_bytes(c, pk, cnt, D, nE, level + 1, keys));
  }
}

// Relinearization inner products (no automorphism) with the ModUp's forward row pass folded in: block
// (tile, extended row o, job) transforms the tile of row o of every digit that targets o (the bridge left
// them after the column stages; a digit's own limbs come from the input in NTT form, a product's formed
// from both operands) and accumulates digit x key in registers, so the extended rows are never written in
// NTT form.  Rows o >= inv_from (the rows the ModDown transforms back) leave after the inverse row pass.
// At most 128 registers (four waves per SIMD) and two tile buffers (68 KiB), so that two workgroups share a
// compute unit and one transforms while the other waits on memory: the first two digits to transform run
// as one pair (row4_fwd_tile2) before any sum is live, further digits one at a time, the row's own digit
// last; the keys are read after each transform, one polynomial at a time; the two sums' inverse row passes
// run as one pair.
__global__ __launch_bounds__(512, 4) void ks_inner_rows_kernel(KsPack jobs, int D, int nE, int nl, int L, int alpha,
                                                               int logN, int S1, size_t key_ds, const DevPrime* P,
                                                               double ptop, int inv_from) {
  __shared__ double sh[kLdsTile4], sh2[kLdsTile4];
  const size_t N = (size_t)1 << logN;
  // block order: the hardware deals consecutive workgroups to the eight XCDs in turn, so with the tile
  // index fastest (N / 4096 tiles, a multiple of 8 from N = 32768) each XCD keeps to its tiles, and with
  // the job next the jobs of one (tile, row), which read the same key tile, run together on one XCD and
  // find it in its L2; rows from the last, so that the special rows (three transforms and two inverse
  // ones against two) start first instead of forming the launch's tail
  const unsigned lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned rest = lin / gridDim.x;
  const int o = (int)gridDim.y - 1 - (int)(rest / gridDim.z);
  const KsJob2 jb = jobs.j[rest % gridDim.z];
  const int prime = o < nl ? o : L + 1 + (o - nl);
  const DevPrime pr = P[prime];
  const size_t t0 = (size_t)(lin % gridDim.x) * 4096;
  const int t = threadIdx.x;
  const int own = o < nl ? o / alpha : -1;   // digit whose own limb this row is
  double a0[8], a1[8];
  // digit j's tile x times its key values, added to the sums (the keys read after x is ready, one
  // polynomial at a time)
  auto mac = [&](int j, double(&x)[8]) {
    const size_t ko = (size_t)j * key_ds + (size_t)prime * N + t0 + t;
    double kv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) kv[k] = gload(jb.kb + ko + 512 * k);
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = reduce_sym(x[k], pr.q, pr.qinv);
#pragma unroll
    for (int k = 0; k < 8; ++k) a0[k] += mul_lazy(x[k], kv[k], pr.q, pr.qinv);
#pragma unroll
    for (int k = 0; k < 8; ++k) kv[k] = gload(jb.ka + ko + 512 * k);
#pragma unroll
    for (int k = 0; k < 8; ++k) a1[k] += mul_lazy(x[k], kv[k], pr.q, pr.qinv);
  };
  auto ext = [&](int j) { return jb.ext + ((size_t)j * nE + o) * N + t0; };
  // the first two digits to transform (not the row's own) as one pair, before any sum is live; the sums
  // are exact, so the digit order changes no bit
  int j = own == 0 ? 1 : 0, jn = D;   // jn: the first digit left after the pair
  if (j < D) {
    int j2 = j + 1;
    if (j2 == own) ++j2;
    if (j2 < D) {
      double x[8], y[8];
      row4_fwd_tile2(ext(j), ext(j2), t0, S1, pr, sh, sh2, x, y);
#pragma unroll
      for (int k = 0; k < 8; ++k) a0[k] = a1[k] = 0.0;
      mac(j, x);
      mac(j2, y);
      jn = j2 + 1;
    } else {
      double x[8];
      row4_fwd_tile(ext(j), t0, S1, pr, sh, x);
#pragma unroll
      for (int k = 0; k < 8; ++k) a0[k] = a1[k] = 0.0;
      mac(j, x);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) a0[k] = a1[k] = 0.0;
  }
  for (int jj = jn; jj < D; ++jj) {   // any further digit one at a time (uniform per workgroup)
    if (jj == own) continue;
    double x[8];
    row4_fwd_tile(ext(jj), t0, S1, pr, sh, x);
    mac(jj, x);
  }
  // the digit whose own limb this row is: its values are the input's in NTT form (a product's: formed
  // from both operands), not transformed
  if (own >= 0) {
    double x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = gload(jb.in + (size_t)o * N + t0 + t + 512 * k);
    if (jb.in_b != nullptr) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        x[k] = mod_mul(x[k], gload(jb.in_b + (size_t)o * N + t0 + t + 512 * k), pr.q, pr.qinv);
    }
    mac(own, x);
  }
  if (jb.top != nullptr && o == nl - 1) {   // uniform: the addend's top limb, all loads issued together
    double u0[8], u1[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t c = t0 + t + 512 * k;
      u0[k] = gload(jb.top + (size_t)o * N + c);
      u1[k] = gload(jb.top + ((size_t)nl + o) * N + c);
    }
    if (jb.top_b != nullptr) {
      double b0[8], b1[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const size_t c = t0 + t + 512 * k;
        b0[k] = gload(jb.top_b + (size_t)o * N + c);
        b1[k] = gload(jb.top_b + ((size_t)nl + o) * N + c);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) ks_tensor_top(u0[k], u1[k], b0[k], b1[k], pr);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a0[k] += mul_lazy(u0[k], ptop, pr.q, pr.qinv);
      a1[k] += mul_lazy(u1[k], ptop, pr.q, pr.qinv);
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a0[k] = canon(reduce_sym(a0[k], pr.q, pr.qinv), pr.q);
    a1[k] = canon(reduce_sym(a1[k], pr.q, pr.qinv), pr.q);
  }
  if (o >= inv_from) {
    // rows the ModDown transforms back (the special rows, and the top data row of a ModDown merged with
    // the switch): the inverse row pass of both sums' tiles here, as the separate row pass would run it
    double x[8], y[8];
    lds_barrier();   // the tile buffers' previous use is over in every wave
    row4_inv_tile2(t0, S1, pr, sh, sh2, a0, a1, x, y);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a0[k] = reduce_sym(x[k], pr.q, pr.qinv);
      a1[k] = reduce_sym(y[k], pr.q, pr.qinv);
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const size_t c = t0 + t + 512 * k;
    jb.acc[(size_t)o * N + c] = a0[k];
    jb.acc[((size_t)nE + o) * N + c] = a1[k];
  }
}

void launch_ks_inner_rows(Context& c, const std::vector<KsJob2>& jobs, int D, int nE, int level, size_t key_ds,
                          double ptop, int inv_from) {
  if (c.log_n < 13) fail(COPSE_EINVAL, "internal: split transform needs N >= 8192");
  if (D > 8) fail(COPSE_EINVAL, "internal: too many digits for the fused inner product");
  const size_t per = c.tune.ks_jobs > 0 ? (size_t)std::min(c.tune.ks_jobs, KsPack::kMax) : KsPack::kMax;
  for (size_t first = 0; first < jobs.size(); first += per) {
    const int cnt = (int)std::min<size_t>(per, jobs.size() - first);
    KsPack pk;
    for (int k = 0; k < cnt; ++k) {
      pk.j[k] = jobs[first + k];
      if (pk.j[k].g != 1) fail(COPSE_EINVAL, "internal: the fused inner product takes no automorphism");
    }
    hipEvent_t ev;
    prof_begin(c, 15, &ev);
    hipLaunchKernelGGL(ks_inner_rows_kernel, dim3((unsigned)(c.N / 4096), nE, cnt), dim3(512), 0, c.stream, pk, D, nE,
                       level + 1, c.L, c.alpha, (int)c.log_n, (int)c.log_n - 12, key_ds, c.d_primes, ptop,
                       inv_from);
    COPSE_HIP(hipGetLastError());
    int keys = 0;
    for (int k = 0; k < cnt; ++k) {
      bool seen = false;
      for (int k2 = 0; k2 < k; ++k2) seen |= pk.j[k2].kb == pk.j[k].kb;
      keys += !seen;
    }
    prof_end(c, 15, ev, ks_pack_bytes(c, pk, cnt, D, nE, level + 1, keys));
  }
}

// Giant-step sums of key-switch inner products (see launch_ks_inner_gsum).  grid: x over coefficients,
// y over extended rows, z over (product, chunk of kB batch elements).  A thread keeps the sums of its chunk's
// kB outputs in registers and runs through the product's steps: per step the key values are loaded once and
// serve every batch element of the chunk (all of them rotate by the same element, so the permuted index is
// shared too), so each key is read once per chunk instead of once per output.
struct GsumPack {
  // 64 x 40 + 16 x 32 bytes: within the 4 KiB of kernel arguments with the other parameters
  static constexpr int kSteps = 64, kProds = 16;
  GsumStep s[kSteps];
  GsumProd p[kProds];
};
// kD: the digit count when it is known at compile time, else (kD = 8) an upper bound of the runtime D_;
// kGsumB: batch elements per thread
template <int kD, int kGsumB>
__global__ __launch_bounds__(256) void ks_inner_gsum_kernel(GsumPack pk, int G, size_t in_bs, size_t ext_bs,
                                                            size_t acc_bs, size_t top_bs, int D_, int nE, int nl,
                                                            int L, int alpha, int logN, size_t key_ds,
                                                            const DevPrime* P, double ptop) {
  const int D = kD < 8 ? kD : D_;
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int o = blockIdx.y;
  const int bchunks = (G + kGsumB - 1) / kGsumB;
  const GsumProd pr_ = pk.p[blockIdx.z / bchunks];
  const int b0 = (int)(blockIdx.z % bchunks) * kGsumB;
  const int nb = min(kGsumB, G - b0);   // uniform
  const int prime = o < nl ? o : L + 1 + (o - nl);
  const DevPrime pr = cload_prime(P + prime);
  const int own = o < nl ? o / alpha : -1;   // digit whose own limb this row is
  double a0[kGsumB], a1[kGsumB];
#pragma unroll
  for (int b = 0; b < kGsumB; ++b) a0[b] = a1[b] = 0.0;
  for (int t = pr_.first; t < pr_.first + pr_.count; ++t) {
    const GsumStep st = pk.s[t];
    const size_t src = st.g == 1 ? i : auto_src((uint32_t)i, st.g, logN);
    double kb[kD], ka[kD], e[kGsumB][kD];
#pragma unroll
    for (int j = 0; j < kD; ++j) {
      if (j < D) {
        const size_t ko = (size_t)j * key_ds + (size_t)prime * N + i;
        kb[j] = st.kb[ko];
        ka[j] = st.ka[ko];
      }
    }
#pragma unroll
    for (int b = 0; b < kGsumB; ++b) {
      if (b < nb) {
#pragma unroll
        for (int j = 0; j < kD; ++j) {
          if (j < D) {
            const double* row = j == own ? st.in + (size_t)(b0 + b) * in_bs + (size_t)o * N
                                         : st.ext + (size_t)(b0 + b) * ext_bs + ((size_t)j * nE + o) * N;
            e[b][j] = row[src];
          }
        }
      }
    }
#pragma unroll
    for (int b = 0; b < kGsumB; ++b) {
      if (b < nb) {
#pragma unroll
        for (int j = 0; j < kD; ++j) {
          if (j < D) {
            a0[b] += mul_lazy(e[b][j], kb[j], pr.q, pr.qinv);
            a1[b] += mul_lazy(e[b][j], ka[j], pr.q, pr.qinv);
          }
        }
        // at most 8 lazy products per step: fold back after each step
        a0[b] = reduce_sym(a0[b], pr.q, pr.qinv);
        a1[b] = reduce_sym(a1[b], pr.q, pr.qinv);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < kGsumB; ++b) {
    if (b < nb) {
      double* acc = pr_.acc + (size_t)(b0 + b) * acc_bs;
      double v0 = a0[b], v1 = a1[b];
      if (pr_.accum) {   // a later chunk: the earlier chunks' canonical sums
        v0 += acc[(size_t)o * N + i];
        v1 += acc[((size_t)nE + o) * N + i];
      } else if (o == nl - 1) {   // uniform per workgroup
        const double* top = pr_.top + (size_t)(b0 + b) * top_bs;
        v0 += mul_lazy(top[(size_t)o * N + i], ptop, pr.q, pr.qinv);
        v1 += mul_lazy(top[((size_t)nl + o) * N + i], ptop, pr.q, pr.qinv);
      }
      acc[(size_t)o * N + i] = canon(reduce_sym(v0, pr.q, pr.qinv), pr.q);
      acc[((size_t)nE + o) * N + i] = canon(reduce_sym(v1, pr.q, pr.qinv), pr.q);
    }
  }
}

void launch_ks_inner_gsum(Context& c, const std::vector<GsumStep>& steps, const std::vector<GsumProd>& prods_in, int G,
                          size_t in_bs, size_t ext_bs, size_t acc_bs, size_t top_bs, int D, int nE, int level,
                          size_t key_ds, double ptop) {
  if (D < 1 || D > 8) fail(COPSE_EINVAL, "internal: digit count of the giant-step sums");
  if (G < 1) return;
  // products with more than kSteps steps run in chunks: chunk r of every product in round r (rounds in stream
  // order, later chunks adding to the accumulator); within a round, packs of at most kProds chunks and kSteps
  // steps
  std::vector<std::vector<GsumProd>> rounds;
  for (const GsumProd& p : prods_in)
    for (int r = 0, done = 0; done < p.count || r == 0; ++r) {
      GsumProd ch = p;
      ch.first = p.first + done;
      ch.count = std::min(GsumPack::kSteps, p.count - done);
      ch.accum = r > 0;
      if ((int)rounds.size() <= r) rounds.emplace_back();
      rounds[r].push_back(ch);
      done += ch.count;
    }
  const int kB = c.tune.gsum_b == 4 ? 4 : 8;
  const int bchunks = (G + kB - 1) / kB;
  for (const auto& prods : rounds)
    for (size_t u0 = 0; u0 < prods.size();) {
      GsumPack pk;
      int np = 0, ns = 0;
      while (u0 + np < prods.size() && np < GsumPack::kProds) {
        const GsumProd& p = prods[u0 + np];
        if (ns + p.count > GsumPack::kSteps) break;
        pk.p[np] = p;
        pk.p[np].first = ns;
        for (int t = 0; t < p.count; ++t) pk.s[ns + t] = steps[p.first + t];
        ns += p.count;
        ++np;
      }
      hipEvent_t ev;
      prof_begin(c, 16, &ev);
      const dim3 grid((unsigned)((c.N + 255) / 256), nE, (unsigned)(np * bchunks));
#define COPSE_KSG(KD, KB)                                                                                       \
  hipLaunchKernelGGL((ks_inner_gsum_kernel<KD, KB>), grid, dim3(256), 0, c.stream, pk, G, in_bs, ext_bs, acc_bs,     \
                     top_bs, D, nE, level + 1, c.L, c.alpha, (int)c.log_n, key_ds, c.d_primes, ptop)
#define COPSE_KSG_D(KB)             \
  switch (D) {                      \
    case 1: COPSE_KSG(1, KB); break; \
    case 2: COPSE_KSG(2, KB); break; \
    case 3: COPSE_KSG(3, KB); break; \
    case 4: COPSE_KSG(4, KB); break; \
    default: COPSE_KSG(8, KB); break; \
  }
      if (kB == 4) {
        COPSE_KSG_D(4)
      } else {
        COPSE_KSG_D(8)
      }
#undef COPSE_KSG_D
#undef COPSE_KSG
      COPSE_HIP(hipGetLastError());
      // per step and batch element: D digit rows read; per output: 2 rows written and the addend's top limb
      // (2 rows) read, or a later chunk's accumulator (2 rows); each step's key (2 D rows) once
      double extra = 0.0;
      for (int u = 0; u < np; ++u) extra += G * (pk.p[u].accum ? 2.0 * nE : 2.0);
      prof_end(c, 16, ev,
               (((double)D * ns * G + 2.0 * np * G + 2.0 * D * ns) * nE + extra) * (double)c.N * 8.0);
      u0 += np;
    }
}

// Sums of automorphisms of c0 parts plus optional unrotated parts (see launch_auto_sum).
// grid: x over coefficients, y over limbs, z over (output, poly) of the pack.
struct AutoSumPack {
  static constexpr int kTerms = 64, kOuts = 16;
  AutoTerm t[kTerms];
  AutoOut o[kOuts];
};
__global__ void auto_sum_kernel(AutoSumPack pk, int nl, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int r = blockIdx.y, u = blockIdx.z >> 1, k = blockIdx.z & 1;
  const AutoOut ou = pk.o[u];
  const DevPrime& pr = P[r];
  const double* f = k == 0 ? ou.f0 : ou.f1;
  const size_t d = ((size_t)k * nl + r) * N + i;
  double v = ou.accum ? ou.dst[d] : f != nullptr ? f[(size_t)r * N + i] : 0.0;
  if (k == 0)
    for (int t = ou.first; t < ou.first + ou.count; ++t) {
      const AutoTerm tm = pk.t[t];
      const size_t src = tm.g == 1 ? i : auto_src((uint32_t)i, tm.g, logN);
      v = mod_add(v, tm.c0[(size_t)r * N + src], pr.q);
    }
  ou.dst[d] = v;
}

void launch_auto_sum(Context& c, const std::vector<AutoTerm>& terms, const std::vector<AutoOut>& outs_in, int nl) {
  // long outputs in chunks, chunk r in round r (see launch_ks_inner_gsum)
  std::vector<std::vector<AutoOut>> rounds;
  for (const AutoOut& o : outs_in)
    for (int r = 0, done = 0; done < o.count || r == 0; ++r) {
      AutoOut ch = o;
      ch.first = o.first + done;
      ch.count = std::min(AutoSumPack::kTerms, o.count - done);
      ch.accum = r > 0;
      if ((int)rounds.size() <= r) rounds.emplace_back();
      rounds[r].push_back(ch);
      done += ch.count;
    }
  for (const auto& outs : rounds)
  for (size_t u0 = 0; u0 < outs.size();) {
    AutoSumPack pk;
    int nu = 0, nt = 0;
    while (u0 + nu < outs.size() && nu < AutoSumPack::kOuts) {
      const AutoOut& o = outs[u0 + nu];
      if (nt + o.count > AutoSumPack::kTerms) break;
      pk.o[nu] = o;
      pk.o[nu].first = nt;
      for (int t = 0; t < o.count; ++t) pk.t[nt + t] = terms[o.first + t];
      nt += o.count;
      ++nu;
    }
    hipEvent_t ev;
    prof_begin(c, 6, &ev);
    hipLaunchKernelGGL(auto_sum_kernel, dim3((unsigned)((c.N + 255) / 256), nl, 2 * nu), dim3(256), 0, c.stream, pk,
                       nl, c.d_primes, (int)c.log_n);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 6, ev, ((double)nt + 4.0 * nu) * nl * (double)c.N * 8.0);
    u0 += nu;
  }
}

// ModDown finish over jobs of 2 polys: out_j[k] = y * P^-1 - w * t P^-1, plus
// mode 1: add_j poly k;  mode 2: for k = 0 add sigma_{g_j}(add_j poly 0)
__global__ void md_finish2_kernel(MPack out, Pack add, GPack gal, const double* acc, const double* w, int nE, int nl,
                                  const double* pinv, const double* tpinv, int add_mode, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int i = blockIdx.y;
  const int z = blockIdx.z;       // job * 2 + k
  const int j = z >> 1, k = z & 1;
  const DevPrime& pi = P[i];
  const double yv = acc[((size_t)z * nE + i) * N + c];
  const double wv = w[((size_t)z * nl + i) * N + c];
  double v = mod_sub(mod_mul(yv, pinv[i], pi.q, pi.qinv), mod_mul(wv, tpinv[i], pi.q, pi.qinv), pi.q);
  if (add_mode == 1) v = mod_add(v, add.p[j][((size_t)k * nl + i) * N + c], pi.q);
  if (add_mode == 2 && k == 0) {
    const size_t src = gal.g[j] == 1 ? c : auto_src((uint32_t)c, gal.g[j], logN);
    v = mod_add(v, add.p[j][(size_t)i * N + src], pi.q);
  }
  out.p[j][((size_t)k * nl + i) * N + c] = v;
}

void launch_md_finish2(Context& c, const std::vector<double*>& out, const std::vector<const double*>& add,
                       const std::vector<uint64_t>& gal, const double* acc, const double* w, int nE, int nl,
                       const double* pinv, const double* tpinv, int add_mode) {
  for (size_t first = 0; first < out.size(); first += kPack) {
    int cnt = (int)std::min<size_t>(kPack, out.size() - first);
    MPack po;
    Pack pa;
    GPack pg;
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k];
      pa.p[k] = add.empty() ? nullptr : add[first + k];
      pg.g[k] = gal.empty() ? 1 : gal[first + k];
    }
    hipEvent_t ev;
    prof_begin(c, 6, &ev);
    hipLaunchKernelGGL(md_finish2_kernel, dim3((unsigned)((c.N + 255) / 256), nl, 2 * cnt), dim3(256), 0, c.stream,
                       po, pa, pg, acc + first * 2 * nE * c.N, w + first * 2 * nl * c.N, nE, nl, pinv, tpinv,
                       add_mode, c.d_primes, (int)c.log_n);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 6, ev, (6.0 + (add_mode == 1 ? 2.0 : add_mode == 2 ? 1.0 : 0.0)) * nl * cnt * (double)c.N * 8.0);
  }
}

// MatMul inner sums (diagonal method, one giant group per output):
//   plaintext model:  out[s][b]     = sum_u baby[u][b] (.) diag(u, s)            (2 polys)
//   encrypted model:  out[s][b]     = sum_u tensor(baby[u][b], diag(u, s))       (3 polys)
// One thread owns one coefficient of one limb of one batch element and keeps the sums of GM giant
// groups in registers, so each baby-step value is read once per launch (per group chunk) instead of
// once per term.  Baby steps with no term in the chunk are skipped (uniform); zero diagonals' products
// are skipped by uniform branches.  The workgroups of one coefficient tile (all batch chunks and all
// giant-group chunks) run back to back on one XCD, so a baby-step tile is fetched from HBM once and the
// other chunks find it in that XCD's L2.  Sums are lazy (|term| < 0.91 q) and folded back with
// reduce_sym every mm_fold_every(q) baby steps.
// grid: x = (N / 64) x giant-group chunks of GM x ceil(G / 4) (XCD-aware, the batch chunk fastest), y = limbs.
constexpr int kMmLanes = 64, kMmWaves = 4;

// How many lazy terms a partial sum takes before it is folded back with reduce_sym, for the limb's prime q:
// a folded sum is below q and every term below c q (c = 1.25 for an encrypted model's operands below 2q,
// 0.91 for a plaintext model's below q), so after K terms a sum is below (1 + c K) q, kept below 2^52:
// exact, and reduce_sym's quotient estimate is off by less than one.  Primes near 2^49 fold every 5 or 7
// terms, primes below 2^42 every 64.
__device__ __forceinline__ int mm_fold_every(double q, bool enc) {
  const double k = (4503599627370496.0 / q - 1.0) / (enc ? 1.25 : 0.91);
  return __builtin_amdgcn_readfirstlane(k >= 64.0 ? 64 : (k < 1.0 ? 1 : (int)k));
}

struct MmPlace {
  size_t i;    // coefficient
  int b;       // batch element of this wave (may be >= G)
  int s0, gm;  // the chunk's first giant group and its group count
};
// kW: waves per workgroup, one batch element each (the batch kernel), or 4 waves sharing one element
template <int GM, int kW = kMmWaves>
__device__ __forceinline__ MmPlace mm_place(int ng, int G, int wv) {
  // consecutive workgroups go to different XCDs: give each XCD a contiguous range of logical blocks
  unsigned bx = blockIdx.x;
  const unsigned nbx = gridDim.x;
  if ((nbx & 7u) == 0) bx = (bx & 7u) * (nbx >> 3) + (bx >> 3);
  const unsigned bchunks = (unsigned)(G + kW - 1) / kW;
  const unsigned per_tile = bchunks * (unsigned)((ng + GM - 1) / GM);
  const unsigned rem = bx % per_tile;
  MmPlace m;
  m.b = (int)(rem % bchunks) * kW + wv;
  m.i = (size_t)(bx / per_tile) * kMmLanes + (threadIdx.x % kMmLanes);
  m.s0 = (int)(rem / bchunks) * GM;
  m.gm = min(GM, ng - m.s0);
  return m;
}

// Encrypted diagonals (Karatsuba): acc = {sum x0 d0, sum (x0 + x1)(d0 + d1), sum x1 d1}; the middle sum
// becomes sum (x0 d1 + x1 d0) = acc[1] - acc[0] - acc[2].  Every term is a lazy product of operands below 2q,
// |term| < 1.25 q (the quotient estimate is off by at most 0.75 for products below 4 q^2 < 2^100).
__device__ __forceinline__ void mm_karatsuba_mid(double (&a)[3], double q, double qinv) {
  const double lo = reduce_sym(a[0], q, qinv), hi = reduce_sym(a[2], q, qinv);
  a[1] = reduce_sym(a[1], q, qinv) - lo - hi;
  a[0] = lo;
  a[2] = hi;
}

// One batch element: the four waves of a workgroup take every fourth baby step of the same coefficients
// (each wave's chain of dependent loads a quarter as long) and add their partial sums through LDS at the
// end.  Per baby step the GM diagonal loads are issued together (a zero diagonal loads the baby value
// again, which is in cache).
template <int GM, bool kEnc>
__global__ __launch_bounds__(256) void mm_inner_kernel(double* __restrict__ out, const double* __restrict__ baby,
                                                       const double* const* __restrict__ tab, int n_u, int ng,
                                                       int nl, size_t baby_slot, const DevPrime* P, int logN,
                                                       const double* b0, int u0) {
  constexpr int kNp = kEnc ? 3 : 2;
  const size_t N = (size_t)1 << logN;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kMmLanes));
  const MmPlace m = mm_place<GM>(ng, 1, 0);
  const size_t i = m.i;
  // N is a multiple of 64, so a workgroup is either wholly in range or wholly out (uniform exit)
  if (i >= N) return;
  const int l = blockIdx.y;
  const int s0 = m.s0, gm = m.gm;
  const DevPrime& pr = P[l];
  const int fold = mm_fold_every(pr.q, kEnc);
  const size_t o = (size_t)l * N + i, ps = (size_t)nl * N;
  double acc[GM][kNp];
#pragma unroll
  for (int s = 0; s < GM; ++s)
#pragma unroll
    for (int p = 0; p < kNp; ++p) acc[s][p] = 0.0;
  int cnt = 0;
  for (int u = wv; u < n_u; u += kMmWaves) {
    // tables carry kMmTabPad trailing entries, so all GM pointers of a row can be fetched together
    const double* const* row = tab + (size_t)u * ng + s0;
    const double* ptr[GM];
    bool any = false;
#pragma unroll
    for (int s = 0; s < GM; ++s) {
      const double* pv = row[s];
      ptr[s] = s < gm ? pv : nullptr;
      any |= ptr[s] != nullptr;
    }
    if (!any) continue;   // uniform: this baby step has no term in the chunk
    // baby step u0 (the rotation by zero) is read from the unrotated input
    const double* bp = u == u0 ? b0 : baby + (size_t)u * baby_slot;
    const double x0 = gload(bp + o), x1 = gload(bp + ps + o);
    double d0[GM], d1[GM];
#pragma unroll
    for (int s = 0; s < GM; ++s) {
      const double* dp = ptr[s] != nullptr ? ptr[s] : bp;
      d0[s] = gload(dp + o);
      if (kEnc) d1[s] = gload(dp + ps + o);
    }
#pragma unroll
    for (int s = 0; s < GM; ++s) {
      if (ptr[s] != nullptr) {
        if (kEnc) {
          acc[s][0] += mul_lazy(x0, d0[s], pr.q, pr.qinv);
          acc[s][1] += mul_lazy(x0 + x1, d0[s] + d1[s], pr.q, pr.qinv);
          acc[s][kNp - 1] += mul_lazy(x1, d1[s], pr.q, pr.qinv);
        } else {
          acc[s][0] += mul_lazy(x0, d0[s], pr.q, pr.qinv);
          acc[s][1] += mul_lazy(x1, d0[s], pr.q, pr.qinv);
        }
      }
    }
    if (++cnt == fold) {
      cnt = 0;
#pragma unroll
      for (int s = 0; s < GM; ++s)
#pragma unroll
        for (int p = 0; p < kNp; ++p) acc[s][p] = reduce_sym(acc[s][p], pr.q, pr.qinv);
    }
  }
  // four groups at a time: every wave leaves its folded partial sums in LDS, wave w completes group w
  __shared__ double red[kMmWaves][kMmWaves][kNp][kMmLanes];
  const int lane = threadIdx.x % kMmLanes;
#pragma unroll
  for (int sb = 0; sb < GM; sb += kMmWaves) {
#pragma unroll
    for (int q = 0; q < kMmWaves; ++q)
      if (sb + q < GM) {
        if constexpr (kEnc) mm_karatsuba_mid(acc[sb + q], pr.q, pr.qinv);
#pragma unroll
        for (int p = 0; p < kNp; ++p) red[wv][q][p][lane] = reduce_sym(acc[sb + q][p], pr.q, pr.qinv);
      }
    lds_barrier();
    const int s = sb + wv;
    if (s < gm) {
      double* op = out + (size_t)(s0 + s) * kNp * ps;
#pragma unroll
      for (int p = 0; p < kNp; ++p) {
        double v = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kMmWaves; ++w2) v += red[w2][wv][p][lane];
        op[(size_t)p * ps + o] = canon(reduce_sym(v, pr.q, pr.qinv), pr.q);
      }
    }
    lds_barrier();
  }
}

// Several batch elements: a workgroup is 64 coefficients x kW batch elements (one per wave; kW = 4 or 8).
// The waves need the same diagonal values, so a baby step's diagonal tile (GM groups x 1 or 2 polys x 64
// coefficients) is fetched once per workgroup, each wave loading every kW-th group, and staged in LDS,
// double-buffered: the next baby step's tile and baby values are in flight while the current step's
// products run, and one barrier per baby step hands the tile over.  Which diagonals of a step are zero
// is a scalar bitmask.  A wave past the end of the batch still loads its share of the tiles.
template <int GM, bool kEnc, int kW>
__global__ __launch_bounds__(64 * kW) void mm_inner_batch_kernel(double* __restrict__ out,
                                                                 const double* __restrict__ baby,
                                                                 const double* const* __restrict__ tab, int n_u,
                                                                 int ng, int G, int nl, size_t baby_slot,
                                                                 size_t baby_b, const DevPrime* P, int logN, Pack b0,
                                                                 int u0) {
  constexpr int kNp = kEnc ? 3 : 2, kNd = kEnc ? 2 : 1;
  constexpr int kPer = (GM + kW - 1) / kW;   // groups of a tile one wave loads
  static_assert(GM <= 32, "one bit per group");
  __shared__ double dl[2][GM][kNd][kMmLanes];
  const size_t N = (size_t)1 << logN;
  const int lane = threadIdx.x % kMmLanes;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kMmLanes));
  const MmPlace m = mm_place<GM, kW>(ng, G, wv);
  const size_t i = m.i;
  if (i >= N) return;   // the whole workgroup (N is a multiple of 64)
  const int b = m.b;
  const bool has_b = b < G;   // uniform per wave
  const int l = blockIdx.y;
  const int s0 = m.s0, gm = m.gm;
  // the prime and the table entries as scalar loads: a vector load's wait inside the products would
  // also wait for the next tile
  const DevPrime pr = cload_prime(P + l);
  const int fold = mm_fold_every(pr.q, kEnc);
  const size_t o = (size_t)l * N + i, ps = (size_t)nl * N;
  // the first baby step at or after u with a term in the chunk (n_u if none) and its bitmask of groups
  auto scan = [&](int u, uint32_t& mask) -> int {
    for (; u < n_u; ++u) {
      const double* const* row = tab + (size_t)u * ng + s0;
      // the whole row at once (the table's kMmTabPad trailing entries keep it in bounds), masked to gm
      uint32_t mk = 0;
#pragma unroll
      for (int s = 0; s < GM; ++s) mk |= (cload(row + s) != nullptr ? 1u : 0u) << s;
      mk &= gm >= 32 ? ~0u : (1u << gm) - 1u;
      if (mk != 0) {
        mask = mk;
        return u;
      }
    }
    mask = 0;
    return n_u;
  };
  // this wave's share of baby step u's tile, and its batch element's baby values, into registers
  double r[kPer][kNd];
  double xn0 = 0.0, xn1 = 0.0;
  auto issue = [&](int u) {
    const double* const* row = tab + (size_t)u * ng + s0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int s = wv + kW * k;
      const double* pv = cload(row + s);   // in bounds as above
      const double* dp = s < gm ? pv : nullptr;   // uniform
      if (dp != nullptr) {
#pragma unroll
        for (int p = 0; p < kNd; ++p) r[k][p] = gload(dp + p * ps + o);
      } else {
#pragma unroll
        for (int p = 0; p < kNd; ++p) r[k][p] = 0.0;
      }
    }
    // unconditional (a wave past the batch reads the last element), so that the loads are issued here,
    // before the products; baby step u0 (the rotation by zero) is read from the unrotated inputs
    const int bl = min(b, G - 1);
    const double* bp = u == u0 ? b0.p[bl] : baby + (size_t)u * baby_slot + (size_t)bl * baby_b;
    xn0 = gload(bp + o);
    xn1 = gload(bp + ps + o);
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int s = wv + kW * k;
      if (s < GM)
#pragma unroll
        for (int p = 0; p < kNd; ++p) dl[buf][s][p][lane] = r[k][p];
    }
  };
  double acc[GM][kNp];
#pragma unroll
  for (int s = 0; s < GM; ++s)
#pragma unroll
    for (int p = 0; p < kNp; ++p) acc[s][p] = 0.0;
  uint32_t mask;
  int u = scan(0, mask);
  if (u < n_u) {
    issue(u);
    stage(0);
  }
  lds_barrier();
  double x0 = xn0, x1 = xn1;
  int buf = 0, cnt = 0;
  while (u < n_u) {   // uniform
    uint32_t mask_n;
    const int un = scan(u + 1, mask_n);
    if (un < n_u) issue(un);   // in flight during this step's products
    const double xs = x0 + x1;   // < 2 q (encrypted model only)
    if (has_b) {
#pragma unroll
      for (int s = 0; s < GM; ++s) {
        // an encrypted model's diagonals are all present: no branches, so the tile's LDS reads run ahead of
        // the products (a slot without a diagonal holds 0.0 and adds exactly zero)
        if (kEnc || ((mask >> s) & 1u)) {
          const double d0 = dl[buf][s][0][lane];
          if (kEnc) {
            // three products (Karatsuba): acc[1] holds sum (x0 + x1)(d0 + d1), and a0 b1 + a1 b0 is formed
            // from it and the other two sums at the end (exact mod q)
            const double d1 = dl[buf][s][kNd - 1][lane];
            acc[s][0] += mul_lazy(x0, d0, pr.q, pr.qinv);
            acc[s][1] += mul_lazy(xs, d0 + d1, pr.q, pr.qinv);
            acc[s][kNp - 1] += mul_lazy(x1, d1, pr.q, pr.qinv);
          } else {
            acc[s][0] += mul_lazy(x0, d0, pr.q, pr.qinv);
            acc[s][1] += mul_lazy(x1, d0, pr.q, pr.qinv);
          }
        }
      }
      if (++cnt == fold) {
        cnt = 0;
#pragma unroll
        for (int s = 0; s < GM; ++s)
#pragma unroll
          for (int p = 0; p < kNp; ++p) acc[s][p] = reduce_sym(acc[s][p], pr.q, pr.qinv);
      }
    }
    if (un < n_u) stage(buf ^ 1);
    // every wave is done with this step's tile and the next one is in place
    lds_barrier();
    buf ^= 1;
    u = un;
    mask = mask_n;
    x0 = xn0;
    x1 = xn1;
  }
  if (!has_b) return;
#pragma unroll
  for (int s = 0; s < GM; ++s) {
    if (s < gm) {
      double* op = out + ((size_t)(s0 + s) * G + b) * kNp * ps;
      if constexpr (kEnc) mm_karatsuba_mid(acc[s], pr.q, pr.qinv);
#pragma unroll
      for (int p = 0; p < kNp; ++p) op[(size_t)p * ps + o] = canon(reduce_sym(acc[s][p], pr.q, pr.qinv), pr.q);
    }
  }
}

template <int GM, bool kEnc>
static void mm_inner_launch(Context& c, double* out, const double* baby, const double* const* tab, int n_u, int ng,
                            int G, int nl, size_t baby_slot, size_t baby_b, const Pack& b0, int u0) {
  const unsigned tiles = (unsigned)((c.N + kMmLanes - 1) / kMmLanes);
  const unsigned gchunks = (unsigned)((ng + GM - 1) / GM);
  if (G == 1) {
    const unsigned nx = tiles * gchunks;
    hipLaunchKernelGGL((mm_inner_kernel<GM, kEnc>), dim3(nx, nl), dim3(256), 0, c.stream, out, baby, tab, n_u, ng,
                       nl, baby_slot, c.d_primes, (int)c.log_n, b0.p[0], u0);
  } else if (G % 8 == 0 && c.tune.mm_waves != 4) {
    // eight batch elements per workgroup: each staged diagonal tile feeds twice the products
    const unsigned nx = tiles * (unsigned)(G / 8) * gchunks;
    hipLaunchKernelGGL((mm_inner_batch_kernel<GM, kEnc, 8>), dim3(nx, nl), dim3(512), 0, c.stream, out, baby, tab,
                       n_u, ng, G, nl, baby_slot, baby_b, c.d_primes, (int)c.log_n, b0, u0);
  } else {
    const unsigned nx = tiles * (unsigned)((G + kMmWaves - 1) / kMmWaves) * gchunks;
    hipLaunchKernelGGL((mm_inner_batch_kernel<GM, kEnc, kMmWaves>), dim3(nx, nl), dim3(256), 0, c.stream, out, baby,
                       tab, n_u, ng, G, nl, baby_slot, baby_b, c.d_primes, (int)c.log_n, b0, u0);
  }
}

void launch_mm_inner(Context& c, double* out, const double* baby, const double* const* tab, int n_u, int ng, int G,
                     int nl, size_t baby_slot, size_t baby_b, bool enc, size_t nnz, int u0,
                     const std::vector<const double*>* b0) {
  if (ng <= 0 || G <= 0) return;
  if (u0 >= 0 && (!b0 || (int)b0->size() != G || G > kPack)) fail(COPSE_EINVAL, "internal: unrotated baby inputs");
  Pack p0{};
  for (int b = 0; u0 >= 0 && b < G; ++b) p0.p[b] = (*b0)[b];
  // one grid row holds every (tile, giant-group chunk, batch chunk); chunks of at least 4 groups
  if ((size_t)((c.N + kMmLanes - 1) / kMmLanes) * (size_t)((G + kMmWaves - 1) / kMmWaves) *
          (size_t)((ng + 3) / 4) * 256 > 0xffffffffu)
    fail(COPSE_EINVAL, "MatMul batch too large");
  hipEvent_t ev;
  prof_begin(c, 9, &ev);
  // giant groups in chunks of at most 24 (12 with three accumulators each, or for one batch element, whose
  // kernel holds a step's loads for every group: more, smaller chunks at higher occupancy measured faster),
  // split evenly
  const int cap = c.tune.mm_cap > 0 ? std::min(32, std::max(4, c.tune.mm_cap)) : (enc || G == 1 ? 12 : 24);
  const int chunks = (ng + cap - 1) / cap;
  const int per = (ng + chunks - 1) / chunks;
  auto run = [&](auto gm_tag) {
    constexpr int GM = decltype(gm_tag)::value;
    if (enc) mm_inner_launch<GM, true>(c, out, baby, tab, n_u, ng, G, nl, baby_slot, baby_b, p0, u0);
    else mm_inner_launch<GM, false>(c, out, baby, tab, n_u, ng, G, nl, baby_slot, baby_b, p0, u0);
  };
  if (per <= 4) run(std::integral_constant<int, 4>());
  else if (per <= 8) run(std::integral_constant<int, 8>());
  else if (per <= 12) run(std::integral_constant<int, 12>());
  else if (per <= 16) run(std::integral_constant<int, 16>());
  else if (per <= 24) run(std::integral_constant<int, 24>());
  else run(std::integral_constant<int, 32>());
  COPSE_HIP(hipGetLastError());
  // every baby step, every nonzero diagonal and every output read or written once
  prof_end(c, 9, ev, ((double)n_u * G * 2 + (double)nnz * (enc ? 2 : 1) + (double)ng * G * (enc ? 3 : 2)) * nl *
                         (double)c.N * 8.0);
}


// out_j = sum_{t < T} terms[j T + t] over rows_per_job rows (row r has prime r % nl)
__global__ void sum_terms_kernel(MPack out, Pack terms, int T, int nl, const DevPrime* P, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int r = blockIdx.y, j = blockIdx.z;
  const DevPrime& pr = P[r % nl];
  const size_t o = (size_t)r * N + i;
  double acc = terms.p[j * T][o];
  for (int t = 1; t < T; ++t) acc = mod_add(acc, terms.p[j * T + t][o], pr.q);
  out.p[j][o] = acc;
}

void launch_sum_terms(Context& c, const std::vector<double*>& out, const std::vector<const double*>& terms, int T,
                      int nl, int rows_per_job) {
  if (T <= 0 || T > kPack) fail(COPSE_EINVAL, "internal: sum of too many terms");
  const int per = kPack / T;
  for (size_t first = 0; first < out.size(); first += per) {
    const int cnt = (int)std::min<size_t>(per, out.size() - first);
    MPack po;
    Pack pt;
    for (int k = 0; k < cnt; ++k) {
      po.p[k] = out[first + k];
      for (int t = 0; t < T; ++t) pt.p[k * T + t] = terms[(first + k) * T + t];
    }
    hipEvent_t ev;
    prof_begin(c, 6, &ev);
    hipLaunchKernelGGL(sum_terms_kernel, dim3((unsigned)((c.N + 255) / 256), rows_per_job, cnt), dim3(256), 0,
                       c.stream, po, pt, T, nl, c.d_primes, (int)c.log_n);
    COPSE_HIP(hipGetLastError());
    prof_end(c, 6, ev, (T + 1.0) * rows_per_job * cnt * (double)c.N * 8.0);
  }
}

// encrypted comparison combine: eq = 2u - xs - ts + 1 (if want_eq), lt = ts - u
__global__ void seccomp_combine_kernel(MPack eq, MPack lt, Pack u, Pack xs, Pack ts, int nl, const DevPrime* P,
                                       int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int r = blockIdx.y, j = blockIdx.z;   // r < 2 nl
  const DevPrime& pr = P[r % nl];
  const size_t o = (size_t)r * N + i;
  const double uv = u.p[j][o], x = xs.p[j][o], tv = ts.p[j][o];
  if (eq.p[j]) {
    double v = mod_sub(mod_sub(mod_add(uv, uv, pr.q), x, pr.q), tv, pr.q);
    if (r < nl) v = mod_add(v, 1.0, pr.q);
    eq.p[j][o] = v;
  }
  lt.p[j][o] = mod_sub(tv, uv, pr.q);
}

void launch_seccomp_combine(Context& c, const std::vector<double*>& eq, const std::vector<double*>& lt,
                            const std::vector<const double*>& u, const std::vector<const double*>& xs,
                            const std::vector<const double*>& ts, int nl) {
  for (size_t first = 0; first < lt.size(); first += kPack) {
    int cnt = (int)std::min<size_t>(kPack, lt.size() - first);
    MPack pe, pl;
    Pack pu, px, pt;
    for (int k = 0; k < cnt; ++k) {
      pe.p[k] = eq[first + k]; pl.p[k] = lt[first + k];
      pu.p[k] = u[first + k]; px.p[k] = xs[first + k]; pt.p[k] = ts[first + k];
    }
    hipLaunchKernelGGL(seccomp_combine_kernel, dim3((unsigned)((c.N + 255) / 256), 2 * nl, cnt), dim3(256), 0,
                       c.stream, pe, pl, pu, px, pt, nl, c.d_primes, (int)c.log_n);
  }
  COPSE_HIP(hipGetLastError());
}

}  // namespace copse

namespace copse {
__global__ void calib_copy_kernel(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
void launch_calib_copy(Context& c, double* dst, const double* src, size_t n) {
  if (n == 0) return;
  const unsigned blocks = (unsigned)std::min<size_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(calib_copy_kernel, dim3(blocks), dim3(256), 0, c.stream, dst, src, n);
  COPSE_HIP(hipGetLastError());
}
}  // namespace copse
