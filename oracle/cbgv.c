/*
 * Plain ring kernels for the CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Every routine works on one residue polynomial (N unsigned 64-bit
 * coefficients) modulo one prime, with exact unsigned __int128 products.
 * Nothing here is shared with the GPU library.  The negacyclic transform
 * evaluates a(X) at the odd powers psi^(2i+1) of a primitive 2N-th root psi,
 * in natural order: out[i] = sum_j a_j psi^((2i+1) j) mod q.  It is used
 * only to multiply in Z_q[X]/(X^N + 1); the tests check it against schoolbook
 * negacyclic multiplication.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

static void bitrev_permute(uint64_t* a, size_t n) {
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
  }
}

/* Textbook iterative radix-2 cyclic transform: a[i] <- sum_j a_j w^(ij). */
static void cyclic_ntt(uint64_t* a, size_t n, uint64_t q, uint64_t w) {
  bitrev_permute(a, n);
  uint64_t* tw = (uint64_t*)malloc(sizeof(uint64_t) * (n / 2 + 1));
  for (size_t len = 2; len <= n; len <<= 1) {
    uint64_t wl = powmod(w, n / len, q);
    tw[0] = 1;
    for (size_t j = 1; j < len / 2; ++j) tw[j] = mulmod(tw[j - 1], wl, q);
    for (size_t i = 0; i < n; i += len) {
      for (size_t j = 0; j < len / 2; ++j) {
        uint64_t u = a[i + j];
        uint64_t v = mulmod(a[i + j + len / 2], tw[j], q);
        a[i + j] = (u + v) % q;
        a[i + j + len / 2] = (u + q - v) % q;
      }
    }
  }
  free(tw);
}

/* Forward negacyclic transform (coefficients -> evaluations at psi^(2i+1)). */
void oc_ntt_fwd(uint64_t* a, size_t n, uint64_t q, uint64_t psi) {
  uint64_t p = 1;
  for (size_t j = 0; j < n; ++j) { a[j] = mulmod(a[j], p, q); p = mulmod(p, psi, q); }
  cyclic_ntt(a, n, q, mulmod(psi, psi, q));
}

/* Inverse of oc_ntt_fwd. */
void oc_ntt_inv(uint64_t* a, size_t n, uint64_t q, uint64_t psi) {
  uint64_t psi_inv = powmod(psi, q - 2, q);
  uint64_t w_inv = mulmod(psi_inv, psi_inv, q);
  cyclic_ntt(a, n, q, w_inv);
  uint64_t n_inv = powmod((uint64_t)n % q, q - 2, q);
  uint64_t p = n_inv;
  for (size_t j = 0; j < n; ++j) { a[j] = mulmod(a[j], p, q); p = mulmod(p, psi_inv, q); }
}

/* out[i] = a[i] * b[i] mod q */
void oc_mul(uint64_t* out, const uint64_t* a, const uint64_t* b, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) out[i] = mulmod(a[i], b[i], q);
}

/* acc[i] = (acc[i] + a[i] * b[i]) mod q */
void oc_mac(uint64_t* acc, const uint64_t* a, const uint64_t* b, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) acc[i] = (uint64_t)(((u128)a[i] * b[i] + acc[i]) % q);
}

/* out[i] = a[i] * s mod q */
void oc_mul_scalar(uint64_t* out, const uint64_t* a, size_t n, uint64_t q, uint64_t s) {
  for (size_t i = 0; i < n; ++i) out[i] = mulmod(a[i], s, q);
}

/*
 * Fast base conversion of one coefficient vector from primes in_q[0..n_in)
 * to primes out_p[0..n_out):
 *   y_i = [x_i * qhat_inv[i]]_{in_q[i]},  out_o = sum_i y_i * qhat_mod[i*n_out+o] mod out_p[o]
 * with qhat_inv[i] = (Q/q_i)^-1 mod q_i and qhat_mod[i][o] = (Q/q_i) mod p_o.
 * in: n_in rows of n; out: n_out rows of n.
 */
void oc_fastbconv(uint64_t* out, const uint64_t* in, size_t n, size_t n_in, const uint64_t* in_q,
                  size_t n_out, const uint64_t* out_p, const uint64_t* qhat_inv,
                  const uint64_t* qhat_mod) {
  uint64_t* y = (uint64_t*)malloc(sizeof(uint64_t) * n_in);
  for (size_t c = 0; c < n; ++c) {
    for (size_t i = 0; i < n_in; ++i) y[i] = mulmod(in[i * n + c], qhat_inv[i], in_q[i]);
    for (size_t o = 0; o < n_out; ++o) {
      u128 acc = 0;
      for (size_t i = 0; i < n_in; ++i) acc += (u128)y[i] * (qhat_mod[i * n_out + o] % out_p[o]);
      out[o * n + c] = (uint64_t)(acc % out_p[o]);
    }
  }
  free(y);
}

/* Schoolbook negacyclic product, used only to pin the transform. */
void oc_negacyclic_schoolbook(uint64_t* out, const uint64_t* a, const uint64_t* b, size_t n, uint64_t q) {
  for (size_t k = 0; k < n; ++k) out[k] = 0;
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j) {
      uint64_t p = mulmod(a[i], b[j], q);
      size_t k = i + j;
      if (k < n) out[k] = (out[k] + p) % q;
      else out[k - n] = (out[k - n] + q - p) % q;
    }
}
