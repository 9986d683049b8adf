// Host utilities: errors, number theory, SHAKE-256 (FIPS 202) and the
// samplers, and the device memory pool.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace copse {

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

// ------------------------------------------------------------------ number theory
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)((unsigned __int128)a * b % m);
}

uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}

// Extended Euclid; m need not be prime.
uint64_t invmod(uint64_t a, uint64_t m) {
  __int128 t0 = 0, t1 = 1, r0 = m, r1 = a % m;
  while (r1 != 0) {
    __int128 qq = r0 / r1, tmp;
    tmp = r0 - qq * r1; r0 = r1; r1 = tmp;
    tmp = t0 - qq * t1; t0 = t1; t1 = tmp;
  }
  if (r0 != 1) fail(COPSE_EINVAL, "value not invertible");
  if (t0 < 0) t0 += m;
  return (uint64_t)t0;
}

// Miller-Rabin with the first twelve primes as bases: deterministic for all 64-bit n.
bool is_prime(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; ++i) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

// An element of exact multiplicative order `order` (a power of two here) mod prime q.
uint64_t root_of_unity(uint64_t order, uint64_t q) {
  if ((q - 1) % order) fail(COPSE_EINVAL, "order does not divide q-1");
  for (uint64_t g = 2; g < q; ++g) {
    uint64_t r = powmod(g, (q - 1) / order, q);
    // order is a power of two: r has exact order iff r^(order/2) = -1
    if (powmod(r, order / 2, q) == q - 1) return r;
  }
  fail(COPSE_EINVAL, "no root of unity");
}

uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

// ------------------------------------------------------------------ Keccak-f[1600] / SHAKE-256
namespace {
struct KeccakConsts {
  uint64_t rc[24];
  int rho[25];
  KeccakConsts() {
    // round constants from the LFSR rc(t) of FIPS 202, Algorithm 5
    auto rcbit = [](int t) -> int {
      if (t % 255 == 0) return 1;
      unsigned R = 0x01;  // bits R[0..7] = 1,0,...,0
      for (int i = 1; i <= t % 255; ++i) {
        R <<= 1;                       // R = 0 || R   (R[8] is the old R[7])
        unsigned r8 = (R >> 8) & 1;
        R ^= r8 | (r8 << 4) | (r8 << 5) | (r8 << 6);
        R &= 0xFF;
      }
      return R & 1;
    };
    for (int ir = 0; ir < 24; ++ir) {
      uint64_t v = 0;
      for (int j = 0; j <= 6; ++j)
        if (rcbit(j + 7 * ir)) v |= 1ULL << ((1 << j) - 1);
      rc[ir] = v;
    }
    // rho offsets (FIPS 202, Algorithm 2)
    for (int i = 0; i < 25; ++i) rho[i] = 0;
    int x = 1, y = 0;
    for (int t = 0; t < 24; ++t) {
      rho[x + 5 * y] = ((t + 1) * (t + 2) / 2) % 64;
      int nx = y, ny = (2 * x + 3 * y) % 5;
      x = nx; y = ny;
    }
  }
};
const KeccakConsts& kc() {
  static KeccakConsts k;
  return k;
}
inline uint64_t rotl(uint64_t v, int r) { return r ? (v << r) | (v >> (64 - r)) : v; }

void keccak_f(uint64_t A[25]) {
  const KeccakConsts& K = kc();
  for (int ir = 0; ir < 24; ++ir) {
    uint64_t C[5], D[5], B[25];
    for (int x = 0; x < 5; ++x) C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];
    for (int x = 0; x < 5; ++x) D[x] = C[(x + 4) % 5] ^ rotl(C[(x + 1) % 5], 1);
    for (int i = 0; i < 25; ++i) A[i] ^= D[i % 5];
    // rho and pi: B[y, 2x+3y] = rot(A[x, y])
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y) B[y + 5 * ((2 * x + 3 * y) % 5)] = rotl(A[x + 5 * y], K.rho[x + 5 * y]);
    for (int x = 0; x < 5; ++x)
      for (int y = 0; y < 5; ++y)
        A[x + 5 * y] = B[x + 5 * y] ^ (~B[(x + 1) % 5 + 5 * y] & B[(x + 2) % 5 + 5 * y]);
    A[0] ^= K.rc[ir];
  }
}
constexpr size_t kRate = 136;

void absorb_all(uint64_t st[25], const uint8_t* msg, size_t len) {
  std::memset(st, 0, 25 * sizeof(uint64_t));
  uint8_t block[kRate];
  size_t off = 0;
  while (true) {
    size_t take = std::min(kRate, len - off);
    std::memset(block, 0, kRate);
    std::memcpy(block, msg + off, take);
    bool last = take < kRate;
    if (last) {
      block[take] ^= 0x1F;          // SHAKE domain bits + first pad bit
      block[kRate - 1] ^= 0x80;     // last pad bit
    }
    for (size_t i = 0; i < kRate / 8; ++i) {
      uint64_t lane = 0;
      for (int b = 0; b < 8; ++b) lane |= (uint64_t)block[8 * i + b] << (8 * b);
      st[i] ^= lane;
    }
    keccak_f(st);
    off += take;
    if (last) break;
  }
}
}  // namespace

void shake256(const uint8_t* msg, size_t len, uint8_t* out, size_t outlen) {
  uint64_t st[25];
  absorb_all(st, msg, len);
  size_t done = 0;
  while (done < outlen) {
    size_t take = std::min(kRate, outlen - done);
    for (size_t i = 0; i < take; ++i) out[done + i] = (uint8_t)(st[i / 8] >> (8 * (i % 8)));
    done += take;
    if (done < outlen) keccak_f(st);
  }
}

ShakeStream::ShakeStream(const uint8_t seed[32], const char* domain, uint64_t obj, uint32_t limb) {
  std::vector<uint8_t> msg(seed, seed + 32);
  for (const char* p = domain; *p; ++p) msg.push_back((uint8_t)*p);
  for (int i = 0; i < 8; ++i) msg.push_back((uint8_t)(obj >> (8 * i)));
  for (int i = 0; i < 4; ++i) msg.push_back((uint8_t)(limb >> (8 * i)));
  absorb_all(st_, msg.data(), msg.size());
  permute_block();
}

void ShakeStream::permute_block() {
  // st_ already permuted: expose its first rate bytes
  for (size_t i = 0; i < kRate; ++i) buf_[i] = (uint8_t)(st_[i / 8] >> (8 * (i % 8)));
  pos_ = 0;
}

void ShakeStream::read(uint8_t* out, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    if (pos_ == kRate) {
      keccak_f(st_);
      permute_block();
    }
    out[i] = buf_[pos_++];
  }
}

void sample_uniform(const uint8_t seed[32], const char* dom, uint64_t obj, uint32_t limb, uint64_t q,
                    size_t n, double* out) {
  ShakeStream s(seed, dom, obj, limb);
  int bits = 64 - __builtin_clzll(q);
  uint64_t mask = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
  size_t got = 0;
  uint8_t b[8];
  while (got < n) {
    s.read(b, 8);
    uint64_t w = 0;
    for (int i = 0; i < 8; ++i) w |= (uint64_t)b[i] << (8 * i);
    w &= mask;
    if (w < q) out[got++] = (double)w;
  }
}

void sample_ternary(const uint8_t seed[32], const char* dom, uint64_t obj, size_t n, int64_t* out) {
  ShakeStream s(seed, dom, obj, 0);
  size_t got = 0;
  uint8_t b;
  while (got < n) {
    s.read(&b, 1);
    if (b == 255) continue;
    int v = b % 3;
    out[got++] = v == 2 ? -1 : v;
  }
}

void sample_cbd21(const uint8_t seed[32], const char* dom, uint64_t obj, size_t n, int64_t* out) {
  ShakeStream s(seed, dom, obj, 0);
  uint8_t b[6];
  for (size_t i = 0; i < n; ++i) {
    s.read(b, 6);
    uint64_t w = 0;
    for (int k = 0; k < 6; ++k) w |= (uint64_t)b[k] << (8 * k);
    int lo = __builtin_popcountll(w & ((1ULL << 21) - 1));
    int hi = __builtin_popcountll((w >> 21) & ((1ULL << 21) - 1));
    out[i] = lo - hi;
  }
}

// ------------------------------------------------------------------ pool
Pool::~Pool() {
  hipSetDevice(device_);
  for (auto& kv : cache_)
    for (void* p : kv.second) (void)hipFree(p);
  for (auto& kv : live_) (void)hipFree(kv.first);
}

static size_t round_size(size_t b) {
  if (b <= 4096) return 4096;
  size_t g = 1ULL << (63 - __builtin_clzll(b));
  size_t step = g / 8;   // 8 size classes per power of two
  return (b + step - 1) / step * step;
}

void* Pool::alloc(size_t bytes) {
  std::lock_guard<std::mutex> lk(mu_);
  size_t sz = round_size(bytes);
  auto it = cache_.find(sz);
  void* p = nullptr;
  if (it != cache_.end() && !it->second.empty()) {
    p = it->second.back();
    it->second.pop_back();
  } else {
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess && !keep_cached_) {
      // release cached blocks and retry once
      for (auto& kv : cache_) {
        for (void* q : kv.second) { (void)hipFree(q); held_ -= kv.first; }
        kv.second.clear();
      }
      (void)hipGetLastError();
      e = hipMalloc(&p, sz);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(COPSE_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
    }
    held_ += sz;
  }
  live_[p] = sz;
  live_bytes_ += sz;
  peak_bytes_ = std::max(peak_bytes_, live_bytes_);
  return p;
}

void Pool::free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto it = live_.find(p);
  if (it == live_.end()) return;
  cache_[it->second].push_back(p);
  live_bytes_ -= it->second;
  live_.erase(it);
}

size_t Pool::live_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return live_bytes_;
}

size_t Pool::peak_bytes() {
  std::lock_guard<std::mutex> lk(mu_);
  return peak_bytes_;
}

void Pool::reset_peak() {
  std::lock_guard<std::mutex> lk(mu_);
  peak_bytes_ = live_bytes_;
}

void Pool::trim() {
  std::lock_guard<std::mutex> lk(mu_);
  if (keep_cached_) return;
  for (auto& kv : cache_) {
    for (void* q : kv.second) { (void)hipFree(q); held_ -= kv.first; }
    kv.second.clear();
  }
}

}  // namespace copse
