// Evaluation without device allocation: copse_evaluate for callers that cannot allocate device memory.
//
// Every temporary of the evaluation comes from one file-scope device array (`scratch`), a fixed
// kScratchBytes per GPU held from the library's load until the process ends.  Host code never uses the
// array's name as an address: when a context is created, its device's copy of the array is looked up
// once with hipGetSymbolAddress (each GPU has its own copy at its own address) and only that pointer is
// handed to kernels and copies.  A call takes the device's array for itself (one call at a time per GPU
// in this process), runs the ordinary batched schedule with a first-fit allocator over the array in place
// of the context's caching pool, copies the result into the caller's ciphertext with a copy kernel,
// waits for the device and releases the array, whose contents then stay as the last call left them.
// Nothing the schedule reads has to start at zero: every scratch buffer is written before it is read.
// The per-level tables are built when the context is created; a row list not cached yet is built inside
// the array for the duration of the call.
#include <algorithm>
#include <map>

#include "compiled.hpp"

namespace copse {

constexpr size_t kScratchBytes = COPSE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

struct DeviceScratch {
  char* ptr = nullptr;   // this device's copy of `scratch`
  std::mutex busy;       // held by the call using it
};

std::mutex g_devices_mu;
std::map<int, std::unique_ptr<DeviceScratch>> g_devices;

DeviceScratch& device_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_devices_mu);
  auto it = g_devices.find(device);
  if (it == g_devices.end() || !it->second->ptr)
    fail(COPSE_EDEVICE, "scratch array of device " + std::to_string(device) + " not looked up");
  return *it->second;
}

// First-fit allocator over [base, base + cap): 256-byte blocks, freed blocks merged with their neighbours.
class ScratchPool : public Pool {
 public:
  ScratchPool(int device, char* base, size_t cap) : Pool(device, true), base_(base), cap_(cap) { free_[0] = cap; }
  void* alloc(size_t bytes) override {
    const size_t sz = std::max<size_t>(256, (bytes + 255) / 256 * 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < sz) continue;
      const size_t off = it->first, rest = it->second - sz;
      free_.erase(it);
      if (rest) free_[off + sz] = rest;
      live_[off] = sz;
      used_ += sz;
      peak_ = std::max(peak_, used_);
      return base_ + off;
    }
    fail(COPSE_ENOMEM, "evaluation needs more than the " + std::to_string(cap_ >> 20) +
                           " MiB scratch array of copse_evaluate_noalloc (" + std::to_string(used_ >> 20) +
                           " MiB in use, " + std::to_string(sz) + " bytes asked)");
  }
  void free(void* p) override {
    if (!p) return;
    auto it = live_.find((size_t)((char*)p - base_));
    if (it == live_.end()) return;
    size_t off = it->first, sz = it->second;
    used_ -= sz;
    live_.erase(it);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + sz == nx->first) {
      sz += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += sz;
        return;
      }
    }
    free_[off] = sz;
  }
  size_t peak() const { return peak_; }

 private:
  char* base_;
  size_t cap_;
  std::map<size_t, size_t> free_;   // offset -> size
  std::map<size_t, size_t> live_;
  size_t used_ = 0, peak_ = 0;
};

// While alive: the context allocates from the scratch pool, records no profiling events and builds
// missing row lists per call.  On exit (also after a failure) it waits for the device, so that nothing
// enqueued by the call still reads the array or a host row list when the next call begins.
struct NoAllocScope {
  Context& c;
  std::shared_ptr<Pool> saved;
  bool prof;
  NoAllocScope(Context& c_, std::shared_ptr<Pool> scratch_pool) : c(c_), saved(c_.pool), prof(c_.profiling) {
    c.pool = std::move(scratch_pool);
    c.profiling = false;
    c.no_alloc = true;
  }
  ~NoAllocScope() {
    (void)hipStreamSynchronize(c.stream);
    c.call_rows.clear();
    c.call_row_bufs.clear();
    c.call_rows_host.clear();
    c.no_alloc = false;
    c.pool = saved;
    c.profiling = prof;
  }
};

}  // namespace

void scratch_acquire(int device) {
  std::lock_guard<std::mutex> lk(g_devices_mu);
  auto& slot = g_devices[device];
  if (!slot) slot = std::make_unique<DeviceScratch>();
  if (slot->ptr) return;
  void* p = nullptr;
  COPSE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  slot->ptr = static_cast<char*>(p);
}

void evaluate_group_noalloc(Context& c, const Model& M, const Keys& k, const std::vector<const Ct*>& planes,
                            Ct& out) {
  if (out.level != 0 || out.npolys != 2 || out.n != c.N)
    fail(COPSE_EINVAL, "result must be one ciphertext of this ring at level 0 with 2 polynomials");
  if (M.noalloc_too_big)
    fail(COPSE_ENOMEM, "this model's evaluation needs more than the " + std::to_string(kScratchBytes >> 20) +
                           " MiB scratch array of copse_evaluate_noalloc");
  DeviceScratch& S = device_scratch(c.device);
  std::lock_guard<std::mutex> lk(S.busy);
  COPSE_HIP(hipSetDevice(c.device));
  auto pool = std::make_shared<ScratchPool>(c.device, S.ptr, kScratchBytes);
  try {
    NoAllocScope scope(c, pool);
    CtPtr r = evaluate_group(c, M, k, planes);
    if (r->level != 0 || r->npolys != 2) fail(COPSE_EINVAL, "internal: result shape");
    launch_copy(c, out.data(), r->data(), out.words());
  } catch (const Error& e) {
    if (e.code == COPSE_ENOMEM) M.noalloc_too_big = true;
    throw;
  }
  M.noalloc_peak = std::max(M.noalloc_peak, pool->peak());
}

}  // namespace copse
