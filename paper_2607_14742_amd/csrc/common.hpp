// Internal declarations shared by the library's translation units.
// Host-side runtime: errors, the device-memory arena, the context, and the
// launch helpers every kernel file uses.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <rocblas/rocblas.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "mpcare.h"

namespace mpcare {

// ----------------------------------------------------------------------------
// errors: internal code throws CareError; the ABI layer converts it to a status
// ----------------------------------------------------------------------------
struct CareError {
  care_status status;
  std::string msg;
};

void set_last_error(const std::string& msg);
const char* last_error_cstr();
[[noreturn]] void fail(care_status st, const std::string& msg);

#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      ::mpcare::fail(_e == hipErrorOutOfMemory ? CARE_ERR_NOMEM : CARE_ERR_DEVICE,        \
                     std::string(#expr) + ": " + hipGetErrorString(_e));                  \
  } while (0)

#define ROCBLAS_CHECK(expr)                                                               \
  do {                                                                                    \
    rocblas_status _s = (expr);                                                           \
    if (_s != rocblas_status_success)                                                     \
      ::mpcare::fail(CARE_ERR_DEVICE, std::string(#expr) + ": rocblas status " +          \
                                          std::to_string((int)_s));                       \
  } while (0)

#define KERNEL_CHECK() HIP_CHECK(hipGetLastError())

// ----------------------------------------------------------------------------
// precision tags
// ----------------------------------------------------------------------------
using bf16 = __hip_bfloat16;
using f16 = _Float16;

// F16 and BF16: FP32 inner solves whose sparse products read the off-diagonal
// values of A in a 16-bit format (F16 with a power-of-two operator scale)
enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

inline Prec prec_from_abi(int32_t p) {
  if (p == CARE_FP64) return Prec::F64;
  if (p == CARE_FP32) return Prec::F32;
  if (p == CARE_BF16_SPMM) return Prec::BF16;
  if (p == CARE_FP16_SPMM) return Prec::F16;
  fail(CARE_ERR_ARG, "unknown precision " + std::to_string(p));
}
inline size_t vec_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }   // Krylov vectors
inline size_t val_bytes(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }

// ----------------------------------------------------------------------------
// device memory arena (grow-only caching allocator owned by a context)
// ----------------------------------------------------------------------------
// Device blocks come from hipMalloc, or from the caller's hooks when the
// context was created with them (care_ctx_create).
struct AllocHooks {
  care_alloc_fn alloc = nullptr;
  care_dealloc_fn dealloc = nullptr;
  void* user = nullptr;
  bool set() const { return alloc != nullptr; }
};

class Arena {
 public:
  Arena(hipStream_t s, const AllocHooks& h) : stream_(s), hooks_(h) {}
  ~Arena();
  void* get(size_t bytes);
  void put(void* p);
  void trim();   // return every cached block to the device (after a stream sync)
  // return cached blocks, largest first, until at most `keep` bytes stay cached
  void trim_to(size_t keep);
  size_t in_use() const { return in_use_; }
  size_t cached() const { return cached_; }

 private:
  void* device_alloc(size_t bytes);
  void device_free(void* p, size_t bytes);
  hipStream_t stream_;
  AllocHooks hooks_;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> live_;
  size_t in_use_ = 0;
  size_t cached_ = 0;
};

// ----------------------------------------------------------------------------
// context
// ----------------------------------------------------------------------------
struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;        // the library's own stream (non-blocking)
  hipStream_t user_stream = nullptr;   // the caller's stream: calls are ordered after it
  hipEvent_t order_event = nullptr;
  rocblas_handle blas = nullptr;
  AllocHooks hooks;                // the caller's device allocator (or none)
  Arena* arena = nullptr;
  void* pinned = nullptr;          // small pinned host staging buffer
  size_t pinned_bytes = 0;
  int num_cu = 256;
  // sparse-product accounting (care_stats)
  int profile = 0;
  int64_t spmm_calls = 0;
  double spmm_bytes = 0.0;
  bool spmm_defer = false;          // bytes of sparse launches counted by the caller
  int64_t spmm_pending[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // deferred launches per sparse-product mode
  int spmm_split = 0;               // BiCGStab products: 0 auto, 1 fused, 2 split
  int spmm_tune = 0;                // 1: time the panel widths of a product shape once, keep the faster
  int krylov_method = 0;            // shifted solves: 0 BiCGStab, 1 restarted GMRES (real shifts)
  int krylov_patient = 0;           // BiCGStab stagnation window max(1000, it/2) (unshifted solves)
  int krylov_graphs = 1;            // 0: no HIP-graph capture of Krylov chunks (batch worker contexts)
  int krylov_rb = 1;                // 1: shifted solves through the red-black reduction where it applies
  int spmm_force_cp = 0;            // 8 / 16: panel width of every wide product (product timing), 0: chosen
  int gram_impl = 2;                // large FP64 Grams: 0 rocBLAS dgemm, 1 the own 128 x 128-tile MFMA
                                    // kernel, 2 the own kernel where measured faster (symmetric Grams)
  int spmm_force_pg = 0;            // > 0: column panels per workgroup (product timing), 0: chosen
  int krylov_compact = 1;           // BiCGStab: gather the still-active columns into fewer panels
  int krylov_restart = 0;           // GMRES restart length (0: 30 in FP32, 50 in FP64)
  int krylov_precond = 0;           // 1: GMRES right-preconditioned by ILU(0) where the operator has it
  // profile mode: the events the next k_spmm launch records at its own start
  // and end (set by SpmmTimer; null otherwise)
  hipEvent_t spmm_ev0 = nullptr, spmm_ev1 = nullptr;
  double t_spmm = 0.0;
  int64_t krylov_iters = 0;
  int64_t krylov_compactions = 0;
  int64_t adi_rotations = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending_events;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
  void reset_counters() {
    spmm_calls = 0;
    spmm_bytes = 0;
    t_spmm = 0;
    krylov_iters = 0;
    krylov_compactions = 0;
    adi_rotations = 0;
  }
  void* host_stage(size_t bytes);  // pinned buffer of at least `bytes`
  void sync();                     // stream synchronize + harvest profile events
  std::pair<hipEvent_t, hipEvent_t> event_pair();
};

// Set up a context on `device`: its own non-blocking stream (default
// priority), the ordering event, a rocBLAS handle and the workspace arena.
// `user_stream` is the caller's stream the context's work is ordered after.
void ctx_init(Ctx& c, int device, hipStream_t user_stream, const AllocHooks& hooks = AllocHooks());
// Release everything ctx_init acquired (waits for the stream first).
void ctx_release(Ctx& c);
// Look up, once per device, the address of the allocation-free entry
// point's fixed device array (called by ctx_init with the device current).
void scratch_setup(int device);
size_t scratch_doubles();


// RAII device buffer from the context arena
template <typename T>
struct DBuf {
  Ctx* ctx = nullptr;
  T* ptr = nullptr;
  size_t count = 0;
  DBuf() = default;
  DBuf(Ctx* c, size_t n) : ctx(c), count(n) {
    ptr = n ? static_cast<T*>(c->arena->get(n * sizeof(T))) : nullptr;
  }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : ctx(o.ctx), ptr(o.ptr), count(o.count) { o.ptr = nullptr; o.count = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    release();
    ctx = o.ctx; ptr = o.ptr; count = o.count;
    o.ptr = nullptr; o.count = 0;
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (ptr && ctx) ctx->arena->put(ptr);
    ptr = nullptr;
    count = 0;
  }
  void resize(Ctx* c, size_t n) {   // discards contents
    if (n <= count && ptr) return;
    release();
    ctx = c;
    count = n;
    ptr = n ? static_cast<T*>(c->arena->get(n * sizeof(T))) : nullptr;
  }
  T* get() const { return ptr; }
};

// copies between host and device on the context stream (synchronous)
void d2h(Ctx* ctx, void* host, const void* dev, size_t bytes);
void h2d(Ctx* ctx, void* dev, const void* host, size_t bytes);
void d2d(Ctx* ctx, void* dst, const void* src, size_t bytes);
void dzero(Ctx* ctx, void* dst, size_t bytes);   // fill kernel, never a memset node

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// leading dimension of internal n x k panels: rows rounded up to 64
inline int64_t pad_ld(int64_t n) { return (n + 63) / 64 * 64; }

// XCD-aware workgroup remap: consecutive logical blocks land on the same XCD
// (8 XCDs, round-robin dispatch), so neighbouring row blocks share an L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned nx = 8;
  unsigned per = nb / nx, rem = nb % nx;
  unsigned x = b % nx, i = b / nx;
  // blocks of XCD x get logical ids [x*per + min(x, rem), ...)
  unsigned base = x * per + (x < rem ? x : rem);
  unsigned cnt = per + (x < rem ? 1u : 0u);
  return i < cnt ? base + i : b;
}

}  // namespace mpcare
