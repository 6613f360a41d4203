// Context, arena and small runtime helpers.
#include "common.hpp"

#include <cstdlib>
#include <cstring>
#include <mutex>

namespace mpcare {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

void fail(care_status st, const std::string& msg) { throw CareError{st, msg}; }

// ---------------------------------------------------------------------------
// Arena
// ---------------------------------------------------------------------------
static size_t round_bytes(size_t b) {
  const size_t g = (b < (size_t(1) << 20)) ? 4096 : (size_t(2) << 20);
  return (b + g - 1) / g * g;
}

void* Arena::device_alloc(size_t bytes) {
  if (hooks_.set()) return hooks_.alloc(bytes, (void*)stream_, hooks_.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void Arena::device_free(void* p, size_t bytes) {
  if (hooks_.set()) hooks_.dealloc(p, bytes, (void*)stream_, hooks_.user);
  else (void)hipFree(p);
}

Arena::~Arena() {
  // blocks may still be read by queued work: wait before handing them back
  (void)hipStreamSynchronize(stream_);
  for (auto& kv : free_) device_free(kv.second, kv.first);
  for (auto& kv : live_) device_free(kv.first, kv.second);
}

void* Arena::get(size_t bytes) {
  size_t rb = round_bytes(bytes ? bytes : 1);
  auto it = free_.lower_bound(rb);
  // reuse a cached block that is not more than 2x too large
  if (it != free_.end() && it->first <= 2 * rb + (size_t(4) << 20)) {
    void* p = it->second;
    size_t sz = it->first;
    free_.erase(it);
    cached_ -= sz;
    live_[p] = sz;
    in_use_ += sz;
    return p;
  }
  void* p = device_alloc(rb);
  if (!p) {
    // release the cache and retry once
    (void)hipStreamSynchronize(stream_);
    for (auto& kv : free_) device_free(kv.second, kv.first);
    free_.clear();
    cached_ = 0;
    p = device_alloc(rb);
    if (!p) fail(CARE_ERR_NOMEM, "device allocation of " + std::to_string(rb) + " bytes failed");
  }
  live_[p] = rb;
  in_use_ += rb;
  return p;
}

void Arena::trim() { trim_to(0); }

void Arena::trim_to(size_t keep) {
  if (cached_ <= keep) return;
  (void)hipStreamSynchronize(stream_);
  while (cached_ > keep && !free_.empty()) {
    auto it = std::prev(free_.end());   // largest cached block
    device_free(it->second, it->first);
    cached_ -= it->first;
    free_.erase(it);
  }
}

void Arena::put(void* p) {
  auto it = live_.find(p);
  if (it == live_.end()) return;
  in_use_ -= it->second;
  cached_ += it->second;
  free_.emplace(it->second, p);
  live_.erase(it);
}

// ---------------------------------------------------------------------------
// Ctx
// ---------------------------------------------------------------------------
void* Ctx::host_stage(size_t bytes) {
  if (bytes > pinned_bytes) {
    // an earlier asynchronous host-to-device copy (h2d returns before its
    // copy has run) may still read the old buffer: wait before freeing it
    if (pinned) {
      HIP_CHECK(hipStreamSynchronize(stream));
      HIP_CHECK(hipHostFree(pinned));
    }
    pinned = nullptr;
    size_t nb = std::max(bytes, size_t(1) << 20);
    HIP_CHECK(hipHostMalloc(&pinned, nb, hipHostMallocDefault));
    pinned_bytes = nb;
  }
  return pinned;
}

std::pair<hipEvent_t, hipEvent_t> Ctx::event_pair() {
  if (!event_pool.empty()) {
    auto e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t a, b;
  HIP_CHECK(hipEventCreate(&a));
  HIP_CHECK(hipEventCreate(&b));
  return {a, b};
}

void Ctx::sync() {
  HIP_CHECK(hipStreamSynchronize(stream));
  for (auto& e : pending_events) {
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e.first, e.second));
    t_spmm += ms * 1e-3;
    event_pool.push_back(e);
  }
  pending_events.clear();
}

void d2h(Ctx* ctx, void* host, const void* dev, size_t bytes) {
  if (!bytes) return;
  void* st = ctx->host_stage(bytes);
  HIP_CHECK(hipMemcpyAsync(st, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  std::memcpy(host, st, bytes);
}

void h2d(Ctx* ctx, void* dev, const void* host, size_t bytes) {
  if (!bytes) return;
  void* st = ctx->host_stage(bytes);
  // the staging buffer may still be read by an earlier async copy
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
  std::memcpy(st, host, bytes);
  HIP_CHECK(hipMemcpyAsync(dev, st, bytes, hipMemcpyHostToDevice, ctx->stream));
  HIP_CHECK(hipStreamSynchronize(ctx->stream));
}

void d2d(Ctx* ctx, void* dst, const void* src, size_t bytes) {
  if (!bytes || dst == src) return;
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0u;
}
__global__ void k_fill_u8(uint8_t* __restrict__ p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void dzero(Ctx* ctx, void* dst, size_t bytes) {
  if (!bytes) return;
  size_t words = bytes / 4;
  if (words) {
    unsigned grid = (unsigned)std::min<size_t>((words + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, ctx->stream, (uint32_t*)dst, words);
    KERNEL_CHECK();
  }
  size_t tail = bytes - words * 4;
  if (tail) {
    hipLaunchKernelGGL(k_fill_u8, dim3(1), dim3(64), 0, ctx->stream, (uint8_t*)dst + words * 4, tail);
    KERNEL_CHECK();
  }
}

void ctx_init(Ctx& c, int device, hipStream_t user_stream, const AllocHooks& hooks) {
  HIP_CHECK(hipSetDevice(device));
  c.device = device;
  c.user_stream = user_stream;
  c.hooks = hooks;
  HIP_CHECK(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));   // default priority
  HIP_CHECK(hipEventCreateWithFlags(&c.order_event, hipEventDisableTiming));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c.num_cu = prop.multiProcessorCount;
  // MPCARE_GRAM=0 / 1 / 2 picks the implementation of the large FP64 Grams
  // (rocBLAS / the own kernel / the own kernel where it is faster, default)
  if (const char* g = std::getenv("MPCARE_GRAM")) {
    const int v = std::atoi(g);
    c.gram_impl = v >= 0 && v <= 2 ? v : 2;
  }
  c.arena = new Arena(c.stream, c.hooks);
  scratch_setup(device);
  if (rocblas_create_handle(&c.blas) != rocblas_status_success) {
    c.blas = nullptr;
    ctx_release(c);
    fail(CARE_ERR_DEVICE, "rocblas_create_handle failed");
  }
  rocblas_set_stream(c.blas, c.stream);
  // reproducible products: no split-K kernels that sum with atomics
  rocblas_set_atomics_mode(c.blas, rocblas_atomics_not_allowed);
}

void ctx_release(Ctx& c) {
  (void)hipSetDevice(c.device);
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  for (auto& e : c.event_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& e : c.pending_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  c.event_pool.clear();
  c.pending_events.clear();
  if (c.blas) rocblas_destroy_handle(c.blas);
  c.blas = nullptr;
  delete c.arena;
  c.arena = nullptr;
  if (c.pinned) (void)hipHostFree(c.pinned);
  c.pinned = nullptr;
  if (c.order_event) (void)hipEventDestroy(c.order_event);
  c.order_event = nullptr;
  if (c.stream) (void)hipStreamDestroy(c.stream);
  c.stream = nullptr;
}

}  // namespace mpcare
