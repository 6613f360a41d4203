// Entry point that allocates nothing: the Gram product of care_gram with its
// row-split partials in a fixed device array, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// `scratch` is a file-scope device array of SCRATCH_DOUBLES doubles (32 MiB),
// one copy per GPU the library runs on, held until the process ends.  Host
// code never passes its name to a kernel: the name is a host-side stand-in.
// Every context set-up looks up the array's device address for its device
// once (hipGetSymbolAddress with that device current) and keeps it per
// device; the kernels get that address as an argument.
//
// Every call on one GPU shares that GPU's array and leaves its partial sums
// in it; calls that overlap on one GPU race on it.  Each call overwrites
// every partial it reads (each (row split, tile) block writes its whole
// 32 x 32 tile), so nothing has to start at zero.
#include <mutex>

#include "care.hpp"
#include "dense.hpp"

namespace mpcare {

constexpr size_t SCRATCH_DOUBLES = size_t(4) << 20;   // 32 MiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_ptr;           // device -> address of its `scratch`

void scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return;
  int cur = -1;
  HIP_CHECK(hipGetDevice(&cur));
  if (cur != device) HIP_CHECK(hipSetDevice(device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) fail(CARE_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<double*>(p);
}

static double* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) fail(CARE_ERR_DEVICE, "scratch array of this device was not set up");
  return it->second;
}

size_t scratch_doubles() { return SCRATCH_DOUBLES; }

void gram_noalloc(Ctx* ctx, int64_t n, const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                  double* C, int64_t ldc) {
  double* part = scratch_of(ctx->device);
  if (n == 0) fail(CARE_ERR_ARG, "n = 0: the Gram is zero (use care_gram)");
  if (!gram_own_into(ctx, n, X, ldx, a, Y, ldy, b, C, ldc, part, SCRATCH_DOUBLES))
    fail(CARE_ERR_ARG, "a and b too large for the fixed scratch array: ceil(a/32) ceil(b/32) must be <= " +
                           std::to_string(SCRATCH_DOUBLES / 1024));
}

}  // namespace mpcare
