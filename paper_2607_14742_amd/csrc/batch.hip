// Batched Framework 1 over independent CARE instances of uneven sizes.
//
// Each instance runs the single-instance solver unchanged.  Concurrency comes
// from W worker threads, each owning a context (non-blocking stream, rocBLAS
// handle, workspace arena) on the same device: the host-side decisions of one
// instance (Krylov polls, eigen-splits) never stall the kernels of another,
// and the sparse products of small instances, which alone cannot fill 256
// CUs, overlap on the device.  Instances are taken largest first from a
// shared list (longest-processing-time order), so the big ones do not start
// last.  A memory budget (60 % of the device memory free at the start) caps
// the estimated peak workspace of the instances running at once: a worker
// takes the largest waiting instance that fits, or waits; an instance runs
// alone when nothing else does.  The estimate can fall short (factor widths
// depend on the problem, and other users of the device hold memory too): an
// instance whose device allocation fails is queued again once, to run alone
// when the other workers are idle.  Running out of device
// memory mid-solve can also starve the runtime's own allocations (kernel
// scratch), which is not an error the library could catch.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>

#include "care.hpp"

namespace mpcare {

void solve_batch(Ctx* ctx, int count, const care_instance* inst, double tol, const care_opts* opts, int workers,
                 care_instance_result* res) {
  if (count < 0) fail(CARE_ERR_ARG, "negative instance count");
  if (count == 0) return;
  if (!inst || !res) fail(CARE_ERR_ARG, "instances or results is NULL");
  const int nw = workers > 0 ? std::min(workers, count) : std::min(count, 8);
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto spec_of = [&](int k) -> OpSpec {
    return inst[k].A ? sparse_spec(inst[k].A) : dense_spec(inst[k].A_dense, inst[k].n_dense, inst[k].lda_dense);
  };
  auto size_of = [&](int k) -> int64_t {
    const OpSpec s = spec_of(k);
    return (s.csr || s.dense) ? s.size() : 0;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return size_of(a) > size_of(b); });
  for (int k = 0; k < count; ++k) {
    std::memset(&res[k], 0, sizeof(res[k]));
    res[k].status = CARE_ERR_DEVICE;   // until a worker has run the instance
    std::strncpy(res[k].message, "not run", sizeof(res[k].message) - 1);
  }

  // estimated peak workspace per instance: the Newton corrections keep a few
  // FP64 n x (hundreds to thousands) panels (ADI factor, Algorithm 2 basis,
  // orthogonalisation remainder); dense instances add one LU per shift
  const int prec = opts ? opts->inner_prec : CARE_FP64;
  const int l0 = opts && opts->penzl_l0 > 0 ? opts->penzl_l0 : 16;
  auto estimate = [&](int k) -> double {
    const OpSpec sp = spec_of(k);
    if (!sp.csr && !sp.dense) return 0.0;
    const double n = (double)sp.size();
    const double per_row = prec == CARE_FP64 ? 64e3 : 128e3;
    double e = n * per_row;
    if (sp.dense) e += n * n * (prec == CARE_FP64 ? 8.0 : 4.0) * (l0 + 2) + 3.0 * n * n * 8.0;
    return e;
  };
  size_t mem_free = 0, mem_total = 0;
  HIP_CHECK(hipMemGetInfo(&mem_free, &mem_total));
  const double budget = 0.6 * (double)mem_free;
  std::mutex mu;
  std::condition_variable cv;
  std::vector<char> taken(count, 0), alone(count, 0);
  int remaining = count, running = 0;
  double in_use = 0.0;
  // next instance for a worker (largest waiting one that fits), or -1 when
  // none is left; blocks while none fits
  auto acquire = [&](double& est) -> int {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      if (remaining == 0) return -1;
      for (int i = 0; i < count; ++i) {
        const int k = order[i];
        if (taken[k]) continue;
        if (alone[k] && running > 0) continue;
        const double e = estimate(k);
        if (running == 0 || in_use + e <= budget) {
          taken[k] = 1;
          --remaining;
          ++running;
          in_use += e;
          est = e;
          return k;
        }
      }
      cv.wait(lk);
    }
  };
  // requeue: an instance that ran out of device memory runs again alone
  // (once); its result is reset under the lock, before another worker can
  // take it
  auto release = [&](double est, int k, bool requeue) {
    {
      std::lock_guard<std::mutex> lk(mu);
      --running;
      in_use -= est;
      if (requeue && !alone[k]) {
        std::memset(&res[k], 0, sizeof(res[k]));
        res[k].status = CARE_ERR_DEVICE;
        std::strncpy(res[k].message, "not run", sizeof(res[k].message) - 1);
        alone[k] = 1;
        taken[k] = 0;
        ++remaining;
      }
    }
    cv.notify_all();
  };
  std::vector<std::string> setup_err(nw);
  auto work = [&](int w) {
    Ctx wc;
    try {
      // the worker threads are the library's own: they allocate with hipMalloc
      // rather than call the caller's allocator hooks from threads the caller
      // did not create (the hooks' contract)
      ctx_init(wc, ctx->device, ctx->stream);
      // no HIP-graph capture in the workers: while one worker's stream is in
      // capture, another worker's device-synchronising calls (hipFree in the
      // per-instance cache trim, pinned staging reallocation, the vendor
      // libraries' workspace allocations) would have to synchronise a
      // capturing stream.  The concurrent workers hide the launch latency the
      // graphs save in a single solve.
      wc.krylov_graphs = 0;
      // ordered after everything the caller queued (ctx->stream waits on it)
      HIP_CHECK(hipEventRecord(wc.order_event, wc.user_stream));
      HIP_CHECK(hipStreamWaitEvent(wc.stream, wc.order_event, 0));
    } catch (const CareError& e) {
      setup_err[w] = e.msg;
      return;
    } catch (...) {
      setup_err[w] = "worker context setup failed";
      return;
    }
    double est = 0.0;
    for (int k; (k = acquire(est)) >= 0;) {
      const care_instance& I = inst[k];
      care_instance_result& R = res[k];
      int r = 0;
      care_status warn = CARE_OK;
      R.message[0] = '\0';
      try {
        const OpSpec spec = spec_of(k);
        if (!spec.csr && !spec.dense) fail(CARE_ERR_ARG, "instance A is NULL");
        if (spec.size() < 1 || (spec.dense && spec.lda < spec.n)) fail(CARE_ERR_ARG, "instance A is empty or invalid");
        care_solve_impl(&wc, spec, I.B, I.m, I.C, I.p, tol, I.shifts, I.nshifts, opts, I.Z, I.ldz, I.rmax, &r,
                        &R.stats, &warn);
        R.status = warn;
      } catch (const CareError& e) {
        R.status = e.status;
        std::strncpy(R.message, e.msg.c_str(), sizeof(R.message) - 1);
      } catch (const std::bad_alloc&) {
        R.status = CARE_ERR_NOMEM;
        std::strncpy(R.message, "host allocation failed", sizeof(R.message) - 1);
      } catch (...) {
        R.status = CARE_ERR_DEVICE;
        std::strncpy(R.message, "internal error", sizeof(R.message) - 1);
      }
      R.r = r;
      try {
        wc.sync();   // a failed instance may leave work queued
      } catch (...) {
      }
      // concurrent workers share the device memory: hand this instance's
      // cached workspace back before the next one
      wc.arena->trim();
      release(est, k, R.status == CARE_ERR_NOMEM);
    }
    ctx_release(wc);
  };
  std::vector<std::thread> th;
  th.reserve(nw);
  for (int w = 0; w < nw; ++w) th.emplace_back(work, w);
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w)
    if (!setup_err[w].empty()) fail(CARE_ERR_DEVICE, "batch worker: " + setup_err[w]);
}

}  // namespace mpcare
