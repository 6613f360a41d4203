// extern "C" entry points: argument checks, context handling, conversion of
// internal errors to status codes.  No exception crosses this boundary.
#include <cstring>

#include "care.hpp"
#include "lu.hpp"

using namespace mpcare;

struct care_ctx {
  Ctx c;
};

namespace {

template <typename F>
care_status guarded(F&& f) {
  try {
    set_last_error("");
    return f();
  } catch (const CareError& e) {
    set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return CARE_ERR_NOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CARE_ERR_DEVICE;
  } catch (...) {
    set_last_error("unknown internal error");
    return CARE_ERR_DEVICE;
  }
}

// Every entry point runs on the context's own non-blocking stream (graph
// capture is not possible on the legacy default stream), ordered after the
// work already queued on the caller's stream.
Ctx* unwrap(care_ctx* c) {
  if (!c) fail(CARE_ERR_ARG, "context is NULL");
  HIP_CHECK(hipSetDevice(c->c.device));
  HIP_CHECK(hipEventRecord(c->c.order_event, c->c.user_stream));
  HIP_CHECK(hipStreamWaitEvent(c->c.stream, c->c.order_event, 0));
  return &c->c;
}

// After a solve the workspace cache may hold tens of GB (wide refinement
// panels): keep a modest amount for the next call, hand the rest back.
void release_cache(Ctx* ctx) { ctx->arena->trim_to(size_t(4) << 30); }

void check_csr_shape(const care_csr* A) {
  if (!A) fail(CARE_ERR_ARG, "A is NULL");
  if (A->n < 1) fail(CARE_ERR_ARG, "A must have n >= 1");
}

}  // namespace

extern "C" {

const char* care_version(void) { return "mpcare 0.1 (gfx950)"; }

care_status care_struct_sizes(int64_t* sizes, int32_t count) {
  return guarded([&]() -> care_status {
    if (!sizes || count < 0 || count > 6) fail(CARE_ERR_ARG, "sizes is NULL or count outside [0, 6]");
    const int64_t all[6] = {(int64_t)sizeof(care_csr),  (int64_t)sizeof(care_shift),
                            (int64_t)sizeof(care_opts), (int64_t)sizeof(care_stats),
                            (int64_t)sizeof(care_instance), (int64_t)sizeof(care_instance_result)};
    for (int i = 0; i < count; ++i) sizes[i] = all[i];
    return CARE_OK;
  });
}

const char* care_last_error(void) { return last_error_cstr(); }

void care_opts_default(care_opts* o, int32_t inner_prec) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->inner_prec = inner_prec;
  o->k_max = 20;
  o->k0_max = 20;
  o->j_max = 50;
  o->eta_r_rel = 1e-4;
  o->eta_s_rel = 10.0 * 1.1102230246251565e-16;
  o->tau_L = 0.0;          // precision default
  o->tau_0 = 0.0;
  o->stagnation = 0.999;
  o->krylov_maxit = 4000;
  o->krylov_tol = 0.0;     // precision default
  o->check_every = 8;
  o->penzl_l0 = 16;
  o->penzl_kp = 20;
  o->penzl_km = 10;
  o->penzl_real = 0;
  o->spmm_split = 0;
  o->krylov_relax = 1;
  o->refine_forcing = 0.25;
  o->tau_L0 = 0.0;         // precision default
  o->spmm_tune = 1;
  o->shift_update = 0;
  o->krylov_method = 0;
  o->krylov_restart = 0;
  o->krylov_compact = 1;
  o->adi_rotate = 1;
  o->profile = 0;
  o->Z_init = nullptr;
  o->ldz_init = 0;
  o->r_init = 0;
  o->adi_deflate = 1;
  o->krylov_block_tol = -1;
  o->krylov_rb = 1;
  o->krylov_precond = 0;
}

care_status care_ctx_create(care_ctx** out, int32_t device, void* stream, care_alloc_fn alloc,
                            care_dealloc_fn dealloc, void* user) {
  return guarded([&]() -> care_status {
    if (!out) fail(CARE_ERR_ARG, "ctx output pointer is NULL");
    *out = nullptr;
    if ((alloc == nullptr) != (dealloc == nullptr)) fail(CARE_ERR_ARG, "alloc and dealloc must both be set or both NULL");
    AllocHooks hooks;
    hooks.alloc = alloc;
    hooks.dealloc = dealloc;
    hooks.user = user;
    int count = 0;
    HIP_CHECK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) fail(CARE_ERR_ARG, "device index out of range");
    care_ctx* c = new care_ctx();
    try {
      ctx_init(c->c, device, (hipStream_t)stream, hooks);
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
    return CARE_OK;
  });
}

void care_ctx_destroy(care_ctx* c) {
  if (!c) return;
  ctx_release(c->c);
  delete c;
}

care_status care_spmm(care_ctx* cx, const care_csr* A, int32_t prec, care_shift p, const double* X, int64_t ldx,
                      int32_t k, double* Y, int64_t ldy) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const Prec pr = prec_from_abi(prec);
    if (k < 0) fail(CARE_ERR_ARG, "k must be >= 0");
    if (k == 0) return CARE_OK;
    if (!X || !Y || ldx < A->n || ldy < A->n) fail(CARE_ERR_ARG, "invalid X / Y");
    if (!std::isfinite(p.re) || !std::isfinite(p.im)) fail(CARE_ERR_ARG, "shift not finite");
    SellOp op;
    build_sell(ctx, A, pr, op);
    const int64_t n = A->n, ld = pad_ld(n);
    const bool cp = p.im != 0.0;
    const int kr = cp ? 2 * k : k;
    std::vector<int> map(kr);
    for (int c = 0; c < kr; ++c) map[c] = cp ? ((c % 2) ? k + c / 2 : c / 2) : c;
    std::vector<int> inv(kr);
    for (int c = 0; c < kr; ++c) inv[map[c]] = c;
    if (pr == Prec::F64) {
      DBuf<double> xi(ctx, (size_t)ld * kr), yi(ctx, (size_t)ld * kr);
      copy_cols<double, double>(ctx, n, kr, X, ldx, xi.get(), ld, map.data());
      spmm_plain(ctx, op, p.re, p.im, xi.get(), ld, kr, yi.get(), ld);
      copy_cols<double, double>(ctx, n, kr, yi.get(), ld, Y, ldy, inv.data());
    } else {
      DBuf<float> xi(ctx, (size_t)ld * kr), yi(ctx, (size_t)ld * kr);
      copy_cols<double, float>(ctx, n, kr, X, ldx, xi.get(), ld, map.data());
      spmm_plain(ctx, op, p.re, p.im, xi.get(), ld, kr, yi.get(), ld);
      copy_cols<float, double>(ctx, n, kr, yi.get(), ld, Y, ldy, inv.data());
    }
    ctx->sync();
    return CARE_OK;
  });
}

care_status care_spmm_timing(care_ctx* cx, const care_csr* A, int32_t prec, care_shift p, int32_t k, int32_t nsets,
                             int32_t reps, int32_t panel, int32_t panels_per_block, double* us_per_product,
                             double* bytes_per_product) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const Prec pr = prec_from_abi(prec);
    if (k < 1 || nsets < 1 || reps < 1) fail(CARE_ERR_ARG, "k, nsets and reps must be >= 1");
    if (panel != 0 && panel != 8 && panel != 16) fail(CARE_ERR_ARG, "panel must be 0, 8 or 16");
    if (panels_per_block < 0) fail(CARE_ERR_ARG, "panels_per_block must be >= 0");
    if (!us_per_product || !bytes_per_product) fail(CARE_ERR_ARG, "output pointer is NULL");
    if (!std::isfinite(p.re) || !std::isfinite(p.im)) fail(CARE_ERR_ARG, "shift not finite");
    const bool cp = p.im != 0.0;
    const int kr = cp ? 2 * k : k;
    std::vector<SellOp> ops(nsets);
    for (auto& op : ops) build_sell(ctx, A, pr, op);
    const int64_t n = A->n, ld = pad_ld(n);
    const size_t vb = vec_bytes(pr);
    DBuf<uint8_t> X(ctx, (size_t)nsets * ld * kr * vb), Y(ctx, (size_t)nsets * ld * kr * vb);
    // inputs of ones (any finite values: the timing does not depend on them)
    if (pr == Prec::F64) fill_const<double>(ctx, (double*)X.get(), (size_t)nsets * ld * kr, 1.0);
    else fill_const<float>(ctx, (float*)X.get(), (size_t)nsets * ld * kr, 1.0);
    ctx->spmm_tune = 0;
    ctx->spmm_force_cp = panel;
    ctx->spmm_force_pg = panels_per_block;
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    auto round = [&]() {
      for (int sI = 0; sI < nsets; ++sI) {
        void* xs = X.get() + (size_t)sI * ld * kr * vb;
        void* ys = Y.get() + (size_t)sI * ld * kr * vb;
        spmm_plain(ctx, ops[sI], p.re, p.im, xs, ld, kr, ys, ld);
      }
    };
    round();   // warm-up (code objects, first touch)
    HIP_CHECK(hipEventRecord(e0, ctx->stream));
    for (int r = 0; r < reps; ++r) round();
    HIP_CHECK(hipEventRecord(e1, ctx->stream));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->spmm_force_cp = 0;
    ctx->spmm_force_pg = 0;
    *us_per_product = 1e3 * (double)ms / ((double)reps * nsets);
    *bytes_per_product = ops[0].bytes(kr, 2);
    ctx->sync();
    return CARE_OK;
  });
}

care_status care_shifted_lu_factor(care_ctx* cx, int32_t prec, int64_t n, const void* M0, const double* shifts,
                                   int32_t nshifts, void* F, int32_t* perm, int32_t* info) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (prec != CARE_FP32 && prec != CARE_FP64) fail(CARE_ERR_ARG, "prec must be CARE_FP32 or CARE_FP64");
    if (n < 1 || n > LU_NMAX) fail(CARE_ERR_ARG, "n must be in [1, " + std::to_string(LU_NMAX) + "]");
    if (nshifts < 0) fail(CARE_ERR_ARG, "nshifts must be >= 0");
    if (nshifts == 0) return CARE_OK;
    if (!M0 || !shifts || !F || !perm || !info) fail(CARE_ERR_ARG, "NULL argument");
    const size_t es = prec == CARE_FP32 ? 4 : 8;
    const size_t mat = (size_t)n * n * es;
    const char* f0 = (const char*)F;
    const char* m0 = (const char*)M0;
    if (f0 < m0 + mat && m0 < f0 + mat * nshifts) fail(CARE_ERR_ARG, "F overlaps M0");
    std::vector<double> sh(shifts, shifts + nshifts);
    for (double v : sh)
      if (!std::isfinite(v)) fail(CARE_ERR_ARG, "shift not finite");
    std::vector<int*> P(nshifts);
    for (int s = 0; s < nshifts; ++s) P[s] = perm + (int64_t)s * n;
    std::vector<int> inf;
    if (prec == CARE_FP32) {
      std::vector<float*> Fs(nshifts);
      for (int s = 0; s < nshifts; ++s) Fs[s] = (float*)F + (int64_t)s * n * n;
      lu_factor_shifted<float>(ctx, (int)n, (const float*)M0, sh, Fs, P, inf);
    } else {
      std::vector<double*> Fs(nshifts);
      for (int s = 0; s < nshifts; ++s) Fs[s] = (double*)F + (int64_t)s * n * n;
      lu_factor_shifted<double>(ctx, (int)n, (const double*)M0, sh, Fs, P, inf);
    }
    for (int s = 0; s < nshifts; ++s) info[s] = inf[s];
    return CARE_OK;
  });
}

care_status care_shifted_lu_solve(care_ctx* cx, int32_t prec, int64_t n, const void* F, const int32_t* perm,
                                  int32_t k, const void* B, int64_t ldb, void* X, int64_t ldx) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (prec != CARE_FP32 && prec != CARE_FP64) fail(CARE_ERR_ARG, "prec must be CARE_FP32 or CARE_FP64");
    if (n < 1 || n > LU_NMAX) fail(CARE_ERR_ARG, "n must be in [1, " + std::to_string(LU_NMAX) + "]");
    if (k < 0) fail(CARE_ERR_ARG, "k must be >= 0");
    if (k == 0) return CARE_OK;
    if (!F || !perm || !B || !X || ldb < n || ldx < n) fail(CARE_ERR_ARG, "invalid F / perm / B / X");
    if (B == X && ldb != ldx) fail(CARE_ERR_ARG, "in-place solve needs ldx == ldb");
    if (prec == CARE_FP32)
      lu_solve<float>(ctx, (int)n, (const float*)F, perm, k, (const float*)B, ldb, (float*)X, ldx);
    else
      lu_solve<double>(ctx, (int)n, (const double*)F, perm, k, (const double*)B, ldb, (double*)X, ldx);
    ctx->sync();
    return CARE_OK;
  });
}

static care_status shifted_solve_entry(care_ctx* cx, const care_csr* A, const double* B, int64_t ldb,
                                       const double* K, int64_t ldk, int32_t m, care_shift p, const double* W,
                                       int64_t ldw, int32_t w, int32_t prec, double tol, int32_t maxit,
                                       const care_opts* km, double* V, int64_t ldv, int32_t* iters) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const Prec pr = prec_from_abi(prec);
    const int64_t n = A->n, ld = pad_ld(n);
    if (w < 0 || m < 0) fail(CARE_ERR_ARG, "w and m must be >= 0");
    // the Krylov method: BiCGStab with the red-black reduction unless km says otherwise
    ctx->krylov_method = km ? km->krylov_method : 0;
    ctx->krylov_restart = km ? km->krylov_restart : 0;
    ctx->krylov_compact = km ? km->krylov_compact : 1;
    ctx->krylov_rb = km ? km->krylov_rb : 1;
    ctx->krylov_precond = km ? km->krylov_precond : 0;
    if (ctx->krylov_method < 0 || ctx->krylov_method > 1) fail(CARE_ERR_ARG, "krylov_method must be 0 or 1");
    if (ctx->krylov_precond < 0 || ctx->krylov_precond > 1) fail(CARE_ERR_ARG, "krylov_precond must be 0 or 1");
    if (w == 0) return CARE_OK;
    if (!W || !V || ldw < n || ldv < n) fail(CARE_ERR_ARG, "invalid W / V");
    const bool smw = K != nullptr && m > 0;
    if (smw && (!B || ldb < n || ldk < n)) fail(CARE_ERR_ARG, "invalid B / K");
    if (!(p.re < 0) || !std::isfinite(p.re) || !std::isfinite(p.im)) fail(CARE_ERR_ARG, "shift needs Re p < 0");
    SellOp op;
    build_sell(ctx, A, pr, op);
    if (ctx->krylov_rb) rb_attach(ctx, rb_analyse(ctx, A), pr, op);
    if (ctx->krylov_precond) ilu_attach(ctx, ilu_analyse(ctx, A), op);
    care_opts d;
    care_opts_default(&d, prec);
    d.krylov_tol = tol;
    d.krylov_maxit = maxit;
    Resolved r = resolve_opts(&d, 1e-10);
    LradiParams lp;
    lp.ktol = r.ktol;
    lp.kmaxit = r.kmaxit;
    lp.check_every = r.check_every;
    const bool cp = p.im != 0.0;
    const int vc = cp ? 2 * w : w;
    std::vector<int> inv(vc);
    for (int c = 0; c < vc; ++c) inv[c] = cp ? ((c < w) ? 2 * c : 2 * (c - w) + 1) : c;
    KrylovResult kr;
    auto run = [&](auto tag) {
      using T = decltype(tag);
      DBuf<T> Bs(ctx, (size_t)ld * std::max(m, 1)), Ks(ctx, (size_t)ld * std::max(m, 1)), Ws(ctx, (size_t)ld * w),
          Vs(ctx, (size_t)ld * vc);
      if (smw) {
        copy_cols<double, T>(ctx, n, m, B, ldb, Bs.get(), ld);
        copy_cols<double, T>(ctx, n, m, K, ldk, Ks.get(), ld);
      }
      copy_cols<double, T>(ctx, n, w, W, ldw, Ws.get(), ld);
      kr = shifted_solve<T>(ctx, op, Bs.get(), smw ? Ks.get() : nullptr, smw ? m : 0, Ws.get(), w, Shift{p.re, p.im},
                            lp, Vs.get());
      copy_cols<T, double>(ctx, n, vc, Vs.get(), ld, V, ldv, inv.data());
    };
    if (pr == Prec::F64) run(double{});
    else run(float{});
    ctx->sync();
    if (iters) *iters = kr.max_iters;
    return kr.unconverged ? CARE_WARN_MAXIT : CARE_OK;
  });
}

care_status care_shifted_solve(care_ctx* cx, const care_csr* A, const double* B, int64_t ldb, const double* K,
                               int64_t ldk, int32_t m, care_shift p, const double* W, int64_t ldw, int32_t w,
                               int32_t prec, double tol, int32_t maxit, double* V, int64_t ldv, int32_t* iters) {
  return shifted_solve_entry(cx, A, B, ldb, K, ldk, m, p, W, ldw, w, prec, tol, maxit, nullptr, V, ldv, iters);
}

care_status care_shifted_solve_opts(care_ctx* cx, const care_csr* A, const double* B, int64_t ldb,
                                    const double* K, int64_t ldk, int32_t m, care_shift p, const double* W,
                                    int64_t ldw, int32_t w, int32_t prec, double tol, int32_t maxit,
                                    const care_opts* opts, double* V, int64_t ldv, int32_t* iters) {
  return shifted_solve_entry(cx, A, B, ldb, K, ldk, m, p, W, ldw, w, prec, tol, maxit, opts, V, ldv, iters);
}

care_status care_ilu0_factor(care_ctx* cx, const care_csr* A, int32_t prec, double p, int32_t* colours,
                             double* off, int64_t noff, double* udiag) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const Prec pr = prec_from_abi(prec);
    if (!std::isfinite(p)) fail(CARE_ERR_ARG, "shift must be finite");
    if (!colours || !udiag || (noff > 0 && !off)) fail(CARE_ERR_ARG, "output pointer is NULL");
    SellOp op;
    build_sell(ctx, A, pr, op);
    const std::shared_ptr<IluHost> h = ilu_analyse(ctx, A);
    ilu_attach(ctx, h, op);
    const std::shared_ptr<IluOp::Factors> f = ilu_factor(ctx, op, p);
    const int64_t n = op.n;
    const int nsl = op.nslices;
    std::vector<int> sptr(nsl + 1), cols((size_t)op.width_total * 64), col(n);
    d2h(ctx, sptr.data(), op.sptr.get(), (nsl + 1) * sizeof(int));
    if (!cols.empty()) d2h(ctx, cols.data(), op.cols.get(), cols.size() * sizeof(int));
    d2h(ctx, col.data(), op.ilu->colour.get(), n * sizeof(int));
    const bool dbl = pr == Prec::F64;
    const size_t vb = vec_bytes(pr);
    std::vector<uint8_t> fo(cols.size() * vb), fd(n * vb);
    if (!fo.empty()) d2h(ctx, fo.data(), f->off.get(), fo.size());
    d2h(ctx, fd.data(), f->dinv.get(), fd.size());
    auto val = [&](const std::vector<uint8_t>& v, size_t e) -> double {
      return dbl ? reinterpret_cast<const double*>(v.data())[e] : (double)reinterpret_cast<const float*>(v.data())[e];
    };
    // the SELL rows hold A^T's off-diagonal entries in column order, padding last
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
      for (int q = sptr[i >> 6]; q < sptr[(i >> 6) + 1]; ++q) cnt += cols[(size_t)q * 64 + (i & 63)] != i;
    if (cnt != noff) fail(CARE_ERR_CAPACITY, "off must hold the " + std::to_string(cnt) +
                                                 " off-diagonal nonzeros of A");
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i) {
      colours[i] = col[i];
      udiag[i] = 1.0 / val(fd, i);
      for (int q = sptr[i >> 6]; q < sptr[(i >> 6) + 1]; ++q) {
        const size_t e = (size_t)q * 64 + (i & 63);
        if (cols[e] != i) off[t++] = val(fo, e);
      }
    }
    return CARE_OK;
  });
}

care_status care_ilu0_apply(care_ctx* cx, const care_csr* A, int32_t prec, double p, const double* X, int64_t ldx,
                            int32_t k, double* Z, int64_t ldz) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const Prec pr = prec_from_abi(prec);
    const int64_t n = A->n, ld = pad_ld(n);
    if (!std::isfinite(p)) fail(CARE_ERR_ARG, "shift must be finite");
    if (k < 0) fail(CARE_ERR_ARG, "k must be >= 0");
    if (k == 0) return CARE_OK;
    if (!X || !Z || ldx < n || ldz < n) fail(CARE_ERR_ARG, "invalid X / Z");
    SellOp op;
    build_sell(ctx, A, pr, op);
    ilu_attach(ctx, ilu_analyse(ctx, A), op);
    const std::shared_ptr<IluOp::Factors> f = ilu_factor(ctx, op, p);
    auto run = [&](auto tag) {
      using T = decltype(tag);
      DBuf<T> Xs(ctx, (size_t)ld * k), Zs(ctx, (size_t)ld * k);
      copy_cols<double, T>(ctx, n, k, X, ldx, Xs.get(), ld);
      ilu_apply<T>(ctx, op, *f, k, Xs.get(), ld, Zs.get(), ld);
      copy_cols<T, double>(ctx, n, k, Zs.get(), ld, Z, ldz);
    };
    if (pr == Prec::F64) run(double{});
    else run(float{});
    ctx->sync();
    return CARE_OK;
  });
}

care_status care_gram(care_ctx* cx, int64_t n, const double* X, int64_t ldx, int32_t a, const double* Y, int64_t ldy,
                      int32_t b, double* Cm, int64_t ldc) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (n < 0 || a < 0 || b < 0) fail(CARE_ERR_ARG, "negative size");
    if (a == 0 || b == 0) return CARE_OK;
    if (!X || !Y || !Cm || ldx < std::max<int64_t>(n, 1) || ldy < std::max<int64_t>(n, 1) || ldc < a)
      fail(CARE_ERR_ARG, "invalid pointers or leading dimensions");
    gram<double, double>(ctx, n, X, ldx, a, Y, ldy, b, Cm, ldc);
    ctx->sync();
    return CARE_OK;
  });
}

care_status care_gram_noalloc(care_ctx* cx, int64_t n, const double* X, int64_t ldx, int32_t a, const double* Y,
                              int64_t ldy, int32_t b, double* Cm, int64_t ldc) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (n < 0 || a < 0 || b < 0) fail(CARE_ERR_ARG, "negative size");
    if (a == 0 || b == 0) return CARE_OK;
    if (!X || !Y || !Cm || ldx < std::max<int64_t>(n, 1) || ldy < std::max<int64_t>(n, 1) || ldc < a)
      fail(CARE_ERR_ARG, "invalid pointers or leading dimensions");
    const int64_t tiles = (int64_t)((a + 31) / 32) * ((b + 31) / 32);
    if (tiles * 1024 > (int64_t)scratch_doubles())
      fail(CARE_ERR_ARG, "a x b beyond the fixed scratch array: ceil(a/32) ceil(b/32) must be <= " +
                             std::to_string(scratch_doubles() / 1024));
    gram_noalloc(ctx, n, X, ldx, a, Y, ldy, b, Cm, ldc);
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    return CARE_OK;
  });
}

care_status care_tsgemm(care_ctx* cx, int64_t n, const double* X, int64_t ldx, int32_t q, const double* S,
                        int64_t lds, int32_t k, double alpha, double beta, double* Y, int64_t ldy) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (n < 0 || q < 0 || k < 0) fail(CARE_ERR_ARG, "negative size");
    if (n == 0 || k == 0) return CARE_OK;
    if (!Y || ldy < n || (q > 0 && (!X || !S || ldx < n || lds < q)))
      fail(CARE_ERR_ARG, "invalid pointers or leading dimensions");
    tsgemm<double, double>(ctx, n, X, ldx, q, S, lds, k, alpha, beta, Y, ldy);
    ctx->sync();
    return CARE_OK;
  });
}

care_status lyap_lradi(care_ctx* cx, const care_csr* A, const double* B, const double* K, int32_t m,
                       const double* W, int64_t ldw, int32_t w, const care_shift* shifts, int32_t nshifts,
                       double tol, const care_opts* opts, double* Z, int64_t ldz, int32_t rmax, int32_t* r_out,
                       care_stats* stats) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const int64_t n = A->n, ld = pad_ld(n);
    if (w < 0 || m < 0) fail(CARE_ERR_ARG, "w and m must be >= 0");
    if (!r_out) fail(CARE_ERR_ARG, "r_out is NULL");
    if (w > 0 && (!W || ldw < n)) fail(CARE_ERR_ARG, "invalid W");
    if (!Z || ldz < n || rmax < 0) fail(CARE_ERR_ARG, "invalid Z");
    const bool smw = K != nullptr && m > 0;
    if (smw && !B) fail(CARE_ERR_ARG, "B is NULL while K is given");
    care_opts d;
    care_opts_default(&d, CARE_FP64);
    const care_opts* o = opts ? opts : &d;
    // nshifts = 0 with shift_update = 2: projection shifts (at most
    // penzl_l0 per set) drawn from W and the run's own iterates
    const bool proj = nshifts == 0 && o->shift_update == 2;
    if (proj && o->penzl_l0 < 1) fail(CARE_ERR_ARG, "projection shifts need penzl_l0 >= 1");
    std::vector<Shift> sh = proj ? std::vector<Shift>() : check_shifts(shifts, nshifts);
    Resolved r = resolve_opts(o, 1e-10);
    LradiParams lp;
    lp.proj_shifts = proj ? o->penzl_l0 : 0;
    lp.tol = tol > 0 ? tol : r.tau_L;
    lp.jmax = r.j_max;
    lp.ktol = r.ktol;
    lp.kmaxit = r.kmaxit;
    lp.check_every = r.check_every;
    lp.deflate = false;      // keep the documented block layout of Z
    lp.relax = o->krylov_relax != 0;
    ctx->reset_counters();
    ctx->profile = o->profile;
    ctx->spmm_split = o->spmm_split;
    ctx->spmm_tune = o->spmm_tune;
    ctx->krylov_method = o->krylov_method;
    ctx->krylov_restart = o->krylov_restart;
    ctx->krylov_compact = o->krylov_compact;
    ctx->krylov_rb = o->krylov_rb;
    ctx->krylov_precond = o->krylov_precond;
    if (ctx->krylov_precond < 0 || ctx->krylov_precond > 1) fail(CARE_ERR_ARG, "krylov_precond must be 0 or 1");
    const double t0 = now_s();
    SellOp op;
    build_sell(ctx, A, r.prec, op);
    if (ctx->krylov_rb) rb_attach(ctx, rb_analyse(ctx, A), r.prec, op);
    if (ctx->krylov_precond) ilu_attach(ctx, ilu_analyse(ctx, A), op);
    LradiOut lo;
    const int zcap = lradi_capacity(w, lp.jmax);
    auto run = [&](auto tag) {
      using T = decltype(tag);
      DBuf<T> Bs(ctx, (size_t)ld * std::max(m, 1)), Ks(ctx, (size_t)ld * std::max(m, 1)),
          Ws(ctx, (size_t)ld * std::max(w, 1));
      ZBuffer<T> Zs;
      Zs.init(ctx, n, std::min(zcap, 16 * std::max(w, 1)));
      if (smw) {
        copy_cols<double, T>(ctx, n, m, B, n, Bs.get(), ld);
        copy_cols<double, T>(ctx, n, m, K, n, Ks.get(), ld);
      }
      copy_cols<double, T>(ctx, n, w, W, ldw, Ws.get(), ld);
      lo = lradi_run<T>(ctx, op, Bs.get(), smw ? Ks.get() : nullptr, smw ? m : 0, Ws.get(), w, sh, lp, Zs, zcap);
      *r_out = lo.zcols;
      if (lo.zcols > rmax) fail(CARE_ERR_CAPACITY, "Z needs " + std::to_string(lo.zcols) + " columns");
      copy_cols<T, double>(ctx, n, lo.zcols, Zs.get(), ld, Z, ldz);
    };
    if (w > 0) {
      if (r.prec == Prec::F64) run(double{});
      else run(float{});
    } else {
      *r_out = 0;
    }
    ctx->sync();
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->iter_outer = 1;
      stats->iter_inner = lo.steps;
      stats->rank = lo.zcols;
      stats->res_rel = lo.res_rel;
      stats->t_total = now_s() - t0;
      stats->spmm_calls = ctx->spmm_calls;
      stats->spmm_bytes = ctx->spmm_bytes;
      stats->t_spmm = ctx->t_spmm;
      stats->krylov_iters = ctx->krylov_iters;
      stats->krylov_compactions = (int32_t)ctx->krylov_compactions;
      stats->adi_rotations = (int32_t)ctx->adi_rotations;
      stats->hist_len = 1;
      stats->res_hist[0] = lo.res_rel;
    }
    release_cache(ctx);
    if (w > 0 && lo.res_rel > lp.tol) return CARE_WARN_MAXIT;
    return lo.krylov_unconverged ? CARE_WARN_MAXIT : CARE_OK;
  });
}

care_status care_residual_factor(care_ctx* cx, const care_csr* A, const double* B, int32_t m, const double* C,
                                 int32_t p, const double* Z, int64_t ldz, int32_t r, double eta_r_rel, double* Cp,
                                 int32_t* rp, double* Cm, int32_t* rm, int64_t ldc, int32_t cap, double* res_fro) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const int64_t n = A->n, ld = pad_ld(n);
    if (m < 0 || p < 0 || r < 0) fail(CARE_ERR_ARG, "m, p, r must be >= 0");
    if ((m > 0 && !B) || (p > 0 && !C) || (r > 0 && (!Z || ldz < n))) fail(CARE_ERR_ARG, "invalid B / C / Z");
    if (!rp || !rm || !res_fro || cap < 0 || ldc < n || (cap > 0 && (!Cp || !Cm)))
      fail(CARE_ERR_ARG, "invalid outputs");
    if (!(eta_r_rel >= 0)) fail(CARE_ERR_ARG, "eta_r_rel must be >= 0");
    SellOp op;
    build_sell(ctx, A, Prec::F64, op);
    DBuf<double> B64(ctx, (size_t)ld * std::max(m, 1)), Ct(ctx, (size_t)ld * std::max(p, 1));
    if (m > 0) copy_cols<double, double>(ctx, n, m, B, n, B64.get(), ld);
    if (p > 0) copy_cols<double, double>(ctx, n, p, C, n, Ct.get(), ld);
    ResidualFactor rf;
    residual_factor(ctx, op, B64.get(), m, Ct.get(), p, Z, ldz, r, eta_r_rel, rf);
    *rp = rf.rp;
    *rm = rf.rm;
    *res_fro = rf.res_fro;
    if (rf.rp > cap || rf.rm > cap)
      fail(CARE_ERR_CAPACITY, "residual factors need " + std::to_string(std::max(rf.rp, rf.rm)) + " columns");
    if (rf.rp) copy_cols<double, double>(ctx, n, rf.rp, rf.Cp.get(), ld, Cp, ldc);
    if (rf.rm) copy_cols<double, double>(ctx, n, rf.rm, rf.Cm.get(), ld, Cm, ldc);
    ctx->sync();
    return CARE_OK;
  });
}

care_status lowrank_truncate(care_ctx* cx, int64_t n, const double* G, int64_t ldg, int32_t s, const int8_t* sign,
                             double eta_s_rel, double* Z, int64_t ldz, int32_t cap, int32_t* r_out, double* eta_n) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (s < 0 || !r_out || cap < 0) fail(CARE_ERR_ARG, "invalid sizes");
    if (s > 0 && (!G || !sign)) fail(CARE_ERR_ARG, "G or sign is NULL");
    if (!(eta_s_rel >= 0)) fail(CARE_ERR_ARG, "eta_s_rel must be >= 0");
    if (n < 1 || ldg < n || ldz < n) fail(CARE_ERR_ARG, "need n >= 1, ldg >= n, ldz >= n");
    std::vector<double> sg(s);
    for (int i = 0; i < s; ++i) {
      if (sign[i] != 1 && sign[i] != -1) fail(CARE_ERR_ARG, "sign entries must be +1 or -1");
      sg[i] = sign[i];
    }
    TruncResult tr;
    signed_truncate(ctx, n, G, ldg, s, sg, eta_s_rel, tr);
    *r_out = tr.r;
    if (eta_n) *eta_n = tr.eta_n;
    if (tr.r > cap) fail(CARE_ERR_CAPACITY, "Z needs " + std::to_string(tr.r) + " columns");
    if (tr.r) copy_cols<double, double>(ctx, n, tr.r, tr.Z.get(), pad_ld(n), Z, ldz);
    ctx->sync();
    return CARE_OK;
  });
}

care_status care_solve(care_ctx* cx, const care_csr* A, const double* B, int32_t m, const double* C, int32_t p,
                       double tol, const care_shift* shifts, int32_t nshifts, const care_opts* opts, double* Z,
                       int64_t ldz, int32_t rmax, int32_t* r_out, care_stats* stats) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    care_stats local;
    care_status warn = CARE_OK;
    care_solve_impl(ctx, sparse_spec(A), B, m, C, p, tol, shifts, nshifts, opts, Z, ldz, rmax, r_out,
                    stats ? stats : &local,
                    &warn);
    release_cache(ctx);
    return warn;
  });
}

care_status care_solve_dense(care_ctx* cx, const double* A, int64_t n, int64_t lda, const double* B, int32_t m,
                             const double* C, int32_t p, double tol, const care_shift* shifts, int32_t nshifts,
                             const care_opts* opts, double* Z, int64_t ldz, int32_t rmax, int32_t* r_out,
                             care_stats* stats) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (!A || n < 1 || lda < n) fail(CARE_ERR_ARG, "invalid dense A");
    care_stats local;
    care_status warn = CARE_OK;
    care_solve_impl(ctx, dense_spec(A, n, lda), B, m, C, p, tol, shifts, nshifts, opts, Z, ldz, rmax, r_out,
                    stats ? stats : &local, &warn);
    release_cache(ctx);
    return warn;
  });
}

care_status care_penzl_shifts(care_ctx* cx, const care_csr* A, int32_t l0, int32_t kp, int32_t km,
                              int32_t real_only, care_shift* out, int32_t* count) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    if (!out || !count || l0 < 1 || kp < 1 || km < 0) fail(CARE_ERR_ARG, "invalid Penzl arguments");
    SellOp op;
    build_sell(ctx, A, Prec::F64, op);
    ctx->krylov_rb = 1;
    rb_attach(ctx, rb_analyse(ctx, A), Prec::F64, op);
    std::vector<Shift> s = penzl_shifts(ctx, op, l0, kp, km, real_only != 0);
    *count = (int)s.size();
    for (size_t i = 0; i < s.size(); ++i) out[i] = care_shift{s[i].re, s[i].im};
    return CARE_OK;
  });
}

care_status care_projection_shifts(care_ctx* cx, const care_csr* A, const double* B, const double* K, int32_t m,
                                   const double* V, int64_t ldv, int32_t s, int32_t l0, int32_t prec,
                                   care_shift* out, int32_t* count) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    check_csr_shape(A);
    const int64_t n = A->n, ld = pad_ld(n);
    if (!out || !count || l0 < 1 || s < 1 || m < 0) fail(CARE_ERR_ARG, "invalid projection-shift arguments");
    if (!V || ldv < n) fail(CARE_ERR_ARG, "invalid V");
    const bool smw = K != nullptr && m > 0;
    if (smw && !B) fail(CARE_ERR_ARG, "B is NULL while K is given");
    const Prec pr = prec_from_abi(prec);
    SellOp op;
    build_sell(ctx, A, pr, op);
    std::vector<Shift> sh;
    auto run = [&](auto tag) {
      using T = decltype(tag);
      DBuf<T> Vs(ctx, (size_t)ld * s), Bs(ctx, (size_t)ld * std::max(m, 1)), Ks(ctx, (size_t)ld * std::max(m, 1));
      copy_cols<double, T>(ctx, n, s, V, ldv, Vs.get(), ld);
      if (smw) {
        copy_cols<double, T>(ctx, n, m, B, n, Bs.get(), ld);
        copy_cols<double, T>(ctx, n, m, K, n, Ks.get(), ld);
      }
      sh = projection_shifts<T>(ctx, op, Bs.get(), smw ? Ks.get() : nullptr, smw ? m : 0, Vs.get(), ld, s, l0);
    };
    if (pr == Prec::F64) run(double{});
    else run(float{});
    *count = (int)sh.size();
    for (size_t i = 0; i < sh.size(); ++i) out[i] = care_shift{sh[i].re, sh[i].im};
    return CARE_OK;
  });
}

care_status care_solve_batch(care_ctx* cx, int32_t count, const care_instance* instances, double tol,
                             const care_opts* opts, int32_t workers, care_instance_result* results) {
  return guarded([&]() -> care_status {
    Ctx* ctx = unwrap(cx);
    if (!(tol > 0)) fail(CARE_ERR_ARG, "tol must be positive");
    solve_batch(ctx, count, instances, tol, opts, workers, results);
    for (int k = 0; k < count; ++k)
      if (results[k].status < 0)
        fail((care_status)results[k].status, "instance " + std::to_string(k) + ": " + results[k].message);
    return CARE_OK;
  });
}

care_status care_ilu0_colouring(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col_idx,
                                int32_t* colours, int32_t* ncolours) {
  return guarded([&]() -> care_status {
    if (!colours || !ncolours) fail(CARE_ERR_ARG, "output pointer is NULL");
    std::vector<int> col;
    const int nc = ilu_colour_host(n, nnz, row_ptr, col_idx, col);
    for (int64_t i = 0; i < n; ++i) colours[i] = col[i];
    *ncolours = nc;
    return CARE_OK;
  });
}

care_status care_ritz_values(const double* H, int32_t k, int64_t ldh, double* re, double* im) {
  return guarded([&]() -> care_status {
    if (k < 0 || (k > 0 && (!H || ldh < k || !re || !im))) fail(CARE_ERR_ARG, "invalid Hessenberg arguments");
    std::vector<std::complex<double>> ev = hessenberg_eigvals(H, k, ldh);
    for (int i = 0; i < k; ++i) {
      re[i] = ev[i].real();
      im[i] = ev[i].imag();
    }
    return CARE_OK;
  });
}

care_status care_penzl_select(const double* re, const double* im, int32_t nr, int32_t l0, care_shift* out,
                              int32_t* count) {
  return guarded([&]() -> care_status {
    if (nr < 1 || l0 < 1 || !re || !out || !count) fail(CARE_ERR_ARG, "invalid selection arguments");
    std::vector<std::complex<double>> R(nr);
    for (int i = 0; i < nr; ++i) R[i] = std::complex<double>(re[i], im ? im[i] : 0.0);
    std::vector<Shift> s = penzl_select(R, l0);
    *count = (int)s.size();
    for (size_t i = 0; i < s.size(); ++i) out[i] = care_shift{s[i].re, s[i].im};
    return CARE_OK;
  });
}

}  // extern "C"
