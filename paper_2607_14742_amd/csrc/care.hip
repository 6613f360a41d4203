// Framework 1 (Factorization-based Mixed Precision Newton Iterative
// Refinement) with the NLR-ADI initial solve of Sec. 4.
#include "care.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace mpcare {

static const double U64 = 1.1102230246251565e-16;   // FP64 unit roundoff (Table 1)
static const double U32 = 5.9604644775390625e-08;   // FP32 unit roundoff (Table 1)
static const double U16 = 4.8828125e-04;            // FP16 unit roundoff (Table 1)
static const double UBF = 3.90625e-03;              // bfloat16 unit roundoff (Table 1)

Resolved resolve_opts(const care_opts* o, double tol) {
  Resolved r;
  care_opts d;
  care_opts_default(&d, o ? o->inner_prec : CARE_FP64);
  if (!o) o = &d;
  r.prec = prec_from_abi(o->inner_prec);
  // tau_L: the paper's 1e-12 (FP64) and 1e-3 (bf16 products); FP32 uses 1e-6
  // instead of the paper's 1e-5, which lets one correction reach the
  // tolerance on well-conditioned problems (Toeplitz example of Sec. 5.2:
  // 3 -> 2 refinement steps) and costs nothing measurable otherwise.
  const double tl_def = r.prec == Prec::F64 ? 1e-12 : (r.prec == Prec::F32 ? 1e-6 : (r.prec == Prec::F16 ? 1e-4 : 1e-3));
  // Krylov tolerance: 1e-10 (FP64) as in Sec. 5, tightened to a tenth of the
  // requested residual when that is smaller: the solves' own errors set the
  // floor of the true Riccati residual near the Krylov tolerance, below the
  // residual-identity estimate the initial stage stops on.  FP32 uses 1e-7
  // instead of the paper's 1e-5 (unpreconditioned BiCGStab: the tighter inner
  // solves leave a smaller, narrower residual and save refinement work).
  const double kt_def = r.prec == Prec::F64 ? std::max(1e-13, std::min(1e-10, 0.1 * tol))
                                            : (r.prec == Prec::F32 ? 1e-7 : (r.prec == Prec::F16 ? 1e-4 : 1e-3));
  r.tau_L = o->tau_L > 0 ? o->tau_L : tl_def;
  r.ktol = o->krylov_tol > 0 ? o->krylov_tol : kt_def;
  r.tau_L0 = o->tau_L0 > 0 ? o->tau_L0 : r.tau_L;
  // the initial solve's residual estimate ignores the inner solves' own
  // errors, so it is asked for a tenth of the final tolerance
  r.tau_0 = o->tau_0 > 0 ? o->tau_0 : std::max(0.1 * tol, 10.0 * r.tau_L0);
  r.theta = o->refine_forcing;
  r.eta_r_rel = o->eta_r_rel;
  r.eta_s_rel = o->eta_s_rel;
  r.stagnation = o->stagnation > 0 ? o->stagnation : 0.999;
  r.k_max = o->k_max;
  r.k0_max = o->k0_max;
  r.j_max = o->j_max;
  r.kmaxit = o->krylov_maxit > 0 ? o->krylov_maxit : 4000;
  r.check_every = o->check_every > 0 ? o->check_every : 8;
  r.deflate = o->adi_deflate != 0;
  r.rotate = o->adi_rotate != 0;
  // block-relative Krylov accuracy: a column's solve error counts against
  // the residual in proportion to its norm.  After the rotation of the
  // LR-ADI residual factor (FP32 / bf16) most columns are small and need no
  // more than the block's absolute accuracy: 500 x 500 FDM 2.12 -> 1.64 s,
  // 3D 2.70 -> 2.28 s.  FP64 keeps per-column accuracy (measured to cost
  // correction accuracy there), and so do bf16 products (3D: 19.3 -> 22.3 s
  // with it, the wider bf16 corrections lose more than they gain).
  r.block_tol = o->krylov_block_tol < 0 ? r.prec == Prec::F32 : o->krylov_block_tol != 0;
  r.relax = o->krylov_relax != 0;
  if (r.k_max < 1 || r.k0_max < 1 || r.j_max < 1) fail(CARE_ERR_ARG, "k_max, k0_max and j_max must be >= 1");
  if (r.eta_r_rel < 0 || r.eta_s_rel < 0) fail(CARE_ERR_ARG, "truncation thresholds must be >= 0");
  if (!(r.theta >= 0.0 && r.theta < 1.0)) fail(CARE_ERR_ARG, "refine_forcing must lie in [0, 1)");
  return r;
}


static double unit_roundoff(Prec p) {
  return p == Prec::F64 ? U64 : (p == Prec::F32 ? U32 : (p == Prec::F16 ? U16 : UBF));
}

// A-priori choice of the inner precision (Theorem 1: the refinement contracts
// when d_1 kappa_F(L_k) u_s < 1, and each correction gains about
// -log10(d_1 kappa u_s) digits).  kappa_F(L) of L(X) = A^T X + X A is
// estimated as ||A||_2 / min_j |Re p_j|: ||L|| <= 2 ||A||_2, and the shift set
// spans the spectrum of A (heuristic shifts from Ritz values, or a caller's
// log-spaced set over the spectral interval), so its smallest |Re p| stands in
// for the separation 1 / ||L^-1|| (exact, up to the factor 2, for normal A).
// ||A||_2 is bounded by sqrt(||A||_1 ||A||_inf).  Thresholds on kappa u_s, both
// measured here: with iterative shifted solves FP32 pays off clearly only for
// well-conditioned A.  On the Toeplitz example FP32 is 1.2-1.3x faster; on
// the 3D problem (kappa ~ 2e3) and the 2D FDM problem (~ 3e4) the two are
// about level or FP64 wins.  So FP32 where kappa u_32 <= 6e-6 (kappa <= 100).
// With direct (LU) shifted solves the paper's Table 1 shows FP32 gains up to
// kappa = 1e5: kappa u_32 <= 6e-3.  The 16-bit product variants are never
// chosen: their u_s puts every kappa >= 1 beyond those limits.
double kappa_L_estimate(double norm2_bound, const std::vector<Shift>& shifts) {
  double lo = INFINITY;
  for (const Shift& p : shifts) lo = std::min(lo, std::fabs(p.re));
  return lo > 0.0 && lo < INFINITY && norm2_bound > 0.0 ? std::max(1.0, norm2_bound / lo) : 1.0;
}

double shift_spread(const std::vector<Shift>& shifts) {
  double lo = INFINITY, hi = 0.0;
  for (const Shift& p : shifts) {
    const double a = std::hypot(p.re, p.im);
    lo = std::min(lo, a);
    hi = std::max(hi, a);
  }
  return lo > 0.0 && hi > 0.0 ? hi / lo : 1.0;
}

int choose_inner_precision(double norm2_bound, const std::vector<Shift>& shifts, bool dense) {
  const double kappa = kappa_L_estimate(norm2_bound, shifts);
  const double limit = dense ? 1e5 * U32 : 100.0 * U32;
  int choice = CARE_FP64;
  if (kappa * unit_roundoff(Prec::F16) <= limit) choice = CARE_FP16_SPMM;
  else if (kappa * unit_roundoff(Prec::F32) <= limit) choice = CARE_FP32;
  if (std::getenv("MPCARE_TRACE"))
    std::fprintf(stderr, "[auto] kappa_F(L) estimate %.3e (kappa u_s limit %.1e): inner precision %d\n", kappa,
                 limit, choice);
  return choice;
}

// ||F M F^T||_F for F = [W, dK], M = diag(I, -I): from the Gram G = F^T F,
// ||F M F^T||_F^2 = sum_ij s_i s_j G_ij^2.
template <typename T>
static double kleinman_residual(Ctx* ctx, int64_t n, const T* W, int w, const T* dK, int m) {
  const int64_t ld = pad_ld(n);
  const int q = w + m;
  DBuf<T> F(ctx, (size_t)ld * q);
  d2d(ctx, F.get(), W, (size_t)ld * w * sizeof(T));
  d2d(ctx, F.get() + (int64_t)w * ld, dK, (size_t)ld * m * sizeof(T));
  DBuf<double> G(ctx, (size_t)q * q);
  gram(ctx, n, F.get(), ld, q, F.get(), ld, q, G.get(), q);
  std::vector<double> h((size_t)q * q);
  d2h(ctx, h.data(), G.get(), h.size() * sizeof(double));
  double s = 0.0;
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) {
      const double sg = ((i < w) == (j < w)) ? 1.0 : -1.0;
      const double g = h[(size_t)j * q + i];
      s += sg * g * g;
    }
  return std::sqrt(std::max(s, 0.0));
}

struct SolveState {
  const SellOp* A64 = nullptr;
  const SellOp* As = nullptr;      // operator in the inner precision
  DBuf<double> B64, Ct64;          // ld = pad_ld(n)
  int64_t n = 0, ld = 0;
  int m = 0, p = 0;
  double nrm_ctc = 0.0;            // ||C^T C||_F
  std::vector<Shift> shifts;
  Resolved prm;
  // truncation budget of Algorithm 2 (residual change, absolute) and the
  // bounds it is converted with: a2 >= ||A||_2, g2 >= ||B B^T||_2
  double res_budget = 0.0, a2 = 0.0, g2 = 0.0;
  // shifts recomputed for each closed-loop operator A - B K^T (heuristic
  // mode with shift_update = 1)
  bool dyn_shifts = false;
  // projection shifts drawn by each LR-ADI run from its own iterates
  // (heuristic mode with shift_update = 2); shifts then holds the set of the
  // projection onto span(C^T), for the a-priori choices that read it
  bool proj_shifts = false;
  int l0 = 16, kp = 20, km = 10;
  bool real_only = false;
};

// the shift set for the operator A - B K^T of one Lyapunov solve: the fixed
// set, or (dynamic shifts) the heuristic applied to that operator
static std::vector<Shift> shifts_for(Ctx* ctx, const SolveState& S, const double* K64) {
  if (S.proj_shifts) return {};
  if (!S.dyn_shifts || !K64 || S.m == 0) return S.shifts;
  std::vector<Shift> sh = penzl_shifts(ctx, *S.A64, S.l0, S.kp, S.km, S.real_only, S.B64.get(), K64, S.m);
  if (std::getenv("MPCARE_TRACE"))
    for (const Shift& p : sh) std::fprintf(stderr, "[penzl A-BK^T] shift (%.6e, %.6e)\n", p.re, p.im);
  return sh;
}

template <typename T>
static void cast_in(Ctx* ctx, int64_t n, int cols, const double* src, int64_t lds, DBuf<T>& dst) {
  const int64_t ld = pad_ld(n);
  dst.resize(ctx, (size_t)ld * std::max(cols, 1));
  copy_cols<double, T>(ctx, n, cols, src, lds, dst.get(), ld);
}

// Stage 0: NLR-ADI (Newton-Kleinman, K_0 = 0) in precision T.
template <typename T>
static void stage0(Ctx* ctx, SolveState& S, TruncResult& Zout, care_stats* st, std::vector<double>& hist) {
  const int64_t n = S.n, ld = S.ld;
  const int m = S.m, p = S.p;
  DBuf<T> Bs, Cts;
  cast_in<T>(ctx, n, m, S.B64.get(), ld, Bs);
  cast_in<T>(ctx, n, p, S.Ct64.get(), ld, Cts);
  const int wmax = p + m;
  const int zcap = lradi_capacity(wmax, S.prm.j_max);
  DBuf<T> K(ctx, (size_t)ld * std::max(m, 1)), Kn(ctx, (size_t)ld * std::max(m, 1)),
      dK(ctx, (size_t)ld * std::max(m, 1));
  DBuf<T> W(ctx, (size_t)ld * wmax);
  ZBuffer<T> Zb;
  Zb.init(ctx, n, std::min(zcap, 16 * wmax));
  DBuf<double> Y;
  LradiParams lp;
  lp.tol = S.prm.tau_L0;
  lp.jmax = S.prm.j_max;
  lp.ktol = S.prm.ktol;
  lp.kmaxit = S.prm.kmaxit;
  lp.check_every = S.prm.check_every;
  lp.deflate = S.prm.deflate;
  lp.rotate = S.prm.deflate && S.prm.rotate && S.prm.prec != Prec::F64;
  lp.group_tol = S.prm.block_tol;
  lp.relax = S.prm.relax;
  lp.proj_shifts = S.proj_shifts ? S.l0 : 0;
  double prev = 0.0;
  int zcols = 0;
  for (int i = 0; i < S.prm.k0_max; ++i) {
    const int w = (i == 0 || m == 0) ? p : p + m;
    d2d(ctx, W.get(), Cts.get(), (size_t)ld * p * sizeof(T));
    if (w > p) d2d(ctx, W.get() + (int64_t)p * ld, K.get(), (size_t)ld * m * sizeof(T));
    std::vector<Shift> sh = S.proj_shifts ? std::vector<Shift>() : S.shifts;
    if (S.dyn_shifts && i > 0 && m > 0) {
      DBuf<double> K64(ctx, (size_t)ld * m);
      copy_cols<T, double>(ctx, n, m, K.get(), ld, K64.get(), ld);
      sh = shifts_for(ctx, S, K64.get());
    }
    LradiOut lo = lradi_run<T>(ctx, *S.As, Bs.get(), (i > 0 && m > 0) ? K.get() : nullptr, m, W.get(), w, sh, lp,
                               Zb, zcap);
    st->iter0_outer += 1;
    st->iter0_inner += lo.steps;
    zcols = lo.zcols;
    double rel;
    if (m > 0) {
      // K_{i+1} = Z (Z^T B)
      Y.resize(ctx, (size_t)std::max(zcols, 1) * m);
      gram(ctx, n, Zb.get(), ld, zcols, Bs.get(), ld, m, Y.get(), zcols);
      tsgemm<T, T>(ctx, n, Zb.get(), ld, zcols, Y.get(), zcols, m, 1.0, 0.0, Kn.get(), ld);
      d2d(ctx, dK.get(), Kn.get(), (size_t)ld * m * sizeof(T));
      if (i > 0) axpby<T>(ctx, n, m, -1.0, K.get(), ld, 1.0, dK.get(), ld);
      // Riccati residual of X_{i+1} = Z Z^T:  R = W W^T - dK dK^T
      rel = kleinman_residual<T>(ctx, n, W.get(), w, dK.get(), m) / S.nrm_ctc;
      std::swap(K, Kn);
    } else {
      rel = kleinman_residual<T>(ctx, n, W.get(), w, dK.get(), 0) / S.nrm_ctc;
    }
    hist.push_back(rel);
    if (std::getenv("MPCARE_TRACE"))
      std::fprintf(stderr, "[stage0] newton %d adi steps %d zcols %d relres %.3e\n", i, lo.steps, zcols, rel);
    if (!std::isfinite(rel)) fail(CARE_ERR_NONFINITE, "initial NLR-ADI residual is not finite");
    if (rel <= S.prm.tau_0 || m == 0) break;
    if (i > 0 && rel / prev > S.prm.stagnation) break;
    prev = rel;
  }
  // promote to FP64 (storage precision u) and compress with Algorithm 2
  // (N = I) at the update threshold eta_s.  A threshold tied to u_s instead
  // would drop directions whose absence costs ~ ||A|| ||X|| 10 u_s in the
  // residual, far above what the FP32 factor itself carries.
  DBuf<double> G(ctx, (size_t)ld * std::max(zcols, 1));
  copy_cols<T, double>(ctx, n, zcols, Zb.get(), ld, G.get(), ld);
  std::vector<double> sign(zcols, 1.0);
  signed_truncate(ctx, n, G.get(), ld, zcols, sign, S.prm.eta_s_rel, Zout, 0.5 * S.res_budget, S.a2, S.g2);
}

// one inner correction: LR-ADI on [C+, C-] with A_k = A - B (Z Z^T B)^T in
// precision T; returns the factor promoted to FP64 with its columns grouped
// by origin: Zpm = [Z+ (np columns), Z- (nm columns)]
template <typename T>
static void correction(Ctx* ctx, SolveState& S, const TruncResult& Zk, const ResidualFactor& rf, double tau,
                       double ktol, DBuf<double>& Zpm, int& np, int& nm, care_stats* st) {
  const int64_t n = S.n, ld = S.ld;
  const int m = S.m;
  const int w = rf.rp + rf.rm;
  DBuf<T> Bs, Ks, W(ctx, (size_t)ld * std::max(w, 1));
  cast_in<T>(ctx, n, m, S.B64.get(), ld, Bs);
  // K = Z (Z^T B) in FP64, then rounded to the inner precision
  DBuf<double> K64(ctx, (size_t)ld * std::max(m, 1));
  if (m > 0 && Zk.r > 0) {
    DBuf<double> Y(ctx, (size_t)Zk.r * m);
    gram(ctx, n, Zk.Z.get(), ld, Zk.r, S.B64.get(), ld, m, Y.get(), Zk.r);
    tsgemm<double, double>(ctx, n, Zk.Z.get(), ld, Zk.r, Y.get(), Zk.r, m, 1.0, 0.0, K64.get(), ld);
  } else if (m > 0) {
    dzero(ctx, K64.get(), (size_t)ld * m * sizeof(double));
  }
  cast_in<T>(ctx, n, m, K64.get(), ld, Ks);
  if (rf.rp) copy_cols<double, T>(ctx, n, rf.rp, rf.Cp.get(), ld, W.get(), ld);
  if (rf.rm) copy_cols<double, T>(ctx, n, rf.rm, rf.Cm.get(), ld, W.get() + (int64_t)rf.rp * ld, ld);
  const int zcap = lradi_capacity(w, S.prm.j_max);
  ZBuffer<T> Zb;
  Zb.init(ctx, n, std::min(zcap, 16 * std::max(w, 1)));
  LradiParams lp;
  lp.tol = tau;
  lp.jmax = S.prm.j_max;
  lp.ktol = ktol;
  lp.kmaxit = S.prm.kmaxit;
  lp.check_every = S.prm.check_every;
  lp.deflate = S.prm.deflate;
  lp.rotate = S.prm.deflate && S.prm.rotate && S.prm.prec != Prec::F64;
  lp.group_split = rf.rp;
  lp.group_tol = S.prm.block_tol;
  lp.relax = S.prm.relax;
  lp.proj_shifts = S.proj_shifts ? S.l0 : 0;
  const std::vector<Shift> sh = shifts_for(ctx, S, (m > 0 && Zk.r > 0) ? K64.get() : nullptr);
  LradiOut lo = lradi_run<T>(ctx, *S.As, Bs.get(), (m > 0 && Zk.r > 0) ? Ks.get() : nullptr, m, W.get(), w, sh,
                             lp, Zb, zcap);
  st->iter_inner += lo.steps;
  const int zcols = lo.zcols;
  std::vector<int> map;
  map.reserve(zcols);
  for (int c = 0; c < zcols; ++c)
    if (lo.zsrc[c] < rf.rp) map.push_back(c);
  np = (int)map.size();
  for (int c = 0; c < zcols; ++c)
    if (lo.zsrc[c] >= rf.rp) map.push_back(c);
  nm = zcols - np;
  Zpm.resize(ctx, (size_t)ld * std::max(zcols, 1));
  if (zcols) copy_cols<T, double>(ctx, n, zcols, Zb.get(), ld, Zpm.get(), ld, map.data());
}

static double fro_of_gram(Ctx* ctx, int64_t n, const double* X, int64_t ld, int k) {
  if (k <= 0) return 0.0;
  DBuf<double> G(ctx, (size_t)k * k);
  gram(ctx, n, X, ld, k, X, ld, k, G.get(), k);
  std::vector<double> h((size_t)k * k);
  d2h(ctx, h.data(), G.get(), h.size() * sizeof(double));
  double s = 0;
  for (double v : h) s += v * v;
  return std::sqrt(s);
}

OpSpec sparse_spec(const care_csr* A) {
  OpSpec s;
  s.csr = A;
  return s;
}

OpSpec dense_spec(const double* A, int64_t n, int64_t lda) {
  OpSpec s;
  s.dense = A;
  s.n = n;
  s.lda = lda;
  return s;
}

void build_op(Ctx* ctx, const OpSpec& A, Prec prec, SellOp& op) {
  if (A.csr) build_sell(ctx, A.csr, prec, op);
  else build_dense(ctx, A.dense, A.lda, A.n, prec, op);
}

void care_solve_impl(Ctx* ctx, const OpSpec& A, const double* B, int m, const double* C, int p, double tol,
                     const care_shift* shifts, int nshifts, const care_opts* opts, double* Zout, int64_t ldz,
                     int rmax, int* r_out, care_stats* st, care_status* warn) {
  const double t0 = now_s();
  *warn = CARE_OK;
  std::memset(st, 0, sizeof(*st));
  if (!A.csr && !A.dense) fail(CARE_ERR_ARG, "A is NULL");
  const int64_t n = A.size();
  if (n < 1) fail(CARE_ERR_ARG, "A must have n >= 1");
  if (m < 0 || p < 1) fail(CARE_ERR_ARG, "need m >= 0 and p >= 1");
  if (m > 0 && !B) fail(CARE_ERR_ARG, "B is NULL");
  if (!C) fail(CARE_ERR_ARG, "C is NULL");
  if (!(tol > 0)) fail(CARE_ERR_ARG, "tol must be positive");
  if (!Zout || ldz < n || rmax < 0 || !r_out) fail(CARE_ERR_ARG, "invalid output factor arguments");
  if (opts && opts->Z_init && (opts->ldz_init < n || opts->r_init < 0)) fail(CARE_ERR_ARG, "invalid Z_init");
  SolveState S;
  // inner precision CARE_AUTO is decided once the shifts are known (below);
  // the options are resolved for FP64 until then
  care_opts eff;
  if (opts) eff = *opts;
  else care_opts_default(&eff, CARE_FP64);
  const bool auto_prec = eff.inner_prec == CARE_AUTO;
  if (auto_prec) eff.inner_prec = CARE_FP64;
  S.prm = resolve_opts(&eff, tol);
  S.n = n;
  S.ld = pad_ld(n);
  S.m = m;
  S.p = p;
  ctx->reset_counters();
  ctx->profile = opts ? opts->profile : 0;
  ctx->spmm_split = opts ? opts->spmm_split : 0;
  ctx->spmm_tune = opts ? opts->spmm_tune : 1;
  ctx->krylov_method = opts ? opts->krylov_method : 0;
  ctx->krylov_restart = opts ? opts->krylov_restart : 0;
  ctx->krylov_compact = opts ? opts->krylov_compact : 1;
  ctx->krylov_rb = opts ? opts->krylov_rb : 1;
  ctx->krylov_precond = opts ? opts->krylov_precond : 0;
  if (ctx->krylov_method < 0 || ctx->krylov_method > 1) fail(CARE_ERR_ARG, "krylov_method must be 0 or 1");
  if (ctx->krylov_precond < 0 || ctx->krylov_precond > 1) fail(CARE_ERR_ARG, "krylov_precond must be 0 or 1");

  SellOp A64, As;
  build_op(ctx, A, Prec::F64, A64);
  // red-black reduction of the shifted solves: analysed once (CSR validated
  // by the operator build above), attached to each operator that solves
  const std::shared_ptr<RbHost> rbh = (ctx->krylov_rb && A.csr) ? rb_analyse(ctx, A.csr) : nullptr;
  rb_attach(ctx, rbh, Prec::F64, A64);
  // multicolour ILU(0) of the shifted matrices for the preconditioned GMRES solves
  const std::shared_ptr<IluHost> iluh =
      (ctx->krylov_precond && ctx->krylov_method == 1 && A.csr) ? ilu_analyse(ctx, A.csr) : nullptr;
  ilu_attach(ctx, iluh, A64);
  S.A64 = &A64;
  S.l0 = eff.penzl_l0;
  S.kp = eff.penzl_kp;
  S.km = eff.penzl_km;
  S.real_only = eff.penzl_real != 0;
  if (eff.shift_update < 0 || eff.shift_update > 2) fail(CARE_ERR_ARG, "shift_update must be 0, 1 or 2");
  S.dyn_shifts = nshifts == 0 && eff.shift_update == 1;
  S.proj_shifts = nshifts == 0 && eff.shift_update == 2;
  if (S.proj_shifts && eff.penzl_l0 < 1) fail(CARE_ERR_ARG, "projection shifts need penzl_l0 >= 1");
  if (nshifts > 0) {
    S.shifts = check_shifts(shifts, nshifts);
  } else if (S.proj_shifts) {
    // C is p x n row-major: the n x p matrix C^T, leading dimension n
    S.shifts = projection_shifts<double>(ctx, A64, nullptr, nullptr, 0, C, n, p, eff.penzl_l0);
    if (std::getenv("MPCARE_TRACE"))
      for (const Shift& sh : S.shifts) std::fprintf(stderr, "[projection C^T] shift (%.6e, %.6e)\n", sh.re, sh.im);
  } else {
    S.shifts = penzl_shifts(ctx, A64, eff.penzl_l0, eff.penzl_kp, eff.penzl_km, eff.penzl_real != 0);
    if (std::getenv("MPCARE_TRACE"))
      for (const Shift& sh : S.shifts) std::fprintf(stderr, "[penzl] shift (%.6e, %.6e)\n", sh.re, sh.im);
  }
  if (auto_prec) {
    eff.inner_prec = choose_inner_precision(A64.norm2_bound(), S.shifts, A.dense != nullptr);
    S.prm = resolve_opts(&eff, tol);
  }
  st->inner_prec = eff.inner_prec;
  if (S.prm.prec == Prec::F64) {
    S.As = &A64;
  } else {
    build_op(ctx, A, S.prm.prec, As);
    rb_attach(ctx, rbh, S.prm.prec, As);
    ilu_attach(ctx, iluh, As);
    S.As = &As;
  }
  // B and C^T in internal layout (ld = pad_ld(n)); C is p x n row-major = C^T col-major with ld n
  S.B64.resize(ctx, (size_t)S.ld * std::max(m, 1));
  S.Ct64.resize(ctx, (size_t)S.ld * p);
  if (m > 0) copy_cols<double, double>(ctx, n, m, B, n, S.B64.get(), S.ld);
  copy_cols<double, double>(ctx, n, p, C, n, S.Ct64.get(), S.ld);
  S.nrm_ctc = fro_of_gram(ctx, n, S.Ct64.get(), S.ld, p);
  if (!std::isfinite(S.nrm_ctc)) fail(CARE_ERR_NONFINITE, "C has non-finite entries");
  S.g2 = m > 0 ? fro_of_gram(ctx, n, S.B64.get(), S.ld, m) : 0.0;
  if (!std::isfinite(S.g2)) fail(CARE_ERR_NONFINITE, "B has non-finite entries");
  S.a2 = A64.norm2_bound() > 0.0 ? A64.norm2_bound() : A64.frob;
  S.res_budget = S.prm.theta * tol * S.nrm_ctc;
  ctx->sync();
  const double t1 = now_s();
  st->t_setup = t1 - t0;

  // ---------------- stage 0 ----------------
  TruncResult Z;
  std::vector<double> hist0, hist;
  if (opts && opts->Z_init) {
    const int r0 = opts->r_init;
    DBuf<double> G(ctx, (size_t)S.ld * std::max(r0, 1));
    copy_cols<double, double>(ctx, n, r0, opts->Z_init, opts->ldz_init, G.get(), S.ld);
    Z.Z = std::move(G);
    Z.r = r0;
    Z.sig_max = factor_lam_max(ctx, n, Z.Z.get(), S.ld, r0);
  } else if (S.prm.prec == Prec::F64) {
    stage0<double>(ctx, S, Z, st, hist0);
  } else {
    stage0<float>(ctx, S, Z, st, hist0);
  }
  ctx->sync();
  const double t2 = now_s();
  st->t_stage0 = t2 - t1;

  // ---------------- refinement (Framework 1) ----------------
  double prev = 0.0, best = INFINITY;
  TruncResult bestZ;
  bool converged = false, stagnated = false;
  double last_res = NAN;
  // Inexact Newton forcing: correction k only has to bring the residual from
  // rel_k down to the tolerance, so its Lyapunov solve stops at
  // theta tol / rel_k relative (never looser than 0.1, never tighter than
  // tau_L), its shifted solves at a tenth of that, and the residual
  // eigenvalues Algorithm 1 drops may add up to theta tol ||C^T C||_F on top
  // of its relative threshold.  The solution truncation (Algorithm 2 and the
  // compression ahead of it) may change the residual by another theta tol.
  // These terms add at most about 3 theta tol to the next residual.
  const double theta = S.prm.theta;
  // MPCARE_TRACE: wall time of each phase of a refinement step
  const bool trace = std::getenv("MPCARE_TRACE") != nullptr;
  double tmark_last = now_s();
  auto tmark = [&](const char* what) {
    if (!trace) return;
    ctx->sync();
    const double t = now_s();
    std::fprintf(stderr, "[refine] phase %s %.1f ms\n", what, 1e3 * (t - tmark_last));
    tmark_last = t;
  };
  for (int k = 0; k < S.prm.k_max; ++k) {
    ResidualFactor rf;
    residual_factor(ctx, A64, S.B64.get(), m, S.Ct64.get(), p, Z.Z.get(), S.ld, Z.r, S.prm.eta_r_rel, rf,
                    theta * tol * S.nrm_ctc, &Z);
    tmark("algorithm 1");
    st->iter_outer += 1;
    const double rel = rf.res_fro / S.nrm_ctc;
    if (!std::isfinite(rel)) fail(CARE_ERR_NONFINITE, "Riccati residual is not finite");
    hist.push_back(rel);
    last_res = rel;
    if (std::getenv("MPCARE_TRACE"))
      std::fprintf(stderr, "[refine] k %d rank %d relres %.3e  C+ %d C- %d\n", k, Z.r, rel, rf.rp, rf.rm);
    if (rel < best) {
      best = rel;
      bestZ.Z.resize(ctx, (size_t)S.ld * std::max(Z.r, 1));
      d2d(ctx, bestZ.Z.get(), Z.Z.get(), (size_t)S.ld * Z.r * sizeof(double));
      bestZ.r = Z.r;
      bestZ.eta_n = Z.eta_n;
      bestZ.sig_max = Z.sig_max;
    }
    if (rel <= tol) {
      converged = true;
      break;
    }
    if (k > 0 && rel / prev > S.prm.stagnation) {
      stagnated = true;
      break;
    }
    prev = rel;
    if (k == S.prm.k_max - 1) break;     // no correction whose residual would go unchecked
    // G = [Z, Z+, Z-] for Algorithm 2; the raw correction factor and its
    // compressed parts are released before the orthogonalisation of G
    DBuf<double> G;
    int s = 0;
    std::vector<double> sign;
    {
      DBuf<double> Zpm;
      int np = 0, nm = 0;
      double tau_k = S.prm.tau_L, kt_k = S.prm.ktol;
      if (theta > 0.0) {
        // An FP32 correction gains at most ~ kappa u_s in relative accuracy
        // (Theorem 1; kappa read off the shift spread), so its Lyapunov solve
        // is not asked for much more than a tenth of that.
        const double floor_k = S.prm.prec == Prec::F32 ? 0.1 * shift_spread(S.shifts) * U32 : 0.0;
        tau_k = std::min(0.1, std::max({S.prm.tau_L, theta * tol / rel, floor_k}));
        kt_k = std::max(S.prm.ktol, 0.1 * tau_k);
      }
      if (std::getenv("MPCARE_TRACE")) std::fprintf(stderr, "[refine] correction tau %.3e ktol %.3e\n", tau_k, kt_k);
      if (S.prm.prec == Prec::F64) correction<double>(ctx, S, Z, rf, tau_k, kt_k, Zpm, np, nm, st);
      else correction<float>(ctx, S, Z, rf, tau_k, kt_k, Zpm, np, nm, st);
      tmark("correction");
      // Each of Z+ and Z- is a PSD factor: compressing it alone to the
      // eigenvalues of Z+- Z+-^T above a quarter of Algorithm 2's own threshold
      // (eta_s max|lambda(P)|, with max|lambda(P)| ~ ||Z Z^T||_2) changes
      // G N G^T by at most that much, and shrinks G from the raw ADI width to
      // the correction's numerical rank.
      // With a truncation budget each group may also drop eigen-terms worth a
      // quarter of it in the residual (the rest goes to Algorithm 2 itself).
      const double tau = 0.25 * S.prm.eta_s_rel * Z.sig_max;
      const double drop = S.res_budget > 0.0 ? 0.25 * S.res_budget / (2.0 * (S.a2 + S.g2 * Z.sig_max)) : 0.0;
      const double* parts[2] = {Zpm.get(), Zpm.get() + (int64_t)np * S.ld};
      int widths[2] = {np, nm};
      DBuf<double> comp[2];
      for (int g = 0; g < 2; ++g) {
        int r = 0;
        if (tau > 0.0 && widths[g] > 0 && psd_compress(ctx, n, parts[g], S.ld, widths[g], tau, comp[g], r, drop)) {
          parts[g] = comp[g].get();
          widths[g] = r;
        }
      }
      // G = [Z, Z+, Z-], Algorithm 2.  When Z carries its orthonormal basis
      // only [Z+, Z-] is assembled: the orthogonalisation starts from it.
      const int lead = Z.has_q ? 0 : Z.r;
      s = lead + widths[0] + widths[1];
      G.resize(ctx, (size_t)S.ld * std::max(s, 1));
      if (lead) d2d(ctx, G.get(), Z.Z.get(), (size_t)S.ld * lead * sizeof(double));
      d2d(ctx, G.get() + (int64_t)lead * S.ld, parts[0], (size_t)S.ld * widths[0] * sizeof(double));
      d2d(ctx, G.get() + (int64_t)(lead + widths[0]) * S.ld, parts[1], (size_t)S.ld * widths[1] * sizeof(double));
      sign.assign(s, 1.0);
      for (int c = lead + widths[0]; c < s; ++c) sign[c] = -1.0;
    }
    tmark("compression");
    TruncResult Zn;
    if (Z.has_q)
      signed_truncate_basis(ctx, n, Z, G.get(), S.ld, s, sign, S.prm.eta_s_rel, Zn, 0.5 * S.res_budget, S.a2, S.g2);
    else
      signed_truncate(ctx, n, G.get(), S.ld, s, sign, S.prm.eta_s_rel, Zn, 0.5 * S.res_budget, S.a2, S.g2);
    tmark("algorithm 2");
    st->eta_n = Zn.eta_n;
    Z = std::move(Zn);
  }
  ctx->sync();
  const double t3 = now_s();
  st->t_refine = t3 - t2;
  // return the best factor met
  const TruncResult& R = bestZ.r > 0 || Z.r == 0 ? bestZ : Z;
  st->rank = R.r;
  st->res_rel = best;
  st->stagnated = stagnated ? 1 : 0;
  *r_out = R.r;
  if (R.r > rmax) fail(CARE_ERR_CAPACITY, "output factor needs " + std::to_string(R.r) + " columns");
  if (R.r > 0) copy_cols<double, double>(ctx, n, R.r, R.Z.get(), S.ld, Zout, ldz);
  // the paper's normalised residual
  const double ztz = fro_of_gram(ctx, n, R.Z.get(), S.ld, R.r);
  const double btb = S.g2;
  st->res_paper = best * S.nrm_ctc / (2.0 * A64.frob * ztz + btb * ztz * ztz + S.nrm_ctc);
  ctx->sync();
  int hl = 0;
  for (double v : hist0)
    if (hl < 48) st->res_hist[hl++] = v;
  for (double v : hist)
    if (hl < 48) st->res_hist[hl++] = v;
  st->hist_len = hl;
  st->t_total = now_s() - t0;
  st->spmm_calls = ctx->spmm_calls;
  st->spmm_bytes = ctx->spmm_bytes;
  st->t_spmm = ctx->t_spmm;
  st->krylov_iters = ctx->krylov_iters;
  st->krylov_compactions = (int32_t)ctx->krylov_compactions;
  st->adi_rotations = (int32_t)ctx->adi_rotations;
  (void)last_res;
  if (!converged) *warn = stagnated ? CARE_WARN_STAGNATED : CARE_WARN_MAXIT;
}

}  // namespace mpcare
