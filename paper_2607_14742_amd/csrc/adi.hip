// LR-ADI driver and its fused update kernel.
#include "adi.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "dense.hpp"

namespace mpcare {

using cplx = std::complex<double>;

std::vector<Shift> check_shifts(const care_shift* s, int count) {
  if (count <= 0 || !s) fail(CARE_ERR_ARG, "empty shift set");
  std::vector<Shift> out;
  for (int i = 0; i < count; ++i) {
    const double re = s[i].re, im = s[i].im;
    if (!(re < 0.0) || !std::isfinite(re) || !std::isfinite(im))
      fail(CARE_ERR_ARG, "shift " + std::to_string(i) + " must have a finite negative real part");
    if (im != 0.0) {
      if (im < 0.0 || i + 1 >= count || s[i + 1].re != re || s[i + 1].im != -im)
        fail(CARE_ERR_ARG, "complex shift " + std::to_string(i) +
                               " must be followed by its conjugate (positive imaginary part first)");
      out.push_back({re, im});
      out.push_back({re, -im});
      ++i;
    } else {
      out.push_back({re, 0.0});
    }
  }
  return out;
}

// Gauss-Jordan inverse of a small complex matrix (column-major), partial pivoting
bool cinv(int m, std::vector<std::complex<double>>& A) {
  std::vector<cplx> I((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::abs(A[(size_t)c * m + r]) > std::abs(A[(size_t)c * m + piv])) piv = r;
    if (std::abs(A[(size_t)c * m + piv]) == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < m; ++j) {
        std::swap(A[(size_t)j * m + c], A[(size_t)j * m + piv]);
        std::swap(I[(size_t)j * m + c], I[(size_t)j * m + piv]);
      }
    const cplx d = A[(size_t)c * m + c];
    for (int j = 0; j < m; ++j) {
      A[(size_t)j * m + c] /= d;
      I[(size_t)j * m + c] /= d;
    }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const cplx f = A[(size_t)c * m + r];
      if (f == 0.0) continue;
      for (int j = 0; j < m; ++j) {
        A[(size_t)j * m + r] -= f * A[(size_t)j * m + c];
        I[(size_t)j * m + r] -= f * I[(size_t)j * m + c];
      }
    }
  }
  A.swap(I);
  return true;
}

// V = Vh + S Y (SMW correction, S: n x m, Y: m x w), then the ADI update.
// Real:    W -= 2 p V;  Z(:, c) = sqrt(-2p) V(:, c)
// Complex: Vh, S interleaved (re, im) column pairs, Y = Yr + i Yi;
//          Vr_hat = Re V + delta Im V;  W -= 4 Re(p) Vr_hat;
//          Z(:, c) = z1 Vr_hat,  Z(:, w + c) = z2 Im V
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) k_adi_update(int64_t n, int w, int m, int64_t ld, const T* __restrict__ Vh,
                                                    const T* __restrict__ S, const double* __restrict__ Yr,
                                                    const double* __restrict__ Yi, T* __restrict__ W,
                                                    T* __restrict__ Z, double c_w, double z1, double z2,
                                                    double delta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= w) return;
  if (!CPLX) {
    double v = (double)Vh[(int64_t)c * ld + i];
    for (int l = 0; l < m; ++l) v += (double)S[(int64_t)l * ld + i] * Yr[(int64_t)c * m + l];
    const int64_t o = (int64_t)c * ld + i;
    W[o] = (T)((double)W[o] - c_w * v);
    Z[o] = (T)(z1 * v);
  } else {
    double vr = (double)Vh[(int64_t)(2 * c) * ld + i];
    double vi = (double)Vh[(int64_t)(2 * c + 1) * ld + i];
    for (int l = 0; l < m; ++l) {
      const double sr = (double)S[(int64_t)(2 * l) * ld + i], si = (double)S[(int64_t)(2 * l + 1) * ld + i];
      const double yr = Yr[(int64_t)c * m + l], yi = Yi[(int64_t)c * m + l];
      vr += sr * yr - si * yi;
      vi += sr * yi + si * yr;
    }
    const double vhat = vr + delta * vi;
    const int64_t o = (int64_t)c * ld + i;
    W[o] = (T)((double)W[o] - c_w * vhat);
    Z[o] = (T)(z1 * vhat);
    Z[(int64_t)(w + c) * ld + i] = (T)(z2 * vi);
  }
}

// ||W^T W||_F and the squared column norms of W
// Eigenvectors of a small symmetric matrix A (k x k, column-major) by the
// cyclic Jacobi method (Golub and Van Loan, Sec. 8.5): rotations J(p, q)
// that zero a_pq are applied as A <- J^T A J and accumulated in Q <- Q J
// until the off-diagonal part is below 1e-15 of the diagonal.  Q returns
// the eigenvectors as columns (column-major); false if Q failed the
// orthogonality check.
static bool jacobi_eig(int k, std::vector<double> A, std::vector<double>& Q) {
  auto a = [&](int r, int c) -> double& { return A[(size_t)c * k + r]; };
  Q.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) Q[(size_t)i * k + i] = 1.0;
  auto q = [&](int r, int c) -> double& { return Q[(size_t)c * k + r]; };
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int c = 0; c < k; ++c)
      for (int r = 0; r < k; ++r) (r == c ? dia : off) += a(r, c) * a(r, c);
    if (off <= 1e-30 * dia) break;
    for (int p = 0; p < k - 1; ++p)
      for (int r = p + 1; r < k; ++r) {
        const double apq = a(p, r);
        if (apq == 0.0) continue;
        const double tau = (a(r, r) - a(p, p)) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        for (int i = 0; i < k; ++i) {   // columns p and r: A J
          const double x = a(i, p), y = a(i, r);
          a(i, p) = cs * x - sn * y;
          a(i, r) = sn * x + cs * y;
        }
        for (int i = 0; i < k; ++i) {   // rows p and r: J^T A
          const double x = a(p, i), y = a(r, i);
          a(p, i) = cs * x - sn * y;
          a(r, i) = sn * x + cs * y;
        }
        for (int i = 0; i < k; ++i) {   // Q J
          const double x = q(i, p), y = q(i, r);
          q(i, p) = cs * x - sn * y;
          q(i, r) = sn * x + cs * y;
        }
      }
  }
  for (int c = 0; c < k; ++c)
    for (int d = 0; d <= c; ++d) {
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += q(i, c) * q(i, d);
      if (std::fabs(s - (c == d ? 1.0 : 0.0)) > 1e-12) return false;
    }
  return true;
}

constexpr int ROTATE_MIN_ITERS = 20;

template <typename T>
static double gram_stats(Ctx* ctx, int64_t n, const T* W, int64_t ld, int w, std::vector<double>& colnorm2,
                         std::vector<double>* full = nullptr) {
  DBuf<double> G(ctx, (size_t)w * w);
  gram(ctx, n, W, ld, w, W, ld, w, G.get(), w);
  std::vector<double> local;
  std::vector<double>& h = full ? *full : local;
  h.resize((size_t)w * w);
  d2h(ctx, h.data(), G.get(), h.size() * sizeof(double));
  double s = 0;
  for (double v : h) s += v * v;
  colnorm2.resize(w);
  for (int c = 0; c < w; ++c) colnorm2[c] = h[(size_t)c * w + c];
  return std::sqrt(s);
}

struct ShiftCache {
  bool ready = false;
  DBuf<uint8_t> S;              // M^{-1} K (T, ld x m, complex: 2m interleaved)
  std::vector<cplx> Tinv;       // (I - B^T S)^{-1}, m x m
};

// One SMW shifted solve: M [Vh, S] = [W, K] (S only when not cached for this
// shift), then Y = T^{-1} (B^T Vh) returned as (yr, yi), m x w column-major.
// rhs / sol: scratch panels of ld x 2 (w + m) entries; Vh is left in sol.
template <typename T>
static KrylovResult smw_step(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, const T* W, int w, Shift p,
                             ShiftCache& sc, const LradiParams& prm, T* rhs, T* sol, std::vector<double>& yr,
                             std::vector<double>& yi) {
  const int64_t n = op.n, ld = pad_ld(n);
  const bool smw = K != nullptr && m > 0;
  const bool cp = p.im != 0.0;
  const bool need_s = smw && !sc.ready;
  const int nrhs = w + (need_s ? m : 0);
  if (!cp) {
    copy_cols<T, T>(ctx, n, w, W, ld, rhs, ld);
    if (need_s) copy_cols<T, T>(ctx, n, m, K, ld, rhs + (int64_t)w * ld, ld);
  } else {
    std::vector<int> map(2 * std::max(w, m));
    for (int c = 0; c < std::max(w, m); ++c) {
      map[2 * c] = c;
      map[2 * c + 1] = -1;
    }
    copy_cols<T, T>(ctx, n, 2 * w, W, ld, rhs, ld, map.data());
    if (need_s) copy_cols<T, T>(ctx, n, 2 * m, K, ld, rhs + (int64_t)2 * w * ld, ld, map.data());
  }
  std::vector<int> groups(nrhs, 0);
  for (int c = w; c < nrhs; ++c) groups[c] = 1;     // the K columns form their own group
  KrylovResult kr = bicgstab<T>(ctx, op, p.re, p.im, (cp ? 2 : 1) * nrhs, rhs, ld, sol, ld, prm.ktol, prm.kmaxit,
                                prm.check_every, prm.group_tol ? &groups : nullptr);
  yr.assign((size_t)std::max(m, 1) * w, 0.0);
  yi.assign((size_t)std::max(m, 1) * w, 0.0);
  if (!smw) return kr;
  if (need_s) {
    const int sc_cols = (cp ? 2 : 1) * m;
    sc.S.resize(ctx, (size_t)ld * sc_cols * sizeof(T));
    d2d(ctx, sc.S.get(), sol + (int64_t)(cp ? 2 : 1) * w * ld, (size_t)ld * sc_cols * sizeof(T));
    DBuf<double> G(ctx, (size_t)m * sc_cols);
    gram(ctx, n, B, ld, m, (const T*)sc.S.get(), ld, sc_cols, G.get(), m);
    std::vector<double> h((size_t)m * sc_cols);
    d2h(ctx, h.data(), G.get(), h.size() * sizeof(double));
    std::vector<cplx> Tm((size_t)m * m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const cplx bs = cp ? cplx(h[(size_t)(2 * j) * m + i], h[(size_t)(2 * j + 1) * m + i])
                           : cplx(h[(size_t)j * m + i], 0.0);
        Tm[(size_t)j * m + i] = (i == j ? 1.0 : 0.0) - bs;
      }
    if (!cinv(m, Tm)) fail(CARE_ERR_BREAKDOWN, "singular SMW capacitance matrix I - B^T (A^T + pI)^{-1} K");
    sc.Tinv = Tm;
    sc.ready = true;
  }
  const int vcols = (cp ? 2 : 1) * w;
  DBuf<double> Gbv(ctx, (size_t)m * vcols);
  gram(ctx, n, B, ld, m, sol, ld, vcols, Gbv.get(), m);
  std::vector<double> h((size_t)m * vcols);
  d2h(ctx, h.data(), Gbv.get(), h.size() * sizeof(double));
  for (int c = 0; c < w; ++c)
    for (int i = 0; i < m; ++i) {
      cplx acc = 0.0;
      for (int l = 0; l < m; ++l) {
        const cplx g = cp ? cplx(h[(size_t)(2 * c) * m + l], h[(size_t)(2 * c + 1) * m + l])
                          : cplx(h[(size_t)c * m + l], 0.0);
        acc += sc.Tinv[(size_t)l * m + i] * g;
      }
      yr[(size_t)c * m + i] = acc.real();
      yi[(size_t)c * m + i] = acc.imag();
    }
  return kr;
}

template <typename T>
LradiOut lradi_run(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, T* W, int w,
                   const std::vector<Shift>& shifts, const LradiParams& prm, ZBuffer<T>& Z, int zmax) {
  LradiOut out;
  const int64_t n = op.n;
  const int64_t ld = pad_ld(n);
  if (w <= 0) return out;
  const bool proj = prm.proj_shifts > 0;
  if (shifts.empty() && !proj) fail(CARE_ERR_ARG, "empty shift set");
  const bool smw = K != nullptr && m > 0;
  std::vector<double> cn;
  out.res0 = gram_stats(ctx, n, W, ld, w, cn);
  if (!std::isfinite(out.res0)) fail(CARE_ERR_NONFINITE, "non-finite right-hand side factor");
  if (out.res0 == 0.0) return out;
  // Projection shifts: the first set from span(W0) unless the caller gave
  // one; each time a set is used up, the next from the span of the most
  // recent blocks of Z (those of the last steps, until they hold l0
  // columns).  A projection without a stable Ritz value keeps the set.
  std::vector<Shift> cur = shifts;
  if (cur.empty()) cur = projection_shifts<T>(ctx, op, B, smw ? K : nullptr, m, W, ld, w, prm.proj_shifts);
  // a dense operator factors A^T + p I for the whole set in one launch
  auto prefactor = [&]() {
    if (!op.dense) return;
    std::vector<double> re;
    for (const Shift& q : cur)
      if (q.im == 0.0) re.push_back(q.re);
    dense_prefactor(ctx, op, re);
  };
  prefactor();
  std::vector<int> step_col;   // first column of Z written by each step

  const int maxcols = smw ? w + m : w;
  DBuf<T> rhs(ctx, (size_t)ld * 2 * maxcols), sol(ctx, (size_t)ld * 2 * maxcols), tmp(ctx, (size_t)ld);
  std::vector<ShiftCache> cache(cur.size());
  DBuf<double> dYr(ctx, (size_t)std::max(m, 1) * w), dYi(ctx, (size_t)std::max(m, 1) * w);
  std::vector<double> yr, yi;
  const bool trace = std::getenv("MPCARE_TRACE") != nullptr;
  // Column deflation: ADI acts on each column of W independently.  The
  // columns kept at the front (physical 0 .. wa-1) are iterated; the others
  // are frozen as they are.  Since W W^T = W_a W_a^T + W_f W_f^T, a frozen set
  // F with ||W_F^T W_F||_F under a quarter of the stopping level
  // tau_L ||W0^T W0||_F can never keep the stopping test (which always
  // covers every column) from being met.  Columns join F smallest first
  // while that Frobenius norm, computed from the Gram of W, allows.
  std::vector<int> perm(w);
  for (int c = 0; c < w; ++c) perm[c] = c;
  int wa = w;
  double frozen2 = 0.0;   // ||W_F^T W_F||_F^2 of the frozen columns
  const double budget = prm.deflate ? 0.25 * prm.tol * out.res0 : 0.0;
  std::vector<double> gfull;

  size_t idx = 0;
  LradiParams sp = prm;   // per-step copy (Krylov tolerance)
  double rot_ref = 1.0;   // residual level of the last rotation of W
  while (out.steps < prm.jmax && wa > 0) {
    if (proj && idx >= cur.size() && out.zcols > 0) {
      int c0 = out.zcols;
      for (int t = (int)step_col.size() - 1; t >= 0; --t) {
        c0 = step_col[t];
        if (out.zcols - c0 >= prm.proj_shifts) break;
      }
      try {
        std::vector<Shift> next =
            projection_shifts<T>(ctx, op, B, smw ? K : nullptr, m, Z.get() + (int64_t)c0 * ld, ld, out.zcols - c0,
                                 prm.proj_shifts);
        cur = std::move(next);
        std::vector<ShiftCache> fresh(cur.size());
        cache.swap(fresh);
        prefactor();
      } catch (const CareError& e) {
        if (e.status != CARE_ERR_UNSTABLE) throw;
      }
      idx = 0;
      if (trace)
        for (const Shift& q : cur) std::fprintf(stderr, "[lradi] projection shift (%.6e, %.6e)\n", q.re, q.im);
    }
    const Shift p = cur[idx % cur.size()];
    ShiftCache& sc = cache[idx % cur.size()];
    // Inexact ADI (relaxation of the inner solves): an inner solve of
    // relative accuracy eps on W_{j-1} perturbs the Lyapunov residual by about
    // eps ||W_{j-1}||^2 = eps res_rel ||W0||^2, so once the residual has
    // dropped, looser solves keep that perturbation at the level of the first
    // step's: tol_j = ktol / (4 res_rel), between ktol and sqrt(ktol).  The
    // solves that also produce the cached SMW block M^{-1} K stay at ktol.
    sp.ktol = prm.ktol;
    if (prm.relax && out.steps > 0 && (sc.ready || !smw))
      sp.ktol = std::min(std::sqrt(prm.ktol), std::max(prm.ktol, prm.ktol / (4.0 * std::max(out.res_rel, 1e-300))));
    const bool cp = p.im != 0.0;
    const int width = (cp ? 2 : 1) * wa;
    if (out.zcols + width > zmax) fail(CARE_ERR_CAPACITY, "LR-ADI factor buffer too small");
    Z.reserve(ctx, out.zcols, out.zcols + width);
    KrylovResult kr = smw_step<T>(ctx, op, B, K, m, W, wa, p, sc, sp, rhs.get(), sol.get(), yr, yi);
    out.krylov_unconverged += kr.unconverged;
    out.krylov_max_iters = std::max(out.krylov_max_iters, kr.max_iters);
    if (smw) {
      h2d(ctx, dYr.get(), yr.data(), (size_t)m * wa * sizeof(double));
      if (cp) h2d(ctx, dYi.get(), yi.data(), (size_t)m * wa * sizeof(double));
    }
    T* Zb = Z.get() + (int64_t)out.zcols * ld;
    step_col.push_back(out.zcols);
    dim3 g(ceil_div(n, 256), wa);
    const T* Sp = smw ? (const T*)sc.S.get() : nullptr;
    if (!cp) {
      const double z1 = std::sqrt(-2.0 * p.re);
      hipLaunchKernelGGL((k_adi_update<T, false>), g, dim3(256), 0, ctx->stream, n, wa, smw ? m : 0, ld,
                         (const T*)sol.get(), Sp, dYr.get(), dYi.get(), W, Zb, 2.0 * p.re, z1, 0.0, 0.0);
      out.steps += 1;
      idx += 1;
    } else {
      const double delta = p.re / p.im;
      const double gam = std::sqrt(-2.0 * p.re);
      const double z1 = std::sqrt(2.0) * gam, z2 = std::sqrt(2.0) * gam * std::sqrt(delta * delta + 1.0);
      hipLaunchKernelGGL((k_adi_update<T, true>), g, dim3(256), 0, ctx->stream, n, wa, smw ? m : 0, ld,
                         (const T*)sol.get(), Sp, dYr.get(), dYi.get(), W, Zb, 4.0 * p.re, z1, z2, delta);
      out.steps += 2;
      idx += 2;
    }
    KERNEL_CHECK();
    out.zcols += width;
    for (int rep = 0; rep < (cp ? 2 : 1); ++rep)
      for (int c = 0; c < wa; ++c) out.zsrc.push_back(perm[c]);
    const double res = gram_stats(ctx, n, W, ld, w, cn, budget > 0.0 ? &gfull : nullptr);
    if (!std::isfinite(res)) fail(CARE_ERR_NONFINITE, "LR-ADI residual became non-finite");
    out.res_rel = res / out.res0;
    if (trace)
      std::fprintf(stderr,
                   "[lradi] step %d p (%.4e, %.4e) w %d smw %d krylov it %d unconv %d restarts %d relres %.2e "
                   "adi res %.3e\n",
                   out.steps, p.re, p.im, wa, smw ? 1 : 0, kr.max_iters, kr.unconverged, kr.restarts,
                   kr.worst_relres, out.res_rel);
    if (out.res_rel > 1e8) fail(CARE_ERR_UNSTABLE, "LR-ADI diverged (is A - B K^T stable?)");
    if (out.res_rel <= prm.tol) break;
    if (budget > 0.0 && prm.rotate && wa > 1 && out.res_rel <= 0.5 * rot_ref && kr.max_iters >= ROTATE_MIN_ITERS) {
      // Rotation of W: any W Q with Q orthogonal is a residual factor of the
      // same residual (W Q Q^T W^T = W W^T), so the next step may start from
      // it.  Each time the ADI residual has halved, the active columns of
      // each group (the factors of C+ and C- in a correction are not mixed)
      // are turned to the eigenvectors of their Gram.  The residual's energy
      // then sits in few columns that hold the slowly converging smooth
      // modes; the other columns converge in few Krylov iterations even at
      // the small shifts (and leave the block solve early, which the
      // compaction turns into fewer panels), and the freezing below can
      // take them once they are small enough.  Where the shifted solves
      // converge in a few iterations anyway (well-conditioned shifted
      // matrices) there is nothing to gain, so the rotation waits for a step
      // whose solves took ROTATE_MIN_ITERS iterations or more.
      rot_ref = out.res_rel;
      bool rotated = false;
      for (int g = 0; g < 2; ++g) {
        std::vector<int> I;
        for (int c = 0; c < wa; ++c)
          if ((prm.group_split > 0 && perm[c] >= prm.group_split ? 1 : 0) == g) I.push_back(c);
        const int k = (int)I.size();
        if (k < 2) continue;
        std::vector<double> Gg((size_t)k * k);
        for (int j = 0; j < k; ++j)
          for (int i = 0; i < k; ++i) Gg[(size_t)j * k + i] = gfull[(size_t)I[j] * w + I[i]];
        DBuf<double> dG(ctx, (size_t)k * k);
        if (k <= 32) {
          // small groups: cyclic Jacobi on the host (no device round trip)
          std::vector<double> Q;
          if (!jacobi_eig(k, Gg, Q)) continue;
          h2d(ctx, dG.get(), Q.data(), Q.size() * sizeof(double));
        } else {
          h2d(ctx, dG.get(), Gg.data(), Gg.size() * sizeof(double));
          std::vector<double> ev;
          dsyevd(ctx, k, dG.get(), k, ev);
        }
        DBuf<T> Wg(ctx, (size_t)ld * k), Wr(ctx, (size_t)ld * k);
        copy_cols<T, T>(ctx, n, k, W, ld, Wg.get(), ld, I.data());
        tsgemm<T, T>(ctx, n, Wg.get(), ld, k, dG.get(), k, k, 1.0, 0.0, Wr.get(), ld);
        for (int j = 0; j < k; ++j) d2d(ctx, W + (int64_t)I[j] * ld, Wr.get() + (int64_t)j * ld, (size_t)n * sizeof(T));
        rotated = true;
        ctx->adi_rotations += 1;
      }
      if (rotated) gram_stats(ctx, n, W, ld, w, cn, &gfull);
    }
    if (budget > 0.0) {
      // freeze the smallest active columns while the frozen budget allows
      std::vector<int> order(wa);
      for (int c = 0; c < wa; ++c) order[c] = c;
      std::sort(order.begin(), order.end(), [&](int a, int b) { return cn[a] < cn[b]; });
      std::vector<char> freeze(wa, 0);
      std::vector<int> fset;     // physical columns of F: the frozen tail and the new ones
      for (int c = wa; c < w; ++c) fset.push_back(c);
      const double b2 = budget * budget;
      for (int c : order) {
        double add = gfull[(size_t)c * w + c] * gfull[(size_t)c * w + c];
        for (int f : fset) add += 2.0 * gfull[(size_t)c * w + f] * gfull[(size_t)c * w + f];
        if (frozen2 + add > b2) break;
        frozen2 += add;
        fset.push_back(c);
        freeze[c] = 1;
      }
      // compact: move frozen columns behind the active ones
      int lo = 0, hi = wa - 1;
      while (true) {
        while (lo <= hi && !freeze[lo]) ++lo;
        while (hi >= lo && freeze[hi]) --hi;
        if (lo >= hi) break;
        d2d(ctx, tmp.get(), W + (int64_t)lo * ld, n * sizeof(T));
        d2d(ctx, W + (int64_t)lo * ld, W + (int64_t)hi * ld, n * sizeof(T));
        d2d(ctx, W + (int64_t)hi * ld, tmp.get(), n * sizeof(T));
        std::swap(perm[lo], perm[hi]);
        std::swap(freeze[lo], freeze[hi]);
        ++lo;
        --hi;
      }
      int na = 0;
      for (int c = 0; c < wa; ++c) na += freeze[c] ? 0 : 1;
      wa = na;   // the cached S = M^{-1} K and T^{-1} do not depend on W
    }
  }
  out.w_final = wa;
  return out;
}

template <typename T>
KrylovResult shifted_solve(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, const T* W, int w, Shift p,
                           const LradiParams& prm, T* V) {
  const int64_t n = op.n, ld = pad_ld(n);
  const bool cp = p.im != 0.0;
  const int maxcols = w + m;
  DBuf<T> rhs(ctx, (size_t)ld * 2 * maxcols), sol(ctx, (size_t)ld * 2 * maxcols);
  ShiftCache sc;
  std::vector<double> yr, yi;
  KrylovResult kr = smw_step<T>(ctx, op, B, K, m, W, w, p, sc, prm, rhs.get(), sol.get(), yr, yi);
  const int vcols = (cp ? 2 : 1) * w;
  d2d(ctx, V, sol.get(), (size_t)ld * vcols * sizeof(T));
  if (K != nullptr && m > 0) {
    // V += S Yhat, Yhat the real form of the complex m x w matrix Y
    const int sr = (cp ? 2 : 1) * m;
    std::vector<double> Yh((size_t)sr * vcols, 0.0);
    for (int c = 0; c < w; ++c)
      for (int l = 0; l < m; ++l) {
        const double a = yr[(size_t)c * m + l], b = yi[(size_t)c * m + l];
        if (!cp) {
          Yh[(size_t)c * sr + l] = a;
        } else {
          Yh[(size_t)(2 * c) * sr + 2 * l] = a;
          Yh[(size_t)(2 * c + 1) * sr + 2 * l] = b;
          Yh[(size_t)(2 * c) * sr + 2 * l + 1] = -b;
          Yh[(size_t)(2 * c + 1) * sr + 2 * l + 1] = a;
        }
      }
    DBuf<double> dY(ctx, Yh.size());
    h2d(ctx, dY.get(), Yh.data(), Yh.size() * sizeof(double));
    tsgemm<T, T>(ctx, n, (const T*)sc.S.get(), ld, sr, dY.get(), sr, vcols, 1.0, 1.0, V, ld);
  }
  ctx->sync();
  return kr;
}

template KrylovResult shifted_solve<double>(Ctx*, const SellOp&, const double*, const double*, int, const double*,
                                            int, Shift, const LradiParams&, double*);
template KrylovResult shifted_solve<float>(Ctx*, const SellOp&, const float*, const float*, int, const float*, int,
                                           Shift, const LradiParams&, float*);

template LradiOut lradi_run<double>(Ctx*, const SellOp&, const double*, const double*, int, double*, int,
                                    const std::vector<Shift>&, const LradiParams&, ZBuffer<double>&, int);
template LradiOut lradi_run<float>(Ctx*, const SellOp&, const float*, const float*, int, float*, int,
                                   const std::vector<Shift>&, const LradiParams&, ZBuffer<float>&, int);

}  // namespace mpcare
