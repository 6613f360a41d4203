// Algorithms 1 and 2 (FP64).
#include "lowrank.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace mpcare {

// Algorithm 1.  The paper factors R(Z) = F M F^T with
// F = [Z, A^T Z, Z Z^T B, C^T].  The third block lies in range(Z)
// (Z Z^T B = Z Y with Y = Z^T B), so the same residual is formed here as
//   R(Z) = F' M' F'^T,   F' = [Z, A^T Z, C^T],
//   M' = [[-Y Y^T, I, 0], [I, 0, 0], [0, 0, I_p]],
// which is identical in exact arithmetic and avoids m exactly dependent
// columns in the thin QR.  Then F' = U T (rank-revealing, Householder
// accuracy), H = T M' T^T, H = Q Lambda Q^T, J+- = {lambda >= eta} / {lambda <= -eta},
// C+ = U Q+ Lambda+^(1/2), C- = U Q- (-Lambda-)^(1/2), ||R||_F = ||Lambda||_2.
// T (k x (r + c), ld k) = [[diag(sqrt(sig)), Trest(0:r, :)], [0, Trest(r:k, :)]]
// for U = [Q, U_new] and a matrix [Q diag(sqrt(sig)), rest]: the coefficients
// of the leading block are exact, those of the rest come from the
// orthogonalisation (Trest, k x c, ld k).
__global__ void k_basis_block(double* __restrict__ T, int k, int r, const double* __restrict__ sq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < k && j < r) T[(int64_t)j * k + i] = i == j ? sq[j] : 0.0;
}

static void basis_coefficients(Ctx* ctx, const TruncResult& Zk, const Orth& o, int c, DBuf<double>& T) {
  const int k = o.k, r = Zk.r;
  T.resize(ctx, (size_t)k * std::max(r + c, 1));
  std::vector<double> sq(r);
  for (int j = 0; j < r; ++j) sq[j] = std::sqrt(std::max(Zk.sig[j], 0.0));
  DBuf<double> dsq(ctx, std::max(r, 1));
  if (r > 0) {
    h2d(ctx, dsq.get(), sq.data(), r * sizeof(double));
    hipLaunchKernelGGL(k_basis_block, dim3(ceil_div(k, 64), r), dim3(64), 0, ctx->stream, T.get(), k, r, dsq.get());
    KERNEL_CHECK();
  }
  if (c > 0) copy_cols<double, double>(ctx, k, c, o.T.get(), k, T.get() + (int64_t)r * k, k);
  ctx->sync();
}

void residual_factor(Ctx* ctx, const SellOp& A64, const double* B, int m, const double* Ct, int p, const double* Z,
                     int64_t ldz, int r, double eta_r_rel, ResidualFactor& out, double drop_fro,
                     const TruncResult* basis) {
  const int64_t n = A64.n;
  const int64_t ld = pad_ld(n);
  const int q = 2 * r + p;
  out.rp = out.rm = 0;
  out.res_fro = 0.0;
  if (q == 0) return;
  DBuf<double> F(ctx, (size_t)ld * q);
  if (r > 0) copy_cols<double, double>(ctx, n, r, Z, ldz, F.get(), ld);
  if (r > 0) spmm_plain(ctx, A64, 0.0, 0.0, Z, ldz, r, F.get() + (int64_t)r * ld, ld);
  if (p > 0) copy_cols<double, double>(ctx, n, p, Ct, ld, F.get() + (int64_t)(2 * r) * ld, ld);

  // M'
  std::vector<double> Mh((size_t)q * q, 0.0);
  if (r > 0 && m > 0) {
    DBuf<double> Y(ctx, (size_t)r * m);
    gram(ctx, n, Z, ldz, r, B, ld, m, Y.get(), r);
    std::vector<double> y((size_t)r * m);
    d2h(ctx, y.data(), Y.get(), y.size() * sizeof(double));
    for (int j = 0; j < r; ++j)
      for (int i = 0; i < r; ++i) {
        double s = 0;
        for (int l = 0; l < m; ++l) s += y[(size_t)l * r + i] * y[(size_t)l * r + j];
        Mh[(size_t)j * q + i] = -s;
      }
  }
  for (int i = 0; i < r; ++i) {
    Mh[(size_t)(r + i) * q + i] = 1.0;
    Mh[(size_t)i * q + (r + i)] = 1.0;
  }
  for (int i = 0; i < p; ++i) Mh[(size_t)(2 * r + i) * q + (2 * r + i)] = 1.0;

  Orth o;
  DBuf<double> Tb;
  const double* T = nullptr;
  if (basis && basis->has_q && basis->r == r && r > 0) {
    // Z = Q diag(sqrt(sig)) with orthonormal Q: orthogonalise [A^T Z, C^T]
    // against Q and among themselves only
    rr_orth(ctx, n, F.get() + (int64_t)r * ld, ld, r + p, o, basis->Q.get(), ld, r);
    if (o.k == 0) return;
    basis_coefficients(ctx, *basis, o, r + p, Tb);
    T = Tb.get();
  } else {
    rr_orth(ctx, n, F.get(), ld, q, o);
    T = o.T.get();
  }
  const int k = o.k;
  if (k == 0) return;
  DBuf<double> M(ctx, (size_t)q * q), TM(ctx, (size_t)k * q), H(ctx, (size_t)k * k), Hs(ctx, (size_t)k * k);
  h2d(ctx, M.get(), Mh.data(), Mh.size() * sizeof(double));
  dgemm(ctx, false, false, k, q, q, 1.0, T, k, M.get(), q, 0.0, TM.get(), k);
  dgemm(ctx, false, true, k, k, q, 1.0, TM.get(), k, T, k, 0.0, H.get(), k);
  {
    const double half = 0.5;
    ROCBLAS_CHECK(rocblas_dgeam(ctx->blas, rocblas_operation_none, rocblas_operation_transpose, k, k, &half, H.get(),
                                k, &half, H.get(), k, Hs.get(), k));
  }
  std::vector<double> lam;
  dsyevd(ctx, k, Hs.get(), k, lam);
  double ss = 0.0, lmax = 0.0;
  for (double v : lam) {
    ss += v * v;
    lmax = std::max(lmax, std::fabs(v));
  }
  out.res_fro = std::sqrt(ss);
  out.lam_max = lmax;
  double eta = eta_r_rel * lmax;
  if (drop_fro > 0.0) {
    // eigenvalues strictly above the cut are kept: nudge eta just past it
    const double cut = frobenius_cut(lam, drop_fro);
    if (cut > 0.0) eta = std::max(eta, std::nextafter(cut, INFINITY));
  }
  std::vector<int> selp, selm;
  std::vector<double> scp, scm;
  for (int i = k - 1; i >= 0; --i) {
    const bool pos = eta > 0 ? lam[i] >= eta : lam[i] > 0;
    if (pos) {
      selp.push_back(i);
      scp.push_back(std::sqrt(lam[i]));
    }
  }
  for (int i = 0; i < k; ++i) {
    const bool neg = eta > 0 ? lam[i] <= -eta : lam[i] < 0;
    if (neg) {
      selm.push_back(i);
      scm.push_back(std::sqrt(-lam[i]));
    }
  }
  out.rp = (int)selp.size();
  out.rm = (int)selm.size();
  DBuf<double> coef(ctx, (size_t)k * std::max(1, out.rp + out.rm));
  if (out.rp) copy_cols<double, double>(ctx, k, out.rp, Hs.get(), k, coef.get(), k, selp.data(), scp.data());
  if (out.rm)
    copy_cols<double, double>(ctx, k, out.rm, Hs.get(), k, coef.get() + (int64_t)out.rp * k, k, selm.data(),
                              scm.data());
  out.Cp.resize(ctx, (size_t)ld * std::max(1, out.rp));
  out.Cm.resize(ctx, (size_t)ld * std::max(1, out.rm));
  if (out.rp) tsgemm(ctx, n, o.U.get(), o.ldu, k, coef.get(), k, out.rp, 1.0, 0.0, out.Cp.get(), ld);
  if (out.rm)
    tsgemm(ctx, n, o.U.get(), o.ldu, k, coef.get() + (int64_t)out.rp * k, k, out.rm, 1.0, 0.0, out.Cm.get(), ld);
  ctx->sync();
}

double frobenius_cut(std::vector<double> v, double drop_fro) {
  for (double& x : v) x = std::fabs(x);
  std::sort(v.begin(), v.end());
  double acc = 0.0, cut = 0.0;
  for (size_t i = 0; i < v.size(); ++i) {
    acc += v[i] * v[i];
    if (acc > drop_fro * drop_fro) break;
    // ties: a magnitude is dropped only together with every entry equal to it
    if (i + 1 == v.size() || v[i + 1] > v[i]) cut = v[i];
  }
  return cut;
}

// Algorithm 2: G = V Gamma, P = Gamma N Gamma^T = Theta Sigma Theta^T,
// keep sigma >= eta_s, Z = V Theta+ Sigma+^(1/2).
// the part of Algorithm 2 after the orthogonalisation G = U T (U: o.U, k
// columns; T: k x s, ld k)
static void truncate_core(Ctx* ctx, int64_t n, const Orth& o, const double* T, int s, const std::vector<double>& sign,
                          double eta_s_rel, TruncResult& out, double res_budget, double a2, double g2) {
  const int64_t ld = pad_ld(n);
  const int k = o.k;
  DBuf<double> GN(ctx, (size_t)k * s), P(ctx, (size_t)k * k), Ps(ctx, (size_t)k * k);
  copy_cols<double, double>(ctx, k, s, T, k, GN.get(), k, nullptr, sign.data());
  dgemm(ctx, false, true, k, k, s, 1.0, GN.get(), k, T, k, 0.0, P.get(), k);
  {
    const double half = 0.5;
    ROCBLAS_CHECK(rocblas_dgeam(ctx->blas, rocblas_operation_none, rocblas_operation_transpose, k, k, &half, P.get(),
                                k, &half, P.get(), k, Ps.get(), k));
  }
  std::vector<double> sig;
  dsyevd(ctx, k, Ps.get(), k, sig);
  double smax = 0.0, all2 = 0.0, neg2 = 0.0;
  for (double v : sig) {
    smax = std::max(smax, std::fabs(v));
    all2 += v * v;
    if (v < 0) neg2 += v * v;
  }
  out.sig_max = smax;
  out.eta_n = all2 > 0 ? std::sqrt(neg2 / all2) : 0.0;
  double eta = eta_s_rel * smax;
  if (res_budget > 0.0 && a2 + g2 * smax > 0.0) {
    std::vector<double> pos;
    for (double v : sig)
      if (v > 0.0) pos.push_back(v);
    const double cut = frobenius_cut(pos, res_budget / (2.0 * (a2 + g2 * smax)));
    if (cut > 0.0) eta = std::max(eta, std::nextafter(cut, INFINITY));
  }
  std::vector<int> sel;
  std::vector<double> sc;
  for (int i = k - 1; i >= 0; --i) {
    const bool keep = eta > 0 ? sig[i] >= eta : sig[i] > 0;
    if (keep) {
      sel.push_back(i);
      sc.push_back(std::sqrt(sig[i]));
    }
  }
  out.r = (int)sel.size();
  out.Z.resize(ctx, (size_t)ld * std::max(1, out.r));
  out.Q.resize(ctx, (size_t)ld * std::max(1, out.r));
  out.sig.resize(out.r);
  for (int j = 0; j < out.r; ++j) out.sig[j] = sig[sel[j]];
  if (out.r) {
    DBuf<double> coef(ctx, (size_t)k * out.r);
    copy_cols<double, double>(ctx, k, out.r, Ps.get(), k, coef.get(), k, sel.data(), sc.data());
    tsgemm(ctx, n, o.U.get(), o.ldu, k, coef.get(), k, out.r, 1.0, 0.0, out.Z.get(), ld);
    copy_cols<double, double>(ctx, k, out.r, Ps.get(), k, coef.get(), k, sel.data());
    tsgemm(ctx, n, o.U.get(), o.ldu, k, coef.get(), k, out.r, 1.0, 0.0, out.Q.get(), ld);
  }
  out.has_q = true;
  ctx->sync();
}

void signed_truncate(Ctx* ctx, int64_t n, const double* G, int64_t ldg, int s, const std::vector<double>& sign,
                     double eta_s_rel, TruncResult& out, double res_budget, double a2, double g2) {
  const int64_t ld = pad_ld(n);
  out.r = 0;
  out.eta_n = 0.0;
  out.has_q = false;
  out.sig.clear();
  if (s <= 0) {
    out.Z.resize(ctx, ld);
    return;
  }
  Orth o;
  rr_orth(ctx, n, G, ldg, s, o);
  if (o.k == 0) {
    out.Z.resize(ctx, ld);
    return;
  }
  truncate_core(ctx, n, o, o.T.get(), s, sign, eta_s_rel, out, res_budget, a2, g2);
}

void signed_truncate_basis(Ctx* ctx, int64_t n, const TruncResult& Zk, const double* Grest, int64_t ldg, int s,
                           const std::vector<double>& sign, double eta_s_rel, TruncResult& out, double res_budget,
                           double a2, double g2) {
  if (!Zk.has_q) fail(CARE_ERR_ARG, "signed_truncate_basis needs a factor with its orthonormal basis");
  const int64_t ld = pad_ld(n);
  out.r = 0;
  out.eta_n = 0.0;
  out.has_q = false;
  out.sig.clear();
  const int r = Zk.r;
  if (r + s <= 0) {
    out.Z.resize(ctx, ld);
    return;
  }
  Orth o;
  rr_orth(ctx, n, Grest, ldg, s, o, Zk.Q.get(), ld, r);
  if (o.k == 0) {
    out.Z.resize(ctx, ld);
    return;
  }
  DBuf<double> T;
  basis_coefficients(ctx, Zk, o, s, T);
  std::vector<double> full(r, 1.0);
  full.insert(full.end(), sign.begin(), sign.end());
  truncate_core(ctx, n, o, T.get(), r + s, full, eta_s_rel, out, res_budget, a2, g2);
}

bool psd_compress(Ctx* ctx, int64_t n, const double* Z, int64_t ldz, int w, double tau_abs, DBuf<double>& out,
                  int& r, double drop_fro) {
  const int64_t ld = pad_ld(n);
  r = 0;
  if (w <= 0) {
    out.resize(ctx, ld);
    return true;
  }
  DBuf<double> G(ctx, (size_t)w * w);
  gram(ctx, n, Z, ldz, w, Z, ldz, w, G.get(), w);
  std::vector<double> lam;
  dsyevd(ctx, w, G.get(), w, lam);
  const double lmax = lam.back();
  if (!(lmax > 0.0)) {
    out.resize(ctx, ld);
    return true;
  }
  if (drop_fro > 0.0) tau_abs = std::max(tau_abs, frobenius_cut(lam, drop_fro));
  if (!(tau_abs >= 1e-14 * lmax)) {
    if (std::getenv("MPCARE_TRACE"))
      std::fprintf(stderr, "[psd_compress] w %d kept whole: tau %.3e below 1e-14 lam_max %.3e\n", w, tau_abs, lmax);
    return false;
  }
  std::vector<int> sel;
  for (int i = w - 1; i >= 0; --i)
    if (lam[i] > tau_abs) sel.push_back(i);
  r = (int)sel.size();
  out.resize(ctx, (size_t)ld * std::max(r, 1));
  if (r) {
    DBuf<double> coef(ctx, (size_t)w * r);
    copy_cols<double, double>(ctx, w, r, G.get(), w, coef.get(), w, sel.data());
    tsgemm(ctx, n, Z, ldz, w, coef.get(), w, r, 1.0, 0.0, out.get(), ld);
  }
  if (std::getenv("MPCARE_TRACE"))
    std::fprintf(stderr, "[psd_compress] w %d -> %d  lam_max %.3e tau %.3e\n", w, r, lmax, tau_abs);
  return true;
}

double factor_lam_max(Ctx* ctx, int64_t n, const double* Z, int64_t ldz, int r) {
  if (r <= 0) return 0.0;
  DBuf<double> G(ctx, (size_t)r * r);
  gram(ctx, n, Z, ldz, r, Z, ldz, r, G.get(), r);
  // a non-finite entry of Z shows in its Gram (the diagonal sums squares)
  std::vector<double> hg((size_t)r * r);
  d2h(ctx, hg.data(), G.get(), hg.size() * sizeof(double));
  for (double g : hg)
    if (!std::isfinite(g)) fail(CARE_ERR_NONFINITE, "the factor has non-finite entries");
  std::vector<double> lam;
  dsyevd(ctx, r, G.get(), r, lam);
  return std::max(lam.back(), 0.0);
}

}  // namespace mpcare
