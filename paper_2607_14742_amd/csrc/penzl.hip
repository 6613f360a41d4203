// Heuristic ADI shifts from Ritz values.  Sec. 5 says only that its shifts
// come from Krylov subspaces, computed as the run goes; read here as Penzl's
// procedure (Penzl 2000, Sec. 5) or as projection shifts (below,
// projection_shifts).  Penzl's procedure:
//   1. kp Arnoldi steps with F = A^T from b0 = ones / sqrt(n) -> Ritz values
//   2. km Arnoldi steps with F^{-1} -> Ritz values, inverted
//   3. candidates: the Ritz values in the open left half-plane
//   4. greedy min-max: the first shift minimises max_t |(t - p)/(t + p)|, then
//      the candidate where prod_{p in P} |(t - p)/(t + p)| is largest joins
//      P until l0 shifts are chosen (a complex one brings its conjugate).
// The Krylov steps run on the GPU (FP64 sparse products, or BiCGStab for
// F^{-1}, classical Gram-Schmidt applied twice through the Gram/tall-skinny
// kernels); the k x k Hessenberg eigenvalues and the greedy choice are small
// host computations.
#include <algorithm>
#include <cfloat>
#include <cstdio>
#include <cmath>
#include <complex>

#include "care.hpp"
#include "dense.hpp"

namespace mpcare {

using cplx = std::complex<double>;

// Eigenvalues of a real upper Hessenberg matrix (column-major, leading
// dimension ldh) by the Francis implicit double-shift QR iteration
// (Golub & Van Loan, Sec. 7.5), eigenvalues only: every transformation is
// confined to the active diagonal block [lo, hi].
std::vector<cplx> hessenberg_eigvals(const double* Hin, int k, int64_t ldh) {
  std::vector<double> a((size_t)k * k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) a[(size_t)j * k + i] = (i <= j + 1) ? Hin[(size_t)j * ldh + i] : 0.0;
  auto A = [&](int i, int j) -> double& { return a[(size_t)j * k + i]; };
  std::vector<cplx> ev(k);
  double anorm = 0.0;
  for (double v : a) anorm += std::fabs(v);
  const double eps = DBL_EPSILON;
  int hi = k - 1, its = 0;
  while (hi >= 0) {
    int lo = hi;
    while (lo > 0) {   // negligible subdiagonal entry splits the matrix
      double s = std::fabs(A(lo - 1, lo - 1)) + std::fabs(A(lo, lo));
      if (s == 0.0) s = anorm;
      if (std::fabs(A(lo, lo - 1)) <= eps * s) {
        A(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {    // 1 x 1 block
      ev[hi] = A(hi, hi);
      --hi;
      its = 0;
      continue;
    }
    if (lo == hi - 1) {   // 2 x 2 block: roots of its characteristic polynomial
      const double a11 = A(hi - 1, hi - 1), a12 = A(hi - 1, hi), a21 = A(hi, hi - 1), a22 = A(hi, hi);
      const double half = 0.5 * (a11 - a22), disc = half * half + a12 * a21;
      const double mid = 0.5 * (a11 + a22);
      if (disc >= 0.0) {
        const double r = std::sqrt(disc);
        const double big = mid + (mid >= 0 ? r : -r);    // the root free of cancellation
        const double det = a11 * a22 - a12 * a21;        // product of the two roots
        ev[hi - 1] = big;
        ev[hi] = big != 0.0 ? det / big : 0.0;
      } else {
        const double r = std::sqrt(-disc);
        ev[hi - 1] = cplx(mid, r);
        ev[hi] = cplx(mid, -r);
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (++its > 100) fail(CARE_ERR_BREAKDOWN, "Hessenberg QR iteration did not converge");
    // shifts: the eigenvalues of the trailing 2 x 2 block (sum s, product t),
    // replaced by an ad hoc pair every tenth iteration
    double s, t;
    if (its % 10 == 0) {
      const double w = std::fabs(A(hi, hi - 1)) + std::fabs(A(hi - 1, hi - 2));
      s = 1.5 * w;
      t = w * w;
    } else {
      s = A(hi - 1, hi - 1) + A(hi, hi);
      t = A(hi - 1, hi - 1) * A(hi, hi) - A(hi - 1, hi) * A(hi, hi - 1);
    }
    // first column of (H - s1 I)(H - s2 I) = H^2 - s H + t I, rows lo..lo+2
    double x = A(lo, lo) * A(lo, lo) + A(lo, lo + 1) * A(lo + 1, lo) - s * A(lo, lo) + t;
    double y = A(lo + 1, lo) * (A(lo, lo) + A(lo + 1, lo + 1) - s);
    double z = A(lo + 1, lo) * A(lo + 2, lo + 1);
    for (int c = lo; c <= hi - 1; ++c) {
      const int nr = c < hi - 1 ? 3 : 2;
      if (c > lo) {
        x = A(c, c - 1);
        y = A(c + 1, c - 1);
        z = nr == 3 ? A(c + 2, c - 1) : 0.0;
      }
      // Householder reflector I - beta v v^T with v = u - alpha e1, u = (x, y, z)
      const double nu = std::sqrt(x * x + y * y + z * z);
      if (nu == 0.0) continue;
      const double alpha = x > 0 ? -nu : nu;
      const double v0 = x - alpha, v1 = y, v2 = z;
      const double beta = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
      for (int j = std::max(lo, c - 1); j <= hi; ++j) {   // from the left
        const double d = beta * (v0 * A(c, j) + v1 * A(c + 1, j) + (nr == 3 ? v2 * A(c + 2, j) : 0.0));
        A(c, j) -= d * v0;
        A(c + 1, j) -= d * v1;
        if (nr == 3) A(c + 2, j) -= d * v2;
      }
      if (c > lo) {
        A(c, c - 1) = alpha;
        A(c + 1, c - 1) = 0.0;
        if (nr == 3) A(c + 2, c - 1) = 0.0;
      }
      const int imax = std::min(c + 3, hi);
      for (int i = lo; i <= imax; ++i) {                  // from the right
        const double d = beta * (A(i, c) * v0 + A(i, c + 1) * v1 + (nr == 3 ? A(i, c + 2) * v2 : 0.0));
        A(i, c) -= d * v0;
        A(i, c + 1) -= d * v1;
        if (nr == 3) A(i, c + 2) -= d * v2;
      }
    }
  }
  return ev;
}

std::vector<Shift> penzl_select(std::vector<cplx> R, int l0) {
  std::vector<cplx> cand;
  for (const cplx& t : R)
    if (t.real() < 0.0 && std::isfinite(t.real()) && std::isfinite(t.imag())) cand.push_back(t);
  if (cand.empty()) fail(CARE_ERR_UNSTABLE, "no Ritz value in the open left half-plane");
  std::stable_sort(cand.begin(), cand.end(), [](const cplx& a, const cplx& b) {
    return a.real() < b.real() || (a.real() == b.real() && a.imag() < b.imag());
  });
  auto ratio = [](const cplx& t, const cplx& p) { return std::abs((t - p) / (t + p)); };
  int first = 0;
  double best = INFINITY;
  for (size_t ip = 0; ip < cand.size(); ++ip) {
    double worst = 0.0;
    for (const cplx& t : cand) worst = std::max(worst, ratio(t, cand[ip]));
    if (worst < best) {
      best = worst;
      first = (int)ip;
    }
  }
  std::vector<cplx> P;
  auto add = [&](const cplx& p) {
    if (p.imag() != 0.0) {
      P.emplace_back(p.real(), std::fabs(p.imag()));
      P.emplace_back(p.real(), -std::fabs(p.imag()));
    } else {
      P.emplace_back(p.real(), 0.0);
    }
  };
  add(cand[first]);
  while ((int)P.size() < l0) {
    int imax = 0;
    double smax = -1.0;
    for (size_t it = 0; it < cand.size(); ++it) {
      double s = 1.0;
      for (const cplx& p : P) s *= ratio(cand[it], p);
      if (s > smax) {
        smax = s;
        imax = (int)it;
      }
    }
    if (smax == 0.0) break;   // every candidate is already a shift
    add(cand[imax]);
  }
  std::vector<Shift> out;
  for (const cplx& p : P) out.push_back(Shift{p.real(), p.imag()});
  return out;
}

// Ritz values of k Arnoldi steps with F = A_k^T = A^T - K B^T (K = NULL or
// m = 0: F = A^T) from ones / sqrt(n).  The inverse F^{-1} is applied by
// BiCGStab on A^T to relative residual 1e-12 plus the Sherman-Morrison-
// Woodbury correction F^{-1} v = M^{-1} v + S (I - B^T S)^{-1} B^T M^{-1} v,
// M = A^T, S = M^{-1} K (Sec. 4).  B, K: FP64, n x m, ld pad_ld(n).
static std::vector<cplx> arnoldi_ritz(Ctx* ctx, const SellOp& op, int k, bool inverse, const double* B,
                                      const double* K, int m) {
  const int64_t n = op.n, ld = pad_ld(n);
  if (!B || !K) m = 0;
  DBuf<double> V(ctx, (size_t)ld * (k + 1)), w(ctx, ld), h1(ctx, k + 1), h2(ctx, k + 1), nn(ctx, 1);
  DBuf<double> bw(ctx, (size_t)std::max(m, 1)), Sm(ctx, (size_t)ld * std::max(m, 1)), coef(ctx, (size_t)std::max(m, 1));
  std::vector<double> Tinv((size_t)m * m);
  auto solve_m = [&](const double* rhs, int cols, double* out) {
    // BiCGStab whatever the context's choice for the ADI solves: the
    // unshifted solves need 1e-12, a long iteration budget and a long
    // stagnation window
    const int method = ctx->krylov_method;
    ctx->krylov_method = 0;
    ctx->krylov_patient = 1;
    KrylovResult kr;
    try {
      kr = bicgstab<double>(ctx, op, 0.0, 0.0, cols, rhs, ld, out, ld, 1e-12, 20000, 8);
    } catch (...) {
      ctx->krylov_method = method;
      ctx->krylov_patient = 0;
      throw;
    }
    ctx->krylov_method = method;
    ctx->krylov_patient = 0;
    if (!(kr.worst_relres < 1e-6)) {
      char msg[160];
      std::snprintf(msg, sizeof msg,
                    "inverse Arnoldi solve with A^T did not converge (relative residual %.2e after %d iterations, "
                    "%d restarts, %d breakdowns)",
                    kr.worst_relres, kr.max_iters, kr.restarts, kr.breakdown);
      fail(CARE_ERR_BREAKDOWN, msg);
    }
  };
  if (inverse && m > 0) {
    // S = M^{-1} K, Tinv = (I - B^T S)^{-1} (host, m x m)
    solve_m(K, m, Sm.get());
    DBuf<double> G(ctx, (size_t)m * m);
    gram(ctx, n, B, ld, m, Sm.get(), ld, m, G.get(), m);
    std::vector<double> g((size_t)m * m);
    d2h(ctx, g.data(), G.get(), g.size() * sizeof(double));
    std::vector<cplx> T((size_t)m * m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) T[(size_t)j * m + i] = (i == j ? 1.0 : 0.0) - g[(size_t)j * m + i];
    if (!cinv(m, T)) fail(CARE_ERR_BREAKDOWN, "singular capacitance matrix I - B^T A^-T K");
    for (size_t e = 0; e < T.size(); ++e) Tinv[e] = T[e].real();
  }
  {
    std::vector<double> b0(n, 1.0 / std::sqrt((double)n));
    h2d(ctx, V.get(), b0.data(), n * sizeof(double));
  }
  std::vector<double> H((size_t)(k + 1) * k, 0.0);   // (k+1) x k, ld k+1
  int steps = k;
  for (int j = 0; j < k; ++j) {
    const double* vj = V.get() + (int64_t)j * ld;
    if (!inverse) {
      spmm_plain(ctx, op, 0.0, 0.0, vj, ld, 1, w.get(), ld);
      if (m > 0) {   // w -= K (B^T v)
        gram(ctx, n, B, ld, m, vj, ld, 1, bw.get(), m);
        tsgemm(ctx, n, K, ld, m, bw.get(), m, 1, -1.0, 1.0, w.get(), ld);
      }
    } else {
      solve_m(vj, 1, w.get());
      if (m > 0) {   // w += S Tinv (B^T w)
        std::vector<double> bt(m), c(m, 0.0);
        gram(ctx, n, B, ld, m, w.get(), ld, 1, bw.get(), m);
        d2h(ctx, bt.data(), bw.get(), m * sizeof(double));
        for (int i = 0; i < m; ++i)
          for (int l = 0; l < m; ++l) c[i] += Tinv[(size_t)l * m + i] * bt[l];
        h2d(ctx, coef.get(), c.data(), m * sizeof(double));
        tsgemm(ctx, n, Sm.get(), ld, m, coef.get(), m, 1, 1.0, 1.0, w.get(), ld);
      }
    }
    // classical Gram-Schmidt, twice
    std::vector<double> hc(j + 1, 0.0), tmp(j + 1);
    for (int rep = 0; rep < 2; ++rep) {
      gram(ctx, n, V.get(), ld, j + 1, w.get(), ld, 1, h1.get(), j + 1);
      tsgemm(ctx, n, V.get(), ld, j + 1, h1.get(), j + 1, 1, -1.0, 1.0, w.get(), ld);
      d2h(ctx, tmp.data(), h1.get(), (j + 1) * sizeof(double));
      for (int i = 0; i <= j; ++i) hc[i] += tmp[i];
    }
    gram(ctx, n, w.get(), ld, 1, w.get(), ld, 1, nn.get(), 1);
    double nrm2 = 0.0;
    d2h(ctx, &nrm2, nn.get(), sizeof(double));
    const double hn = std::sqrt(std::max(nrm2, 0.0));
    if (!std::isfinite(hn)) fail(CARE_ERR_NONFINITE, "non-finite Arnoldi vector");
    double colnorm = hn * hn;
    for (int i = 0; i <= j; ++i) {
      H[(size_t)j * (k + 1) + i] = hc[i];
      colnorm += hc[i] * hc[i];
    }
    H[(size_t)j * (k + 1) + j + 1] = hn;
    if (hn <= 1e-12 * std::sqrt(colnorm)) {   // invariant subspace: the Ritz values are exact
      steps = j + 1;
      break;
    }
    axpby<double>(ctx, n, 1, 1.0 / hn, w.get(), ld, 0.0, V.get() + (int64_t)(j + 1) * ld, ld);
  }
  std::vector<cplx> ev = hessenberg_eigvals(H.data(), steps, k + 1);
  if (inverse)
    for (cplx& t : ev) t = 1.0 / t;
  return ev;
}

// Reduction of a real k x k matrix (column-major, leading dimension k) to
// upper Hessenberg form by Householder similarity transformations
// (Golub & Van Loan, Sec. 7.4.3): the eigenvalues are unchanged.  Host.
static void hessenberg_reduce(std::vector<double>& a, int k) {
  auto A = [&](int i, int j) -> double& { return a[(size_t)j * k + i]; };
  std::vector<double> v(k);
  for (int c = 0; c + 2 < k; ++c) {
    double alpha = 0.0;
    for (int i = c + 1; i < k; ++i) alpha += A(i, c) * A(i, c);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (A(c + 1, c) > 0.0) alpha = -alpha;
    const int len = k - c - 1;
    double vn2 = 0.0;
    for (int t = 0; t < len; ++t) {
      v[t] = A(c + 1 + t, c) - (t == 0 ? alpha : 0.0);
      vn2 += v[t] * v[t];
    }
    if (vn2 == 0.0) continue;
    const double beta = 2.0 / vn2;
    for (int j = c; j < k; ++j) {            // rows c+1.. from the left
      double d = 0.0;
      for (int t = 0; t < len; ++t) d += v[t] * A(c + 1 + t, j);
      d *= beta;
      for (int t = 0; t < len; ++t) A(c + 1 + t, j) -= d * v[t];
    }
    for (int i = 0; i < k; ++i) {            // columns c+1.. from the right
      double d = 0.0;
      for (int t = 0; t < len; ++t) d += A(i, c + 1 + t) * v[t];
      d *= beta;
      for (int t = 0; t < len; ++t) A(i, c + 1 + t) -= d * v[t];
    }
    for (int i = c + 2; i < k; ++i) A(i, c) = 0.0;
  }
}

// Projection shifts (Benner, Kuerschner and Saak, ETNA 43, 2014): the other
// reading of Sec. 5's Krylov-subspace shifts, in which each LR-ADI run draws
// its shifts from its own iterates as it goes.  Steps:
//   1. the dominant directions of span(V): V^T V = U L U^T,
//      Q = V U_k L_k^{-1/2} over the eigenvalues above 1e-10 max L (<= 64);
//   2. H = Q^T F Q with F = A^T - K B^T (sparse product, Gram);
//   3. the eigenvalues of H (host: Hessenberg reduction, Francis QR);
//   4. mirrored into the open left half-plane, Penzl's greedy choice of at
//      most l0 among them.
template <typename T>
std::vector<Shift> projection_shifts(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, const T* V,
                                     int64_t ldv, int s, int l0) {
  const int64_t n = op.n, ld = pad_ld(n);
  if (s < 1 || l0 < 1) fail(CARE_ERR_ARG, "projection shifts need s >= 1 and l0 >= 1");
  if (!V || ldv < n) fail(CARE_ERR_ARG, "invalid projection basis");
  if ((op.prec == Prec::F64) != (sizeof(T) == 8)) fail(CARE_ERR_ARG, "projection basis precision mismatch");
  DBuf<double> G(ctx, (size_t)s * s);
  gram<T, T>(ctx, n, V, ldv, s, V, ldv, s, G.get(), s);
  std::vector<double> lam;
  dsyevd(ctx, s, G.get(), s, lam);
  const double lmax = lam.back();
  if (!(lmax > 0.0) || !std::isfinite(lmax)) fail(CARE_ERR_BREAKDOWN, "projection basis is zero or not finite");
  std::vector<int> sel;
  std::vector<double> isq;
  for (int i = s - 1; i >= 0 && (int)sel.size() < 64; --i)
    if (lam[i] > 1e-10 * lmax) {
      sel.push_back(i);
      isq.push_back(1.0 / std::sqrt(lam[i]));
    }
  const int k = (int)sel.size();
  DBuf<double> Uk(ctx, (size_t)s * k);
  copy_cols<double, double>(ctx, s, k, G.get(), s, Uk.get(), s, sel.data(), isq.data());
  DBuf<T> Q(ctx, (size_t)ld * k), Y(ctx, (size_t)ld * k);
  tsgemm<T, T>(ctx, n, V, ldv, s, Uk.get(), s, k, 1.0, 0.0, Q.get(), ld);
  spmm_plain(ctx, op, 0.0, 0.0, Q.get(), ld, k, Y.get(), ld);
  if (B && K && m > 0) {   // Y -= K (B^T Q)
    DBuf<double> Cq(ctx, (size_t)m * k);
    gram<T, T>(ctx, n, B, ld, m, Q.get(), ld, k, Cq.get(), m);
    tsgemm<T, T>(ctx, n, K, ld, m, Cq.get(), m, k, -1.0, 1.0, Y.get(), ld);
  }
  DBuf<double> H(ctx, (size_t)k * k);
  gram<T, T>(ctx, n, Q.get(), ld, k, Y.get(), ld, k, H.get(), k);
  std::vector<double> h((size_t)k * k);
  d2h(ctx, h.data(), H.get(), h.size() * sizeof(double));
  for (double x : h)
    if (!std::isfinite(x)) fail(CARE_ERR_NONFINITE, "projected matrix is not finite");
  hessenberg_reduce(h, k);
  std::vector<cplx> ev = hessenberg_eigvals(h.data(), k, k);
  for (cplx& t : ev)
    if (t.real() > 0.0) t = -std::conj(t);
  return penzl_select(ev, l0);
}

template std::vector<Shift> projection_shifts<double>(Ctx*, const SellOp&, const double*, const double*, int,
                                                      const double*, int64_t, int, int);
template std::vector<Shift> projection_shifts<float>(Ctx*, const SellOp&, const float*, const float*, int,
                                                     const float*, int64_t, int, int);

std::vector<Shift> penzl_shifts(Ctx* ctx, const SellOp& A64, int l0, int kp, int km, bool real_only, const double* B,
                                const double* K, int m) {
  if (A64.prec != Prec::F64) fail(CARE_ERR_ARG, "Ritz values need the FP64 operator");
  if (l0 < 1 || kp < 1 || km < 0) fail(CARE_ERR_ARG, "need l0 >= 1, kp >= 1, km >= 0");
  const int kcap = (int)std::min<int64_t>(A64.n, 1000);
  std::vector<cplx> R = arnoldi_ritz(ctx, A64, std::min(kp, kcap), false, B, K, m);
  if (km > 0) {
    std::vector<cplx> Ri = arnoldi_ritz(ctx, A64, std::min(km, kcap), true, B, K, m);
    R.insert(R.end(), Ri.begin(), Ri.end());
  }
  if (real_only)
    for (cplx& t : R) t = cplx(t.real(), 0.0);
  ctx->sync();
  return penzl_select(R, l0);
}

}  // namespace mpcare
