// Column-batched restarted GMRES(m) for real shifts, the inner solver of
// Sec. 5, optionally right-preconditioned by the multicolour ILU(0) of the
// shifted matrix as there (ilu.hip).
//
// Every right-hand-side column runs its own Arnoldi process; the columns
// share each launch.  One Arnoldi step is one sparse product of the whole
// panel, classical Gram-Schmidt applied twice against the column's basis
// (per-column dot products and updates, FP64 accumulation), and a column
// norm.  The small Hessenberg least-squares problems are updated with Givens
// rotations on the host, one per column and step.  A column leaves the active
// set when its residual estimate meets the tolerance; at the end of a cycle
// the solution update x += V y is applied, and the next cycle restarts from
// the true residual b - M x.
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "dense.hpp"
#include "krylov.hpp"

namespace mpcare {

namespace {

// rows per thread in the dot kernel (measured on the 500 x 500 problem's
// paper-setting solves: 8 is fastest in FP32, 4 in FP64) and rows per block
template <typename T>
constexpr int gm_rows() { return sizeof(T) == 8 ? 4 : 8; }
template <typename T>
constexpr int gm_chunk() { return 256 * gm_rows<T>(); }

// part[(c Jo + i) nb + blk] = sum over the block's rows of V_i[row, c] w[row, c]
// for i < J (V_i = V + i bstride) and, with self = 1, i = J: the block's part
// of w[:, c]^T w[:, c] (Jo = J + self).  The block's rows of w stay in
// registers; each dot is reduced inside its wave by shuffles, and the four
// wave sums meet once in LDS (fixed order), so the block synchronises once
// for all J dots.
template <typename T>
__global__ void __launch_bounds__(256) k_gm_multidot(int64_t n, int J, int self, const T* __restrict__ V, int64_t ld,
                                                     int64_t bstride, const T* __restrict__ w, int64_t ldw,
                                                     const int* __restrict__ active, double* __restrict__ part,
                                                     int nb) {
  const int c = blockIdx.y, blk = blockIdx.x;
  extern __shared__ double gm_sh[];          // (J + self) x 4 wave sums
  const int Jo = J + self;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool on = active[c] != 0;
  constexpr int GM_ROWS = gm_rows<T>();
  double wv[GM_ROWS];
  int64_t rows[GM_ROWS];
#pragma unroll
  for (int u = 0; u < GM_ROWS; ++u) {
    rows[u] = (int64_t)blk * gm_chunk<T>() + u * 256 + threadIdx.x;
    wv[u] = (on && rows[u] < n) ? (double)w[(int64_t)c * ldw + rows[u]] : 0.0;
  }
  for (int i = 0; i < Jo; ++i) {
    double s = 0.0;
    if (on) {
      if (i < J) {
        const T* vi = V + (int64_t)i * bstride + (int64_t)c * ld;
#pragma unroll
        for (int u = 0; u < GM_ROWS; ++u)
          if (rows[u] < n) s += (double)vi[rows[u]] * wv[u];
      } else {
#pragma unroll
        for (int u = 0; u < GM_ROWS; ++u) s += wv[u] * wv[u];
      }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) gm_sh[i * 4 + wave] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < Jo; i += 256)
    part[((int64_t)c * Jo + i) * nb + blk] = (gm_sh[i * 4] + gm_sh[i * 4 + 1]) + (gm_sh[i * 4 + 2] + gm_sh[i * 4 + 3]);
}

// h[t] = sum_blk part[t nb + blk] for t < total: one wave per output, the
// lanes take strided blocks and a shuffle tree combines them (fixed order)
__global__ void __launch_bounds__(256) k_gm_reduce(int total, int nb, const double* __restrict__ part,
                                                   double* __restrict__ h) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= total) return;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[(int64_t)t * nb + b];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) h[t] = s;
}

// y[:, c] += alpha sum_{i < J} coef[c cstride + i] V_i[:, c] for active columns
template <typename T>
__global__ void __launch_bounds__(256) k_gm_multiaxpy(int64_t n, int J, const T* __restrict__ V, int64_t ld,
                                                      int64_t bstride, const double* __restrict__ coef, int cstride,
                                                      double alpha, T* __restrict__ y, int64_t ldy,
                                                      const int* __restrict__ active) {
  const int c = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= n || !active[c]) return;
  double acc = 0.0;
#pragma unroll 4
  for (int i = 0; i < J; ++i)
    acc += coef[(int64_t)c * cstride + i] * (double)V[(int64_t)i * bstride + (int64_t)c * ld + row];
  T* yc = y + (int64_t)c * ldy + row;
  *yc = (T)((double)*yc + alpha * acc);
}

// out[:, c] = s[c] * in[:, c]
template <typename T>
__global__ void __launch_bounds__(256) k_gm_scale(int64_t n, const T* __restrict__ in, int64_t ldi,
                                                  const double* __restrict__ s, T* __restrict__ out, int64_t ldo) {
  const int c = blockIdx.y;
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  out[(int64_t)c * ldo + row] = (T)(s[c] * (double)in[(int64_t)c * ldi + row]);
}

}  // namespace

template <typename T>
KrylovResult gmres(Ctx* ctx, const SellOp& op, double pr, int ncols, const T* b, int64_t ldb, T* x, int64_t ldx,
                   double tol, int maxit, int restart, const std::vector<int>* groups) {
  KrylovResult res;
  if (ncols <= 0) return res;
  const int64_t n = op.n, ld = pad_ld(n);
  const int k = ncols;
  const int m = std::min(1000, std::max(1, restart));   // LDS of the dot kernel: (m + 1) x 4 doubles
  const int nb = (int)ceil_div(n, (int64_t)gm_chunk<T>());
  const int64_t bstride = ld * k;
  DBuf<T> V(ctx, (size_t)bstride * (m + 1)), w(ctx, (size_t)bstride);
  DBuf<double> part(ctx, (size_t)nb * k * (m + 1)), hdev(ctx, (size_t)k * (m + 1)), sdev(ctx, (size_t)k);
  DBuf<int> act(ctx, (size_t)k);
  std::vector<int> hact(k, 1);
  dim3 gcol(ceil_div(n, 256), k);
  // right preconditioner (factored once per shift and kept on the operator)
  std::shared_ptr<IluOp::Factors> pre;
  if (ctx->krylov_precond == 1 && op.ilu) pre = ilu_factor(ctx, op, pr);
  DBuf<T> zt(ctx, pre ? (size_t)bstride : 0);

  // per-column sums of squares of an n x k panel (ld = ldp)
  auto colsq = [&](const T* P, int64_t ldp, std::vector<double>& out) {
    std::vector<int> all(k, 1);
    h2d(ctx, act.get(), all.data(), k * sizeof(int));
    hipLaunchKernelGGL(k_gm_multidot<T>, dim3(nb, k), dim3(256), 4 * sizeof(double), ctx->stream, n, 0, 1, P, ldp,
                       (int64_t)0, P, ldp, act.get(), part.get(), nb);
    KERNEL_CHECK();
    hipLaunchKernelGGL(k_gm_reduce, dim3(ceil_div(k, 4)), dim3(256), 0, ctx->stream, k, nb, part.get(),
                       hdev.get());
    KERNEL_CHECK();
    out.resize(k);
    d2h(ctx, out.data(), hdev.get(), k * sizeof(double));
  };

  // targets: ||r_c|| <= tol ||b_c|| (or the largest ||b|| of its group)
  std::vector<double> bn2;
  colsq(b, ldb, bn2);
  std::vector<double> bnorm(k), target(k);
  for (int c = 0; c < k; ++c) bnorm[c] = std::sqrt(std::max(bn2[c], 0.0));
  std::map<int, double> gmax;
  if (groups)
    for (int c = 0; c < k; ++c) gmax[(*groups)[c]] = std::max(gmax[(*groups)[c]], bnorm[c]);
  for (int c = 0; c < k; ++c) target[c] = tol * (groups ? gmax[(*groups)[c]] : bnorm[c]);

  for (int c = 0; c < k; ++c) dzero(ctx, x + (int64_t)c * ldx, n * sizeof(T));
  std::vector<int> iters(k, 0), stalled(k, 0);
  std::vector<double> rnorm(bnorm);
  const T* r0 = b;      // residual of the current cycle (first cycle: b itself)
  int64_t ldr = ldb;
  int total = 0;
  std::vector<double> H, cs, sn, g, hv;
  while (total < maxit) {
    // active columns and V_0 = r / ||r||
    std::vector<double> scale(k, 0.0);
    int nact = 0;
    for (int c = 0; c < k; ++c) {
      hact[c] = !stalled[c] && rnorm[c] > target[c] && rnorm[c] > 0.0 && std::isfinite(rnorm[c]) ? 1 : 0;
      if (hact[c]) {
        scale[c] = 1.0 / rnorm[c];
        ++nact;
      }
    }
    if (nact == 0) break;
    h2d(ctx, sdev.get(), scale.data(), k * sizeof(double));
    hipLaunchKernelGGL(k_gm_scale<T>, gcol, dim3(256), 0, ctx->stream, n, r0, ldr, sdev.get(), V.get(), ld);
    KERNEL_CHECK();
    h2d(ctx, act.get(), hact.data(), k * sizeof(int));
    const std::vector<int> cycle_act = hact;
    H.assign((size_t)k * (m + 1) * m, 0.0);
    cs.assign((size_t)k * m, 0.0);
    sn.assign((size_t)k * m, 0.0);
    g.assign((size_t)k * (m + 1), 0.0);
    std::vector<int> jdone(k, -1);   // last Arnoldi step of each column in this cycle
    for (int c = 0; c < k; ++c) g[(size_t)c * (m + 1)] = rnorm[c];
    int j = 0;
    for (; j < m && total < maxit; ++j) {
      // w = M V_j, or M P^{-1} V_j
      if (pre) {
        ilu_apply<T>(ctx, op, *pre, k, V.get() + (int64_t)j * bstride, ld, zt.get(), ld);
        spmm_plain(ctx, op, pr, 0.0, zt.get(), ld, k, w.get(), ld);
      } else {
        spmm_plain(ctx, op, pr, 0.0, V.get() + (int64_t)j * bstride, ld, k, w.get(), ld);
      }
      // classical Gram-Schmidt against V_0..V_j.  The first pass also returns
      // ||w||^2; a column gets a second pass only when its norm after the
      // first, estimated as ||w||^2 - sum_i h_i^2, fell below 1/sqrt(2) of
      // it (the reorthogonalisation test of Daniel, Gragg, Kaufman and
      // Stewart); the others are orthogonal to working accuracy already.
      const int J = j + 1;
      std::vector<double> hsum((size_t)k * J, 0.0);
      std::vector<int> redo(k, 0);
      for (int rep = 0; rep < 2; ++rep) {
        const int self = rep == 0 ? 1 : 0, Jo = J + self;
        if (rep == 1) {
          if (std::none_of(redo.begin(), redo.end(), [](int v) { return v != 0; })) break;
          h2d(ctx, act.get(), redo.data(), k * sizeof(int));
        }
        hipLaunchKernelGGL(k_gm_multidot<T>, dim3(nb, k), dim3(256), (size_t)Jo * 4 * sizeof(double), ctx->stream,
                           n, J, self, V.get(), ld, bstride, w.get(), ld, act.get(), part.get(), nb);
        KERNEL_CHECK();
        hipLaunchKernelGGL(k_gm_reduce, dim3(ceil_div(k * Jo, 4)), dim3(256), 0, ctx->stream, k * Jo, nb,
                           part.get(), hdev.get());
        KERNEL_CHECK();
        hipLaunchKernelGGL(k_gm_multiaxpy<T>, gcol, dim3(256), 0, ctx->stream, n, J, V.get(), ld, bstride,
                           hdev.get(), Jo, -1.0, w.get(), ld, act.get());
        KERNEL_CHECK();
        hv.resize((size_t)k * Jo);
        d2h(ctx, hv.data(), hdev.get(), hv.size() * sizeof(double));
        for (int c = 0; c < k; ++c) {
          if (!(rep == 0 ? hact[c] : redo[c])) continue;
          double h2 = 0.0;
          for (int i = 0; i < J; ++i) {
            const double h = hv[(size_t)c * Jo + i];
            hsum[(size_t)c * J + i] += h;
            h2 += h * h;
          }
          if (rep == 0) {
            const double w2 = hv[(size_t)c * Jo + J];
            redo[c] = (w2 - h2 < 0.5 * w2) ? 1 : 0;
          }
        }
        if (rep == 1) h2d(ctx, act.get(), hact.data(), k * sizeof(int));
      }
      std::vector<double> wn2;
      {
        // ||w_c||^2 over the active columns
        hipLaunchKernelGGL(k_gm_multidot<T>, dim3(nb, k), dim3(256), 4 * sizeof(double), ctx->stream, n, 0, 1,
                           w.get(), ld, (int64_t)0, w.get(), ld, act.get(), part.get(), nb);
        KERNEL_CHECK();
        hipLaunchKernelGGL(k_gm_reduce, dim3(ceil_div(k, 4)), dim3(256), 0, ctx->stream, k, nb, part.get(),
                           hdev.get());
        KERNEL_CHECK();
        wn2.resize(k);
        d2h(ctx, wn2.data(), hdev.get(), k * sizeof(double));
      }
      ++total;
      std::vector<double> inv(k, 0.0);
      for (int c = 0; c < k; ++c) {
        if (!hact[c]) continue;
        iters[c] += 1;
        double* Hc = &H[(size_t)c * (m + 1) * m + (size_t)j * (m + 1)];
        for (int i = 0; i < J; ++i) Hc[i] = hsum[(size_t)c * J + i];
        const double hn = std::sqrt(std::max(wn2[c], 0.0));
        Hc[J] = hn;
        // earlier rotations, then a new one that zeroes Hc[J]
        for (int i = 0; i < j; ++i) {
          const double a = Hc[i], bb = Hc[i + 1];
          Hc[i] = cs[(size_t)c * m + i] * a + sn[(size_t)c * m + i] * bb;
          Hc[i + 1] = -sn[(size_t)c * m + i] * a + cs[(size_t)c * m + i] * bb;
        }
        const double a = Hc[j], bb = Hc[J];
        const double rr = std::hypot(a, bb);
        const double cj = rr > 0.0 ? a / rr : 1.0, sj = rr > 0.0 ? bb / rr : 0.0;
        cs[(size_t)c * m + j] = cj;
        sn[(size_t)c * m + j] = sj;
        Hc[j] = rr;
        Hc[J] = 0.0;
        double* gc = &g[(size_t)c * (m + 1)];
        gc[J] = -sj * gc[j];
        gc[j] = cj * gc[j];
        jdone[c] = j;
        const double est = std::fabs(gc[J]);
        if (!(est > target[c]) || !(hn > 1e-300) || !std::isfinite(est)) {
          hact[c] = 0;            // converged (or happy breakdown): no further steps this cycle
        } else {
          inv[c] = 1.0 / hn;
        }
      }
      // V_{j+1} = w / ||w|| for the columns that go on
      h2d(ctx, sdev.get(), inv.data(), k * sizeof(double));
      hipLaunchKernelGGL(k_gm_scale<T>, gcol, dim3(256), 0, ctx->stream, n, w.get(), ld, sdev.get(),
                         V.get() + (int64_t)(j + 1) * bstride, ld);
      KERNEL_CHECK();
      h2d(ctx, act.get(), hact.data(), k * sizeof(int));
      if (std::none_of(hact.begin(), hact.end(), [](int v) { return v != 0; })) {
        ++j;
        break;
      }
    }
    // y = R^{-1} g per column over its own steps, then x += V y
    const int J = std::max(1, j);
    std::vector<double> Y((size_t)k * J, 0.0);
    std::vector<int> upd(k, 0);
    for (int c = 0; c < k; ++c) {
      if (!cycle_act[c] || jdone[c] < 0) continue;
      const int jc = jdone[c] + 1;   // coefficients 0 .. jc-1
      const double* Hc = &H[(size_t)c * (m + 1) * m];
      const double* gc = &g[(size_t)c * (m + 1)];
      for (int i = jc - 1; i >= 0; --i) {
        double s = gc[i];
        for (int l = i + 1; l < jc; ++l) s -= Hc[(size_t)l * (m + 1) + i] * Y[(size_t)c * J + l];
        const double d = Hc[(size_t)i * (m + 1) + i];
        Y[(size_t)c * J + i] = d != 0.0 ? s / d : 0.0;
      }
      upd[c] = 1;
    }
    h2d(ctx, hdev.get(), Y.data(), Y.size() * sizeof(double));
    h2d(ctx, act.get(), upd.data(), k * sizeof(int));
    if (pre) {
      // x += P^{-1} (V y): columns without an update stay zero in zt
      dzero(ctx, zt.get(), (size_t)bstride * sizeof(T));
      hipLaunchKernelGGL(k_gm_multiaxpy<T>, gcol, dim3(256), 0, ctx->stream, n, J, V.get(), ld, bstride,
                         hdev.get(), J, 1.0, zt.get(), ld, act.get());
      KERNEL_CHECK();
      ilu_apply<T>(ctx, op, *pre, k, zt.get(), ld, w.get(), ld);
      axpby<T>(ctx, n, k, 1.0, w.get(), ld, 1.0, x, ldx);
    } else {
      hipLaunchKernelGGL(k_gm_multiaxpy<T>, gcol, dim3(256), 0, ctx->stream, n, J, V.get(), ld, bstride,
                         hdev.get(), J, 1.0, x, ldx, act.get());
      KERNEL_CHECK();
    }
    // true residual for the next cycle (and the report)
    spmm_plain(ctx, op, pr, 0.0, x, ldx, k, w.get(), ld);
    axpby<T>(ctx, n, k, 1.0, b, ldb, -1.0, w.get(), ld);   // w = b - M x
    std::vector<double> rn2;
    colsq(w.get(), ld, rn2);
    for (int c = 0; c < k; ++c) {
      const double rn = std::sqrt(std::max(rn2[c], 0.0));
      // a cycle that cut the true residual by less than 10 % marks the
      // column stagnant (the working precision's floor, or a restart length
      // too short for the spectrum): it keeps its iterate
      if (cycle_act[c] && !(rn < 0.9 * rnorm[c])) stalled[c] = 1;
      rnorm[c] = rn;
    }
    r0 = w.get();
    ldr = ld;
    // the next cycle's V_0 is formed from w before w is overwritten
    res.restarts += 1;
    bool any = false;
    for (int c = 0; c < k; ++c) any = any || (!stalled[c] && rnorm[c] > target[c]);
    if (!any) break;
  }
  res.restarts = std::max(0, res.restarts - 1);
  for (int c = 0; c < k; ++c) {
    if (!std::isfinite(rnorm[c])) fail(CARE_ERR_NONFINITE, "non-finite value in the GMRES iteration");
    const bool ok = rnorm[c] <= target[c] || bnorm[c] == 0.0;
    res.max_iters = std::max(res.max_iters, iters[c]);
    ctx->krylov_iters += iters[c];
    const double rel = bnorm[c] > 0.0 ? rnorm[c] / bnorm[c] : 0.0;
    res.col_ok.push_back(ok ? 1 : 0);
    res.col_relres.push_back(rel);
    res.col_bnorm.push_back(bnorm[c]);
    res.worst_relres = std::max(res.worst_relres, rel);
    if (!ok) res.unconverged += 1;
  }
  return res;
}

template KrylovResult gmres<double>(Ctx*, const SellOp&, double, int, const double*, int64_t, double*, int64_t,
                                    double, int, int, const std::vector<int>*);
template KrylovResult gmres<float>(Ctx*, const SellOp&, double, int, const float*, int64_t, float*, int64_t, double,
                                   int, int, const std::vector<int>*);

}  // namespace mpcare
