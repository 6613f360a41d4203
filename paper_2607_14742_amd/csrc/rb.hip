// Red-black reduction of the shifted solves (A^T + p I) x = b.
//
// Two-colour the pattern of A (breadth-first search over the undirected
// graph of its off-diagonal entries); when no off-diagonal entry joins two
// rows of the same colour and the diagonal of A is one constant d, order the
// unknowns red then black:
//
//   A^T + p I = [[(d + p) I, E], [F, (d + p) I]].
//
// Eliminating the red unknowns is exact:
//
//   ((d + p) I - F E / (d + p)) x_b = b_b - F b_r / (d + p),
//
// and multiplying by -(d + p) gives a shifted system in the same form as the
// original one, with the operator G = F E (black x black, its own diagonal
// kept) and the shift p' = -(d + p)^2:
//
//   (G + p' I) x_b = F b_r - (d + p) b_b,     x_r = (b_r - E x_b) / (d + p).
//
// So the reduced system runs through the same SELL products and Krylov
// solvers.  It has half the unknowns, and for the diffusion-dominated spectra
// of the FDM operators about a quarter of the condition number (the
// eigenvalues d + p +- mu of the two-cyclic matrix map to
// (d + p - mu)(d + p + mu)), so the Krylov solves take fewer and cheaper
// iterations.  This is the two-colour (red-black) block factorisation that a
// multicolour incomplete LU of a five- or seven-point stencil starts from,
// with the black block's fill kept: the preconditioning of the paper's
// ILU(0)-Krylov inner solves, here exact.
#include <algorithm>
#include <cmath>
#include <queue>

#include "krylov.hpp"

namespace mpcare {

struct RbHost {
  int64_t n = 0, nr = 0, nb = 0;
  double d = 0.0;
  std::vector<int> red, blk;                    // original indices
  std::vector<int> frp, fci;                    // F rows (black), original red columns
  std::vector<double> fv;
  std::vector<int> erp, eci;                    // E rows (red), reduced black columns
  std::vector<double> ev;
  std::vector<int> gtrp, gtci;                  // CSR of G^T (reduced black indices, sorted)
  std::vector<double> gtv;
};

std::shared_ptr<RbHost> rb_analyse(Ctx* ctx, const care_csr* A) {
  if (!A || A->n < 2 || A->nnz <= 0) return nullptr;
  const int64_t n = A->n, nnz = A->nnz;
  std::vector<int> rp(n + 1), ci(nnz);
  std::vector<double> va(nnz);
  d2h(ctx, rp.data(), A->row_ptr, (n + 1) * sizeof(int));
  d2h(ctx, ci.data(), A->col_idx, nnz * sizeof(int));
  d2h(ctx, va.data(), A->val, nnz * sizeof(double));
  if (rp[0] != 0 || rp[n] != nnz) return nullptr;
  // constant diagonal
  double d = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    bool found = false;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= n) return nullptr;
      if (ci[e] == i) {
        if (i == 0) d = va[e];
        if (va[e] != d) return nullptr;
        found = true;
      }
    }
    if (!found) return nullptr;
  }
  if (d == 0.0 || !std::isfinite(d)) return nullptr;
  // A^T (rows of A^T = columns of A)
  std::vector<int> tp(n + 1, 0), tc(nnz);
  std::vector<double> tv(nnz);
  for (int64_t e = 0; e < nnz; ++e) tp[ci[e] + 1] += 1;
  for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
  {
    std::vector<int> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int pos = fill[ci[e]]++;
        tc[pos] = (int)i;
        tv[pos] = va[e];
      }
  }
  // two-colouring of the undirected off-diagonal graph
  std::vector<signed char> col(n, -1);
  std::vector<int> queue;
  queue.reserve(n);
  for (int64_t s = 0; s < n; ++s) {
    if (col[s] >= 0) continue;
    col[s] = 0;
    queue.clear();
    queue.push_back((int)s);
    for (size_t h = 0; h < queue.size(); ++h) {
      const int i = queue[h];
      auto visit = [&](int j) -> bool {
        if (j == i) return true;
        if (col[j] < 0) {
          col[j] = (signed char)(1 - col[i]);
          queue.push_back(j);
          return true;
        }
        return col[j] != col[i];
      };
      for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (!visit(ci[e])) return nullptr;
      for (int e = tp[i]; e < tp[i + 1]; ++e)
        if (!visit(tc[e])) return nullptr;
    }
  }
  auto h = std::make_shared<RbHost>();
  h->n = n;
  h->d = d;
  int64_t c1 = 0;
  for (int64_t i = 0; i < n; ++i) c1 += col[i];
  const int black_colour = (c1 <= n - c1) ? 1 : 0;   // the reduced system takes the smaller colour
  std::vector<int> pos(n);
  for (int64_t i = 0; i < n; ++i) {
    if (col[i] == black_colour) {
      pos[i] = (int)h->blk.size();
      h->blk.push_back((int)i);
    } else {
      pos[i] = (int)h->red.size();
      h->red.push_back((int)i);
    }
  }
  h->nb = (int64_t)h->blk.size();
  h->nr = (int64_t)h->red.size();
  if (h->nb == 0) return nullptr;
  // F: rows of A^T at black rows (red columns, original indices); E: rows of
  // A^T at red rows (black columns, reduced indices)
  h->frp.assign(1, 0);
  for (int i : h->blk) {
    for (int e = tp[i]; e < tp[i + 1]; ++e)
      if (tc[e] != i) {
        h->fci.push_back(tc[e]);
        h->fv.push_back(tv[e]);
      }
    h->frp.push_back((int)h->fci.size());
  }
  h->erp.assign(1, 0);
  for (int j : h->red) {
    for (int e = tp[j]; e < tp[j + 1]; ++e)
      if (tc[e] != j) {
        h->eci.push_back(pos[tc[e]]);
        h->ev.push_back(tv[e]);
      }
    h->erp.push_back((int)h->eci.size());
  }
  // G = F E (black x black) by a sparse accumulator per row
  std::vector<int> grp(1, 0), gci;
  std::vector<double> gv;
  std::vector<double> acc(h->nb, 0.0);
  std::vector<char> mark(h->nb, 0);
  std::vector<int> touched;
  for (int64_t bi = 0; bi < h->nb; ++bi) {
    touched.clear();
    for (int e = h->frp[bi]; e < h->frp[bi + 1]; ++e) {
      const int rj = pos[h->fci[e]];
      const double f = h->fv[e];
      for (int u = h->erp[rj]; u < h->erp[rj + 1]; ++u) {
        const int k = h->eci[u];
        if (!mark[k]) {
          mark[k] = 1;
          touched.push_back(k);
        }
        acc[k] += f * h->ev[u];
      }
    }
    // every black row keeps a diagonal entry (the SELL build needs none, but
    // an isolated black row then still has its G_ii = 0)
    std::sort(touched.begin(), touched.end());
    for (int k : touched) {
      gci.push_back(k);
      gv.push_back(acc[k]);
      acc[k] = 0.0;
      mark[k] = 0;
    }
    grp.push_back((int)gci.size());
  }
  // CSR of G^T (the SELL build takes CSR(M) and stores M^T)
  const int64_t gnnz = (int64_t)gci.size();
  h->gtrp.assign(h->nb + 1, 0);
  h->gtci.resize(gnnz);
  h->gtv.resize(gnnz);
  for (int64_t e = 0; e < gnnz; ++e) h->gtrp[gci[e] + 1] += 1;
  for (int64_t i = 0; i < h->nb; ++i) h->gtrp[i + 1] += h->gtrp[i];
  {
    std::vector<int> fill(h->gtrp.begin(), h->gtrp.end() - 1);
    for (int64_t r = 0; r < h->nb; ++r)
      for (int e = grp[r]; e < grp[r + 1]; ++e) {
        const int p = fill[gci[e]]++;
        h->gtci[p] = (int)r;
        h->gtv[p] = gv[e];
      }
  }
  return h;
}

template <typename T>
static void upload_vals(Ctx* ctx, const std::vector<double>& v, DBuf<uint8_t>& dst) {
  std::vector<T> t(v.begin(), v.end());
  dst.resize(ctx, std::max<size_t>(t.size(), 1) * sizeof(T));
  if (!t.empty()) h2d(ctx, dst.get(), t.data(), t.size() * sizeof(T));
}

static void upload_ints(Ctx* ctx, const std::vector<int>& v, DBuf<int>& dst) {
  dst.resize(ctx, std::max<size_t>(v.size(), 1));
  if (!v.empty()) h2d(ctx, dst.get(), v.data(), v.size() * sizeof(int));
}

void rb_attach(Ctx* ctx, const std::shared_ptr<RbHost>& h, Prec prec, SellOp& op) {
  if (!h || op.dense) return;
  auto rb = std::make_shared<RbOp>();
  rb->d = h->d;
  rb->nr = h->nr;
  rb->nb = h->nb;
  upload_ints(ctx, h->red, rb->red);
  upload_ints(ctx, h->blk, rb->blk);
  upload_ints(ctx, h->frp, rb->frp);
  upload_ints(ctx, h->fci, rb->fci);
  upload_ints(ctx, h->erp, rb->erp);
  upload_ints(ctx, h->eci, rb->eci);
  if (prec == Prec::F64) {
    upload_vals<double>(ctx, h->fv, rb->fval);
    upload_vals<double>(ctx, h->ev, rb->eval);
  } else {
    upload_vals<float>(ctx, h->fv, rb->fval);
    upload_vals<float>(ctx, h->ev, rb->eval);
  }
  DBuf<int> grp, gci;
  upload_ints(ctx, h->gtrp, grp);
  upload_ints(ctx, h->gtci, gci);
  DBuf<double> gv(ctx, std::max<size_t>(h->gtv.size(), 1));
  if (!h->gtv.empty()) h2d(ctx, gv.get(), h->gtv.data(), h->gtv.size() * sizeof(double));
  care_csr g;
  g.n = h->nb;
  g.nnz = (int64_t)h->gtci.size();
  g.row_ptr = grp.get();
  g.col_idx = gci.get();
  g.val = gv.get();
  build_sell(ctx, &g, prec, rb->G);
  // the preconditioned GMRES solves run on the reduced system: ILU(0) of G + p' I
  if (ctx->krylov_precond && ctx->krylov_method == 1) ilu_attach(ctx, ilu_analyse(ctx, &g), rb->G);
  ctx->sync();
  op.rb = rb;
}

// bh[:, c] = F b_r - (d + p) b_b over the black rows (complex: interleaved
// (re, im) column pairs, g = d + p complex)
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) k_rb_rhs(int64_t nb, int nlog, const int* __restrict__ frp,
                                                const int* __restrict__ fci, const T* __restrict__ fv,
                                                const int* __restrict__ blk, const T* __restrict__ b, int64_t ldb,
                                                T* __restrict__ bh, int64_t ldh, double gr, double gi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= nb || c >= nlog) return;
  const int cr = CPLX ? 2 * c : c;
  const T* br = b + (int64_t)cr * ldb;
  T sr = (T)0, si = (T)0;
  for (int e = frp[i]; e < frp[i + 1]; ++e) {
    const int j = fci[e];
    sr += fv[e] * br[j];
    if (CPLX) si += fv[e] * br[j + ldb];
  }
  const int ib = blk[i];
  const T xr = br[ib], xi = CPLX ? br[ib + ldb] : (T)0;
  bh[(int64_t)cr * ldh + i] = sr - ((T)gr * xr - (T)gi * xi);
  if (CPLX) bh[(int64_t)(cr + 1) * ldh + i] = si - ((T)gr * xi + (T)gi * xr);
}

// x_r = (b_r - E x_b) / (d + p) over the red rows, x_b scattered to the black
// rows (grid rows: nr red rows then nb black rows)
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) k_rb_back(int64_t nr, int64_t nb, int nlog, const int* __restrict__ erp,
                                                 const int* __restrict__ eci, const T* __restrict__ ev,
                                                 const int* __restrict__ red, const int* __restrict__ blk,
                                                 const T* __restrict__ b, int64_t ldb, const T* __restrict__ xh,
                                                 int64_t ldh, T* __restrict__ x, int64_t ldx, double qr, double qi) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= nr + nb || c >= nlog) return;
  const int cr = CPLX ? 2 * c : c;
  const T* xhr = xh + (int64_t)cr * ldh;
  T* xr = x + (int64_t)cr * ldx;
  if (r >= nr) {
    const int64_t i = r - nr;
    xr[blk[i]] = xhr[i];
    if (CPLX) xr[blk[i] + ldx] = xhr[i + ldh];
    return;
  }
  const T* brc = b + (int64_t)cr * ldb;
  const int j = red[r];
  T sr = brc[j], si = CPLX ? brc[j + ldb] : (T)0;
  for (int e = erp[r]; e < erp[r + 1]; ++e) {
    const int k = eci[e];
    sr -= ev[e] * xhr[k];
    if (CPLX) si -= ev[e] * xhr[k + ldh];
  }
  // times q = 1 / (d + p)
  xr[j] = (T)qr * sr - (T)qi * si;
  if (CPLX) xr[j + ldx] = (T)qr * si + (T)qi * sr;
}

template <typename T>
KrylovResult bicgstab_rb(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols, const T* b, int64_t ldb, T* x,
                         int64_t ldx, double tol, int maxit, int check_every, const std::vector<int>* groups) {
  const RbOp& rb = *op.rb;
  const bool cplx = pi != 0.0;
  const double gr = rb.d + pr, gi = pi;              // g = d + p
  const double g2 = gr * gr + gi * gi;
  const double spr = -(gr * gr - gi * gi), spi = -2.0 * gr * gi;   // p' = -g^2
  const int nlog = cplx ? ncols / 2 : ncols;
  const int64_t ldh = pad_ld(rb.nb);
  DBuf<T> bh(ctx, (size_t)ldh * ncols), xh(ctx, (size_t)ldh * ncols);
  if (nlog > 0) {
    const dim3 g1(ceil_div(rb.nb, 256), nlog);
    if (cplx)
      hipLaunchKernelGGL((k_rb_rhs<T, true>), g1, dim3(256), 0, ctx->stream, rb.nb, nlog, rb.frp.get(), rb.fci.get(),
                         (const T*)rb.fval.get(), rb.blk.get(), b, ldb, bh.get(), ldh, gr, gi);
    else
      hipLaunchKernelGGL((k_rb_rhs<T, false>), g1, dim3(256), 0, ctx->stream, rb.nb, nlog, rb.frp.get(), rb.fci.get(),
                         (const T*)rb.fval.get(), rb.blk.get(), b, ldb, bh.get(), ldh, gr, gi);
    KERNEL_CHECK();
  }
  KrylovResult kr = bicgstab<T>(ctx, rb.G, spr, spi, ncols, bh.get(), ldh, xh.get(), ldh, tol, maxit, check_every,
                                groups);
  if (nlog > 0) {
    const double qr = gr / g2, qi = -gi / g2;        // 1 / g
    const dim3 g2d(ceil_div(rb.nr + rb.nb, 256), nlog);
    if (cplx)
      hipLaunchKernelGGL((k_rb_back<T, true>), g2d, dim3(256), 0, ctx->stream, rb.nr, rb.nb, nlog, rb.erp.get(),
                         rb.eci.get(), (const T*)rb.eval.get(), rb.red.get(), rb.blk.get(), b, ldb, xh.get(), ldh, x,
                         ldx, qr, qi);
    else
      hipLaunchKernelGGL((k_rb_back<T, false>), g2d, dim3(256), 0, ctx->stream, rb.nr, rb.nb, nlog, rb.erp.get(),
                         rb.eci.get(), (const T*)rb.eval.get(), rb.red.get(), rb.blk.get(), b, ldb, xh.get(), ldh, x,
                         ldx, qr, qi);
    KERNEL_CHECK();
  }
  return kr;
}

// whether a shifted solve can take the reduction: the scaling d + p must be
// nonzero, and a complex shift must stay complex after the reduction (the
// reduced system's right-hand side is complex)
bool rb_usable(const SellOp& op, double pr, double pi) {
  if (!op.rb || op.dense) return false;
  const double gr = op.rb->d + pr, gi = pi;
  if (gr == 0.0 && gi == 0.0) return false;
  if (pi != 0.0 && gr * gi == 0.0) return false;
  return true;
}

template KrylovResult bicgstab_rb<double>(Ctx*, const SellOp&, double, double, int, const double*, int64_t, double*,
                                          int64_t, double, int, int, const std::vector<int>*);
template KrylovResult bicgstab_rb<float>(Ctx*, const SellOp&, double, double, int, const float*, int64_t, float*,
                                         int64_t, double, int, int, const std::vector<int>*);

}  // namespace mpcare
