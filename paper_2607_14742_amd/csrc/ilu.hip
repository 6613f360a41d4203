// ILU(0) of the shifted matrices M = A^T + p I in a multicolour order: the
// preconditioner of the restarted-GMRES inner solves of Sec. 5 ("Performance
// Analysis on GPU"), where the factorisation and the triangular solves run on
// the GPU.
//
// Ordering.  The unknowns are coloured first-fit in their natural order over
// the undirected graph of the off-diagonal entries of A (host analysis of the
// pattern, once per matrix): row i takes the smallest colour that none of its
// already coloured neighbours holds.  Rows of one colour are never coupled,
// so in the order "colour 0, colour 1, ..." (natural order inside a colour)
// the diagonal blocks of M are diagonal and every colour is one parallel step
// of the factorisation and of each triangular solve.  Five- and seven-point
// stencils take two colours (red-black), the band of the Toeplitz example four.
//
// Storage.  The factors live at the positions of the operator's SELL-64
// layout of A^T (same column indices, one value array per shift in the vector
// precision): an entry (i, j) holds l_ij when j's colour is below i's and
// u_ij when it is above; the pivots are kept apart as 1 / u_ii.
//
// Factorisation (one launch per colour, one thread per row, rows of lower
// colours final): row i starts from its row of M; for each lower neighbour k
// in increasing (colour, index) order the multiplier l_ik = m_ik / u_kk is
// formed and m_ij -= l_ik u_kj for every later position j of row i that row
// k's U part holds (the diagonal included); fill outside the pattern is never
// formed.  This is the IKJ form of ILU(0) in the multicolour order.
//
// Solve z = (L U)^{-1} x, one launch per colour and sweep: forward over
// colours 1 .. C-1 (y = x on colour 0), the last colour fused with its
// backward step, then backward over colours C-2 .. 0.  2C - 2 launches (one
// for C = 1), each a gather over the row's entries for a group of columns.
#include <algorithm>
#include <cmath>

#include "krylov.hpp"

namespace mpcare {

struct IluHost {
  int64_t n = 0;
  int ncol = 0;
  std::vector<int> colour;   // per row
  std::vector<int> rows;     // rows grouped by colour, increasing index inside a colour
  std::vector<int> coff;     // colour c holds rows[coff[c] .. coff[c + 1])
};

namespace {

constexpr int ILU_MAX_COLOURS = 1024;
constexpr int ILU_NT = 256;
constexpr int ILU_KC = 8;            // right-hand-side columns per thread in the solves
constexpr size_t ILU_CACHE = 64;     // factorisations kept per operator

// One colour of the factorisation: thread t factors row rows[t].
template <typename TV, typename T>
__global__ void __launch_bounds__(ILU_NT) k_ilu_factor(int cnt, const int* __restrict__ rows, int c, int64_t n,
                                                       const int* __restrict__ sptr, const int* __restrict__ cols,
                                                       const TV* __restrict__ vals, float vscale,
                                                       const T* __restrict__ diag, T shift,
                                                       const int* __restrict__ colour, T* off, T* dinv,
                                                       int* __restrict__ bad) {
  const int t = blockIdx.x * ILU_NT + threadIdx.x;
  if (t >= cnt) return;
  const int i = rows[t];
  const int l = i & 63;
  const int b = sptr[i >> 6], w = sptr[(i >> 6) + 1] - b;
  for (int q = 0; q < w; ++q) {
    const int64_t e = (int64_t)(b + q) * 64 + l;
    off[e] = load_entry<T, TV>(vals, e, vscale);
  }
  T dg = diag[i] + shift;
  int64_t last = -1;
  for (;;) {
    // the next lower neighbour in (colour, index) order
    int64_t best = INT64_MAX;
    int64_t ebest = -1;
    for (int q = 0; q < w; ++q) {
      const int64_t e = (int64_t)(b + q) * 64 + l;
      const int j = cols[e];
      if (j == i) continue;                     // padding
      const int cj = colour[j];
      if (cj >= c) continue;
      const int64_t key = (int64_t)cj * n + j;
      if (key > last && key < best) {
        best = key;
        ebest = e;
      }
    }
    if (ebest < 0) break;
    last = best;
    const int k = cols[ebest];
    const T lik = off[ebest] * dinv[k];
    off[ebest] = lik;
    const int lk = k & 63;
    const int bk = sptr[k >> 6], wk = sptr[(k >> 6) + 1] - bk;
    const int ck = colour[k];
    for (int q = 0; q < wk; ++q) {
      const int64_t ek = (int64_t)(bk + q) * 64 + lk;
      const int j = cols[ek];
      if (j == k || colour[j] <= ck) continue;  // padding, or not in row k's U part
      const T ukj = off[ek];
      if (j == i) {
        dg -= lik * ukj;
        continue;
      }
      for (int r = 0; r < w; ++r) {
        const int64_t e = (int64_t)(b + r) * 64 + l;
        if (cols[e] == j) {
          off[e] -= lik * ukj;
          break;
        }
      }
    }
  }
  if (!(dg != T(0)) || !isfinite((double)dg)) atomicMax(bad, 1);
  dinv[i] = T(1) / dg;
}

// Forward step of colour c >= 1: y_i = x_i - sum_{colour(j) < c} l_ij y_j with
// y = x on colour 0 and y = Z elsewhere; the last colour also divides by u_ii.
template <typename T>
__global__ void __launch_bounds__(ILU_NT) k_ilu_fwd(int cnt, const int* __restrict__ rows, int c, bool last,
                                                    const int* __restrict__ sptr, const int* __restrict__ cols,
                                                    const T* __restrict__ off, const T* __restrict__ dinv,
                                                    const int* __restrict__ colour, int k, const T* __restrict__ X,
                                                    int64_t ldx, T* Z, int64_t ldz) {
  const int t = blockIdx.x * ILU_NT + threadIdx.x;
  if (t >= cnt) return;
  const int c0 = blockIdx.y * ILU_KC, kc = min(ILU_KC, k - c0);
  const int i = rows[t];
  const int l = i & 63;
  const int b = sptr[i >> 6], w = sptr[(i >> 6) + 1] - b;
  T acc[ILU_KC];
#pragma unroll
  for (int q = 0; q < ILU_KC; ++q) acc[q] = q < kc ? X[(int64_t)(c0 + q) * ldx + i] : T(0);
  for (int r = 0; r < w; ++r) {
    const int64_t e = (int64_t)(b + r) * 64 + l;
    const int j = cols[e];
    if (j == i) continue;
    const int cj = colour[j];
    if (cj >= c) continue;
    const T v = off[e];
    const T* src = cj == 0 ? X : Z;
    const int64_t ls = cj == 0 ? ldx : ldz;
#pragma unroll
    for (int q = 0; q < ILU_KC; ++q)
      if (q < kc) acc[q] -= v * src[(int64_t)(c0 + q) * ls + j];
  }
  const T s = last ? dinv[i] : T(1);
#pragma unroll
  for (int q = 0; q < ILU_KC; ++q)
    if (q < kc) Z[(int64_t)(c0 + q) * ldz + i] = acc[q] * s;
}

// Backward step of colour c: z_i = (y_i - sum_{colour(j) > c} u_ij z_j) / u_ii
// with y_i = x_i on colour 0 and Z_i elsewhere.
template <typename T>
__global__ void __launch_bounds__(ILU_NT) k_ilu_bwd(int cnt, const int* __restrict__ rows, int c,
                                                    const int* __restrict__ sptr, const int* __restrict__ cols,
                                                    const T* __restrict__ off, const T* __restrict__ dinv,
                                                    const int* __restrict__ colour, int k, const T* __restrict__ X,
                                                    int64_t ldx, T* Z, int64_t ldz) {
  const int t = blockIdx.x * ILU_NT + threadIdx.x;
  if (t >= cnt) return;
  const int c0 = blockIdx.y * ILU_KC, kc = min(ILU_KC, k - c0);
  const int i = rows[t];
  const int l = i & 63;
  const int b = sptr[i >> 6], w = sptr[(i >> 6) + 1] - b;
  const T* y = c == 0 ? X : Z;
  const int64_t ly = c == 0 ? ldx : ldz;
  T acc[ILU_KC];
#pragma unroll
  for (int q = 0; q < ILU_KC; ++q) acc[q] = q < kc ? y[(int64_t)(c0 + q) * ly + i] : T(0);
  for (int r = 0; r < w; ++r) {
    const int64_t e = (int64_t)(b + r) * 64 + l;
    const int j = cols[e];
    if (j == i || colour[j] <= c) continue;
    const T v = off[e];
#pragma unroll
    for (int q = 0; q < ILU_KC; ++q)
      if (q < kc) acc[q] -= v * Z[(int64_t)(c0 + q) * ldz + j];
  }
  const T s = dinv[i];
#pragma unroll
  for (int q = 0; q < ILU_KC; ++q)
    if (q < kc) Z[(int64_t)(c0 + q) * ldz + i] = acc[q] * s;
}

template <typename TV, typename T>
void factor_launch(Ctx* ctx, const SellOp& op, const IluOp& il, double p, IluOp::Factors& f, int* bad) {
  for (int c = 0; c < il.ncol; ++c) {
    const int cnt = il.coff[c + 1] - il.coff[c];
    if (cnt == 0) continue;
    hipLaunchKernelGGL((k_ilu_factor<TV, T>), dim3(ceil_div(cnt, ILU_NT)), dim3(ILU_NT), 0, ctx->stream, cnt,
                       il.rows.get() + il.coff[c], c, op.n, op.sptr.get(), op.cols.get(),
                       (const TV*)op.vals.get(), op.val_scale, (const T*)op.diag.get(), (T)p, il.colour.get(),
                       (T*)f.off.get(), (T*)f.dinv.get(), bad);
    KERNEL_CHECK();
  }
}

}  // namespace

int ilu_colour_host(int64_t n, int64_t nnz, const int* rp, const int* ci, std::vector<int>& colour) {
  if (n < 1 || nnz < 0 || !rp || (nnz > 0 && !ci)) fail(CARE_ERR_ARG, "invalid CSR pattern");
  if (rp[0] != 0 || rp[n] != nnz) fail(CARE_ERR_ARG, "CSR row_ptr must start at 0 and end at nnz");
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) fail(CARE_ERR_ARG, "CSR row_ptr is not monotone");
  for (int64_t e = 0; e < nnz; ++e)
    if (ci[e] < 0 || ci[e] >= n) fail(CARE_ERR_ARG, "CSR column index out of range");
  // rows of A^T (the other direction of each edge)
  std::vector<int> tp(n + 1, 0), tc(std::max<int64_t>(nnz, 1));
  for (int64_t e = 0; e < nnz; ++e) tp[ci[e] + 1] += 1;
  for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
  {
    std::vector<int> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int e = rp[i]; e < rp[i + 1]; ++e) tc[fill[ci[e]]++] = (int)i;
  }
  colour.assign(n, -1);
  std::vector<int64_t> stamp(ILU_MAX_COLOURS + 1, -1);
  int ncol = 0;
  for (int64_t i = 0; i < n; ++i) {
    auto mark = [&](int j) {
      if (j != i && colour[j] >= 0) stamp[colour[j]] = i;
    };
    for (int e = rp[i]; e < rp[i + 1]; ++e) mark(ci[e]);
    for (int e = tp[i]; e < tp[i + 1]; ++e) mark(tc[e]);
    int c = 0;
    while (stamp[c] == i) ++c;
    if (c >= ILU_MAX_COLOURS)
      fail(CARE_ERR_NOT_IMPLEMENTED, "ILU(0): the pattern needs more than 1024 colours");
    colour[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

std::shared_ptr<IluHost> ilu_analyse(Ctx* ctx, const care_csr* A) {
  if (!A || A->n < 1) return nullptr;
  const int64_t n = A->n, nnz = A->nnz;
  std::vector<int> rp(n + 1), ci(std::max<int64_t>(nnz, 1));
  d2h(ctx, rp.data(), A->row_ptr, (n + 1) * sizeof(int));
  if (nnz) d2h(ctx, ci.data(), A->col_idx, nnz * sizeof(int));
  auto h = std::make_shared<IluHost>();
  h->n = n;
  const int ncol = ilu_colour_host(n, nnz, rp.data(), ci.data(), h->colour);
  h->ncol = ncol;
  h->coff.assign(ncol + 1, 0);
  for (int64_t i = 0; i < n; ++i) h->coff[h->colour[i] + 1] += 1;
  for (int c = 0; c < ncol; ++c) h->coff[c + 1] += h->coff[c];
  h->rows.resize(n);
  {
    std::vector<int> fill(h->coff.begin(), h->coff.end() - 1);
    for (int64_t i = 0; i < n; ++i) h->rows[fill[h->colour[i]]++] = (int)i;
  }
  return h;
}

void ilu_attach(Ctx* ctx, const std::shared_ptr<IluHost>& h, SellOp& op) {
  if (!h || op.dense || h->n != op.n) return;
  auto il = std::make_shared<IluOp>();
  il->ncol = h->ncol;
  il->coff = h->coff;
  il->rows.resize(ctx, h->n);
  il->colour.resize(ctx, h->n);
  h2d(ctx, il->rows.get(), h->rows.data(), h->n * sizeof(int));
  h2d(ctx, il->colour.get(), h->colour.data(), h->n * sizeof(int));
  op.ilu = il;
}

std::shared_ptr<IluOp::Factors> ilu_factor(Ctx* ctx, const SellOp& op, double p) {
  if (!op.ilu) fail(CARE_ERR_ARG, "ILU(0) requested for an operator without its colouring");
  IluOp& il = *op.ilu;
  auto it = il.fac.find(p);
  if (it != il.fac.end()) return it->second;
  if (il.fac.size() >= ILU_CACHE) il.fac.clear();
  auto f = std::make_shared<IluOp::Factors>();
  const size_t vb = vec_bytes(op.prec);
  f->off.resize(ctx, std::max<size_t>((size_t)op.width_total * 64 * vb, vb));
  f->dinv.resize(ctx, (size_t)op.n * vb);
  DBuf<int> bad(ctx, 1);
  dzero(ctx, bad.get(), sizeof(int));
  switch (op.prec) {
    case Prec::F64: factor_launch<double, double>(ctx, op, il, p, *f, bad.get()); break;
    case Prec::F32: factor_launch<float, float>(ctx, op, il, p, *f, bad.get()); break;
    case Prec::BF16: factor_launch<bf16, float>(ctx, op, il, p, *f, bad.get()); break;
    case Prec::F16: factor_launch<f16, float>(ctx, op, il, p, *f, bad.get()); break;
  }
  int hb = 0;
  d2h(ctx, &hb, bad.get(), sizeof(int));
  if (hb) fail(CARE_ERR_BREAKDOWN, "ILU(0): zero or non-finite pivot");
  il.fac[p] = f;
  return f;
}

template <typename T>
void ilu_apply(Ctx* ctx, const SellOp& op, const IluOp::Factors& f, int k, const T* X, int64_t ldx, T* Z,
               int64_t ldz) {
  if (k <= 0) return;
  const IluOp& il = *op.ilu;
  const int C = il.ncol;
  const unsigned gy = ceil_div(k, ILU_KC);
  const T* off = (const T*)f.off.get();
  const T* dinv = (const T*)f.dinv.get();
  auto rows_of = [&](int c) { return il.coff[c + 1] - il.coff[c]; };
  for (int c = 1; c < C; ++c) {
    const int cnt = rows_of(c);
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_ilu_fwd<T>, dim3(ceil_div(cnt, ILU_NT), gy), dim3(ILU_NT), 0, ctx->stream, cnt,
                       il.rows.get() + il.coff[c], c, c == C - 1, op.sptr.get(), op.cols.get(), off, dinv,
                       il.colour.get(), k, X, ldx, Z, ldz);
    KERNEL_CHECK();
  }
  for (int c = C >= 2 ? C - 2 : 0; c >= 0; --c) {
    const int cnt = rows_of(c);
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_ilu_bwd<T>, dim3(ceil_div(cnt, ILU_NT), gy), dim3(ILU_NT), 0, ctx->stream, cnt,
                       il.rows.get() + il.coff[c], c, op.sptr.get(), op.cols.get(), off, dinv, il.colour.get(), k,
                       X, ldx, Z, ldz);
    KERNEL_CHECK();
  }
}

template void ilu_apply<double>(Ctx*, const SellOp&, const IluOp::Factors&, int, const double*, int64_t, double*,
                                int64_t);
template void ilu_apply<float>(Ctx*, const SellOp&, const IluOp::Factors&, int, const float*, int64_t, float*,
                               int64_t);

}  // namespace mpcare
