// Set-up of the sparse operator (CSR(A) -> SELL-64 of A^T, per precision)
// and the launcher of the sparse-product kernel template.
#include "sparse.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstdio>

#include <hip/hip_ext.h>
#include <hipcub/hipcub.hpp>

namespace mpcare {

// ---------------------------------------------------------------------------
// input validation (before any kernel indexes through the caller's arrays)
// ---------------------------------------------------------------------------
__global__ void k_check_rowptr(const int* __restrict__ rp, int64_t n, int64_t nnz, int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  const int v = rp[i];
  bool ok = v >= 0 && v <= nnz;
  if (i == 0) ok = ok && v == 0;
  if (i == n) ok = ok && v == nnz;
  if (i < n) ok = ok && rp[i + 1] >= v;
  if (!ok) atomicOr(bad, 1);
}

__global__ void k_check_cols(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
                             int64_t n, int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int prev = -1;
  int flag = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int c = ci[e];
    if (c < 0 || c >= n) flag |= 2;
    else if (c <= prev) flag |= 4;
    prev = c;
    const double v = val[e];
    if (!__builtin_isfinite(v)) flag |= 8;
  }
  if (flag) atomicOr(bad, flag);
}

// ---------------------------------------------------------------------------
// transpose CSR(A) -> CSR(A^T)
// ---------------------------------------------------------------------------
__global__ void k_count_cols(const int* __restrict__ ci, int64_t nnz, int* __restrict__ cnt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}

__global__ void k_scatter_t(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ val,
                            int64_t n, const int* __restrict__ rpt, int* __restrict__ fill,
                            int* __restrict__ ct, double* __restrict__ vt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int j = ci[e];
    const int pos = rpt[j] + atomicAdd(&fill[j], 1);
    ct[pos] = (int)i;
    vt[pos] = val[e];
  }
}

// sort each row of A^T by column index (insertion sort; rows are short)
__global__ void k_sort_rows(const int* __restrict__ rpt, int64_t n, int* __restrict__ ct, double* __restrict__ vt) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int b = rpt[j], e = rpt[j + 1];
  for (int u = b + 1; u < e; ++u) {
    const int c = ct[u];
    const double v = vt[u];
    int w = u - 1;
    while (w >= b && ct[w] > c) {
      ct[w + 1] = ct[w];
      vt[w + 1] = vt[w];
      --w;
    }
    ct[w + 1] = c;
    vt[w + 1] = v;
  }
}

// off-diagonal row length of A^T, padded to whole slices
__global__ void k_slice_width(const int* __restrict__ rpt, const int* __restrict__ ct, int64_t n, int nslices,
                              int* __restrict__ width) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int w = 0;
  for (int l = 0; l < 64; ++l) {
    const int64_t i = (int64_t)s * 64 + l;
    if (i >= n) break;
    int len = rpt[i + 1] - rpt[i];
    for (int e = rpt[i]; e < rpt[i + 1]; ++e)
      if (ct[e] == i) { --len; break; }
    w = len > w ? len : w;
  }
  width[s] = w;
}

template <typename TV, typename T>
__global__ void k_fill_sell(const int* __restrict__ rpt, const int* __restrict__ ct, const double* __restrict__ vt,
                            int64_t n, int nslices, const int* __restrict__ sptr, int* __restrict__ cols,
                            TV* __restrict__ vals, T* __restrict__ diag, double inv_scale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nslices * 64) return;
  const int s = (int)(i >> 6), lane = (int)(i & 63);
  const int base = sptr[s], w = sptr[s + 1] - base;
  int t = 0;
  double d = 0.0;
  const int self = (int)(i < n ? i : n - 1);
  if (i < n) {
    for (int e = rpt[i]; e < rpt[i + 1]; ++e) {
      if (ct[e] == i) {
        d = vt[e];
      } else {
        const int64_t o = (int64_t)(base + t) * 64 + lane;
        cols[o] = ct[e];
        vals[o] = (TV)(vt[e] * inv_scale);
        ++t;
      }
    }
    diag[i] = (T)d;
  }
  for (; t < w; ++t) {
    const int64_t o = (int64_t)(base + t) * 64 + lane;
    cols[o] = self;
    vals[o] = (TV)0.0;
  }
}

__global__ void k_sumsq(const double* __restrict__ v, int64_t n, double* __restrict__ part) {
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    s += v[e] * v[e];
  double vv[1] = {s};
  block_reduce_to<1>(vv, [&](int, double val) { part[blockIdx.x] = val; });
}

// largest absolute row sum, one partial maximum per block (blockDim 256)
__global__ void __launch_bounds__(256) k_rowabs_max(const int32_t* __restrict__ rp, const double* __restrict__ val,
                                                    int64_t n, double* __restrict__ part) {
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) s += fabs(val[e]);
    mx = fmax(mx, s);
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <typename T>
static void exclusive_scan(Ctx* ctx, const T* in, T* out, int64_t count) {
  size_t tmp = 0;
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, (int)count, ctx->stream));
  DBuf<uint8_t> t(ctx, tmp + 16);
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(t.get(), tmp, in, out, (int)count, ctx->stream));
}

void build_sell(Ctx* ctx, const care_csr* A, Prec prec, SellOp& op) {
  if (!A) fail(CARE_ERR_ARG, "A is NULL");
  const int64_t n = A->n, nnz = A->nnz;
  if (n < 1 || n >= (int64_t(1) << 31) / 2) fail(CARE_ERR_ARG, "n out of range");
  if (nnz < 0 || nnz >= (int64_t(1) << 31)) fail(CARE_ERR_ARG, "nnz out of range");
  if (!A->row_ptr || (nnz > 0 && (!A->col_idx || !A->val))) fail(CARE_ERR_ARG, "CSR pointer is NULL");
  hipStream_t st = ctx->stream;

  DBuf<int> flag(ctx, 1);
  dzero(ctx, flag.get(), sizeof(int));
  hipLaunchKernelGGL(k_check_rowptr, dim3(ceil_div(n + 1, 256)), dim3(256), 0, st, A->row_ptr, n, nnz, flag.get());
  KERNEL_CHECK();
  int bad = 0;
  d2h(ctx, &bad, flag.get(), sizeof(int));
  if (bad) fail(CARE_ERR_ARG, "CSR row_ptr is not a valid monotone offset array");
  if (nnz > 0) {
    hipLaunchKernelGGL(k_check_cols, dim3(ceil_div(n, 256)), dim3(256), 0, st, A->row_ptr, A->col_idx, A->val, n,
                       flag.get());
    KERNEL_CHECK();
    d2h(ctx, &bad, flag.get(), sizeof(int));
    if (bad & 2) fail(CARE_ERR_ARG, "CSR column index out of range");
    if (bad & 4) fail(CARE_ERR_ARG, "CSR column indices not strictly increasing within a row");
    if (bad & 8) fail(CARE_ERR_NONFINITE, "A has a NaN or Inf value");
  }

  // transpose
  DBuf<int> cnt(ctx, n + 1), rpt(ctx, n + 1), fill(ctx, n);
  DBuf<int> ct(ctx, nnz ? nnz : 1);
  DBuf<double> vt(ctx, nnz ? nnz : 1);
  dzero(ctx, cnt.get(), (n + 1) * sizeof(int));
  dzero(ctx, fill.get(), n * sizeof(int));
  if (nnz) {
    hipLaunchKernelGGL(k_count_cols, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, A->col_idx, nnz, cnt.get());
    KERNEL_CHECK();
  }
  exclusive_scan(ctx, cnt.get(), rpt.get(), n + 1);
  hipLaunchKernelGGL(k_scatter_t, dim3(ceil_div(n, 256)), dim3(256), 0, st, A->row_ptr, A->col_idx, A->val, n,
                     rpt.get(), fill.get(), ct.get(), vt.get());
  KERNEL_CHECK();
  hipLaunchKernelGGL(k_sort_rows, dim3(ceil_div(n, 256)), dim3(256), 0, st, rpt.get(), n, ct.get(), vt.get());
  KERNEL_CHECK();

  // slice widths and offsets
  const int nsl = (int)((n + 63) / 64);
  DBuf<int> width(ctx, nsl + 1);
  dzero(ctx, width.get(), (nsl + 1) * sizeof(int));
  hipLaunchKernelGGL(k_slice_width, dim3(ceil_div(nsl, 256)), dim3(256), 0, st, rpt.get(), ct.get(), n, nsl,
                     width.get());
  KERNEL_CHECK();
  op.sptr.resize(ctx, nsl + 1);
  exclusive_scan(ctx, width.get(), op.sptr.get(), nsl + 1);
  int total = 0;
  d2h(ctx, &total, op.sptr.get() + nsl, sizeof(int));
  {
    std::vector<int> hw(nsl);
    d2h(ctx, hw.data(), width.get(), nsl * sizeof(int));
    op.max_width = nsl ? *std::max_element(hw.begin(), hw.end()) : 0;
  }

  // ||A||_F
  if (nnz) {
    const int nb = 256;
    DBuf<double> part(ctx, nb);
    hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(256), 0, st, A->val, nnz, part.get());
    KERNEL_CHECK();
    std::vector<double> h(nb);
    d2h(ctx, h.data(), part.get(), nb * sizeof(double));
    double s = 0;
    for (double v : h) s += v;
    op.frob = std::sqrt(s);
    // ||A||_inf from the rows of A (row_ptr was validated above), ||A||_1
    // from the rows of the transpose built above
    hipLaunchKernelGGL(k_rowabs_max, dim3(nb), dim3(256), 0, st, A->row_ptr, A->val, n, part.get());
    KERNEL_CHECK();
    d2h(ctx, h.data(), part.get(), nb * sizeof(double));
    op.norm_inf = *std::max_element(h.begin(), h.end());
    hipLaunchKernelGGL(k_rowabs_max, dim3(nb), dim3(256), 0, st, (const int32_t*)rpt.get(), vt.get(), n, part.get());
    KERNEL_CHECK();
    d2h(ctx, h.data(), part.get(), nb * sizeof(double));
    op.norm_one = *std::max_element(h.begin(), h.end());
  }
  // F16 values: a power-of-two scale that maps max |a_ij| <= min(||A||_1,
  // ||A||_inf) into [2^13, 2^14], within half precision's range (65504);
  // entries below 2^-38 max |a_ij| fall to zero
  op.val_scale = 1.0f;
  if (prec == Prec::F16 && nnz) {
    const double bound = std::min(op.norm_inf, op.norm_one);
    if (bound > 0.0) op.val_scale = std::ldexp(1.0f, (int)std::ceil(std::log2(bound)) - 14);
  }
  op.n = n;
  op.nnz = nnz;
  op.nslices = nsl;
  op.width_total = total;
  op.prec = prec;
  const int64_t ents = (int64_t)total * 64;
  op.cols.resize(ctx, ents ? ents : 1);
  op.vals.resize(ctx, (ents ? ents : 1) * val_bytes(prec));
  op.diag.resize(ctx, n * vec_bytes(prec));
  dim3 g(ceil_div((int64_t)nsl * 64, 256));
  if (prec == Prec::F64) {
    hipLaunchKernelGGL((k_fill_sell<double, double>), g, dim3(256), 0, st, rpt.get(), ct.get(), vt.get(), n, nsl,
                       op.sptr.get(), op.cols.get(), (double*)op.vals.get(), (double*)op.diag.get(), 1.0);
  } else if (prec == Prec::F32) {
    hipLaunchKernelGGL((k_fill_sell<float, float>), g, dim3(256), 0, st, rpt.get(), ct.get(), vt.get(), n, nsl,
                       op.sptr.get(), op.cols.get(), (float*)op.vals.get(), (float*)op.diag.get(), 1.0);
  } else if (prec == Prec::BF16) {
    hipLaunchKernelGGL((k_fill_sell<bf16, float>), g, dim3(256), 0, st, rpt.get(), ct.get(), vt.get(), n, nsl,
                       op.sptr.get(), op.cols.get(), (bf16*)op.vals.get(), (float*)op.diag.get(), 1.0);
  } else {
    hipLaunchKernelGGL((k_fill_sell<f16, float>), g, dim3(256), 0, st, rpt.get(), ct.get(), vt.get(), n, nsl,
                       op.sptr.get(), op.cols.get(), (f16*)op.vals.get(), (float*)op.diag.get(),
                       1.0 / (double)op.val_scale);
  }
  KERNEL_CHECK();

  ctx->sync();
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
// Launch target of the sparse products: the stream and, in profile mode, the
// events the kernel records at its own start and end (hipExtLaunchKernelGGL:
// the timestamps are the kernel's, without the gaps between launches).
struct LaunchAt {
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

template <typename K, typename T>
static void launch_one(K kernel, const LaunchAt& at, dim3 g, const SpmmArgs<T>& a) {
  if (at.e0) hipExtLaunchKernelGGL(kernel, g, dim3(256), 0, at.st, at.e0, at.e1, 0, a);
  else hipLaunchKernelGGL(kernel, g, dim3(256), 0, at.st, a);
}

template <typename TV, typename T, int CP, bool CPLX, int WMAX>
static void launch_mode(const LaunchAt& at, dim3 g, int mode, const SpmmArgs<T>& a) {
  if (mode == MODE_PLAIN) launch_one(k_spmm<TV, T, CP, MODE_PLAIN, CPLX, WMAX>, at, g, a);
  else if (mode == MODE_DOT1) launch_one(k_spmm<TV, T, CP, MODE_DOT1, CPLX, WMAX>, at, g, a);
  else if (mode == MODE_DOT2) launch_one(k_spmm<TV, T, CP, MODE_DOT2, CPLX, WMAX>, at, g, a);
  // the fused BiCGStab modes stream their entries (one panel per workgroup)
  else if (mode == MODE_BICG_P) launch_one(k_spmm<TV, T, CP, MODE_BICG_P, CPLX, 0>, at, g, a);
  else launch_one(k_spmm<TV, T, CP, MODE_BICG_S, CPLX, 0>, at, g, a);
}

// Row-width class: rows of at most 4 entries are preloaded at every panel
// width; rows of at most 8 only for panels of at most 4 columns, since wider
// panels then hold 8 x panel gathers in flight per thread and the register
// cost (one or two waves per SIMD) outweighs the shorter load chain.
template <typename TV, typename T, int CP, bool CPLX>
static void launch_w(const LaunchAt& at, dim3 g, int mode, int wmax, const SpmmArgs<T>& a) {
  if (wmax == 4) launch_mode<TV, T, CP, CPLX, 4>(at, g, mode, a);
  else if (wmax == 8 && CP <= 4) launch_mode<TV, T, CP, CPLX, (CP <= 4 ? 8 : 0)>(at, g, mode, a);
  else launch_mode<TV, T, CP, CPLX, 0>(at, g, mode, a);
}

template <typename TV, typename T, int CP>
static void launch_cp(const LaunchAt& at, dim3 g, int mode, bool cplx, int wmax, const SpmmArgs<T>& a) {
  if constexpr (CP >= 2) {
    if (cplx) {
      launch_w<TV, T, CP, true>(at, g, mode, wmax, a);
      return;
    }
  }
  launch_w<TV, T, CP, false>(at, g, mode, wmax, a);
}

static int default_cp(int k, bool cplx) {
  int cp = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
  if (cplx && cp < 2) cp = 2;
  return cp;
}

// Panels per workgroup: one where few row blocks exist (the grid needs the
// panels for parallelism), else as many as keep about 1024 workgroups, in
// groups of equal size; the fused modes keep one panel per workgroup.
static int panels_per_block(int64_t nrb, int panels, int mode, int force) {
  if (mode == MODE_BICG_P || mode == MODE_BICG_S || panels <= 1) return 1;
  if (force > 0) return std::min(force, panels);
  const int target = (int)std::max<int64_t>(1, std::min<int64_t>(panels, nrb * panels / 1024));
  const int groups = (panels + target - 1) / target;
  return (panels + groups - 1) / groups;
}

template <typename TV, typename T>
static void launch_tv(const LaunchAt& at, int64_t n, int mode, bool cplx, SpmmArgs<T> a, int cp, int wmax,
                      int force_pg) {
  const int k = a.ncols;
  const int panels = ceil_div(k, cp);
  a.pg = panels_per_block(spmm_rowblocks(n), panels, mode, force_pg);
  dim3 g(spmm_rowblocks(n), ceil_div(panels, a.pg));
  switch (cp) {
    case 1: launch_cp<TV, T, 1>(at, g, mode, cplx, wmax, a); break;
    case 2: launch_cp<TV, T, 2>(at, g, mode, cplx, wmax, a); break;
    case 4: launch_cp<TV, T, 4>(at, g, mode, cplx, wmax, a); break;
    case 8: launch_cp<TV, T, 8>(at, g, mode, cplx, wmax, a); break;
    default: launch_cp<TV, T, 16>(at, g, mode, cplx, wmax, a); break;
  }
}

template <typename T>
static void launch_prec(Ctx* ctx, const SellOp& op, int mode, bool cplx, const SpmmArgs<T>& a, int cp, int pg = 0) {
  const int wmax = op.max_width <= 4 ? 4 : (op.max_width <= 8 ? 8 : 0);
  const int fpg = ctx->spmm_force_pg > 0 ? ctx->spmm_force_pg : pg;
  LaunchAt at;
  at.st = ctx->stream;
  at.e0 = ctx->spmm_ev0;
  at.e1 = ctx->spmm_ev1;
  if constexpr (sizeof(T) == 8) {
    if (op.prec != Prec::F64) fail(CARE_ERR_ARG, "FP64 vectors need the FP64 operator");
    launch_tv<double, double>(at, op.n, mode, cplx, a, cp, wmax, fpg);
  } else {
    if (op.prec == Prec::F32) launch_tv<float, float>(at, op.n, mode, cplx, a, cp, wmax, fpg);
    else if (op.prec == Prec::BF16) launch_tv<bf16, float>(at, op.n, mode, cplx, a, cp, wmax, fpg);
    else launch_tv<f16, float>(at, op.n, mode, cplx, a, cp, wmax, fpg);
  }
  KERNEL_CHECK();
}

// Autotuner of the product's tile: panel width and panels per workgroup.  A
// product of k > 8 columns runs in panels of 16 or of 8 columns, and a
// workgroup runs one panel or a group of them over its row slice (the
// matrix entries loaded once for the group).  Wider panels and larger groups
// read the matrix fewer times; narrower panels keep fewer gathers in flight
// per thread, and single panels give the grid more workgroups.  Which wins
// depends on the matrix, the precision and k.  The first launch of a shape
// (operator, precision, mode, real/complex, k rounded up to 16) runs each
// distinct candidate (16 or 8 columns; the default group or one panel per
// workgroup) twice with HIP events around each and keeps the fastest for that
// shape.  Only modes whose outputs every launch overwrites completely (plain
// product, split BiCGStab products) are tuned: the extra launches then leave
// the same results behind, since neither choice changes any column's
// arithmetic.  Launches inside a stream capture use the stored choice or the
// default.  Returns the panel width; *pg receives the panels per workgroup
// (0: the default rule).
template <typename T>
static int tuned_cp(Ctx* ctx, const SellOp& op, int mode, bool cplx, const SpmmArgs<T>& a, int* pg) {
  *pg = 0;
  const int k = a.ncols;
  const int cp0 = default_cp(k, cplx);
  if (cp0 == 16 && ctx->spmm_force_cp) return ctx->spmm_force_cp;
  if (!ctx->spmm_tune || cp0 != 16 || !(mode == MODE_PLAIN || mode == MODE_DOT1 || mode == MODE_DOT2)) return cp0;
  const int key = mode | (cplx ? 8 : 0) | (std::min((int)ceil_div(k, 16), 64) << 4) | (sizeof(T) == 8 ? 1 << 12 : 0);
  auto it = op.cp_choice.find(key);
  if (it != op.cp_choice.end()) {
    *pg = it->second >> 8;
    return it->second & 0xff;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_CHECK(hipStreamIsCapturing(ctx->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return cp0;
  // distinct candidates (cp, pg); pg = 0 is the default rule
  std::vector<std::pair<int, int>> cand;
  for (int cp : {16, 8}) {
    const int panels = ceil_div(k, cp);
    const int dflt = panels_per_block(spmm_rowblocks(op.n), panels, mode, 0);
    cand.push_back({cp, 0});
    if (dflt > 1) cand.push_back({cp, 1});
  }
  const int nc = (int)cand.size();
  std::vector<hipEvent_t> ev(2 * nc + 1);
  for (auto& e : ev) HIP_CHECK(hipEventCreate(&e));
  HIP_CHECK(hipEventRecord(ev[0], ctx->stream));
  for (int v = 0; v < 2 * nc; ++v) {
    launch_prec<T>(ctx, op, mode, cplx, a, cand[v % nc].first, cand[v % nc].second);
    HIP_CHECK(hipEventRecord(ev[v + 1], ctx->stream));
  }
  HIP_CHECK(hipEventSynchronize(ev[2 * nc]));
  std::vector<float> best(nc, INFINITY);
  for (int v = 0; v < 2 * nc; ++v) {
    float t = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&t, ev[v], ev[v + 1]));
    best[v % nc] = std::min(best[v % nc], t);
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  // the default (16 columns, default groups) unless another is 3 % faster
  int pick = 0;
  for (int c = 1; c < nc; ++c)
    if (best[c] < 0.97f * best[pick] && best[c] < best[0] * 0.97f) pick = c;
  const int cp = cand[pick].first;
  *pg = cand[pick].second;
  op.cp_choice[key] = cp | (*pg << 8);
  if (std::getenv("MPCARE_TRACE")) {
    std::fprintf(stderr, "[spmm-tune] n %lld mode %d cplx %d k %d fp%d:", (long long)op.n, mode, cplx ? 1 : 0, k,
                 (int)(8 * sizeof(T)));
    for (int c = 0; c < nc; ++c)
      std::fprintf(stderr, " %d cols/%s %.1f us", cand[c].first, cand[c].second ? "1 panel" : "default",
                   1e3f * best[c]);
    std::fprintf(stderr, " -> %d cols/%s\n", cp, *pg ? "1 panel" : "default");
  }
  return cp;
}

template <typename T>
int launch_spmm(Ctx* ctx, const SellOp& op, int mode, bool cplx, SpmmArgs<T>& a) {
  a.n = (int)op.n;
  a.sptr = op.sptr.get();
  a.cols = op.cols.get();
  a.vals = op.vals.get();
  a.diag = (const T*)op.diag.get();
  a.vscale = op.val_scale;
  a.nrb = spmm_rowblocks(op.n);
  if (a.ncols <= 0) return a.nrb;
  if (cplx && (a.ncols % 2)) fail(CARE_ERR_ARG, "complex panel with an odd number of real columns");
  int pg = 0;
  const int cp = tuned_cp<T>(ctx, op, mode, cplx, a, &pg);
  SpmmTimer timer(ctx, op, a.ncols, mode);
  launch_prec<T>(ctx, op, mode, cplx, a, cp, pg);
  return a.nrb;
}

template int launch_spmm<double>(Ctx*, const SellOp&, int, bool, SpmmArgs<double>&);
template int launch_spmm<float>(Ctx*, const SellOp&, int, bool, SpmmArgs<float>&);

SpmmTimer::SpmmTimer(Ctx* c, const SellOp& op, int k_real, int mode) : ctx(c) {
  ctx->spmm_calls += 1;
  if (ctx->spmm_defer && mode >= 0 && mode < 5) ctx->spmm_pending[mode] += 1;
  else ctx->spmm_bytes += op.bytes(k_real, spmm_vec_passes(mode));
  if (ctx->profile) {
    // recorded by the launch itself, at the kernel's start and end
    ev = ctx->event_pair();
    ctx->spmm_ev0 = ev.first;
    ctx->spmm_ev1 = ev.second;
  }
}

SpmmTimer::~SpmmTimer() {
  if (ctx->profile && ev.first) {
    ctx->spmm_ev0 = ctx->spmm_ev1 = nullptr;
    ctx->pending_events.push_back(ev);
  }
}

void spmm_plain(Ctx* ctx, const SellOp& op, double pr, double pi, const void* X, int64_t ldx, int k_real,
                void* Y, int64_t ldy) {
  if (op.dense) {
    dense_apply(ctx, op, pr, pi, X, ldx, k_real, Y, ldy);
    return;
  }
  const bool cplx = pi != 0.0;
  if (op.prec == Prec::F64) {
    SpmmArgs<double> a;
    a.ncols = k_real;
    a.sr = pr;
    a.si = pi;
    a.X = (const double*)X;
    a.ldx = ldx;
    a.Y = (double*)Y;
    a.ldy = ldy;
    launch_spmm<double>(ctx, op, MODE_PLAIN, cplx, a);
  } else {
    SpmmArgs<float> a;
    a.ncols = k_real;
    a.sr = pr;
    a.si = pi;
    a.X = (const float*)X;
    a.ldx = ldx;
    a.Y = (float*)Y;
    a.ldy = ldy;
    launch_spmm<float>(ctx, op, MODE_PLAIN, cplx, a);
  }
}

}  // namespace mpcare
