// Dense operator for the dense CARE instances: A^T stored as an n x n
// column-major matrix in the inner precision.  Products y = (A^T + p I) x
// are rocBLAS GEMMs (MFMA) plus a shift; shifted solves factor A^T + p I
// once per real shift with a partially pivoted LU in the inner precision and
// reuse the factors for every right-hand side block of every Newton step,
// since with the SMW form the base matrix does not change (Sec. 4).  Up to
// order LU_NMAX the factorisations of a whole shift set are one launch of the
// hand-written batched LU (lu.hip); its triangular-solve kernel serves orders
// up to LU_OWN_SOLVE_MAX and rocSOLVER getrs (on the same factors) larger
// ones; beyond LU_NMAX rocSOLVER getrf / getrs per shift.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.hpp"
#include "krylov.hpp"
#include "lu.hpp"

namespace mpcare {

template <typename T>
__global__ void k_add_diag(int64_t n, T* a, int64_t lda, T p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i * lda + i] += p;
}

// absolute column sums (one block per column) and row sums (one thread per
// row) of a column-major n x n matrix
__global__ void __launch_bounds__(256) k_abs_colsum(int64_t n, const double* __restrict__ a,
                                                    double* __restrict__ out) {
  const int64_t j = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += fabs(a[j * n + i]);
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sh[0];
}
__global__ void k_abs_rowsum(int64_t n, const double* __restrict__ a, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = 0; j < n; ++j) s += fabs(a[j * n + i]);
  out[i] = s;
}

void build_dense(Ctx* ctx, const double* A, int64_t lda, int64_t n, Prec prec, SellOp& op) {
  if (!A || n < 1 || lda < n) fail(CARE_ERR_ARG, "invalid dense A");
  if (n > 46340) fail(CARE_ERR_ARG, "dense A larger than 46340 x 46340");
  if (prec == Prec::BF16 || prec == Prec::F16)
    fail(CARE_ERR_NOT_IMPLEMENTED, "the 16-bit product variants apply to sparse operators only");
  op = SellOp();
  op.n = n;
  op.nnz = n * n;
  op.prec = prec;
  op.dense = true;
  DBuf<double> t(ctx, (size_t)n * n);
  const double one = 1.0, zero = 0.0;
  // A^T, leading dimension n
  ROCBLAS_CHECK(rocblas_dgeam(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, (int)n, (int)n, &one, A,
                              (int)lda, &zero, A, (int)lda, t.get(), (int)n));
  double nrm = 0.0;
  ROCBLAS_CHECK(rocblas_dnrm2(ctx->blas, (int)(n * n), t.get(), 1, &nrm));
  op.frob = nrm;
  if (!std::isfinite(nrm)) fail(CARE_ERR_NONFINITE, "A has non-finite entries");
  {
    // t = A^T: its column sums are the row sums of A and vice versa
    DBuf<double> sums(ctx, (size_t)n);
    std::vector<double> h((size_t)n);
    hipLaunchKernelGGL(k_abs_colsum, dim3((unsigned)n), dim3(256), 0, ctx->stream, n, (const double*)t.get(),
                       sums.get());
    KERNEL_CHECK();
    d2h(ctx, h.data(), sums.get(), (size_t)n * sizeof(double));
    op.norm_inf = *std::max_element(h.begin(), h.end());
    hipLaunchKernelGGL(k_abs_rowsum, dim3(ceil_div(n, 256)), dim3(256), 0, ctx->stream, n, (const double*)t.get(),
                       sums.get());
    KERNEL_CHECK();
    d2h(ctx, h.data(), sums.get(), (size_t)n * sizeof(double));
    op.norm_one = *std::max_element(h.begin(), h.end());
  }
  if (prec == Prec::F64) {
    op.dmat.resize(ctx, (size_t)n * n * sizeof(double));
    d2d(ctx, op.dmat.get(), t.get(), (size_t)n * n * sizeof(double));
  } else {
    op.dmat.resize(ctx, (size_t)n * n * sizeof(float));
    copy_cols<double, float>(ctx, n, (int)n, t.get(), n, (float*)op.dmat.get(), n);
  }
  ctx->sync();
}

void dense_apply(Ctx* ctx, const SellOp& op, double pr, double pi, const void* X, int64_t ldx, int k, void* Y,
                 int64_t ldy) {
  if (pi != 0.0) fail(CARE_ERR_NOT_IMPLEMENTED, "complex shifts with a dense operator");
  if (k <= 0) return;
  const int n = (int)op.n;
  if (op.prec == Prec::F64) {
    const double one = 1.0, zero = 0.0;
    ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, n, k, n, &one,
                                (const double*)op.dmat.get(), n, (const double*)X, (int)ldx, &zero, (double*)Y,
                                (int)ldy));
    if (pr != 0.0) axpby<double>(ctx, n, k, pr, (const double*)X, ldx, 1.0, (double*)Y, ldy);
  } else {
    const float one = 1.0f, zero = 0.0f;
    ROCBLAS_CHECK(rocblas_sgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, n, k, n, &one,
                                (const float*)op.dmat.get(), n, (const float*)X, (int)ldx, &zero, (float*)Y,
                                (int)ldy));
    if (pr != 0.0) axpby<float>(ctx, n, k, pr, (const float*)X, ldx, 1.0, (float*)Y, ldy);
  }
}

static rocblas_status getrf(rocblas_handle h, int n, double* a, int* ipiv, int* info) {
  return rocsolver_dgetrf(h, n, n, a, n, ipiv, info);
}
static rocblas_status getrf(rocblas_handle h, int n, float* a, int* ipiv, int* info) {
  return rocsolver_sgetrf(h, n, n, a, n, ipiv, info);
}
static rocblas_status getrf_batched(rocblas_handle h, int n, double* const a[], int* ipiv, int* info, int count) {
  return rocsolver_dgetrf_batched(h, n, n, a, n, ipiv, n, info, count);
}
static rocblas_status getrf_batched(rocblas_handle h, int n, float* const a[], int* ipiv, int* info, int count) {
  return rocsolver_sgetrf_batched(h, n, n, a, n, ipiv, n, info, count);
}

// From this order on the shift set is factored by rocSOLVER's batched getrf,
// which spreads each matrix over many compute units, instead of the
// one-workgroup-per-matrix kernel: measured 1.7x faster at n = 1024 and 3x at
// n = 2048 (16 FP32 shifts), slower below n = 512.
constexpr int LU_BATCHED_MIN = 1024;
static rocblas_status getrs(rocblas_handle h, int n, int k, double* a, const int* ipiv, double* x, int ldx) {
  return rocsolver_dgetrs(h, rocblas_operation_none, n, k, a, n, ipiv, x, ldx);
}
static rocblas_status getrs(rocblas_handle h, int n, int k, float* a, const int* ipiv, float* x, int ldx) {
  return rocsolver_sgetrs(h, rocblas_operation_none, n, k, a, n, ipiv, x, ldx);
}

// Factor A^T + p I for every listed real shift not factored yet: one launch
// of the hand-written batched LU for all of them below LU_BATCHED_MIN, else
// one call of rocSOLVER's batched getrf.
template <typename T>
static void factor_shifts(Ctx* ctx, const SellOp& op, const std::vector<double>& want) {
  const int n = (int)op.n;
  std::vector<double> todo;
  for (double p : want)
    if (op.lu.find(p) == op.lu.end() && std::find(todo.begin(), todo.end(), p) == todo.end()) todo.push_back(p);
  if (todo.empty()) return;
  if (n < LU_BATCHED_MIN && n <= LU_NMAX) {
    std::vector<std::shared_ptr<SellOp::DenseLU>> fs;
    std::vector<T*> F;
    std::vector<int*> P;
    std::vector<int*> I;
    for (size_t s = 0; s < todo.size(); ++s) {
      auto f = std::make_shared<SellOp::DenseLU>();
      f->a.resize(ctx, (size_t)n * n * sizeof(T));
      f->perm.resize(ctx, n);
      f->ipiv.resize(ctx, n);
      f->own = true;
      F.push_back((T*)f->a.get());
      P.push_back(f->perm.get());
      I.push_back(f->ipiv.get());
      fs.push_back(f);
    }
    std::vector<int> info;
    lu_factor_shifted<T>(ctx, n, (const T*)op.dmat.get(), todo, F, P, info, I);
    for (size_t s = 0; s < todo.size(); ++s) {
      if (info[s] > 0) fail(CARE_ERR_BREAKDOWN, "A^T + p I is singular in the inner precision");
      op.lu[todo[s]] = fs[s];
    }
    return;
  }
  // rocSOLVER's batched getrf over the whole shift set
  const int ns = (int)todo.size();
  std::vector<std::shared_ptr<SellOp::DenseLU>> fs;
  std::vector<T*> ptrs;
  for (double pr : todo) {
    auto f = std::make_shared<SellOp::DenseLU>();
    f->a.resize(ctx, (size_t)n * n * sizeof(T));
    f->ipiv.resize(ctx, n);
    d2d(ctx, f->a.get(), op.dmat.get(), (size_t)n * n * sizeof(T));
    // the shift is added in the operator precision (I is kept in A's type)
    hipLaunchKernelGGL(k_add_diag<T>, dim3(ceil_div(n, 256)), dim3(256), 0, ctx->stream, (int64_t)n,
                       (T*)f->a.get(), (int64_t)n, (T)pr);
    KERNEL_CHECK();
    ptrs.push_back((T*)f->a.get());
    fs.push_back(f);
  }
  DBuf<T*> dptr(ctx, (size_t)ns);
  DBuf<int> piv(ctx, (size_t)n * ns), info(ctx, (size_t)ns);
  h2d(ctx, dptr.get(), ptrs.data(), (size_t)ns * sizeof(T*));
  ROCBLAS_CHECK(getrf_batched(ctx->blas, n, dptr.get(), piv.get(), info.get(), ns));
  std::vector<int> hinfo(ns);
  d2h(ctx, hinfo.data(), info.get(), (size_t)ns * sizeof(int));
  for (int s = 0; s < ns; ++s) {
    if (hinfo[s] > 0) fail(CARE_ERR_BREAKDOWN, "A^T + p I is singular in the inner precision");
    d2d(ctx, fs[s]->ipiv.get(), piv.get() + (size_t)s * n, (size_t)n * sizeof(int));
    op.lu[todo[s]] = fs[s];
  }
}

void dense_prefactor(Ctx* ctx, const SellOp& op, const std::vector<double>& shifts) {
  if (!op.dense) return;
  if (op.prec == Prec::F64) factor_shifts<double>(ctx, op, shifts);
  else factor_shifts<float>(ctx, op, shifts);
}

template <typename T>
KrylovResult dense_solve(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols, const T* b, int64_t ldb, T* x,
                         int64_t ldx) {
  KrylovResult res;
  if (ncols <= 0) return res;
  if (pi != 0.0) fail(CARE_ERR_NOT_IMPLEMENTED, "complex shifts with a dense operator");
  if ((op.prec == Prec::F64) != (sizeof(T) == 8)) fail(CARE_ERR_ARG, "dense solve precision mismatch");
  const int n = (int)op.n;
  factor_shifts<T>(ctx, op, {pr});
  const std::shared_ptr<SellOp::DenseLU>& f = op.lu.at(pr);
  if (f->own && n <= LU_OWN_SOLVE_MAX) {
    lu_solve<T>(ctx, n, (const T*)f->a.get(), f->perm.get(), ncols, b, ldb, x, ldx);
  } else {
    copy_cols<T, T>(ctx, n, ncols, b, ldb, x, ldx);
    ROCBLAS_CHECK(getrs(ctx->blas, n, ncols, (T*)f->a.get(), f->ipiv.get(), x, (int)ldx));
  }
  res.col_ok.assign(ncols, 1);
  res.col_relres.assign(ncols, 0.0);
  res.col_bnorm.assign(ncols, 0.0);
  return res;
}

template KrylovResult dense_solve<double>(Ctx*, const SellOp&, double, double, int, const double*, int64_t, double*,
                                          int64_t);
template KrylovResult dense_solve<float>(Ctx*, const SellOp&, double, double, int, const float*, int64_t, float*,
                                         int64_t);

}  // namespace mpcare
