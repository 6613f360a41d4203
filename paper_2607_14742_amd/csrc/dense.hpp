// Dense tall-skinny kernels (FP64 MFMA on gfx950) and small dense helpers.
//
//   gram     C = X^T Y        X: n x a, Y: n x b (FP64 or FP32 inputs),
//                             FP64 accumulation, split over rows with a
//                             fixed-order reduction (deterministic)
//   tsgemm   Y = alpha X S + beta Y    X: n x q, S: q x k small FP64
//   copy_cols  typed column copies with optional column map and scaling
//
// Small q x q work (products, symmetric eigenproblems) runs on the GPU
// through rocBLAS dgemm and rocSOLVER dsyevd.
#pragma once

#include "common.hpp"

namespace mpcare {

template <typename TX, typename TY>
void gram(Ctx* ctx, int64_t n, const TX* X, int64_t ldx, int a, const TY* Y, int64_t ldy, int b, double* C,
          int64_t ldc);

// The library's own MFMA Gram (every output tile, no symmetry shortcut) with
// its row-split partials in `part` (part_doubles doubles, device memory of
// the caller): allocates nothing.  false = the partials of one split do not
// fit (ceil(a/32) ceil(b/32) 1024 > part_doubles); nothing is launched then.
bool gram_own_into(Ctx* ctx, int64_t n, const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                   double* C, int64_t ldc, double* part, size_t part_doubles);

// care_gram_noalloc: gram_own_into with the partials in the library's fixed
// device array (noalloc.hip)
void gram_noalloc(Ctx* ctx, int64_t n, const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                  double* C, int64_t ldc);

// Y = alpha X S + beta Y  (beta == 0: Y is not read)
template <typename TX, typename TY>
void tsgemm(Ctx* ctx, int64_t n, const TX* X, int64_t ldx, int q, const double* S, int64_t lds, int k,
            double alpha, double beta, TY* Y, int64_t ldy);

// out[:, c] = scale[c] * in[:, map[c]]  (map[c] < 0 -> zero column).  map and
// scale are HOST arrays (may be NULL: identity / 1).
template <typename TI, typename TO>
void copy_cols(Ctx* ctx, int64_t n, int ncols, const TI* in, int64_t ldi, TO* out, int64_t ldo,
               const int* map = nullptr, const double* scale = nullptr);

// p[0..count) = v
template <typename T>
void fill_const(Ctx* ctx, T* p, size_t count, double v);

// Y = a X + b Y on n x ncols panels (same type)
template <typename T>
void axpby(Ctx* ctx, int64_t n, int ncols, double a, const T* X, int64_t ldx, double b, T* Y, int64_t ldy);

// small dense helpers on device, column-major FP64
// C = alpha op(A) op(B) + beta C via rocBLAS
void dgemm(Ctx* ctx, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc);
// symmetric eigen-decomposition A = Q diag(w) Q^T in place (A -> Q),
// eigenvalues ascending, copied to the host vector w
void dsyevd(Ctx* ctx, int n, double* A, int lda, std::vector<double>& w);

// Rank-revealing orthogonalisation of a tall-skinny FP64 matrix:
// F (n x q) = U T + E with U^T U = I (n x k), T = U^T F (k x q) and E at the
// FP64 noise level of F's columns.  See dense.hip for the algorithm.
struct Orth {
  DBuf<double> U;      // n x k, ld = ldu
  DBuf<double> T;      // k x q, ld = k
  int64_t ldu = 0;
  int k = 0;
};
void rr_orth(Ctx* ctx, int64_t n, const double* F, int64_t ldf, int q, Orth& out);
// The same with a known orthonormal basis U0 (n x k0, ld ldu0) of part of
// the column space: U = [U0, U_new] with U_new orthogonal to U0, and
// T = U^T F (k x q) for the q columns of F only.
void rr_orth(Ctx* ctx, int64_t n, const double* F, int64_t ldf, int q, Orth& out, const double* U0, int64_t ldu0,
             int k0);

}  // namespace mpcare
