// Batched LU with partial pivoting of shifted dense matrices and its
// triangular solves (lu.hip).
#pragma once

#include <vector>

#include "common.hpp"

namespace mpcare {

// largest order the hand-written factorisation and solve take (two panel rows
// per thread of a 1024-thread workgroup; the solve keeps n x KB values in LDS)
constexpr int LU_NMAX = 2048;

// Factor M_s = M0 + shifts[s] I for every s in one launch, one workgroup per
// matrix.  M0: device n x n column-major (ld n) in T; F[s]: device n x n (ld n,
// not overlapping M0) receiving the LAPACK getrf layout; perm[s]: device n
// ints with (P M_s)[i] = M_s[perm[s][i]]; info[s]: 0, or the 1-based index of
// the first zero pivot; ipiv (optional, one device array of n ints per
// shift): the row exchanges, 1-based as getrf's (for rocSOLVER getrs).  The
// shift is rounded to T before it is added.
template <typename T>
void lu_factor_shifted(Ctx* ctx, int n, const T* M0, const std::vector<double>& shifts, const std::vector<T*>& F,
                       const std::vector<int*>& perm, std::vector<int>& info, const std::vector<int*>& ipiv = {});

// Largest order at which the dense shifted solves use lu_solve; beyond it
// rocSOLVER getrs on the same factors is faster (measured: FP32, k = 8..16,
// 150 vs 180 us at n = 512, 354 vs 275 us at n = 1024).
constexpr int LU_OWN_SOLVE_MAX = 512;

// X = M^{-1} B for k columns with the factors of one matrix (B and X may be
// the same storage with the same leading dimension).  Asynchronous on the
// context's stream.
template <typename T>
void lu_solve(Ctx* ctx, int n, const T* F, const int* perm, int k, const T* B, int64_t ldb, T* X, int64_t ldx);

}  // namespace mpcare
