// Column-batched BiCGStab for the shifted block solves (A^T + p I) X = B
// that dominate LR-ADI (Sec. 4: "the dominant computation is the application
// of M_alpha^{-1} to block right hand sides").  The paper uses restarted
// GMRES; this library uses BiCGStab (two sparse products and a handful of
// fused vector passes per iteration, no basis storage) with one independent
// recurrence per right-hand-side column, all columns sharing each launch.
#pragma once

#include "sparse.hpp"

namespace mpcare {

struct KrylovResult {
  int max_iters = 0;        // largest per-column iteration count
  int unconverged = 0;      // columns that stopped above tol
  int breakdown = 0;        // columns stopped by a breakdown
  int restarts = 0;         // restart rounds performed
  int compactions = 0;      // times the still-active columns were gathered into fewer panels
  double worst_relres = 0;  // largest ||r|| / ||b|| at exit (recursive residual)
  std::vector<int> col_ok;          // per logical column: reached its tolerance
  std::vector<double> col_relres;   // per logical column: ||r|| / ||b||
  std::vector<double> col_bnorm;    // per logical column: ||b||
};

// Solve (A^T + p I) x_c = b_c for every column c.  T = double needs an FP64
// operator, T = float an FP32 or BF16 operator.  Complex p (pi != 0): b and
// x hold ncols_real/2 complex columns as interleaved (re, im) column pairs.
// x is overwritten (zero initial guess).  Columns with b_c = 0 return 0.
//
// groups (optional, one id per logical column): the stopping test of column
// c becomes ||r_c|| <= tol max_{c' in group(c)} ||b_c'||, i.e. accuracy
// relative to the largest right-hand side of its group rather than to its
// own norm (the block is used as a whole by LR-ADI).  NULL: ||r_c|| <= tol ||b_c||.
template <typename T>
KrylovResult bicgstab(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols_real, const T* b,
                      int64_t ldb, T* x, int64_t ldx, double tol, int maxit, int check_every,
                      const std::vector<int>* groups = nullptr);

// The same solve through the red-black reduction of op (rb.hip): the
// reduced system (G + p' I) x_b = F b_r - (d + p) b_b goes to bicgstab with
// the operator G, then x_r = (b_r - E x_b) / (d + p).  Tolerances apply to
// the reduced right-hand side.  bicgstab() dispatches here when the context
// enables the reduction and rb_usable() holds.
template <typename T>
KrylovResult bicgstab_rb(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols_real, const T* b, int64_t ldb,
                         T* x, int64_t ldx, double tol, int maxit, int check_every, const std::vector<int>* groups);
bool rb_usable(const SellOp& op, double pr, double pi);

// Restarted GMRES(restart) for a real shift (gmres.hip): the same contract as
// bicgstab (zero initial guess, per-column or per-group tolerance); maxit
// counts Arnoldi steps over all cycles.  bicgstab() dispatches here when the
// context selects it and the shift is real.
template <typename T>
KrylovResult gmres(Ctx* ctx, const SellOp& op, double pr, int ncols, const T* b, int64_t ldb, T* x, int64_t ldx,
                   double tol, int maxit, int restart, const std::vector<int>* groups);

// Direct shifted solve for a dense operator (dense_op.hip): LU of A^T + p I
// in the operator precision, cached per real shift on the operator.
template <typename T>
KrylovResult dense_solve(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols, const T* b, int64_t ldb, T* x,
                         int64_t ldx);

}  // namespace mpcare
