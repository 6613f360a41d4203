// Residual-based LR-ADI with SMW shifted solves (the inner solver of Sec. 4).
//
// For  A_k^T X + X A_k + W0 W0^T = 0,  A_k = A - B K^T,  F = A_k^T:
//   real p:        V = (F + p I)^{-1} W,  W <- W - 2 p V,  Z <- [Z, sqrt(-2p) V]
//   pair (p, p*):  V = (F + p I)^{-1} W (complex), delta = Re p / Im p,
//                  Vh = Re V + delta Im V,  W <- W - 4 Re(p) Vh,
//                  Z <- [Z, sqrt(2) g Vh, sqrt(2) g sqrt(delta^2 + 1) Im V],
//                  g = sqrt(-2 Re p)
// and ||residual||_F = ||W^T W||_F after every step.  (F + p I)^{-1} is applied
// through the Sherman-Morrison-Woodbury formula of Sec. 4 with M = A^T + p I:
//   M [Vh, S] = [W, K],  T = I_m - B^T S,  V = Vh + S T^{-1} B^T Vh,
// where S = M^{-1} K and T^{-1} are cached per shift for the whole solve.
#pragma once

#include <algorithm>
#include <complex>

#include "krylov.hpp"

namespace mpcare {

struct Shift {
  double re, im;
};

struct LradiParams {
  double tol = 1e-12;        // ||W^T W||_F <= tol ||W0^T W0||_F
  int jmax = 50;
  double ktol = 1e-10;       // Krylov relative residual per column
  int kmaxit = 4000;
  int check_every = 8;
  bool deflate = true;       // freeze converged columns of W (see lradi_run)
  bool group_tol = true;     // Krylov accuracy relative to the block's largest column
  bool relax = false;        // inexact ADI: looser solves as the ADI residual shrinks (lradi_run)
  bool rotate = false;       // with deflate: rotate W to its principal directions (lradi_run)
  int group_split = 0;       // W0 columns [0, group_split) and the rest form separate groups
  int proj_shifts = 0;       // > 0: projection shifts, at most this many per set (lradi_run)
};

struct LradiOut {
  int steps = 0;             // ADI steps (a complex pair counts 2)
  int zcols = 0;             // columns written to Z
  double res_rel = 0.0;      // final ||W^T W||_F / ||W0^T W0||_F
  double res0 = 0.0;         // ||W0^T W0||_F
  int krylov_unconverged = 0;
  int krylov_max_iters = 0;
  int w_final = 0;           // columns still iterated at the end
  std::vector<int> zsrc;     // column of W0 that each column of Z comes from
};

// in-place inverse of a small m x m complex matrix (column-major, partial
// pivoting); false if singular
bool cinv(int m, std::vector<std::complex<double>>& A);

// shift list checks: Re < 0, complex shifts as (p, conj p) with Im p > 0 first
std::vector<Shift> check_shifts(const care_shift* s, int count);

// Projection shifts (penzl.hip): the Ritz values of F = A^T - K B^T (K = NULL
// or m = 0: A^T) on the span of the s columns of V (n x s, leading dimension
// ldv; in the vector precision T of the operator's solves), restricted to
// the dominant directions of V (eigenvalues of V^T V above 1e-10 of the
// largest, at most 64 of them).  Ritz values in the right half-plane are
// mirrored into the left one; at most l0 shifts are then chosen among them
// by Penzl's greedy min-max rule.  B, K: n x m, ld pad_ld(n).
template <typename T>
std::vector<Shift> projection_shifts(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, const T* V,
                                     int64_t ldv, int s, int l0);

// Growable n x cap column buffer (ld pad_ld(n)) for the LR-ADI factor: the
// factor's final width is known only at the end (column deflation), so the
// buffer starts small and grows by half again when full, keeping the columns
// already written.
template <typename T>
struct ZBuffer {
  DBuf<T> buf;
  int64_t ld = 0;
  int cap = 0;
  void init(Ctx* ctx, int64_t n, int cap0) {
    ld = pad_ld(n);
    cap = std::max(cap0, 1);
    buf = DBuf<T>(ctx, (size_t)ld * cap);
  }
  void reserve(Ctx* ctx, int used, int need) {
    if (need <= cap) return;
    const int nc = std::max(need, cap + cap / 2);
    DBuf<T> nb(ctx, (size_t)ld * nc);
    if (used > 0) d2d(ctx, nb.get(), buf.get(), (size_t)ld * used * sizeof(T));
    buf = std::move(nb);
    cap = nc;
  }
  T* get() const { return buf.get(); }
};

// Run LR-ADI in vector precision T (double or float) on the prepared
// operator.  B, K: n x m (K may be NULL), W: n x w, all with leading
// dimension pad_ld(n); W is overwritten by the final residual factor.  Z
// receives the factor blocks (growing as needed up to zmax columns).
template <typename T>
LradiOut lradi_run(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, T* W, int w,
                   const std::vector<Shift>& shifts, const LradiParams& prm, ZBuffer<T>& Z, int zmax);

// One SMW shifted solve (A_k^T + p I) V = W (the building block of
// lradi_run), V explicit: n x w real, or n x 2w interleaved for complex p.
template <typename T>
KrylovResult shifted_solve(Ctx* ctx, const SellOp& op, const T* B, const T* K, int m, const T* W, int w, Shift p,
                           const LradiParams& prm, T* V);

// largest number of factor columns lradi_run can write for jmax steps
inline int lradi_capacity(int w, int jmax) { return w * (jmax + 2); }

}  // namespace mpcare
