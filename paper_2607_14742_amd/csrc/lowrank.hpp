// Algorithm 1 (residual factor decomposition) and Algorithm 2 (solution
// factor decomposition) in FP64 on the GPU.
#pragma once

#include "dense.hpp"
#include "sparse.hpp"

namespace mpcare {

struct ResidualFactor {
  DBuf<double> Cp, Cm;      // n x rp, n x rm, ld = pad_ld(n)
  int rp = 0, rm = 0;
  double res_fro = 0.0;     // ||R(Z Z^T)||_F = ||H||_F before truncation
  double lam_max = 0.0;
};

// Algorithm 1.  A64: FP64 operator; B (n x m) and Ct = C^T (n x p) FP64 with
// leading dimension pad_ld(n); Z: n x r (ldz).  Eigenvalues of H below
// eta_r_rel max|lambda(H)| in magnitude are dropped; with drop_fro > 0 so are
// the smallest ones whose joint Frobenius norm is at most drop_fro.
struct TruncResult;
void residual_factor(Ctx* ctx, const SellOp& A64, const double* B, int m, const double* Ct, int p,
                     const double* Z, int64_t ldz, int r, double eta_r_rel, ResidualFactor& out,
                     double drop_fro = 0.0, const TruncResult* basis = nullptr);

// Algorithm 2 for a general signature: Z Z^T = positive part of G N G^T
// above eta_s_rel * max|lambda(P)|.  Output Z: n x *r (ld pad_ld(n)).
// Z = Q diag(sqrt(sig)) with orthonormal Q (kept when has_q): a later
// Algorithm 1 or 2 on a matrix whose leading block is Z starts its
// orthogonalisation from Q (residual_factor's `basis`, signed_truncate_basis).
struct TruncResult {
  DBuf<double> Z;
  int r = 0;
  double eta_n = 0.0;
  double sig_max = 0.0;
  DBuf<double> Q;               // n x r, ld pad_ld(n)
  std::vector<double> sig;      // r kept eigenvalues of Z Z^T
  bool has_q = false;
};
// With res_budget > 0 the smallest kept eigenvalues are dropped as well while
// the Frobenius norm E of everything dropped from the positive part stays
// within res_budget / (2 (a2 + g2 sig_max)): removing E from X changes the
// Riccati residual by at most 2 (||A||_2 + ||B B^T||_2 ||X||_2) ||E||_F
// (to first order), so a2 >= ||A||_2 and g2 >= ||B B^T||_2 keep that change
// within res_budget.
void signed_truncate(Ctx* ctx, int64_t n, const double* G, int64_t ldg, int s, const std::vector<double>& sign,
                     double eta_s_rel, TruncResult& out, double res_budget = 0.0, double a2 = 0.0,
                     double g2 = 0.0);

// Algorithm 2 for G = [Zk, Grest] with signature [+1 (Zk.r times), sign]:
// the orthogonalisation starts from Zk's orthonormal basis (Zk.has_q).
void signed_truncate_basis(Ctx* ctx, int64_t n, const TruncResult& Zk, const double* Grest, int64_t ldg, int s,
                           const std::vector<double>& sign, double eta_s_rel, TruncResult& out,
                           double res_budget = 0.0, double a2 = 0.0, double g2 = 0.0);

// The largest magnitude c such that all of |v| <= c together stay within
// drop_fro in the Frobenius norm (0 when even the smallest does not).
double frobenius_cut(std::vector<double> v, double drop_fro);

// Compression of one positive semidefinite factor ahead of Algorithm 2:
// Z Z^T = U diag(lam) U^T from the FP64 Gram Z^T Z = V diag(lam) V^T; keeps
// lam > tau_abs and returns Zc = Z V_sel (n x r, ld pad_ld(n), orthogonal
// columns), so that ||Z Z^T - Zc Zc^T||_2 <= tau_abs + O(u lam_max): the
// dropped part is exactly the sum of the dropped eigen-terms, so only the
// FP64 Gram's own rounding adds to it.  Returns false, and leaves out
// untouched, when tau_abs lies below 1e-14 lam_max, where that rounding would
// no longer be small next to it.
// With drop_fro > 0 the smallest eigen-terms whose joint Frobenius norm is at
// most drop_fro are dropped as well.
bool psd_compress(Ctx* ctx, int64_t n, const double* Z, int64_t ldz, int w, double tau_abs, DBuf<double>& out,
                  int& r, double drop_fro = 0.0);

// largest eigenvalue of Z Z^T (0 for an empty factor)
double factor_lam_max(Ctx* ctx, int64_t n, const double* Z, int64_t ldz, int r);

}  // namespace mpcare
