// Framework 1 driver: NLR-ADI initial solve in the inner precision, then the
// FP64 residual / inner correction / FP64 update loop.
#pragma once

#include "adi.hpp"
#include "lowrank.hpp"

namespace mpcare {

struct Resolved {
  Prec prec = Prec::F64;
  double tau_L = 1e-12, tau_L0 = 1e-12, tau_0 = 1e-10, ktol = 1e-10, theta = 0.25;
  double eta_r_rel = 1e-4, eta_s_rel = 1.1102230246251565e-15, stagnation = 0.999;
  int k_max = 20, k0_max = 20, j_max = 50, kmaxit = 4000, check_every = 8;
  bool deflate = true, block_tol = false, relax = false, rotate = true;
};

Resolved resolve_opts(const care_opts* o, double tol);
// max|p| / min|p| over a shift set (1 for an empty or degenerate set)
double shift_spread(const std::vector<Shift>& shifts);
// ||A||_2 / min |Re p|: the estimate of kappa_F(L) behind CARE_AUTO
double kappa_L_estimate(double norm2_bound, const std::vector<Shift>& shifts);
// CARE_FP32 or CARE_FP64 for inner_prec = CARE_AUTO, from that estimate
int choose_inner_precision(double norm2_bound, const std::vector<Shift>& shifts, bool dense);

// The operator of one solve: a sparse CSR of A, or a dense column-major A.
struct OpSpec {
  const care_csr* csr = nullptr;
  const double* dense = nullptr;   // device, n x n, leading dimension lda
  int64_t n = 0, lda = 0;
  int64_t size() const { return csr ? csr->n : n; }
};
OpSpec sparse_spec(const care_csr* A);
OpSpec dense_spec(const double* A, int64_t n, int64_t lda);
void build_op(Ctx* ctx, const OpSpec& A, Prec prec, SellOp& op);

void care_solve_impl(Ctx* ctx, const OpSpec& A, const double* B, int m, const double* C, int p, double tol,
                     const care_shift* shifts, int nshifts, const care_opts* opts, double* Z, int64_t ldz, int rmax,
                     int* r_out, care_stats* stats, care_status* warn);

// Batched solve of independent instances on concurrent worker streams
// (batch.hip); per-instance outcomes in res.
void solve_batch(Ctx* ctx, int count, const care_instance* inst, double tol, const care_opts* opts, int workers,
                 care_instance_result* res);

// Penzl's heuristic (penzl.hip): Ritz values of A^T and A^-T on the GPU, then
// the greedy min-max choice of l0 shifts; real_only keeps real parts.
// shift heuristic (Penzl) from Ritz values of A_k^T = A^T - K B^T and its
// inverse; K = NULL (or m = 0) gives the shifts of A itself
std::vector<Shift> penzl_shifts(Ctx* ctx, const SellOp& A64, int l0, int kp, int km, bool real_only,
                                const double* B = nullptr, const double* K = nullptr, int m = 0);
// host steps of the heuristic
std::vector<std::complex<double>> hessenberg_eigvals(const double* H, int k, int64_t ldh);
std::vector<Shift> penzl_select(std::vector<std::complex<double>> R, int l0);

}  // namespace mpcare
