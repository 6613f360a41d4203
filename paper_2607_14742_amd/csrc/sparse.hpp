// Sparse operator M = A^T + p I used by every shifted solve (Sec. 4).
//
// Layout in HBM: A^T is stored once per precision in SELL-64 form (sliced
// ELLPACK, 64 rows per slice = one wavefront, rows in their original order):
//   * slice s covers rows [64 s, 64 s + 64); its width w_s is the largest
//     off-diagonal row length of A^T in the slice;
//   * entry t of row 64 s + l is at offset (sptr[s] + t) * 64 + l of `cols`
//     and `vals`, so one wavefront reads 64 consecutive column indices and
//     values per step (coalesced 256 B / 128 B / 512 B loads);
//   * padding entries point at the row itself with value 0;
//   * the diagonal is kept apart in the vector precision (`diag`), so the
//     shift is applied as (d_i + p) x_i in that precision and the bf16
//     variant rounds only off-diagonal values.
// Dense n x k panels (Krylov vectors, ADI factors) are column-major with a
// leading dimension rounded up to 64 rows.
#pragma once

#include <cmath>

#include <map>
#include <memory>

#include "common.hpp"
#include "spmm_kernel.hpp"

namespace mpcare {

struct RbOp;
struct IluOp;

struct SellOp {
  int64_t n = 0, nnz = 0;          // of A
  int nslices = 0;
  int64_t width_total = 0;         // sum of slice widths
  int max_width = 0;               // widest slice (off-diagonal entries per row)
  float val_scale = 1.0f;          // F16: values stored as a_ij / val_scale (a power of two)
  Prec prec = Prec::F64;
  DBuf<int> sptr;                  // nslices + 1
  DBuf<int> cols;                  // width_total * 64
  DBuf<uint8_t> vals;              // width_total * 64 * val_bytes
  DBuf<uint8_t> diag;              // n * vec_bytes
  double frob = 0.0;               // ||A||_F (FP64)
  double norm_inf = 0.0;           // ||A||_inf = max_i sum_j |a_ij| (FP64)
  double norm_one = 0.0;           // ||A||_1 = max_j sum_i |a_ij| = ||A^T||_inf (FP64)
  // panel width chosen by the autotuner per product shape (launch_spmm)
  mutable std::map<int, int> cp_choice;
  // sqrt(||A||_1 ||A||_inf) >= ||A||_2
  double norm2_bound() const { return std::sqrt(norm_one * norm_inf); }
  // Dense operator (dense_op.hip): A^T held as an n x n column-major matrix
  // (leading dimension n) in the operator precision; shifted solves use LU
  // factorisations of A^T + p I cached per real shift.
  bool dense = false;
  DBuf<uint8_t> dmat;
  struct DenseLU {
    DBuf<uint8_t> a;               // LU factors, n x n
    DBuf<int> ipiv;                // 1-based row exchanges (for getrs)
    DBuf<int> perm;                // hand-written factors: (P M)[i] = M[perm[i]]
    bool own = false;              // factors from lu_factor_shifted
  };
  mutable std::map<double, std::shared_ptr<DenseLU>> lu;
  // Red-black reduction of A^T + p I (rb.hip), present when A is two-colourable
  // with a constant diagonal and the context enables it
  std::shared_ptr<RbOp> rb;
  // Multicolour ILU(0) of A^T + p I (ilu.hip): the colouring of A's pattern,
  // present when the context asks for the preconditioned GMRES solves
  std::shared_ptr<IluOp> ilu;
  // algorithmic bytes of one product with k real columns: the CSR formula
  // nnz (s_v + 4) + 4 (n + 1) plus `passes` n-vectors per column (2 for
  // y = M x; the fused BiCGStab modes move more, see spmm_vec_passes)
  double bytes(int k, int passes = 2) const {
    return double(nnz) * (double(val_bytes(prec)) + 4.0) + 4.0 * double(n + 1) +
           double(passes) * double(n) * double(k) * double(vec_bytes(prec));
  }
};

// Build A^T in SELL-64 form at precision `prec` from the caller's CSR(A).
void build_sell(Ctx* ctx, const care_csr* A, Prec prec, SellOp& op);

// Red-black reduction (rb.hip).  When the pattern of A is two-colourable
// (red / black, every off-diagonal entry couples the two colours; five- and
// seven-point stencils) and its diagonal is one constant d, the shifted solve
//   (A^T + p I) x = b,   A^T = [[d I, E], [F, d I]] in red / black order,
// eliminates the red unknowns exactly: with G = F E (black x black),
//   (G + p' I) x_b = F b_r - (d + p) b_b,   p' = -(d + p)^2,
//   x_r = (b_r - E x_b) / (d + p).
// G + p' I has half the rows and about a quarter of the condition number of
// A^T + p I.  The host analysis of CSR(A) (two-colouring, G) is done once and
// attached to every operator built from the same A.
struct RbHost;
std::shared_ptr<RbHost> rb_analyse(Ctx* ctx, const care_csr* A);   // nullptr: not applicable
void rb_attach(Ctx* ctx, const std::shared_ptr<RbHost>& h, Prec prec, SellOp& op);
struct RbOp {
  double d = 0.0;                  // the constant diagonal of A
  int64_t nr = 0, nb = 0;          // red / black rows
  DBuf<int> red, blk;              // original index of each red / black row
  DBuf<int> frp, fci;              // F: rows of A^T at black rows, red columns (original indices)
  DBuf<int> erp, eci;              // E: rows of A^T at red rows, black columns (reduced indices)
  DBuf<uint8_t> fval, eval;        // values in the operator's vector precision
  SellOp G;                        // G = F E over the black rows (SELL-64, diagonal kept apart)
};

// Multicolour ILU(0) of A^T + p I (ilu.hip).  ilu_analyse colours the
// pattern of A first-fit in natural order (host, once per matrix; fails with
// CARE_ERR_NOT_IMPLEMENTED past 1024 colours); ilu_attach uploads the colour
// classes to an operator built from the same A.  ilu_factor returns the
// factors of A^T + p I for a real shift, factored once per shift and kept on
// the operator; a zero pivot fails with CARE_ERR_BREAKDOWN.  ilu_apply sets
// Z = (L U)^{-1} X for k columns (X, Z distinct, vector precision of op).
struct IluHost;
std::shared_ptr<IluHost> ilu_analyse(Ctx* ctx, const care_csr* A);
// The colouring alone, on a host CSR pattern (validated here): colour[i] for
// every row, returns the number of colours.
int ilu_colour_host(int64_t n, int64_t nnz, const int* rp, const int* ci, std::vector<int>& colour);
void ilu_attach(Ctx* ctx, const std::shared_ptr<IluHost>& h, SellOp& op);
struct IluOp {
  int ncol = 0;
  std::vector<int> coff;           // colour c holds rows[coff[c] .. coff[c + 1]) (host)
  DBuf<int> rows;                  // rows grouped by colour, increasing index inside a colour
  DBuf<int> colour;                // colour of each row
  struct Factors {
    DBuf<uint8_t> off;             // l_ij / u_ij at the SELL positions of A^T
    DBuf<uint8_t> dinv;            // 1 / u_ii
  };
  std::map<double, std::shared_ptr<Factors>> fac;
};
std::shared_ptr<IluOp::Factors> ilu_factor(Ctx* ctx, const SellOp& op, double p);
template <typename T>
void ilu_apply(Ctx* ctx, const SellOp& op, const IluOp::Factors& f, int k, const T* X, int64_t ldx, T* Z,
               int64_t ldz);

// Y = (A^T + p I) X for k real columns (complex shift: k complex columns in
// interleaved [re, im] column pairs, i.e. 2k real columns).  X, Y in the
// operator's vector precision.
void spmm_plain(Ctx* ctx, const SellOp& op, double pr, double pi, const void* X, int64_t ldx,
                int k_real, void* Y, int64_t ldy);

// Dense operators (dense_op.hip): build A^T from a dense column-major A
// (device, leading dimension lda) in precision prec (FP64 or FP32), and
// Y = (A^T + p I) X by GEMM (real p only).
void build_dense(Ctx* ctx, const double* A, int64_t lda, int64_t n, Prec prec, SellOp& op);
// Factor A^T + p I of a dense operator for every listed real shift not
// factored yet (one launch of the batched LU for orders up to LU_NMAX).
void dense_prefactor(Ctx* ctx, const SellOp& op, const std::vector<double>& shifts);
void dense_apply(Ctx* ctx, const SellOp& op, double pr, double pi, const void* X, int64_t ldx, int k, void* Y,
                 int64_t ldy);

// Launch one sparse product in `mode` (see spmm_kernel.hpp) with the panel
// width picked from the column count; fills grid-dependent fields of `a`
// (n, sptr, cols, vals, diag, nrb).  Returns the number of row blocks.
template <typename T>
int launch_spmm(Ctx* ctx, const SellOp& op, int mode, bool cplx, SpmmArgs<T>& a);

inline int spmm_rowblocks(int64_t n) { return (int)((n + 255) / 256); }

// record the algorithmic traffic of a product (and bracket it with events
// when profiling is on)
// n-vector passes per real column of one launch in each mode: y = M x reads
// x and writes y; MODE_BICG_P reads r, p, v, rhat and writes p, v (4 on a
// column's first iteration, where p and v are not read); MODE_BICG_S reads
// r, v and writes s, t; the split second halves read x (and rhat) and write y.
inline int spmm_vec_passes(int mode, bool first = false) {
  switch (mode) {
    case 1: return first ? 4 : 6;   // MODE_BICG_P
    case 2: return 4;               // MODE_BICG_S
    case 3: return 3;               // MODE_DOT1: x, rhat read; y written
    default: return 2;              // MODE_PLAIN, MODE_DOT2: x read; y written
  }
}

// Counts a launch and, when the context profiles, brackets it with HIP events
// on the library stream.  While ctx->spmm_defer is set the launch's bytes are
// left to the caller, which knows how many columns were still active.
struct SpmmTimer {
  Ctx* ctx;
  std::pair<hipEvent_t, hipEvent_t> ev{};
  SpmmTimer(Ctx* c, const SellOp& op, int k_real, int mode);
  ~SpmmTimer();
};

}  // namespace mpcare
