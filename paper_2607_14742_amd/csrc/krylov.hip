// Column-batched BiCGStab (real and complex shifts).
//
// One iteration = three fused passes over the n x k panels plus three tiny
// per-column scalar kernels, all enqueued without host synchronisation:
//   K1  v = M p~,  p~ = r + beta (p - omega v_old)          partial <rhat, v>
//   S1  alpha = rho / <rhat, v>
//   K2  t = M s,   s = r - alpha v                           partials <t, s>, <t, t>
//   S2  omega = <t, s> / <t, t>
//   K3  x += alpha p~ + omega s,  r = s - omega t            partials <rhat, r>, <r, r>
//   S3  beta = (rho_new / rho)(alpha / omega), convergence test
// rhat = b (the right-hand side itself, never copied).  Columns that reach
// ||r|| <= tol ||b|| are frozen by their status flag; every kernel skips them.
// The host polls the status array every `check_every` iterations.
#include "krylov.hpp"

#include <cstdlib>
#include <map>

#include "dense.hpp"

namespace mpcare {

enum { FLAG_NONE = 0, FLAG_CONVERGED = 1, FLAG_BREAKDOWN = 2, FLAG_NONFINITE = 3, FLAG_STAGNATED = 4, FLAG_DIVERGED = 5 };
// a column stops when its residual norm has not dropped by 10 % for
// max(STALL_MAX, iterations / 4) iterations in FP64, max(STALL_MAX_F32,
// iterations / 8) in FP32 (the attainable accuracy of the working precision
// is reached, or BiCGStab stagnates; see the restarts), or when it exceeds
// 1e3 x the smallest residual met (divergence); it then returns the best
// checkpointed iterate.  FP32 columns meet their precision's floor often (at
// small shifts the floor lies above the requested tolerance), so their window
// is shorter; FP64 keeps the longer one.  The unshifted solves of the shift
// heuristic's inverse Arnoldi (condition number up to kappa(A)) go through
// long plateaus and use max(STALL_MAX_PATIENT, iterations / 2).
constexpr int STALL_MAX = 150;
constexpr int STALL_MAX_PATIENT = 1000;
constexpr int STALL_MAX_F32 = 50;
constexpr double DIVERGE_RR = 1e6;
enum { UPD_INIT = 0, UPD_XR = 1 };

template <typename T>
struct ElemArgs {
  int n = 0, ncols = 0, nrb = 0;
  int64_t ld = 0;                 // Krylov workspace leading dimension
  const T* b = nullptr;
  int64_t ldb = 0;
  T* x = nullptr;
  int64_t ldx = 0;
  T* r = nullptr;
  const T* p = nullptr;
  const T* s = nullptr;
  const T* t = nullptr;
  const double* sc = nullptr;
  const int* st = nullptr;
  double* part = nullptr;
};

// elementwise BiCGStab passes with fused column dots
template <typename T, int CP, int UMODE, bool CPLX>
__global__ void __launch_bounds__(256) k_bicg_elem(ElemArgs<T> a) {
  constexpr int NL = CPLX ? CP / 2 : CP;
  constexpr int NDOT = UMODE == UPD_INIT ? 1 : 2;
  const int rb = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = rb * 256 + threadIdx.x;
  const int c0 = blockIdx.y * CP;
  T dots[NDOT * CP];
#pragma unroll
  for (int k = 0; k < NDOT * CP; ++k) dots[k] = (T)0;

  if (UMODE == UPD_INIT) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int cr = c0 + (CPLX ? 2 * q : q);
      if (cr >= a.ncols || i >= a.n) continue;
      const int64_t ob = (int64_t)cr * a.ldb + i, ox = (int64_t)cr * a.ldx + i, o = (int64_t)cr * a.ld + i;
      const T br = a.b[ob];
      a.r[o] = br;
      a.x[ox] = (T)0;
      if (!CPLX) {
        dots[q] = br * br;
      } else {
        const T bi = a.b[ob + a.ldb];
        a.r[o + a.ld] = bi;
        a.x[ox + a.ldx] = (T)0;
        dots[2 * q] = br * br + bi * bi;
        dots[2 * q + 1] = (T)0;
      }
    }
  } else {
    // all loads first, without a branch per column (inactive columns read the
    // panel's first active column), then the stores of the active columns
    bool act[NL];
    int colq[NL];
    int qa = -1;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int cr = c0 + (CPLX ? 2 * q : q);
      act[q] = cr < a.ncols && a.st[(int64_t)(CPLX ? cr / 2 : cr) * KI + KI_ACTIVE] != 0;
      if (qa < 0 && act[q]) qa = q;
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) colq[q] = act[q] ? c0 + (CPLX ? 2 * q : q) : c0 + (CPLX ? 2 * qa : qa);
    if (qa >= 0 && i < a.n) {
      T pr[NL], pim[NL], sr[NL], sim[NL], tr[NL], tim[NL], xr[NL], xim[NL], hr[NL], hi[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int cr = colq[q];
        const int64_t ob = (int64_t)cr * a.ldb + i, ox = (int64_t)cr * a.ldx + i, o = (int64_t)cr * a.ld + i;
        pr[q] = a.p[o];
        sr[q] = a.s[o];
        tr[q] = a.t[o];
        xr[q] = a.x[ox];
        hr[q] = a.b[ob];
        pim[q] = sim[q] = tim[q] = xim[q] = hi[q] = (T)0;
        if (CPLX) {
          pim[q] = a.p[o + a.ld];
          sim[q] = a.s[o + a.ld];
          tim[q] = a.t[o + a.ld];
          xim[q] = a.x[ox + a.ldx];
          hi[q] = a.b[ob + a.ldb];
        }
      }
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        if (!act[q]) continue;
        const int cr = c0 + (CPLX ? 2 * q : q);
        const int lc = CPLX ? cr / 2 : cr;
        const int64_t ox = (int64_t)cr * a.ldx + i, o = (int64_t)cr * a.ld + i;
        const double* sc = a.sc + (int64_t)lc * KS;
        if (!CPLX) {
          const T al = (T)sc[KS_ALPHA], om = (T)sc[KS_OMEGA];
          a.x[ox] = xr[q] + (al * pr[q] + om * sr[q]);
          const T rv = sr[q] - om * tr[q];
          a.r[o] = rv;
          dots[q] = hr[q] * rv;               // <rhat, r>
          dots[CP + q] = rv * rv;             // <r, r>
        } else {
          const T alr = (T)sc[KS_ALPHA], ali = (T)sc[KS_ALPHA + 1];
          const T omr = (T)sc[KS_OMEGA], omi = (T)sc[KS_OMEGA + 1];
          a.x[ox] = xr[q] + ((alr * pr[q] - ali * pim[q]) + (omr * sr[q] - omi * sim[q]));
          a.x[ox + a.ldx] = xim[q] + ((alr * pim[q] + ali * pr[q]) + (omr * sim[q] + omi * sr[q]));
          const T rr = sr[q] - (omr * tr[q] - omi * tim[q]);
          const T ri = sim[q] - (omr * tim[q] + omi * tr[q]);
          a.r[o] = rr;
          a.r[o + a.ld] = ri;
          dots[2 * q] = hr[q] * rr + hi[q] * ri;          // conj(rhat) r
          dots[2 * q + 1] = hr[q] * ri - hi[q] * rr;
          dots[CP + 2 * q] = rr * rr + ri * ri;           // |r|^2
          dots[CP + 2 * q + 1] = (T)0;
        }
      }
    }
  }
  block_reduce_to<NDOT * CP>(dots, [&](int kk, double val) {
    const int dot = kk / CP, c = c0 + kk % CP;
    if (c < a.ncols) a.part[((int64_t)dot * a.ncols + c) * a.nrb + rb] = val;
  });
}

// sum of the row-block partials of (dot, real column c): one wavefront,
// fixed order
// (SCALAR_THREADS threads; four independent loads in flight per thread, then
// a fixed-order tree: the result is the same on every thread)
constexpr int SCALAR_THREADS = 256;
__device__ __forceinline__ double wave_sum_partials(const double* __restrict__ part, int ncols, int nrb, int dot,
                                                    int c) {
  const double* p = part + ((int64_t)dot * ncols + c) * nrb;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int t = threadIdx.x;
  for (int rb = t; rb < nrb; rb += 4 * SCALAR_THREADS) {
    const int r1 = rb + SCALAR_THREADS, r2 = rb + 2 * SCALAR_THREADS, r3 = rb + 3 * SCALAR_THREADS;
    const double a0 = p[rb];
    const double a1 = r1 < nrb ? p[r1] : 0.0;
    const double a2 = r2 < nrb ? p[r2] : 0.0;
    const double a3 = r3 < nrb ? p[r3] : 0.0;
    s0 += a0;
    s1 += a1;
    s2 += a2;
    s3 += a3;
  }
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double wsum[SCALAR_THREADS / 64];
  __syncthreads();
  if ((t & 63) == 0) wsum[t >> 6] = s;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int w = 0; w < SCALAR_THREADS / 64; ++w) tot += wsum[w];
  return tot;
}

// (not written as v - v == 0: floating-point contraction may turn that into
// fma(a, b, -(a b)) for v = a b, which is the product's rounding error)
__device__ __forceinline__ bool finite_d(double v) { return __builtin_isfinite(v); }

// complex helpers (re, im) on doubles
__device__ __forceinline__ void cdiv(double ar, double ai, double br, double bi, double& qr, double& qi) {
  // (ar + i ai) / (br + i bi), scaled (Smith's method)
  if (fabs(br) >= fabs(bi)) {
    const double r = bi / br, d = br + bi * r;
    qr = (ar + ai * r) / d;
    qi = (ai - ar * r) / d;
  } else {
    const double r = br / bi, d = bi + br * r;
    qr = (ar * r + ai) / d;
    qi = (ai * r - ar) / d;
  }
}

// PHASE 0: init (bnrm2, rho); 1: alpha; 2: omega; 3: beta + convergence
template <int PHASE, bool CPLX>
__global__ void __launch_bounds__(SCALAR_THREADS) k_bicg_scalar(double* __restrict__ scv, int* __restrict__ stv,
                                                    const double* __restrict__ part, int ncols, int nrb, double tol2,
                                                    int stall_min, int stall_div) {
  const int lc = blockIdx.x;
  const int cr = CPLX ? 2 * lc : lc;
  double* sc = scv + (int64_t)lc * KS;
  int* st = stv + (int64_t)lc * KI;
  if (PHASE != 0 && st[KI_ACTIVE] == 0) return;   // uniform per block
  if (PHASE == 0) {
    const double bb = wave_sum_partials(part, ncols, nrb, 0, cr);
    if (threadIdx.x == 0) {
      for (int k = 0; k < KS; ++k) sc[k] = 0.0;
      sc[KS_BNRM2] = bb;
      sc[KS_RNRM2] = bb;
      sc[KS_RHO] = bb;              // <rhat, r0> = ||b||^2
      sc[KS_OMEGA] = 1.0;
      sc[KS_RMIN] = bb;
      sc[KS_RREF] = bb;
      sc[KS_RCKPT] = bb;            // the checkpoint starts as x0 = 0
      sc[KS_TOL2] = tol2;           // stop at ||r||^2 <= TOL2 ||b||^2
      st[KI_ITERS] = 0;
      st[KI_STALL] = 0;
      const bool ok = finite_d(bb);
      st[KI_ACTIVE] = (ok && bb > 0.0) ? 1 : 0;
      st[KI_FLAG] = ok ? (bb > 0.0 ? FLAG_NONE : FLAG_CONVERGED) : FLAG_NONFINITE;
    }
    return;
  }
  if (PHASE == 1) {
    const double vr = wave_sum_partials(part, ncols, nrb, 0, cr);
    const double vi = CPLX ? wave_sum_partials(part, ncols, nrb, 0, cr + 1) : 0.0;
    if (threadIdx.x == 0) {
      double ar, ai;
      if (!CPLX) {
        ar = sc[KS_RHO] / vr;
        ai = 0.0;
      } else {
        cdiv(sc[KS_RHO], sc[KS_RHO + 1], vr, vi, ar, ai);
      }
      if ((vr == 0.0 && vi == 0.0) || !finite_d(ar) || !finite_d(ai)) {
        st[KI_ACTIVE] = 0;
        st[KI_FLAG] = FLAG_BREAKDOWN;
      } else {
        sc[KS_ALPHA] = ar;
        sc[KS_ALPHA + 1] = ai;
      }
    }
    return;
  }
  if (PHASE == 2) {
    const double tsr = wave_sum_partials(part, ncols, nrb, 0, cr);
    const double tsi = CPLX ? wave_sum_partials(part, ncols, nrb, 0, cr + 1) : 0.0;
    const double tt = wave_sum_partials(part, ncols, nrb, 1, cr);
    if (threadIdx.x == 0) {
      double wr = 0.0, wi = 0.0;
      if (tt > 0.0) {
        wr = tsr / tt;
        wi = tsi / tt;
      }
      if (!finite_d(wr) || !finite_d(wi)) {
        st[KI_ACTIVE] = 0;
        st[KI_FLAG] = FLAG_NONFINITE;
        return;
      }
      sc[KS_OMEGA] = wr;
      sc[KS_OMEGA + 1] = wi;
    }
    return;
  }
  // PHASE 3
  const double rhr = wave_sum_partials(part, ncols, nrb, 0, cr);
  const double rhi = CPLX ? wave_sum_partials(part, ncols, nrb, 0, cr + 1) : 0.0;
  const double rr = wave_sum_partials(part, ncols, nrb, 1, cr);
  if (threadIdx.x == 0) {
    st[KI_ITERS] += 1;
    sc[KS_RNRM2] = rr;
    sc[KS_LAST_RHR] = rhr;
    if (!finite_d(rr)) {
      st[KI_ACTIVE] = 0;
      st[KI_FLAG] = FLAG_NONFINITE;
      return;
    }
    if (rr <= sc[KS_TOL2] * sc[KS_BNRM2]) {
      st[KI_ACTIVE] = 0;
      st[KI_FLAG] = FLAG_CONVERGED;
      return;
    }
    const double rmin = sc[KS_RMIN];
    if (rr < 0.81 * sc[KS_RREF]) {      // norm dropped by 10 % since the reference
      st[KI_STALL] = 0;
      sc[KS_RREF] = rr;
    } else {
      st[KI_STALL] += 1;
    }
    if (rr < rmin) sc[KS_RMIN] = rr;
    if (rr > DIVERGE_RR * rmin) {
      st[KI_ACTIVE] = 0;
      st[KI_FLAG] = FLAG_DIVERGED;
      return;
    }
    if (st[KI_STALL] > stall_min && st[KI_STALL] > st[KI_ITERS] / stall_div) {
      st[KI_ACTIVE] = 0;
      st[KI_FLAG] = FLAG_STAGNATED;
      return;
    }
    const double wr = sc[KS_OMEGA], wi = sc[KS_OMEGA + 1];
    if (wr == 0.0 && wi == 0.0) {
      st[KI_ACTIVE] = 0;
      st[KI_FLAG] = FLAG_BREAKDOWN;
      return;
    }
    // beta = (rho_new / rho) (alpha / omega)
    double q1r, q1i, q2r, q2i;
    if (!CPLX) {
      q1r = rhr / sc[KS_RHO];
      q1i = 0.0;
      q2r = sc[KS_ALPHA] / wr;
      q2i = 0.0;
    } else {
      cdiv(rhr, rhi, sc[KS_RHO], sc[KS_RHO + 1], q1r, q1i);
      cdiv(sc[KS_ALPHA], sc[KS_ALPHA + 1], wr, wi, q2r, q2i);
    }
    const double br = q1r * q2r - q1i * q2i, bi = q1r * q2i + q1i * q2r;
    if ((rhr == 0.0 && rhi == 0.0) || !finite_d(br) || !finite_d(bi)) {
      st[KI_ACTIVE] = 0;
      st[KI_FLAG] = FLAG_BREAKDOWN;
      return;
    }
    sc[KS_BETA] = br;
    sc[KS_BETA + 1] = bi;
    sc[KS_RHO] = rhr;
    sc[KS_RHO + 1] = rhi;
  }
}

// Checkpoint (RESTORE = false): active columns whose current residual is the
// smallest checkpointed so far copy x -> xb.  Restore (RESTORE = true):
// columns stopped without convergence whose checkpoint is better copy
// xb -> x.  The per-column decision reads scalars that only this launch's
// first row block changes, and only towards an equal value, so every block
// takes the same decision.
template <typename T, bool RESTORE, bool CPLX>
__global__ void __launch_bounds__(256) k_bicg_ckpt(int n, int ncols, T* __restrict__ x, int64_t ldx,
                                                   T* __restrict__ xb, int64_t ld, double* __restrict__ scv,
                                                   const int* __restrict__ stv) {
  const int c = blockIdx.y;
  const int lc = CPLX ? c / 2 : c;
  double* sc = scv + (int64_t)lc * KS;
  const int* st = stv + (int64_t)lc * KI;
  const double rr = sc[KS_RNRM2], rk = sc[KS_RCKPT];
  bool go;
  if (!RESTORE) {
    go = st[KI_ACTIVE] != 0 && rr <= rk;
  } else {
    const int f = st[KI_FLAG];
    go = f != FLAG_CONVERGED && rk < rr;
  }
  if (!go) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    if (!RESTORE) xb[(int64_t)c * ld + i] = x[(int64_t)c * ldx + i];
    else x[(int64_t)c * ldx + i] = xb[(int64_t)c * ld + i];
  }
  if (!RESTORE && blockIdx.x == 0 && threadIdx.x == 0 && (!CPLX || (c % 2) == 0)) sc[KS_RCKPT] = rr;
}

template <typename T, bool RESTORE>
static void ckpt(Ctx* ctx, bool cplx, int n, int ncols, T* x, int64_t ldx, T* xb, int64_t ld, double* sc,
                 const int* st) {
  dim3 g(ceil_div(n, 256), ncols);
  if (cplx)
    hipLaunchKernelGGL((k_bicg_ckpt<T, RESTORE, true>), g, dim3(256), 0, ctx->stream, n, ncols, x, ldx, xb, ld, sc, st);
  else
    hipLaunchKernelGGL((k_bicg_ckpt<T, RESTORE, false>), g, dim3(256), 0, ctx->stream, n, ncols, x, ldx, xb, ld, sc,
                       st);
  KERNEL_CHECK();
}

// First half of a split MODE_BICG_P / MODE_BICG_S (see spmm_kernel.hpp): the
// input of the sparse product formed once per row, with the fused modes'
// formulas: p_new = r + beta (p - omega v) (r on a column's first iteration),
// or s = r - alpha v.
template <typename T, int CP, int WHICH, bool CPLX>
__global__ void __launch_bounds__(256) k_bicg_pre(SpmmArgs<T> a) {
  constexpr int NL = CPLX ? CP / 2 : CP;
  const int rb = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int i = rb * 256 + threadIdx.x;
  const int c0 = blockIdx.y * CP;
  if (i >= a.n) return;
  // loads of every column first (inactive ones read the first active column),
  // then the stores of the active columns
  bool act[NL], first[NL];
  int colq[NL];
  int qa = -1;
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int cr = c0 + (CPLX ? 2 * q : q);
    const int* st = a.st + (int64_t)(CPLX ? cr / 2 : cr) * KI;
    act[q] = cr < a.ncols && st[KI_ACTIVE] != 0;
    first[q] = act[q] && st[KI_ITERS] == 0;
    if (qa < 0 && act[q]) qa = q;
  }
  if (qa < 0) return;
#pragma unroll
  for (int q = 0; q < NL; ++q) colq[q] = act[q] ? c0 + (CPLX ? 2 * q : q) : c0 + (CPLX ? 2 * qa : qa);
  T rr[NL], ri[NL], vr[NL], vi[NL], pr[NL], pi[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int64_t o = (int64_t)colq[q] * a.ld + i;
    rr[q] = a.r[o];
    vr[q] = a.vold[o];
    pr[q] = WHICH == MODE_BICG_P ? a.pold[o] : (T)0;
    ri[q] = vi[q] = pi[q] = (T)0;
    if (CPLX) {
      ri[q] = a.r[o + a.ld];
      vi[q] = a.vold[o + a.ld];
      if (WHICH == MODE_BICG_P) pi[q] = a.pold[o + a.ld];
    }
  }
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    if (!act[q]) continue;
    const int cr = c0 + (CPLX ? 2 * q : q);
    const double* sc = a.sc + (int64_t)(CPLX ? cr / 2 : cr) * KS;
    const int64_t o = (int64_t)cr * a.ld + i;
    if (WHICH == MODE_BICG_P) {
      // the fused modes' formula; on a column's first iteration p = r
      const T br = (T)sc[KS_BETA], bi = (T)sc[KS_BETA + 1];
      const T wr = (T)sc[KS_OMEGA], wi = (T)sc[KS_OMEGA + 1];
      if (!CPLX) {
        a.pnew[o] = first[q] ? rr[q] : rr[q] + br * (pr[q] - wr * vr[q]);
      } else {
        const T ur = pr[q] - (wr * vr[q] - wi * vi[q]);
        const T ui = pi[q] - (wr * vi[q] + wi * vr[q]);
        a.pnew[o] = first[q] ? rr[q] : rr[q] + (br * ur - bi * ui);
        a.pnew[o + a.ld] = first[q] ? ri[q] : ri[q] + (br * ui + bi * ur);
      }
    } else {
      const T ar = (T)sc[KS_ALPHA], ai = (T)sc[KS_ALPHA + 1];
      if (!CPLX) {
        a.s[o] = rr[q] - ar * vr[q];
      } else {
        a.s[o] = rr[q] - (ar * vr[q] - ai * vi[q]);
        a.s[o + a.ld] = ri[q] - (ar * vi[q] + ai * vr[q]);
      }
    }
  }
}

template <typename T, int WHICH>
static void launch_pre(Ctx* ctx, const SellOp& op, bool cplx, SpmmArgs<T> a) {
  a.n = (int)op.n;
  const int k = a.ncols;
  if (k <= 0 || a.n <= 0) return;
  const int cp = k <= 2 ? 2 : (k <= 4 ? 4 : 8);
  dim3 g(spmm_rowblocks(a.n), ceil_div(k, cp));
  if (cplx) {
    if (cp == 2) hipLaunchKernelGGL((k_bicg_pre<T, 2, WHICH, true>), g, dim3(256), 0, ctx->stream, a);
    else if (cp == 4) hipLaunchKernelGGL((k_bicg_pre<T, 4, WHICH, true>), g, dim3(256), 0, ctx->stream, a);
    else hipLaunchKernelGGL((k_bicg_pre<T, 8, WHICH, true>), g, dim3(256), 0, ctx->stream, a);
  } else {
    if (cp == 2) hipLaunchKernelGGL((k_bicg_pre<T, 2, WHICH, false>), g, dim3(256), 0, ctx->stream, a);
    else if (cp == 4) hipLaunchKernelGGL((k_bicg_pre<T, 4, WHICH, false>), g, dim3(256), 0, ctx->stream, a);
    else hipLaunchKernelGGL((k_bicg_pre<T, 8, WHICH, false>), g, dim3(256), 0, ctx->stream, a);
  }
  KERNEL_CHECK();
}

// Split or fused BiCGStab products: split when the fused kernel's gathered
// vectors (3 for the p step) for the rows of one panel that a single XCD holds
// would fill more than half of that XCD's 4 MB L2.
static bool use_split(const Ctx* ctx, const SellOp& op, int ncols, bool cplx) {
  if (ctx->spmm_split == 1) return false;
  if (ctx->spmm_split == 2) return true;
  const int k = ncols;
  int cp = k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : 16;
  if (cplx && cp < 2) cp = 2;
  const double rows_per_xcd = double(op.n) / 8.0;
  const double ws = rows_per_xcd * cp * 3.0 * double(vec_bytes(op.prec));
  return ws > 2.0 * 1024 * 1024;
}

template <typename T, int CP, int UMODE, bool CPLX>
static void launch_elem(Ctx* ctx, const ElemArgs<T>& a) {
  dim3 g(spmm_rowblocks(a.n), ceil_div(a.ncols, CP));
  hipLaunchKernelGGL((k_bicg_elem<T, CP, UMODE, CPLX>), g, dim3(256), 0, ctx->stream, a);
  KERNEL_CHECK();
}

template <typename T, int UMODE>
static void elem(Ctx* ctx, bool cplx, const ElemArgs<T>& a) {
  const int k = a.ncols;
  if (cplx) {
    if (k <= 2) launch_elem<T, 2, UMODE, true>(ctx, a);
    else if (k <= 4) launch_elem<T, 4, UMODE, true>(ctx, a);
    else launch_elem<T, 8, UMODE, true>(ctx, a);
  } else {
    if (k <= 1) launch_elem<T, 1, UMODE, false>(ctx, a);
    else if (k <= 2) launch_elem<T, 2, UMODE, false>(ctx, a);
    else if (k <= 4) launch_elem<T, 4, UMODE, false>(ctx, a);
    else launch_elem<T, 8, UMODE, false>(ctx, a);
  }
}

template <int PHASE>
static void scalar(Ctx* ctx, bool cplx, double* sc, int* st, const double* part, int ncols, int nrb, double tol2,
                   bool fp32) {
  const int nl = cplx ? ncols / 2 : ncols;
  int smin = fp32 ? STALL_MAX_F32 : STALL_MAX, sdiv = fp32 ? 8 : 4;
  if (ctx->krylov_patient) {
    smin = STALL_MAX_PATIENT;
    sdiv = 2;
  }
  if (cplx)
    hipLaunchKernelGGL((k_bicg_scalar<PHASE, true>), dim3(nl), dim3(SCALAR_THREADS), 0, ctx->stream, sc, st, part,
                       ncols, nrb, tol2, smin, sdiv);
  else
    hipLaunchKernelGGL((k_bicg_scalar<PHASE, false>), dim3(nl), dim3(SCALAR_THREADS), 0, ctx->stream, sc, st, part,
                       ncols, nrb, tol2, smin, sdiv);
  KERNEL_CHECK();
}

template <typename T>
static KrylovResult bicgstab_core(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols, const T* b,
                                  int64_t ldb, T* x, int64_t ldx, double tol, int maxit, int check_every,
                                  const std::vector<int>* groups, const std::vector<double>* target2) {
  KrylovResult res;
  if (ncols <= 0) return res;
  const bool cplx = pi != 0.0;
  if (cplx && (ncols % 2)) fail(CARE_ERR_ARG, "complex solve needs an even number of real columns");
  const int64_t n = op.n;
  const int64_t ld = pad_ld(n);
  const char* tr_env = std::getenv("MPCARE_TRACE");
  const bool trace = tr_env && std::atoi(tr_env) >= 2;
  int nl = cplx ? ncols / 2 : ncols;
  const int per = cplx ? 2 : 1;
  const int nl0 = nl;
  const int nrb = spmm_rowblocks(n);
  const size_t panel = (size_t)ld * ncols;
  DBuf<T> r(ctx, panel), P0(ctx, panel), P1(ctx, panel), V0(ctx, panel), V1(ctx, panel), S(ctx, panel),
      Tt(ctx, panel), Xb(ctx, panel);
  dzero(ctx, Xb.get(), panel * sizeof(T));
  DBuf<double> part(ctx, (size_t)2 * ncols * nrb);
  DBuf<double> sc(ctx, (size_t)nl * KS);
  DBuf<int> st(ctx, (size_t)nl * KI);
  T* Pb[2] = {P0.get(), P1.get()};
  T* Vb[2] = {V0.get(), V1.get()};
  const double tol2 = tol * tol;
  // Column compaction: once the columns still iterating fit in fewer
  // 16-column panels, they are gathered to the front of fresh panels and the
  // solve continues on those alone (the sparse products and elementwise
  // passes work in panels, and a panel with one active column costs nearly as
  // much as a full one).  Every column's arithmetic is unchanged.  orig[c]: the caller's logical
  // column of working column c; xcur / bcur: the working x and right-hand
  // side (the caller's arrays until the first compaction); fsc / fst: final
  // scalars and status of the columns that left the working set.
  std::vector<int> orig(nl);
  for (int c = 0; c < nl; ++c) orig[c] = c;
  T* xcur = x;
  int64_t ldxcur = ldx;
  const T* bcur = b;
  int64_t ldbcur = ldb;
  DBuf<T> xw, bw;
  std::vector<double> fsc((size_t)nl0 * KS);
  std::vector<int> fst((size_t)nl0 * KI);

  ElemArgs<T> ea;
  ea.n = (int)n;
  ea.ncols = ncols;
  ea.nrb = nrb;
  ea.ld = ld;
  ea.b = b;
  ea.ldb = ldb;
  ea.x = x;
  ea.ldx = ldx;
  ea.r = r.get();
  ea.sc = sc.get();
  ea.st = st.get();
  ea.part = part.get();
  auto dump = [&](const char* tag) {   // MPCARE_TRACE: scalars of the first columns
    std::vector<double> hs((size_t)nl * KS);
    std::vector<int> hi((size_t)nl * KI);
    d2h(ctx, hs.data(), sc.get(), hs.size() * sizeof(double));
    d2h(ctx, hi.data(), st.get(), hi.size() * sizeof(int));
    for (int c = 0; c < std::min(nl, 2); ++c) {
      const double* v = &hs[(size_t)c * KS];
      const int* s = &hi[(size_t)c * KI];
      std::fprintf(stderr,
                   "[bicg %s col %d] rho %.3e %.3e alpha %.3e %.3e omega %.3e %.3e beta %.3e %.3e bb %.3e rr %.3e "
                   "rhr %.3e act %d it %d flag %d\n",
                   tag, c, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], v[9], v[10], s[0], s[1], s[2]);
    }
  };
  elem<T, UPD_INIT>(ctx, cplx, ea);
  scalar<0>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2, sizeof(T) == 4);
  if (groups || target2) {
    // tolerance relative to the largest right-hand side of each group, or an
    // absolute target ||r_c||^2 <= target2[c] (restarts)
    if ((groups && (int)groups->size() != nl) || (target2 && (int)target2->size() != nl))
      fail(CARE_ERR_ARG, "per-column tolerances do not match the columns");
    std::vector<double> hs((size_t)nl * KS);
    std::vector<int> hi((size_t)nl * KI);
    d2h(ctx, hs.data(), sc.get(), hs.size() * sizeof(double));
    d2h(ctx, hi.data(), st.get(), hi.size() * sizeof(int));
    std::map<int, double> gmax;
    if (groups)
      for (int c = 0; c < nl; ++c)
        gmax[(*groups)[c]] = std::max(gmax[(*groups)[c]], hs[(size_t)c * KS + KS_BNRM2]);
    for (int c = 0; c < nl; ++c) {
      const double bb = hs[(size_t)c * KS + KS_BNRM2];
      if (bb <= 0.0 || !hi[(size_t)c * KI + KI_ACTIVE]) continue;
      const double t2 = target2 ? (*target2)[c] / bb : tol2 * gmax[(*groups)[c]] / bb;
      hs[(size_t)c * KS + KS_TOL2] = t2;
      if (t2 >= 1.0) {                 // x = 0 already meets the group tolerance
        hi[(size_t)c * KI + KI_ACTIVE] = 0;
        hi[(size_t)c * KI + KI_FLAG] = FLAG_CONVERGED;
      }
    }
    h2d(ctx, sc.get(), hs.data(), hs.size() * sizeof(double));
    h2d(ctx, st.get(), hi.data(), hi.size() * sizeof(int));
  }
  if (trace) dump("S0");

  std::vector<int> hst((size_t)nl * KI);
  int it = 0;
  check_every = check_every > 0 ? check_every : 8;
  int next_check = 1;   // first poll right after one iteration (trivial columns)
  bool done = false;
  const bool split = use_split(ctx, op, ncols, cplx);
  auto iteration = [&](int it) {
    SpmmArgs<T> a1;
    a1.ncols = ncols;
    a1.sr = pr;
    a1.si = pi;
    a1.ld = ld;
    a1.r = r.get();
    a1.pold = Pb[it & 1];
    a1.vold = Vb[it & 1];
    a1.pnew = Pb[(it + 1) & 1];
    a1.vnew = Vb[(it + 1) & 1];
    a1.rhat = bcur;
    a1.ldrhat = ldbcur;
    a1.sc = sc.get();
    a1.st = st.get();
    a1.part = part.get();
    if (split) {
      launch_pre<T, MODE_BICG_P>(ctx, op, cplx, a1);
      SpmmArgs<T> d1 = a1;
      d1.X = a1.pnew;
      d1.ldx = ld;
      d1.Y = a1.vnew;
      d1.ldy = ld;
      launch_spmm<T>(ctx, op, MODE_DOT1, cplx, d1);
    } else {
      launch_spmm<T>(ctx, op, MODE_BICG_P, cplx, a1);
    }
    scalar<1>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2, sizeof(T) == 4);
    if (trace && it < 3) dump("S1");

    SpmmArgs<T> a2 = a1;
    a2.vold = Vb[(it + 1) & 1];
    a2.s = S.get();
    a2.t = Tt.get();
    if (split) {
      launch_pre<T, MODE_BICG_S>(ctx, op, cplx, a2);
      SpmmArgs<T> d2 = a2;
      d2.X = a2.s;
      d2.ldx = ld;
      d2.Y = a2.t;
      d2.ldy = ld;
      launch_spmm<T>(ctx, op, MODE_DOT2, cplx, d2);
    } else {
      launch_spmm<T>(ctx, op, MODE_BICG_S, cplx, a2);
    }
    scalar<2>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2, sizeof(T) == 4);
    if (trace && it < 3) dump("S2");

    ElemArgs<T> e3 = ea;
    e3.p = Pb[(it + 1) & 1];
    e3.s = S.get();
    e3.t = Tt.get();
    elem<T, UPD_XR>(ctx, cplx, e3);
    scalar<3>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2, sizeof(T) == 4);
    if (trace && it < 3) dump("S3");
  };
  // Profiling: the bytes of the launches since the previous poll are counted
  // for the columns still active at this poll, a lower bound for each of
  // them (columns only ever leave the active set).
  bool first_chunk = true;
  auto account = [&](int active) {
    if (!ctx->spmm_defer) return;
    const int kr = active * (cplx ? 2 : 1);
    for (int md = MODE_BICG_P; md <= MODE_DOT2; ++md) {
      const int passes = md == MODE_BICG_P ? spmm_vec_passes(md, first_chunk) : spmm_vec_passes(md);
      ctx->spmm_bytes += double(ctx->spmm_pending[md]) * op.bytes(kr, passes);
      ctx->spmm_pending[md] = 0;
    }
    first_chunk = false;
  };
  auto poll = [&]() {
    ckpt<T, false>(ctx, cplx, (int)n, ncols, xcur, ldxcur, Xb.get(), ld, sc.get(), st.get());
    d2h(ctx, hst.data(), st.get(), hst.size() * sizeof(int));
    int active = 0;
    for (int c = 0; c < nl; ++c) active += hst[(size_t)c * KI + KI_ACTIVE];
    account(active);
    done = active == 0;
  };
  // Compaction at a poll (hst holds the status of the working columns; `it`
  // iterations are done, so p and v live in Pb[it & 1], Vb[it & 1]).
  auto compact = [&]() -> bool {
    if (!ctx->krylov_compact) return false;
    std::vector<int> keep;
    for (int c = 0; c < nl; ++c)
      if (hst[(size_t)c * KI + KI_ACTIVE]) keep.push_back(c);
    const int na = (int)keep.size();
    if (na == 0 || ceil_div(na * per, 16) >= ceil_div(nl * per, 16)) return false;   // no panel saved
    std::vector<double> hs((size_t)nl * KS);
    d2h(ctx, hs.data(), sc.get(), hs.size() * sizeof(double));
    // columns leaving the working set are final: their scalars are kept, and
    // x (or the better checkpoint, as the final restore would choose it) goes
    // to the caller's column
    for (int c = 0; c < nl; ++c) {
      if (hst[(size_t)c * KI + KI_ACTIVE]) continue;
      const int o = orig[c];
      std::copy(hs.begin() + (size_t)c * KS, hs.begin() + (size_t)(c + 1) * KS, fsc.begin() + (size_t)o * KS);
      std::copy(hst.begin() + (size_t)c * KI, hst.begin() + (size_t)(c + 1) * KI, fst.begin() + (size_t)o * KI);
      const double* v = &hs[(size_t)c * KS];
      const bool restore = hst[(size_t)c * KI + KI_FLAG] != FLAG_CONVERGED && v[KS_RCKPT] < v[KS_RNRM2];
      for (int e = 0; e < per; ++e) {
        const T* src = restore ? Xb.get() + (int64_t)(c * per + e) * ld : xcur + (int64_t)(c * per + e) * ldxcur;
        d2d(ctx, x + (int64_t)(o * per + e) * ldx, src, (size_t)n * sizeof(T));
      }
    }
    const int ncn = na * per;
    std::vector<int> map(ncn);
    for (int j = 0; j < na; ++j)
      for (int e = 0; e < per; ++e) map[j * per + e] = keep[j] * per + e;
    auto gather = [&](const T* src, int64_t lds) {
      DBuf<T> t(ctx, (size_t)ld * ncn);
      copy_cols<T, T>(ctx, n, ncn, src, lds, t.get(), ld, map.data());
      return t;
    };
    const int cur = it & 1;
    DBuf<T> nr = gather(r.get(), ld), np = gather(Pb[cur], ld), nv = gather(Vb[cur], ld);
    DBuf<T> nxb = gather(Xb.get(), ld), nx = gather(xcur, ldxcur), nb = gather(bcur, ldbcur);
    r = std::move(nr);
    Xb = std::move(nxb);
    xw = std::move(nx);
    bw = std::move(nb);
    if (cur == 0) {
      P0 = std::move(np);
      V0 = std::move(nv);
    } else {
      P1 = std::move(np);
      V1 = std::move(nv);
    }
    Pb[0] = P0.get();
    Pb[1] = P1.get();
    Vb[0] = V0.get();
    Vb[1] = V1.get();
    xcur = xw.get();
    ldxcur = ld;
    bcur = bw.get();
    ldbcur = ld;
    std::vector<double> hs2((size_t)na * KS);
    std::vector<int> hi2((size_t)na * KI);
    std::vector<int> no(na);
    for (int j = 0; j < na; ++j) {
      std::copy(hs.begin() + (size_t)keep[j] * KS, hs.begin() + (size_t)(keep[j] + 1) * KS, hs2.begin() + (size_t)j * KS);
      std::copy(hst.begin() + (size_t)keep[j] * KI, hst.begin() + (size_t)(keep[j] + 1) * KI,
                hi2.begin() + (size_t)j * KI);
      no[j] = orig[keep[j]];
    }
    h2d(ctx, sc.get(), hs2.data(), hs2.size() * sizeof(double));
    h2d(ctx, st.get(), hi2.data(), hi2.size() * sizeof(int));
    orig = no;
    nl = na;
    ncols = ncn;
    hst.assign((size_t)nl * KI, 0);
    std::copy(hi2.begin(), hi2.end(), hst.begin());
    ea.ncols = ncols;
    ea.b = bcur;
    ea.ldb = ldbcur;
    ea.x = xcur;
    ea.ldx = ldxcur;
    ea.r = r.get();
    res.compactions += 1;
    ctx->krylov_compactions += 1;
    return true;
  };
  // The first check_every iterations (and everything when profiling) are
  // launched directly, with polls after the first iteration and then every
  // check_every iterations.  The steady state runs chunks of CHUNK iterations
  // plus the checkpoint kernel, with a host poll after each chunk: replayed as
  // one captured HIP graph (no memset nodes: the loop holds kernels only), or,
  // where graphs are off (batch worker contexts), the same launches issued
  // directly, so both give the same results.  A chunk never runs past maxit:
  // the iterations left below a whole chunk are launched directly.
  const int CHUNK = 8;
  const bool chunked = !ctx->profile && !trace && maxit > 2 * CHUNK;
  const bool graphs = chunked && ctx->krylov_graphs;
  ctx->spmm_defer = ctx->profile != 0;
  for (int md = 0; md < 5; ++md) ctx->spmm_pending[md] = 0;
  auto direct_until = [&](int limit, bool stop_at_check) {
    while (it < limit && !done && (!stop_at_check || it < check_every)) {
      iteration(it);
      ++it;
      if (it >= next_check || it >= limit) {
        poll();
        next_check = it + check_every;
        if (!done && it < limit) compact();
      }
    }
  };
  direct_until(maxit, chunked);
  if (!done && chunked && it + CHUNK + 1 <= maxit) {
    if (it % 2) {          // the ping-pong buffers repeat with period 2
      iteration(it);
      ++it;
    }
    // a compaction changes the launches: the chunk is captured again (the
    // polls stay every CHUNK iterations, so the checkpoints are those of an
    // uncompacted solve)
    bool recapture = true;
    while (recapture && !done && it + CHUNK <= maxit) {
      recapture = false;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      int64_t dcalls = 0;
      double dbytes = 0.0;
      if (graphs) {
        const int64_t calls0 = ctx->spmm_calls;
        const double bytes0 = ctx->spmm_bytes;
        HIP_CHECK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        for (int c = 0; c < CHUNK; ++c) iteration(it + c);
        ckpt<T, false>(ctx, cplx, (int)n, ncols, xcur, ldxcur, Xb.get(), ld, sc.get(), st.get());
        HIP_CHECK(hipStreamEndCapture(ctx->stream, &graph));
        dcalls = ctx->spmm_calls - calls0;
        dbytes = ctx->spmm_bytes - bytes0;
        ctx->spmm_calls = calls0;
        ctx->spmm_bytes = bytes0;
        HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      }
      while (it + CHUNK <= maxit && !done) {
        if (graphs) {
          HIP_CHECK(hipGraphLaunch(exec, ctx->stream));
          ctx->spmm_calls += dcalls;
          ctx->spmm_bytes += dbytes;
        } else {
          for (int c = 0; c < CHUNK; ++c) iteration(it + c);
          ckpt<T, false>(ctx, cplx, (int)n, ncols, xcur, ldxcur, Xb.get(), ld, sc.get(), st.get());
        }
        it += CHUNK;
        d2h(ctx, hst.data(), st.get(), hst.size() * sizeof(int));
        int active = 0;
        for (int c = 0; c < nl; ++c) active += hst[(size_t)c * KI + KI_ACTIVE];
        done = active == 0;
        if (!done && it < maxit && compact()) {
          recapture = true;
          break;
        }
      }
      if (graphs) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
      }
    }
    next_check = it + check_every;
  }
  direct_until(maxit, false);
  account(0);
  ctx->spmm_defer = false;
  // columns that stopped without converging fall back to their best checkpoint
  ckpt<T, true>(ctx, cplx, (int)n, ncols, xcur, ldxcur, Xb.get(), ld, sc.get(), st.get());
  {
    std::vector<double> hsc((size_t)nl * KS);
    d2h(ctx, hsc.data(), sc.get(), hsc.size() * sizeof(double));
    d2h(ctx, hst.data(), st.get(), hst.size() * sizeof(int));
    for (int c = 0; c < nl; ++c) {
      const int o = orig[c];
      std::copy(hsc.begin() + (size_t)c * KS, hsc.begin() + (size_t)(c + 1) * KS, fsc.begin() + (size_t)o * KS);
      std::copy(hst.begin() + (size_t)c * KI, hst.begin() + (size_t)(c + 1) * KI, fst.begin() + (size_t)o * KI);
      if (xcur != x)
        for (int e = 0; e < per; ++e)
          d2d(ctx, x + (int64_t)(o * per + e) * ldx, xcur + (int64_t)(c * per + e) * ldxcur, (size_t)n * sizeof(T));
    }
    ctx->sync();
  }
  for (int c = 0; c < nl0; ++c) {
    const int* s = &fst[(size_t)c * KI];
    const double* v = &fsc[(size_t)c * KS];
    res.max_iters = std::max(res.max_iters, s[KI_ITERS]);
    ctx->krylov_iters += s[KI_ITERS];
    const double rfin = s[KI_FLAG] == FLAG_CONVERGED ? v[KS_RNRM2] : std::min(v[KS_RNRM2], v[KS_RCKPT]);
    const double rel = v[KS_BNRM2] > 0 ? std::sqrt(rfin / v[KS_BNRM2]) : 0.0;
    res.worst_relres = std::max(res.worst_relres, rel);
    if (s[KI_FLAG] == FLAG_NONFINITE) fail(CARE_ERR_NONFINITE, "non-finite value in the Krylov iteration");
    const bool ok = s[KI_FLAG] == FLAG_CONVERGED || rfin <= v[KS_TOL2] * v[KS_BNRM2];
    res.col_ok.push_back(ok ? 1 : 0);
    res.col_relres.push_back(rel);
    res.col_bnorm.push_back(std::sqrt(std::max(v[KS_BNRM2], 0.0)));
    if (!ok) {
      res.unconverged += 1;
      if (s[KI_FLAG] == FLAG_BREAKDOWN) res.breakdown += 1;
    }
  }
  return res;
}

// Restarted solve: columns that stop above their tolerance (stagnation,
// breakdown, divergence or the iteration cap) are solved again on their
// true residual b - M x with a fresh shadow vector, up to MAX_RESTARTS
// rounds, and the correction is added to x.
constexpr int MAX_RESTARTS = 2;

// per-column sums of squares, one partial per block (blockDim 256)
template <typename T>
__global__ void __launch_bounds__(256) k_colsumsq(int64_t n, const T* __restrict__ x, int64_t ldx,
                                                  double* __restrict__ part) {
  const int64_t c = blockIdx.y;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = (double)x[c * ldx + i];
    s += v * v;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c * gridDim.x + blockIdx.x] = sh[0];
}

template <typename T>
static std::vector<double> col_norms(Ctx* ctx, int64_t n, int ncols, const T* x, int64_t ldx) {
  const int nb = (int)std::min<int64_t>(64, ceil_div(n, 256));
  DBuf<double> part(ctx, (size_t)nb * ncols);
  hipLaunchKernelGGL(k_colsumsq<T>, dim3(nb, ncols), dim3(256), 0, ctx->stream, n, x, ldx, part.get());
  KERNEL_CHECK();
  std::vector<double> h((size_t)nb * ncols), out(ncols, 0.0);
  d2h(ctx, h.data(), part.get(), h.size() * sizeof(double));
  for (int c = 0; c < ncols; ++c) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += h[(size_t)c * nb + b];
    out[c] = std::sqrt(s);
  }
  return out;
}

template <typename T>
KrylovResult bicgstab(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols, const T* b, int64_t ldb, T* x,
                      int64_t ldx, double tol, int maxit, int check_every, const std::vector<int>* groups) {
  if (op.dense) return dense_solve<T>(ctx, op, pr, pi, ncols, b, ldb, x, ldx);
  if (ctx->krylov_rb && rb_usable(op, pr, pi))
    return bicgstab_rb<T>(ctx, op, pr, pi, ncols, b, ldb, x, ldx, tol, maxit, check_every, groups);
  if (ctx->krylov_method == 1 && pi == 0.0) {
    const int restart = ctx->krylov_restart > 0 ? ctx->krylov_restart : (sizeof(T) == 8 ? 50 : 30);
    return gmres<T>(ctx, op, pr, ncols, b, ldb, x, ldx, tol, maxit, restart, groups);
  }
  KrylovResult res = bicgstab_core<T>(ctx, op, pr, pi, ncols, b, ldb, x, ldx, tol, maxit, check_every, groups,
                                      nullptr);
  const bool cplx = pi != 0.0;
  const int per = cplx ? 2 : 1;
  const int nl = ncols / per;
  const int64_t n = op.n, ld = pad_ld(n);
  // absolute target of each column: ||r_c||^2 <= tgt2_c
  std::vector<double> tgt2(nl);
  std::map<int, double> gmax;
  if (groups)
    for (int c = 0; c < nl; ++c) gmax[(*groups)[c]] = std::max(gmax[(*groups)[c]], res.col_bnorm[c]);
  for (int c = 0; c < nl; ++c) {
    const double ref = groups ? gmax[(*groups)[c]] : res.col_bnorm[c];
    tgt2[c] = tol * tol * ref * ref;
  }
  // A column that stopped near the attainable accuracy of the working
  // precision gains nothing from a restart: the true residual b - M x
  // evaluated in precision T carries rounding errors of about
  // u_T (||A^T||_inf + |p|) ||x_c|| (and BiCGStab's recursive residual drifts
  // from it by as much), so a column within 10 times that level of ||b_c||,
  // or within 1e4 u_T, is left as it is.
  const double u_t = sizeof(T) == 8 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
  std::vector<double> floor_rel(nl, 1e4 * u_t);
  if (op.norm_one > 0.0 && res.unconverged > 0) {
    const std::vector<double> xn = col_norms<T>(ctx, n, ncols, x, ldx);
    const double mnorm = op.norm_one + std::hypot(pr, pi);
    for (int c = 0; c < nl; ++c) {
      const double xx = cplx ? std::hypot(xn[2 * c], xn[2 * c + 1]) : xn[c];
      if (res.col_bnorm[c] > 0.0)
        floor_rel[c] = std::max(floor_rel[c], 10.0 * u_t * mnorm * xx / res.col_bnorm[c]);
    }
  }
  for (int round = 0; round < MAX_RESTARTS; ++round) {
    // the restart rounds share the caller's iteration budget
    const int left = maxit - res.max_iters;
    if (left <= 0) break;
    std::vector<int> cols;
    for (int c = 0; c < nl; ++c)
      if (!res.col_ok[c] && res.col_relres[c] > floor_rel[c]) cols.push_back(c);
    if (cols.empty()) break;
    const int nc = (int)cols.size(), ncr = nc * per;
    std::vector<int> map(ncr);
    for (int j = 0; j < nc; ++j)
      for (int e = 0; e < per; ++e) map[j * per + e] = cols[j] * per + e;
    DBuf<T> Xc(ctx, (size_t)ld * ncr), Rc(ctx, (size_t)ld * ncr), Bc(ctx, (size_t)ld * ncr), D(ctx, (size_t)ld * ncr);
    copy_cols<T, T>(ctx, n, ncr, x, ldx, Xc.get(), ld, map.data());
    copy_cols<T, T>(ctx, n, ncr, b, ldb, Bc.get(), ld, map.data());
    spmm_plain(ctx, op, pr, pi, Xc.get(), ld, ncr, Rc.get(), ld);
    axpby<T>(ctx, n, ncr, 1.0, Bc.get(), ld, -1.0, Rc.get(), ld);    // Rc = b - M x
    std::vector<double> ct2(nc);
    for (int j = 0; j < nc; ++j) ct2[j] = tgt2[cols[j]];
    KrylovResult r2 = bicgstab_core<T>(ctx, op, pr, pi, ncr, Rc.get(), ld, D.get(), ld, tol, left, check_every,
                                       nullptr, &ct2);
    for (int e = 0; e < ncr; ++e)
      axpby<T>(ctx, n, 1, 1.0, D.get() + (int64_t)e * ld, ld, 1.0, x + (int64_t)map[e] * ldx, ldx);
    res.max_iters += r2.max_iters;
    res.restarts += 1;
    for (int j = 0; j < nc; ++j) {
      const int c = cols[j];
      res.col_ok[c] = r2.col_ok[j];
      const double rn = r2.col_relres[j] * r2.col_bnorm[j];
      res.col_relres[c] = res.col_bnorm[c] > 0 ? rn / res.col_bnorm[c] : 0.0;
    }
  }
  res.unconverged = 0;
  res.worst_relres = 0;
  for (int c = 0; c < nl; ++c) {
    res.unconverged += res.col_ok[c] ? 0 : 1;
    res.worst_relres = std::max(res.worst_relres, res.col_relres[c]);
  }
  return res;
}

template KrylovResult bicgstab<double>(Ctx*, const SellOp&, double, double, int, const double*, int64_t, double*,
                                       int64_t, double, int, int, const std::vector<int>*);
template KrylovResult bicgstab<float>(Ctx*, const SellOp&, double, double, int, const float*, int64_t, float*,
                                      int64_t, double, int, int, const std::vector<int>*);

}  // namespace mpcare
