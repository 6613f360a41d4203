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

namespace mpcare {

enum { FLAG_NONE = 0, FLAG_CONVERGED = 1, FLAG_BREAKDOWN = 2, FLAG_NONFINITE = 3, FLAG_STAGNATED = 4, FLAG_DIVERGED = 5 };
// a column stops when its residual norm has not dropped by 10 % for
// STALL_MAX iterations (the attainable accuracy of the working precision is
// reached), or when it exceeds 1e3 x the smallest residual met (divergence);
// it then returns the best checkpointed iterate
constexpr int STALL_MAX = 200;
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

#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int cr = c0 + (CPLX ? 2 * q : q);
    if (cr >= a.ncols || i >= a.n) continue;
    const int lc = CPLX ? cr / 2 : cr;
    const int64_t ob = (int64_t)cr * a.ldb + i, ox = (int64_t)cr * a.ldx + i, o = (int64_t)cr * a.ld + i;
    if (UMODE == UPD_INIT) {
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
    } else {
      if (a.st[(int64_t)lc * KI + KI_ACTIVE] == 0) continue;
      const double* sc = a.sc + (int64_t)lc * KS;
      if (!CPLX) {
        const T al = (T)sc[KS_ALPHA], om = (T)sc[KS_OMEGA];
        const T sv = a.s[o], tv = a.t[o];
        a.x[ox] += al * a.p[o] + om * sv;
        const T rv = sv - om * tv;
        a.r[o] = rv;
        dots[q] = a.b[ob] * rv;             // <rhat, r>
        dots[CP + q] = rv * rv;             // <r, r>
      } else {
        const T alr = (T)sc[KS_ALPHA], ali = (T)sc[KS_ALPHA + 1];
        const T omr = (T)sc[KS_OMEGA], omi = (T)sc[KS_OMEGA + 1];
        const T pr = a.p[o], pim = a.p[o + a.ld];
        const T sr = a.s[o], sim = a.s[o + a.ld];
        const T tr = a.t[o], tim = a.t[o + a.ld];
        a.x[ox] += (alr * pr - ali * pim) + (omr * sr - omi * sim);
        a.x[ox + a.ldx] += (alr * pim + ali * pr) + (omr * sim + omi * sr);
        const T rr = sr - (omr * tr - omi * tim);
        const T ri = sim - (omr * tim + omi * tr);
        a.r[o] = rr;
        a.r[o + a.ld] = ri;
        const T hr = a.b[ob], hi = a.b[ob + a.ldb];
        dots[2 * q] = hr * rr + hi * ri;          // conj(rhat) r
        dots[2 * q + 1] = hr * ri - hi * rr;
        dots[CP + 2 * q] = rr * rr + ri * ri;     // |r|^2
        dots[CP + 2 * q + 1] = (T)0;
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
__device__ __forceinline__ double wave_sum_partials(const double* __restrict__ part, int ncols, int nrb, int dot,
                                                    int c) {
  const double* p = part + ((int64_t)dot * ncols + c) * nrb;
  double s = 0.0;
  for (int rb = threadIdx.x; rb < nrb; rb += 64) s += p[rb];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
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
__global__ void __launch_bounds__(64) k_bicg_scalar(double* __restrict__ scv, int* __restrict__ stv,
                                                    const double* __restrict__ part, int ncols, int nrb, double tol2) {
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
    if (rr <= tol2 * sc[KS_BNRM2]) {
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
    if (st[KI_STALL] > STALL_MAX) {
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
static void scalar(Ctx* ctx, bool cplx, double* sc, int* st, const double* part, int ncols, int nrb, double tol2) {
  const int nl = cplx ? ncols / 2 : ncols;
  if (cplx)
    hipLaunchKernelGGL((k_bicg_scalar<PHASE, true>), dim3(nl), dim3(64), 0, ctx->stream, sc, st, part, ncols, nrb, tol2);
  else
    hipLaunchKernelGGL((k_bicg_scalar<PHASE, false>), dim3(nl), dim3(64), 0, ctx->stream, sc, st, part, ncols, nrb, tol2);
  KERNEL_CHECK();
}

template <typename T>
KrylovResult bicgstab(Ctx* ctx, const SellOp& op, double pr, double pi, int ncols, const T* b, int64_t ldb, T* x,
                      int64_t ldx, double tol, int maxit, int check_every) {
  KrylovResult res;
  if (ncols <= 0) return res;
  const bool cplx = pi != 0.0;
  if (cplx && (ncols % 2)) fail(CARE_ERR_ARG, "complex solve needs an even number of real columns");
  const int64_t n = op.n;
  const int64_t ld = pad_ld(n);
  const char* tr_env = std::getenv("MPCARE_TRACE");
  const bool trace = tr_env && std::atoi(tr_env) >= 2;
  const int nl = cplx ? ncols / 2 : ncols;
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
  scalar<0>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2);
  if (trace) dump("S0");

  std::vector<int> hst((size_t)nl * KI);
  int it = 0;
  check_every = check_every > 0 ? check_every : 8;
  int next_check = 1;   // first poll right after one iteration (trivial columns)
  bool done = false;
  while (it < maxit && !done) {
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
    a1.rhat = b;
    a1.ldrhat = ldb;
    a1.sc = sc.get();
    a1.st = st.get();
    a1.part = part.get();
    launch_spmm<T>(ctx, op, MODE_BICG_P, cplx, a1);
    scalar<1>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2);
    if (trace && it < 3) dump("S1");

    SpmmArgs<T> a2 = a1;
    a2.vold = Vb[(it + 1) & 1];
    a2.s = S.get();
    a2.t = Tt.get();
    launch_spmm<T>(ctx, op, MODE_BICG_S, cplx, a2);
    scalar<2>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2);
    if (trace && it < 3) dump("S2");

    ElemArgs<T> e3 = ea;
    e3.p = Pb[(it + 1) & 1];
    e3.s = S.get();
    e3.t = Tt.get();
    elem<T, UPD_XR>(ctx, cplx, e3);
    scalar<3>(ctx, cplx, sc.get(), st.get(), part.get(), ncols, nrb, tol2);
    if (trace && it < 3) dump("S3");
    ++it;

    if (it >= next_check || it >= maxit) {
      ckpt<T, false>(ctx, cplx, (int)n, ncols, x, ldx, Xb.get(), ld, sc.get(), st.get());
      d2h(ctx, hst.data(), st.get(), hst.size() * sizeof(int));
      int active = 0;
      for (int c = 0; c < nl; ++c) active += hst[(size_t)c * KI + KI_ACTIVE];
      done = active == 0;
      next_check = it + check_every;
    }
  }
  // columns that stopped without converging fall back to their best checkpoint
  ckpt<T, true>(ctx, cplx, (int)n, ncols, x, ldx, Xb.get(), ld, sc.get(), st.get());
  std::vector<double> hsc((size_t)nl * KS);
  d2h(ctx, hsc.data(), sc.get(), hsc.size() * sizeof(double));
  d2h(ctx, hst.data(), st.get(), hst.size() * sizeof(int));
  for (int c = 0; c < nl; ++c) {
    const int* s = &hst[(size_t)c * KI];
    const double* v = &hsc[(size_t)c * KS];
    res.max_iters = std::max(res.max_iters, s[KI_ITERS]);
    ctx->krylov_iters += s[KI_ITERS];
    const double rfin = s[KI_FLAG] == FLAG_CONVERGED ? v[KS_RNRM2] : std::min(v[KS_RNRM2], v[KS_RCKPT]);
    const double rel = v[KS_BNRM2] > 0 ? std::sqrt(rfin / v[KS_BNRM2]) : 0.0;
    res.worst_relres = std::max(res.worst_relres, rel);
    if (s[KI_FLAG] == FLAG_NONFINITE) fail(CARE_ERR_NONFINITE, "non-finite value in the Krylov iteration");
    if (s[KI_FLAG] != FLAG_CONVERGED) {
      if (rel > tol) res.unconverged += 1;
      if (s[KI_FLAG] == FLAG_BREAKDOWN) res.breakdown += 1;
    }
  }
  return res;
}

template KrylovResult bicgstab<double>(Ctx*, const SellOp&, double, double, int, const double*, int64_t, double*,
                                       int64_t, double, int, int);
template KrylovResult bicgstab<float>(Ctx*, const SellOp&, double, double, int, const float*, int64_t, float*,
                                      int64_t, double, int, int);

}  // namespace mpcare
