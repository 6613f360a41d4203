// SELL-64 sparse-product kernel template (gfx950, wave64).
//
// One thread owns one row i of M = A^T + p I and a panel of CP real columns;
// a wavefront owns one SELL slice, so the column-index and value loads of a
// step are 64 consecutive entries, and the gathers X[j, c] of a stencil-like
// matrix are contiguous across lanes because neighbouring rows have
// neighbouring column indices.  Workgroups (256 rows) are remapped so that
// consecutive row blocks run on the same XCD and share its L2.
//
// The same body serves three input/epilogue modes:
//   MODE_PLAIN   y = (A^T + p I) x
//   MODE_BICG_P  BiCGStab search direction formed on the fly:
//                x~ = r + beta (p - omega v)   (x~ = r on a column's first
//                iteration); writes p_new = x~, v = M x~, partial <rhat, v>
//   MODE_BICG_S  x~ = s = r - alpha v formed on the fly; writes s, t = M s,
//                partials <t, s>, <t, t>
//   MODE_DOT1    the second half of a split MODE_BICG_P: x~ = X already
//                formed (k_bicg_pre), writes Y = M x~, partial <rhat, Y>
//   MODE_DOT2    the second half of a split MODE_BICG_S: writes Y = M X,
//                partials <Y, X>, <Y, Y>
// The fused modes gather r, p, v (or r, v) at every neighbour row and form
// x~ there again; when a panel's rows in flight on one XCD outgrow its L2,
// those gathers miss repeatedly, and the split form (x~ written once by an
// elementwise pass, then one gathered vector) moves fewer bytes.
// With CPLX the panel holds CP/2 complex columns as interleaved (re, im)
// column pairs; the shift is complex and dots are <u, v> = sum conj(u) v.
#pragma once

#include "common.hpp"

#include <type_traits>

namespace mpcare {

enum SpmmMode { MODE_PLAIN = 0, MODE_BICG_P = 1, MODE_BICG_S = 2, MODE_DOT1 = 3, MODE_DOT2 = 4 };

// per-logical-column BiCGStab scalars, KS doubles per column
// (RMIN: smallest ||r||^2 met; RCKPT: ||r||^2 of the checkpointed iterate)
enum {
  KS_RHO = 0, KS_ALPHA = 2, KS_OMEGA = 4, KS_BETA = 6, KS_BNRM2 = 8, KS_RNRM2 = 9, KS_LAST_RHR = 10,
  KS_RMIN = 11, KS_RCKPT = 12, KS_RREF = 13, KS_TOL2 = 14, KS = 16
};
// per-logical-column status, KI ints per column (STALL: iterations since the
// residual norm last dropped by 10 %)
enum { KI_ACTIVE = 0, KI_ITERS = 1, KI_FLAG = 2, KI_STALL = 3, KI = 4 };

template <typename T>
struct SpmmArgs {
  int n = 0;
  int ncols = 0;                 // real columns
  const int* sptr = nullptr;
  const int* cols = nullptr;
  const void* vals = nullptr;
  const T* diag = nullptr;
  double sr = 0.0, si = 0.0;     // shift
  int64_t ld = 0;                // leading dimension of Krylov panels
  // plain mode
  const T* X = nullptr;
  int64_t ldx = 0;
  T* Y = nullptr;
  int64_t ldy = 0;
  // BiCGStab modes
  const T* r = nullptr;
  const T* pold = nullptr;
  const T* vold = nullptr;
  T* pnew = nullptr;
  T* vnew = nullptr;
  const T* rhat = nullptr;
  int64_t ldrhat = 0;
  T* s = nullptr;
  T* t = nullptr;
  const double* sc = nullptr;
  const int* st = nullptr;
  double* part = nullptr;        // [(dot * ncols + col) * nrb + rowblock]
  int nrb = 0;
  int pg = 1;                    // column panels per workgroup (grid y = ceil(panels / pg))
  float vscale = 1.0f;           // F16 values: the operator's power-of-two scale
};

template <typename T, typename TV>
__device__ __forceinline__ T load_val(const TV* p, int64_t e) {
  return (T)p[e];
}
template <>
__device__ __forceinline__ float load_val<float, bf16>(const bf16* p, int64_t e) {
  return __bfloat162float(p[e]);
}
template <>
__device__ __forceinline__ float load_val<float, f16>(const f16* p, int64_t e) {
  return (float)p[e];
}
// one off-diagonal value of the operator; F16 values are unscaled by the
// operator's power of two (an exact product)
template <typename T, typename TV>
__device__ __forceinline__ T load_entry(const TV* p, int64_t e, float vscale) {
  if constexpr (std::is_same<TV, f16>::value) return load_val<T, TV>(p, e) * vscale;
  else return load_val<T, TV>(p, e);
}

// Reduce NV per-thread values over the 256-thread block in a fixed order
// (LDS transpose, 16 lanes per value) and hand value k of the block to
// dst(k, sum) on one lane.
template <int NV, typename T, typename Dst>
__device__ __forceinline__ void block_reduce_to(const T (&v)[NV], Dst dst) {
  constexpr int CH = NV < 16 ? NV : 16;
  __shared__ T red[CH][257];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k0 = 0; k0 < NV; k0 += CH) {
#pragma unroll
    for (int k = 0; k < CH; ++k)
      if (k0 + k < NV) red[k][tid] = v[k0 + k];
    __syncthreads();
    const int nk = (NV - k0) < CH ? (NV - k0) : CH;
    if (tid < nk * 16) {
      const int k = tid >> 4, q = tid & 15;
      T s = (T)0;
#pragma unroll
      for (int u = 0; u < 16; ++u) s += red[k][u * 16 + q];
      s += __shfl_xor(s, 8, 16);
      s += __shfl_xor(s, 4, 16);
      s += __shfl_xor(s, 2, 16);
      s += __shfl_xor(s, 1, 16);
      if (q == 0) dst(k0 + k, (double)s);
    }
    __syncthreads();
  }
}

// Complex products with their roundings fixed: re = fma(ar, br, -(ai bi)),
// im = fma(ar, bi, ai br).
template <typename T>
__device__ __forceinline__ T cmul_re(T ar, T ai, T br, T bi) {
#pragma clang fp contract(off)
  return fma(ar, br, -(ai * bi));
}
template <typename T>
__device__ __forceinline__ T cmul_im(T ar, T ai, T br, T bi) {
#pragma clang fp contract(off)
  return fma(ar, bi, ai * br);
}

template <typename TV, typename T, int CP, int MODE, bool CPLX, int WMAX>
__global__ void __launch_bounds__(256) k_spmm(SpmmArgs<T> a) {
  // Every fused multiply-add below is written out and no other is formed, so
  // a column's arithmetic is the same in every instance of the kernel (panel
  // width, row-width class, panels per workgroup): results do not depend on
  // how the columns are grouped into panels.
#pragma clang fp contract(off)
  constexpr int NDOT = MODE == MODE_PLAIN ? 0 : ((MODE == MODE_BICG_P || MODE == MODE_DOT1) ? 1 : 2);
  constexpr bool XIN = MODE == MODE_PLAIN || MODE == MODE_DOT1 || MODE == MODE_DOT2;   // input read from X
  constexpr int NL = CPLX ? CP / 2 : CP;          // logical columns in the panel
  static_assert(!CPLX || (CP % 2 == 0), "complex panels hold column pairs");

  // grid: (row block, group of pg panels); consecutive row blocks share an
  // XCD (and the halo rows of the neighbouring blocks in its L2)
  const int rb = (int)xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int i = rb * 256 + tid;
  const int64_t ld = a.ld;

  // The row's off-diagonal entries.  With WMAX > 0 (operators whose slices
  // hold at most WMAX entries per row) they are loaded once, before the
  // panels, padded with zero entries at the row itself: every gather of a
  // panel can then be issued at once (no chain of index loads), and the
  // matrix is read once for all the workgroup's panels.  WMAX = 0 streams the
  // entries panel by panel.
  int sbeg = 0, send = 0;
  if (i < a.n) {
    sbeg = a.sptr[i >> 6];
    send = a.sptr[(i >> 6) + 1];
  }
  int cj[WMAX > 0 ? WMAX : 1];
  T cv[WMAX > 0 ? WMAX : 1];
  if constexpr (WMAX > 0) {
    const TV* vals = (const TV*)a.vals;
    const int lane = i & 63;
#pragma unroll
    for (int t = 0; t < WMAX; ++t) {
      cj[t] = i < a.n ? i : 0;
      cv[t] = (T)0;
      if (sbeg + t < send) {
        const int64_t e = (int64_t)(sbeg + t) * 64 + lane;
        cj[t] = a.cols[e];
        cv[t] = load_entry<T, TV>(vals, e, a.vscale);
      }
    }
  }

  for (int pgi = 0; pgi < a.pg; ++pgi) {
  const int c0 = (blockIdx.y * a.pg + pgi) * CP;    // first real column of the panel
  if (c0 >= a.ncols) break;                         // uniform over the workgroup

  bool act[NL];
  bool first[NL];
  T sA_r[NL], sA_i[NL], sB_r[NL], sB_i[NL];       // mode scalars (beta/omega or alpha)
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int cr = c0 + (CPLX ? 2 * q : q);         // real column of the (re) part
    const int lc = CPLX ? cr / 2 : cr;              // logical column
    act[q] = cr < a.ncols;
    first[q] = false;
    sA_r[q] = sA_i[q] = sB_r[q] = sB_i[q] = (T)0;
    if (MODE != MODE_PLAIN && act[q]) {
      const int* st = a.st + (int64_t)lc * KI;
      act[q] = st[KI_ACTIVE] != 0;
      first[q] = st[KI_ITERS] == 0;
      const double* sc = a.sc + (int64_t)lc * KS;
      if (MODE == MODE_BICG_P) {
        sA_r[q] = (T)sc[KS_BETA];
        sA_i[q] = (T)sc[KS_BETA + 1];
        sB_r[q] = (T)sc[KS_OMEGA];
        sB_i[q] = (T)sc[KS_OMEGA + 1];
      } else if (MODE == MODE_BICG_S) {
        sA_r[q] = (T)sc[KS_ALPHA];
        sA_i[q] = (T)sc[KS_ALPHA + 1];
      }
    }
  }

  // Every load below is issued without a per-column branch: a column that is
  // inactive (converged, or past ncols in the last panel) reads the rows of
  // the panel's first active column instead, i.e. cache lines that are being
  // fetched anyway, and its results are dropped.  A branch per column would
  // make the compiler wait for each gather before issuing the next one.
  int colq[NL];
  int qa = -1;
#pragma unroll
  for (int q = 0; q < NL; ++q)
    if (qa < 0 && act[q]) qa = q;
  const int cra = c0 + (CPLX ? 2 * (qa < 0 ? 0 : qa) : (qa < 0 ? 0 : qa));
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int cr = c0 + (CPLX ? 2 * q : q);
    colq[q] = act[q] ? cr : cra;
  }

  // input value of logical column q at row j: (re, im)
  auto input = [&](int q, int64_t j, T& xr, T& xi) {
    const int cr = colq[q];
    const int64_t o = (int64_t)cr * ld + j;
    if (XIN) {
      xr = a.X[(int64_t)cr * a.ldx + j];
      xi = CPLX ? a.X[(int64_t)(cr + 1) * a.ldx + j] : (T)0;
    } else if (MODE == MODE_BICG_P) {
      // p and v are read on every iteration and the result selected, so that
      // the first iteration needs no branch (their contents are then unused)
      if (!CPLX) {
        const T rv = a.r[o];
        const T upd = fma(sA_r[q], fma(-sB_r[q], a.vold[o], a.pold[o]), rv);
        xr = first[q] ? rv : upd;
        xi = (T)0;
      } else {
        const T rr = a.r[o], ri = a.r[o + ld];
        const T pr = a.pold[o], pi = a.pold[o + ld];
        const T vr = a.vold[o], vi = a.vold[o + ld];
        const T ur = pr - cmul_re(sB_r[q], sB_i[q], vr, vi);
        const T ui = pi - cmul_im(sB_r[q], sB_i[q], vr, vi);
        const T ar = rr + cmul_re(sA_r[q], sA_i[q], ur, ui);
        const T ai = ri + cmul_im(sA_r[q], sA_i[q], ur, ui);
        xr = first[q] ? rr : ar;
        xi = first[q] ? ri : ai;
      }
    } else {  // MODE_BICG_S
      if (!CPLX) {
        xr = fma(-sA_r[q], a.vold[o], a.r[o]);
        xi = (T)0;
      } else {
        const T vr = a.vold[o], vi = a.vold[o + ld];
        xr = a.r[o] - cmul_re(sA_r[q], sA_i[q], vr, vi);
        xi = a.r[o + ld] - cmul_im(sA_r[q], sA_i[q], vr, vi);
      }
    }
  };

  T acc_r[NL], acc_i[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) acc_r[q] = acc_i[q] = (T)0;

  T dots[NDOT > 0 ? NDOT * CP : 1];
#pragma unroll
  for (int k = 0; k < (NDOT > 0 ? NDOT * CP : 1); ++k) dots[k] = (T)0;

  // plain product and the first split product need the row's own input only
  // for the diagonal term: it seeds the accumulators before the gathers, so
  // those inputs are not live across the loop
  constexpr bool DIAG_FIRST = MODE == MODE_PLAIN || MODE == MODE_DOT1;
  if (DIAG_FIRST && i < a.n && qa >= 0) {
    const T d0 = a.diag[i] + (T)a.sr;
    const T sim0 = (T)a.si;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      T x0r, x0i;
      input(q, i, x0r, x0i);
      if (!CPLX) {
        acc_r[q] = d0 * x0r;
      } else {
        acc_r[q] = cmul_re(d0, sim0, x0r, x0i);
        acc_i[q] = cmul_im(d0, sim0, x0r, x0i);
      }
    }
  }
  if (i < a.n && qa >= 0) {
    const int lane = i & 63;
    const int beg = sbeg, end = send;
    const TV* vals = (const TV*)a.vals;
    if constexpr (WMAX > 0) {
      // all entries' gathers issued without a branch (padding entries read
      // the row itself, already fetched, with value zero)
#pragma unroll
      for (int t = 0; t < WMAX; ++t) {
        T xr[NL], xi[NL];
#pragma unroll
        for (int q = 0; q < NL; ++q) input(q, cj[t], xr[q], xi[q]);
#pragma unroll
        for (int q = 0; q < NL; ++q) {
          acc_r[q] = fma(cv[t], xr[q], acc_r[q]);
          if (CPLX) acc_i[q] = fma(cv[t], xi[q], acc_i[q]);
        }
      }
    }
    // software pipeline: the next entry's column index and value are loaded
    // after this entry's gathers have been issued
    int jn = i;
    T avn = (T)0;
    if (WMAX == 0 && beg < end) {
      const int64_t e = (int64_t)beg * 64 + lane;
      jn = a.cols[e];
      avn = load_entry<T, TV>(vals, e, a.vscale);
    }
    for (int t = beg; WMAX == 0 && t < end; ++t) {
      const int j = jn;
      const T av = avn;
      T xr[NL], xi[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) input(q, j, xr[q], xi[q]);
      if (t + 1 < end) {
        const int64_t e = (int64_t)(t + 1) * 64 + lane;
        jn = a.cols[e];
        avn = load_entry<T, TV>(vals, e, a.vscale);
      }
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        acc_r[q] = fma(av, xr[q], acc_r[q]);
        if (CPLX) acc_i[q] = fma(av, xi[q], acc_i[q]);
      }
    }
    const T d = a.diag[i] + (T)a.sr;
    const T sim = (T)a.si;
    T xr[NL], xi[NL], hr[NL], hi[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      xr[q] = xi[q] = (T)0;
      if (!DIAG_FIRST) input(q, i, xr[q], xi[q]);
      hr[q] = hi[q] = (T)0;
      if (MODE == MODE_BICG_P || MODE == MODE_DOT1) {
        const int64_t oh = (int64_t)colq[q] * a.ldrhat + i;
        hr[q] = a.rhat[oh];
        if (CPLX) hi[q] = a.rhat[oh + a.ldrhat];
      }
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      if (!act[q]) continue;
      T yr, yi = (T)0;
      if (DIAG_FIRST) {
        yr = acc_r[q];
        yi = CPLX ? acc_i[q] : (T)0;
      } else if (!CPLX) {
        yr = fma(d, xr[q], acc_r[q]);
      } else {
        yr = fma(-sim, xi[q], fma(d, xr[q], acc_r[q]));
        yi = fma(sim, xr[q], fma(d, xi[q], acc_i[q]));
      }
      const int cr = c0 + (CPLX ? 2 * q : q);
      const int64_t o = (int64_t)cr * ld + i;
      if (MODE == MODE_PLAIN) {
        a.Y[(int64_t)cr * a.ldy + i] = yr;
        if (CPLX) a.Y[(int64_t)(cr + 1) * a.ldy + i] = yi;
      } else if (MODE == MODE_DOT1 || MODE == MODE_BICG_P) {
        if (MODE == MODE_DOT1) {
          a.Y[(int64_t)cr * a.ldy + i] = yr;
          if (CPLX) a.Y[(int64_t)(cr + 1) * a.ldy + i] = yi;
        } else {
          a.pnew[o] = xr[q];
          a.vnew[o] = yr;
          if (CPLX) {
            a.pnew[o + ld] = xi[q];
            a.vnew[o + ld] = yi;
          }
        }
        if (!CPLX) {
          dots[q] = hr[q] * yr;                      // <rhat, v>
        } else {
          dots[2 * q] = fma(hr[q], yr, hi[q] * yi);       // conj(rhat) v
          dots[2 * q + 1] = fma(hr[q], yi, -(hi[q] * yr));
        }
      } else {   // MODE_DOT2, MODE_BICG_S
        if (MODE == MODE_DOT2) {
          a.Y[(int64_t)cr * a.ldy + i] = yr;
          if (CPLX) a.Y[(int64_t)(cr + 1) * a.ldy + i] = yi;
        } else {
          a.s[o] = xr[q];
          a.t[o] = yr;
          if (CPLX) {
            a.s[o + ld] = xi[q];
            a.t[o + ld] = yi;
          }
        }
        if (!CPLX) {
          dots[q] = yr * xr[q];                      // <t, s>
          dots[CP + q] = yr * yr;                    // <t, t>
        } else {
          dots[2 * q] = fma(yr, xr[q], yi * xi[q]);       // conj(t) s
          dots[2 * q + 1] = fma(yr, xi[q], -(yi * xr[q]));
          dots[CP + 2 * q] = fma(yr, yr, yi * yi);        // |t|^2
          dots[CP + 2 * q + 1] = (T)0;
        }
      }
    }
  }
  if constexpr (NDOT > 0) {
    block_reduce_to<NDOT * CP>(dots, [&](int kk, double val) {
      const int dot = kk / CP, c = c0 + kk % CP;
      if (c < a.ncols) a.part[((int64_t)dot * a.ncols + c) * a.nrb + rb] = val;
    });
  }
  }   // panels of the workgroup
}

}  // namespace mpcare
