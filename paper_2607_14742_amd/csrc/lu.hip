// Batched LU factorisation with partial pivoting of shifted dense matrices
// M_s = M0 + p_s I and the triangular solves that reuse them: the direct
// shifted solves of the dense problems (Sec. 5.1 solves its dense examples
// with LU factorisations; with the Sherman-Morrison-Woodbury form of Sec. 4
// the base matrix A^T + p I is the same at every Newton step, so one
// factorisation per shift serves the whole solve).
//
// k_lu_factor: one workgroup owns one matrix for its whole factorisation
// (a single launch covers every shift of a set).  Right-looking blocked LU
// with panels of NB columns:
//   * the panel (rows j0..n-1; NB = 16 columns in FP32, 8 in FP64, so that
//     it fits the 128 registers a thread of a 1024-thread workgroup has)
//     sits in registers, two rows per thread; each
//     column takes an arg-max over the workgroup (ties: smallest row), a row
//     exchange through LDS and a rank-1 update of the rest of the panel;
//   * the panel's row exchanges are applied to every other column, in order;
//   * U12 = L11^{-1} A12 by one thread per column (L11 in LDS), staged in LDS;
//   * A22 -= L21 U12 on the matrix cores (16 x 16 x 4 MFMA): each wave keeps
//     the L21 operands of a 32-row strip in registers and sweeps the column
//     tiles, reading the U12 operands from LDS.
// The result has the LAPACK getrf layout (unit L below the diagonal, U on and
// above it, ipiv the sequential row exchanges), plus perm with
// (P M)[i] = M[perm[i]] for the solves.
//
// k_lu_solve: one workgroup per group of KB right-hand sides; the permuted
// right-hand sides live in LDS, the factors stream through in 64-row blocks
// (each block's triangle is solved by one wave per column with lane
// broadcasts, then the rows below (forward) or above (backward) are updated).
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "lu.hpp"

namespace mpcare {

typedef float lu_float4 __attribute__((ext_vector_type(4)));
typedef double lu_double4 __attribute__((ext_vector_type(4)));

constexpr int LU_NT = 1024;     // threads per workgroup
constexpr int LU_R = 2;         // panel rows per thread (n <= LU_NT * LU_R)
constexpr int LU_CB = 512;      // columns of the trailing matrix per U12 stage
constexpr int LU_PU = LU_CB + 16;   // LDS pitch of the staged U12 rows

template <typename T>
struct LuMma;
// v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// lane l holds D[4 (l / 16) + v][l % 16], v = 0..3
template <>
struct LuMma<float> {
  using V = lu_float4;
  static constexpr int NB = 16;
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int g, int v) { return 4 * g + v; }
};
// v_mfma_f64_16x16x4f64: same operand layout; lane l holds D[(l / 16) + 4 v][l % 16]
template <>
struct LuMma<double> {
  using V = lu_double4;
  static constexpr int NB = 8;
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int g, int v) { return g + 4 * v; }
};

__device__ __forceinline__ float lane_bcast(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One column C of the panel factorisation (compile-time C, so the panel
// stays in registers): arg-max pivot, row exchange, scaling and the rank-1
// update of the panel's later columns.
template <typename T, int NB, int C>
__device__ __forceinline__ void lu_panel_column(T (&pr)[LU_R][NB], int j0, int n, int nb, int tid, int lane,
                                                int wave, T (*redv)[LU_NT / 64], int (*redi)[LU_NT / 64],
                                                T (*sRow)[2][NB], int* spiv, int* sinfo) {
  constexpr int c = C;
  if (c >= nb) return;   // uniform; a short panel only at the end
  const int jc = j0 + c, buf = c & 1;
  T best = T(-1);
  int bi = 0x7fffffff;
#pragma unroll
  for (int r = 0; r < LU_R; ++r) {
    const int i = j0 + tid + r * LU_NT;
    const T a = fabs(pr[r][c]);
    if (i >= jc && i < n && a > best) {
      best = a;
      bi = i;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const T ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    redv[buf][wave] = best;
    redi[buf][wave] = bi;
  }
  __syncthreads();
  best = redv[buf][0];
  bi = redi[buf][0];
#pragma unroll
  for (int w = 1; w < LU_NT / 64; ++w) {
    const T ob = redv[buf][w];
    const int oi = redi[buf][w];
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  // no candidate above -1 only if every entry is NaN: keep the diagonal
  const int piv = bi == 0x7fffffff ? jc : bi;
  const int oj = (jc - j0) % LU_NT, rj = (jc - j0) / LU_NT;
  const int op = (piv - j0) % LU_NT, rp = (piv - j0) / LU_NT;
  T* rowA = sRow[buf][0];   // the pivot row, at jc after the exchange
  T* rowB = sRow[buf][1];   // the old row jc, at piv after the exchange
  // (branches, not selects: a select between two rows would become a
  // dynamic index into the register panel)
  if (tid == op) {
    if (rp == 0) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) rowA[cc] = pr[0][cc];
    } else {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) rowA[cc] = pr[1][cc];
    }
  }
  if (tid == oj && piv != jc) {
    if (rj == 0) {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) rowB[cc] = pr[0][cc];
    } else {
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) rowB[cc] = pr[1][cc];
    }
  }
  __syncthreads();
  if (piv != jc && (tid == oj || tid == op)) {
    // both register rows are rewritten with value selects (a store into a
    // row chosen at run time would push the panel out of registers)
    const bool tj0 = tid == oj && rj == 0, tj1 = tid == oj && rj == 1;
    const bool tp0 = tid == op && rp == 0, tp1 = tid == op && rp == 1;
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      const T a = rowA[cc], b = rowB[cc];
      pr[0][cc] = tj0 ? a : (tp0 ? b : pr[0][cc]);
      pr[1][cc] = tj1 ? a : (tp1 ? b : pr[1][cc]);
    }
  }
  const T d = rowA[c];
  if (tid == 0) {
    spiv[c] = piv;
    if (d == T(0) && *sinfo == 0) *sinfo = jc + 1;
  }
#pragma unroll
  for (int r = 0; r < LU_R; ++r) {
    const int i = j0 + tid + r * LU_NT;
    if (i > jc && i < n) {
      const T l = d != T(0) ? pr[r][c] / d : pr[r][c];
      pr[r][c] = l;
#pragma unroll
      for (int cc = c + 1; cc < NB; ++cc) pr[r][cc] = fma(-l, rowA[cc], pr[r][cc]);
    }
  }
}

template <typename T, int NB, int... Cs>
__device__ __forceinline__ void lu_panel(std::integer_sequence<int, Cs...>, T (&pr)[LU_R][NB], int j0, int n, int nb,
                                         int tid, int lane, int wave, T (*redv)[LU_NT / 64],
                                         int (*redi)[LU_NT / 64], T (*sRow)[2][NB], int* spiv, int* sinfo) {
  (lu_panel_column<T, NB, Cs>(pr, j0, n, nb, tid, lane, wave, redv, redi, sRow, spiv, sinfo), ...);
}

template <typename T>
__global__ void __launch_bounds__(LU_NT) k_lu_factor(int n, const T* __restrict__ M0, const T* __restrict__ shifts,
                                                     T* const* __restrict__ Fp, int* const* __restrict__ Pp,
                                                     int* __restrict__ ipiv_all, int* __restrict__ info) {
  constexpr int NB = LuMma<T>::NB;
  using V = typename LuMma<T>::V;
  __shared__ T sU[NB * LU_PU];
  __shared__ T sL11[NB * NB];
  __shared__ T sRow[2][2][NB];
  __shared__ T redv[2][LU_NT / 64];
  __shared__ int redi[2][LU_NT / 64];
  __shared__ int spiv[NB];
  __shared__ int sperm[LU_NT * LU_R];
  __shared__ int sinfo;

  const int mat = blockIdx.x;
  T* __restrict__ M = Fp[mat];
  int* __restrict__ ipiv = ipiv_all + (int64_t)mat * n;
  const T p = shifts[mat];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;

  // M = M0 + p I (the shift in the operator precision)
  for (int col = 0; col < n; ++col)
    for (int i = tid; i < n; i += LU_NT) {
      const T v = M0[(int64_t)col * n + i];
      M[(int64_t)col * n + i] = i == col ? v + p : v;
    }
  for (int i = tid; i < n; i += LU_NT) sperm[i] = i;
  if (tid == 0) sinfo = 0;
  __syncthreads();

  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nb = min(NB, n - j0);
    // ---- panel: rows j0 + tid + r LU_NT, columns j0 .. j0 + nb - 1
    T pr[LU_R][NB];
#pragma unroll
    for (int r = 0; r < LU_R; ++r) {
      const int i = j0 + tid + r * LU_NT;
#pragma unroll
      for (int c = 0; c < NB; ++c) pr[r][c] = (i < n && c < nb) ? M[(int64_t)(j0 + c) * n + i] : T(0);
    }
    lu_panel<T, NB>(std::make_integer_sequence<int, NB>(), pr, j0, n, nb, tid, lane, wave, redv, redi, sRow, spiv,
                    &sinfo);
    // ---- panel back to memory; L11 to LDS; the exchanges to perm
#pragma unroll
    for (int r = 0; r < LU_R; ++r) {
      const int i = j0 + tid + r * LU_NT;
      if (i < n) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nb) M[(int64_t)(j0 + c) * n + i] = pr[r][c];
      }
    }
    if (tid < nb) {
#pragma unroll
      for (int c = 0; c < NB; ++c) sL11[tid * NB + c] = pr[0][c];
    }
    __syncthreads();
    if (tid < nb) ipiv[j0 + tid] = spiv[tid];
    if (tid == 0) {
      for (int c = 0; c < nb; ++c) {
        const int a = j0 + c, b = spiv[c];
        const int t = sperm[a];
        sperm[a] = sperm[b];
        sperm[b] = t;
      }
    }
    // ---- the exchanges on the columns left of the panel (L, LAPACK layout)
    for (int col = tid; col < j0; col += LU_NT) {
      T* Mc = M + (int64_t)col * n;
      for (int c = 0; c < nb; ++c) {
        const int pv = spiv[c];
        if (pv != j0 + c) {
          const T a = Mc[j0 + c], b = Mc[pv];
          Mc[j0 + c] = b;
          Mc[pv] = a;
        }
      }
    }
    // ---- trailing matrix, LU_CB columns at a time
    const int r0 = j0 + nb;
    const int nstrips = (n - r0 + 31) / 32;
    for (int cb0 = r0; cb0 < n; cb0 += LU_CB) {
      const int cbn = min(LU_CB, n - cb0);
      if (tid < cbn) {
        T* Mc = M + (int64_t)(cb0 + tid) * n;
        for (int c = 0; c < nb; ++c) {
          const int pv = spiv[c];
          if (pv != j0 + c) {
            const T a = Mc[j0 + c], b = Mc[pv];
            Mc[j0 + c] = b;
            Mc[pv] = a;
          }
        }
        T u[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) u[c] = c < nb ? Mc[j0 + c] : T(0);
        // column-oriented forward substitution; the empty asm keeps the
        // scheduler from hoisting all NB (NB - 1) / 2 LDS reads of L11 at once
#pragma unroll
        for (int t = 0; t < NB - 1; ++t) {
          asm volatile("" ::: "memory");
#pragma unroll
          for (int c = t + 1; c < NB; ++c) u[c] = fma(-sL11[c * NB + t], u[t], u[c]);
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          // rows past a short last panel stay zero (their L11 rows are stale)
          if (c >= nb) u[c] = T(0);
          else Mc[j0 + c] = u[c];
          sU[c * LU_PU + tid] = u[c];
        }
      }
      __syncthreads();
      const int nct = (cbn + 31) / 32;
      for (int s = wave; s < nstrips; s += LU_NT / 64) {
        T a[2][NB / 4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const int row = r0 + 32 * s + 16 * rt + li;
#pragma unroll
          for (int t = 0; t < NB / 4; ++t) {
            const int k = 4 * t + lg;
            a[rt][t] = (row < n && k < nb) ? -M[(int64_t)(j0 + k) * n + row] : T(0);
          }
        }
        for (int ct = 0; ct < nct; ++ct) {
          V acc[2][2];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
              const int col = cb0 + 32 * ct + 16 * cc + li;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int row = r0 + 32 * s + 16 * rt + LuMma<T>::row(lg, v);
                acc[rt][cc][v] = (row < n && col < cb0 + cbn) ? M[(int64_t)col * n + row] : T(0);
              }
            }
#pragma unroll
          for (int t = 0; t < NB / 4; ++t) {
            const T b0 = sU[(4 * t + lg) * LU_PU + 32 * ct + li];
            const T b1 = sU[(4 * t + lg) * LU_PU + 32 * ct + 16 + li];
            acc[0][0] = LuMma<T>::mma(a[0][t], b0, acc[0][0]);
            acc[0][1] = LuMma<T>::mma(a[0][t], b1, acc[0][1]);
            acc[1][0] = LuMma<T>::mma(a[1][t], b0, acc[1][0]);
            acc[1][1] = LuMma<T>::mma(a[1][t], b1, acc[1][1]);
          }
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
              const int col = cb0 + 32 * ct + 16 * cc + li;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int row = r0 + 32 * s + 16 * rt + LuMma<T>::row(lg, v);
                if (row < n && col < cb0 + cbn) M[(int64_t)col * n + row] = acc[rt][cc][v];
              }
            }
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += LU_NT) Pp[mat][i] = sperm[i];
  if (tid == 0) info[mat] = sinfo;
}

template <typename T, int KB>
__global__ void __launch_bounds__(LU_NT) k_lu_solve(int n, const T* __restrict__ F, const int* __restrict__ perm,
                                                    int k, const T* __restrict__ Bm, int64_t ldb, T* __restrict__ X,
                                                    int64_t ldx) {
  __shared__ T xs[KB * LU_NT * LU_R];
  __shared__ T sD[64 * 65];
  const int c0 = blockIdx.x * KB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int j = 0; j < KB; ++j)
    for (int i = tid; i < n; i += LU_NT)
      xs[j * n + i] = c0 + j < k ? Bm[(int64_t)(c0 + j) * ldb + perm[i]] : T(0);
  __syncthreads();
  // forward: L y = P b with unit lower L
  for (int b0 = 0; b0 < n; b0 += 64) {
    const int bs = min(64, n - b0);
    for (int e = tid; e < bs * 64; e += LU_NT) {
      const int t = e >> 6, i = e & 63;
      sD[t * 65 + i] = i < bs ? F[(int64_t)(b0 + t) * n + b0 + i] : T(0);
    }
    __syncthreads();
    if (wave < KB) {
      T xv = lane < bs ? xs[wave * n + b0 + lane] : T(0);
      for (int t = 0; t < bs; ++t) {
        const T xt = lane_bcast(xv, t);
        if (lane > t) xv = fma(-sD[t * 65 + lane], xt, xv);
      }
      if (lane < bs) xs[wave * n + b0 + lane] = xv;
    }
    __syncthreads();
    for (int i = b0 + bs + tid; i < n; i += LU_NT) {
      T acc[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) acc[j] = T(0);
      for (int t = 0; t < bs; ++t) {
        const T l = F[(int64_t)(b0 + t) * n + i];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = fma(l, xs[j * n + b0 + t], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < KB; ++j) xs[j * n + i] -= acc[j];
    }
    __syncthreads();
  }
  // backward: U x = y
  for (int b0 = (n - 1) / 64 * 64; b0 >= 0; b0 -= 64) {
    const int bs = min(64, n - b0);
    for (int e = tid; e < bs * 64; e += LU_NT) {
      const int t = e >> 6, i = e & 63;
      sD[t * 65 + i] = i < bs ? F[(int64_t)(b0 + t) * n + b0 + i] : T(0);
    }
    __syncthreads();
    if (wave < KB) {
      T xv = lane < bs ? xs[wave * n + b0 + lane] : T(0);
      for (int t = bs - 1; t >= 0; --t) {
        if (lane == t) xv = xv / sD[t * 65 + t];
        const T xt = lane_bcast(xv, t);
        if (lane < t) xv = fma(-sD[t * 65 + lane], xt, xv);
      }
      if (lane < bs) xs[wave * n + b0 + lane] = xv;
    }
    __syncthreads();
    for (int i = tid; i < b0; i += LU_NT) {
      T acc[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) acc[j] = T(0);
      for (int t = 0; t < bs; ++t) {
        const T u = F[(int64_t)(b0 + t) * n + i];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = fma(u, xs[j * n + b0 + t], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < KB; ++j) xs[j * n + i] -= acc[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < KB; ++j)
    if (c0 + j < k)
      for (int i = tid; i < n; i += LU_NT) X[(int64_t)(c0 + j) * ldx + i] = xs[j * n + i];
}

template <typename T>
void lu_factor_shifted(Ctx* ctx, int n, const T* M0, const std::vector<double>& shifts, const std::vector<T*>& F,
                       const std::vector<int*>& perm, std::vector<int>& info) {
  const int nm = (int)shifts.size();
  info.assign(nm, 0);
  if (nm == 0) return;
  if (n < 1 || n > LU_NMAX) fail(CARE_ERR_ARG, "lu_factor_shifted: n must be in [1, " + std::to_string(LU_NMAX) + "]");
  if ((int)F.size() != nm || (int)perm.size() != nm) fail(CARE_ERR_ARG, "lu_factor_shifted: one output per shift");
  std::vector<T> hs(nm);
  for (int s = 0; s < nm; ++s) {
    if (!F[s] || !perm[s]) fail(CARE_ERR_ARG, "lu_factor_shifted: NULL output");
    hs[s] = (T)shifts[s];
  }
  DBuf<T> ds(ctx, nm);
  DBuf<T*> dF(ctx, nm);
  DBuf<int*> dP(ctx, nm);
  DBuf<int> dipiv(ctx, (size_t)nm * n), dinfo(ctx, nm);
  h2d(ctx, ds.get(), hs.data(), nm * sizeof(T));
  h2d(ctx, dF.get(), F.data(), nm * sizeof(T*));
  h2d(ctx, dP.get(), perm.data(), nm * sizeof(int*));
  hipLaunchKernelGGL(k_lu_factor<T>, dim3(nm), dim3(LU_NT), 0, ctx->stream, n, M0, (const T*)ds.get(),
                     (T* const*)dF.get(), (int* const*)dP.get(), dipiv.get(), dinfo.get());
  KERNEL_CHECK();
  d2h(ctx, info.data(), dinfo.get(), nm * sizeof(int));
}

template <typename T>
void lu_solve(Ctx* ctx, int n, const T* F, const int* perm, int k, const T* B, int64_t ldb, T* X, int64_t ldx) {
  if (k <= 0) return;
  if (n < 1 || n > LU_NMAX) fail(CARE_ERR_ARG, "lu_solve: n must be in [1, " + std::to_string(LU_NMAX) + "]");
  if (ldb < n || ldx < n) fail(CARE_ERR_ARG, "lu_solve: leading dimension below n");
  constexpr int KB = sizeof(T) == 4 ? 4 : 2;
  hipLaunchKernelGGL((k_lu_solve<T, KB>), dim3(ceil_div(k, KB)), dim3(LU_NT), 0, ctx->stream, n, F, perm, k, B, ldb,
                     X, ldx);
  KERNEL_CHECK();
}

template void lu_factor_shifted<float>(Ctx*, int, const float*, const std::vector<double>&, const std::vector<float*>&,
                                       const std::vector<int*>&, std::vector<int>&);
template void lu_factor_shifted<double>(Ctx*, int, const double*, const std::vector<double>&,
                                        const std::vector<double*>&, const std::vector<int*>&, std::vector<int>&);
template void lu_solve<float>(Ctx*, int, const float*, const int*, int, const float*, int64_t, float*, int64_t);
template void lu_solve<double>(Ctx*, int, const double*, const int*, int, const double*, int64_t, double*, int64_t);

}  // namespace mpcare
