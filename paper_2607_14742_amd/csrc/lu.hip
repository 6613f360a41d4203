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
//   * the panel (rows j0..n-1; NB = 16 columns in FP32, 8 in FP64) sits in
//     registers, four rows per thread of a 512-thread workgroup; each
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
// k_lu_solve: one workgroup per group of KB right-hand sides (2 in FP32, 1 in
// FP64: the FMA work of a workgroup is n^2 KB, so narrow groups spread it
// over more compute units); the permuted
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

constexpr int LU_NT = 512;      // threads per workgroup
constexpr int LU_R = 4;         // panel rows per thread (n <= LU_NT * LU_R)
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

// element idx (< 2^32 / sizeof(T)) of a matrix through a 32-bit byte offset,
// so that loads and stores can take the uniform base in scalar registers
template <typename T>
__device__ __forceinline__ T& at(T* base, int idx) {
  return *(T*)((char*)base + (uint32_t)idx * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T at(const T* base, int idx) {
  return *(const T*)((const char*)base + (uint32_t)idx * (uint32_t)sizeof(T));
}

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
  // Rows are picked out of the register panel with value selects only (an
  // access through a row index known at run time would move the panel to
  // scratch memory).
  if (tid == op || (tid == oj && piv != jc)) {
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      T va = pr[0][cc], vb = pr[0][cc];
#pragma unroll
      for (int r = 1; r < LU_R; ++r) {
        va = rp == r ? pr[r][cc] : va;
        vb = rj == r ? pr[r][cc] : vb;
      }
      if (tid == op) rowA[cc] = va;
      if (tid == oj && piv != jc) rowB[cc] = vb;
    }
  }
  __syncthreads();
  if (piv != jc && (tid == oj || tid == op)) {
#pragma unroll
    for (int cc = 0; cc < NB; ++cc) {
      const T a = rowA[cc], b = rowB[cc];
#pragma unroll
      for (int r = 0; r < LU_R; ++r) {
        const bool tj = tid == oj && rj == r, tp = tid == op && rp == r;
        pr[r][cc] = tj ? a : (tp ? b : pr[r][cc]);
      }
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
                                                     int* const* __restrict__ Ip, int* __restrict__ info) {
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
    if (Ip && tid < nb) Ip[mat][j0 + tid] = spiv[tid] + 1;   // 1-based, as getrf's
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
      // The product is formed transposed, C^T -= U12^T L21^T, so that the 16
      // consecutive lanes of an accumulator register hold 16 consecutive rows
      // of one column of C (contiguous in memory).  Lane (li, lg) holds
      // C[row0 + li][col0 + LuMma<T>::row(lg, v)] in register v.  The next
      // column tile's loads are issued before the current tile's MFMAs.
      const int nct = (cbn + 31) / 32;
      const int cend = cb0 + cbn;
      for (int s = wave; s < nstrips; s += LU_NT / 64) {
        const int rbase = r0 + 32 * s;
        T bl[2][NB / 4];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          const int row = rbase + 16 * rt + li;
#pragma unroll
          for (int t = 0; t < NB / 4; ++t) {
            const int k = 4 * t + lg;
            bl[rt][t] = (row < n && k < nb) ? -at(M, (j0 + k) * n + row) : T(0);
          }
        }
        auto load_c = [&](V (&acc)[2][2], int ct) {
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
              const int row = rbase + 16 * rt + li;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int col = cb0 + 32 * ct + 16 * cc + LuMma<T>::row(lg, v);
                acc[rt][cc][v] = (row < n && col < cend) ? at(M, col * n + row) : T(0);
              }
            }
        };
        auto update_store = [&](V (&acc)[2][2], int ct) {
#pragma unroll
          for (int t = 0; t < NB / 4; ++t) {
            const T u0 = sU[(4 * t + lg) * LU_PU + 32 * ct + li];
            const T u1 = sU[(4 * t + lg) * LU_PU + 32 * ct + 16 + li];
            acc[0][0] = LuMma<T>::mma(u0, bl[0][t], acc[0][0]);
            acc[0][1] = LuMma<T>::mma(u1, bl[0][t], acc[0][1]);
            acc[1][0] = LuMma<T>::mma(u0, bl[1][t], acc[1][0]);
            acc[1][1] = LuMma<T>::mma(u1, bl[1][t], acc[1][1]);
          }
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
              const int row = rbase + 16 * rt + li;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int col = cb0 + 32 * ct + 16 * cc + LuMma<T>::row(lg, v);
                if (row < n && col < cend) at(M, col * n + row) = acc[rt][cc][v];
              }
            }
        };
        V accA[2][2], accB[2][2];
        load_c(accA, 0);
        for (int ct = 0; ct < nct; ct += 2) {
          if (ct + 1 < nct) load_c(accB, ct + 1);
          update_store(accA, ct);
          if (ct + 1 < nct) {
            if (ct + 2 < nct) load_c(accA, ct + 2);
            update_store(accB, ct + 1);
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

// ---------------------------------------------------------------------------
// triangular solves
// ---------------------------------------------------------------------------
constexpr int LS_NT = 1024;   // threads of a solve workgroup; thread t owns rows t and t + LS_NT
template <typename T>
constexpr int LS_GS = 32;     // factor entries of a row loaded together (FP32)
template <>
constexpr int LS_GS<double> = 16;

// One sweep over the 64-row blocks of a triangular factor (forward: unit
// lower L, blocks top to bottom, rows below updated; backward: upper U,
// bottom to top, rows above updated).  The KB right-hand sides live in LDS
// (xs, columns of np entries).  Per block:
//   1. the diagonal block (staged in LDS during the previous block) is solved
//      by one wave per column, lane i holding row i, with lane broadcasts;
//   2. each thread's rows outside the block take x[i] -= F[i, block] x_block,
//      the 64 factor entries of a row loaded in groups (32 in FP32, 16 in
//      FP64), the block's x values read from LDS.
// The next diagonal block is loaded during step 2.
// A short last block is padded with the identity (diagonal) and zeros.
template <typename T, int KB, bool FWD>
__device__ __forceinline__ void lu_sweep(int n, int np, const T* F, T* xs, T (*sD)[64 * 65]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = (n + 63) / 64;
  auto blk_start = [&](int q) { return FWD ? 64 * q : 64 * (nblk - 1 - q); };
  // rows of this thread taking part in the update of block b0 (bs rows)
  auto takes_part = [&](int i, int b0, int bs) { return i < n && (FWD ? i >= b0 + bs : i < b0); };
  T dpre[(64 * 64) / LS_NT];
  // (loads go to clamped, always valid addresses and unused values are
  // zeroed afterwards: conditional loads would each need a branch)
  auto load_diag = [&](int b0, int bs) {
#pragma unroll
    for (int e = 0; e < (64 * 64) / LS_NT; ++e) {
      const int idx = tid + e * LS_NT, t = idx >> 6, i = idx & 63;
      const T v = at(F, (b0 + min(t, bs - 1)) * n + b0 + min(i, bs - 1));
      dpre[e] = (i < bs && t < bs) ? v : (i == t ? T(1) : T(0));
    }
  };
  auto store_diag = [&](int buf) {
#pragma unroll
    for (int e = 0; e < (64 * 64) / LS_NT; ++e) {
      const int idx = tid + e * LS_NT, t = idx >> 6, i = idx & 63;
      sD[buf][t * 65 + i] = dpre[e];
    }
  };
  constexpr int GS = LS_GS<T>;
  {
    const int b0 = blk_start(0), bs = min(64, n - b0);
    load_diag(b0, bs);
    store_diag(0);
  }
  for (int q = 0; q < nblk; ++q) {
    const int b0 = blk_start(q), bs = min(64, n - b0), buf = q & 1;
    __syncthreads();   // sD[buf] staged; x of the block final
    if (wave < KB) {
      const T* D = sD[buf];
      T xv = lane < bs ? xs[wave * np + b0 + lane] : T(0);
      if (FWD) {
#pragma unroll 8
        for (int t = 0; t < 64; ++t) {
          const T xt = lane_bcast(xv, t);
          if (lane > t) xv = fma(-D[t * 65 + lane], xt, xv);
        }
      } else {
#pragma unroll 8
        for (int t = 63; t >= 0; --t) {
          if (lane == t) xv = xv / D[t * 65 + t];
          const T xt = lane_bcast(xv, t);
          if (lane < t) xv = fma(-D[t * 65 + lane], xt, xv);
        }
      }
      if (lane < bs) xs[wave * np + b0 + lane] = xv;
    }
    const bool more = q + 1 < nblk;
    if (more) {
      const int nb0 = blk_start(q + 1);
      load_diag(nb0, min(64, n - nb0));
    }
    __syncthreads();   // the block's x final for every thread
    // rows outside the block: x[i] -= F[i, block] x_block (the block's x
    // values are LDS broadcasts); the factor entries of a row come in groups
    // of GS, each group's loads issued together
    T acc[2][KB];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < KB; ++j) acc[r][j] = T(0);
    bool part[2];
    int ic[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int i = tid + r * LS_NT;
      part[r] = takes_part(i, b0, bs);
      ic[r] = min(i, n - 1);
    }
    if (part[0] || part[1]) {
#pragma unroll 1
      for (int g0 = 0; g0 < 64; g0 += GS) {
        T gv[2][GS];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int t = 0; t < GS; ++t) {
            const int c = g0 + t;
            const T v = at(F, (b0 + min(c, bs - 1)) * n + ic[r]);
            gv[r][t] = (part[r] && c < bs) ? v : T(0);
          }
#pragma unroll
        for (int t = 0; t < GS; ++t)
#pragma unroll
          for (int j = 0; j < KB; ++j) {
            const T xv = xs[j * np + b0 + g0 + t];
            acc[0][j] = fma(gv[0][t], xv, acc[0][j]);
            acc[1][j] = fma(gv[1][t], xv, acc[1][j]);
          }
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (part[r]) {
#pragma unroll
          for (int j = 0; j < KB; ++j) xs[j * np + tid + r * LS_NT] -= acc[r][j];
        }
    }
    if (more) store_diag(buf ^ 1);
  }
  __syncthreads();
}

template <typename T, int KB>
__global__ void __launch_bounds__(LS_NT) k_lu_solve(int n, const T* F, const int* __restrict__ perm,
                                                    int k, const T* __restrict__ Bm, int64_t ldb, T* __restrict__ X,
                                                    int64_t ldx) {
  // xs holds columns of np = n + 64 entries (the entries past n are zero)
  __shared__ T xs[KB * (LU_NMAX + 64)];
  __shared__ T sD[2][64 * 65];
  const int c0 = blockIdx.x * KB, np = n + 64;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < KB; ++j)
    for (int i = tid; i < np; i += LS_NT)
      xs[j * np + i] = (c0 + j < k && i < n) ? Bm[(int64_t)(c0 + j) * ldb + perm[i]] : T(0);
  lu_sweep<T, KB, true>(n, np, F, xs, sD);    // L y = P b
  lu_sweep<T, KB, false>(n, np, F, xs, sD);   // U x = y
#pragma unroll
  for (int j = 0; j < KB; ++j)
    if (c0 + j < k)
      for (int i = tid; i < n; i += LS_NT) X[(int64_t)(c0 + j) * ldx + i] = xs[j * np + i];
}

template <typename T>
void lu_factor_shifted(Ctx* ctx, int n, const T* M0, const std::vector<double>& shifts, const std::vector<T*>& F,
                       const std::vector<int*>& perm, std::vector<int>& info, const std::vector<int*>& ipiv) {
  const int nm = (int)shifts.size();
  info.assign(nm, 0);
  if (nm == 0) return;
  if (n < 1 || n > LU_NMAX) fail(CARE_ERR_ARG, "lu_factor_shifted: n must be in [1, " + std::to_string(LU_NMAX) + "]");
  if ((int)F.size() != nm || (int)perm.size() != nm || (!ipiv.empty() && (int)ipiv.size() != nm))
    fail(CARE_ERR_ARG, "lu_factor_shifted: one output per shift");
  std::vector<T> hs(nm);
  for (int s = 0; s < nm; ++s) {
    if (!F[s] || !perm[s] || (!ipiv.empty() && !ipiv[s])) fail(CARE_ERR_ARG, "lu_factor_shifted: NULL output");
    hs[s] = (T)shifts[s];
  }
  DBuf<T> ds(ctx, nm);
  DBuf<T*> dF(ctx, nm);
  DBuf<int*> dP(ctx, nm), dI(ctx, nm);
  DBuf<int> dinfo(ctx, nm);
  h2d(ctx, ds.get(), hs.data(), nm * sizeof(T));
  h2d(ctx, dF.get(), F.data(), nm * sizeof(T*));
  h2d(ctx, dP.get(), perm.data(), nm * sizeof(int*));
  if (!ipiv.empty()) h2d(ctx, dI.get(), ipiv.data(), nm * sizeof(int*));
  hipLaunchKernelGGL(k_lu_factor<T>, dim3(nm), dim3(LU_NT), 0, ctx->stream, n, M0, (const T*)ds.get(),
                     (T* const*)dF.get(), (int* const*)dP.get(), ipiv.empty() ? nullptr : (int* const*)dI.get(),
                     dinfo.get());
  KERNEL_CHECK();
  d2h(ctx, info.data(), dinfo.get(), nm * sizeof(int));
}

template <typename T>
void lu_solve(Ctx* ctx, int n, const T* F, const int* perm, int k, const T* B, int64_t ldb, T* X, int64_t ldx) {
  if (k <= 0) return;
  if (n < 1 || n > LU_NMAX) fail(CARE_ERR_ARG, "lu_solve: n must be in [1, " + std::to_string(LU_NMAX) + "]");
  if (ldb < n || ldx < n) fail(CARE_ERR_ARG, "lu_solve: leading dimension below n");
  constexpr int KB = sizeof(T) == 4 ? 2 : 1;
  hipLaunchKernelGGL((k_lu_solve<T, KB>), dim3(ceil_div(k, KB)), dim3(LS_NT), 0, ctx->stream, n, F, perm, k, B, ldb,
                     X, ldx);
  KERNEL_CHECK();
}

template void lu_factor_shifted<float>(Ctx*, int, const float*, const std::vector<double>&, const std::vector<float*>&,
                                       const std::vector<int*>&, std::vector<int>&, const std::vector<int*>&);
template void lu_factor_shifted<double>(Ctx*, int, const double*, const std::vector<double>&,
                                        const std::vector<double*>&, const std::vector<int*>&, std::vector<int>&,
                                        const std::vector<int*>&);
template void lu_solve<float>(Ctx*, int, const float*, const int*, int, const float*, int64_t, float*, int64_t);
template void lu_solve<double>(Ctx*, int, const double*, const int*, int, const double*, int64_t, double*, int64_t);

}  // namespace mpcare
