// Dense tall-skinny kernels on the FP64 matrix cores of gfx950, the small
// dense helpers, and the rank-revealing orthogonalisation used by
// Algorithms 1 and 2.
#include "dense.hpp"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdlib>
#include <numeric>

namespace mpcare {

typedef double double4_t __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operand layout (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the 16 x 16 result is returned as
// four doubles per lane, D[(l / 16) + 4 v][l % 16], v = 0..3 (checked on
// gfx950 against a host product).
__device__ __forceinline__ double4_t mfma16(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ double ldg_d(const T* p) {
  return (double)*p;
}

// ---------------------------------------------------------------------------
// Gram  C = X^T Y
// ---------------------------------------------------------------------------
// Grid: x = output tile (32 x 32) index, y = row split.  Each of the 4 waves
// accumulates the whole tile over every 4th 16-row group of its split; the
// waves are then summed through LDS and the tile is written to
// part[split][tile][32 x 32].  Row k of a 16-row group is fed to MFMA t from
// lane group g with k = 4 g + t, so each lane reads 4 consecutive rows of
// one column (32 B) per operand.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_gram(int64_t n, const TX* __restrict__ X, int64_t ldx, int a,
                                              const TY* __restrict__ Y, int64_t ldy, int b, int tiles_j,
                                              int64_t rows_per_split, const int* __restrict__ tile_list,
                                              double* __restrict__ part) {
  const int tl = blockIdx.x;
  const int tcode = tile_list ? tile_list[tl] : tl;   // no list: every tile, in order
  const int ti = tcode / tiles_j, tj = tcode % tiles_j;
  const int i0 = ti * 32, j0 = tj * 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_split;
  const int64_t rend = min(n, rbeg + rows_per_split);

  double4_t acc[2][2];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = (double4_t){0.0, 0.0, 0.0, 0.0};

  // column pointers (clamped; out-of-range columns are zeroed by a flag)
  const int xc0 = i0 + cl, xc1 = i0 + 16 + cl, yc0 = j0 + cl, yc1 = j0 + 16 + cl;
  const bool xv0 = xc0 < a, xv1 = xc1 < a, yv0 = yc0 < b, yv1 = yc1 < b;
  const TX* xp0 = X + (int64_t)(xv0 ? xc0 : 0) * ldx;
  const TX* xp1 = X + (int64_t)(xv1 ? xc1 : 0) * ldx;
  const TY* yp0 = Y + (int64_t)(yv0 ? yc0 : 0) * ldy;
  const TY* yp1 = Y + (int64_t)(yv1 ? yc1 : 0) * ldy;

  for (int64_t r0 = rbeg + (int64_t)wave * 16; r0 < rend; r0 += 64) {
    const int64_t rr = r0 + 4 * g;
    double x0[4], x1[4], y0[4], y1[4];
    if (rr + 3 < rend) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        x0[t] = xv0 ? ldg_d(xp0 + rr + t) : 0.0;
        x1[t] = xv1 ? ldg_d(xp1 + rr + t) : 0.0;
        y0[t] = yv0 ? ldg_d(yp0 + rr + t) : 0.0;
        y1[t] = yv1 ? ldg_d(yp1 + rr + t) : 0.0;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool ok = rr + t < rend;
        x0[t] = (xv0 && ok) ? ldg_d(xp0 + rr + t) : 0.0;
        x1[t] = (xv1 && ok) ? ldg_d(xp1 + rr + t) : 0.0;
        y0[t] = (yv0 && ok) ? ldg_d(yp0 + rr + t) : 0.0;
        y1[t] = (yv1 && ok) ? ldg_d(yp1 + rr + t) : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[0][0] = mfma16(x0[t], y0[t], acc[0][0]);
      acc[0][1] = mfma16(x0[t], y1[t], acc[0][1]);
      acc[1][0] = mfma16(x1[t], y0[t], acc[1][0]);
      acc[1][1] = mfma16(x1[t], y1[t], acc[1][1]);
    }
  }
  // reduce the 4 waves through LDS: tile element (i, j) at red[i * 33 + j]
  __shared__ double red[3][32 * 33];
  if (wave > 0) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = 16 * u + g + 4 * e, jj = 16 * v + cl;
          red[wave - 1][ii * 33 + jj] = acc[u][v][e];
        }
  }
  __syncthreads();
  if (wave == 0) {
    double* out = part + ((int64_t)blockIdx.y * gridDim.x + tl) * 1024;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ii = 16 * u + g + 4 * e, jj = 16 * v + cl;
          double s = acc[u][v][e];
          s += red[0][ii * 33 + jj];
          s += red[1][ii * 33 + jj];
          s += red[2][ii * 33 + jj];
          out[ii * 32 + jj] = s;
        }
  }
}

// C(i, j) = sum over splits (fixed order); symmetric: mirror the upper tiles.
// Grid (tiles, 4): one thread per element of a 32 x 32 tile; the split loop
// is unrolled so that several partials are in flight while the sum keeps its
// order.
__global__ void __launch_bounds__(256) k_gram_reduce(const double* __restrict__ part, int ntl, int nsplit,
                                                     const int* __restrict__ tile_list, int tiles_j, int a, int b,
                                                     int sym, double* __restrict__ C, int64_t ldc) {
  const int tl = blockIdx.x;
  const int tcode = tile_list ? tile_list[tl] : tl;
  const int ti = tcode / tiles_j, tj = tcode % tiles_j;
  const int e = blockIdx.y * 256 + threadIdx.x;
  const int ii = e >> 5, jj = e & 31;
  const int i = ti * 32 + ii, j = tj * 32 + jj;
  if (i >= a || j >= b) return;
  const double* p = part + (int64_t)tl * 1024 + e;
  const int64_t stride = (int64_t)ntl * 1024;
  double s = 0.0;
#pragma unroll 8
  for (int sp = 0; sp < nsplit; ++sp) s += p[sp * stride];
  C[(int64_t)j * ldc + i] = s;
  if (sym && ti != tj) C[(int64_t)i * ldc + j] = s;
}

// C(i, j) = sum_s W_s(i, j), s = 0 .. nsplit-1 in order (W_s: a x b, ld a);
// sym: the lower triangle mirrors the upper one, so C is exactly symmetric
__global__ void k_sum_partials(int a, int b, int nsplit, const double* __restrict__ W, double* __restrict__ C,
                               int64_t ldc, int sym) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= a || j >= b) return;
  const int64_t ab = (int64_t)a * b, o = (sym && i > j) ? (int64_t)i * a + j : (int64_t)j * a + i;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += W[k * ab + o];
  C[(int64_t)j * ldc + i] = s;
}

// ---------------------------------------------------------------------------
// Gram C = X^T Y in 128 x 128 output tiles (FP64)
// ---------------------------------------------------------------------------
// One workgroup (4 waves, 2 x 2) per output tile and row split; each wave
// owns a 64 x 64 quarter as 4 x 4 MFMA tiles (16 accumulators).  Rows come
// 16 at a time: the 16 x 128 slices of X and Y are staged in LDS (double
// buffered; the next slices' global loads are issued before the current
// slices' MFMAs), row k of the slice feeding MFMA step k / 4 from lane group
// k % 4.  The tile's partial sum goes to part (column-major 128 x 128 per
// tile and split) and k_gram128_reduce adds the splits in a fixed order.
constexpr int G128_PITCH = 128 + 2;   // LDS row pitch (doubles)

// Tile t of a ti x tj grid of 128 x 128 tiles, row by row; with sym only the
// tiles on and above the diagonal (ti == tj) are enumerated.
__device__ __forceinline__ void g128_tile(int t, int ti, int tj, int sym, int& I, int& J) {
  if (!sym) {
    I = t / tj;
    J = t % tj;
    return;
  }
  I = 0;
  while (t >= ti - I) {
    t -= ti - I;
    ++I;
  }
  J = I + t;
}

__global__ void __launch_bounds__(256) k_gram128(int64_t n, const double* __restrict__ X, int64_t ldx, int a,
                                                 const double* __restrict__ Y, int64_t ldy, int b, int ti, int tj,
                                                 int sym, int64_t rows_per_split, double* __restrict__ part) {
  __shared__ double xs[2][16 * G128_PITCH];
  __shared__ double ys[2][16 * G128_PITCH];
  const int tl = blockIdx.x;
  int TI, TJ;
  g128_tile(tl, ti, tj, sym, TI, TJ);
  const int i0 = TI * 128, j0 = TJ * 128;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  const int64_t rbeg = (int64_t)blockIdx.y * rows_per_split;
  const int64_t rend = min(n, rbeg + rows_per_split);

  // global -> register staging: thread t loads rows 8 (t % 2) .. + 7 of
  // column t / 2 of the X and Y slices
  const int sc = tid >> 1, sr = (tid & 1) * 8;
  const bool xok = i0 + sc < a, yok = j0 + sc < b;
  const double* xp = X + (int64_t)(xok ? i0 + sc : 0) * ldx;
  const double* yp = Y + (int64_t)(yok ? j0 + sc : 0) * ldy;
  double xr[8], yr[8];
  auto load = [&](int64_t r0) {
    const int64_t r = r0 + sr;
    if (r + 7 < rend) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        xr[e] = xok ? xp[r + e] : 0.0;
        yr[e] = yok ? yp[r + e] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool ok = r + e < rend;
        xr[e] = (xok && ok) ? xp[r + e] : 0.0;
        yr[e] = (yok && ok) ? yp[r + e] : 0.0;
      }
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      xs[buf][(sr + e) * G128_PITCH + sc] = xr[e];
      ys[buf][(sr + e) * G128_PITCH + sc] = yr[e];
    }
  };
  double4_t acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = (double4_t){0.0, 0.0, 0.0, 0.0};

  // 16 x 16 sub-tiles wholly past a or b (a ragged last tile) skip their MFMAs
  bool live[4], livej[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    live[u] = i0 + wi + 16 * u < a;
    livej[u] = j0 + wj + 16 * u < b;
  }
  int buf = 0;
  if (rbeg < rend) {
    load(rbeg);
    stage(0);
  }
  __syncthreads();
  for (int64_t r0 = rbeg; r0 < rend; r0 += 16) {
    const bool more = r0 + 16 < rend;
    if (more) load(r0 + 16);
    const double* xb = xs[buf];
    const double* yb = ys[buf];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 4 * t + lg;
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = xb[k * G128_PITCH + wi + 16 * u + li];
#pragma unroll
      for (int v = 0; v < 4; ++v) bv[v] = yb[k * G128_PITCH + wj + 16 * v + li];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (live[u] && livej[v]) acc[u][v] = mfma16(av[u], bv[v], acc[u][v]);
    }
    if (more) stage(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* out = part + ((int64_t)blockIdx.y * gridDim.x + tl) * (128 * 128);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ii = wi + 16 * u + lg + 4 * e, jj = wj + 16 * v + li;
        out[jj * 128 + ii] = acc[u][v][e];
      }
}

// C(i, j) = sum over the splits (in order) of the tile partials; with sym the
// entries below the diagonal take the value computed for (j, i), so C is
// exactly symmetric.
__global__ void k_gram128_reduce(const double* __restrict__ part, int ntl, int nsplit, int ti, int tj, int a, int b,
                                 int sym, double* __restrict__ C, int64_t ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= a || j >= b) return;
  const int si = (sym && i > j) ? j : i, sj = (sym && i > j) ? i : j;
  const int I = si >> 7, J = sj >> 7;
  // inverse of g128_tile
  const int tl = sym ? I * ti - I * (I - 1) / 2 + (J - I) : I * tj + J;
  const int64_t o = (int64_t)(sj & 127) * 128 + (si & 127);
  double s = 0.0;
#pragma unroll 8
  for (int sp = 0; sp < nsplit; ++sp) s += part[((int64_t)sp * ntl + tl) * (128 * 128) + o];
  C[(int64_t)j * ldc + i] = s;
}

static void gram128(Ctx* ctx, int64_t n, const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                    double* C, int64_t ldc) {
  const bool sym = X == Y && ldx == ldy && a == b;
  const int ti = (a + 127) / 128, tj = (b + 127) / 128;
  const int ntl = sym ? ti * (ti + 1) / 2 : ti * tj;
  // about two workgroups per compute unit, at least 512 rows per split
  const int64_t want = std::max<int64_t>(1, (int64_t)2 * ctx->num_cu / ntl);
  int64_t rps = std::max<int64_t>(512, (n + want - 1) / want);
  rps = (rps + 15) / 16 * 16;
  const int nsplit = (int)((n + rps - 1) / rps);
  DBuf<double> part(ctx, (size_t)nsplit * ntl * 128 * 128);
  hipLaunchKernelGGL(k_gram128, dim3(ntl, nsplit), dim3(256), 0, ctx->stream, n, X, ldx, a, Y, ldy, b, ti, tj,
                     sym ? 1 : 0, rps, part.get());
  KERNEL_CHECK();
  hipLaunchKernelGGL(k_gram128_reduce, dim3(ceil_div(a, 256), b), dim3(256), 0, ctx->stream, (const double*)part.get(),
                     ntl, nsplit, ti, tj, a, b, sym ? 1 : 0, C, ldc);
  KERNEL_CHECK();
}

template <typename TX, typename TY>
void gram(Ctx* ctx, int64_t n, const TX* X, int64_t ldx, int a, const TY* Y, int64_t ldy, int b, double* C,
          int64_t ldc) {
  if (a <= 0 || b <= 0) return;
  if (n <= 0) {
    for (int j = 0; j < b; ++j) dzero(ctx, C + (int64_t)j * ldc, a * sizeof(double));
    return;
  }
  if constexpr (sizeof(TX) == 8 && sizeof(TY) == 8) {
    // The own 128 x 128-tile kernel for the symmetric Grams X^T X where it
    // was measured faster than rocBLAS (it computes only the tiles on and
    // above the diagonal): up to 512 columns, or while X stays within
    // 1.5 GB (beyond, its per-tile re-reads of X from HBM dominate; n =
    // 250000: q = 206 / 417 take 0.51 / 1.65 ms against 0.54 / 1.98 ms,
    // q = 1026 10.8 ms against 10.3 ms; n = 125000, q = 1218: 4.8 against
    // 6.4 ms).  gram_impl 1 uses it for every large Gram, 0 never.
    const bool symx = (const void*)X == (const void*)Y && ldx == ldy && a == b;
    const bool own = ctx->gram_impl == 1 ||
                     (ctx->gram_impl == 2 && symx && (a <= 512 || (double)n * a * 8.0 <= 1.5e9));
    if (own && (int64_t)a * b >= 32 * 32 && a < 65536 && b < 65536) {
      gram128(ctx, n, (const double*)X, ldx, a, (const double*)Y, ldy, b, C, ldc);
      return;
    }
    // large FP64 Grams: rocBLAS dgemm (MFMA) over row chunks (split-K as a
    // strided batch), partial products summed in a fixed order, so the result
    // is reproducible (atomics are also disabled on the context's handle)
    if ((int64_t)a * b >= 32 * 32 && n <= INT32_MAX && ldx <= INT32_MAX && ldy <= INT32_MAX) {
      const int64_t tiles = (int64_t)((a + 127) / 128) * ((b + 127) / 128);
      int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>(64, (2048 + tiles - 1) / tiles));
      nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, n / 2048));
      const double one = 1.0, zero = 0.0;
      const bool sym = (const void*)X == (const void*)Y && ldx == ldy && a == b;
      if (nsplit <= 1 && !sym) {
        ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, a, b, (int)n, &one,
                                    (const double*)X, (int)ldx, (const double*)Y, (int)ldy, &zero, C, (int)ldc));
        return;
      }
      // nsplit equal chunks of rc rows in one strided batch, the remainder
      // (< 64 nsplit rows) as one more partial product
      const int64_t rc = nsplit > 1 ? n / nsplit / 64 * 64 : n;
      const int64_t rem = n - nsplit * rc;
      const int64_t ab = (int64_t)a * b;
      const int nparts = (int)nsplit + (rem > 0 ? 1 : 0);
      DBuf<double> W(ctx, (size_t)(ab * nparts));
      ROCBLAS_CHECK(rocblas_dgemm_strided_batched(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, a, b,
                                                  (int)rc, &one, (const double*)X, (int)ldx, rc, (const double*)Y,
                                                  (int)ldy, rc, &zero, W.get(), a, ab, (int)nsplit));
      if (rem > 0)
        ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none, a, b, (int)rem,
                                    &one, (const double*)X + nsplit * rc, (int)ldx, (const double*)Y + nsplit * rc,
                                    (int)ldy, &zero, W.get() + nsplit * ab, a));
      dim3 g(ceil_div(a, 256), b);
      hipLaunchKernelGGL(k_sum_partials, g, dim3(256), 0, ctx->stream, a, b, nparts, (const double*)W.get(), C, ldc,
                         sym ? 1 : 0);
      KERNEL_CHECK();
      return;
    }
  }
  const bool sym = (const void*)X == (const void*)Y && ldx == ldy && a == b && sizeof(TX) == sizeof(TY);
  const int tiles_i = (a + 31) / 32, tiles_j = (b + 31) / 32;
  std::vector<int> tl;
  for (int i = 0; i < tiles_i; ++i)
    for (int j = 0; j < tiles_j; ++j)
      if (!sym || j >= i) tl.push_back(i * tiles_j + j);
  const int ntl = (int)tl.size();
  // aim at ~4 workgroups per CU, at least 256 rows per split
  int64_t want = std::max<int64_t>(1, (int64_t)4 * ctx->num_cu / ntl);
  int64_t rps = std::max<int64_t>(256, (n + want - 1) / want);
  rps = (rps + 63) / 64 * 64;
  const int nsplit = (int)((n + rps - 1) / rps);
  DBuf<int> dtl(ctx, ntl);
  h2d(ctx, dtl.get(), tl.data(), ntl * sizeof(int));
  DBuf<double> part(ctx, (size_t)nsplit * ntl * 1024);
  hipLaunchKernelGGL((k_gram<TX, TY>), dim3(ntl, nsplit), dim3(256), 0, ctx->stream, n, X, ldx, a, Y, ldy, b, tiles_j,
                     rps, dtl.get(), part.get());
  KERNEL_CHECK();
  hipLaunchKernelGGL(k_gram_reduce, dim3(ntl, 4), dim3(256), 0, ctx->stream, part.get(), ntl, nsplit, dtl.get(),
                     tiles_j, a, b, sym ? 1 : 0, C, ldc);
  KERNEL_CHECK();
}

// The library's own FP64 MFMA Gram over every 32 x 32 output tile, with the
// row-split partials in a caller-provided buffer of `part_doubles` doubles;
// no allocation and no host-to-device copy.  Returns false (nothing
// launched) when one row split of partials does not fit.
bool gram_own_into(Ctx* ctx, int64_t n, const double* X, int64_t ldx, int a, const double* Y, int64_t ldy, int b,
                   double* C, int64_t ldc, double* part, size_t part_doubles) {
  const int tiles_i = (a + 31) / 32, tiles_j = (b + 31) / 32;
  const int64_t ntl = (int64_t)tiles_i * tiles_j;
  if (ntl * 1024 > (int64_t)part_doubles) return false;
  // aim at ~4 workgroups per CU, at least 256 rows per split, within the buffer
  const int64_t cap = (int64_t)part_doubles / (ntl * 1024);
  int64_t want = std::max<int64_t>(1, std::min<int64_t>(cap, (int64_t)4 * ctx->num_cu / ntl));
  int64_t rps = std::max<int64_t>(256, (n + want - 1) / want);
  rps = (rps + 63) / 64 * 64;
  int64_t nsplit = (n + rps - 1) / rps;
  while (nsplit > cap) {           // rounding of rps up can leave one split too many
    rps += 64;
    nsplit = (n + rps - 1) / rps;
  }
  nsplit = std::max<int64_t>(nsplit, 1);
  hipLaunchKernelGGL((k_gram<double, double>), dim3((unsigned)ntl, (unsigned)nsplit), dim3(256), 0, ctx->stream, n, X,
                     ldx, a, Y, ldy, b, tiles_j, rps, (const int*)nullptr, part);
  KERNEL_CHECK();
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)ntl, 4), dim3(256), 0, ctx->stream, (const double*)part, (int)ntl,
                     (int)nsplit, (const int*)nullptr, tiles_j, a, b, 0, C, ldc);
  KERNEL_CHECK();
  return true;
}

// ---------------------------------------------------------------------------
// tall-skinny GEMM  Y = alpha X S + beta Y
// ---------------------------------------------------------------------------
// Each wave computes a 16-row x 64-column block of Y as Y^T = S^T X^T:
// A' = S^T (lane: S[k][j0 + l % 16]), B' = X^T (lane: X[r0 + l % 16][k]),
// result lane l, v -> Y[r0 + l % 16][j0 + (l / 16) + 4 v], so every store
// instruction writes 16 consecutive rows of a column.
template <typename TX, typename TY>
__global__ void __launch_bounds__(256) k_tsgemm(int64_t n, const TX* __restrict__ X, int64_t ldx, int q,
                                                const double* __restrict__ S, int64_t lds, int k, double alpha,
                                                double beta, TY* __restrict__ Yp, int64_t ldy) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int64_t r0 = ((int64_t)xcd_remap(blockIdx.x, gridDim.x) * 4 + wave) * 16;
  const int jbase = blockIdx.y * 64;
  if (r0 >= n) return;
  const int64_t row = r0 + cl;
  const bool rv = row < n;
  double4_t acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = (double4_t){0.0, 0.0, 0.0, 0.0};
  int jc[4];
  bool jv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    jc[u] = jbase + 16 * u + cl;
    jv[u] = jc[u] < k;
  }
  for (int k0 = 0; k0 < q; k0 += 16) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int kk = k0 + 4 * g + t;       // row of S / column of X fed by this lane
      const bool kv = kk < q;
      const double xb = (kv && rv) ? ldg_d(X + (int64_t)kk * ldx + row) : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double sa = (kv && jv[u]) ? S[(int64_t)jc[u] * lds + kk] : 0.0;
        acc[u] = mfma16(sa, xb, acc[u]);
      }
    }
  }
  // lane holds Y[r0 + cl][jbase + 16 u + g + 4 v]
  if (!rv) return;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = jbase + 16 * u + g + 4 * v;
      if (j < k) {
        TY* yp = Yp + (int64_t)j * ldy + row;
        double val = alpha * acc[u][v];
        if (beta != 0.0) val += beta * (double)*yp;
        *yp = (TY)val;
      }
    }
}

template <typename TX, typename TY>
void tsgemm(Ctx* ctx, int64_t n, const TX* X, int64_t ldx, int q, const double* S, int64_t lds, int k, double alpha,
            double beta, TY* Y, int64_t ldy) {
  if (n <= 0 || k <= 0) return;
  if (q <= 0) {   // X S is empty: Y = beta Y
    if (beta == 0.0) {
      for (int j = 0; j < k; ++j) dzero(ctx, Y + (int64_t)j * ldy, n * sizeof(TY));
    } else if (beta != 1.0) {
      axpby<TY>(ctx, n, k, 0.0, Y, ldy, beta, Y, ldy);
    }
    return;
  }
  if constexpr (sizeof(TX) == 8 && sizeof(TY) == 8) {
    if ((int64_t)q * k >= 64 * 64 && n <= INT32_MAX && ldx <= INT32_MAX && ldy <= INT32_MAX) {
      ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, rocblas_operation_none, rocblas_operation_none, (int)n, k, q, &alpha,
                                  (const double*)X, (int)ldx, S, (int)lds, &beta, (double*)Y, (int)ldy));
      return;
    }
  }
  dim3 grid(ceil_div(n, 64), ceil_div(k, 64));
  hipLaunchKernelGGL((k_tsgemm<TX, TY>), grid, dim3(256), 0, ctx->stream, n, X, ldx, q, S, lds, k, alpha, beta, Y,
                     ldy);
  KERNEL_CHECK();
}

template <typename T>
__global__ void k_fill_const(T* __restrict__ p, size_t count, T v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
void fill_const(Ctx* ctx, T* p, size_t count, double v) {
  if (!count) return;
  const unsigned grid = (unsigned)std::min<size_t>((count + 255) / 256, 16384);
  hipLaunchKernelGGL((k_fill_const<T>), dim3(grid), dim3(256), 0, ctx->stream, p, count, (T)v);
  KERNEL_CHECK();
}
template void fill_const<double>(Ctx*, double*, size_t, double);
template void fill_const<float>(Ctx*, float*, size_t, double);

// ---------------------------------------------------------------------------
// column copies
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ void k_copy_cols(int64_t n, int ncols, const TI* __restrict__ in, int64_t ldi, TO* __restrict__ out,
                            int64_t ldo, const int* __restrict__ map, const double* __restrict__ scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= ncols) return;
  const int src = map ? map[c] : c;
  double v = 0.0;
  if (src >= 0) v = (double)in[(int64_t)src * ldi + i];
  if (scale) v *= scale[c];
  out[(int64_t)c * ldo + i] = (TO)v;
}

template <typename TI, typename TO>
void copy_cols(Ctx* ctx, int64_t n, int ncols, const TI* in, int64_t ldi, TO* out, int64_t ldo, const int* map,
               const double* scale) {
  if (n <= 0 || ncols <= 0) return;
  DBuf<int> dmap;
  DBuf<double> dscale;
  if (map) {
    dmap.resize(ctx, ncols);
    h2d(ctx, dmap.get(), map, ncols * sizeof(int));
  }
  if (scale) {
    dscale.resize(ctx, ncols);
    h2d(ctx, dscale.get(), scale, ncols * sizeof(double));
  }
  for (int c0 = 0; c0 < ncols; c0 += 65535) {
    const int nc = std::min(ncols - c0, 65535);
    dim3 g(ceil_div(n, 256), nc);
    hipLaunchKernelGGL((k_copy_cols<TI, TO>), g, dim3(256), 0, ctx->stream, n, nc, in, ldi, out + (int64_t)c0 * ldo,
                       ldo, map ? dmap.get() + c0 : nullptr, scale ? dscale.get() + c0 : nullptr);
    KERNEL_CHECK();
  }
}

template <typename T>
__global__ void k_axpby(int64_t n, int ncols, double a, const T* __restrict__ X, int64_t ldx, double b,
                        T* __restrict__ Y, int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= ncols) return;
  T* y = Y + (int64_t)c * ldy + i;
  const double xv = (double)X[(int64_t)c * ldx + i];
  *y = (T)(a * xv + (b != 0.0 ? b * (double)*y : 0.0));
}

template <typename T>
void axpby(Ctx* ctx, int64_t n, int ncols, double a, const T* X, int64_t ldx, double b, T* Y, int64_t ldy) {
  if (n <= 0 || ncols <= 0) return;
  dim3 g(ceil_div(n, 256), ncols);
  hipLaunchKernelGGL((k_axpby<T>), g, dim3(256), 0, ctx->stream, n, ncols, a, X, ldx, b, Y, ldy);
  KERNEL_CHECK();
}
template void axpby<double>(Ctx*, int64_t, int, double, const double*, int64_t, double, double*, int64_t);
template void axpby<float>(Ctx*, int64_t, int, double, const float*, int64_t, double, float*, int64_t);

#define INST_GRAM(TX, TY) \
  template void gram<TX, TY>(Ctx*, int64_t, const TX*, int64_t, int, const TY*, int64_t, int, double*, int64_t);
INST_GRAM(double, double)
INST_GRAM(float, float)
INST_GRAM(float, double)
INST_GRAM(double, float)
#define INST_TS(TX, TY)                                                                                      \
  template void tsgemm<TX, TY>(Ctx*, int64_t, const TX*, int64_t, int, const double*, int64_t, int, double, \
                               double, TY*, int64_t);
INST_TS(double, double)
INST_TS(float, float)
INST_TS(double, float)
INST_TS(float, double)
#define INST_CP(TI, TO) \
  template void copy_cols<TI, TO>(Ctx*, int64_t, int, const TI*, int64_t, TO*, int64_t, const int*, const double*);
INST_CP(double, double)
INST_CP(double, float)
INST_CP(float, double)
INST_CP(float, float)

// ---------------------------------------------------------------------------
// small dense helpers
// ---------------------------------------------------------------------------
void dgemm(Ctx* ctx, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda, const double* B,
           int ldb, double beta, double* C, int ldc) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0) {
    if (beta == 0.0)
      for (int j = 0; j < n; ++j) dzero(ctx, C + (int64_t)j * ldc, m * sizeof(double));
    return;
  }
  ROCBLAS_CHECK(rocblas_dgemm(ctx->blas, ta ? rocblas_operation_transpose : rocblas_operation_none,
                              tb ? rocblas_operation_transpose : rocblas_operation_none, m, n, k, &alpha, A, lda, B,
                              ldb, &beta, C, ldc));
}

void dsyevd(Ctx* ctx, int n, double* A, int lda, std::vector<double>& w) {
  w.assign(n, 0.0);
  if (n <= 0) return;
  DBuf<double> D(ctx, n), E(ctx, n);
  DBuf<int> info(ctx, 1);
  ROCBLAS_CHECK(rocsolver_dsyevd(ctx->blas, rocblas_evect_original, rocblas_fill_upper, n, A, lda, D.get(), E.get(),
                                 info.get()));
  int hinfo = 0;
  d2h(ctx, &hinfo, info.get(), sizeof(int));
  if (hinfo != 0) fail(CARE_ERR_DEVICE, "rocsolver_dsyevd did not converge (info " + std::to_string(hinfo) + ")");
  d2h(ctx, w.data(), D.get(), n * sizeof(double));
}

__global__ void k_scale_sym(double* __restrict__ G, int64_t ldg, int q, const double* __restrict__ s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < q) G[(int64_t)j * ldg + i] *= s[i] * s[j];
}
__global__ void k_scale_rows(double* __restrict__ A, int64_t lda, int m, int ncols, const double* __restrict__ s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < m && j < ncols) A[(int64_t)j * lda + i] *= s[i];
}

// ---------------------------------------------------------------------------
// rank-revealing orthogonalisation
// ---------------------------------------------------------------------------
// Pass structure (all FP64):
//   E_0 = F.  Pass p: G = E_p^T E_p, scaled by the inverse column norms of F
//   (so thresholds are relative to each column of F); G~ = W L W^T.  Keep
//   directions with l > max(1e-11 max l, noise), noise = (64 u)^2 q: they
//   give U_new = E_p S W_sel L_sel^{-1/2}, whose Gram has condition number
//   <= 1e11 * (1 + O(u)), so one Cholesky polish makes it orthonormal.  U_new
//   is made orthogonal to the previous U (two Gram-Schmidt passes), then
//   E_{p+1} = F - U U^T F (two passes).  The loop ends when E carries no
//   direction above the noise level; T = U^T F.  Unlike Cholesky QR this
//   handles rank-deficient F (columns of Z Z^T B lie in range(Z); ADI blocks
//   are nearly collinear) and keeps the small directions that carry the
//   Riccati residual, to the accuracy of Householder QR.
// Re-orthonormalise the k nearly orthonormal columns of U in place:
// U^T U = V D V^T, U <- U V D^{-1/2} over the eigenvalues D > 1e-8 max D.
// Returns the number of columns kept (at the front of U); a column that the
// projection against earlier passes reduced to noise is dropped here and
// its direction, if real, is met again by the next pass.
static int polish(Ctx* ctx, int64_t n, double* U, int64_t ldu, int k, bool trace) {
  if (k <= 0) return 0;
  DBuf<double> G(ctx, (size_t)k * k);
  gram(ctx, n, U, ldu, k, U, ldu, k, G.get(), k);
  {
    // Fast path: when Gershgorin puts every eigenvalue of U^T U in [0.5, 2]
    // (condition <= 4), the Cholesky factor U^T U = L L^T re-orthonormalises
    // U <- U L^{-T} to O(u kappa) = O(u); its blocked factorisation has far
    // fewer sequential steps than the eigen-decomposition below.  A fresh
    // block of the first pass typically has eigenvalues within 1e-4 of 1.
    std::vector<double> hg((size_t)k * k);
    d2h(ctx, hg.data(), G.get(), hg.size() * sizeof(double));
    double lo = INFINITY, hi = 0.0;
    for (int i = 0; i < k; ++i) {
      double off = 0.0;
      for (int j = 0; j < k; ++j)
        if (j != i) off += std::fabs(hg[(size_t)j * k + i]);
      lo = std::min(lo, hg[(size_t)i * k + i] - off);
      hi = std::max(hi, hg[(size_t)i * k + i] + off);
    }
    if (lo >= 0.5 && hi <= 2.0 && n <= INT32_MAX && ldu <= INT32_MAX) {
      DBuf<int> info(ctx, 1);
      ROCBLAS_CHECK(rocsolver_dpotrf(ctx->blas, rocblas_fill_lower, k, G.get(), k, info.get()));
      int hinfo = 0;
      d2h(ctx, &hinfo, info.get(), sizeof(int));
      if (hinfo == 0) {
        const double one = 1.0;
        ROCBLAS_CHECK(rocblas_dtrsm(ctx->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                                    rocblas_diagonal_non_unit, (int)n, k, &one, G.get(), k, U, (int)ldu));
        if (trace)
          std::fprintf(stderr, "[rr_orth] polish k %d by Cholesky, Gershgorin [%.3e, %.3e]\n", k, lo, hi);
        return k;
      }
      gram(ctx, n, U, ldu, k, U, ldu, k, G.get(), k);   // the factorisation overwrote G
    }
  }
  std::vector<double> d;
  dsyevd(ctx, k, G.get(), k, d);
  const double dmax = d.empty() ? 0.0 : d.back();
  std::vector<int> sel;
  std::vector<double> isq;
  for (int i = k - 1; i >= 0; --i)
    if (d[i] > 1e-8 * dmax) {
      sel.push_back(i);
      isq.push_back(1.0 / std::sqrt(d[i]));
    }
  if (trace)
    std::fprintf(stderr, "[rr_orth] polish k %d kept %zu eig [%.3e, %.3e]\n", k, sel.size(), d.empty() ? 0.0 : d[0],
                 dmax);
  const int kk = (int)sel.size();
  if (kk == 0) return 0;
  DBuf<double> B(ctx, (size_t)k * kk);
  copy_cols<double, double>(ctx, k, kk, G.get(), k, B.get(), k, sel.data(), isq.data());
  DBuf<double> tmp(ctx, (size_t)pad_ld(n) * kk);
  tsgemm(ctx, n, U, ldu, k, B.get(), k, kk, 1.0, 0.0, tmp.get(), pad_ld(n));
  copy_cols<double, double>(ctx, n, kk, tmp.get(), pad_ld(n), U, ldu);
  return kk;
}

// out[j] = sum_i (s_i G_ij s_j)^2, one block per column j
__global__ void __launch_bounds__(256) k_scaled_colsq(const double* __restrict__ G, int64_t ldg, int q,
                                                      const double* __restrict__ s, double* __restrict__ out) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < q; i += 256) {
    const double v = s[i] * G[(int64_t)j * ldg + i] * s[j];
    acc += v * v;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sh[0];
}

void rr_orth(Ctx* ctx, int64_t n, const double* F, int64_t ldf, int q, Orth& out) {
  rr_orth(ctx, n, F, ldf, q, out, nullptr, 0, 0);
}

void rr_orth(Ctx* ctx, int64_t n, const double* F, int64_t ldf, int q, Orth& out, const double* U0, int64_t ldu0,
             int k0) {
  const double u = 1.1102230246251565e-16;
  const bool trace = std::getenv("MPCARE_TRACE") != nullptr;
  const int64_t ld = pad_ld(n);
  if (!U0) k0 = 0;
  const int kcap = k0 + q;           // rank bound of [U0, F]
  out.ldu = ld;
  out.k = 0;
  out.U.resize(ctx, (size_t)ld * std::max(kcap, 1));
  out.T.resize(ctx, (size_t)std::max(kcap, 1) * std::max(q, 1));
  if (k0 > 0) copy_cols<double, double>(ctx, n, k0, U0, ldu0, out.U.get(), ld);
  if (q <= 0) {
    out.k = k0;
    return;
  }

  // column norms of F -> s = 1 / ||F_j|| (0 for zero columns)
  DBuf<double> G(ctx, (size_t)q * q);
  gram(ctx, n, F, ldf, q, F, ldf, q, G.get(), q);
  std::vector<double> hG((size_t)q * q);
  d2h(ctx, hG.data(), G.get(), hG.size() * sizeof(double));
  std::vector<double> s(q);
  for (int j = 0; j < q; ++j) {
    const double d = hG[(size_t)j * q + j];
    s[j] = d > 0 ? 1.0 / std::sqrt(d) : 0.0;
  }
  DBuf<double> ds(ctx, q);
  h2d(ctx, ds.get(), s.data(), q * sizeof(double));

  // E: the remainder F - U (U^T F), updated in place block by block
  DBuf<double> E(ctx, (size_t)ld * q);
  copy_cols<double, double>(ctx, n, q, F, ldf, E.get(), ld);
  const double* Ecur = E.get();
  const int64_t lde = ld;
  const double noise = (64.0 * u) * (64.0 * u) * q;
  DBuf<double> W(ctx, (size_t)q * q), B(ctx, (size_t)q * q), Tf(ctx, (size_t)kcap * q), T2(ctx, (size_t)kcap * q);
  // search-space bases of the passes (see below) and their work space
  DBuf<double> Rest(ctx, (size_t)q * q), RestNext(ctx, (size_t)q * q), Tmp(ctx, (size_t)q * q),
      Hred(ctx, (size_t)q * q);
  bool have_rest = false;
  int nrest = 0;
  // T = U^T F with rows added block by block (leading dimension kcap)
  DBuf<double> Tacc(ctx, (size_t)kcap * q);
  dzero(ctx, Tacc.get(), (size_t)kcap * q * sizeof(double));
  std::vector<double> lam;
  // For the block U_b = U(:, c0:c1) just added: E -= U_b (U_b^T E), twice
  // (block classical Gram-Schmidt with reorthogonalisation), and its rows of
  // T are U_b^T E summed over both sweeps.  E is already orthogonal to the
  // earlier columns and so is U_b, so U_b^T F = U_b^T E to rounding, and the
  // earlier blocks need no second look.
  auto project_block = [&](int c0, int c1) {
    const int kb = c1 - c0;
    if (kb <= 0) return;
    const double* Ub = out.U.get() + (int64_t)c0 * ld;
    for (int rep = 0; rep < 2; ++rep) {
      gram(ctx, n, Ub, ld, kb, E.get(), ld, q, Tf.get(), kb);
      tsgemm(ctx, n, Ub, ld, kb, Tf.get(), kb, q, -1.0, 1.0, E.get(), ld);
      axpby<double>(ctx, kb, q, 1.0, Tf.get(), kb, 1.0, Tacc.get() + c0, kcap);
    }
  };
  if (k0 > 0) {
    out.k = k0;
    project_block(0, k0);
  }
  DBuf<double> csq(ctx, q);
  std::vector<double> hcsq(q);
  // Frobenius norm of the scaled Gram of the current remainder (G holds
  // the Gram afterwards); it bounds the remainder's largest eigenvalue
  auto remainder_fro = [&]() {
    gram(ctx, n, Ecur, lde, q, Ecur, lde, q, G.get(), q);
    hipLaunchKernelGGL(k_scaled_colsq, dim3(q), dim3(256), 0, ctx->stream, G.get(), (int64_t)q, q, ds.get(),
                       csq.get());
    KERNEL_CHECK();
    d2h(ctx, hcsq.data(), csq.get(), (size_t)q * sizeof(double));
    double fro2 = 0.0;
    for (double v : hcsq) fro2 += v;
    return std::sqrt(fro2);
  };
  // Each pass resolves about eleven decades of the scaled Gram's spectrum
  // and the noise floor lies about 28 decades down, so three passes
  // normally suffice; the loop ends earlier when the remainder reaches the
  // noise level or F's rank is exhausted.
  const int max_passes = 6;
  bool complete = false;
  for (int pass = 0; pass < max_passes; ++pass) {
    if (pass > 0 || k0 > 0) {
      // a remainder at the noise level ends the loop here, as the eigen-
      // decomposition below would (it selects nothing when lmax <= noise)
      const double fro = remainder_fro();
      if (fro <= noise) {
        if (trace)
          std::fprintf(stderr, "[rr_orth] n %lld q %d pass %d ||G||_F %.3e at noise: done\n", (long long)n, q, pass,
                       fro);
        complete = true;
        break;
      }
    }
    d2d(ctx, W.get(), G.get(), (size_t)q * q * sizeof(double));
    dim3 gs(ceil_div(q, 64), q);
    hipLaunchKernelGGL(k_scale_sym, gs, dim3(64), 0, ctx->stream, W.get(), (int64_t)q, q, ds.get());
    KERNEL_CHECK();
    // Search space of this pass, in the scaled coordinates of F's columns:
    // all of R^q, or, after a pass whose new columns were all kept, the
    // directions that pass left unselected (Rest, q x nrest, orthonormal).
    // The remainder E S then lies in span(Rest) up to rounding: the pass took
    // out exactly span(E S W_sel), and E S = (E S W_sel) W_sel^T +
    // (E S Rest) Rest^T.  The eigen-decomposition then has order nrest
    // instead of q.
    const bool reduced = have_rest;
    const int nb = reduced ? nrest : q;
    if (reduced && nb == 0) {
      complete = true;
      break;
    }
    double* Hm = W.get();
    if (reduced) {
      dgemm(ctx, false, false, q, nb, q, 1.0, W.get(), q, Rest.get(), q, 0.0, Tmp.get(), q);
      dgemm(ctx, true, false, nb, nb, q, 1.0, Rest.get(), q, Tmp.get(), q, 0.0, Hred.get(), nb);
      Hm = Hred.get();
    }
    dsyevd(ctx, nb, Hm, nb, lam);
    const double lmax = *std::max_element(lam.begin(), lam.end());
    const double thr = std::max(1e-11 * lmax, noise);
    std::vector<int> sel, rest;
    std::vector<double> isq;
    for (int i = nb - 1; i >= 0; --i) {
      if (lam[i] > thr && out.k + (int)sel.size() < kcap) {
        sel.push_back(i);
        isq.push_back(1.0 / std::sqrt(lam[i]));
      } else {
        rest.push_back(i);
      }
    }
    if (sel.empty()) {
      complete = true;
      break;
    }
    const int kk = (int)sel.size();
    // the next search space and B = S W_sel L_sel^{-1/2}, with W_sel the
    // selected eigenvectors in R^q (Rest times those of the reduced matrix)
    const int nr = (int)rest.size();
    if (reduced) {
      copy_cols<double, double>(ctx, nb, kk, Hm, nb, Tmp.get(), nb, sel.data(), isq.data());
      dgemm(ctx, false, false, q, kk, nb, 1.0, Rest.get(), q, Tmp.get(), nb, 0.0, B.get(), q);
      if (nr > 0) {
        copy_cols<double, double>(ctx, nb, nr, Hm, nb, Tmp.get(), nb, rest.data());
        dgemm(ctx, false, false, q, nr, nb, 1.0, Rest.get(), q, Tmp.get(), nb, 0.0, RestNext.get(), q);
      }
    } else {
      copy_cols<double, double>(ctx, q, kk, W.get(), q, B.get(), q, sel.data(), isq.data());
      if (nr > 0) copy_cols<double, double>(ctx, q, nr, W.get(), q, RestNext.get(), q, rest.data());
    }
    dim3 gr(ceil_div(q, 64), kk);
    hipLaunchKernelGGL(k_scale_rows, gr, dim3(64), 0, ctx->stream, B.get(), (int64_t)q, q, kk, ds.get());
    KERNEL_CHECK();
    double* Unew = out.U.get() + (int64_t)out.k * ld;
    tsgemm(ctx, n, Ecur, lde, q, B.get(), q, kk, 1.0, 0.0, Unew, ld);
    if (out.k > 0) {
      for (int rep = 0; rep < 2; ++rep) {   // Unew -= U (U^T Unew)
        gram(ctx, n, out.U.get(), ld, out.k, Unew, ld, kk, T2.get(), out.k);
        tsgemm(ctx, n, out.U.get(), ld, out.k, T2.get(), out.k, kk, -1.0, 1.0, Unew, ld);
      }
    }
    if (trace)
      std::fprintf(stderr, "[rr_orth] n %lld q %d pass %d search %d lmax %.3e thr %.3e new %d\n", (long long)n, q,
                   pass, nb, lmax, thr, kk);
    const int kept = polish(ctx, n, Unew, ld, kk, trace);
    if (kept == 0) {
      complete = true;      // what is left projects to noise (polish dropped it)
      break;
    }
    // a polish that dropped columns leaves part of span(E S W_sel) in the
    // remainder: the next pass searches all of R^q again
    have_rest = kept == kk;
    nrest = nr;
    if (have_rest) std::swap(Rest, RestNext);
    const int kold = out.k;
    out.k += kept;
    project_block(kold, out.k);
    if (out.k >= kcap) {
      complete = true;      // the basis spans [U0, F]
      break;
    }
  }
  // The pass cap must not leave a part of F above the noise level out of T:
  // Algorithm 1 would then underestimate ||R||_F, Framework 1's stop test.
  if (!complete && remainder_fro() > noise)
    fail(CARE_ERR_BREAKDOWN, "rank-revealing orthogonalisation left a remainder above the noise level after " +
                                 std::to_string(max_passes) + " passes");
  if (out.k == 0) return;
  copy_cols<double, double>(ctx, out.k, q, Tacc.get(), kcap, out.T.get(), out.k);
  ctx->sync();
}

}  // namespace mpcare
