// Algorithm 1, first step, in float64: the Gram matrix G = B^T B of the
// preconditioned m x n matrix. Only the upper 16 x 16 tiles are formed
// (symmetric rank-k update). Grid = row chunks; a workgroup of 4 waves
// stages 64-row panels of B in LDS (row-major, coalesced column loads) and
// each wave accumulates its share of the upper tiles with float64 MFMA
// 16x16x4. Per-chunk partials are summed in a second kernel in fixed order
// (deterministic, no atomics).
#include "common.hpp"

namespace mrcqr {

constexpr int GR_THREADS = 256;
constexpr int GR_PANEL = 64;
constexpr int GR_NMAX = 128;
constexpr int GR_NB = GR_NMAX / 16;
constexpr int GR_LDR = 66;  // column stride (doubles) of the LDS panel

// Each wave owns the upper tiles of block rows I1 = w and I2 = nb-1-w
// (9 tiles per wave for nb = 8). Per K step it loads every block column it
// needs once (the A and B operand layouts coincide for B^T B) and issues
// one MFMA per tile. The panel is column-major in LDS with a 66-double
// column stride: coalesced 64-row column stores and the operand reads
// (16 columns x 4 rows per wave) both hit distinct banks.
__global__ __launch_bounds__(GR_THREADS) void syrk_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, int rows_per_chunk,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ double tile[2][GR_NMAX * GR_LDR];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nb = (n + 15) / 16;
  const int64_t tstart = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t tend = min((int64_t)m, tstart + rows_per_chunk);
  const int npan = (int)((tend - tstart + GR_PANEL - 1) / GR_PANEL);
  const int I1 = w, I2 = nb - 1 - w;
  const bool has1 = I1 < nb && I1 <= I2, has2 = I2 > I1;
  const int xmin = has2 ? I1 : (has1 ? I1 : nb);

  f64x4 acc1[GR_NB], acc2[GR_NB];
#pragma unroll
  for (int J = 0; J < GR_NB; ++J) { acc1[J] = f64x4{0, 0, 0, 0}; acc2[J] = f64x4{0, 0, 0, 0}; }

  constexpr int EPT = GR_PANEL * GR_NMAX / GR_THREADS;  // 32 columns per thread, one row
  double regs[EPT];
  auto load_panel = [&](int64_t t0) {
    const int64_t t = t0 + l;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int col = w + 4 * e;
      regs[e] = (t < tend && col < n) ? B[t + (int64_t)col * ldb] : 0.0;
    }
  };
  if (npan > 0) load_panel(tstart);
  for (int p = 0; p < npan; ++p) {
    const int buf = p & 1;
#pragma unroll
    for (int e = 0; e < EPT; ++e) tile[buf][(w + 4 * e) * GR_LDR + l] = regs[e];
    if (p + 1 < npan) load_panel(tstart + (int64_t)(p + 1) * GR_PANEL);
    __syncthreads();
    const double* tb = tile[buf] + c16 * GR_LDR + g;
#pragma unroll 2
    for (int kk = 0; kk < GR_PANEL / 4; ++kk) {
      const double* tk = tb + 4 * kk;
      double op[GR_NB];
#pragma unroll
      for (int X = 0; X < GR_NB; ++X) op[X] = (X >= xmin && X < nb) ? tk[16 * X * GR_LDR] : 0.0;
      const double a1 = has1 ? tk[16 * I1 * GR_LDR] : 0.0;
      const double a2 = has2 ? tk[16 * I2 * GR_LDR] : 0.0;
#pragma unroll
      for (int J = 0; J < GR_NB; ++J) {
        if (has1 && J >= I1 && J < nb) acc1[J] = mfma_f64(a1, op[J], acc1[J]);
        if (has2 && J >= I2 && J < nb) acc2[J] = mfma_f64(a2, op[J], acc2[J]);
      }
    }
  }
  // Gpart[chunk][col][row] for the upper tiles (f64 D layout)
  double* Gp = Gpart + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int J = 0; J < GR_NB; ++J)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = 16 * J + c16;
      if (has1 && J >= I1 && J < nb) {
        const int row = 16 * I1 + d_row_f64(l, r);
        if (row < n && col < n) Gp[(int64_t)col * n + row] = acc1[J][r];
      }
      if (has2 && J >= I2 && J < nb) {
        const int row = 16 * I2 + d_row_f64(l, r);
        if (row < n && col < n) Gp[(int64_t)col * n + row] = acc2[J][r];
      }
    }
}

// G[i, j] = G[j, i] = sum over chunks of the upper partial (i <= j). One
// block per column j; its 4 waves sum 4 contiguous chunk ranges (lanes over
// rows i), combined in LDS in fixed order (deterministic).
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ Gpart, int chunks, int n,
                                                          double* __restrict__ G, int64_t ldg,
                                                          const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  __shared__ double part[4][64];
  const int j = blockIdx.x;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int per = (chunks + 3) / 4;
  const int c0 = w * per, c1 = min(chunks, c0 + per);
  for (int i0 = 0; i0 <= j; i0 += 64) {
    const int i = i0 + l;
    double acc = 0.0;
    if (i <= j) {
      const double* p = Gpart + (int64_t)j * n + i;
      const int64_t str = (int64_t)n * n;
      int c = c0;
      for (; c + 8 <= c1; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(c + u) * str];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
      }
      for (; c < c1; ++c) acc += p[(int64_t)c * str];
    }
    part[w][l] = acc;
    __syncthreads();
    if (w == 0 && i <= j) {
      const double tot = ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
      G[i + (int64_t)j * ldg] = tot;
      G[j + (int64_t)i * ldg] = tot;
    }
    __syncthreads();
  }
}

struct GramGeom { int chunks, rows_per_chunk; };

GramGeom gram_geometry(int64_t m) {
  const int64_t npan = (m + GR_PANEL - 1) / GR_PANEL;
  const int64_t target = 512;
  const int64_t per = (npan + target - 1) / target;
  GramGeom gg;
  gg.rows_per_chunk = (int)(per * GR_PANEL);
  gg.chunks = (int)((m + gg.rows_per_chunk - 1) / gg.rows_per_chunk);
  return gg;
}

size_t gram_partial_bytes(int64_t m, int64_t n) {
  GramGeom gg = gram_geometry(m);
  return (size_t)gg.chunks * (size_t)n * (size_t)n * sizeof(double);
}

hipError_t launch_gram(const double* B, int m, int n, int64_t ldb, double* Gpart, double* G, int64_t ldg,
                       const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > GR_NMAX) return hipErrorInvalidValue;
  GramGeom gg = gram_geometry(m);
  hipLaunchKernelGGL(syrk_kernel, dim3(gg.chunks), dim3(GR_THREADS), 0, st, B, m, n, ldb, gg.rows_per_chunk, Gpart, ctrl, phase);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(n), dim3(256), 0, st, (const double*)Gpart, gg.chunks, n, G, ldg, ctrl, phase);
  return hipGetLastError();
}

}  // namespace mrcqr
