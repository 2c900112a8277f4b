// Algorithm 1, first step, in float64: the Gram matrix G = B^T B of the
// preconditioned m x n matrix. Only the upper 16 x 16 tiles are formed
// (symmetric rank-k update). Grid = row chunks; a workgroup of 8 waves
// (2 per SIMD) stages 64-row panels of B in LDS (coalesced column loads)
// and each wave accumulates its share of the upper tiles with float64 MFMA
// 16x16x4. Per-chunk partials are summed in a second kernel in fixed order
// (deterministic, no atomics).
#include "batch.hpp"

namespace mrcqr {

constexpr int GR_THREADS = 512;
constexpr int GR_PANEL = 64;
constexpr int GR_SLAB = 256;  // rows per slab (the solve's rows per workgroup pass)
constexpr int GR_NMAX = 128;
constexpr int GR_NB = GR_NMAX / 16;
constexpr int GR_LDR = 65;  // column stride (doubles) of the LDS panel (odd: conflict-free operand reads)
constexpr int GR_TPW = 5;   // upper tiles per wave (at most)

// Upper tile u of wave w (8 waves, 8 x 8 tile grid, 36 tiles): waves 0-3
// take tiles (p, p..p+4) of block row p = w; waves 4-7 take the rest of
// block row p = w - 4, (p, p+5..7), and block row 7 - p, (7-p, 7-p..7).
// Waves w and w + 4 share a SIMD and hold 9 tiles together. Tiles beyond
// the block count nb are skipped.
__device__ __forceinline__ void gr_tile(int w, int u, int& I, int& J) {
  if (w < 4) { I = w; J = w + u; return; }
  const int p = w - 4, r1 = 3 - p;  // tiles left in block row p
  if (u < r1) { I = p; J = p + 5 + u; }
  else if (u - r1 <= p) { I = 7 - p; J = 7 - p + (u - r1); }
  else { I = GR_NB; J = GR_NB; }  // no tile
}

// The panel is column-major in LDS with a 65-double column stride:
// coalesced 64-row column stores and the operand reads (16 columns x 4 rows
// per wave) both hit distinct banks. Per K step (4 rows) a wave reads the A
// operand of each of its block rows once and one B operand per tile, and
// issues one float64 MFMA 16x16x4 per tile.
// Rows are taken in slabs of GR_SLAB: chunk c owns slabs c, c + chunks,
// c + 2 chunks, ... (the slabs the triangular solve's workgroup c writes, in
// the same 256-row units) and reads them last-written first, so that its
// first panels are still in the memory-side cache.
template <bool FULL>
__device__ __forceinline__ void syrk_body(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ double tile[2][GR_NMAX * GR_LDR];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nb = (n + 15) / 16;
  const int64_t nslab = ((int64_t)m + GR_SLAB - 1) / GR_SLAB;
  const int c = blockIdx.x;
  const int nsc = (int)((nslab - c + chunks - 1) / chunks);  // slabs of this chunk
  constexpr int PPS = GR_SLAB / GR_PANEL;                    // panels per slab
  const int npan = nsc * PPS;
  // first row of this chunk's panel i (slabs in reverse order)
  auto panel_row = [&](int i) -> int64_t {
    const int64_t slab = c + (int64_t)chunks * (nsc - 1 - i / PPS);
    return slab * GR_SLAB + (int64_t)GR_PANEL * (i % PPS);
  };
  const int64_t tend = m;

  int ti[GR_TPW], tj[GR_TPW];
  bool has[GR_TPW];
#pragma unroll
  for (int u = 0; u < GR_TPW; ++u) {
    gr_tile(w, u, ti[u], tj[u]);
    has[u] = ti[u] < nb && tj[u] < nb;
    if (!has[u]) { ti[u] = 0; tj[u] = 0; }
  }
  // FULL: all 8 x 8 block columns exist (n > 112). Otherwise the products of
  // tiles that do not exist are skipped (their accumulators are never
  // stored), and a wave without tiles skips the K loop.
  bool any = FULL;
#pragma unroll
  for (int u = 0; u < GR_TPW; ++u) any = any || has[u];
  f64x4 acc[GR_TPW];
#pragma unroll
  for (int u = 0; u < GR_TPW; ++u) acc[u] = f64x4{0, 0, 0, 0};

  constexpr int EPT = GR_PANEL * GR_NMAX / GR_THREADS;  // 16 columns per thread, one row
  constexpr int CST = GR_THREADS / 64;                  // column stride of a thread's columns
  double regs[EPT];
  auto load_panel = [&](int64_t t0) {
    const int64_t t = t0 + l;
    if (t0 + GR_PANEL <= tend && n == GR_NMAX) {
      const double* bp = B + t + (int64_t)w * ldb;
#pragma unroll
      for (int e = 0; e < EPT; ++e) regs[e] = bp[(int64_t)(CST * e) * ldb];
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int col = w + CST * e;
        regs[e] = (t < tend && col < n) ? B[t + (int64_t)col * ldb] : 0.0;
      }
    }
  };
  if (npan > 0) load_panel(panel_row(0));
  for (int p = 0; p < npan; ++p) {
    const int buf = p & 1;
#pragma unroll
    for (int e = 0; e < EPT; ++e) tile[buf][(w + CST * e) * GR_LDR + l] = regs[e];
    if (p + 1 < npan) load_panel(panel_row(p + 1));
    __syncthreads();
    const double* tb = tile[buf] + c16 * GR_LDR + g;
    // no branches in the K loop: a tile that does not exist (beyond nb)
    // reads block 0 and its accumulator is never stored
    if (!any) {
      // no tile of this wave exists
    } else if (w < 4) {
      // one block row: one A operand, B operands of blocks p..p+4
#pragma unroll 4
      for (int kk = 0; kk < GR_PANEL / 4; ++kk) {
        const double* tk = tb + 4 * kk;
        double bo[GR_TPW];
#pragma unroll
        for (int u = 0; u < GR_TPW; ++u) bo[u] = tk[16 * tj[u] * GR_LDR];
        const double a = tk[16 * ti[0] * GR_LDR];
#pragma unroll
        for (int u = 0; u < GR_TPW; ++u)
          if (FULL || has[u]) acc[u] = mfma_f64(a, bo[u], acc[u]);
      }
    } else {
#pragma unroll 4
      for (int kk = 0; kk < GR_PANEL / 4; ++kk) {
        const double* tk = tb + 4 * kk;
        double ao[GR_TPW - 1], bo[GR_TPW - 1];
#pragma unroll
        for (int u = 0; u < GR_TPW - 1; ++u) {
          ao[u] = tk[16 * ti[u] * GR_LDR];
          bo[u] = tk[16 * tj[u] * GR_LDR];
        }
#pragma unroll
        for (int u = 0; u < GR_TPW - 1; ++u)
          if (FULL || has[u]) acc[u] = mfma_f64(ao[u], bo[u], acc[u]);
      }
    }
  }
  // Gpart[chunk][col][row] for the upper tiles (f64 D layout)
  double* Gp = Gpart + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int u = 0; u < GR_TPW; ++u) {
    if (!has[u]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = 16 * tj[u] + c16, row = 16 * ti[u] + d_row_f64(l, r);
      if (row < n && col < n) Gp[(int64_t)col * n + row] = acc[u][r];
    }
  }
}

// n <= 16 NB with NB = 1, 2, 4: the panel holds only the 16 NB columns
// that can exist, and the NB (NB + 1) / 2 upper tiles go to the waves in
// order (wave w takes tiles w and w + 8). Every tile sees the same panels in
// the same order, as the same MFMA sequence, as in syrk_body, so the
// partial sums are bitwise the same; registers and LDS shrink with NB.
template <int NB>
__device__ __forceinline__ void syrk_small_body(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  constexpr int NC = 16 * NB;              // columns staged
  constexpr int NTILE = NB * (NB + 1) / 2;  // upper tiles
  constexpr int TPW = (NTILE + 7) / 8;      // tiles per wave
  __shared__ double tile[2][NC * GR_LDR];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nb = (n + 15) / 16;
  const int64_t nslab = ((int64_t)m + GR_SLAB - 1) / GR_SLAB;
  const int c = blockIdx.x;
  const int nsc = (int)((nslab - c + chunks - 1) / chunks);
  constexpr int PPS = GR_SLAB / GR_PANEL;
  const int npan = nsc * PPS;
  auto panel_row = [&](int i) -> int64_t {
    const int64_t slab = c + (int64_t)chunks * (nsc - 1 - i / PPS);
    return slab * GR_SLAB + (int64_t)GR_PANEL * (i % PPS);
  };
  const int64_t tend = m;

  int ti[TPW], tj[TPW];
  bool has[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    int t = w + 8 * u, I = 0;
    has[u] = t < NTILE;
    if (has[u]) {
      while (t >= NB - I) { t -= NB - I; ++I; }
    }
    ti[u] = has[u] ? I : 0;
    tj[u] = has[u] ? I + t : 0;
    if (!(ti[u] < nb && tj[u] < nb)) { has[u] = false; ti[u] = 0; tj[u] = 0; }
  }
  f64x4 acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = f64x4{0, 0, 0, 0};

  constexpr int CST = GR_THREADS / 64;           // column stride of a thread's columns
  constexpr int EPT = NC / CST > 0 ? NC / CST : 1;  // columns per thread, one row
  double regs[EPT];
  auto load_panel = [&](int64_t t0) {
    const int64_t t = t0 + l;
    if (t0 + GR_PANEL <= tend && n == NC && NC >= CST) {
      const double* bp = B + t + (int64_t)w * ldb;
#pragma unroll
      for (int e = 0; e < EPT; ++e) regs[e] = bp[(int64_t)(CST * e) * ldb];
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int col = w + CST * e;
        regs[e] = (t < tend && col < n) ? B[t + (int64_t)col * ldb] : 0.0;
      }
    }
  };
  if (npan > 0) load_panel(panel_row(0));
  for (int p = 0; p < npan; ++p) {
    const int buf = p & 1;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int col = w + CST * e;
      if (col < NC) tile[buf][col * GR_LDR + l] = regs[e];
    }
    if (p + 1 < npan) load_panel(panel_row(p + 1));
    __syncthreads();
    const double* tb = tile[buf] + c16 * GR_LDR + g;
    if (has[0]) {
#pragma unroll 4
      for (int kk = 0; kk < GR_PANEL / 4; ++kk) {
        const double* tk = tb + 4 * kk;
#pragma unroll
        for (int u = 0; u < TPW; ++u) {
          if (!has[u]) continue;
          const double a = tk[16 * ti[u] * GR_LDR], b = tk[16 * tj[u] * GR_LDR];
          acc[u] = mfma_f64(a, b, acc[u]);
        }
      }
    }
  }
  double* Gp = Gpart + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    if (!has[u]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = 16 * tj[u] + c16, row = 16 * ti[u] + d_row_f64(l, r);
      if (row < n && col < n) Gp[(int64_t)col * n + row] = acc[u][r];
    }
  }
}

template <int NB>
__global__ __launch_bounds__(GR_THREADS) void syrk_small_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  syrk_small_body<NB>(B, m, n, ldb, chunks, Gpart, ctrl, phase);
}

__global__ __launch_bounds__(GR_THREADS) void syrk_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  syrk_body<true>(B, m, n, ldb, chunks, Gpart, ctrl, phase);
}

__global__ __launch_bounds__(GR_THREADS) void syrk_part_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  syrk_body<false>(B, m, n, ldb, chunks, Gpart, ctrl, phase);
}

// Grouped: blockIdx.x is the member's chunk; members are grouped by the
// variant a single call of their shape uses.
template <bool FULL>
__global__ __launch_bounds__(GR_THREADS) void syrk_grouped(const BatchInst* __restrict__ bi,
                                                           const int32_t* __restrict__ members, BatchCall call,
                                                           int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.gram_chunks) return;
  syrk_body<FULL>(bat_ptr<const double>(call, d, d.off_B), d.m, d.n, d.m, d.gram_chunks,
                  bat_ptr<double>(call, d, d.off_Gpart), bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase);
}

template <int NB>
__global__ __launch_bounds__(GR_THREADS) void syrk_small_grouped(const BatchInst* __restrict__ bi,
                                                                 const int32_t* __restrict__ members, BatchCall call,
                                                                 int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.gram_chunks) return;
  syrk_small_body<NB>(bat_ptr<const double>(call, d, d.off_B), d.m, d.n, d.m, d.gram_chunks,
                      bat_ptr<double>(call, d, d.off_Gpart), bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase);
}

// G[i, j] = G[j, i] = sum over chunks of the upper partial (i <= j). One
// block per column j; its 4 waves sum 4 contiguous chunk ranges (lanes over
// rows i), combined in LDS in fixed order (deterministic).
__device__ __forceinline__ void gram_reduce_body(const double* __restrict__ Gpart, int chunks, int n,
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

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ Gpart, int chunks, int n,
                                                          double* __restrict__ G, int64_t ldg,
                                                          const Ctrl* __restrict__ ctrl, int phase) {
  gram_reduce_body(Gpart, chunks, n, G, ldg, ctrl, phase);
}

__global__ __launch_bounds__(256) void gram_reduce_grouped(const BatchInst* __restrict__ bi,
                                                           const int32_t* __restrict__ members, BatchCall call,
                                                           int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.n) return;
  gram_reduce_body(bat_ptr<const double>(call, d, d.off_Gpart), d.gram_chunks, d.n, bat_ptr<double>(call, d, d.off_G),
                   d.n, bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase);
}

// Kernel variant of the Gram of an n-column B: 0, 1, 2 = the small-n
// kernel for n <= 16, 32, 64; 3 = skipped tiles past n; 4 = every tile.
int syrk_variant(int n) {
  if (n <= 16) return 0;
  if (n <= 32) return 1;
  if (n <= 64) return 2;
  return n > GR_NMAX - 16 ? 4 : 3;
}

// one workgroup per compute unit, at most one per slab
static int gram_chunks(int64_t m) {
  const int64_t nslab = (m + GR_SLAB - 1) / GR_SLAB;
  return (int)(nslab < 256 ? nslab : 256);
}

int gram_batch_chunks(int64_t m) { return gram_chunks(m); }

hipError_t launch_gram_grouped(int variant, const BatchInst* bi, const int32_t* members, int count, int max_chunks,
                               int max_n, const BatchCall& call, int phase, hipStream_t st) {
  const dim3 grid(max_chunks, count), block(GR_THREADS);
  switch (variant) {
    case 0: hipLaunchKernelGGL(syrk_small_grouped<1>, grid, block, 0, st, bi, members, call, phase); break;
    case 1: hipLaunchKernelGGL(syrk_small_grouped<2>, grid, block, 0, st, bi, members, call, phase); break;
    case 2: hipLaunchKernelGGL(syrk_small_grouped<4>, grid, block, 0, st, bi, members, call, phase); break;
    case 3: hipLaunchKernelGGL(syrk_grouped<false>, grid, block, 0, st, bi, members, call, phase); break;
    default: hipLaunchKernelGGL(syrk_grouped<true>, grid, block, 0, st, bi, members, call, phase); break;
  }
  hipLaunchKernelGGL(gram_reduce_grouped, dim3(max_n, count), dim3(256), 0, st, bi, members, call, phase);
  return hipGetLastError();
}

size_t gram_partial_bytes(int64_t m, int64_t n) {
  return (size_t)gram_chunks(m) * (size_t)n * (size_t)n * sizeof(double);
}

hipError_t launch_gram(const double* B, int m, int n, int64_t ldb, double* Gpart, double* G, int64_t ldg,
                       const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > GR_NMAX) return hipErrorInvalidValue;
  const int chunks = gram_chunks(m);
  const dim3 grid(chunks), block(GR_THREADS);
  switch (syrk_variant(n)) {
    case 0: hipLaunchKernelGGL(syrk_small_kernel<1>, grid, block, 0, st, B, m, n, ldb, chunks, Gpart, ctrl, phase); break;
    case 1: hipLaunchKernelGGL(syrk_small_kernel<2>, grid, block, 0, st, B, m, n, ldb, chunks, Gpart, ctrl, phase); break;
    case 2: hipLaunchKernelGGL(syrk_small_kernel<4>, grid, block, 0, st, B, m, n, ldb, chunks, Gpart, ctrl, phase); break;
    case 3: hipLaunchKernelGGL(syrk_part_kernel, grid, block, 0, st, B, m, n, ldb, chunks, Gpart, ctrl, phase); break;
    default: hipLaunchKernelGGL(syrk_kernel, grid, block, 0, st, B, m, n, ldb, chunks, Gpart, ctrl, phase); break;
  }
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(n), dim3(256), 0, st, (const double*)Gpart, chunks, n, G, ldg, ctrl, phase);
  return hipGetLastError();
}

}  // namespace mrcqr
