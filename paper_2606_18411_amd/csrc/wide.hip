// The path for 128 < n <= 512 on column panels of 128 (32 or 64 for the
// sketch QR): every n x n object of the path outgrows one workgroup's
// registers and LDS, so each step is taken panel by panel with the kernels
// of the n <= 128 path plus the ones here.
//   Sketch QR (Algorithm 2, SketchQR): blocked Householder QR in the
//     sketch's QR precision; a panel of 32 or 64 columns is factored by one
//     workgroup (LAPACK geqr2 order, reflectors left in place below the
//     diagonal), its reflectors are applied to the columns to its right
//     from LDS, and upper_copy_kernel and the finish kernel take R (rows
//     with a negative pivot flipped), the checks and the condition
//     estimate of Rs.
//   B = A Rs^{-1} (Stage 2): per 128-column panel P, the update
//     C = A_P - B_{<P} Rs_{<P,P} (gemm_resident_kernel for K = 128,
//     gemm_panel_kernel beyond) and the solve of the n <= 128 path with the
//     diagonal panel, in place.
//   G = B^T B (Algorithm 1 step 1): the diagonal 128 x 128 blocks by the
//     n <= 128 Gram kernels, the blocks above them by gram_pair_kernel.
//   G = Rc^T Rc (Algorithm 1 step 2): right-looking over 128-column panels:
//     the n <= 128 Cholesky of the diagonal block, the panel
//     X = G_{rest,P} Rc_PP^{-1} by the solve, Rc_{P,rest} = X^T, and the
//     trailing update G_{rest,rest} -= X X^T (the panel GEMM).
//   X = Rc^{-1}, R = Rc Rs, the posterior power steps (many workgroups, two
//     launches per step) and Q = B X (the panel GEMM per panel of Q), each
//     for n <= 512.
// Every kernel is gated by the control block like the n <= 128 ones.
#include "batch.hpp"
#include "ice.hpp"

namespace mrcqr {

constexpr int WD_NMAX = 512;
constexpr int WD_PANEL = 128;  // column panel of the solve, Gram, Cholesky and product

// ---------------------------------------------------------------------------
// C = beta C0 + alpha Bs W: rows x nc (nc <= 128) from Bs (rows x K) and W
// (K x nc; W(k, j) = W[k + j ldw], or W[j + k ldw] when TW). K is taken in
// chunks of 16; entries with k >= kvalid read as zero (Bs and W are never
// read there). C0 may be C (each entry is read before it is written by the
// same lane); beta == 0 reads no C0.
// Each wave owns 16 rows and all 8 column blocks of 16; 8 waves (two per
// SIMD) share a workgroup and two workgroups a compute unit, so that one
// workgroup's stores overlap the other's products. The transposed product
// C^T = W^T Bs^T runs as float64 MFMA 16x16x4 with W (staged in LDS in
// A-operand order, double-buffered, each chunk loaded into registers one
// chunk ahead) as A operand and the rows of Bs (loaded one chunk ahead, and
// the next pass's first chunk during the last one) as B operand.
constexpr int GP_THREADS = 512;
constexpr int GP_ROWS = (GP_THREADS / 64) * 16;
constexpr int GP_WST = 2048 / GP_THREADS;  // W entries a thread stages per chunk

template <bool TW>
__global__ __launch_bounds__(GP_THREADS, 4) void gemm_panel_kernel(
    const double* __restrict__ Bs, int64_t ldb, int K, int kvalid, const double* __restrict__ W, int64_t ldw,
    const double* C0, int64_t ldc0, double* C, int64_t ldc, int rows, int nc, double alpha, double beta,
    const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ __attribute__((aligned(16))) double Wl[2][2048];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nch = (K + 15) / 16;
  // W staging: entry e = tid + GP_THREADS q of a chunk sits at (k-step e / 512,
  // column block (e / 64) % 8, lane e % 64) of the A-operand order
  double wr[GP_WST];
  // a lane's W base (row g, column c16 of a 4 x 16 piece) plus wave-uniform
  // offsets: entry (k-step ks, column block b) of the chunk at k0
  const double* Wlane = W + (TW ? c16 + (int64_t)g * ldw : g + (int64_t)c16 * ldw);
  auto wload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < GP_WST; ++q) {
      const int e0 = 64 * w + GP_THREADS * q;  // first entry of this wave's q-th piece
      const int ks = e0 >> 9, b = (e0 >> 6) & 7;
      int64_t u = TW ? 16 * b + (int64_t)(k0 + 4 * ks) * ldw : (k0 + 4 * ks) + (int64_t)(16 * b) * ldw;
      asm volatile("" : "+s"(u));
      const bool in = 16 * b + c16 < nc && k0 + 4 * ks + g < kvalid;
      wr[q] = in ? Wlane[u] : 0.0;
    }
  };
  auto wstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < GP_WST; ++q) Wl[buf][tid + GP_THREADS * q] = wr[q];
  };
  const double* Bl = Bs + c16 + (int64_t)g * ldb;
  const double* C0l = C0 + c16 + (int64_t)g * ldc0;
  double* Cl = C + c16 + (int64_t)g * ldc;
  double bd[4];
  auto loadb = [&](int64_t r0, int k0) {
    const bool row_in = r0 + c16 < rows;
    int64_t u = r0 + (int64_t)k0 * ldb;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      asm volatile("" : "+s"(u));
      const bool in = row_in && k0 + 4 * ks + g < kvalid;
      bd[ks] = in ? __builtin_nontemporal_load(&Bl[u]) : 0.0;
      u += 4 * ldb;
    }
  };
  int64_t pan = blockIdx.x;
  if (pan * GP_ROWS >= rows) return;
  wload(0);
  loadb(pan * GP_ROWS + 16 * w, 0);
  for (; pan * GP_ROWS < rows; pan += gridDim.x) {
    const int64_t r0 = pan * GP_ROWS + 16 * w;
    const int64_t rn = r0 + (int64_t)gridDim.x * GP_ROWS;  // this wave's rows in the next pass
    const bool more = (pan + gridDim.x) * GP_ROWS < rows;
    f64x4 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    wstore(0);
    if (nch > 1) wload(16);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      double cur[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) cur[ks] = bd[ks];
      if (c + 1 < nch) loadb(r0, 16 * (c + 1));
      else if (more) loadb(rn, 0);
      const double* Wb = Wl[c & 1];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] = mfma_f64(Wb[(ks * 8 + b) * 64 + l], cur[ks], acc[b]);
      if (c + 1 < nch) {
        wstore((c + 1) & 1);
        if (c + 2 < nch) wload(16 * (c + 2));
        else if (more) wload(0);
      } else if (nch == 1 && more) {
        wload(0);
      }
      __syncthreads();
    }
    const bool row_in = r0 + c16 < rows;
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t uc = r0 + (int64_t)(16 * b + 4 * r) * ldc, u0 = r0 + (int64_t)(16 * b + 4 * r) * ldc0;
        asm volatile("" : "+s"(uc), "+s"(u0));
        const bool in = row_in && 16 * b + 4 * r + g < nc;
        if (in) {
          double v = alpha * acc[b][r];
          if (beta != 0.0) v = fma(beta, __builtin_nontemporal_load(&C0l[u0]), v);
          __builtin_nontemporal_store(v, &Cl[uc]);
        }
      }
  }
}

// The same product for K <= 128 with all of W (128 KB at K = 128) staged
// once in LDS for the whole kernel, in A-operand order: no restaging per
// pass and no barrier after the staging; 16 waves per workgroup, one
// workgroup per CU (each wave's stores overlap the other waves' products).
// Chunks, k-steps and column blocks are taken in the order of
// gemm_panel_kernel, so both give the same sums.
constexpr int GRS_THREADS = 1024;
constexpr int GRS_ROWS = (GRS_THREADS / 64) * 16;  // 256 rows per pass
constexpr int GRS_KMAX = 128;

template <bool TW>
__global__ __launch_bounds__(GRS_THREADS, 4) void gemm_resident_kernel(
    const double* __restrict__ Bs, int64_t ldb, int K, int kvalid, const double* __restrict__ W, int64_t ldw,
    const double* C0, int64_t ldc0, double* C, int64_t ldc, int rows, int nc, double alpha, double beta,
    const Ctrl* __restrict__ ctrl, int phase) {
  extern __shared__ __attribute__((aligned(16))) double Wl[];  // (K/4) k-steps x 8 blocks x 64
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nks = (K + 3) / 4;  // k-steps of 4
  const int nch4 = (nks + 3) / 4 * 4;  // k-steps staged (whole chunks, zero past kvalid)
  // stage W: entry (ks, b, lane) = W(4 ks + lane / 16, 16 b + lane % 16)
  for (int e = tid; e < nch4 * 512; e += GRS_THREADS) {
    const int ks = e >> 9, b = (e >> 6) & 7, ll = e & 63;
    const int k = 4 * ks + (ll >> 4), j = 16 * b + (ll & 15);
    double v = 0.0;
    if (j < nc && k < kvalid) v = TW ? W[j + (int64_t)k * ldw] : W[k + (int64_t)j * ldw];
    Wl[e] = v;
  }
  __syncthreads();
  const double* Bl = Bs + c16 + (int64_t)g * ldb;
  const double* C0l = C0 + c16 + (int64_t)g * ldc0;
  double* Cl = C + c16 + (int64_t)g * ldc;
  const int nch = (nks + 3) / 4;  // chunks of 4 k-steps (16 k)
  for (int64_t pan = blockIdx.x; pan * GRS_ROWS < rows; pan += gridDim.x) {
    const int64_t r0 = pan * GRS_ROWS + 16 * w;
    const bool row_in = r0 + c16 < rows;
    f64x4 acc[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    double bd[4];
    auto loadb = [&](int c) {
      int64_t u = r0 + (int64_t)(16 * c) * ldb;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        asm volatile("" : "+s"(u));
        const bool in = row_in && 16 * c + 4 * ks + g < kvalid;
        bd[ks] = in ? __builtin_nontemporal_load(&Bl[u]) : 0.0;
        u += 4 * ldb;
      }
    };
    loadb(0);
    for (int c = 0; c < nch; ++c) {
      double cur[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) cur[ks] = bd[ks];
      if (c + 1 < nch) loadb(c + 1);
      const double* Wc = Wl + (size_t)(16 * c) * 128;  // 4 k-steps x 512 entries
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] = mfma_f64(Wc[(ks * 8 + b) * 64 + l], cur[ks], acc[b]);
    }
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t uc = r0 + (int64_t)(16 * b + 4 * r) * ldc, u0 = r0 + (int64_t)(16 * b + 4 * r) * ldc0;
        asm volatile("" : "+s"(uc), "+s"(u0));
        const bool in = row_in && 16 * b + 4 * r + g < nc;
        if (in) {
          double v = alpha * acc[b][r];
          if (beta != 0.0) v = fma(beta, __builtin_nontemporal_load(&C0l[u0]), v);
          __builtin_nontemporal_store(v, &Cl[uc]);
        }
      }
  }
}

hipError_t launch_gemm_panel(bool tw, const double* Bs, int64_t ldb, int K, int kvalid, const double* W, int64_t ldw,
                             const double* C0, int64_t ldc0, double* C, int64_t ldc, int rows, int nc, double alpha,
                             double beta, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (nc < 1 || nc > 128 || rows < 1 || K < 1) return hipErrorInvalidValue;
  if (K <= GRS_KMAX) {
    const int nch = ((K + 3) / 4 + 3) / 4;
    const size_t lds = (size_t)nch * 4 * 512 * sizeof(double);
    const int64_t passes = ((int64_t)rows + GRS_ROWS - 1) / GRS_ROWS;
    const dim3 grid((unsigned)(passes < 256 ? passes : 256)), block(GRS_THREADS);
    if (tw) {
      allow_dynamic_lds((const void*)gemm_resident_kernel<true>, lds);
      hipLaunchKernelGGL(gemm_resident_kernel<true>, grid, block, lds, st, Bs, ldb, K, kvalid, W, ldw, C0, ldc0, C,
                         ldc, rows, nc, alpha, beta, ctrl, phase);
    } else {
      allow_dynamic_lds((const void*)gemm_resident_kernel<false>, lds);
      hipLaunchKernelGGL(gemm_resident_kernel<false>, grid, block, lds, st, Bs, ldb, K, kvalid, W, ldw, C0, ldc0, C,
                         ldc, rows, nc, alpha, beta, ctrl, phase);
    }
    return hipGetLastError();
  }
  const int64_t panels = ((int64_t)rows + GP_ROWS - 1) / GP_ROWS;
  const int64_t cap = 512;
  const dim3 grid((unsigned)(panels < cap ? panels : cap)), block(GP_THREADS);
  if (tw)
    hipLaunchKernelGGL(gemm_panel_kernel<true>, grid, block, 0, st, Bs, ldb, K, kvalid, W, ldw, C0, ldc0, C, ldc, rows,
                       nc, alpha, beta, ctrl, phase);
  else
    hipLaunchKernelGGL(gemm_panel_kernel<false>, grid, block, 0, st, Bs, ldb, K, kvalid, W, ldw, C0, ldc0, C, ldc,
                       rows, nc, alpha, beta, ctrl, phase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram blocks above the diagonal: partial sums over row chunks of
// G_IJ = B_I^T B_J (128 x 128, I < J, column panels of B), one workgroup per
// (chunk, pair). 32-row steps of B_I and B_J are staged in LDS
// (column-major, odd 33-double stride: conflict-free stores and operand
// reads), double-buffered, each step loaded into registers one step ahead;
// each of the 8 waves owns 2 x 4 of the 64 tiles (A operand B_I^T from two
// column tiles, B operand B_J from four).
constexpr int GPR_THREADS = 512;
constexpr int GPR_ROWS = 32;                   // rows per step
constexpr int GPR_LD = GPR_ROWS + 1;
constexpr int GPR_EPT = 2 * GPR_ROWS * WD_PANEL / GPR_THREADS;  // staged entries per thread (both panels)

// Pair pr of the blocks above the diagonal, row by row: (0,1), (0,2), ...,
// (1,2), ...
__device__ __forceinline__ void pair_of(int pr, int n, int& I, int& J) {
  const int np = (n + WD_PANEL - 1) / WD_PANEL;
  I = 0;
  while (pr >= np - 1 - I) { pr -= np - 1 - I; ++I; }
  J = I + 1 + pr;
}

// Grid: 8 npr ceil(chunks / 8) workgroups. Workgroups are dispatched to the
// 8 XCDs round-robin; the npr pairs of one row chunk get ids 8 apart, so
// they run on one XCD and share its L2 for the chunk's rows.
__global__ __launch_bounds__(GPR_THREADS, 2) void gram_pair_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks, int rows_per_chunk, int npr,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ double Bt[2][2 * WD_PANEL * GPR_LD];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int bid = blockIdx.x, xcd = bid & 7, rest = bid >> 3;
  const int pr = rest % npr, chunk = (rest / npr) * 8 + xcd;
  if (chunk >= chunks) return;
  int I, J;
  pair_of(pr, n, I, J);
  const int ci0 = WD_PANEL * I, cj0 = WD_PANEL * J;
  const int nci = min(WD_PANEL, n - ci0), ncj = min(WD_PANEL, n - cj0);
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int ta0 = 2 * (w % 4), tb0 = 4 * (w / 4);
  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t rbeg = (int64_t)chunk * rows_per_chunk;
  const int64_t rend = min((int64_t)m, rbeg + rows_per_chunk);
  // staged entry q of this thread: row l % ROWS, column (panel-local)
  // c = (64 q + tid) / ROWS over the 256 columns of both panels
  constexpr int CPI = 64 / GPR_ROWS;  // columns per wave instruction
  const int lr = l % GPR_ROWS, lc = l / GPR_ROWS;
  double regs[GPR_EPT];
  // a lane's base (row lr, column lc) plus wave-uniform offsets; entry q
  // of a wave covers columns CW q + CPI w + (0..CPI-1) of the 256 (panel I
  // then panel J), so its panel is uniform
  constexpr int CW = GPR_THREADS / GPR_ROWS;
  const double* Bl = B + lr + (int64_t)lc * ldb;
  auto load = [&](int64_t p0) {
    const bool rin = p0 + lr < rend;
#pragma unroll
    for (int q = 0; q < GPR_EPT; ++q) {
      const int c0 = CW * q + CPI * w;          // uniform
      const bool second = c0 >= WD_PANEL;       // uniform
      const int cl0 = second ? c0 - WD_PANEL : c0;
      int64_t u = p0 + (int64_t)((second ? cj0 : ci0) + cl0) * ldb;
      asm volatile("" : "+s"(u));
      const bool ok = rin && cl0 + lc < (second ? ncj : nci);
      regs[q] = ok ? __builtin_nontemporal_load(&Bl[u]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < GPR_EPT; ++q) {
      const int c = (GPR_THREADS / GPR_ROWS) * q + CPI * w + lc;
      Bt[buf][c * GPR_LD + lr] = regs[q];
    }
  };
  const int nsteps = (int)((rend - rbeg + GPR_ROWS - 1) / GPR_ROWS);
  if (nsteps > 0) load(rbeg);
  for (int s = 0; s < nsteps; ++s) {
    const int buf = s & 1;
    store(buf);
    if (s + 1 < nsteps) load(rbeg + (int64_t)(s + 1) * GPR_ROWS);
    __syncthreads();
    const double* bi = Bt[buf] + c16 * GPR_LD + g;
    const double* bj = Bt[buf] + (WD_PANEL + c16) * GPR_LD + g;
#pragma unroll
    for (int ks = 0; ks < GPR_ROWS / 4; ++ks) {
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = bi[16 * (ta0 + a) * GPR_LD + 4 * ks];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = bj[16 * (tb0 + b) * GPR_LD + 4 * ks];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma_f64(av[a], bv[b], acc[a][b]);
    }
  }
  double* out = Gpart + ((int64_t)pr * chunks + chunk) * (WD_PANEL * WD_PANEL);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * (ta0 + a) + 4 * r + g, j = 16 * (tb0 + b) + c16;
        out[i + (int64_t)j * WD_PANEL] = acc[a][b][r];
      }
}

// Sum of the chunk partials of every pair in fixed order; writes G_IJ and
// its mirror G_JI. A workgroup of 4 waves takes 64 entries of one pair;
// wave w sums its quarter of the chunks (8 loads in flight), and the four
// quarter sums are added in order.
__global__ __launch_bounds__(256) void gram_pair_reduce_kernel(const double* __restrict__ Gpart, int chunks, int n,
                                                               double* __restrict__ G, int64_t ldg,
                                                               const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  __shared__ double part[4][64];
  const int pr = blockIdx.y;
  int I, J;
  pair_of(pr, n, I, J);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int e = blockIdx.x * 64 + l;
  const int per = (chunks + 3) / 4;
  const int c0 = w * per, c1 = min(chunks, c0 + per);
  double acc = 0.0;
  if (e < WD_PANEL * WD_PANEL) {
    const double* p = Gpart + (int64_t)pr * chunks * (WD_PANEL * WD_PANEL) + e;
    constexpr int64_t str = WD_PANEL * WD_PANEL;
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
  if (w != 0 || e >= WD_PANEL * WD_PANEL) return;
  const int i = e % WD_PANEL, j = e / WD_PANEL;
  const int gi = WD_PANEL * I + i, gj = WD_PANEL * J + j;
  if (gi >= n || gj >= n) return;
  const double sum = ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
  G[gi + (int64_t)gj * ldg] = sum;
  G[gj + (int64_t)gi * ldg] = sum;
}

// Row chunks per pair: about 768 workgroups over all pairs (three per
// compute unit), at most 512 chunks.
static int gpr_max_chunks(int npr) {
  const int c = (768 / (npr > 0 ? npr : 1) + 7) / 8 * 8;
  return c > 512 ? 512 : c;
}

int wide_panels(int n) { return (n + WD_PANEL - 1) / WD_PANEL; }
int wide_pairs(int n) { const int np = wide_panels(n); return np * (np - 1) / 2; }

size_t gram_pair_partial_bytes(int n) {
  return (size_t)wide_pairs(n) * gpr_max_chunks(wide_pairs(n)) * WD_PANEL * WD_PANEL * sizeof(double) + 256;
}

hipError_t launch_gram(const double* B, int m, int n, int64_t ldb, double* Gpart, double* G, int64_t ldg,
                       const Ctrl* ctrl, int phase, hipStream_t st);

// Gram for n <= 512: diagonal blocks by launch_gram (Gpart_diag: the n <=
// 128 partials), the others by the pair kernel (Gpart_pairs).
hipError_t launch_gram_wide(const double* B, int m, int n, int64_t ldb, double* Gpart_diag, double* Gpart_pairs,
                            double* G, int64_t ldg, const Ctrl* ctrl, int phase, hipStream_t st) {
  const int np = wide_panels(n);
  for (int P = 0; P < np; ++P) {
    const int c0 = WD_PANEL * P, nc = min(WD_PANEL, n - c0);
    const hipError_t e = launch_gram(B + (int64_t)c0 * ldb, m, nc, ldb, Gpart_diag, G + c0 + (int64_t)c0 * ldg, ldg,
                                     ctrl, phase, st);
    if (e != hipSuccess) return e;
  }
  const int npr = wide_pairs(n);
  if (npr > 0) {
    const int maxc = gpr_max_chunks(npr);
    const int rpc = (int)((((int64_t)m + maxc - 1) / maxc + 63) / 64 * 64);
    const int chunks = (int)(((int64_t)m + rpc - 1) / rpc);
    const int chunks8 = (chunks + 7) / 8 * 8;
    hipLaunchKernelGGL(gram_pair_kernel, dim3(chunks8 * npr), dim3(GPR_THREADS), 0, st, B, m, n, ldb, chunks, rpc,
                       npr, Gpart_pairs, ctrl, phase);
    hipLaunchKernelGGL(gram_pair_reduce_kernel, dim3((WD_PANEL * WD_PANEL + 63) / 64, npr), dim3(256), 0, st,
                       (const double*)Gpart_pairs, chunks, n, G, ldg, ctrl, phase);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked Householder QR of the sketch Y (s x n, float64 storage of values
// of type T), in place: R in the upper triangle, the reflectors below it
// (LAPACK convention, v_j = 1 implicit), tau[j].
//
// Panel kernel: one workgroup of 16 waves factors Y[j0:s, j0:j0+nb] (nb <=
// 16 CPW): wave w holds columns w + 16 q (q < CPW), lane l rows j0 + l + 64 i
// (i < RPL), in registers, scaled by 2^es (es from the panel's largest
// magnitude, undone on R); the wave owning column j forms its reflector
// (larfg: beta = -sign(alpha) ||x||) and publishes v in LDS; every wave
// then updates its columns to the right (one dot product per column: a
// wave sum).
template <typename T, int RPL, int CPW>
__global__ __launch_bounds__(1024) void hh_panel_kernel(double* __restrict__ Y, int s, int n, int64_t ldy, int j0,
                                                        int nb, double* __restrict__ tau, int* __restrict__ flags,
                                                        const Ctrl* __restrict__ ctrl, int slot, int phase) {
  __shared__ T vsh[2][64 * RPL];
  __shared__ T tsh[2];
  __shared__ double wmax[16];
  __shared__ int wnf[16];
  if (skip_launch(ctrl, slot, phase)) return;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int sp = s - j0;  // rows of the panel
  T y[CPW][RPL];
  double lm = 0.0;
  bool nf = false;
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 16 * q;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = l + 64 * i;
      const double v = (c < nb && r < sp) ? Y[(j0 + r) + (int64_t)(j0 + c) * ldy] : 0.0;
      lm = fmax(lm, fabs(v));
      nf = nf || !isfinite(v);
      y[q][i] = (T)v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) lm = fmax(lm, __shfl_xor(lm, o));
  const bool wave_nf = __ballot(nf) != 0;
  if (l == 0) { wmax[w] = lm; wnf[w] = wave_nf; }
  __syncthreads();
  int es = 0;
  {
    double gm = 0.0;
    bool anf = false;
    for (int k = 0; k < 16; ++k) { gm = fmax(gm, wmax[k]); anf = anf || wnf[k]; }
    if (gm > 0.0 && isfinite(gm)) { int E; (void)frexp(gm, &E); es = -E; }
    if (anf && tid == 0) atomicOr(flags, 2);  // a non-finite sketch entry
  }
#pragma unroll
  for (int q = 0; q < CPW; ++q)
#pragma unroll
    for (int i = 0; i < RPL; ++i) y[q][i] = (T)ldexp((double)y[q][i], es);

  for (int j = 0; j < nb; ++j) {
    const int buf = j & 1;
    if (w == (j & 15)) {
      const int q = j >> 4;
      // reflector of column j (rows j.. of the panel)
      T alpha_l = (T)0, ss = (T)0;
#pragma unroll
      for (int qq = 0; qq < CPW; ++qq) {
        if (qq != q) continue;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = l + 64 * i;
          alpha_l = (r == j) ? y[qq][i] : alpha_l;
          ss += (r > j) ? y[qq][i] * y[qq][i] : (T)0;
        }
      }
      const T alpha = wave_sum_dpp(alpha_l);
      const T sig = wave_sum_dpp(ss);
      T tv, beta, scal;
      if (sig == (T)0) { tv = (T)0; beta = alpha; scal = (T)0; }
      else {
        const T nrm = sqrt(alpha * alpha + sig);
        beta = signbit(alpha) ? nrm : -nrm;
        tv = (beta - alpha) / beta;
        scal = (T)1 / (alpha - beta);
      }
#pragma unroll
      for (int qq = 0; qq < CPW; ++qq) {
        if (qq != q) continue;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = l + 64 * i;
          const T v = (r > j) ? y[qq][i] * scal : (r == j ? (T)1 : (T)0);
          vsh[buf][r] = v;
          y[qq][i] = (r == j) ? beta : ((r > j) ? v : y[qq][i]);  // v stays below the diagonal
        }
      }
      if (l == 0) {
        tsh[buf] = tv;
        tau[j0 + j] = (double)tv;
      }
    }
    __syncthreads();
    const T tv = tsh[buf];
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      const int c = w + 16 * q;
      if (c > j && c < nb) {
        T dp = (T)0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) dp += vsh[buf][l + 64 * i] * y[q][i];
        const T f = tv * wave_sum_dpp(dp);
#pragma unroll
        for (int i = 0; i < RPL; ++i) y[q][i] -= f * vsh[buf][l + 64 * i];
      }
    }
  }
  // back to Y: R (upper part, scaled back) and the reflectors below it
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    const int c = w + 16 * q;
    if (c >= nb) continue;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = l + 64 * i;
      if (r < sp) {
        const double v = (r <= c) ? ldexp((double)y[q][i], -es) : (double)y[q][i];
        Y[(j0 + r) + (int64_t)(j0 + c) * ldy] = v;
      }
    }
  }
}

// Apply the panel's reflectors (columns j0..j0+nb-1 of Y, below the
// diagonal, tau) to column c of Y (c >= j0 + nb), rows j0..s-1, in order;
// one wave per column, arithmetic in T. A workgroup of 16 waves (16
// columns) stages the reflectors in LDS, HH_KB of them at a time (128 KB),
// so that the serial chain of a column reads no global memory.
template <typename T, int RPL>
__global__ __launch_bounds__(1024) void hh_apply_kernel(double* __restrict__ Y, int s, int n, int64_t ldy, int j0,
                                                        int nb, const double* __restrict__ tau,
                                                        const Ctrl* __restrict__ ctrl, int slot, int phase) {
  constexpr int LEN = 64 * RPL;
  constexpr int HH_KB = (128 * 1024) / (LEN * (int)sizeof(T));
  __shared__ T vs[HH_KB][LEN];
  if (skip_launch(ctrl, slot, phase)) return;
  const int tid = threadIdx.x, l = tid & 63;
  const int c = j0 + nb + blockIdx.x * 16 + (tid >> 6);
  const bool have = c < n;
  const int sp = s - j0;
  T y[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = l + 64 * i;
    y[i] = (have && r < sp) ? (T)Y[(j0 + r) + (int64_t)c * ldy] : (T)0;
  }
  for (int k0 = 0; k0 < nb; k0 += HH_KB) {
    const int kb = min(HH_KB, nb - k0);
    __syncthreads();  // the previous stage's reflectors are applied
    for (int e = tid; e < kb * LEN; e += 1024) {
      const int kk = e / LEN, r = e % LEN, k = k0 + kk;
      const double* vk = Y + j0 + (int64_t)(j0 + k) * ldy;
      vs[kk][r] = (r > k && r < sp) ? (T)vk[r] : (r == k ? (T)1 : (T)0);
    }
    __syncthreads();
    if (have) {
      for (int kk = 0; kk < kb; ++kk) {
        T dp = (T)0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) dp += vs[kk][l + 64 * i] * y[i];
        const T f = (T)tau[j0 + k0 + kk] * wave_sum_dpp(dp);
#pragma unroll
        for (int i = 0; i < RPL; ++i) y[i] -= f * vs[kk][l + 64 * i];
      }
    }
  }
  if (!have) return;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = l + 64 * i;
    if (r < sp) Y[(j0 + r) + (int64_t)c * ldy] = (double)y[i];
  }
}

// Upper triangle of an n x n matrix into dst (below it zero; everything
// zero when one of the np pivots in fails[] is set) and into a row-major
// copy Rt (row r at Rt + r n) for the condition estimate, by 32 x 32 tiles
// transposed through LDS. flip: row r is multiplied by the sign of
// src(r, r) (R with a positive diagonal from a Householder factor), and a
// diagonal entry that is not positive and finite or an off-diagonal entry
// that is not finite sets bit 4 of *flags.
__global__ __launch_bounds__(256) void upper_copy_kernel(const double* src, int64_t lds, double* dst, int64_t ldd,
                                                         double* __restrict__ Rt, int n, int flip,
                                                         const int32_t* __restrict__ fails, int np,
                                                         int* __restrict__ flags, const Ctrl* __restrict__ ctrl,
                                                         int slot, int phase) {
  __shared__ double tile[32][33];
  if (skip_launch(ctrl, slot, phase)) return;
  bool zero_all = false;
  if (fails)
    for (int P = 0; P < np; ++P) zero_all = zero_all || fails[P] >= 0;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + tx, c = c0 + ty + 8 * k;
    double v = 0.0;
    if (r < n && c < n && r <= c && !zero_all) {
      v = src[r + (int64_t)c * lds];
      if (flip) {
        v = (src[r + (int64_t)r * lds] < 0.0 ? -1.0 : 1.0) * v;
        if (r == c && !(v > 0.0 && isfinite(v))) bad = true;
        if (r < c && !isfinite(v)) bad = true;
      }
    }
    if (r < n && c < n) dst[r + (int64_t)c * ldd] = v;
    tile[ty + 8 * k][tx] = v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + ty + 8 * k, c = c0 + tx;
    if (r < n && c < n) Rt[(int64_t)r * n + c] = tile[tx][ty + 8 * k];
  }
  if (flags && bad) atomicOr(flags, 4);
}

static void launch_upper_copy(const double* src, int64_t lds, double* dst, int64_t ldd, double* Rt, int n, bool flip,
                              const int32_t* fails, int np, int* flags, const Ctrl* ctrl, int slot, int phase,
                              hipStream_t st) {
  const dim3 grid((n + 31) / 32, (n + 31) / 32), block(256);
  hipLaunchKernelGGL(upper_copy_kernel, grid, block, 0, st, src, lds, dst, ldd, Rt, n, flip ? 1 : 0, fails, np, flags,
                     ctrl, slot, phase);
}

// Clear the flags word of the sketch QR (a small fill kernel, so the
// sequence records no memset).
__global__ void wide_flags_clear_kernel(int* flags, const Ctrl* __restrict__ ctrl, int slot, int phase) {
  if (skip_launch(ctrl, slot, phase)) return;
  if (threadIdx.x == 0) *flags = 0;
}

// The checks and the condition estimate of Rs with the AUTO escalation (the
// epilogue of the n <= 128 sketch QR), after upper_copy_kernel has written
// Rs (diag(Rs) > 0), its row-major copy Rt and the flags.
__global__ __launch_bounds__(256) void hh_finish_kernel(const double* __restrict__ Rt, int n,
                                                         const int* __restrict__ flags,
                                                         double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl,
                                                         int slot, int phase, int want_kappa) {
  if (skip_launch(ctrl, slot, phase)) return;
  const int fl = *flags;
  const bool nonfinite = (fl & 2) != 0;
  const bool bad = (fl & 4) != 0 || nonfinite;
  const bool auto_here = ctrl != nullptr && ctrl->auto_mode;
  double kappa = ice_kappa_rows(Rt, n, !bad && (auto_here || want_kappa));
  if (bad) kappa = __builtin_inf();
  if (threadIdx.x != 0) return;
  if (kappa_out) *kappa_out = kappa;
  if (!ctrl) return;
  ctrl->kappa_rs = kappa;
  const int p = ctrl->cur_prec;
  const bool can_escalate = ctrl->auto_mode && (p == P_FP16 || p == P_FP32);
  const double tau_p = (p == P_FP16) ? TAU_FP16 : (p == P_FP32 ? TAU_FP32 : __builtin_inf());
  if (bad) {
    if (can_escalate) { ctrl->cur_prec = (p == P_FP16) ? P_FP32 : P_FP64; ctrl->escalations += 1; }
    else ctrl->status = nonfinite ? ST_NONFINITE : ST_SINGULAR;
  } else if (can_escalate && kappa >= tau_p) {
    ctrl->cur_prec = (p == P_FP16) ? P_FP32 : P_FP64;
    ctrl->escalations += 1;
  }
}

// Panels of 16 CPW columns; CPW = 2 where 4 would not fit the 128
// registers of a 1024-thread workgroup (float64, or 16 rows per lane).
template <typename T, int RPL>
static hipError_t hh_panels(double* Y, int s, int n, int64_t ldy, double* tau, int* flags, const Ctrl* ctrl,
                            int slot, int phase, hipStream_t st) {
  constexpr int CPW = (sizeof(T) == 8 || RPL > 8) ? 2 : 4;
  for (int j0 = 0; j0 < n; j0 += 16 * CPW) {
    const int nb = min(16 * CPW, n - j0);
    hipLaunchKernelGGL((hh_panel_kernel<T, RPL, CPW>), dim3(1), dim3(1024), 0, st, Y, s, n, ldy, j0, nb, tau, flags,
                       ctrl, slot, phase);
    const int rest = n - j0 - nb;
    if (rest > 0)
      hipLaunchKernelGGL((hh_apply_kernel<T, RPL>), dim3((rest + 15) / 16), dim3(1024), 0, st, Y, s, n, ldy, j0,
                         nb, (const double*)tau, ctrl, slot, phase);
  }
  return hipGetLastError();
}

// The sketch QR for n > 128: Y (s x n, ld ldy) is overwritten.
hipError_t launch_sketch_qr_wide(bool f64, double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                                 double* tau, int* flags, double* Rt, double* kappa, Ctrl* ctrl, int slot, int phase,
                                 hipStream_t st) {
  if (n > WD_NMAX || s > 16 * 64 || s < n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wide_flags_clear_kernel, dim3(1), dim3(64), 0, st, flags, (const Ctrl*)ctrl, slot, phase);
  const int rpl = (s + 63) / 64;
  hipError_t e;
  if (f64) {
    if (rpl <= 8) e = hh_panels<double, 8>(Y, s, n, ldy, tau, flags, ctrl, slot, phase, st);
    else e = hh_panels<double, 16>(Y, s, n, ldy, tau, flags, ctrl, slot, phase, st);
  } else {
    if (rpl <= 8) e = hh_panels<float, 8>(Y, s, n, ldy, tau, flags, ctrl, slot, phase, st);
    else e = hh_panels<float, 16>(Y, s, n, ldy, tau, flags, ctrl, slot, phase, st);
  }
  if (e != hipSuccess) return e;
  launch_upper_copy(Y, ldy, Rs, ldr, Rt, n, true, nullptr, 0, flags, ctrl, slot, phase, st);
  hipLaunchKernelGGL(hh_finish_kernel, dim3(1), dim3(256), 0, st, (const double*)Rt, n, (const int*)flags, kappa,
                     ctrl, slot, phase, kappa != nullptr ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_trsm(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr, double* X,
                       int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st);

// X = A R^{-1} for n <= 512 by 128-column panels: X_P = (A_P - X_{<P}
// R_{<P,P}) R_PP^{-1}, the update by gemm_panel_kernel into X_P, the solve
// in place.
hipError_t launch_trsm_wide(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr, double* X,
                            int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st) {
  const int np = wide_panels(n);
  for (int P = 0; P < np; ++P) {
    const int c0 = WD_PANEL * P, nc = min(WD_PANEL, n - c0);
    const double* Ap = A + (int64_t)c0 * lda;
    double* Xp = X + (int64_t)c0 * ldx;
    hipError_t e;
    if (P > 0) {
      e = launch_gemm_panel(false, X, ldx, c0, c0, R + (int64_t)c0 * ldr, ldr, Ap, lda, Xp, ldx, m, nc, -1.0, 1.0,
                            ctrl, phase, st);
      if (e != hipSuccess) return e;
      e = launch_trsm(Xp, m, nc, ldx, R + c0 + (int64_t)c0 * ldr, ldr, Xp, ldx, ws, ctrl, phase, st);
    } else {
      e = launch_trsm(Ap, m, nc, lda, R, ldr, Xp, ldx, ws, ctrl, phase, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Q = B X (X upper triangular, n <= 512): Q_P = B_{<=P} X_{<=P,P}.
hipError_t launch_qform_wide(const double* B, int m, int n, int64_t ldb, const double* X, int64_t ldx, double* Q,
                             int64_t ldq, const Ctrl* ctrl, int phase, hipStream_t st) {
  const int np = wide_panels(n);
  for (int P = 0; P < np; ++P) {
    const int c0 = WD_PANEL * P, nc = min(WD_PANEL, n - c0);
    const int K = c0 + nc;
    const hipError_t e = launch_gemm_panel(false, B, ldb, K, K, X + (int64_t)c0 * ldx, ldx, nullptr, 0,
                                           Q + (int64_t)c0 * ldq, ldq, m, nc, 1.0, 0.0, ctrl, phase, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_cholesky(const double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                           double* kappa, Ctrl* ctrl, int phase, hipStream_t st);

// Rc_{P,rest} = T^T (T: rest x nc, ld ldt).
__global__ void wide_transpose_kernel(const double* __restrict__ T, int64_t ldt, int rest, int nc,
                                      double* __restrict__ Rc, int64_t ldr, const Ctrl* __restrict__ ctrl,
                                      int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rest * nc) return;
  const int k = e % nc, j = e / nc;
  Rc[k + (int64_t)j * ldr] = T[j + (int64_t)k * ldt];
}

// The factorization's outcome: the first failing pivot over the panels (in
// the whole matrix's numbering) and the ICE of Rc (from its row-major copy
// Rt; upper_copy_kernel has cleared the lower triangle), into the control
// block as the n <= 128 Cholesky kernel leaves them.
__global__ __launch_bounds__(256) void chol_wide_finish_kernel(const int32_t* __restrict__ fails, int np, int n,
                                                               const double* __restrict__ Rt,
                                                               int32_t* __restrict__ fail_out,
                                                               double* __restrict__ kappa_out,
                                                               Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  int f = -1;
  for (int P = 0; P < np; ++P)
    if (fails[P] >= 0) { f = WD_PANEL * P + fails[P]; break; }
  double kappa = ice_kappa_rows(Rt, n, f < 0);
  if (f >= 0) kappa = __builtin_inf();
  if (threadIdx.x != 0) return;
  if (fail_out) *fail_out = f;
  if (kappa_out) *kappa_out = kappa;
  if (ctrl) {
    ctrl->kappa_rc = kappa;
    ctrl->pass_fail = f;
  }
}

// G = Rc^T Rc for n <= 512, right-looking over 128-column panels. G is
// overwritten (trailing updates); T (n x 128, ld n), fails (np ints) and Rt
// (n x n) are scratch; Tw the solve's staging workspace.
hipError_t launch_cholesky_wide(double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                                double* kappa, double* T, int32_t* fails, double* Rt, void* Tw, Ctrl* ctrl, int phase,
                                hipStream_t st) {
  const int np = wide_panels(n);
  for (int P = 0; P < np; ++P) {
    const int c0 = WD_PANEL * P, nc = min(WD_PANEL, n - c0);
    hipError_t e = launch_cholesky(G + c0 + (int64_t)c0 * ldg, nc, ldg, Rc + c0 + (int64_t)c0 * ldr, ldr, fails + P,
                                   nullptr, ctrl, phase, st);
    if (e != hipSuccess) return e;
    const int o = c0 + nc, rest = n - o;
    if (rest <= 0) continue;
    // T = G_{rest,P} Rc_PP^{-1} = Rc_{P,rest}^T
    e = launch_trsm(G + o + (int64_t)c0 * ldg, rest, nc, ldg, Rc + c0 + (int64_t)c0 * ldr, ldr, T, n, Tw, ctrl,
                    phase, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(wide_transpose_kernel, dim3((rest * nc + 255) / 256), dim3(256), 0, st, (const double*)T,
                       (int64_t)n, rest, nc, Rc + c0 + (int64_t)o * ldr, ldr, (const Ctrl*)ctrl, phase);
    // G_{rest,rest} -= T T^T
    for (int cb = 0; cb < rest; cb += WD_PANEL) {
      const int ncb = min(WD_PANEL, rest - cb);
      double* Cb = G + o + (int64_t)(o + cb) * ldg;
      e = launch_gemm_panel(true, T, n, nc, nc, T + cb, n, Cb, ldg, Cb, ldg, rest, ncb, -1.0, 1.0, ctrl, phase, st);
      if (e != hipSuccess) return e;
    }
  }
  launch_upper_copy(Rc, ldr, Rc, ldr, Rt, n, false, fails, np, nullptr, ctrl, P_AUTO, phase, st);
  hipLaunchKernelGGL(chol_wide_finish_kernel, dim3(1), dim3(256), 0, st, (const int32_t*)fails, np, n,
                     (const double*)Rt, fail, kappa, ctrl, phase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// X = R^{-1} (R upper triangular, n <= 512): one wave per column j, lane l
// holding rows l + 64 q; x_i is formed on the lane holding row i and read
// by the others (back substitution in column order). The columns of R are
// read TI_DEPTH steps ahead of the serial chain.
__global__ __launch_bounds__(64) void trinv_wide_kernel(const double* __restrict__ R, int n, int64_t ldr,
                                                        double* __restrict__ X, int64_t ldx,
                                                        const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  constexpr int Q = WD_NMAX / 64;
  constexpr int TI_DEPTH = 4;
  const int j = blockIdx.x, l = threadIdx.x;
  double sv[Q], rinv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = l + 64 * q;
    const int rc = min(r, n - 1);
    rinv[q] = 1.0 / R[rc + (int64_t)rc * ldr];
    sv[q] = (r == j) ? 1.0 : 0.0;
  }
  // ring[d]: entries r < i of column i of R
  double ring[TI_DEPTH][Q];
  auto load = [&](int i, int slot) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = l + 64 * q;
      ring[slot][q] = (i >= 0 && r < i) ? R[r + (int64_t)i * ldr] : 0.0;
    }
  };
#pragma unroll
  for (int d = 0; d < TI_DEPTH; ++d) load(j - d, d);
  for (int i0 = j; i0 >= 0; i0 -= TI_DEPTH) {
#pragma unroll
    for (int d = 0; d < TI_DEPTH; ++d) {
      const int i = i0 - d;
      if (i >= 0) {
        double col[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) col[q] = ring[d][q];
        load(i - TI_DEPTH, d);
        const int qi = i >> 6;
        double own = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (q == qi) own = sv[q] * rinv[q];
        const double x = readlane_t(own, i & 63);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int r = l + 64 * q;
          if (r == i) sv[q] = x;
          else if (r < i) sv[q] = fma(-col[q], x, sv[q]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = l + 64 * q;
    if (r < n) X[r + (int64_t)j * ldx] = (r <= j) ? sv[q] : 0.0;
  }
}

// R = R2 R1 (both upper triangular, n <= 512): one thread per entry.
__global__ void trmm_wide_kernel(const double* __restrict__ R2, int64_t ld2, const double* __restrict__ R1,
                                 int64_t ld1, int n, double* __restrict__ R, int64_t ldr,
                                 const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int i = e % n, j = e / n;
  double v = 0.0;
  for (int k = i; k <= j; ++k) v = fma(R2[i + (int64_t)k * ld2], R1[k + (int64_t)j * ld1], v);
  R[i + (int64_t)j * ldr] = v;
}

hipError_t launch_rc_tail_wide(const double* Rc, int n, int64_t ldc, const double* Rs, int64_t lds_, double* X,
                               int64_t ldx, double* R, int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st) {
  hipLaunchKernelGGL(trinv_wide_kernel, dim3(n), dim3(64), 0, st, Rc, n, ldc, X, ldx, ctrl, phase);
  if (R)
    hipLaunchKernelGGL(trmm_wide_kernel, dim3((n * n + 255) / 256), dim3(256), 0, st, Rc, ldc, Rs, lds_, n, R, ldr,
                       ctrl, phase);
  return hipGetLastError();
}

hipError_t launch_trinv_wide(const double* R, int n, int64_t ldr, double* X, int64_t ldx, const Ctrl* ctrl, int phase,
                             hipStream_t st) {
  hipLaunchKernelGGL(trinv_wide_kernel, dim3(n), dim3(64), 0, st, R, n, ldr, X, ldx, ctrl, phase);
  return hipGetLastError();
}

hipError_t launch_trmm_wide(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int n, double* R,
                            int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st) {
  hipLaunchKernelGGL(trmm_wide_kernel, dim3((n * n + 255) / 256), dim3(256), 0, st, R2, ld2, R1, ld1, n, R, ldr,
                     ctrl, phase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The posterior check for n <= 512 (the n <= 128 kernel's estimate and
// decision): sigma_max(Rc) and sigma_max(X) from POSTERIOR_STEPS power steps
// on M^T M from the normalized all-ones vector. Each step is two launches
// over 16-row (16-column) blocks of both matrices, so that the n x n
// matrices stream through many compute units: y = M x with x = z / ||z||
// (every workgroup forms ||z|| itself, in one fixed order), then z = M^T y.
// A last y = M x and a one-workgroup decision follow. Vectors live in ws:
// z[2][WD_NMAX], then y[2][WD_NMAX].
constexpr int PW_THREADS = 256;
constexpr size_t POSTERIOR_WS_DOUBLES = 4 * WD_NMAX;

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  v = wave_sum_dpp(v);
  const int t = threadIdx.x;
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// y = M x: workgroup (block, k), k = 0 for Rc and 1 for X; thread t takes
// row 16 block + t % 16 and the columns j = t / 16 (mod 16), j >= row.
__global__ __launch_bounds__(PW_THREADS) void power_mv_kernel(const double* __restrict__ Rc,
                                                              const double* __restrict__ X, int n, int64_t ld,
                                                              double* __restrict__ ws, int first,
                                                              const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ double xs[WD_NMAX];
  __shared__ double part[16][17];
  __shared__ double red[4];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int k = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
  const double* M = k ? X : Rc;
  const double* z = ws + k * WD_NMAX;
  double* y = ws + (2 + k) * WD_NMAX;
  if (first) {
    for (int i = t; i < n; i += PW_THREADS) xs[i] = 1.0 / sqrt((double)n);
  } else {
    double s = 0.0;
    for (int i = t; i < n; i += PW_THREADS) s = fma(z[i], z[i], s);
    const double nz = sqrt(block_sum_256(s, red));
    for (int i = t; i < n; i += PW_THREADS) xs[i] = z[i] / nz;
  }
  __syncthreads();
  const int r = t & 15, sl = t >> 4, i = 16 * blk + r;
  double acc = 0.0;
  if (i < n)
    for (int j = sl; j < n; j += 16)
      if (j >= i) acc = fma(M[i + (int64_t)j * ld], xs[j], acc);
  part[sl][r] = acc;
  __syncthreads();
  if (t < 16 && 16 * blk + t < n) {
    double v = 0.0;
    for (int q = 0; q < 16; ++q) v += part[q][t];
    y[16 * blk + t] = v;
  }
}

// z = M^T y: thread t takes column 16 block + t / 16 and the rows
// i = t % 16 (mod 16), i <= column; the 16 partial sums of a column are one
// group of 16 lanes.
__global__ __launch_bounds__(PW_THREADS) void power_tmv_kernel(const double* __restrict__ Rc,
                                                               const double* __restrict__ X, int n, int64_t ld,
                                                               double* __restrict__ ws,
                                                               const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int k = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
  const double* M = k ? X : Rc;
  double* z = ws + k * WD_NMAX;
  const double* y = ws + (2 + k) * WD_NMAX;
  const int sl = t & 15, j = 16 * blk + (t >> 4);
  double acc = 0.0;
  if (j < n)
    for (int i = sl; i <= j; i += 16) acc = fma(M[i + (int64_t)j * ld], y[i], acc);
  acc = group_sum_dpp(acc, 16);
  if (sl == 0 && j < n) z[j] = acc;
}

// ||M x|| after the last step, the estimate and the decision.
__global__ __launch_bounds__(PW_THREADS) void posterior_decide_kernel(const double* __restrict__ ws, int n,
                                                                      Ctrl* __restrict__ ctrl, int phase,
                                                                      double* __restrict__ kappa_out) {
  __shared__ double red[4];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int t = threadIdx.x;
  double est[2];
  for (int k = 0; k < 2; ++k) {
    const double* y = ws + (2 + k) * WD_NMAX;
    double s = 0.0;
    for (int i = t; i < n; i += PW_THREADS) s = fma(y[i], y[i], s);
    est[k] = sqrt(block_sum_256(s, red));
  }
  if (t != 0) return;
  const bool broken = ctrl != nullptr && ctrl->pass_fail >= 0;
  const double kpow = est[0] * est[1];
  double kappa = __builtin_inf();
  if (!broken) {
    const double kice = ctrl ? ctrl->kappa_rc : 0.0;
    if (isfinite(kpow) && isfinite(kice)) kappa = fmax(kice, kpow);
  }
  if (kappa_out) *kappa_out = kappa;
  if (!ctrl) return;
  ctrl->kappa_rc = kappa;
  const int f = ctrl->pass_fail;
  const bool bad = broken || !(kappa <= TAU_POSTERIOR);
  const int p = ctrl->cur_prec;
  if (phase != PH_RERUN2 && ctrl->auto_mode && bad && ctrl->status == ST_OK && (p == P_FP16 || p == P_FP32)) {
    ctrl->retry += 1;
    ctrl->cur_prec = (p == P_FP16) ? P_FP32 : P_FP64;
    ctrl->escalations += 1;
  } else {
    if (ctrl->status == ST_OK) {
      if (f >= 0) { ctrl->status = ST_CHOL; ctrl->chol_fail = f; }
      else if (!(kappa <= TAU_POSTERIOR)) ctrl->status = ST_POSTERIOR;
    }
    ctrl_carry_record(ctrl);
  }
}

size_t posterior_wide_ws_bytes() { return POSTERIOR_WS_DOUBLES * sizeof(double); }

hipError_t launch_posterior_wide(const double* Rc, const double* X, int n, int64_t ld, double* ws, Ctrl* ctrl,
                                 int phase, double* kappa_out, hipStream_t st) {
  if (n > WD_NMAX || ws == nullptr) return hipErrorInvalidValue;
  const dim3 grid((n + 15) / 16, 2), block(PW_THREADS);
  for (int it = 0; it <= POSTERIOR_STEPS; ++it) {
    hipLaunchKernelGGL(power_mv_kernel, grid, block, 0, st, Rc, X, n, ld, ws, it == 0 ? 1 : 0, (const Ctrl*)ctrl,
                       phase);
    if (it < POSTERIOR_STEPS)
      hipLaunchKernelGGL(power_tmv_kernel, grid, block, 0, st, Rc, X, n, ld, ws, (const Ctrl*)ctrl, phase);
  }
  hipLaunchKernelGGL(posterior_decide_kernel, dim3(1), block, 0, st, (const double*)ws, n, ctrl, phase, kappa_out);
  return hipGetLastError();
}

}  // namespace mrcqr
