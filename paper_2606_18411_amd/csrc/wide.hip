// The path for 128 < n <= 512 on column panels of 128 (64 for the sketch
// QR) or 32: every n x n object of the path outgrows one workgroup's registers
// and LDS, so each step is taken panel by panel with the kernels of the
// n <= 128 path plus the ones here.
//   Sketch QR (Algorithm 2, SketchQR): blocked Householder QR in the
//     sketch's QR precision; a panel of 64 columns is factored by one
//     workgroup (LAPACK geqr2 order, reflectors left in place below the
//     diagonal), its reflectors are applied to the columns to its right,
//     and the finish kernel takes R (rows with a negative pivot flipped),
//     the checks and the condition estimate of Rs.
//   B = A Rs^{-1} (Stage 2): per 128-column panel P, the update
//     C = A_P - B_{<P} Rs_{<P,P} (gemm_panel_kernel) and the solve of the
//     n <= 128 path with the diagonal panel, in place.
//   G = B^T B (Algorithm 1 step 1): the diagonal 128 x 128 blocks by the
//     n <= 128 Gram kernels, the blocks above them by gram_pair_kernel.
//   G = Rc^T Rc (Algorithm 1 step 2): right-looking over 128-column panels:
//     the n <= 128 Cholesky of the diagonal block, the panel
//     X = G_{rest,P} Rc_PP^{-1} by the solve, Rc_{P,rest} = X^T, and the
//     trailing update G_{rest,rest} -= X X^T (gemm_panel_kernel).
//   X = Rc^{-1}, R = Rc Rs, the posterior power steps and Q = B X, each for
//     n <= 512.
// Every kernel is gated by the control block like the n <= 128 ones.
#include "batch.hpp"
#include "ice.hpp"

namespace mrcqr {

constexpr int WD_NMAX = 512;
constexpr int WD_PANEL = 128;  // column panel of the solve, Gram, Cholesky and product

// ---------------------------------------------------------------------------
// C = beta C0 + alpha Bs W: rows x nc (nc <= 128) from Bs (rows x K) and W
// (K x nc; W(k, j) = W[k + j ldw], or W[j + k ldw] when TW). K is taken in
// steps of 16; entries with k >= kvalid read as zero (Bs and W are never
// read there). C0 may be C (each entry is read before it is written by the
// same lane); beta == 0 reads no C0.
// Each wave owns 16 rows (one tile) and all 8 column blocks of 16, 16 waves
// (four per SIMD) share a workgroup; the transposed product C^T = W^T Bs^T
// runs as float64 MFMA 16x16x4 with W (staged in LDS in A-operand order, 16
// k at a time, double-buffered) as A operand and the rows of Bs as B
// operand.
constexpr int GP_THREADS = 1024;
constexpr int GP_TILES = 1;
constexpr int GP_ROWS = (GP_THREADS / 64) * 16 * GP_TILES;

template <bool TW>
__global__ __launch_bounds__(GP_THREADS, 1) void gemm_panel_kernel(
    const double* __restrict__ Bs, int64_t ldb, int K, int kvalid, const double* __restrict__ W, int64_t ldw,
    const double* C0, int64_t ldc0, double* C, int64_t ldc, int rows, int nc, double alpha, double beta,
    const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ __attribute__((aligned(16))) double Wl[2][4 * 8 * 64];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nch = (K + 15) / 16;
  auto stage = [&](int buf, int k0) {
    for (int e = tid; e < 4 * 8 * 64; e += GP_THREADS) {
      const int ks = e / 512, b = (e / 64) % 8, ll = e % 64;
      const int k = k0 + 4 * ks + ll / 16, j = 16 * b + ll % 16;
      double v = 0.0;
      if (j < nc && k < kvalid) v = TW ? W[j + (int64_t)k * ldw] : W[k + (int64_t)j * ldw];
      Wl[buf][e] = v;
    }
  };
  // a lane's addresses: its own base (row l%16, column l/16) plus
  // wave-uniform offsets, stepped opaquely so that the optimizer does not
  // keep per-lane 64-bit offsets of every k-step live
  const double* Bl = Bs + c16 + (int64_t)g * ldb;
  const double* C0l = C0 + c16 + (int64_t)g * ldc0;
  double* Cl = C + c16 + (int64_t)g * ldc;
  for (int64_t pan = blockIdx.x; pan * GP_ROWS < rows; pan += gridDim.x) {
    const int64_t r0 = pan * GP_ROWS + 16 * GP_TILES * w;
    const bool row_in = r0 + c16 < rows;
    double bd[4][GP_TILES];
    auto loadb = [&](int k0) {
      int64_t u = r0 + (int64_t)k0 * ldb;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        asm volatile("" : "+s"(u));
        const bool in = row_in && k0 + 4 * ks + g < kvalid;
#pragma unroll
        for (int t = 0; t < GP_TILES; ++t) bd[ks][t] = in ? Bl[u + 16 * t] : 0.0;
        u += 4 * ldb;
      }
    };
    f64x4 acc[8][GP_TILES];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int t = 0; t < GP_TILES; ++t) acc[b][t] = f64x4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();  // the previous pass is done with Wl
    stage(0, 0);
    loadb(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      double cur[4][GP_TILES];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int t = 0; t < GP_TILES; ++t) cur[ks][t] = bd[ks][t];
      if (c + 1 < nch) {
        stage((c + 1) & 1, 16 * (c + 1));
        loadb(16 * (c + 1));
      }
      const double* Wb = Wl[c & 1];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const double ra = Wb[(ks * 8 + b) * 64 + l];
#pragma unroll
          for (int t = 0; t < GP_TILES; ++t) acc[b][t] = mfma_f64(ra, cur[ks][t], acc[b][t]);
        }
      __syncthreads();
    }
    // element (row 16 t + l%16, column 16 b + 4 r + l/16)
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t uc = r0 + (int64_t)(16 * b + 4 * r) * ldc, u0 = r0 + (int64_t)(16 * b + 4 * r) * ldc0;
        asm volatile("" : "+s"(uc), "+s"(u0));
        const bool in = row_in && 16 * b + 4 * r + g < nc;
#pragma unroll
        for (int t = 0; t < GP_TILES; ++t) {
          if (in) {
            double v = alpha * acc[b][t][r];
            if (beta != 0.0) v = fma(beta, C0l[u0 + 16 * t], v);
            Cl[uc + 16 * t] = v;
          }
        }
      }
  }
}

hipError_t launch_gemm_panel(bool tw, const double* Bs, int64_t ldb, int K, int kvalid, const double* W, int64_t ldw,
                             const double* C0, int64_t ldc0, double* C, int64_t ldc, int rows, int nc, double alpha,
                             double beta, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (nc < 1 || nc > 128 || rows < 1 || K < 1) return hipErrorInvalidValue;
  const int64_t panels = ((int64_t)rows + GP_ROWS - 1) / GP_ROWS;
  const dim3 grid((unsigned)(panels < 256 ? panels : 256)), block(GP_THREADS);
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
// (chunk, pair). 64-row panels of B_I and B_J are staged in LDS
// (column-major, 65-double stride); each of the 8 waves owns 2 x 4 of the
// 64 tiles (A operand B_I^T from two column tiles, B operand B_J from four).
constexpr int GPR_THREADS = 512;
constexpr int GPR_LD = 65;

// Pair pr of the blocks above the diagonal, row by row: (0,1), (0,2), ...,
// (1,2), ...
__device__ __forceinline__ void pair_of(int pr, int n, int& I, int& J) {
  const int np = (n + WD_PANEL - 1) / WD_PANEL;
  I = 0;
  while (pr >= np - 1 - I) { pr -= np - 1 - I; ++I; }
  J = I + 1 + pr;
}

__global__ __launch_bounds__(GPR_THREADS, 1) void gram_pair_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, int chunks, int rows_per_chunk,
    double* __restrict__ Gpart, const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ double Bi[128 * GPR_LD];
  __shared__ double Bj[128 * GPR_LD];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int chunk = blockIdx.x, pr = blockIdx.y;
  int I, J;
  pair_of(pr, n, I, J);
  const int ci0 = WD_PANEL * I, cj0 = WD_PANEL * J;
  const int nci = min(WD_PANEL, n - ci0), ncj = min(WD_PANEL, n - cj0);
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  const int ta0 = 2 * (w % 4), tb0 = 4 * (w / 4);
  f64x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t rbeg = (int64_t)chunk * rows_per_chunk;
  const int64_t rend = min((int64_t)m, rbeg + rows_per_chunk);
  for (int64_t p0 = rbeg; p0 < rend; p0 += 64) {
    __syncthreads();
    for (int e = tid; e < 64 * 128; e += GPR_THREADS) {
      const int r = e % 64, c = e / 64;
      const int64_t row = p0 + r;
      const bool rin = row < rend;
      Bi[c * GPR_LD + r] = (rin && c < nci) ? B[row + (int64_t)(ci0 + c) * ldb] : 0.0;
      Bj[c * GPR_LD + r] = (rin && c < ncj) ? B[row + (int64_t)(cj0 + c) * ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ks = 0; ks < 16; ++ks) {
      const int k = 4 * ks + g;
      double av[2], bv[4];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Bi[(16 * (ta0 + a) + c16) * GPR_LD + k];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bj[(16 * (tb0 + b) + c16) * GPR_LD + k];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma_f64(av[a], bv[b], acc[a][b]);
    }
  }
  // D[i][j] = (B_I^T B_J)[16 ta + i][16 tb + j]: lane l, register r holds
  // D[4 r + l/16][l%16]
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
// its mirror G_JI.
__global__ void gram_pair_reduce_kernel(const double* __restrict__ Gpart, int chunks, int n,
                                        double* __restrict__ G, int64_t ldg, const Ctrl* __restrict__ ctrl,
                                        int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int pr = blockIdx.y;
  int I, J;
  pair_of(pr, n, I, J);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= WD_PANEL * WD_PANEL) return;
  const int i = e % WD_PANEL, j = e / WD_PANEL;
  const int gi = WD_PANEL * I + i, gj = WD_PANEL * J + j;
  if (gi >= n || gj >= n) return;
  const double* p = Gpart + (int64_t)pr * chunks * (WD_PANEL * WD_PANEL) + e;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += p[(int64_t)c * (WD_PANEL * WD_PANEL)];
  G[gi + (int64_t)gj * ldg] = s;
  G[gj + (int64_t)gi * ldg] = s;
}

constexpr int GPR_CHUNKS = 256;

int wide_panels(int n) { return (n + WD_PANEL - 1) / WD_PANEL; }
int wide_pairs(int n) { const int np = wide_panels(n); return np * (np - 1) / 2; }

size_t gram_pair_partial_bytes(int n) {
  return (size_t)wide_pairs(n) * GPR_CHUNKS * WD_PANEL * WD_PANEL * sizeof(double) + 256;
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
    const int rpc = (int)((((int64_t)m + GPR_CHUNKS - 1) / GPR_CHUNKS + 63) / 64 * 64);
    const int chunks = (int)(((int64_t)m + rpc - 1) / rpc);
    hipLaunchKernelGGL(gram_pair_kernel, dim3(chunks, npr), dim3(GPR_THREADS), 0, st, B, m, n, ldb, chunks, rpc,
                       Gpart_pairs, ctrl, phase);
    hipLaunchKernelGGL(gram_pair_reduce_kernel, dim3((WD_PANEL * WD_PANEL + 255) / 256, npr), dim3(256), 0, st,
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
// one wave per column, arithmetic in T.
template <typename T, int RPL>
__global__ __launch_bounds__(256) void hh_apply_kernel(double* __restrict__ Y, int s, int n, int64_t ldy, int j0,
                                                       int nb, const double* __restrict__ tau,
                                                       const Ctrl* __restrict__ ctrl, int slot, int phase) {
  if (skip_launch(ctrl, slot, phase)) return;
  const int l = threadIdx.x & 63;
  const int c = j0 + nb + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const int sp = s - j0;
  T y[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = l + 64 * i;
    y[i] = (r < sp) ? (T)Y[(j0 + r) + (int64_t)c * ldy] : (T)0;
  }
  for (int k = 0; k < nb; ++k) {
    const double* vk = Y + j0 + (int64_t)(j0 + k) * ldy;
    T v[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = l + 64 * i;
      v[i] = (r > k && r < sp) ? (T)vk[r] : (r == k ? (T)1 : (T)0);
    }
    T dp = (T)0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) dp += v[i] * y[i];
    const T f = (T)tau[j0 + k] * wave_sum_dpp(dp);
#pragma unroll
    for (int i = 0; i < RPL; ++i) y[i] -= f * v[i];
  }
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = l + 64 * i;
    if (r < sp) Y[(j0 + r) + (int64_t)c * ldy] = (double)y[i];
  }
}

// Clear the flags word of the sketch QR (a small fill kernel, so the
// sequence records no memset).
__global__ void wide_flags_clear_kernel(int* flags, const Ctrl* __restrict__ ctrl, int slot, int phase) {
  if (skip_launch(ctrl, slot, phase)) return;
  if (threadIdx.x == 0) *flags = 0;
}

// R from the factored Y with diag(R) > 0 (rows with a negative pivot
// flipped), the singular / non-finite checks and the condition estimate of
// Rs with the AUTO escalation (the epilogue of the n <= 128 sketch QR).
__global__ __launch_bounds__(256) void hh_finish_kernel(const double* __restrict__ Y, int n, int64_t ldy,
                                                         double* __restrict__ Rs, int64_t ldr,
                                                         const int* __restrict__ flags,
                                                         double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl,
                                                         int slot, int phase, int want_kappa) {
  __shared__ int bad_sh;
  if (skip_launch(ctrl, slot, phase)) return;
  if (threadIdx.x == 0) bad_sh = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e % n, c = e / n;
    double v = 0.0;
    if (r <= c) {
      const double d = Y[r + (int64_t)r * ldy];
      v = (d < 0.0 ? -1.0 : 1.0) * Y[r + (int64_t)c * ldy];
      if (r == c && !(v > 0.0 && isfinite(v))) bad_sh = 1;
      if (r < c && !isfinite(v)) bad_sh = 1;
    }
    Rs[r + (int64_t)c * ldr] = v;
  }
  __syncthreads();
  const bool nonfinite = (*flags & 2) != 0;
  const bool bad = bad_sh != 0 || nonfinite;
  const bool auto_here = ctrl != nullptr && ctrl->auto_mode;
  double kappa = ice_kappa_block_wide(Rs, n, 1, (int)ldr, !bad && (auto_here || want_kappa));
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
      hipLaunchKernelGGL((hh_apply_kernel<T, RPL>), dim3((rest + 3) / 4), dim3(256), 0, st, Y, s, n, ldy, j0, nb,
                         (const double*)tau, ctrl, slot, phase);
  }
  return hipGetLastError();
}

// The sketch QR for n > 128: Y (s x n, ld ldy) is overwritten.
hipError_t launch_sketch_qr_wide(bool f64, double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                                 double* tau, int* flags, double* kappa, Ctrl* ctrl, int slot, int phase,
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
  hipLaunchKernelGGL(hh_finish_kernel, dim3(1), dim3(256), 0, st, (const double*)Y, n, ldy, Rs, ldr,
                     (const int*)flags, kappa, ctrl, slot, phase, kappa != nullptr ? 1 : 0);
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
// the whole matrix's numbering), the lower triangle cleared, and the ICE of
// Rc, into the control block as the n <= 128 Cholesky kernel leaves them.
__global__ __launch_bounds__(256) void chol_wide_finish_kernel(const int32_t* __restrict__ fails, int np, int n,
                                                               double* __restrict__ Rc, int64_t ldr,
                                                               int32_t* __restrict__ fail_out,
                                                               double* __restrict__ kappa_out,
                                                               Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  int f = -1;
  for (int P = 0; P < np; ++P)
    if (fails[P] >= 0) { f = WD_PANEL * P + fails[P]; break; }
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e % n, c = e / n;
    if (r > c || f >= 0) Rc[r + (int64_t)c * ldr] = 0.0;
  }
  __syncthreads();
  double kappa = ice_kappa_block_wide(Rc, n, 1, (int)ldr, f < 0);
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
// overwritten (trailing updates); T (n x 128, ld n) and fails (np ints) are
// scratch; Tw the solve's staging workspace.
hipError_t launch_cholesky_wide(double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                                double* kappa, double* T, int32_t* fails, void* Tw, Ctrl* ctrl, int phase,
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
  hipLaunchKernelGGL(chol_wide_finish_kernel, dim3(1), dim3(256), 0, st, (const int32_t*)fails, np, n, Rc, ldr, fail,
                     kappa, ctrl, phase);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// X = R^{-1} (R upper triangular, n <= 512): one wave per column j, lane l
// holding rows l + 64 q; x_i is formed on the lane holding row i and read
// by the others (back substitution in column order).
__global__ __launch_bounds__(64) void trinv_wide_kernel(const double* __restrict__ R, int n, int64_t ldr,
                                                        double* __restrict__ X, int64_t ldx,
                                                        const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  constexpr int Q = WD_NMAX / 64;
  const int j = blockIdx.x, l = threadIdx.x;
  double sv[Q], rinv[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = l + 64 * q;
    const int rc = min(r, n - 1);
    rinv[q] = 1.0 / R[rc + (int64_t)rc * ldr];
    sv[q] = (r == j) ? 1.0 : 0.0;
  }
  for (int i = j; i >= 0; --i) {
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
      else if (r < i) sv[q] = fma(-R[r + (int64_t)i * ldr], x, sv[q]);
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
// on M^T M from the normalized all-ones vector, threads 0..511 for Rc and
// 512..1023 for X (thread i forms y_i = (M x)_i, then z_i = (M^T y)_i).
__global__ __launch_bounds__(1024) void posterior_wide_kernel(const double* __restrict__ Rc,
                                                              const double* __restrict__ X, int n, int64_t ld,
                                                              Ctrl* __restrict__ ctrl, int phase,
                                                              double* __restrict__ kappa_out) {
  __shared__ double xs[2][WD_NMAX];
  __shared__ double ys[2][WD_NMAX];
  __shared__ double red[2][8];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int t = threadIdx.x, k = t >> 9, i = t & (WD_NMAX - 1), l = t & 63, wk = (t >> 6) & 7;
  const bool broken = ctrl != nullptr && ctrl->pass_fail >= 0;
  const double* M = k == 0 ? Rc : X;
  double est[2] = {__builtin_inf(), __builtin_inf()};
  if (!broken) {
    xs[k][i] = i < n ? 1.0 / sqrt((double)n) : 0.0;
    __syncthreads();
    double y = 0.0;
    for (int it = 0;; ++it) {
      y = 0.0;
      if (i < n)
        for (int j = i; j < n; ++j) y = fma(M[i + (int64_t)j * ld], xs[k][j], y);
      if (it == POSTERIOR_STEPS) break;
      ys[k][i] = y;
      __syncthreads();
      double z = 0.0;
      if (i < n)
        for (int r = 0; r <= i; ++r) z = fma(M[r + (int64_t)i * ld], ys[k][r], z);
      const double s2 = wave_sum_dpp(z * z);
      if (l == 0) red[k][wk] = s2;
      __syncthreads();
      double nz2 = 0.0;
      for (int q = 0; q < 8; ++q) nz2 += red[k][q];
      xs[k][i] = z / sqrt(nz2);
      __syncthreads();
    }
    const double q2 = wave_sum_dpp(y * y);
    if (l == 0) red[k][wk] = q2;
    __syncthreads();
    for (int kk = 0; kk < 2; ++kk) {
      double s = 0.0;
      for (int q = 0; q < 8; ++q) s += red[kk][q];
      est[kk] = sqrt(s);
    }
  }
  if (t != 0) return;
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

hipError_t launch_posterior_wide(const double* Rc, const double* X, int n, int64_t ld, Ctrl* ctrl, int phase,
                                 double* kappa_out, hipStream_t st) {
  if (n > WD_NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(posterior_wide_kernel, dim3(1), dim3(1024), 0, st, Rc, X, n, ld, ctrl, phase, kappa_out);
  return hipGetLastError();
}

}  // namespace mrcqr
