// Stage 2 triangular solves X = A R^{-1} (R upper triangular, n x n): the
// preconditioning solve A1 = A Rs^{-1} and Q = A1 R2^{-1} (Algorithm 2,
// Stage 2, and Algorithm 1, third step). The paper requires a solve, not a
// product with an explicitly inverted Rs (Section "Algorithm Description"),
// so every 16 x 16 diagonal block is handled by substitution.
//
// A prep kernel stages R once per call into two padded, pre-negated operand
// arrays (no bound checks remain in the main loop):
//   Rop: off-diagonal blocks in MFMA A-operand order,
//        Rop[off(J, q) + lane] = -R[4q + lane/16][16J + lane%16];
//   Dg:  diagonal blocks row-major, Dg[J][k][j] = -R[16J+k][16J+j] (j > k),
//        1/R[16J+k][16J+k] on the diagonal, zero elsewhere and beyond n.
// Main kernel: each wave owns 64 rows (4 row tiles of 16). Columns go in
// blocks J of 16. In the transposed form X_J^T = R_JJ^{-T}(A_J^T -
// R_{<J,J}^T X_{<J}^T) the update runs as float64 MFMA 16x16x4 with Rop
// (staged in LDS) as A operand and the solved columns (kept in registers in
// B-operand layout) as B operand. The result goes through a per-wave LDS
// tile to one row per lane, the 64 lanes run the forward substitution with
// wave-uniform diagonal-block rows (scalar loads), and the solved columns
// return to B-operand registers and to X.
#include "batch.hpp"

namespace mrcqr {

constexpr int TR_THREADS = 256;
constexpr int TR_WROWS = 64;                 // rows per wave
constexpr int TR_ROWS = 4 * TR_WROWS;        // rows per workgroup pass
constexpr int TR_TLD = 17;                   // leading dimension of the per-wave LDS tile
constexpr int TR_NMAX = 128;

__host__ __device__ constexpr int tr_off(int J, int q) { return 64 * (2 * J * (J - 1) + q); }
__host__ __device__ constexpr int tr_rop_size(int nb) { return nb > 1 ? tr_off(nb, 0) : 64; }

size_t trsm_workspace_bytes(int n) {
  const int nb = (n + 15) / 16;
  return ((size_t)tr_rop_size(nb) + (size_t)nb * 256) * sizeof(double) + 256;
}

__device__ __forceinline__ void trsm_prep_body(const double* __restrict__ R, int n, int64_t ldr,
                                               double* __restrict__ Rop, double* __restrict__ Dg,
                                               const Ctrl* __restrict__ ctrl, int phase, int bx, int gx) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int nb = (n + 15) / 16;
  const int nrop = tr_rop_size(nb);
  for (int e = bx * blockDim.x + threadIdx.x; e < nrop + nb * 256; e += gx * blockDim.x) {
    if (e < nrop) {
      // invert off(J, q) + lane
      int J = 1;
      while (J < nb && e >= tr_off(J + 1, 0)) ++J;
      const int rem = e - tr_off(J, 0);
      const int q = rem / 64, lane = rem % 64;
      const int row = 4 * q + lane / 16, col = 16 * J + lane % 16;
      Rop[e] = (nb > 1 && row < n && col < n) ? -R[row + (int64_t)col * ldr] : 0.0;
    } else {
      const int d = e - nrop;
      const int J = d / 256, k = (d % 256) / 16, j = d % 16;
      const int row = 16 * J + k, col = 16 * J + j;
      double v = 0.0;
      if (row < n && col < n) {
        if (j > k) v = -R[row + (int64_t)col * ldr];
        else if (j == k) v = 1.0 / R[row + (int64_t)row * ldr];
      }
      Dg[d] = v;
    }
  }
}

__global__ void trsm_prep_kernel(const double* __restrict__ R, int n, int64_t ldr, double* __restrict__ Rop,
                                 double* __restrict__ Dg, const Ctrl* __restrict__ ctrl, int phase) {
  trsm_prep_body(R, n, ldr, Rop, Dg, ctrl, phase, blockIdx.x, gridDim.x);
}

// Grouped: Rs of each member into its operand arrays (grid-stride over the
// largest member's element count).
__global__ void trsm_prep_grouped(const BatchInst* __restrict__ bi, const int32_t* __restrict__ members,
                                  BatchCall call, int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  double* Rop = bat_ptr<double>(call, d, d.off_Tw);
  trsm_prep_body(bat_ptr<const double>(call, d, d.off_Rs), d.n, d.n, Rop, Rop + tr_rop_size((d.n + 15) / 16),
                 bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NMAX>
__device__ __forceinline__ void trsm_body(
    const double* __restrict__ A, int m, int n, int64_t lda,
    const double* __restrict__ Rop, const double* __restrict__ Dg,
    double* __restrict__ X, int64_t ldx, const Ctrl* __restrict__ ctrl, int phase, int bx, int gx) {
  constexpr int NB = NMAX / 16;
  constexpr int RSZ = tr_rop_size(NB);
  __shared__ __attribute__((aligned(16))) double Rl[RSZ];
  __shared__ double Tt[4][TR_WROWS * TR_TLD];
  if (skip_launch(ctrl, P_AUTO, phase)) return;

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nb = (n + 15) / 16;
  const int rsz = tr_rop_size(nb);
  for (int e = tid; e < rsz; e += TR_THREADS) Rl[e] = Rop[e];
  __syncthreads();

  double* Tw = Tt[w];
  for (int64_t pan = bx; pan * TR_ROWS < m; pan += gx) {
    const int64_t r0 = pan * TR_ROWS + TR_WROWS * w;
    double xb[4 * NB][4];
    double an[4][4];
    auto load_a = [&](int J) {
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 16 * nt + c16;
          const int col = 16 * J + d_row_f64(l, r);
          an[nt][r] = (row < m && col < n) ? A[row + (int64_t)col * lda] : 0.0;
        }
    };
    load_a(0);
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      if (J >= nb) break;
      f64x4 acc[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = f64x4{an[nt][0], an[nt][1], an[nt][2], an[nt][3]};
      if (J + 1 < nb) load_a(J + 1);
#pragma unroll
      for (int q = 0; q < 4 * J; ++q) {
        const double ra = Rl[tr_off(J, q) + l];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma_f64(ra, xb[q][nt], acc[nt]);
      }
      // to one row per lane: Tw[row_local][col_local]
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) Tw[(16 * nt + c16) * TR_TLD + d_row_f64(l, r)] = acc[nt][r];
      wave_lds_sync();
      double y[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) y[k] = Tw[l * TR_TLD + k];
      const double* Dr = Dg + J * 256;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double xk = y[k] * Dr[17 * k];
        y[k] = xk;
#pragma unroll
        for (int jj = k + 1; jj < 16; ++jj) y[jj] = fma(xk, Dr[16 * k + jj], y[jj]);
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) Tw[l * TR_TLD + k] = y[k];
      wave_lds_sync();
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const double v = Tw[(16 * nt + c16) * TR_TLD + 4 * qq + g];
          xb[4 * J + qq][nt] = v;
          const int64_t row = r0 + 16 * nt + c16;
          const int col = 16 * J + 4 * qq + g;
          if (row < m && col < n) X[row + (int64_t)col * ldx] = v;
        }
      wave_lds_sync();
    }
  }
}

template <int NMAX>
__global__ __launch_bounds__(TR_THREADS, NMAX == 64 ? 2 : (NMAX == 32 ? 4 : 1)) void trsm_kernel(
    const double* __restrict__ A, int m, int n, int64_t lda,
    const double* __restrict__ Rop, const double* __restrict__ Dg,
    double* __restrict__ X, int64_t ldx, const Ctrl* __restrict__ ctrl, int phase) {
  trsm_body<NMAX>(A, m, n, lda, Rop, Dg, X, ldx, ctrl, phase, blockIdx.x, gridDim.x);
}

// Grouped: B = A Rs^{-1} of each member; a member uses its own block count.
template <int NMAX>
__global__ __launch_bounds__(TR_THREADS, NMAX == 64 ? 2 : (NMAX == 32 ? 4 : 1)) void trsm_grouped(const BatchInst* __restrict__ bi,
                                                           const int32_t* __restrict__ members, BatchCall call,
                                                           int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.trsm_blocks) return;
  const double* Rop = bat_ptr<const double>(call, d, d.off_Tw);
  trsm_body<NMAX>(call.A[i], d.m, d.n, call.lda[i], Rop, Rop + tr_rop_size((d.n + 15) / 16),
                  bat_ptr<double>(call, d, d.off_B), d.m, bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase, blockIdx.x,
                  d.trsm_blocks);
}

// Blocks of the solve for an m-row member of a batch: about four row panels
// per workgroup, at most one workgroup per compute unit.
int trsm_batch_blocks(int64_t m) {
  const int64_t panels = (m + TR_ROWS - 1) / TR_ROWS;
  const int64_t b = (panels + 3) / 4;
  return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

hipError_t launch_trsm_grouped(int nmax, const BatchInst* bi, const int32_t* members, int count, int max_elems,
                               int max_blocks, const BatchCall& call, int phase, hipStream_t st) {
  hipLaunchKernelGGL(trsm_prep_grouped, dim3((max_elems + 255) / 256, count), dim3(256), 0, st, bi, members, call,
                     phase);
  const dim3 grid(max_blocks, count);
  if (nmax == 32) hipLaunchKernelGGL(trsm_grouped<32>, grid, dim3(TR_THREADS), 0, st, bi, members, call, phase);
  else if (nmax == 64) hipLaunchKernelGGL(trsm_grouped<64>, grid, dim3(TR_THREADS), 0, st, bi, members, call, phase);
  else if (nmax == 128) hipLaunchKernelGGL(trsm_grouped<128>, grid, dim3(TR_THREADS), 0, st, bi, members, call, phase);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

int trsm_prep_elems(int n) {
  const int nb = (n + 15) / 16;
  return tr_rop_size(nb) + nb * 256;
}

hipError_t launch_trsm(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr,
                       double* X, int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > TR_NMAX) return hipErrorInvalidValue;
  const int nb = (n + 15) / 16;
  double* Rop = static_cast<double*>(ws);
  double* Dg = Rop + tr_rop_size(nb);
  const int prep_elems = tr_rop_size(nb) + nb * 256;
  hipLaunchKernelGGL(trsm_prep_kernel, dim3((prep_elems + 255) / 256), dim3(256), 0, st, R, n, ldr, Rop, Dg,
                     ctrl, phase);
  const int64_t panels = ((int64_t)m + TR_ROWS - 1) / TR_ROWS;
  // one workgroup per CU per wave the instance fits on a SIMD (1 at n > 64,
  // 2 at n <= 64, 4 at n <= 32: see the launch bounds)
  const int64_t cap = 256 * (n <= 32 ? 4 : (n <= 64 ? 2 : 1));
  const int grid = (int)(panels < cap ? panels : cap);
  if (grid < 1) return hipGetLastError();
  if (n <= 32) hipLaunchKernelGGL(trsm_kernel<32>, dim3(grid), dim3(TR_THREADS), 0, st, A, m, n, lda, Rop, Dg, X, ldx, ctrl, phase);
  else if (n <= 64) hipLaunchKernelGGL(trsm_kernel<64>, dim3(grid), dim3(TR_THREADS), 0, st, A, m, n, lda, Rop, Dg, X, ldx, ctrl, phase);
  else hipLaunchKernelGGL(trsm_kernel<128>, dim3(grid), dim3(TR_THREADS), 0, st, A, m, n, lda, Rop, Dg, X, ldx, ctrl, phase);
  return hipGetLastError();
}

}  // namespace mrcqr
