// Stage 2 triangular solves X = A R^{-1} (R upper triangular, n x n): the
// preconditioning solve A1 = A Rs^{-1} and Q = A1 R2^{-1} (Algorithm 2,
// Stage 2, and Algorithm 1, third step). The paper requires a solve, not a
// product with an explicitly inverted Rs (Section "Algorithm Description"),
// so every 16 x 16 diagonal block is handled by substitution.
//
// Each wave owns 32 rows. Columns go in blocks J of 16. For block J the
// wave computes, in the transposed form X_J^T = R_JJ^{-T}(A_J^T -
// R_{<J,J}^T X_{<J}^T), the update as float64 MFMA 16x16x4 with the
// negated off-diagonal blocks of R (staged once per workgroup in LDS) as A
// operand and the already solved columns (kept in registers in B-operand
// layout) as B operand; the result goes through a per-wave LDS tile into
// one-row-per-lane layout, where lanes 0..31 run the forward substitution
// with the diagonal block (uniform, scalar-loaded entries of R and
// reciprocals of its diagonal), and back into B-operand registers and to X.
#include "common.hpp"

namespace mrcqr {

constexpr int TR_THREADS = 256;
constexpr int TR_ROWS = 128;  // rows per workgroup pass (4 waves x 32)
constexpr int TR_TLD = 17;    // leading dimension of the per-wave LDS tile

__host__ __device__ constexpr int tr_off(int J, int q) { return 64 * (2 * J * (J - 1) + q); }

template <int NMAX>
__global__ __launch_bounds__(TR_THREADS) void trsm_kernel(
    const double* __restrict__ A, int m, int n, int64_t lda,
    const double* __restrict__ R, int64_t ldr, double* __restrict__ X, int64_t ldx,
    const Ctrl* __restrict__ ctrl, int phase) {
  constexpr int NB = NMAX / 16;
  constexpr int RSZ = (NB > 1) ? tr_off(NB, 0) : 64;
  __shared__ double Rl[RSZ];
  __shared__ double invd[NMAX];
  __shared__ double Tt[4][32 * TR_TLD];
  if (skip_launch(ctrl, P_AUTO, phase)) return;

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nb = (n + 15) / 16;

  // stage -R[4q + g][16J + c16] for J >= 1, q < 4J (zero outside n x n)
  for (int J = 1; J < nb; ++J)
    for (int q = w; q < 4 * J; q += 4) {
      const int row = 4 * q + g, col = 16 * J + c16;
      Rl[tr_off(J, q) + l] = (row < n && col < n) ? -R[row + (int64_t)col * ldr] : 0.0;
    }
  for (int j = tid; j < NMAX; j += TR_THREADS) invd[j] = (j < n) ? 1.0 / R[j + (int64_t)j * ldr] : 0.0;
  __syncthreads();

  double* Tw = Tt[w];
  for (int64_t pan = blockIdx.x; pan * TR_ROWS < m; pan += gridDim.x) {
    const int64_t r0 = pan * TR_ROWS + 32 * w;
    double xb[4 * NB][2];
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      if (J >= nb) break;
      f64x4 acc[2];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 16 * nt + c16;
          const int col = 16 * J + d_row_f64(l, r);
          acc[nt][r] = (row < m && col < n) ? A[row + (int64_t)col * lda] : 0.0;
        }
#pragma unroll
      for (int q = 0; q < 4 * J; ++q) {
        const double ra = Rl[tr_off(J, q) + l];
        acc[0] = mfma_f64(ra, xb[q][0], acc[0]);
        acc[1] = mfma_f64(ra, xb[q][1], acc[1]);
      }
      // transpose through LDS: Tw[row_local][col_local]
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) Tw[(16 * nt + c16) * TR_TLD + d_row_f64(l, r)] = acc[nt][r];
      __syncthreads();
      if (l < 32) {
        double y[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = Tw[l * TR_TLD + k];
        const int base = 16 * J;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (base + k < n) {
            const double xk = y[k] * invd[base + k];
            y[k] = xk;
#pragma unroll
            for (int jj = k + 1; jj < 16; ++jj)
              if (base + jj < n) y[jj] = fma(-xk, R[(base + k) + (int64_t)(base + jj) * ldr], y[jj]);
          }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) Tw[l * TR_TLD + k] = y[k];
      }
      __syncthreads();
#pragma unroll
      for (int qq = 0; qq < 4; ++qq)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const double v = Tw[(16 * nt + c16) * TR_TLD + 4 * qq + g];
          xb[4 * J + qq][nt] = v;
          const int64_t row = r0 + 16 * nt + c16;
          const int col = 16 * J + 4 * qq + g;
          if (row < m && col < n) X[row + (int64_t)col * ldx] = v;
        }
      __syncthreads();
    }
  }
}

hipError_t launch_trsm(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr,
                       double* X, int64_t ldx, const Ctrl* ctrl, int phase, hipStream_t st) {
  const int64_t panels = ((int64_t)m + TR_ROWS - 1) / TR_ROWS;
  const int grid = (int)(panels < 1024 ? panels : 1024);
  if (grid < 1) return hipSuccess;
  if (n <= 32) hipLaunchKernelGGL(trsm_kernel<32>, dim3(grid), dim3(TR_THREADS), 0, st, A, m, n, lda, R, ldr, X, ldx, ctrl, phase);
  else if (n <= 64) hipLaunchKernelGGL(trsm_kernel<64>, dim3(grid), dim3(TR_THREADS), 0, st, A, m, n, lda, R, ldr, X, ldx, ctrl, phase);
  else if (n <= 128) hipLaunchKernelGGL(trsm_kernel<128>, dim3(grid), dim3(TR_THREADS), 0, st, A, m, n, lda, R, ldr, X, ldx, ctrl, phase);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mrcqr
