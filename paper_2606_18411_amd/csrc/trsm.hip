// Stage 2 triangular solves X = A R^{-1} (R upper triangular, n x n): the
// preconditioning solve A1 = A Rs^{-1} and Q = A1 R2^{-1} (Algorithm 2,
// Stage 2, and Algorithm 1, third step). The paper requires a solve, not a
// product with an explicitly inverted Rs (Section "Algorithm Description");
// the solve here is block forward substitution over column blocks of 16,
// where each 16 x 16 diagonal block is applied through its own inverse, as
// GPU BLAS triangular solves do. Rs as a whole is never inverted: the
// inverses are of the diagonal blocks only, each formed by substitution.
//
// A prep kernel stages R once per call into two operand arrays, padded with
// zeros beyond n:
//   Rop: off-diagonal blocks, pre-negated, in MFMA A-operand order,
//        Rop[off(J, q) + lane] = -R[4q + lane/16][16J + lane%16];
//   Dinv: the inverse of every diagonal block in MFMA A-operand order,
//        Dinv[256 J + 64 k + lane] = inv(R_JJ)[4k + lane/16][lane%16].
// Main kernel: each wave owns 32 rows (two row tiles of 16) and two waves
// share a SIMD. In the transposed form X_J^T = inv(R_JJ)^T (A_J^T -
// R_{<J,J}^T X_{<J}^T) both products run as float64 MFMA 16x16x4 with the
// staged operands (in LDS) as A operand. The D layout of a 16x16x4 f64
// result (lane l, register r: column 4r + l/16, row l%16 of the tile) is
// the B-operand layout of the four k-steps over those columns, so every
// solved block feeds the later blocks straight from its result registers,
// and the whole solve has no transposes and no vector arithmetic. The
// blocks of A stream through TR_DEPTH register buffers, TR_DEPTH blocks
// ahead of the solve, across row panels.
#include "batch.hpp"

namespace mrcqr {

constexpr int TR_THREADS = 256;              // 4 waves; two workgroups per CU
constexpr int TR_WROWS = 32;                 // rows per wave
constexpr int TR_NT = TR_WROWS / 16;         // row tiles per wave
constexpr int TR_ROWS = 4 * TR_WROWS;        // rows per workgroup pass
constexpr int TR_DEPTH = 4;                  // column blocks in flight per wave
constexpr int TR_NMAX = 128;

__host__ __device__ constexpr int tr_off(int J, int q) { return 64 * (2 * J * (J - 1) + q); }
__host__ __device__ constexpr int tr_rop_size(int nb) { return nb > 1 ? tr_off(nb, 0) : 64; }

size_t trsm_workspace_bytes(int n) {
  const int nb = (n + 15) / 16;
  return ((size_t)tr_rop_size(nb) + (size_t)nb * 256) * sizeof(double) + 256;
}

// Elements the prep spreads over its threads (Rop; every workgroup also
// takes its share of the diagonal blocks).
int trsm_prep_elems(int n) {
  const int nb = (n + 15) / 16;
  return tr_rop_size(nb);
}

// Rop by a grid-stride loop; the inverse of diagonal block J by workgroup
// J mod gx: the block is staged in LDS and 16 threads form one column each
// by back substitution. Launched with 256 threads per workgroup.
__device__ __forceinline__ void trsm_prep_body(const double* __restrict__ R, int n, int64_t ldr,
                                               double* __restrict__ Rop, double* __restrict__ Dinv,
                                               const Ctrl* __restrict__ ctrl, int phase, int bx, int gx) {
  __shared__ double Rb[16][17];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int nb = (n + 15) / 16;
  const int nrop = tr_rop_size(nb);
  const int t = threadIdx.x;
  for (int e = bx * blockDim.x + t; e < nrop; e += gx * blockDim.x) {
    // invert off(J, q) + lane
    int J = 1;
    while (J < nb && e >= tr_off(J + 1, 0)) ++J;
    const int rem = e - tr_off(J, 0);
    const int q = rem / 64, lane = rem % 64;
    const int row = 4 * q + lane / 16, col = 16 * J + lane % 16;
    Rop[e] = (nb > 1 && row < n && col < n) ? -R[row + (int64_t)col * ldr] : 0.0;
  }
  for (int J = bx; J < nb; J += gx) {
    const int o = 16 * J, r = t % 16, c = t / 16;
    Rb[r][c] = (o + r < n && o + c < n) ? R[(o + r) + (int64_t)(o + c) * ldr] : 0.0;
    __syncthreads();
    if (t < 16) {
      // column i = t of inv(R_JJ), zero beyond n (fixed trip counts with
      // predicates keep x in registers)
      const int i = t;
      const bool live = o + i < n;
      double x[16];
#pragma unroll
      for (int k = 15; k >= 0; --k) {
        double acc = 0.0;
#pragma unroll
        for (int u = k + 1; u < 16; ++u) acc = u <= i ? fma(Rb[k][u], x[u], acc) : acc;
        x[k] = !live || k > i ? 0.0 : (k == i ? 1.0 : -acc) / Rb[k][k];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) Dinv[256 * J + 64 * (k / 4) + 16 * (k % 4) + i] = x[k];
    }
    __syncthreads();
  }
}

__global__ void trsm_prep_kernel(const double* __restrict__ R, int n, int64_t ldr, double* __restrict__ Rop,
                                 double* __restrict__ Dinv, const Ctrl* __restrict__ ctrl, int phase) {
  trsm_prep_body(R, n, ldr, Rop, Dinv, ctrl, phase, blockIdx.x, gridDim.x);
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

// NB column blocks are compiled in. EXACT: the matrix has exactly NB blocks
// (the single-matrix launch picks the instance); otherwise (grouped launch,
// members of different widths) the block count is read at run time and
// blocks past it are skipped.
template <int NB, bool EXACT>
__device__ __forceinline__ void trsm_body(
    const double* __restrict__ A, int m, int n, int64_t lda,
    const double* __restrict__ Rop, const double* __restrict__ Dinv,
    double* __restrict__ X, int64_t ldx, const Ctrl* __restrict__ ctrl, int phase, int bx, int gx) {
  constexpr int RSZ = tr_rop_size(NB);
  constexpr int D = TR_DEPTH;
  constexpr int NSMAX = (NB + D - 1) / D * D;
  __shared__ __attribute__((aligned(16))) double Rl[RSZ];
  __shared__ __attribute__((aligned(16))) double Dl[NB * 256];
  if (skip_launch(ctrl, P_AUTO, phase)) return;

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const int nb = EXACT ? NB : (n + 15) / 16;
  const int rsz = tr_rop_size(nb);
  for (int e = tid; e < rsz; e += TR_THREADS) Rl[e] = Rop[e];
  for (int e = tid; e < nb * 256; e += TR_THREADS) Dl[e] = Dinv[e];
  __syncthreads();

  // Element (row 16 nt + l%16, column 16 J + 4 r + l/16) of a block goes to
  // register r of tile nt (the D layout). A lane's address is its own base
  // (row l%16, column l/16) plus a wave-uniform offset, stepped opaquely to
  // the optimizer so that it does not keep every block's offsets live.
  // Lanes outside the matrix read zero and store nothing (zero columns meet
  // zero coefficients; rows are independent). A and X are touched once:
  // non-temporal accesses.
  const double* Al = A + c16 + (int64_t)g * lda;
  double* Xl = X + c16 + (int64_t)g * ldx;
  // Slot J of a panel holds block J in ab[J % D]; once block J is solved
  // the block D slots later (this panel or the next) is loaded into that
  // buffer. A panel has a multiple of D slots; the ones past the last block
  // are empty.
  const int ns = (nb + D - 1) / D * D;
  f64x4 ab[D][TR_NT];
  auto load_blk = [&](int slot, int64_t pan, int J) {
    const int64_t rb = pan * TR_ROWS + TR_WROWS * w;
    if (rb >= m || J >= nb) return;  // never used
    int64_t u = rb + (int64_t)(16 * J) * lda;
    asm volatile("" : "+s"(u));
    const int64_t rows = m - rb;  // rows of the matrix from rb on
    const int cols = n - 16 * J;  // columns of the matrix from 16 J on
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int nt = 0; nt < TR_NT; ++nt) {
        const bool in = 16 * nt + c16 < rows && 4 * r + g < cols;
        ab[slot][nt][r] = in ? __builtin_nontemporal_load(&Al[u + 16 * nt + (int64_t)(4 * r) * lda]) : 0.0;
      }
  };
#pragma unroll
  for (int j = 0; j < D; ++j) load_blk(j, bx, j);
  for (int64_t pan = bx; pan * TR_ROWS < m; pan += gx) {
    const int64_t r0 = pan * TR_ROWS + TR_WROWS * w;
    f64x4 xb[NB][TR_NT];  // solved blocks (B-operand layout)
#pragma unroll
    for (int J = 0; J < NSMAX; ++J) {
      if (J < nb) {  // not an empty slot
        f64x4 acc[TR_NT];
#pragma unroll
        for (int nt = 0; nt < TR_NT; ++nt) acc[nt] = ab[J % D][nt];
#pragma unroll
        for (int K = 0; K < J; ++K)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double ra = Rl[tr_off(J, 4 * K + r) + l];
#pragma unroll
            for (int nt = 0; nt < TR_NT; ++nt) acc[nt] = mfma_f64(ra, xb[K][nt][r], acc[nt]);
          }
        f64x4 x[TR_NT];
#pragma unroll
        for (int nt = 0; nt < TR_NT; ++nt) x[nt] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double da = Dl[256 * J + 64 * k + l];
#pragma unroll
          for (int nt = 0; nt < TR_NT; ++nt) x[nt] = mfma_f64(da, acc[nt][k], x[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < TR_NT; ++nt) xb[J][nt] = x[nt];
        int64_t u = r0 + (int64_t)(16 * J) * ldx;
        asm volatile("" : "+s"(u));
        const int64_t rows = m - r0;
        const int cols = n - 16 * J;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int nt = 0; nt < TR_NT; ++nt)
            if (16 * nt + c16 < rows && 4 * r + g < cols) __builtin_nontemporal_store(x[nt][r], &Xl[u + 16 * nt + (int64_t)(4 * r) * ldx]);
      }
      if (J < ns) {
        const bool here = J + D < ns;
        load_blk(J % D, here ? pan : pan + gx, here ? J + D : J + D - ns);
      }
    }
  }
}

template <int NB>
__global__ __launch_bounds__(TR_THREADS, 2) void trsm_kernel(
    const double* __restrict__ A, int m, int n, int64_t lda,
    const double* __restrict__ Rop, const double* __restrict__ Dinv,
    double* __restrict__ X, int64_t ldx, const Ctrl* __restrict__ ctrl, int phase) {
  trsm_body<NB, true>(A, m, n, lda, Rop, Dinv, X, ldx, ctrl, phase, blockIdx.x, gridDim.x);
}

// Grouped: B = A Rs^{-1} of each member; a member uses its own block count.
template <int NB>
__global__ __launch_bounds__(TR_THREADS, 2) void trsm_grouped(const BatchInst* __restrict__ bi,
                                                              const int32_t* __restrict__ members, BatchCall call,
                                                              int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.trsm_blocks) return;
  const double* Rop = bat_ptr<const double>(call, d, d.off_Tw);
  trsm_body<NB, false>(call.A[i], d.m, d.n, call.lda[i], Rop, Rop + tr_rop_size((d.n + 15) / 16),
                             bat_ptr<double>(call, d, d.off_B), d.m, bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase,
                             blockIdx.x, d.trsm_blocks);
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
  if (nmax == 32) hipLaunchKernelGGL(trsm_grouped<2>, grid, dim3(TR_THREADS), 0, st, bi, members, call, phase);
  else if (nmax == 64) hipLaunchKernelGGL(trsm_grouped<4>, grid, dim3(TR_THREADS), 0, st, bi, members, call, phase);
  else if (nmax == 128) hipLaunchKernelGGL(trsm_grouped<8>, grid, dim3(TR_THREADS), 0, st, bi, members, call, phase);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_trsm(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr,
                       double* X, int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > TR_NMAX) return hipErrorInvalidValue;
  const int nb = (n + 15) / 16;
  double* Rop = static_cast<double*>(ws);
  double* Dinv = Rop + tr_rop_size(nb);
  const int prep_elems = trsm_prep_elems(n);
  hipLaunchKernelGGL(trsm_prep_kernel, dim3((prep_elems + 255) / 256), dim3(256), 0, st, R, n, ldr, Rop, Dinv,
                     ctrl, phase);
  // two workgroups per CU (two waves per SIMD: see the launch bounds)
  const int64_t panels = ((int64_t)m + TR_ROWS - 1) / TR_ROWS;
  const dim3 gr((unsigned)(panels < 512 ? panels : 512)), bl(TR_THREADS);
#define MRCQR_TRSM_CASE(NBV) \
  case NBV: hipLaunchKernelGGL(trsm_kernel<NBV>, gr, bl, 0, st, A, m, n, lda, Rop, Dinv, X, ldx, ctrl, phase); break;
  switch (nb) {
    MRCQR_TRSM_CASE(1) MRCQR_TRSM_CASE(2) MRCQR_TRSM_CASE(3) MRCQR_TRSM_CASE(4)
    MRCQR_TRSM_CASE(5) MRCQR_TRSM_CASE(6) MRCQR_TRSM_CASE(7) default: MRCQR_TRSM_CASE(8)
  }
#undef MRCQR_TRSM_CASE
  return hipGetLastError();
}

}  // namespace mrcqr
