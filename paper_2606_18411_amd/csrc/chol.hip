// Algorithm 1, second step: Cholesky factorization G = Rc^T Rc (float64),
// with breakdown detection (a pivot that is not positive or not finite,
// the failure mode the paper describes for Cholesky-QR), the posterior
// condition estimate of Rc = the condition number of A Rs^{-1} (Section
// "Adaptive Precision Selection": an underestimated precision shows up as
// lost orthogonality), Stage 3's product R = Rc Rs, and the small
// per-call control kernels.
#include "common.hpp"
#include "ice.hpp"

namespace mrcqr {

constexpr int CH_THREADS = 1024;
constexpr int CH_NMAX = 128;
constexpr int TRMM_NMAX = 128;

// Right-looking Cholesky of the upper triangle of G (n <= 128), register
// resident: thread (ty, tx) owns L[i][k] for rows i = ty + 16a (a < 8) and
// columns k = tx + 64b (b < 2). Row j, updated by steps < j, sits in LDS
// (double-buffered); at step j every thread applies
// L[i][k] -= L[j][i] L[j][k] / piv_j to all its entries, without a mask
// (the update is uniform work; rows i <= j hold garbage afterwards), and
// the owners of row j + 1 publish it and copy it to Rl, where the final
// rows collect. One barrier per step. The rows are scaled by 1/sqrt(piv)
// at the end, which gives the textbook
// R[j][k] = (G[j][k] - sum_i R[i][j] R[i][k]) / R[j][j].
__global__ __launch_bounds__(CH_THREADS) void chol_kernel(
    const double* __restrict__ G, int n, int64_t ldg, double* __restrict__ Rc, int64_t ldr,
    int32_t* __restrict__ fail_out, double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  constexpr int TY = CH_THREADS / 64;   // 16 row groups
  constexpr int NA = CH_NMAX / TY;      // 8 rows per thread
  constexpr int NBK = CH_NMAX / 64;     // 2 columns per thread
  constexpr int LDR = CH_NMAX + 1;
  __shared__ double prow[2][CH_NMAX];   // published pivot rows (double-buffered)
  __shared__ double Rl[CH_NMAX * LDR];  // row-major
  __shared__ double rscale[CH_NMAX];
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;
  double Lr[NA][NBK];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      const int i = ty + TY * a, k = tx + 64 * b;
      Lr[a][b] = (i < n && k < n && i <= k) ? G[i + (int64_t)k * ldg] : 0.0;
    }
  if (ty == 0) {
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      prow[0][tx + 64 * b] = Lr[0][b];
      Rl[tx + 64 * b] = Lr[0][b];
    }
  }
  __syncthreads();
  const int tyu = __builtin_amdgcn_readfirstlane(ty);
  int f = -1;
  for (int j = 0; j < n; ++j) {
    const int buf = j & 1;
    const double piv = prow[buf][j];
    double ri[NA], pk[NBK];
#pragma unroll
    for (int a = 0; a < NA; ++a) ri[a] = prow[buf][tyu + TY * a];
#pragma unroll
    for (int b = 0; b < NBK; ++b) pk[b] = prow[buf][tx + 64 * b];
    if (!(piv > 0.0) || !isfinite(piv)) { f = j; break; }
    const double inv = rcp_nr(piv);
    double rk[NBK];
#pragma unroll
    for (int b = 0; b < NBK; ++b) rk[b] = pk[b] * inv;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NBK; ++b) Lr[a][b] = fma(-ri[a], rk[b], Lr[a][b]);
    const int jn = j + 1;
    if (jn < n && tyu == jn % TY) {
      const int an = jn / TY;
#pragma unroll
      for (int a = 0; a < NA; ++a)
        if (a == an) {
#pragma unroll
          for (int b = 0; b < NBK; ++b) {
            prow[buf ^ 1][tx + 64 * b] = Lr[a][b];
            Rl[jn * LDR + tx + 64 * b] = Lr[a][b];
          }
        }
    }
    __syncthreads();
  }
  // rows i < nrows = (f < 0 ? n : f) of Rl hold the Schur rows; zero the
  // strict lower triangle and the rows past a breakdown, scale row i by
  // 1/sqrt(piv_i) (diagonal: sqrt(piv_i))
  const int nrows = (f < 0) ? n : f;
  __syncthreads();
  if (tid < n) {
    const double d = Rl[tid * LDR + tid];
    rscale[tid] = (tid < nrows) ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += CH_THREADS) {
    const int i = e / n, k = e % n;
    double v = 0.0;
    if (i < nrows && k >= i) v = (k == i) ? sqrt(Rl[i * LDR + i]) : Rl[i * LDR + k] * rscale[i];
    Rl[i * LDR + k] = v;
  }
  __syncthreads();
  for (int k = tx; k < n; k += 64)
    for (int i = ty; i < n; i += TY) Rc[i + (int64_t)k * ldr] = (f < 0) ? Rl[i * LDR + k] : 0.0;
  {
    double kappa = ice_kappa_block(Rl, n, LDR, 1, f < 0);
    if (f >= 0) kappa = __builtin_inf();
    if (tid == 0) {
      if (fail_out) *fail_out = f;
      if (kappa_out) *kappa_out = kappa;
      if (ctrl) {
        ctrl->kappa_rc = kappa;
        const bool bad = (f >= 0) || !(kappa <= TAU_POSTERIOR);
        const int p = ctrl->cur_prec;
        if (phase == PH_FIRST && ctrl->auto_mode && bad && ctrl->status == ST_OK &&
            (p == P_FP16 || p == P_FP32)) {
          // self-correcting rerun one precision higher (Section "Adaptive
          // Precision Selection"): the rerun pass is enabled on the device
          ctrl->retry = 1;
          ctrl->cur_prec = (p == P_FP16) ? P_FP32 : P_FP64;
          ctrl->escalations += 1;
        } else if (ctrl->status == ST_OK) {
          if (f >= 0) { ctrl->status = ST_CHOL; ctrl->chol_fail = f; }
          else if (!(kappa <= TAU_POSTERIOR)) ctrl->status = ST_POSTERIOR;
        }
      }
    }
  }
}

// R = R2 R1 (upper x upper), each entry sum_{j=i..k} R2[i][j] R1[j][k]
// accumulated in index order.
__global__ __launch_bounds__(64) void trmm_kernel(const double* __restrict__ R2, int64_t ld2,
                                                  const double* __restrict__ R1, int64_t ld1, int n,
                                                  double* __restrict__ R, int64_t ldr,
                                                  const Ctrl* __restrict__ ctrl, int phase) {
  // one wave per (64-row block, 16-column block): lane l accumulates row
  // i = 64 blockIdx.y + l of the 16 columns c0..c0+15. The needed parts of
  // R2 (rows i0..i0+63, columns i0..jend-1) and of R1 (rows 0..jend-1,
  // the 16 columns) are staged in LDS first. Only the upper triangles of
  // R1 and R2 are read as values.
  __shared__ __attribute__((aligned(16))) double r1s[TRMM_NMAX * 16];
  __shared__ __attribute__((aligned(16))) double r2s[64 * TRMM_NMAX];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int l = threadIdx.x;
  const int c0 = 16 * blockIdx.x, i0 = 64 * blockIdx.y;
  const int i = i0 + l;
  const int jend = min(n, c0 + 16);  // R1[j][c] = 0 for j > c
  // loads with clamped (always valid) addresses and no branches, so that
  // they are all in flight together; the masks are applied afterwards
  {
    double v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int e = l + 64 * u, j = min(e / 16, n - 1), c = e % 16;
      v[u] = R1[j + (int64_t)min(c0 + c, n - 1) * ld1];
    }
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int e = l + 64 * u, j = e / 16, c = e % 16;
      if (e < jend * 16) r1s[e] = (c0 + c < n && j <= c0 + c) ? v[u] : 0.0;
    }
  }
  // R2[i][j] for j in [i0, jend), column-major in LDS (64 rows per column).
  // A full 64-row block with an even leading dimension is copied by direct
  // global-to-LDS loads (two columns of 16-byte pairs per instruction, all
  // in flight together); otherwise element by element.
  const bool direct = (i0 + 64 <= n) && ((ld2 & 1) == 0) && ((reinterpret_cast<uintptr_t>(R2) & 15) == 0);
  if (direct) {
    typedef __attribute__((address_space(3))) void lds_t;
    const int ncol = jend - i0;
    for (int k = 0; 2 * k < ncol; ++k) {
      const int jj = min(2 * k + (l >> 5), ncol - 1);
      const double* src = R2 + (i0 + 2 * (l & 31)) + (int64_t)(i0 + jj) * ld2;
      __builtin_amdgcn_global_load_lds(src, (lds_t*)(r2s + 128 * k), 16, 0, 0);
    }
    __builtin_amdgcn_s_waitcnt(0);
  } else {
    const int ic = min(i, n - 1);
    for (int j0 = i0; j0 < jend; j0 += 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = R2[ic + (int64_t)min(j0 + u, n - 1) * ld2];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (j0 + u < jend) r2s[(j0 + u - i0) * 64 + l] = v[u];
    }
  }
  __syncthreads();
  // only the upper triangle of R2 is a value: zero row i's entries j < i
  // (all of them for rows past n), then the product loop has no branches
  const int ncol = jend - i0;
  const int zlim = (i < n) ? min(l, ncol) : ncol;
  for (int jj = 0; jj < zlim; ++jj) r2s[jj * 64 + l] = 0.0;
  __syncthreads();
  double acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0;
#pragma unroll 4
  for (int jj = 0; jj < ncol; ++jj) {
    const double a = r2s[jj * 64 + l];
    const double* rr = r1s + (i0 + jj) * 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = fma(a, rr[c], acc[c]);
  }
  if (i < n) {
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c0 + c < n) R[i + (int64_t)(c0 + c) * ldr] = acc[c];
  }
}

__global__ void ctrl_init_kernel(Ctrl* ctrl, int prec, int auto_mode) {
  if (threadIdx.x == 0) {
    ctrl->cur_prec = prec;
    ctrl->status = ST_OK;
    ctrl->chol_fail = -1;
    ctrl->escalations = 0;
    ctrl->auto_mode = auto_mode;
    ctrl->retry = 0;
    ctrl->kappa_rs = 0.0;
    ctrl->kappa_rc = 0.0;
  }
}

struct InfoOut {
  int32_t status, precision_used, chol_fail_index, escalations;
  double kappa_rs_est, kappa_rc_est;
};

__global__ void ctrl_finalize_kernel(const Ctrl* ctrl, InfoOut* info) {
  if (threadIdx.x == 0) {
    info->status = ctrl->status;
    info->precision_used = ctrl->cur_prec;
    info->chol_fail_index = ctrl->chol_fail;
    info->escalations = ctrl->escalations;
    info->kappa_rs_est = ctrl->kappa_rs;
    info->kappa_rc_est = ctrl->kappa_rc;
  }
}



hipError_t launch_cholesky(const double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                           double* kappa, Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > CH_NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(CH_THREADS), 0, st, G, n, ldg, Rc, ldr, fail, kappa, ctrl, phase);
  return hipGetLastError();
}

hipError_t launch_trmm(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int n, double* R,
                       int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > TRMM_NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trmm_kernel, dim3((n + 15) / 16, (n + 63) / 64), dim3(64), 0, st, R2, ld2, R1, ld1, n, R, ldr,
                     ctrl, phase);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl* ctrl, int prec, int auto_mode, hipStream_t st) {
  hipLaunchKernelGGL(ctrl_init_kernel, dim3(1), dim3(64), 0, st, ctrl, prec, auto_mode);
  return hipGetLastError();
}

hipError_t launch_ctrl_finalize(const Ctrl* ctrl, void* info, hipStream_t st) {
  hipLaunchKernelGGL(ctrl_finalize_kernel, dim3(1), dim3(64), 0, st, ctrl, (InfoOut*)info);
  return hipGetLastError();
}

}  // namespace mrcqr
