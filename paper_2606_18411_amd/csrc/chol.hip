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

constexpr int CH_THREADS = 512;
constexpr int CH_NMAX = 128;

// Right-looking Cholesky of the upper triangle of G (n <= 128), register
// resident: thread (ty, tx) owns L[i][k] for rows i = ty + 8a (a < 16) and
// columns k = tx + 64b (b < 2). At step j the owners of row j publish it
// (already updated by steps < j) in LDS; every thread then updates its
// trailing entries L[i][k] -= L[j][i] L[j][k] / piv_j. One barrier per step;
// the rows are scaled by 1/sqrt(piv) at the end, which gives the textbook
// R[j][k] = (G[j][k] - sum_i R[i][j] R[i][k]) / R[j][j].
__global__ __launch_bounds__(CH_THREADS) void chol_kernel(
    const double* __restrict__ G, int n, int64_t ldg, double* __restrict__ Rc, int64_t ldr,
    int32_t* __restrict__ fail_out, double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  constexpr int TY = CH_THREADS / 64;   // 8 row groups
  constexpr int NA = CH_NMAX / TY;      // 16 rows per thread
  constexpr int NBK = CH_NMAX / 64;     // 2 columns per thread
  __shared__ double prow[2][CH_NMAX];   // published pivot rows (double-buffered)
  __shared__ double Rl[CH_NMAX * (CH_NMAX + 1)];
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
  int f = -1;
  for (int j = 0; j < n; ++j) {
    const int buf = j & 1;
    if (ty == (j % TY)) {
      const int aj = j / TY;
#pragma unroll
      for (int a = 0; a < NA; ++a)
        if (a == aj) {
#pragma unroll
          for (int b = 0; b < NBK; ++b) prow[buf][tx + 64 * b] = Lr[a][b];
        }
    }
    __syncthreads();
    const double piv = prow[buf][j];
    if (!(piv > 0.0) || !isfinite(piv)) { f = j; break; }
    const double inv = 1.0 / piv;
    double rk[NBK], ri[NA];
#pragma unroll
    for (int b = 0; b < NBK; ++b) rk[b] = prow[buf][tx + 64 * b] * inv;
#pragma unroll
    for (int a = 0; a < NA; ++a) ri[a] = prow[buf][min(ty + TY * a, CH_NMAX - 1)];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NBK; ++b) {
        const int i = ty + TY * a, k = tx + 64 * b;
        const bool upd = (i > j) && (k >= i);
        Lr[a][b] = upd ? fma(-ri[a], rk[b], Lr[a][b]) : Lr[a][b];
      }
  }
  // rows j < (f < 0 ? n : f) hold G's Schur rows; scale them into R
  const int nrows = (f < 0) ? n : f;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NBK; ++b) {
      const int i = ty + TY * a, k = tx + 64 * b;
      if (i < n && k < n) Rl[i * (CH_NMAX + 1) + k] = (i <= k && i < nrows) ? Lr[a][b] : 0.0;
    }
  __syncthreads();
  for (int i = ty; i < nrows; i += TY) {
    const double d = Rl[i * (CH_NMAX + 1) + i];
    const double rinv = 1.0 / sqrt(d);
    for (int k = i + tx; k < n; k += 64) Rl[i * (CH_NMAX + 1) + k] = (k == i) ? sqrt(d) : Rl[i * (CH_NMAX + 1) + k] * rinv;
  }
  __syncthreads();
  for (int k = tx; k < n; k += 64)
    for (int i = ty; i < n; i += TY) Rc[i + (int64_t)k * ldr] = (f < 0 && i <= k) ? Rl[i * (CH_NMAX + 1) + k] : 0.0;
  if (tid < 64) {
    double kappa = __builtin_inf();
    if (f < 0) kappa = ice_kappa(Rl, n, CH_NMAX + 1, 1);
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

// R = R2 R1 (upper x upper): one block per column k; column k of R1 is
// staged in LDS and thread i forms sum_{j=i..k} R2[i][j] R1[j][k] in index
// order (coalesced reads of R2 across threads).
__global__ __launch_bounds__(256) void trmm_kernel(const double* __restrict__ R2, int64_t ld2,
                                                   const double* __restrict__ R1, int64_t ld1, int n,
                                                   double* __restrict__ R, int64_t ldr,
                                                   const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  extern __shared__ double col[];
  const int k = blockIdx.x;
  for (int j = threadIdx.x; j <= k; j += blockDim.x) col[j] = R1[j + (int64_t)k * ld1];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc = 0.0;
    if (i <= k)
      for (int j = i; j <= k; ++j) acc = fma(R2[i + (int64_t)j * ld2], col[j], acc);
    R[i + (int64_t)k * ldr] = acc;
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
  allow_dynamic_lds(reinterpret_cast<const void*>(&trmm_kernel), (size_t)n * 8);
  hipLaunchKernelGGL(trmm_kernel, dim3(n), dim3(n < 256 ? ((n + 63) / 64) * 64 : 256), (size_t)n * 8, st, R2, ld2,
                     R1, ld1, n, R, ldr, ctrl, phase);
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
