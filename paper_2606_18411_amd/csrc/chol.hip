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

// Right-looking Cholesky of the upper triangle of G, held row-major in LDS.
// Step j keeps row j unscaled and updates the trailing triangle with
// L[i][k] -= L[j][i] * L[j][k] / piv_j (one barrier per step); the rows are
// scaled by 1/sqrt(piv) at the end, which gives the textbook
// R[j][k] = (G[j][k] - sum_i R[i][j] R[i][k]) / R[j][j].
__global__ __launch_bounds__(CH_THREADS) void chol_kernel(
    const double* __restrict__ G, int n, int64_t ldg, double* __restrict__ Rc, int64_t ldr,
    int32_t* __restrict__ fail_out, double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double* L = reinterpret_cast<double*>(smem);
  const int ld = n + 1;
  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;   // ty is wave-uniform
  constexpr int TY = CH_THREADS / 64;
  for (int k = tx; k < n; k += 64)
    for (int i = ty; i < n; i += TY) L[i * ld + k] = (i <= k) ? G[i + (int64_t)k * ldg] : 0.0;
  __syncthreads();
  int f = -1;
  for (int j = 0; j < n; ++j) {
    const double piv = L[j * ld + j];
    if (!(piv > 0.0) || !isfinite(piv)) { f = j; break; }
    const double inv = 1.0 / piv;
    for (int k = j + 1 + tx; k < n; k += 64) {
      const double ljk = L[j * ld + k] * inv;
      for (int i = j + 1 + ty; i <= k; i += TY) L[i * ld + k] = fma(-L[j * ld + i], ljk, L[i * ld + k]);
    }
    __syncthreads();
  }
  // scale rows: R[j][k] = L[j][k] / sqrt(L[j][j])
  const int nrows = (f < 0) ? n : f;
  for (int i = ty; i < nrows; i += TY) {
    const double rinv = 1.0 / sqrt(L[i * ld + i]);
    for (int k = i + tx; k < n; k += 64) L[i * ld + k] = (k == i) ? sqrt(L[i * ld + i]) : L[i * ld + k] * rinv;
  }
  __syncthreads();
  for (int k = tx; k < n; k += 64)
    for (int i = ty; i < n; i += TY) Rc[i + (int64_t)k * ldr] = (f < 0 && i <= k) ? L[i * ld + k] : 0.0;
  if (tid < 64) {
    double kappa = __builtin_inf();
    if (f < 0) kappa = ice_kappa(L, n, ld, 1);
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

// R = R2 R1 (upper x upper), one thread per entry, summed in index order.
__global__ void trmm_kernel(const double* __restrict__ R2, int64_t ld2, const double* __restrict__ R1,
                            int64_t ld1, int n, double* __restrict__ R, int64_t ldr,
                            const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = idx % n, k = idx / n;
  double acc = 0.0;
  if (i <= k)
    for (int j = i; j <= k; ++j) acc = fma(R2[i + (int64_t)j * ld2], R1[j + (int64_t)k * ld1], acc);
  R[i + (int64_t)k * ldr] = acc;
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

size_t chol_smem_bytes(int n) { return (size_t)n * (n + 1) * 8 + 64; }

hipError_t launch_cholesky(const double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                           double* kappa, Ctrl* ctrl, int phase, hipStream_t st) {
  allow_dynamic_lds(reinterpret_cast<const void*>(&chol_kernel), chol_smem_bytes(n));
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(CH_THREADS), chol_smem_bytes(n), st, G, n, ldg, Rc, ldr,
                     fail, kappa, ctrl, phase);
  return hipGetLastError();
}

hipError_t launch_trmm(const double* R2, int64_t ld2, const double* R1, int64_t ld1, int n, double* R,
                       int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st) {
  const int tot = n * n;
  hipLaunchKernelGGL(trmm_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, R2, ld2, R1, ld1, n, R, ldr,
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
