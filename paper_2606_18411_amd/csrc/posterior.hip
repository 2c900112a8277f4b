// Posterior check of the adaptive precision policy (Section "Adaptive
// Precision Selection": a precision chosen too low shows up as lost
// orthogonality, and the factorization is rerun at the next higher level).
// Cholesky-QR loses orthogonality like kappa(Rc)^2 u, with Rc the Cholesky
// factor of the preconditioned B = A Rs^{-1}, so the check bounds an
// estimate of kappa_2(Rc) by TAU_POSTERIOR.
//
// The estimate is the larger of two lower bounds of kappa_2(Rc): the ICE
// estimate the Cholesky kernel leaves in the control block, and
// sigma_max(Rc) sigma_max(X) from POSTERIOR_STEPS power steps (Golub and
// Van Loan, Section 8.2) on Rc^T Rc and X^T X, X = Rc^{-1} (formed for Q
// anyway), both started from the normalized all-ones vector. ICE alone can
// underestimate kappa(Rc) several-fold on these well-conditioned factors.
//
// One workgroup of 1024 threads holds both matrices in registers: thread t
// owns the 4 x 4 block at rows 4 (t / 32), columns 4 (t % 32) of each.
// y = M x sums over the 32 threads of a row block (one half-wave, DPP);
// z = M^T y sums over the 32 row blocks through LDS in a fixed order.
#include "batch.hpp"

namespace mrcqr {

constexpr int PO_THREADS = 1024;
constexpr int PO_NMAX = 128;

__device__ __forceinline__ void posterior_body(const double* __restrict__ Rc, const double* __restrict__ X, int n,
                                               int64_t ld, Ctrl* __restrict__ ctrl, int phase,
                                               double* __restrict__ kappa_out) {
  __shared__ double part[2][32][PO_NMAX];
  __shared__ double xs[2][PO_NMAX];
  __shared__ double red[2][16];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int rb = t >> 5, cb = t & 31;
  const bool broken = ctrl != nullptr && ctrl->pass_fail >= 0;
  double est[2] = {__builtin_inf(), __builtin_inf()};
  if (!broken) {
    double M[2][4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = 4 * rb + a, j = 4 * cb + b;
        const bool in = i < n && j < n && i <= j;
        const int64_t o = in ? i + (int64_t)j * ld : 0;
        M[0][a][b] = in ? Rc[o] : 0.0;
        M[1][a][b] = in ? X[o] : 0.0;
      }
    if (t < 2 * PO_NMAX) {
      const int col = t & (PO_NMAX - 1);
      xs[t >> 7][col] = col < n ? 1.0 / sqrt((double)n) : 0.0;
    }
    __syncthreads();
    double y[2][4];
    for (int it = 0;; ++it) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        double xv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) xv[b] = xs[k][4 * cb + b];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          double v = 0.0;
#pragma unroll
          for (int b = 0; b < 4; ++b) v = fma(M[k][a][b], xv[b], v);
          y[k][a] = group_sum_dpp(v, 32);
        }
      }
      if (it == POSTERIOR_STEPS) break;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          double v = 0.0;
#pragma unroll
          for (int a = 0; a < 4; ++a) v = fma(M[k][a][b], y[k][a], v);
          part[k][rb][4 * cb + b] = v;
        }
      __syncthreads();
      double z = 0.0;
      if (t < 2 * PO_NMAX) {
        const int k = t >> 7, col = t & (PO_NMAX - 1);
        for (int r = 0; r < 32; ++r) z += part[k][r][col];
        const double s2 = wave_sum_dpp(z * z);
        if (l == 0) red[k][w & 1] = s2;
      }
      __syncthreads();
      if (t < 2 * PO_NMAX) {
        const int k = t >> 7, col = t & (PO_NMAX - 1);
        const double nz = sqrt(red[k][0] + red[k][1]);
        xs[k][col] = z / nz;
      }
      __syncthreads();
    }
    // ||M x|| of the last iterate: row block rb's y sits in its 32 threads;
    // lanes 0 and 32 of each wave carry the wave's two row blocks
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double q = ((y[k][0] * y[k][0] + y[k][1] * y[k][1]) + (y[k][2] * y[k][2] + y[k][3] * y[k][3]));
      const double s = readlane_t(q, 0) + readlane_t(q, 32);
      if (l == 0) red[k][w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      double s = 0.0;
      for (int i = 0; i < PO_THREADS / 64; ++i) s += red[k][i];
      est[k] = sqrt(s);
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
    // rerun one precision higher; the next pass is enabled on the device
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

__global__ __launch_bounds__(PO_THREADS) void posterior_kernel(const double* __restrict__ Rc,
                                                              const double* __restrict__ X, int n, int64_t ld,
                                                              Ctrl* __restrict__ ctrl, int phase,
                                                              double* __restrict__ kappa_out) {
  posterior_body(Rc, X, n, ld, ctrl, phase, kappa_out);
}

// Grouped: one workgroup per member.
__global__ __launch_bounds__(PO_THREADS) void posterior_grouped(const BatchInst* __restrict__ bi,
                                                               const int32_t* __restrict__ members, BatchCall call,
                                                               int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  posterior_body(bat_ptr<const double>(call, d, d.off_Rc), bat_ptr<const double>(call, d, d.off_Rci), d.n, d.n,
                 bat_ptr<Ctrl>(call, d, d.off_ctrl), phase, nullptr);
}

hipError_t launch_posterior(const double* Rc, const double* X, int n, int64_t ld, Ctrl* ctrl, int phase,
                            double* kappa_out, hipStream_t st) {
  if (n > PO_NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(posterior_kernel, dim3(1), dim3(PO_THREADS), 0, st, Rc, X, n, ld, ctrl, phase, kappa_out);
  return hipGetLastError();
}

hipError_t launch_posterior_grouped(const BatchInst* bi, const int32_t* members, int count, const BatchCall& call,
                                    int phase, hipStream_t st) {
  hipLaunchKernelGGL(posterior_grouped, dim3(1, count), dim3(PO_THREADS), 0, st, bi, members, call, phase);
  return hipGetLastError();
}

}  // namespace mrcqr
