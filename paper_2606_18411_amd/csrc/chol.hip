// Algorithm 1, second step: Cholesky factorization G = Rc^T Rc (float64),
// with breakdown detection (a pivot that is not positive or not finite,
// the failure mode the paper describes for Cholesky-QR), the ICE part of the
// posterior condition estimate of Rc = the condition number of A Rs^{-1}
// (Section "Adaptive Precision Selection": an underestimated precision shows
// up as lost orthogonality; the decision is taken in posterior.hip), Stage
// 3's product R = Rc Rs, and the small per-call control kernels.
#include "batch.hpp"
#include "ice.hpp"
#include "small.hpp"

namespace mrcqr {

constexpr int CH_THREADS = 512;
constexpr int CH_NMAX = 128;

// Blocked right-looking Cholesky of the upper triangle of G (n <= 128),
// 16-column blocks, all of it in LDS (row-major, stride 129). Block step K:
//   A. wave 0 factors the 16 x 16 diagonal block: lane c holds column c of
//      the block, and step j forms r_jj = sqrt(pivot), scales row j and
//      takes r_ji r_jc off every entry (i, c), j < i <= c (r_ji read from
//      lane i);
//   B. the row panel R[K, >K] = R_KK^{-T} G[K, >K], one thread per column
//      (forward substitution);
//   C. the trailing upper tiles lose R[K, I]^T R[K, J] (float64 MFMA
//      16x16x4, 16 waves).
// Each entry ends as the textbook R[j][k] = (G[j][k] - sum_{i<j} R[i][j]
// R[i][k]) / R[j][j], summed in another order. A pivot that is not
// positive and finite stops the factorization (its index is reported).
__device__ __forceinline__ void chol_body(
    const double* __restrict__ G, int n, int64_t ldg, double* __restrict__ Rc, int64_t ldr,
    int32_t* __restrict__ fail_out, double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  constexpr int LDR = CH_NMAX + 1;
  __shared__ double Rl[CH_NMAX * LDR];  // row-major
  __shared__ double dinv[16];           // 1 / r_jj of the current diagonal block
  __shared__ int fail_sh;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  // upper triangle of G, zero elsewhere (coalesced over the rows of a
  // column; all of a thread's loads in flight together)
  {
    constexpr int PER = CH_NMAX * CH_NMAX / CH_THREADS;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * CH_THREADS, i = e % CH_NMAX, j = e / CH_NMAX;
      v[u] = (i <= j && j < n) ? G[i + (int64_t)j * ldg] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * CH_THREADS, i = e % CH_NMAX, j = e / CH_NMAX;
      Rl[i * LDR + j] = v[u];
    }
  }
  if (tid == 0) fail_sh = -1;
  __syncthreads();
  // The condition estimate of Rc runs on the last two waves (sigma_max,
  // sigma_min), row by row as the rows become final: the rows of block
  // K - 1 during phases A and B of block step K, the last block's at the
  // end. Those waves take no part in phase C.
  constexpr int NW = CH_THREADS / 64;
  const bool ice_wave = w >= NW - 2;
  IceWave<2> ice;
  int ice_row = 0;  // next row of R for the estimate
  auto ice_rows = [&](int upto) {
    for (; ice_row < upto; ++ice_row) {
      if (ice_row == 0) ice.start(Rl, n, 1, w == NW - 2);
      else ice.step(Rl, n, LDR, 1, ice_row);
    }
  };
  const int nb = (n + 15) / 16;
  for (int K = 0; K < nb; ++K) {
    const int k0 = 16 * K, kb = min(16, n - k0);
    if (ice_wave && K > 0) ice_rows(k0 - 5);
    if (w == 0) {
      const int c = c16;
      double col[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) col[i] = Rl[(k0 + i) * LDR + k0 + c];
      int f = -1;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        // (wave-uniform conditions; no early exit, so the loops unroll)
        const double piv = readlane_t(col[j], j);
        if (j < kb && f < 0 && (!(piv > 0.0) || !isfinite(piv))) f = k0 + j;
        if (j < kb && f < 0) {
          const double inv = rsqrt_nr(piv), r = piv * inv;
          col[j] = (c == j) ? r : col[j] * inv;
          if (l == 0) dinv[j] = inv;
#pragma unroll
          for (int i = j + 1; i < 16; ++i) {
            const double rji = readlane_t(col[j], i);
            col[i] = fma(-rji, col[j], col[i]);
          }
        }
      }
      if (l < kb) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i <= c) Rl[(k0 + i) * LDR + k0 + c] = col[i];
      }
      if (l == 0 && f >= 0) fail_sh = f;
    }
    __syncthreads();
    if (fail_sh >= 0) break;
    const int cb = k0 + kb;  // first column right of the block
    if (cb >= n) break;
    if (ice_wave && K > 0) ice_rows(k0);
    for (int c = cb + tid; c < n; c += CH_THREADS) {
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = Rl[(k0 + i) * LDR + c];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        x[i] *= dinv[i];
#pragma unroll
        for (int k = i + 1; k < 16; ++k) x[k] = fma(-Rl[(k0 + i) * LDR + k0 + k], x[i], x[k]);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Rl[(k0 + i) * LDR + c] = x[i];
    }
    __syncthreads();
    // trailing tiles (I, J), K < I <= J < nb, numbered row by row
    const int nt = nb - K - 1;
    for (int t = w; t < nt * (nt + 1) / 2 && !ice_wave; t += NW - 2) {
      int a = 0, rem = t;
      while (rem >= nt - a) { rem -= nt - a; ++a; }
      const int I = K + 1 + a, J = I + rem;
      f64x4 acc = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double* rk = Rl + (k0 + 4 * s + g) * LDR;
        acc = mfma_f64(rk[16 * I + c16], rk[16 * J + c16], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Rl[(16 * I + 4 * r + g) * LDR + 16 * J + c16] -= acc[r];
    }
    __syncthreads();
  }
  // Rc leaves from the other waves while the estimate takes the last rows
  const int f = fail_sh;
  __shared__ double ice_res[2];
  if (ice_wave) {
    if (f < 0) {
      ice_rows(n);
      if (l == 0) ice_res[w - (NW - 2)] = ice.estimate();
    }
  } else {
    for (int e = tid; e < n * n; e += CH_THREADS - 128) {
      const int i = e % n, k = e / n;
      Rc[i + (int64_t)k * ldr] = (f < 0 && i <= k) ? Rl[i * LDR + k] : 0.0;
    }
  }
  __syncthreads();
  {
    double kappa = __builtin_inf();
    if (f < 0) {
      const double eM = ice_res[0], em = ice_res[1];
      kappa = (!isfinite(eM) || !isfinite(em) || !(em > 0.0)) ? __builtin_inf() : eM / em;
    }
    if (tid == 0) {
      if (fail_out) *fail_out = f;
      if (kappa_out) *kappa_out = kappa;
      // the posterior kernel combines this estimate with power steps and
      // takes the rerun decision once Rc^{-1} is formed
      if (ctrl) {
        ctrl->kappa_rc = kappa;
        ctrl->pass_fail = f;
      }
    }
  }
}

__global__ __launch_bounds__(CH_THREADS) void chol_kernel(
    const double* __restrict__ G, int n, int64_t ldg, double* __restrict__ Rc, int64_t ldr,
    int32_t* __restrict__ fail_out, double* __restrict__ kappa_out, Ctrl* __restrict__ ctrl, int phase) {
  chol_body(G, n, ldg, Rc, ldr, fail_out, kappa_out, ctrl, phase);
}

// Grouped: one workgroup per member.
__global__ __launch_bounds__(CH_THREADS) void chol_grouped(const BatchInst* __restrict__ bi,
                                                           const int32_t* __restrict__ members, BatchCall call,
                                                           int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  chol_body(bat_ptr<const double>(call, d, d.off_G), d.n, d.n, bat_ptr<double>(call, d, d.off_Rc), d.n, nullptr,
            nullptr, bat_ptr<Ctrl>(call, d, d.off_ctrl), phase);
}

// Stage 3, stand-alone: R = R2 R1 (see trmm_tile).
__global__ __launch_bounds__(64) void trmm_kernel(const double* __restrict__ R2, int64_t ld2,
                                                  const double* __restrict__ R1, int64_t ld1, int n,
                                                  double* __restrict__ R, int64_t ldr,
                                                  const Ctrl* __restrict__ ctrl, int phase) {
  __shared__ __attribute__((aligned(16))) double lds[TRMM_LDS_DOUBLES];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  trmm_tile(R2, ld2, R1, ld1, n, R, ldr, blockIdx.x, blockIdx.y, lds);
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



__global__ void ctrl_finalize_grouped(const BatchInst* __restrict__ bi, const int32_t* __restrict__ members,
                                      BatchCall call) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if (threadIdx.x == 0 && call.info) {
    const Ctrl* ctrl = bat_ptr<const Ctrl>(call, d, d.off_ctrl);
    InfoOut* info = reinterpret_cast<InfoOut*>(call.info) + i;
    info->status = ctrl->status;
    info->precision_used = ctrl->cur_prec;
    info->chol_fail_index = ctrl->chol_fail;
    info->escalations = ctrl->escalations;
    info->kappa_rs_est = ctrl->kappa_rs;
    info->kappa_rc_est = ctrl->kappa_rc;
  }
}

// Outcome of CholQR2 (two Cholesky factorizations, fail[0] and fail[1]):
// breakdown of the first pass, else of the second (its index is a pivot of
// the Gram matrix of Q1), else ok.
__global__ void cholqr2_finalize_kernel(const int32_t* __restrict__ fail, InfoOut* __restrict__ info) {
  if (threadIdx.x == 0) {
    const int f = fail[0] >= 0 ? fail[0] : fail[1];
    info->status = f >= 0 ? ST_CHOL : ST_OK;
    info->precision_used = P_FP64;
    info->chol_fail_index = f;
    info->escalations = 0;
    info->kappa_rs_est = __builtin_nan("");
    info->kappa_rc_est = __builtin_nan("");
  }
}

hipError_t launch_cholqr2_finalize(const int32_t* fail, void* info, hipStream_t st) {
  hipLaunchKernelGGL(cholqr2_finalize_kernel, dim3(1), dim3(64), 0, st, fail, (InfoOut*)info);
  return hipGetLastError();
}

hipError_t launch_cholesky_grouped(const BatchInst* bi, const int32_t* members, int count, const BatchCall& call,
                                   int phase, hipStream_t st) {
  hipLaunchKernelGGL(chol_grouped, dim3(1, count), dim3(CH_THREADS), 0, st, bi, members, call, phase);
  return hipGetLastError();
}

hipError_t launch_finalize_grouped(const BatchInst* bi, const int32_t* members, int count, const BatchCall& call,
                                   hipStream_t st) {
  hipLaunchKernelGGL(ctrl_finalize_grouped, dim3(1, count), dim3(64), 0, st, bi, members, call);
  return hipGetLastError();
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

hipError_t launch_ctrl_finalize(const Ctrl* ctrl, void* info, hipStream_t st) {
  hipLaunchKernelGGL(ctrl_finalize_kernel, dim3(1), dim3(64), 0, st, ctrl, (InfoOut*)info);
  return hipGetLastError();
}

}  // namespace mrcqr
