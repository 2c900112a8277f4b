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
constexpr int TRMM_NMAX = 128;

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
__global__ __launch_bounds__(CH_THREADS) void chol_kernel(
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
