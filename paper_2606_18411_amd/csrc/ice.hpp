// Incremental condition estimation (C. Bischof, "Incremental condition
// estimation", SIAM J. Matrix Anal. Appl. 11(2), 1990) of an upper-
// triangular n x n matrix, used for the sketch-precision regime (Section
// "Adaptive Precision Selection") and for the posterior check on Rc.
//
// With L = R^T and a unit x such that ||L_j x|| = est_j, appending row
// [w^T, gamma] of L and taking [s x; c] gives ||.||^2 = [s c] M [s c]^T,
// M = [[est^2 + alpha^2, alpha gamma], [alpha gamma, gamma^2]],
// alpha = w^T x. The new estimate is the square root of M's largest (for
// sigma_max) or smallest (sigma_min) eigenvalue, (s, c) its eigenvector.
// M is scaled by 2^(-2E) with 2^E the power of two just above
// rho = max(est, |alpha|, |gamma|) (exact scaling); the smallest eigenvalue
// is det(M) / lam_max = (est gamma)^2 / lam_max.
#pragma once
#include "common.hpp"

namespace mrcqr {

// Reciprocal, reciprocal square root and square root refined from the
// hardware estimates by Newton steps (two for the reciprocal and the
// reciprocal square root, one more residual correction for the square
// root): a few units in the last place, with a third of the latency of the
// correctly rounded library sequences. Arguments are finite; x > 0
// (rsqrt_nr), x >= 0 (sqrt_nr).
__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  double e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  e = fma(-d, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double xh = -0.5 * x;
  double r = fma(xh * y, y, 0.5);
  y = fma(y, r, y);
  r = fma(xh * y, y, 0.5);
  return fma(y, r, y);
}
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = rsqrt_nr(x);
  double q = x * y;
  q = fma(fma(-q, q, x), 0.5 * y, q);
  return x > 0.0 ? q : 0.0;
}

// Reciprocal and reciprocal square root with one Newton step from the
// hardware estimates, for the condition estimate only (a loose quantity:
// the step doubles the estimate's correct bits, which is ample here).
__device__ __forceinline__ double rcp1(double d) {
  const double y = __builtin_amdgcn_rcp(d);
  return fma(y, fma(-d, y, 1.0), y);
}
__device__ __forceinline__ double rsqrt1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}

// One ICE update. The estimate is kept as est = sqrt(es2) 2^F (es2 < 4),
// so that no square root sits on its chain and no square overflows: with
// 2^E >= rho = max(est, |alpha|, |gamma|) (E from exponents only; exact
// power-of-two scaling) M = [[e^2 + a^2, a g], [a g, g^2]] for the scaled
// values, lam_max from the closed form, lam_min = (e g)^2 / lam_max, (s, c)
// the unit eigenvector of the chosen eigenvalue, and the new estimate is
// sqrt(lam) 2^E. Branch-free so that the sigma_max and sigma_min updates
// run interleaved.
__device__ __forceinline__ void ice_step(double& es2, int& F, double alpha, double gamma, bool largest,
                                         double& s, double& c) {
  int ke, ka, kg;
  (void)frexp(es2, &ke);
  (void)frexp(alpha, &ka);
  (void)frexp(gamma, &kg);
  const int E = max(max(F + ((ke + 1) >> 1), ka), kg);
  const double e2s = ldexp(es2, 2 * (F - E)), a = ldexp(alpha, -E), g = ldexp(gamma, -E);
  const double A = fma(a, a, e2s), B = a * g, C = g * g;
  const double hd = 0.5 * (A - C);
  const double disc = fma(hd, hd, B * B);
  const double lmax = 0.5 * (A + C) + (disc > 0.0 ? disc * rsqrt1(disc) : 0.0);
  const double lam = largest ? lmax : (e2s * C) * rcp1(lmax > 0.0 ? lmax : 1.0);
  const double v1a = lam - C, v2b = lam - A;
  const double n1 = fma(v1a, v1a, B * B), n2 = fma(v2b, v2b, B * B);
  const bool first = n1 >= n2;
  const double va = first ? v1a : B, vb = first ? B : v2b, nn = first ? n1 : n2;
  const bool deg = !(nn > 0.0);
  const double r = rsqrt1(deg ? 1.0 : nn);
  s = deg ? (largest ? 0.0 : 1.0) : va * r;
  c = deg ? (largest ? 1.0 : 0.0) : vb * r;
  const bool zero = es2 == 0.0 && alpha == 0.0 && gamma == 0.0;
  if (zero) { s = 1.0; c = 0.0; }
  es2 = zero ? 0.0 : fmax(lam, 0.0);
  F = zero ? F : E;
}

// ICE of sigma_max (largest) or sigma_min of R (element (i, j) at
// R[i*si + j*sj], n <= 64 * XPL) by one full wave, row by row: start()
// takes row 0, step(j) row j (rows in order), estimate() the result (NaN
// when R holds a non-finite value). Right-looking form of
// alpha_j = R[0:j, j]^T x: lane l keeps beta_k = R[0:j, k]^T x for its
// columns k = l + 64 q, and the step that turns x into [s x; c] updates
// beta_k <- s beta_k + c R[j, k]. alpha_j is read from the lane holding
// column j, so no reduction sits on the serial chain; rows of R are read
// contiguously when si = ld, sj = 1. A caller may interleave the steps with
// other work, once the rows they read are final.
template <int XPL>
struct IceWave {
  double b[XPL];
  double es2;
  int F;
  bool bad, largest;

  __device__ void start(const double* R, int n, int sj, bool lg) {
    largest = lg;
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < XPL; ++q) {
      const int k = l + 64 * q;
      b[q] = (k < n) ? R[k * sj] : 0.0;  // x = [1]: beta_k = R[0, k]
    }
    const double r00 = R[0];
    const double m00 = frexp(r00, &F);  // |r00| = |m00| 2^F
    es2 = m00 * m00;
    bad = !isfinite(r00);
  }
  __device__ void step(const double* R, int n, int si, int sj, int j) {
    const int l = threadIdx.x & 63;
    double row[XPL];
#pragma unroll
    for (int q = 0; q < XPL; ++q) {
      const int k = l + 64 * q;
      row[q] = (k > j && k < n) ? R[j * si + k * sj] : 0.0;
    }
    const double gma = R[j * si + j * sj];
    const int jq = j >> 6;
    double v = b[0];
#pragma unroll
    for (int q = 1; q < XPL; ++q)
      if (q == jq) v = b[q];
    const double alpha = readlane_t(v, j & 63);
    bad |= !isfinite(gma) || !isfinite(alpha);
    double sn, cs;
    ice_step(es2, F, alpha, gma, largest, sn, cs);
#pragma unroll
    for (int q = 0; q < XPL; ++q) b[q] = fma(sn, b[q], cs * row[q]);
  }
  __device__ double estimate() const { return bad ? __builtin_nan("") : ldexp(sqrt(es2), F); }
};

template <int XPL, bool LARGEST>
__device__ double ice_est_wave(const double* R, int n, int si, int sj) {
  IceWave<XPL> ice;
  ice.start(R, n, sj, LARGEST);
  for (int j = 1; j < n; ++j) ice.step(R, n, si, sj, j);
  return ice.estimate();
}

// kappa estimate est_max / est_min of R: sigma_max on wave 0 and sigma_min
// on wave 1 of the block (blockDim.x >= 128), run only when RUN; every
// thread of the block calls it and receives the result (NaN when not RUN,
// +inf for a singular or non-finite R).
__device__ double ice_kappa_block(const double* R, int n, int si, int sj, bool run) {
  __shared__ double ice_res[2];
  const int w = threadIdx.x >> 6;
  if (run && w < 2) {
    double est;
    if (n <= 64) est = (w == 0) ? ice_est_wave<1, true>(R, n, si, sj) : ice_est_wave<1, false>(R, n, si, sj);
    else est = (w == 0) ? ice_est_wave<2, true>(R, n, si, sj) : ice_est_wave<2, false>(R, n, si, sj);
    if ((threadIdx.x & 63) == 0) ice_res[w] = est;
  }
  __syncthreads();
  if (!run) return __builtin_nan("");
  const double eM = ice_res[0], em = ice_res[1];
  if (!isfinite(eM) || !isfinite(em) || !(em > 0.0)) return __builtin_inf();
  return eM / em;
}

// ICE for n <= 512 on a row-major copy Rt of R (row j at Rt + j n, so a
// wave reads each row contiguously), with the rows read DEPTH steps ahead
// of the serial chain; the kernels of the column-panel path for n > 128
// call it, so that the register budget of the n <= 128 kernels stays as
// it is.
template <int XPL, bool LARGEST>
__device__ double ice_est_rows(const double* __restrict__ Rt, int n) {
  constexpr int DEPTH = 4;
  const int l = threadIdx.x & 63;
  IceWave<XPL> ice;
  ice.start(Rt, n, 1, LARGEST);
  double ring[DEPTH][XPL], gring[DEPTH];
  auto load = [&](int j, int slot) {
#pragma unroll
    for (int q = 0; q < XPL; ++q) {
      const int k = l + 64 * q;
      const bool in = j < n && k > j && k < n;
      ring[slot][q] = load_or_zero(Rt + (in ? (int64_t)j * n + k : 0), in);
    }
    gring[slot] = load_or_zero(Rt + (j < n ? (int64_t)j * n + j : 0), j < n);
  };
  // consume row j from slot d, then refill the slot with row j + DEPTH (the
  // refill is issued once the slot's values are dead, so that it lands in
  // the same registers and nothing is moved at the loop's back edge)
  auto step = [&](int j, int d) {
    const double* row = ring[d];
    const double gma = gring[d];
    const int jq = j >> 6;
    double v = ice.b[0];
#pragma unroll
    for (int q = 1; q < XPL; ++q)
      if (q == jq) v = ice.b[q];
    const double alpha = readlane_t(v, j & 63);
    ice.bad |= !isfinite(gma) || !isfinite(alpha);
    double sn, cs;
    ice_step(ice.es2, ice.F, alpha, gma, LARGEST, sn, cs);
#pragma unroll
    for (int q = 0; q < XPL; ++q) ice.b[q] = fma(sn, ice.b[q], cs * row[q]);
    load(j + DEPTH, d);
  };
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) load(1 + d, d);
  // whole groups of DEPTH rows without branches (the loads stay in flight
  // across iterations), then the remaining rows
  int j0 = 1;
  for (; j0 + DEPTH <= n; j0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) step(j0 + d, d);
  }
#pragma unroll
  for (int d = 0; d < DEPTH; ++d)
    if (j0 + d < n) step(j0 + d, d);
  return ice.estimate();
}

// kappa estimate est_max / est_min of R (n <= 512) from its row-major copy
// Rt: sigma_max on wave 0 and sigma_min on wave 1 (blockDim.x >= 128), run
// only when RUN; every thread of the block calls it and receives the
// result (NaN when not RUN, +inf for a singular or non-finite R).
__device__ double ice_kappa_rows(const double* __restrict__ Rt, int n, bool run) {
  __shared__ double ice_res_w[2];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (run && w < 2) {
    double est;
    if (n <= 256) est = (w == 0) ? ice_est_rows<4, true>(Rt, n) : ice_est_rows<4, false>(Rt, n);
    else est = (w == 0) ? ice_est_rows<8, true>(Rt, n) : ice_est_rows<8, false>(Rt, n);
    if ((threadIdx.x & 63) == 0) ice_res_w[w] = est;
  }
  __syncthreads();
  if (!run) return __builtin_nan("");
  const double eM = ice_res_w[0], em = ice_res_w[1];
  if (!isfinite(eM) || !isfinite(em) || !(em > 0.0)) return __builtin_inf();
  return eM / em;
}

}  // namespace mrcqr
