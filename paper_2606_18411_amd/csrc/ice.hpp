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

// One ICE update (s, c, est_new) from est, alpha = w^T x and gamma, written
// without branches so that the sigma_max and sigma_min updates of a step
// run interleaved.
__device__ __forceinline__ void ice_step(double est, double alpha, double gamma, bool largest,
                                         double& s, double& c, double& est_new) {
  const double rho = fmax(fmax(est, fabs(alpha)), fabs(gamma));
  // rho is scaled by a power of two so the scaling is exact
  int erho;
  (void)frexp(rho, &erho);
  const double e = ldexp(est, -erho), a = ldexp(alpha, -erho), g = ldexp(gamma, -erho);
  const double A = fma(e, e, a * a), B = a * g, C = g * g;
  const double hd = 0.5 * (A - C);
  const double lmax = 0.5 * (A + C) + sqrt_nr(fma(hd, hd, B * B));
  const double eg = e * g;
  const double lam = largest ? lmax : (eg * eg) * rcp_nr(lmax > 0.0 ? lmax : 1.0);
  const double v1a = lam - C, v2b = lam - A;
  const double n1 = fma(v1a, v1a, B * B), n2 = fma(v2b, v2b, B * B);
  const bool first = n1 >= n2;
  const double va = first ? v1a : B, vb = first ? B : v2b, nn = first ? n1 : n2;
  const bool deg = !(nn > 0.0);
  const double r = rsqrt_nr(deg ? 1.0 : nn);
  s = deg ? (largest ? 0.0 : 1.0) : va * r;
  c = deg ? (largest ? 1.0 : 0.0) : vb * r;
  est_new = ldexp(sqrt_nr(fmax(lam, 0.0)), erho);
  if (rho == 0.0) { s = 1.0; c = 0.0; est_new = 0.0; }
}

// ICE estimate of sigma_max (LARGEST) or sigma_min of R (element (i, j) at
// R[i*si + j*sj]) by one full wave; n <= 64 * XPL. Returns NaN when R holds
// a non-finite value. Right-looking form of alpha_j = R[0:j, j]^T x: lane l
// keeps beta_k = R[0:j, k]^T x for its columns k = l + 64 q, and the step
// that turns x into [s x; c] updates beta_k <- s beta_k + c R[j, k].
// alpha_j is then read from the lane holding column j, so no reduction sits
// on the serial chain; rows of R are read contiguously when si = ld, sj = 1.
template <int XPL, bool LARGEST>
__device__ double ice_est_wave(const double* R, int n, int si, int sj) {
  const int l = threadIdx.x & 63;
  double b[XPL];
#pragma unroll
  for (int q = 0; q < XPL; ++q) {
    const int k = l + 64 * q;
    b[q] = (k < n) ? R[k * sj] : 0.0;  // x = [1]: beta_k = R[0, k]
  }
  double est = fabs(R[0]);
  bool bad = !isfinite(est);
  for (int j = 1; j < n; ++j) {
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
    ice_step(est, alpha, gma, LARGEST, sn, cs, est);
#pragma unroll
    for (int q = 0; q < XPL; ++q) b[q] = fma(sn, b[q], cs * row[q]);
  }
  return bad ? __builtin_nan("") : est;
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

}  // namespace mrcqr
