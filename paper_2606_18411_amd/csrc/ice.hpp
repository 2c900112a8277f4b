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

__device__ __forceinline__ void ice_step(double est, double alpha, double gamma, bool largest,
                                         double& s, double& c, double& est_new) {
  const double rho = fmax(fmax(est, fabs(alpha)), fabs(gamma));
  if (rho == 0.0) { s = 1.0; c = 0.0; est_new = 0.0; return; }
  // rho is scaled by a power of two so the division by it is exact
  int erho;
  (void)frexp(rho, &erho);
  const double e = ldexp(est, -erho), a = ldexp(alpha, -erho), g = ldexp(gamma, -erho);
  const double scale = ldexp(1.0, erho);
  const double A = e * e + a * a, B = a * g, C = g * g;
  const double hd = 0.5 * (A - C);
  const double lmax = 0.5 * (A + C) + sqrt(hd * hd + B * B);
  const double lam = largest ? lmax : (lmax > 0.0 ? (e * g) * (e * g) / lmax : 0.0);
  const double v1a = lam - C, v1b = B, v2a = B, v2b = lam - A;
  const double n1 = v1a * v1a + v1b * v1b, n2 = v2a * v2a + v2b * v2b;
  if (n1 == 0.0 && n2 == 0.0) { s = largest ? 0.0 : 1.0; c = largest ? 1.0 : 0.0; }
  else if (n1 >= n2) { const double r = 1.0 / sqrt(n1); s = v1a * r; c = v1b * r; }
  else { const double r = 1.0 / sqrt(n2); s = v2a * r; c = v2b * r; }
  est_new = sqrt(fmax(lam, 0.0)) * scale;
}


// kappa estimate est_max / est_min of R (element (i, j) at R[i*si + j*sj]),
// executed by one full wave; n <= 64 * XPL. Returns +inf for a singular or
// non-finite R.
template <int XPL>
__device__ double ice_kappa_wave(const double* R, int n, int si, int sj) {
  const int l = threadIdx.x & 63;
  double xM[XPL], xm[XPL];
#pragma unroll
  for (int q = 0; q < XPL; ++q) { xM[q] = (l + 64 * q == 0) ? 1.0 : 0.0; xm[q] = xM[q]; }
  double estM = fabs(R[0]), estm = estM;
  for (int j = 1; j < n; ++j) {
    double aM = 0.0, am = 0.0;
#pragma unroll
    for (int q = 0; q < XPL; ++q) {
      const int i = l + 64 * q;
      if (i < j) { const double r = R[i * si + j * sj]; aM += r * xM[q]; am += r * xm[q]; }
    }
    aM = wave_sum_dpp(aM);
    am = wave_sum_dpp(am);
    const double gma = R[j * si + j * sj];
    double sM, cM, sm, cm;
    ice_step(estM, aM, gma, true, sM, cM, estM);
    ice_step(estm, am, gma, false, sm, cm, estm);
#pragma unroll
    for (int q = 0; q < XPL; ++q) {
      const int i = l + 64 * q;
      xM[q] = (i == j) ? cM : xM[q] * sM;
      xm[q] = (i == j) ? cm : xm[q] * sm;
    }
  }
  if (!isfinite(estM) || !isfinite(estm) || !(estm > 0.0)) return __builtin_inf();
  return estM / estm;
}

__device__ __forceinline__ double ice_kappa(const double* R, int n, int si, int sj) {
  return (n <= 64) ? ice_kappa_wave<1>(R, n, si, sj) : ice_kappa_wave<2>(R, n, si, sj);
}

}  // namespace mrcqr
