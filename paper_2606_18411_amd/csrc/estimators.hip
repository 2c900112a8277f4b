// The two other condition estimators of Section "Adaptive Precision
// Selection", next to the ICE estimate the adaptive policy uses:
//   * the block 1-norm estimator (Higham and Tisseur, SIAM J. Matrix Anal.
//     Appl. 21, 2000, Algorithm 2.4, with t = 2 columns and at most 5
//     iterations) of ||B||_1 for B = R^{-1} (kappa_1(R) of a triangular
//     factor) or B = (R^T R)^{-1} (the paper's regime bound kappa_2(A)^2 <=
//     n ||A^T A||_1 ||(A^T A)^{-1}||_1 from the Cholesky factor R of A^T A);
//   * the CholQR probe: one pass of Algorithm 1 on A and the bound
//     kappa_2(A) >= sqrt(q / (u (1 + q))), q = ||I - Q^T Q||_2, here with q
//     from power steps on the symmetric I - Q^T Q (a lower estimate of q,
//     so the bound stays a lower bound).
#include "batch.hpp"

namespace mrcqr {

hipError_t launch_gram(const double* B, int m, int n, int64_t ldb, double* Gpart, double* G, int64_t ldg,
                       const Ctrl* ctrl, int phase, hipStream_t st);
size_t gram_partial_bytes(int64_t m, int64_t n);
hipError_t launch_cholesky(const double* G, int n, int64_t ldg, double* Rc, int64_t ldr, int32_t* fail,
                           double* kappa, Ctrl* ctrl, int phase, hipStream_t st);
hipError_t launch_trsm(const double* A, int m, int n, int64_t lda, const double* R, int64_t ldr, double* X,
                       int64_t ldx, void* ws, const Ctrl* ctrl, int phase, hipStream_t st);
size_t trsm_workspace_bytes(int n);

constexpr int EST_NMAX = 128;
constexpr int EST_T = 2;
constexpr int EST_ITMAX = 5;
constexpr int EST_TRIES = 16;  // random draws for a column before keeping the last one

// ---- one wave: lane l holds entries l and l + 64 of each n-vector ---------
__device__ __forceinline__ double est_sum(double v) { return wave_sum_dpp(v); }
__device__ __forceinline__ double est_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// B X for the two columns of X (in place): B = R^{-1} (back substitution),
// its transpose R^{-T} (forward substitution), or (R^T R)^{-1} (both).
__device__ void est_solve(const double* __restrict__ R, int64_t ldr, int n, double (&x)[EST_T][2], bool trans) {
  const int l = threadIdx.x & 63;
  if (!trans) {
    for (int i = n - 1; i >= 0; --i) {
      const double rii = R[i + (int64_t)i * ldr];
#pragma unroll
      for (int j = 0; j < EST_T; ++j) {
        const double own = (i < 64) ? x[j][0] : x[j][1];
        const double xi = readlane_t(own, i & 63) / rii;
        if (l == (i & 63)) { if (i < 64) x[j][0] = xi; else x[j][1] = xi; }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = l + 64 * h;
          if (k < i) x[j][h] = fma(-R[k + (int64_t)i * ldr], xi, x[j][h]);
        }
      }
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const double rii = R[i + (int64_t)i * ldr];
#pragma unroll
      for (int j = 0; j < EST_T; ++j) {
        const double own = (i < 64) ? x[j][0] : x[j][1];
        const double xi = readlane_t(own, i & 63) / rii;
        if (l == (i & 63)) { if (i < 64) x[j][0] = xi; else x[j][1] = xi; }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = l + 64 * h;
          if (k > i && k < n) x[j][h] = fma(-R[i + (int64_t)k * ldr], xi, x[j][h]);
        }
      }
    }
  }
}

__device__ __forceinline__ void est_apply(const double* R, int64_t ldr, int n, double (&x)[EST_T][2], bool trans,
                                          bool gram) {
  if (gram) {  // (R^T R)^{-1} = R^{-1} R^{-T}, symmetric
    est_solve(R, ldr, n, x, true);
    est_solve(R, ldr, n, x, false);
  } else {
    est_solve(R, ldr, n, x, trans);
  }
}

// +-1 entries of the random column `col` (counter-based generator, stream
// 3, counter col * n + i), zero past n
__device__ __forceinline__ void est_fresh(uint64_t key3, int col, int n, double (&v)[2]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = l + 64 * h;
    v[h] = (i < n) ? (((hash_at(key3, (uint64_t)col * n + i) >> 63) == 0) ? 1.0 : -1.0) : 0.0;
  }
}

__device__ __forceinline__ bool est_parallel(const double (&a)[2], const double (&b)[2], int n) {
  return fabs(est_sum(a[0] * b[0] + a[1] * b[1])) == (double)n;
}

// index of the largest v over entries not excluded (ties: smallest index);
// -1 if every entry is excluded
__device__ int est_argmax(const double (&v)[2], const bool (&excl)[2], int n) {
  const int l = threadIdx.x & 63;
  double c0 = (!excl[0] && l < n) ? v[0] : -1.0, c1 = (!excl[1] && l + 64 < n) ? v[1] : -1.0;
  const double mx = est_max(fmax(c0, c1));
  if (mx < 0.0) return -1;
  const uint64_t b0 = __ballot(c0 == mx), b1 = __ballot(c1 == mx);
  if (b0) return __builtin_ctzll(b0);
  return 64 + __builtin_ctzll(b1);
}

// Block 1-norm estimate of B (see the header); one wave.
__device__ double onenorm_est_wave(const double* R, int64_t ldr, int n, bool gram, uint64_t seed) {
  const int l = threadIdx.x & 63;
  const uint64_t key3 = stream_key(seed, 3);
  double X[EST_T][2], S[EST_T][2], Sold[EST_T][2];
  if (n == 1) {
    const double r = R[0];
    return gram ? 1.0 / (r * r) : fabs(1.0 / r);
  }
  int rcol = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) X[0][h] = (l + 64 * h < n) ? 1.0 : 0.0;
  {
    double c[2];
    for (int tries = 0; tries < EST_TRIES; ++tries) {
      est_fresh(key3, rcol++, n, c);
      if (!est_parallel(c, X[0], n)) break;
    }
    X[1][0] = c[0]; X[1][1] = c[1];
  }
#pragma unroll
  for (int j = 0; j < EST_T; ++j) { X[j][0] /= n; X[j][1] /= n; Sold[j][0] = Sold[j][1] = 0.0; }
  int hist[EST_T * (EST_ITMAX + 1)];
  int nhist = 0, ind_best = 0, ind_cur[EST_T] = {0, 0};
  double est = 0.0, est_old = 0.0;
  for (int k = 1; k <= EST_ITMAX + 1; ++k) {
    est_apply(R, ldr, n, X, false, gram);  // X now holds Y = B X
    double norms[EST_T];
#pragma unroll
    for (int j = 0; j < EST_T; ++j) norms[j] = est_sum(fabs(X[j][0]) + fabs(X[j][1]));
    est = fmax(norms[0], norms[1]);
    const int jbest = (norms[0] >= norms[1]) ? 0 : 1;
    if ((est > est_old || k == 2) && k >= 2) ind_best = ind_cur[jbest];
    if (k >= 2 && est <= est_old) { est = est_old; break; }
    est_old = est;
    if (k > EST_ITMAX) break;
#pragma unroll
    for (int j = 0; j < EST_T; ++j)
#pragma unroll
      for (int h = 0; h < 2; ++h) S[j][h] = (l + 64 * h < n) ? (X[j][h] >= 0.0 ? 1.0 : -1.0) : 0.0;
    if (k > 1) {
      bool all = true;
#pragma unroll
      for (int j = 0; j < EST_T; ++j) all = all && (est_parallel(S[j], Sold[0], n) || est_parallel(S[j], Sold[1], n));
      if (all) break;
    }
#pragma unroll
    for (int j = 0; j < EST_T; ++j) {
      for (int tries = 0; tries < EST_TRIES; ++tries) {
        bool par = (j == 1) && est_parallel(S[1], S[0], n);
        if (k > 1) par = par || est_parallel(S[j], Sold[0], n) || est_parallel(S[j], Sold[1], n);
        if (!par) break;
        est_fresh(key3, rcol++, n, S[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < EST_T; ++j) { Sold[j][0] = S[j][0]; Sold[j][1] = S[j][1]; X[j][0] = S[j][0]; X[j][1] = S[j][1]; }
    est_apply(R, ldr, n, X, true, gram);  // X now holds Z = B^T S
    double hv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) hv[h] = fmax(fabs(X[0][h]), fabs(X[1][h]));
    const double hmax = est_max(fmax(l < n ? hv[0] : 0.0, l + 64 < n ? hv[1] : 0.0));
    if (k >= 2 && hmax == readlane_t(ind_best < 64 ? hv[0] : hv[1], ind_best & 63)) break;
    // the t largest h (ties: smaller index first) all seen before: stop
    bool excl[2] = {false, false};
    int top[EST_T];
#pragma unroll
    for (int j = 0; j < EST_T; ++j) {
      top[j] = est_argmax(hv, excl, n);
      if (top[j] >= 0 && l == (top[j] & 63)) { if (top[j] < 64) excl[0] = true; else excl[1] = true; }
    }
    bool seen_all = true;
#pragma unroll
    for (int j = 0; j < EST_T; ++j) {
      bool seen = false;
      for (int q = 0; q < nhist; ++q) seen = seen || hist[q] == top[j];
      seen_all = seen_all && seen;
    }
    if (seen_all) break;
    // the t largest not seen before become the unit vectors of X
    excl[0] = excl[1] = false;
    for (int q = 0; q < nhist; ++q)
      if (l == (hist[q] & 63)) { if (hist[q] < 64) excl[0] = true; else excl[1] = true; }
    int got = 0;
#pragma unroll
    for (int j = 0; j < EST_T; ++j) {
      const int i = est_argmax(hv, excl, n);
      if (i < 0) break;
      ind_cur[j] = i;
      ++got;
      if (l == (i & 63)) { if (i < 64) excl[0] = true; else excl[1] = true; }
    }
    if (got < EST_T) break;
#pragma unroll
    for (int j = 0; j < EST_T; ++j) {
      X[j][0] = (l == ind_cur[j]) ? 1.0 : 0.0;
      X[j][1] = (l + 64 == ind_cur[j]) ? 1.0 : 0.0;
      hist[nhist++] = ind_cur[j];
    }
  }
  return est;
}

// kappa_1(R) (G == nullptr) or the Gram bound sqrt(n ||G||_1 est), R the
// Cholesky factor of G (both n x n, leading dimension ld). One wave.
__global__ __launch_bounds__(64) void onenorm_condest_kernel(const double* __restrict__ R,
                                                            const double* __restrict__ G, int n, int64_t ld,
                                                            uint64_t seed, double* __restrict__ kappa_out) {
  const int l = threadIdx.x;
  const bool gram = G != nullptr;
  const double inv = onenorm_est_wave(R, ld, n, gram, seed);
  // ||R||_1 (upper triangle) or ||G||_1: the largest column sum of |entries|
  double cs[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = l + 64 * h;
    if (j < n) {
      const double* col = (gram ? G : R) + (int64_t)j * ld;
      const int top = gram ? n : j + 1;
      double a = 0.0;
      for (int i = 0; i < top; ++i) a += fabs(col[i]);
      cs[h] = a;
    }
  }
  const double nrm = est_max(fmax(cs[0], cs[1]));
  if (l == 0) {
    double k = gram ? sqrt((double)n * nrm * inv) : nrm * inv;
    if (!isfinite(k)) k = __builtin_inf();
    *kappa_out = k;
  }
}

hipError_t launch_onenorm_condest(const double* R, const double* G, int n, int64_t ld, uint64_t seed,
                                  double* kappa, hipStream_t st) {
  if (n > EST_NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(onenorm_condest_kernel, dim3(1), dim3(64), 0, st, R, G, n, ld, seed, kappa);
  return hipGetLastError();
}

// ---- CholQR probe ----------------------------------------------------------
// q = ||E x|| after POSTERIOR_STEPS normalized applications of E = I - G_Q
// (symmetric, G_Q = Q^T Q) to x0 = ones / sqrt(n); then the paper's bound.
// +inf when the Cholesky of the pass broke down. 256 threads; E in LDS,
// column-major with stride n + 1 (thread r reads row r: conflict-free).
__global__ __launch_bounds__(256) void probe_kernel(const double* __restrict__ GQ, int n, int64_t ld,
                                                   const int32_t* __restrict__ fail, double* __restrict__ kappa_out) {
  __shared__ double E[EST_NMAX * (EST_NMAX + 1)];
  __shared__ double x[EST_NMAX];
  __shared__ double red[4];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  if (*fail >= 0) {
    if (t == 0) *kappa_out = __builtin_inf();
    return;
  }
  for (int e = t; e < n * n; e += 256) {
    const int i = e % n, j = e / n;
    E[i + j * (n + 1)] = (i == j ? 1.0 : 0.0) - GQ[i + (int64_t)j * ld];
  }
  if (t < n) x[t] = 1.0 / sqrt((double)n);
  __syncthreads();
  double q = 0.0;
  for (int it = 0; it <= POSTERIOR_STEPS; ++it) {
    double z = 0.0;
    if (t < n) {
      for (int c = 0; c < n; ++c) z = fma(E[t + c * (n + 1)], x[c], z);
    }
    const double s2 = wave_sum_dpp(t < n ? z * z : 0.0);
    if (l == 0) red[w] = s2;
    __syncthreads();
    const double nz = sqrt((red[0] + red[1]) + (red[2] + red[3]));
    if (it == POSTERIOR_STEPS) { q = nz; break; }
    if (t < n) x[t] = z / nz;
    __syncthreads();
  }
  if (t == 0) {
    const double u = 0x1p-53;
    double k = sqrt(q / (u * (1.0 + q)));
    if (!isfinite(k)) k = __builtin_inf();
    *kappa_out = k;
  }
}

// Workspace of the probe: G (n x n), Rg (n x n), Gram partials, solve
// staging, the breakdown index, Q (m x n).
struct ProbeLayout { size_t G, R, Gpart, Tw, fail, Q, total; };
static size_t est_align(size_t x) { return (x + 255) & ~(size_t)255; }
static ProbeLayout probe_layout(int64_t m, int64_t n) {
  ProbeLayout L;
  size_t o = 0;
  auto take = [&](size_t b) { size_t at = o; o = est_align(o + b); return at; };
  L.G = take((size_t)n * n * 8);
  L.R = take((size_t)n * n * 8);
  L.Gpart = take(gram_partial_bytes(m, n));
  L.Tw = take(trsm_workspace_bytes((int)n));
  L.fail = take(sizeof(int32_t));
  L.Q = take((size_t)m * n * 8);
  L.total = o;
  return L;
}

size_t probe_workspace_bytes(int64_t m, int64_t n) { return probe_layout(m, n).total; }

hipError_t launch_cholqr_probe(const double* A, int m, int n, int64_t lda, void* ws, double* kappa,
                               hipStream_t st) {
  if (n > EST_NMAX) return hipErrorInvalidValue;
  const ProbeLayout L = probe_layout(m, n);
  char* w = static_cast<char*>(ws);
  double* G = reinterpret_cast<double*>(w + L.G);
  double* R = reinterpret_cast<double*>(w + L.R);
  double* Gpart = reinterpret_cast<double*>(w + L.Gpart);
  int32_t* fail = reinterpret_cast<int32_t*>(w + L.fail);
  double* Q = reinterpret_cast<double*>(w + L.Q);
  hipError_t e;
  if ((e = launch_gram(A, m, n, lda, Gpart, G, n, nullptr, PH_FIRST, st)) != hipSuccess) return e;
  if ((e = launch_cholesky(G, n, n, R, n, fail, nullptr, nullptr, PH_FIRST, st)) != hipSuccess) return e;
  if ((e = launch_trsm(A, m, n, lda, R, n, Q, m, w + L.Tw, nullptr, PH_FIRST, st)) != hipSuccess) return e;
  if ((e = launch_gram(Q, m, n, m, Gpart, G, n, nullptr, PH_FIRST, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(probe_kernel, dim3(1), dim3(256), 0, st, G, n, (int64_t)n, fail, kappa);
  return hipGetLastError();
}

}  // namespace mrcqr
