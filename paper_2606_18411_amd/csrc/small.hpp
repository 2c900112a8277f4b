// Small n x n steps shared by the stand-alone entry points and the fused
// tail launch of the factorization: Stage 3's R = Rc Rs and the columns of
// Rc^{-1} (Algorithm 1, third step, with an explicit inverse). Both run on
// one 64-thread workgroup each.
#pragma once
#include "common.hpp"

namespace mrcqr {

constexpr int TRMM_NMAX = 128;
constexpr int TRMM_LDS_DOUBLES = TRMM_NMAX * 16 + 64 * TRMM_NMAX;

// R = R2 R1 (upper x upper), each entry sum_{j=i..k} R2[i][j] R1[j][k]
// accumulated in index order. One wave per (64-row block by, 16-column
// block bx): lane l accumulates row i = 64 by + l of the 16 columns
// c0..c0+15. The needed parts of R2 (rows i0..i0+63, columns i0..jend-1)
// and of R1 (rows 0..jend-1, the 16 columns) are staged in LDS first
// (lds: TRMM_LDS_DOUBLES doubles, 16-byte aligned). Only the upper
// triangles of R1 and R2 are read as values.
__device__ __forceinline__ void trmm_tile(const double* __restrict__ R2, int64_t ld2, const double* __restrict__ R1,
                                          int64_t ld1, int n, double* __restrict__ R, int64_t ldr, int bx, int by,
                                          double* lds) {
  double* r1s = lds;
  double* r2s = lds + TRMM_NMAX * 16;
  const int l = threadIdx.x;
  const int c0 = 16 * bx, i0 = 64 * by;
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

// Column j of X = R^{-1} for upper-triangular R (one wave): solves R x = e_j
// by back substitution (x_i = (e_j - sum_{k>i} r_ik x_k)_i / r_ii,
// i = j..0) in column order: once x_i is known, r_ki x_i is taken off the
// right-hand side of every row k < i. Lane l holds rows l and l + 64; x_i
// is formed on the lane holding row i (with that lane's reciprocal of
// r_ii) and read from there. Only the upper triangle of R is read.
__device__ __forceinline__ void trinv_column(const double* __restrict__ R, int n, int64_t ldr, double* __restrict__ X,
                                             int64_t ldx, int j) {
  constexpr int U = 8;
  const int l = threadIdx.x & 63;
  const int ra = min(l, n - 1), rb = min(l + 64, n - 1);  // clamped: always valid addresses
  const double rinv0 = 1.0 / R[ra + (int64_t)ra * ldr], rinv1 = 1.0 / R[rb + (int64_t)rb * ldr];
  double s0 = (l == j) ? 1.0 : 0.0, s1 = (l + 64 == j) ? 1.0 : 0.0;
  double pa[U], pb[U];
  auto fetch = [&](int i0) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = max(i0 - u, 0);
      pa[u] = R[ra + i * ldr];
      pb[u] = R[rb + i * ldr];
    }
  };
  fetch(j);
  for (int i0 = j; i0 >= 0; i0 -= U) {
    double ca[U], cb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) { ca[u] = pa[u]; cb[u] = pb[u]; }
    if (i0 - U >= 0) fetch(i0 - U);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 - u;
      if (i < 0) break;
      const double own = (i < 64) ? s0 * rinv0 : s1 * rinv1;
      const double x = readlane_t(own, i & 63);
      s0 = (l == i) ? x : ((l < i) ? fma(-ca[u], x, s0) : s0);
      s1 = (l + 64 == i) ? x : ((l + 64 < i) ? fma(-cb[u], x, s1) : s1);
    }
  }
  if (l < n) X[l + (int64_t)j * ldx] = s0;
  if (l + 64 < n) X[l + 64 + (int64_t)j * ldx] = s1;
}

}  // namespace mrcqr
