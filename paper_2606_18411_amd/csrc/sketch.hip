// Algorithm 2, Stage 1: DiagMult (sign flip + cast to p), the transform
// along the rows, and Select (the s sampled rows), computed as one dense
// contraction Y = C_S * fl_p(D A) on the matrix cores, with the rows C_S of
// the transform generated on the fly:
//   DCT-II (default):  C_S[i, t] = cos(pi (2t+1) k / (2m)),  k = S[i] < m;
//   real part of the DFT (the paper's operator, Algorithm 2 FFT + Select):
//                      C_S[i, t] = cos(2 pi k t / m),       k = S[i] <= m/2.
// Both are cos((pi/2) phi / m) of an integer phase phi = (a t + b) k mod 4m,
// (a, b) = (2, 1) and (4, 0).
//
// Work decomposition: grid (row chunks, column blocks of 128, sketch-row
// blocks of 256). A workgroup of 8 waves (for n <= 16, 32, 64: 1, 2, 4
// waves, 16 columns and 32 sketch rows each, so that no wave idles) streams
// its row chunk in panels of 64 rows: the panel is loaded once (coalesced, 512 B per column), signed,
// block-prescaled and cast, and written to LDS in the layout of the MFMA B
// operand; each wave generates the coefficients of its 32 sketch rows
// straight into A-operand registers and multiplies against the whole panel.
// Partial sums per row chunk are reduced in a second kernel in fixed order.
//
// Coefficients: the phase (2t+1)k mod 4m is tracked in exact integer
// arithmetic and evaluated (quadrant reduction + Taylor polynomials on
// [0, pi/4], float64) only to seed rotation recurrences: FP16/BF16 rotate in
// float32 along runs of 8 consecutive rows and advance the run base by one
// panel per panel, re-seeding exactly every 8 panels (error ~2e-6, far below
// the 2^-11 / 2^-8 unit roundoff of the target format); FP32/FP64 rotate in
// float64 along the lane's stride-4 row sequence and re-seed every 4 panels
// (64 rotations, error ~1e-14).
#include "batch.hpp"

namespace mrcqr {

constexpr int SK_SBLK = 256;
constexpr int SK_NBLK = 128;
constexpr int SK_PANEL = 64;

template <int P> struct SkT;
template <> struct SkT<P_FP16> { using elem = _Float16; using acc = float; static constexpr int KSTEP = 32; static constexpr int LD = 72; };
template <> struct SkT<P_BF16> { using elem = __bf16;   using acc = float; static constexpr int KSTEP = 32; static constexpr int LD = 72; };
template <> struct SkT<P_FP32> { using elem = float;    using acc = float; static constexpr int KSTEP = 4;  static constexpr int LD = 66; };
template <> struct SkT<P_FP64> { using elem = double;   using acc = double; static constexpr int KSTEP = 4; static constexpr int LD = 65; };

// ---- cos/sin of the DCT-II phase --------------------------------------
// angle = (pi/2) * phi / m for an integer phase phi in [0, 4m).
// Taylor series of cos and sin on [0, pi/4] (truncation below 1.2e-10 in
// float, below 4e-21 in double).
__device__ __forceinline__ void taylor_f32(float th, float& c, float& s) {
  const float t2 = th * th;
  c = 1.0f + t2 * (-1.0f / 2 + t2 * (1.0f / 24 + t2 * (-1.0f / 720 + t2 * (1.0f / 40320 + t2 * (-1.0f / 3628800)))));
  s = th * (1.0f + t2 * (-1.0f / 6 + t2 * (1.0f / 120 + t2 * (-1.0f / 5040 + t2 * (1.0f / 362880 + t2 * (-1.0f / 39916800))))));
}
__device__ __forceinline__ void taylor_f64(double th, double& c, double& s) {
  const double t2 = th * th;
  c = 1.0 + t2 * (-1.0 / 2 + t2 * (1.0 / 24 + t2 * (-1.0 / 720 + t2 * (1.0 / 40320 + t2 * (-1.0 / 3628800
      + t2 * (1.0 / 479001600.0 + t2 * (-1.0 / 87178291200.0 + t2 * (1.0 / 20922789888000.0
      + t2 * (-1.0 / 6402373705728000.0)))))))));
  s = th * (1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040 + t2 * (1.0 / 362880 + t2 * (-1.0 / 39916800.0
      + t2 * (1.0 / 6227020800.0 + t2 * (-1.0 / 1307674368000.0 + t2 * (1.0 / 355687428096000.0
      + t2 * (-1.0 / 121645100408832000.0))))))))));
}

template <typename F>
__device__ __forceinline__ void phase_sincos(uint32_t phi, uint32_t m, F inv_m, F& cs, F& sn) {
  const uint32_t q = (uint32_t)(phi >= m) + (uint32_t)(phi >= 2u * m) + (uint32_t)(phi >= 3u * m);
  const uint32_t r = phi - q * m;
  const bool swap = 2u * r > m;
  const uint32_t rr = swap ? m - r : r;
  const F th = (F)rr * inv_m * (F)1.5707963267948966192;
  F c0, s0;
  if constexpr (sizeof(F) == 4) taylor_f32(th, c0, s0); else taylor_f64(th, c0, s0);
  const F ca = swap ? s0 : c0;  // cos and sin of the angle inside the quadrant
  const F sa = swap ? c0 : s0;
  cs = (q == 0) ? ca : (q == 1) ? -sa : (q == 2) ? -ca : sa;
  sn = (q == 0) ? sa : (q == 1) ? ca : (q == 2) ? -sa : -ca;
}

__device__ __forceinline__ uint32_t phase_of(uint64_t t, uint64_t k, uint64_t m4, uint64_t pa, uint64_t pb) {
  return (uint32_t)(((pa * t + pb) * k) % m4);
}
__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t m4) {
  uint32_t c = a + b;
  return c >= m4 ? c - m4 : c;
}

// Block power-of-two exponent: mu * 2^e in [2^14, 2^15), clamped to
// [-100, 100]; 0 when mu is 0 or not finite.
__device__ __forceinline__ int block_exp(double mu) {
  if (!(mu > 0.0) || !isfinite(mu)) return 0;
  int E;
  (void)frexp(mu, &E);
  int e = 15 - E;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// The same exponent from the largest biased exponent field F of a block:
// mu = 0.1xx..b * 2^(F - 1022) for normal mu gives e = 15 - (F - 1022);
// F = 0 (zeros or subnormals) gives the clamp 100 (all-zero blocks give
// zero values whatever e is); F = 0x7FF (inf, NaN) gives 0.
__device__ __forceinline__ int block_exp_field(uint32_t F) {
  if (F == 0x7FFu) return 0;
  const int e = 1037 - (int)F;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

__device__ __forceinline__ uint32_t group8_max_u32_dpp(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  return v;
}

template <int P, int NTL, bool FULL>
__device__ __forceinline__ void sketch_body(
    const double* __restrict__ A, int64_t lda, int m, int n,
    const int32_t* __restrict__ S, int s, uint64_t seed, int rows_per_chunk,
    typename SkT<P>::acc* __restrict__ Ypart, const Ctrl* __restrict__ ctrl, int phase,
    int chunk, int cblk, int sblk, int xform) {
  using T = SkT<P>;
  using elem = typename T::elem;
  using acc_t = typename T::acc;
  constexpr int KSTEP = T::KSTEP;
  constexpr int LD = T::LD;
  constexpr int NKS = SK_PANEL / KSTEP;
  constexpr bool LOWP = (P != P_FP64);

  if (skip_launch(ctrl, P, phase)) return;

  __shared__ __attribute__((aligned(16))) elem tile[2][16 * NTL * LD];
  __shared__ float esc[2][16 * NTL];
  __shared__ uint64_t sgnm[2];

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  const int cbase = cblk * SK_NBLK;
  // NTL waves per block: wave w loads columns 16 w .. 16 w + 15 of the panel
  // and owns sketch rows 32 w .. 32 w + 31 of the block's 32 NTL rows
  const int sbase = sblk * (32 * NTL) + w * 32;
  // FULL: the block's 128 columns and 256 sketch rows all exist. Otherwise
  // column tiles at or past n and M tiles of rows at or past s are skipped
  // (their products were zero and never stored; every stored sum goes
  // through the same products in the same order either way).
  const int ncol = FULL ? SK_NBLK : min(n - cbase, 16 * NTL);
  const int ntile = FULL ? NTL : (ncol + 15) >> 4;
  const bool wload = FULL || w * 16 < ncol;  // this wave loads columns that exist
  bool mt_on[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) mt_on[mt] = FULL || sbase + 16 * mt < s;
  const int64_t tstart = (int64_t)chunk * rows_per_chunk;
  const int64_t tend = min((int64_t)m, tstart + rows_per_chunk);
  const int npanels = (int)((tend - tstart + SK_PANEL - 1) / SK_PANEL);
  const uint32_t um = (uint32_t)m, m4 = 4u * (uint32_t)m;
  const uint64_t key0 = stream_key(seed, 0);
  const uint64_t pa = xform ? 4 : 2, pb = xform ? 0 : 1;  // phase (pa t + pb) k

  // ---- this lane's two sketch rows (one per M tile) and their phases ----
  // phi[mt]: exact phase (2t+1)k mod 4m at the lane's first row of the
  // current panel (t0 + 8g for the K=32 forms, t0 + g for the K=4 forms).
  uint32_t phi[2], inc_p[2];
  bool kvalid[2];
  // rotation state: (cb, sb) = cos/sin at the lane's first row of the panel
  typedef typename std::conditional<KSTEP == 32, float, double>::type rot_t;
  rot_t cb[2], sb[2];       // current base
  rot_t c1[2], s1[2];       // rotation by one row step of the lane's sequence
  rot_t cK[2], sK[2];       // rotation by 32 rows (K=32 forms only)
  rot_t cP[2], sP[2];       // rotation by one panel (64 rows)
  float tc1[2];             // 2 cos(one row step), K=32 forms
  const double inv_md = 1.0 / (double)m;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int row = sbase + 16 * mt + c16;
    kvalid[mt] = row < s;
    const uint32_t k = kvalid[mt] ? (uint32_t)S[row] : 0u;
    const uint64_t tl = (uint64_t)tstart + (KSTEP == 32 ? 8 * g : g);
    phi[mt] = phase_of(tl, k, m4, pa, pb);
    inc_p[mt] = (uint32_t)((pa * SK_PANEL * k) % m4);
    // the lane steps 1 row (K=32: 8 consecutive rows) or 4 rows (K=4) at a time
    const uint32_t step = (uint32_t)((pa * (KSTEP == 32 ? 1 : 4) * k) % m4);
    double c, sn;
    phase_sincos<double>(step, um, inv_md, c, sn); c1[mt] = (rot_t)c; s1[mt] = (rot_t)sn;
    tc1[mt] = (float)(2.0 * c);
    phase_sincos<double>((uint32_t)((pa * 32 * k) % m4), um, inv_md, c, sn); cK[mt] = (rot_t)c; sK[mt] = (rot_t)sn;
    phase_sincos<double>(inc_p[mt], um, inv_md, c, sn); cP[mt] = (rot_t)c; sP[mt] = (rot_t)sn;
    phase_sincos<double>(phi[mt], um, inv_md, c, sn); cb[mt] = (rot_t)c; sb[mt] = (rot_t)sn;
  }

  // ---- accumulators ----
  typedef typename std::conditional<LOWP, f32x4, f64x4>::type accv;
  accv acc[2][NTL];
  accv accp[2][NTL];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NTL; ++b) { acc[a][b] = accv{0, 0, 0, 0}; accp[a][b] = accv{0, 0, 0, 0}; }

  // ---- panel loader: thread covers columns cl_r = w*16 + r*8 + l/8 (r = 0,1),
  //      rows 8*(l%8) .. +7 of the panel ----
  double regs[16];
  const int lrow = 8 * (l & 7);
  auto load_panel = [&](int64_t t0) {
    if (!wload) return;
    if (t0 + SK_PANEL <= tend && cbase + 16 * NTL <= n) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const double* ap = A + t0 + lrow + (int64_t)(cbase + w * 16 + r * 8 + (l >> 3)) * lda;
#pragma unroll
        for (int i = 0; i < 8; ++i) regs[r * 8 + i] = ap[i];
      }
    } else {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int col = cbase + w * 16 + r * 8 + (l >> 3);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int64_t t = t0 + lrow + i;
          regs[r * 8 + i] = (col < n && t < tend) ? A[t + (int64_t)col * lda] : 0.0;
        }
      }
    }
  };
  // Rademacher signs of the panel's 64 rows as one ballot mask (bit i = row t0+i)
  auto signs_for = [&](int64_t t0, int buf) {
    if (w == 0) {
      const int64_t t = t0 + l;
      const bool neg = (t < tend) && (hash_at(key0, (uint64_t)t) >> 63);
      const uint64_t msk = __ballot(neg);
      if (l == 0) sgnm[buf] = msk;
    }
  };

  if (npanels > 0) {
    load_panel(tstart);
    signs_for(tstart, 0);
  }
  __syncthreads();

  for (int p = 0; p < npanels; ++p) {
    const int buf = p & 1;
    const int64_t t0 = tstart + (int64_t)p * SK_PANEL;
    // 1. sign, prescale, cast, store to LDS
    const uint32_t smask = (uint32_t)(sgnm[buf] >> lrow) & 0xFFu;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (!wload) continue;
      const int cl = w * 16 + r * 8 + (l >> 3);
      int e = 0;
      if constexpr (LOWP) {
        // the largest biased exponent field of the block decides e (the
        // element of largest magnitude has it); 0x7FF = inf or NaN
        uint32_t fm = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) fm = max(fm, ((uint32_t)__double2hiint(regs[r * 8 + i]) >> 20) & 0x7FFu);
        fm = group8_max_u32_dpp(fm);
        e = block_exp_field(fm);
        if ((l & 7) == 0) esc[buf][cl] = ldexpf(1.0f, -e);
      }
      elem* dst = &tile[buf][cl * LD + lrow];
      typedef typename std::conditional<P == P_BF16, bf16x8, half8>::type vec8s;
      vec8s pk;  // the 8 half-width values of this lane, one 16-byte LDS write
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double x = regs[r * 8 + i];
        const double v = __hiloint2double(__double2hiint(x) ^ (int)(((smask >> i) & 1u) << 31), __double2loint(x));
        if constexpr (LOWP) {
          // two roundings, float64 -> float32 -> p (the barrier keeps the
          // compiler from fusing them into one float64 -> p conversion)
          float f = (float)ldexp(v, e);
          asm volatile("" : "+v"(f));
          if constexpr (KSTEP == 32) pk[i] = (elem)f;
          else dst[i] = (elem)f;
        } else {
          dst[i] = v;
        }
      }
      if constexpr (KSTEP == 32) *reinterpret_cast<vec8s*>(dst) = pk;
    }
    // 2. prefetch the next panel
    if (p + 1 < npanels) {
      load_panel(t0 + SK_PANEL);
      signs_for(t0 + SK_PANEL, buf ^ 1);
    }
    __syncthreads();

    // exact re-seed of the rotation bases every 8 panels (K=32 forms, float)
    // or every 4 panels (K=4 forms, double)
    if (p > 0 && (p & (KSTEP == 32 ? 7 : 3)) == 0) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        double c, sn;
        phase_sincos<double>(phi[mt], um, inv_md, c, sn);
        cb[mt] = (rot_t)c; sb[mt] = (rot_t)sn;
      }
    }

    // 3. contraction of this panel
    const elem* tb = tile[buf];
    if constexpr (KSTEP == 32) {
      typedef typename std::conditional<P == P_FP16, half8, bf16x8>::type vec8;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        vec8 bop[NTL];
#pragma unroll
        for (int nt = 0; nt < NTL; ++nt)
          if (nt < ntile) bop[nt] = *reinterpret_cast<const vec8*>(&tb[(16 * nt + c16) * LD + KSTEP * ks + 8 * g]);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          if (!mt_on[mt]) continue;
          // run of 8 consecutive rows starting 32*ks rows after the base:
          // first two values by rotation, the rest by the three-term
          // recurrence cos((t+1)w) = 2 cos(w) cos(tw) - cos((t-1)w). Rows
          // of sketch rows >= s are computed too and never stored.
          float c = cb[mt], sn = sb[mt];
          if (ks == 1) { const float cn = c * cK[mt] - sn * sK[mt]; sn = sn * cK[mt] + c * sK[mt]; c = cn; }
          vec8 aop;
          float cprev = c, ccur = c * c1[mt] - sn * s1[mt];
          aop[0] = (elem)cprev;
          aop[1] = (elem)ccur;
#pragma unroll
          for (int j = 2; j < 8; ++j) {
            const float cn = fmaf(tc1[mt], ccur, -cprev);
            cprev = ccur;
            ccur = cn;
            aop[j] = (elem)ccur;
          }
#pragma unroll
          for (int nt = 0; nt < NTL; ++nt) {
            if (nt >= ntile) continue;
            const accv cin = (ks == 0) ? accv{0, 0, 0, 0} : accp[mt][nt];
            if constexpr (P == P_FP16) accp[mt][nt] = mfma_f16(aop, bop[nt], cin);
            else accp[mt][nt] = mfma_bf16(aop, bop[nt], cin);
          }
        }
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        const float cn = cb[mt] * cP[mt] - sb[mt] * sP[mt];
        sb[mt] = sb[mt] * cP[mt] + cb[mt] * sP[mt];
        cb[mt] = cn;
      }
    } else {
      // the lane's rows t0 + g + 4 ks: one rotation by 4 rows per K step; after
      // 16 steps the base sits at the next panel's first row
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        elem bop[NTL];
#pragma unroll
        for (int nt = 0; nt < NTL; ++nt)
          if (nt < ntile) bop[nt] = tb[(16 * nt + c16) * LD + KSTEP * ks + g];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const elem a = kvalid[mt] ? (elem)cb[mt] : (elem)0.0;
#pragma unroll
          for (int nt = 0; nt < NTL; ++nt) {
            if (!mt_on[mt] || nt >= ntile) continue;
            if constexpr (P == P_FP32) accp[mt][nt] = mfma_f32(a, bop[nt], accp[mt][nt]);
            else acc[mt][nt] = mfma_f64(a, bop[nt], acc[mt][nt]);
          }
          const double cn = cb[mt] * c1[mt] - sb[mt] * s1[mt];
          sb[mt] = sb[mt] * c1[mt] + cb[mt] * s1[mt];
          cb[mt] = cn;
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) phi[mt] = add_mod(phi[mt], inc_p[mt], m4);
    if constexpr (LOWP) {
      // undo the block prescale of this panel (one power of two per column)
#pragma unroll
      for (int nt = 0; nt < NTL; ++nt) {
        if (nt >= ntile) continue;
        const float sc = esc[buf][16 * nt + c16];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          if (!mt_on[mt]) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[mt][nt][r] = fmaf(accp[mt][nt][r], sc, acc[mt][nt][r]);
          if constexpr (KSTEP != 32) accp[mt][nt] = accv{0, 0, 0, 0};
        }
      }
    }
  }

  // ---- partial sums of this row chunk: Ypart[(chunk*n + col)*s + srow] ----
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < NTL; ++nt) {
      const int col = cbase + 16 * nt + c16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int srow = sbase + 16 * mt + (LOWP ? d_row_f32(l, r) : d_row_f64(l, r));
        if (col < n && srow < s)
          Ypart[((int64_t)chunk * n + col) * s + srow] = acc[mt][nt][r];
      }
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin in linear order
// (x fastest). With several sketch-row blocks, the blocks that read the
// same rows and columns of A get linear ids 8 apart (one XCD, dispatched
// together), so that A comes from HBM once and from that XCD's L2 for the
// others; `remap` needs chunks x column blocks to be a multiple of 8.
template <int P, int NTL, bool FULL>
__global__ __launch_bounds__(64 * NTL) void sketch_kernel(
    const double* __restrict__ A, int64_t lda, int m, int n,
    const int32_t* __restrict__ S, int s, uint64_t seed, int rows_per_chunk,
    typename SkT<P>::acc* __restrict__ Ypart, const Ctrl* __restrict__ ctrl, int phase, int xform, int remap) {
  int chunk = blockIdx.x, cb = blockIdx.y, sb = blockIdx.z;
  if (remap) {
    const int L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int q = L >> 3, nsb = gridDim.z;
    const int pr = (q / nsb) * 8 + (L & 7);
    sb = q % nsb;
    chunk = pr % gridDim.x;
    cb = pr / gridDim.x;
  }
  sketch_body<P, NTL, FULL>(A, lda, m, n, S, s, seed, rows_per_chunk, Ypart, ctrl, phase, chunk, cb, sb, xform);
}

// Grouped (members with n <= 128 and s <= 256: one column block and one
// sketch-row block each); blockIdx.x is the row chunk. Members are grouped
// by the variant a single call of their shape uses (FULL when n = 128 and
// s = 256), since the two may round the coefficients differently.
template <int P, int NTL, bool FULL>
__global__ __launch_bounds__(64 * NTL) void sketch_grouped(const BatchInst* __restrict__ bi,
                                                             const int32_t* __restrict__ members, BatchCall call,
                                                             int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.sk_chunks) return;
  sketch_body<P, NTL, FULL>(call.A[i], call.lda[i], d.m, d.n, bat_ptr<int32_t>(call, d, d.off_S), d.s, call.seed[i],
                       d.sk_rows, bat_ptr<typename SkT<P>::acc>(call, d, d.off_Ypart),
                       bat_ptr<Ctrl>(call, d, d.off_ctrl), phase, blockIdx.x, 0, 0, 0);
}

// Y[srow, col] = scale * sum over chunks (float64, fixed order), then
// rounded to float32 for the low-precision sketches (flags bit 0); scale =
// gamma_k = sqrt(1/s) (k = 0) or sqrt(2/s) for the DCT-II, sqrt(s/m) for
// the real part of the DFT (flags bit 1; the paper's sqrt(c/m)). A block covers 64
// consecutive (col, srow) entries; its 4 waves sum 4 contiguous chunk
// ranges, combined in LDS in fixed order.
template <typename AccT>
__device__ __forceinline__ void sketch_reduce_body(const AccT* __restrict__ Ypart, int chunks, int n, int s,
                                     const int32_t* __restrict__ S, double* __restrict__ Y, int64_t ldy,
                                     int flags, int m, const Ctrl* __restrict__ ctrl, int slot, int phase) {
  if (skip_launch(ctrl, slot, phase)) return;
  const int round_f32 = flags & 1;
  __shared__ double part[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t idx = (int64_t)blockIdx.x * 64 + l;
  const int64_t tot = (int64_t)n * s;
  const int per = (chunks + 3) / 4;
  const int c0 = w * per, c1 = min(chunks, c0 + per);
  double acc = 0.0;
  if (idx < tot) {
    const AccT* p = Ypart + idx;
    int c = c0;
    for (; c + 8 <= c1; c += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (double)p[(int64_t)(c + u) * tot];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; c < c1; ++c) acc += (double)p[(int64_t)c * tot];
  }
  part[w][l] = acc;
  __syncthreads();
  if (w == 0 && idx < tot) {
    const int col = (int)(idx / s), srow = (int)(idx % s);
    const double sum = ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
    const double gamma = (flags & 2) ? sqrt((double)s / (double)m)
                                     : ((S[srow] == 0) ? sqrt(1.0 / (double)s) : sqrt(2.0 / (double)s));
    double y = gamma * sum;
    if (round_f32) y = (double)(float)y;
    Y[srow + (int64_t)col * ldy] = y;
  }
}

template <typename AccT>
__global__ __launch_bounds__(256) void sketch_reduce_kernel(const AccT* __restrict__ Ypart, int chunks, int n, int s,
                                     const int32_t* __restrict__ S, double* __restrict__ Y, int64_t ldy,
                                     int flags, int m, const Ctrl* __restrict__ ctrl, int slot, int phase) {
  sketch_reduce_body<AccT>(Ypart, chunks, n, s, S, Y, ldy, flags, m, ctrl, slot, phase);
}

template <typename AccT>
__global__ __launch_bounds__(256) void sketch_reduce_grouped(const BatchInst* __restrict__ bi,
                                                             const int32_t* __restrict__ members, BatchCall call,
                                                             int round_f32, int slot, int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int64_t)blockIdx.x * 64 >= (int64_t)d.n * d.s) return;
  sketch_reduce_body<AccT>(bat_ptr<const AccT>(call, d, d.off_Ypart), d.sk_chunks, d.n, d.s,
                           bat_ptr<const int32_t>(call, d, d.off_S), bat_ptr<double>(call, d, d.off_Y), d.s, round_f32, d.m,
                           bat_ptr<const Ctrl>(call, d, d.off_ctrl), slot, phase);
}

// ---- host-side launch -------------------------------------------------
struct SketchGeom { int chunks, rows_per_chunk; };

// Kernel variant of an (n, s) sketch: the column tiles a block holds in
// registers and LDS (NTL = 1, 2, 4 for n <= 16, 32, 64, else 8), and FULL
// when every block covers 128 existing columns and 256 existing sketch rows.
// variant = 0, 1, 2 (NTL = 1, 2, 4), 3 (NTL = 8), 4 (NTL = 8, FULL).
int sketch_variant(int n, int s) {
  if (n <= 16) return 0;
  if (n <= 32) return 1;
  if (n <= 64) return 2;
  return (n % SK_NBLK == 0 && s % SK_SBLK == 0) ? 4 : 3;
}

// waves per block (= column tiles held) of a variant
static int sketch_waves(int v) { return v == 0 ? 1 : v == 1 ? 2 : v == 2 ? 4 : 8; }

template <int P>
static void launch_sketch_v(int v, dim3 grid, hipStream_t st, const double* A, int64_t lda, int m, int n,
                            const int32_t* S, int s, uint64_t seed, int rows_per_chunk, typename SkT<P>::acc* Ypart,
                            const Ctrl* ctrl, int phase, int xform) {
  const dim3 block(64 * sketch_waves(v));
  const int remap = (grid.z > 1 && (grid.x * grid.y) % 8 == 0) ? 1 : 0;
  switch (v) {
    case 0: hipLaunchKernelGGL((sketch_kernel<P, 1, false>), grid, block, 0, st, A, lda, m, n, S, s, seed, rows_per_chunk, Ypart, ctrl, phase, xform, remap); break;
    case 1: hipLaunchKernelGGL((sketch_kernel<P, 2, false>), grid, block, 0, st, A, lda, m, n, S, s, seed, rows_per_chunk, Ypart, ctrl, phase, xform, remap); break;
    case 2: hipLaunchKernelGGL((sketch_kernel<P, 4, false>), grid, block, 0, st, A, lda, m, n, S, s, seed, rows_per_chunk, Ypart, ctrl, phase, xform, remap); break;
    case 3: hipLaunchKernelGGL((sketch_kernel<P, 8, false>), grid, block, 0, st, A, lda, m, n, S, s, seed, rows_per_chunk, Ypart, ctrl, phase, xform, remap); break;
    default: hipLaunchKernelGGL((sketch_kernel<P, 8, true>), grid, block, 0, st, A, lda, m, n, S, s, seed, rows_per_chunk, Ypart, ctrl, phase, xform, remap); break;
  }
}

template <int P>
static void launch_sketch_grouped_v(int v, dim3 grid, hipStream_t st, const BatchInst* bi, const int32_t* members,
                                    const BatchCall& call, int phase) {
  const dim3 block(64 * sketch_waves(v));
  switch (v) {
    case 0: hipLaunchKernelGGL((sketch_grouped<P, 1, false>), grid, block, 0, st, bi, members, call, phase); break;
    case 1: hipLaunchKernelGGL((sketch_grouped<P, 2, false>), grid, block, 0, st, bi, members, call, phase); break;
    case 2: hipLaunchKernelGGL((sketch_grouped<P, 4, false>), grid, block, 0, st, bi, members, call, phase); break;
    case 3: hipLaunchKernelGGL((sketch_grouped<P, 8, false>), grid, block, 0, st, bi, members, call, phase); break;
    default: hipLaunchKernelGGL((sketch_grouped<P, 8, true>), grid, block, 0, st, bi, members, call, phase); break;
  }
}

SketchGeom sketch_geometry(int64_t m) {
  const int64_t npan = (m + SK_PANEL - 1) / SK_PANEL;
  const int64_t target = 256;
  const int64_t per = (npan + target - 1) / target;
  SketchGeom gg;
  gg.rows_per_chunk = (int)(per * SK_PANEL);
  gg.chunks = (int)((m + gg.rows_per_chunk - 1) / gg.rows_per_chunk);
  return gg;
}

size_t sketch_partial_bytes(int64_t m, int64_t n, int64_t s, int prec) {
  SketchGeom gg = sketch_geometry(m);
  const size_t el = (prec == P_FP64) ? sizeof(double) : sizeof(float);
  return (size_t)gg.chunks * (size_t)n * (size_t)s * el;
}

hipError_t launch_sketch(int prec, const double* A, int64_t lda, int m, int n, const int32_t* S, int s,
                         uint64_t seed, void* Ypart, double* Y, int64_t ldy, const Ctrl* ctrl, int phase,
                         hipStream_t st, int xform) {
  const int fl = 1 | (xform ? 2 : 0), fl64 = xform ? 2 : 0;
  SketchGeom gg = sketch_geometry(m);
  const int v = sketch_variant(n, s);
  const int srows = 32 * sketch_waves(v);  // sketch rows per block
  dim3 grid(gg.chunks, (n + SK_NBLK - 1) / SK_NBLK, (s + srows - 1) / srows);
  const int rb = 256;
  const int64_t tot = (int64_t)n * s;
  dim3 rgrid((unsigned)((tot + 63) / 64));
  switch (prec) {
    case P_FP16:
      launch_sketch_v<P_FP16>(v, grid, st, A, lda, m, n, S, s, seed, gg.rows_per_chunk, (float*)Ypart, ctrl, phase, xform);
      hipLaunchKernelGGL(sketch_reduce_kernel<float>, rgrid, dim3(rb), 0, st, (const float*)Ypart, gg.chunks, n, s, S, Y, ldy, fl, m, ctrl, (int)P_FP16, phase);
      break;
    case P_BF16:
      launch_sketch_v<P_BF16>(v, grid, st, A, lda, m, n, S, s, seed, gg.rows_per_chunk, (float*)Ypart, ctrl, phase, xform);
      hipLaunchKernelGGL(sketch_reduce_kernel<float>, rgrid, dim3(rb), 0, st, (const float*)Ypart, gg.chunks, n, s, S, Y, ldy, fl, m, ctrl, (int)P_BF16, phase);
      break;
    case P_FP32:
      launch_sketch_v<P_FP32>(v, grid, st, A, lda, m, n, S, s, seed, gg.rows_per_chunk, (float*)Ypart, ctrl, phase, xform);
      hipLaunchKernelGGL(sketch_reduce_kernel<float>, rgrid, dim3(rb), 0, st, (const float*)Ypart, gg.chunks, n, s, S, Y, ldy, fl, m, ctrl, (int)P_FP32, phase);
      break;
    case P_FP64:
      launch_sketch_v<P_FP64>(v, grid, st, A, lda, m, n, S, s, seed, gg.rows_per_chunk, (double*)Ypart, ctrl, phase, xform);
      hipLaunchKernelGGL(sketch_reduce_kernel<double>, rgrid, dim3(rb), 0, st, (const double*)Ypart, gg.chunks, n, s, S, Y, ldy, fl64, m, ctrl, (int)P_FP64, phase);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Stage 1's sketch for every member of a batch at precision prec: grid
// (largest chunk count, members), then the reduction.
hipError_t launch_sketch_grouped(int prec, int variant, const BatchInst* bi, const int32_t* members, int count,
                                 int max_chunks, int64_t max_ns, const BatchCall& call, int phase, hipStream_t st) {
  const dim3 grid(max_chunks, count), rgrid((unsigned)((max_ns + 63) / 64), count);
  switch (prec) {
    case P_FP16:
      launch_sketch_grouped_v<P_FP16>(variant, grid, st, bi, members, call, phase);
      hipLaunchKernelGGL(sketch_reduce_grouped<float>, rgrid, dim3(256), 0, st, bi, members, call, 1, (int)P_FP16, phase);
      break;
    case P_BF16:
      launch_sketch_grouped_v<P_BF16>(variant, grid, st, bi, members, call, phase);
      hipLaunchKernelGGL(sketch_reduce_grouped<float>, rgrid, dim3(256), 0, st, bi, members, call, 1, (int)P_BF16, phase);
      break;
    case P_FP32:
      launch_sketch_grouped_v<P_FP32>(variant, grid, st, bi, members, call, phase);
      hipLaunchKernelGGL(sketch_reduce_grouped<float>, rgrid, dim3(256), 0, st, bi, members, call, 1, (int)P_FP32, phase);
      break;
    case P_FP64:
      launch_sketch_grouped_v<P_FP64>(variant, grid, st, bi, members, call, phase);
      hipLaunchKernelGGL(sketch_reduce_grouped<double>, rgrid, dim3(256), 0, st, bi, members, call, 0, (int)P_FP64, phase);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mrcqr
