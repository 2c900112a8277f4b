// Algorithm 1, third step, Q = B Rc^{-1}, formed as a product with an
// explicit inverse of Rc. Rc is the Cholesky factor of the Gram matrix of
// the preconditioned B = A Rs^{-1}, whose condition number the sketch keeps
// O(1) (Section "Mixed-Precision Justification"), so kappa(Rc) = kappa(B)
// is a small constant (about 3 at the headline shape, at most the
// posterior threshold when the result is accepted). Applying an explicit
// inverse squares the condition number in the error bound (the reason
// Section "Algorithm Description" keeps the solve with Rs); for Rc that
// costs a few units of roundoff, and it turns the dependent substitution
// into a streaming float64 MFMA contraction. Rs is never inverted:
// B = A Rs^{-1} stays a substitution.
//
// trinv_kernel / rc_tail_kernel: X = R^{-1} for upper-triangular R, one
// wave per column (trinv_column); in the factorization the same launch also
// forms R = Rc Rs.
//
// qform_kernel<NB>: Q = B X with X upper triangular (NB = ceil(n / 16)
// blocks of 16 columns). X is staged once per workgroup in LDS in MFMA
// A-operand order, Xl[off(J, q) + lane] = X[4q + lane / 16][16J + lane % 16]
// for the K steps q < 4(J + 1) that reach column block J (the rest of X is
// zero). Each wave owns 32 rows (two interleaved 16-row tiles: even and
// odd rows) and all NB column blocks; the B operand is read straight from
// HBM (32 rows x 4 columns per 16-byte-per-lane load, 256-byte segments)
// and Q leaves from the accumulators the same way. K steps are taken in
// pairs (q, 4 NB - 1 - q), which cost the same NB + 1 MFMAs per tile
// whatever q is, in chunks of 8 steps; up to three chunks ahead (of this
// tile or the next) are loaded while one is multiplied.
#include "batch.hpp"
#include "small.hpp"

namespace mrcqr {

constexpr int QF_NMAX = 128;
constexpr int QF_NT = 2;  // 16-row tiles per wave (1 wave per SIMD; 2 waves per SIMD with NT = 1 measured slower)
constexpr int QF_CH = 4;  // K-step pairs per chunk

__host__ __device__ constexpr int qf_off(int J, int q) { return 64 * (2 * J * (J + 1) + q); }

// Stand-alone X = R^{-1}: one 64-thread workgroup per column (see
// trinv_column).
__global__ __launch_bounds__(64) void trinv_kernel(const double* __restrict__ R, int n, int64_t ldr,
                                                   double* __restrict__ X, int64_t ldx,
                                                   const Ctrl* __restrict__ ctrl, int phase) {
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  trinv_column(R, n, ldr, X, ldx, blockIdx.x);
}

// The small steps after the Cholesky of the factorization in one launch:
// workgroups 0..n-1 form the columns of Rc^{-1} for Q, the rest the tiles of
// Stage 3's R = Rc Rs (independent of each other).
__device__ __forceinline__ void rc_tail_body(const double* __restrict__ Rc, int n, int64_t ldc,
                                             const double* __restrict__ Rs, int64_t lds_,
                                             double* __restrict__ X, int64_t ldx, double* __restrict__ R,
                                             int64_t ldr, const Ctrl* __restrict__ ctrl, int phase, int b) {
  __shared__ __attribute__((aligned(16))) double lds[TRMM_LDS_DOUBLES];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  if (b < n) {
    trinv_column(Rc, n, ldc, X, ldx, b);
    return;
  }
  const int t = b - n, nbx = (n + 15) / 16;
  trmm_tile(Rc, ldc, Rs, lds_, n, R, ldr, t % nbx, t / nbx, lds);
}

__global__ __launch_bounds__(64) void rc_tail_kernel(const double* __restrict__ Rc, int n, int64_t ldc,
                                                     const double* __restrict__ Rs, int64_t lds_,
                                                     double* __restrict__ X, int64_t ldx, double* __restrict__ R,
                                                     int64_t ldr, const Ctrl* __restrict__ ctrl, int phase) {
  rc_tail_body(Rc, n, ldc, Rs, lds_, X, ldx, R, ldr, ctrl, phase, blockIdx.x);
}

__host__ __device__ inline int rc_tail_blocks(int n) { return n + ((n + 15) / 16) * ((n + 63) / 64); }

// Grouped: a member uses n + (its trmm tiles) workgroups.
__global__ __launch_bounds__(64) void rc_tail_grouped(const BatchInst* __restrict__ bi,
                                                      const int32_t* __restrict__ members, BatchCall call,
                                                      int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= rc_tail_blocks(d.n)) return;
  rc_tail_body(bat_ptr<const double>(call, d, d.off_Rc), d.n, d.n, bat_ptr<const double>(call, d, d.off_Rs), d.n,
               bat_ptr<double>(call, d, d.off_Rci), d.n, call.R[i], call.ldr[i], bat_ptr<const Ctrl>(call, d, d.off_ctrl),
               phase, blockIdx.x);
}

template <int NB, int NT>
__device__ __forceinline__ void qform_body(
    const double* __restrict__ B, int m, int n, int64_t ldb, const double* __restrict__ X, int64_t ldx,
    double* __restrict__ Q, int64_t ldq, const Ctrl* __restrict__ ctrl, int phase, int bx, int gx) {
  constexpr int THREADS = NT == 2 ? 256 : 512;
  constexpr int WROWS = 16 * NT;                // rows per wave
  constexpr int ROWS = THREADS / 64 * WROWS;    // rows per workgroup pass
  constexpr int NQ = 4 * NB;                    // K steps of 4 rows of X
  constexpr int NP = NQ / 2;                    // step pairs
  constexpr int NCH = (NP + QF_CH - 1) / QF_CH;
  constexpr int XSZ = qf_off(NB, 0);
  __shared__ double Xl[XSZ];
  if (skip_launch(ctrl, P_AUTO, phase)) return;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;

  // X in operand order; only its upper triangle (rows and columns < n) is read
  for (int e = tid; e < XSZ; e += THREADS) {
    const int p = e >> 6, lane = e & 63;
    int J = 0;
    while (p >= 2 * (J + 1) * (J + 2)) ++J;
    const int q = p - 2 * J * (J + 1);
    const int row = 4 * q + (lane >> 4), col = 16 * J + (lane & 15);
    Xl[e] = (row <= col && col < n) ? X[row + (int64_t)col * ldx] : 0.0;
  }
  __syncthreads();

  const int64_t npass = ((int64_t)m + ROWS - 1) / ROWS;
  int64_t pass = bx;
  if (pass >= npass) return;

  // K step of pair p, half h: q = p (h = 0) or NQ - 1 - p (h = 1)
  auto kstep = [](int p, int h) { return h == 0 ? p : NQ - 1 - p; };
  typedef const __attribute__((address_space(1))) double* gcptr;
  typedef __attribute__((address_space(1))) double* gptr;
  typedef const __attribute__((address_space(1))) char* gbytes;
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) d2* gcptr2;
  typedef __attribute__((address_space(1))) d2* gptr2;
  const gcptr Bg = (gcptr)B;
  const gptr Qg = (gptr)Q;
  // The NT 16-row tiles of a wave interleave: tile nt holds rows
  // r0 + NT c16 + nt, so that a lane moves its rows of a column with one
  // access. Full passes (all rows inside m, n = 16 NB, leading dimensions
  // below 2^27, for NT = 2 even and with 16-byte aligned B and Q) address B
  // and Q as a wave-uniform base (scalar registers) plus a per-lane 32-bit
  // byte offset (NT c16 + g ld) * 8.
  const bool aligned = NT == 1 || (((ldb | ldq) & 1) == 0 &&
                                   ((reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(Q)) & 15) == 0);
  const bool fast_cfg = ldb < ((int64_t)1 << 27) && ldq < ((int64_t)1 << 27) && aligned && 16 * NB == n;
  const int64_t nfull = fast_cfg ? (int64_t)m / ROWS : 0;
  const uint32_t offB = (uint32_t)(NT * c16 + (int64_t)g * ldb) * 8u;
  const uint32_t offQ = (uint32_t)(NT * c16 + (int64_t)g * ldq) * 8u;

  typedef double Buf[QF_CH][2][NT];
  auto load_fast = [&](Buf& buf, int c, int64_t r0) {
    // bases of the two K steps of a pair, stepped by 4 columns per pair
    // (opaque to the optimizer, so that it keeps one running pointer
    // instead of a precomputed address per K step)
    gcptr lo = Bg + r0 + (int64_t)(4 * kstep(c * QF_CH, 0)) * ldb;
    gcptr hi = Bg + r0 + (int64_t)(4 * kstep(c * QF_CH, 1)) * ldb;
    const int64_t st = 4 * ldb;
#pragma unroll
    for (int pp = 0; pp < QF_CH; ++pp) {
      if (c * QF_CH + pp < NP) {
        asm volatile("" : "+s"(lo), "+s"(hi));
        if constexpr (NT == 2) {
          const d2 vlo = *(gcptr2)((gbytes)lo + offB);
          const d2 vhi = *(gcptr2)((gbytes)hi + offB);
          buf[pp][0][0] = vlo.x;
          buf[pp][0][1] = vlo.y;
          buf[pp][1][0] = vhi.x;
          buf[pp][1][1] = vhi.y;
        } else {
          buf[pp][0][0] = *(gcptr)((gbytes)lo + offB);
          buf[pp][1][0] = *(gcptr)((gbytes)hi + offB);
        }
        lo += st;
        hi -= st;
      }
    }
  };
  // any tile: rows past m read row m - 1 and columns past n read column
  // n - 1 (valid addresses: the X rows they meet are zero and those Q rows
  // are not stored)
  auto load_any = [&](Buf& buf, int c, int64_t r0) {
#pragma unroll
    for (int pp = 0; pp < QF_CH; ++pp) {
      const int p = c * QF_CH + pp;
      if (p < NP) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          int64_t cofs = (int64_t)min(4 * kstep(p, h) + g, n - 1) * ldb;
          asm volatile("" : "+v"(cofs));
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int64_t row = min(r0 + NT * c16 + nt, (int64_t)m - 1);
            buf[pp][h][nt] = B[row + cofs];
          }
        }
      }
    }
  };

  f64x4 acc[NB][NT];
  auto mma_chunk = [&](int c, Buf& buf) {
#pragma unroll
    for (int pp = 0; pp < QF_CH; ++pp) {
      const int p = c * QF_CH + pp;
      if (p < NP) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int q = kstep(p, h);
#pragma unroll
          for (int J = q / 4; J < NB; ++J) {
            const double a = Xl[qf_off(J, q) + l];
            // K step 0 reaches every block first: it starts the sums
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[J][nt] = mfma_f64(a, buf[pp][h][nt], q == 0 ? f64x4{0, 0, 0, 0} : acc[J][nt]);
          }
        }
      }
    }
  };
  // Q rows r0 + NT c16 + nt, columns 16 J + 4 r + g
  auto store_fast = [&](int64_t r0) {
    gptr sq = Qg + r0;
    const int64_t st = 4 * ldq;
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        asm volatile("" : "+s"(sq));
        if constexpr (NT == 2) *(gptr2)((gbytes)sq + offQ) = d2{acc[J][0][r], acc[J][1][r]};
        else *(gptr)((gbytes)sq + offQ) = acc[J][0][r];
        sq += st;
      }
  };
  auto store_any = [&](int64_t r0) {
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int64_t row = r0 + NT * c16 + nt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * J + d_row_f64(l, r);
          if (row < m && col < n) Q[row + (int64_t)col * ldq] = acc[J][nt][r];
        }
      }
  };

  if (pass < nfull) {
    // full passes, software-pipelined: chunk c of a pass lives in buffer
    // c, and D chunks (of this pass or the next) are in flight while one is
    // multiplied
    constexpr int NBUF = NCH >= 2 ? NCH : 2;
    constexpr int D = NBUF - 1;
    Buf bufs[NBUF];
    int64_t r0 = pass * ROWS + WROWS * w;
    static_for<D>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c < NCH) load_fast(bufs[c], c, r0);
    });
    for (;;) {
      const int64_t next = pass + gx;
      const bool more = next < nfull;
      const int64_t r0n = next * ROWS + WROWS * w;
      // X stays in LDS: its operand reads must not be hoisted out of the
      // pass loop (they would need 2 NB (NB + 1) more registers)
      asm volatile("" ::: "memory");
      static_for<NCH>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int cl = c + D;
        if constexpr (cl < NCH) load_fast(bufs[cl % NBUF], cl, r0);
        else if (more) load_fast(bufs[cl % NBUF], cl - NCH, r0n);
        mma_chunk(c, bufs[c % NBUF]);
      });
      store_fast(r0);
      pass = next;
      if (!more) break;
      r0 = r0n;
      if constexpr (NCH == 1) {
        // the single chunk of the next pass went to buffer 1: move it to 0
#pragma unroll
        for (int pp = 0; pp < QF_CH; ++pp)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bufs[0][pp][h][nt] = bufs[1][pp][h][nt];
      }
    }
  }
  // the ragged last pass, and every pass of other shapes
  for (; pass < npass; pass += gx) {
    const int64_t r0 = pass * ROWS + WROWS * w;
    Buf buf;
    asm volatile("" ::: "memory");
    static_for<NCH>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      load_any(buf, c, r0);
      mma_chunk(c, buf);
    });
    store_any(r0);
  }
}

template <int NB, int NT>
__global__ __launch_bounds__(NT == 2 ? 256 : 512, NB <= 2 ? 4 : 1) void qform_kernel(
    const double* __restrict__ B, int m, int n, int64_t ldb, const double* __restrict__ X, int64_t ldx,
    double* __restrict__ Q, int64_t ldq, const Ctrl* __restrict__ ctrl, int phase) {
  qform_body<NB, NT>(B, m, n, ldb, X, ldx, Q, ldq, ctrl, phase, blockIdx.x, gridDim.x);
}

// Grouped: Q = B X of each member; a member uses its own block count.
template <int NB, int NT>
__global__ __launch_bounds__(NT == 2 ? 256 : 512, NB <= 2 ? 4 : 1) void qform_grouped(const BatchInst* __restrict__ bi,
                                                                     const int32_t* __restrict__ members,
                                                                     BatchCall call, int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  if ((int)blockIdx.x >= d.qform_blocks) return;
  qform_body<NB, NT>(bat_ptr<const double>(call, d, d.off_B), d.m, d.n, d.m, bat_ptr<const double>(call, d, d.off_Rci),
                     d.n, call.Q[i], call.ldq[i], bat_ptr<const Ctrl>(call, d, d.off_ctrl), phase, blockIdx.x,
                     d.qform_blocks);
}

// Row passes per workgroup of Q = B X for an m-row member of a batch: about
// four, at most one workgroup per compute unit.
int qform_batch_blocks(int64_t m) {
  constexpr int rows = (QF_NT == 2 ? 256 : 512) / 64 * 16 * QF_NT;
  const int64_t npass = (m + rows - 1) / rows;
  const int64_t b = (npass + 3) / 4;
  return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

hipError_t launch_rc_tail_grouped(const BatchInst* bi, const int32_t* members, int count, int max_n,
                                  const BatchCall& call, int phase, hipStream_t st) {
  hipLaunchKernelGGL(rc_tail_grouped, dim3(rc_tail_blocks(max_n), count), dim3(64), 0, st, bi, members, call, phase);
  return hipGetLastError();
}

// members share nb = ceil(n / 16)
hipError_t launch_qform_grouped(int nb, const BatchInst* bi, const int32_t* members, int count, int max_blocks,
                                const BatchCall& call, int phase, hipStream_t st) {
  constexpr int NT = QF_NT;
  const dim3 grid(max_blocks, count), block(NT == 2 ? 256 : 512);
  switch (nb) {
#define QF_CASE(K) \
  case K: hipLaunchKernelGGL((qform_grouped<K, NT>), grid, block, 0, st, bi, members, call, phase); break;
    QF_CASE(1) QF_CASE(2) QF_CASE(3) QF_CASE(4) QF_CASE(5) QF_CASE(6) QF_CASE(7) QF_CASE(8)
#undef QF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_trinv(const double* R, int n, int64_t ldr, double* X, int64_t ldx, const Ctrl* ctrl, int phase,
                        hipStream_t st) {
  if (n > QF_NMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(trinv_kernel, dim3(n), dim3(64), 0, st, R, n, ldr, X, ldx, ctrl, phase);
  return hipGetLastError();
}

hipError_t launch_rc_tail(const double* Rc, int n, int64_t ldc, const double* Rs, int64_t ldrs, double* X, int64_t ldx,
                          double* R, int64_t ldr, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > QF_NMAX || n > TRMM_NMAX) return hipErrorInvalidValue;
  const int tiles = ((n + 15) / 16) * ((n + 63) / 64);
  hipLaunchKernelGGL(rc_tail_kernel, dim3(n + tiles), dim3(64), 0, st, Rc, n, ldc, Rs, ldrs, X, ldx, R, ldr, ctrl,
                     phase);
  return hipGetLastError();
}

hipError_t launch_qform(const double* B, int m, int n, int64_t ldb, const double* X, int64_t ldx, double* Q,
                        int64_t ldq, const Ctrl* ctrl, int phase, hipStream_t st) {
  if (n > QF_NMAX) return hipErrorInvalidValue;
  constexpr int NT = QF_NT;
  constexpr int rows = (NT == 2 ? 256 : 512) / 64 * 16 * NT;
  const int64_t npass = ((int64_t)m + rows - 1) / rows;
  // one workgroup per CU per wave the instance fits on a SIMD (4 at n <= 32)
  const int64_t cap = 256 * (n <= 32 ? 4 : 1);
  const int grid = (int)(npass < cap ? npass : cap);
  if (grid < 1) return hipGetLastError();
  const int nb = (n + 15) / 16;
  const dim3 block(NT == 2 ? 256 : 512);
  switch (nb) {
#define QF_CASE(K) \
  case K: hipLaunchKernelGGL((qform_kernel<K, NT>), dim3(grid), block, 0, st, B, m, n, ldb, X, ldx, Q, ldq, ctrl, phase); break;
    QF_CASE(1) QF_CASE(2) QF_CASE(3) QF_CASE(4) QF_CASE(5) QF_CASE(6) QF_CASE(7) QF_CASE(8)
#undef QF_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mrcqr
