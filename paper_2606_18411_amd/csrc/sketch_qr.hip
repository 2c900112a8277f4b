// Algorithm 2, Stage 1, SketchQR and the promotion of Rs to float64, plus
// the condition estimate that drives the adaptive precision choice
// (Section "Adaptive Precision Selection").
//
// Householder thin QR of the s x n sketch Y in one workgroup of 1024
// threads. Y lives in registers: thread t owns column t / TPC and rows
// (t % TPC) + TPC * i, i < RB (TPC threads per column sit in one wave, so
// column reductions are wave shuffles). Step j: the owner group of column j
// forms the reflector (LAPACK larfg convention: beta = -sign(alpha) ||x||,
// tau = (beta - alpha) / beta, v = x / (alpha - beta), v_j = 1), publishes v
// and tau in LDS (double-buffered, one barrier per step), and every column
// c > j applies H = I - tau v v^T. Arithmetic is float32 for FP16/BF16/FP32
// sketches and float64 for FP64 sketches. Rs gets diag >= 0 by flipping
// rows and is widened to float64.
//
// The ICE estimate (Bischof 1990) of kappa_2 runs in wave 0 afterwards.
#include "batch.hpp"
#include "ice.hpp"

namespace mrcqr {

constexpr int QR_THREADS = 1024;

// Condition estimate of Rs (held row-major in LDS) and the AUTO
// escalation rule, called by every thread after Rs is complete: a sketch
// holding inf or NaN, a singular Rs or an estimate at or above the regime
// bound of the current precision moves the call one precision up (FP16 ->
// FP32 -> FP64); with nothing left to escalate to, a non-finite sketch
// (non-finite input, or input beyond the range of the precision) or a
// singular Rs is reported.
__device__ void sketch_qr_epilogue(const double* Rl, int n, bool bad, bool nonfinite, double* __restrict__ kappa_out,
                                   Ctrl* __restrict__ ctrl, int want_kappa) {
  bad = bad || nonfinite;
  const bool auto_here = ctrl != nullptr && ctrl->auto_mode;
  double kappa = ice_kappa_block(Rl, n, n, 1, !bad && (auto_here || want_kappa));
  if (bad) kappa = __builtin_inf();
  if (threadIdx.x != 0) return;
  if (kappa_out) *kappa_out = kappa;
  if (!ctrl) return;
  ctrl->kappa_rs = kappa;
  const int p = ctrl->cur_prec;
  const bool can_escalate = ctrl->auto_mode && (p == P_FP16 || p == P_FP32);
  const double tau_p = (p == P_FP16) ? TAU_FP16 : (p == P_FP32 ? TAU_FP32 : __builtin_inf());
  if (bad) {
    if (can_escalate) { ctrl->cur_prec = (p == P_FP16) ? P_FP32 : P_FP64; ctrl->escalations += 1; }
    else ctrl->status = nonfinite ? ST_NONFINITE : ST_SINGULAR;
  } else if (can_escalate && kappa >= tau_p) {
    ctrl->cur_prec = (p == P_FP16) ? P_FP32 : P_FP64;
    ctrl->escalations += 1;
  }
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int tpc) { return group_sum_dpp(v, tpc); }

template <typename T, int RB, int NT>
__global__ __launch_bounds__(NT) void householder_kernel(
    const double* __restrict__ Y, int s, int n, int64_t ldy, int tpc,
    double* __restrict__ Rs, int64_t ldr, double* __restrict__ kappa_out,
    Ctrl* __restrict__ ctrl, int slot, int phase, int want_kappa) {
  if (skip_launch(ctrl, slot, phase)) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int vlen = tpc * RB;
  double* Rl = reinterpret_cast<double*>(smem);          // n * n, row-major
  T* vbuf = reinterpret_cast<T*>(Rl + (size_t)n * n);    // 2 * vlen
  T* taus = vbuf + 2 * vlen;                             // 2
  float* dsign = reinterpret_cast<float*>(taus + 2);     // n
  __shared__ int bad_flag;
  __shared__ double wmax[NT / 64];
  __shared__ int wnf[NT / 64];

  // thread -> column c, contiguous row block [rb*RB, rb*RB + RB)
  const int tid = threadIdx.x;
  const int c = tid / tpc, rb = tid % tpc;
  const bool active = c < n;
  const int r0 = rb * RB;
  T y[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int r = r0 + i;
    y[i] = (active && r < s) ? (T)Y[r + (int64_t)c * ldy] : (T)0;
  }
  if (tid == 0) bad_flag = 0;

  // Exact power-of-two prescale so that squares stay in range: Y * 2^es has
  // max magnitude in [0.5, 1); R is scaled back by 2^-es at the end.
  {
    double lm = 0.0;
    bool nf = false;
#pragma unroll
    for (int i = 0; i < RB; ++i) { lm = fmax(lm, fabs((double)y[i])); nf = nf || !isfinite(y[i]); }
    // wave max via the group sum machinery is not needed: use LDS per wave
    for (int o = 32; o > 0; o >>= 1) lm = fmax(lm, __shfl_xor(lm, o));
    const bool wave_nf = __ballot(nf) != 0;
    if ((tid & 63) == 0) { wmax[tid >> 6] = lm; wnf[tid >> 6] = wave_nf; }
  }
  __syncthreads();
  int es = 0;
  bool nonfinite = false;
  {
    double gm = 0.0;
    for (int w = 0; w < NT / 64; ++w) { gm = fmax(gm, wmax[w]); nonfinite = nonfinite || wnf[w]; }
    if (gm > 0.0 && isfinite(gm)) { int E; (void)frexp(gm, &E); es = -E; }
  }
#pragma unroll
  for (int i = 0; i < RB; ++i) y[i] = (T)ldexp((double)y[i], es);

  // Reflector of column j, formed by the tpc threads that own it (LAPACK
  // larfg convention); v is zero above row j and below row s.
  auto reflector = [&](int j, int buf) {
    T alpha_l = (T)0, sp[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = r0 + i;
      alpha_l = (r == j) ? y[i] : alpha_l;
      sp[i & 3] += (r > j) ? y[i] * y[i] : (T)0;
    }
    const T alpha = group_sum(alpha_l, tpc);
    const T sig = group_sum((sp[0] + sp[1]) + (sp[2] + sp[3]), tpc);
    T tau, beta, scal;
    if (sig == (T)0) { tau = (T)0; beta = alpha; scal = (T)0; }
    else {
      const T nrm = sqrt(alpha * alpha + sig);
      beta = signbit(alpha) ? nrm : -nrm;
      tau = (beta - alpha) / beta;
      scal = (T)1 / (alpha - beta);
    }
    T* v = vbuf + buf * vlen + r0;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = r0 + i;
      v[i] = (r > j) ? y[i] * scal : (r == j ? (T)1 : (T)0);
      y[i] = (r == j) ? beta : y[i];
    }
    if (rb == 0) taus[buf] = tau;
  };

  if (c == 0) reflector(0, 0);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int buf = j & 1;
    if (active && c > j) {
      const T tau = taus[buf];
      const T* v = vbuf + buf * vlen + r0;
      T dp[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
      for (int i = 0; i < RB; ++i) dp[i & 3] += v[i] * y[i];
      const T d = group_sum((dp[0] + dp[1]) + (dp[2] + dp[3]), tpc);
      const T f = tau * d;
#pragma unroll
      for (int i = 0; i < RB; ++i) y[i] -= f * v[i];
      // look-ahead: the owners of column j+1 form its reflector now, while
      // the other columns are still being updated
      if (c == j + 1) reflector(j + 1, buf ^ 1);
    }
    __syncthreads();
  }

  // diag(R) >= 0: flip rows with a negative pivot; widen to float64.
  if (active) {
#pragma unroll
    for (int i = 0; i < RB; ++i)
      if (r0 + i == c) dsign[c] = (y[i] < (T)0) ? -1.0f : 1.0f;
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = r0 + i;
      if (r < n) {
        const double val = (r <= c) ? ldexp((double)y[i] * (double)dsign[r], -es) : 0.0;
        Rs[r + (int64_t)c * ldr] = val;
        Rl[r * n + c] = val;
        if (r == c && !(val > 0.0 && isfinite(val))) bad_flag = 1;
        if (r < c && !isfinite(val)) bad_flag = 1;
      }
    }
  }
  __syncthreads();
  sketch_qr_epilogue(Rl, n, bad_flag != 0, nonfinite, kappa_out, ctrl, want_kappa);
}


// Main path for s <= 512: NT threads in groups of 16 lanes (one DPP row).
// Group g owns columns g + NT/16 k (k < CPT) over all rows; lane t of a group
// owns rows VEC (t + 16 i) + e (i < RPT / VEC, e < VEC), VEC = 16 bytes /
// sizeof(T). The published reflector v is read as 16-byte vectors: the 16
// lanes of a group read 256 consecutive bytes and the 4 groups of a wave
// read the same ones (broadcast, no bank conflicts). Per step each thread
// reads its RPT entries of v once and applies them to its CPT columns
// (LDS traffic per step: NT * RPT entries);
// column sums are 4 DPP stages inside the group. The column j + 1 is
// updated first by its group, which then forms the next reflector while
// the other columns are still being updated (one barrier per step).
template <typename T, int NT, int CPT, int RPT>
__device__ __forceinline__ void householder16_body(
    const double* __restrict__ Y, int s, int n, int64_t ldy,
    double* __restrict__ Rs, int64_t ldr, double* __restrict__ kappa_out,
    Ctrl* __restrict__ ctrl, int slot, int phase, int want_kappa) {
  if (skip_launch(ctrl, slot, phase)) return;
  constexpr int TPG = 16, NG = NT / TPG;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int NI = RPT / VEC;
  constexpr int SP = TPG * RPT;  // padded rows
  static_assert(RPT % VEC == 0, "RPT must be a multiple of the vector width");
  typedef T vec_t __attribute__((ext_vector_type(VEC)));
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* vbuf = reinterpret_cast<T*>(smem);                   // 2 * SP
  double* Rl = reinterpret_cast<double*>(vbuf + 2 * SP);  // n * n, row-major
  T* taus = reinterpret_cast<T*>(Rl + (size_t)n * n);     // 2
  float* dsign = reinterpret_cast<float*>(taus + 2);      // n
  __shared__ int bad_flag;
  __shared__ double wmax[NT / 64];
  __shared__ int wnf[NT / 64];

  const int tid = threadIdx.x, grp = tid / TPG, t = tid % TPG;
  auto row_of = [&](int i, int e) { return VEC * (t + TPG * i) + e; };
  T y[CPT][RPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = grp + NG * k;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int r = row_of(i, e);
        y[k][VEC * i + e] = (c < n && r < s) ? (T)Y[r + (int64_t)c * ldy] : (T)0;
      }
  }
  if (tid == 0) bad_flag = 0;

  // exact power-of-two prescale: max |Y| * 2^es in [0.5, 1)
  {
    double lm = 0.0;
    bool nf = false;
#pragma unroll
    for (int k = 0; k < CPT; ++k)
#pragma unroll
      for (int i = 0; i < RPT; ++i) { lm = fmax(lm, fabs((double)y[k][i])); nf = nf || !isfinite(y[k][i]); }
    for (int o = 32; o > 0; o >>= 1) lm = fmax(lm, __shfl_xor(lm, o));
    const bool wave_nf = __ballot(nf) != 0;
    if ((tid & 63) == 0) { wmax[tid >> 6] = lm; wnf[tid >> 6] = wave_nf; }
  }
  __syncthreads();
  int es = 0;
  bool nonfinite = false;
  {
    double gm = 0.0;
    for (int w = 0; w < NT / 64; ++w) { gm = fmax(gm, wmax[w]); nonfinite = nonfinite || wnf[w]; }
    if (gm > 0.0 && isfinite(gm)) { int E; (void)frexp(gm, &E); es = -E; }
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int i = 0; i < RPT; ++i) y[k][i] = (T)ldexp((double)y[k][i], es);

  // reflector of column jj = grp + NG * K from this group's registers
  // (LAPACK larfg convention), published to vbuf[buf] and taus[buf]
  auto reflector = [&](auto kc, int jj, int buf) {
    constexpr int K = decltype(kc)::value;
    T alpha_l = (T)0, sp = (T)0;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int r = row_of(i, e);
        const T v = y[K][VEC * i + e];
        alpha_l = (r == jj) ? v : alpha_l;
        sp += (r > jj) ? v * v : (T)0;
      }
    const T alpha = group_sum_dpp(alpha_l, TPG);
    const T sig = group_sum_dpp(sp, TPG);
    T tau, beta, scal;
    if (sig == (T)0) { tau = (T)0; beta = alpha; scal = (T)0; }
    else {
      const T nrm = sqrt(alpha * alpha + sig);
      beta = signbit(alpha) ? nrm : -nrm;
      tau = (beta - alpha) / beta;
      scal = (T)1 / (alpha - beta);
    }
    T* vb = vbuf + buf * SP;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      vec_t vv;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int r = row_of(i, e);
        const T yv = y[K][VEC * i + e];
        vv[e] = (r > jj) ? yv * scal : (r == jj ? (T)1 : (T)0);
        y[K][VEC * i + e] = (r == jj) ? beta : yv;
      }
      *reinterpret_cast<vec_t*>(vb + VEC * (t + TPG * i)) = vv;
    }
    if (t == 0) taus[buf] = tau;
  };

  if (grp == 0) reflector(std::integral_constant<int, 0>{}, 0, 0);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int buf = j & 1;
    const T tau = taus[buf];
    T v[RPT];
    const T* vb = vbuf + buf * SP;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const vec_t vv = *reinterpret_cast<const vec_t*>(vb + VEC * (t + TPG * i));
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[VEC * i + e] = vv[e];
    }
    auto apply = [&](auto kc) {
      constexpr int K = decltype(kc)::value;
      const int c = grp + NG * K;
      if (c > j && c < n) {
        T dp[2] = {(T)0, (T)0};
#pragma unroll
        for (int i = 0; i < RPT; ++i) dp[i & 1] += v[i] * y[K][i];
        const T d = group_sum_dpp(dp[0] + dp[1], TPG);
        const T f = tau * d;
#pragma unroll
        for (int i = 0; i < RPT; ++i) y[K][i] -= f * v[i];
        if (c == j + 1) reflector(kc, j + 1, buf ^ 1);
      }
    };
    static_for<CPT>(apply);
    __syncthreads();
  }

  // diag(R) >= 0: flip rows with a negative pivot; widen to float64.
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = grp + NG * k;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (c < n && row_of(i, e) == c) dsign[c] = (y[k][VEC * i + e] < (T)0) ? -1.0f : 1.0f;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const int c = grp + NG * k;
    if (c >= n) continue;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int r = row_of(i, e);
        if (r < n) {
          const double val = (r <= c) ? ldexp((double)y[k][VEC * i + e] * (double)dsign[r], -es) : 0.0;
          Rs[r + (int64_t)c * ldr] = val;
          Rl[r * n + c] = val;
          if (r == c && !(val > 0.0 && isfinite(val))) bad_flag = 1;
          if (r < c && !isfinite(val)) bad_flag = 1;
        }
      }
  }
  __syncthreads();
  sketch_qr_epilogue(Rl, n, bad_flag != 0, nonfinite, kappa_out, ctrl, want_kappa);
}

// Stand-alone ICE of an upper-triangular matrix (two waves).
template <typename T, int NT, int CPT, int RPT>
__global__ __launch_bounds__(NT) void householder16_kernel(
    const double* __restrict__ Y, int s, int n, int64_t ldy,
    double* __restrict__ Rs, int64_t ldr, double* __restrict__ kappa_out,
    Ctrl* __restrict__ ctrl, int slot, int phase, int want_kappa) {
  householder16_body<T, NT, CPT, RPT>(Y, s, n, ldy, Rs, ldr, kappa_out, ctrl, slot, phase, want_kappa);
}

// Grouped: one workgroup per member (all members share the configuration).
template <typename T, int NT, int CPT, int RPT>
__global__ __launch_bounds__(NT) void householder16_grouped(const BatchInst* __restrict__ bi,
                                                            const int32_t* __restrict__ members, BatchCall call,
                                                            int slot, int phase) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  householder16_body<T, NT, CPT, RPT>(bat_ptr<const double>(call, d, d.off_Y), d.s, d.n, d.s,
                                      bat_ptr<double>(call, d, d.off_Rs), d.n, nullptr,
                                      bat_ptr<Ctrl>(call, d, d.off_ctrl), slot, phase, 0);
}

__global__ void condest_kernel(const double* __restrict__ R, int n, int64_t ldr, double* __restrict__ kappa_out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double* Rl = reinterpret_cast<double*>(smem);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;  // coalesced reads, row-major copy
    Rl[i * n + j] = (i <= j) ? R[i + (int64_t)j * ldr] : 0.0;
  }
  __syncthreads();
  const double k = ice_kappa_block(Rl, n, n, 1, true);
  if (threadIdx.x == 0) *kappa_out = k;
}

// Threads per column: a power of two <= 64 with tpc * n <= NT. Register
// rows per thread RB >= ceil(s / tpc). Large RB runs with 512 threads so
// that each thread may use 256 registers.
static int qr_tpc(int n, int nt) {
  int t = 64;
  while (t > 1 && t * n > nt) t >>= 1;
  return t;
}

size_t qr_smem_bytes(int vlen, int n, bool f64) {
  const size_t el = f64 ? 8 : 4;
  return (size_t)n * n * 8 + 2 * (size_t)vlen * el + 2 * el + (size_t)n * 4 + 64;
}

bool qr_supported(int s, int n) {
  if (n < 1 || n > 128) return false;
  const int tpc = qr_tpc(n, 512);
  return (s + tpc - 1) / tpc <= 64;
}

template <typename T, int RB, int NT>
static hipError_t launch_qr_rb(const double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                               double* kappa, Ctrl* ctrl, int slot, int phase, hipStream_t st) {
  const size_t sm = qr_smem_bytes(qr_tpc(n, NT) * RB, n, sizeof(T) == 8);
  allow_dynamic_lds(reinterpret_cast<const void*>(&householder_kernel<T, RB, NT>), sm);
  hipLaunchKernelGGL((householder_kernel<T, RB, NT>), dim3(1), dim3(NT), sm, st,
                     Y, s, n, ldy, qr_tpc(n, NT), Rs, ldr, kappa, ctrl, slot, phase, kappa != nullptr ? 1 : 0);
  return hipGetLastError();
}

template <typename T, int NT, int CPT, int RPT>
static hipError_t launch_qr16(const double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                              double* kappa, Ctrl* ctrl, int slot, int phase, hipStream_t st) {
  const size_t sm = 2 * (size_t)16 * RPT * sizeof(T) + (size_t)n * n * 8 + 2 * sizeof(T) + (size_t)n * 4 + 64;
  allow_dynamic_lds(reinterpret_cast<const void*>(&householder16_kernel<T, NT, CPT, RPT>), sm);
  hipLaunchKernelGGL((householder16_kernel<T, NT, CPT, RPT>), dim3(1), dim3(NT), sm, st,
                     Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, kappa != nullptr ? 1 : 0);
  return hipGetLastError();
}

// Configuration of the 16-lane-group kernel for (s, n): rows per lane RPT =
// s / 16 rounded up to {4, 8, 16, 32}; 1024 threads (64 groups, CPT <= 2)
// when the register arrays (y: CPT * RPT, v: RPT entries) stay within
// about 80 registers, else 512 threads (32 groups, CPT <= 4, about 200).
// Returns false when the shape needs the general kernel.
template <typename T>
static bool qr16_config(int s, int n, int& nt, int& cpt, int& rpt) {
  rpt = 4;
  while (rpt * 16 < s) rpt *= 2;
  if (rpt > 32) return false;
  const int wsz = (int)sizeof(T) / 4;
  cpt = (n + 63) / 64;
  if (cpt <= 2 && (cpt * rpt + rpt) * wsz <= 80) { nt = 1024; return true; }
  cpt = (n + 31) / 32 > 2 ? 4 : 2;
  if ((cpt * rpt + rpt) * wsz <= 200) { nt = 512; return true; }
  return false;
}

template <typename T, int NT, int CPT, int RPT>
static hipError_t launch_qr16_grouped(const BatchInst* bi, const int32_t* members, int count, int max_n,
                                      const BatchCall& call, int slot, int phase, hipStream_t st) {
  const size_t sm = 2 * (size_t)16 * RPT * sizeof(T) + (size_t)max_n * max_n * 8 + 2 * sizeof(T) + (size_t)max_n * 4 + 64;
  allow_dynamic_lds(reinterpret_cast<const void*>(&householder16_grouped<T, NT, CPT, RPT>), sm);
  hipLaunchKernelGGL((householder16_grouped<T, NT, CPT, RPT>), dim3(1, count), dim3(NT), sm, st, bi, members, call,
                     slot, phase);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_qr_t(const double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                              double* kappa, Ctrl* ctrl, int slot, int phase, hipStream_t st) {
  int nt, cpt, rpt;
  if (qr16_config<T>(s, n, nt, cpt, rpt)) {
#define QR16(N, C, R) \
  if (nt == N && cpt == C && rpt == R) return launch_qr16<T, N, C, R>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st)
    if constexpr (sizeof(T) == 4) {
      QR16(1024, 1, 4); QR16(1024, 1, 8); QR16(1024, 1, 16); QR16(1024, 1, 32);
      QR16(1024, 2, 4); QR16(1024, 2, 8); QR16(1024, 2, 16);
    } else {
      QR16(1024, 1, 4); QR16(1024, 1, 8); QR16(1024, 1, 16);
      QR16(1024, 2, 4); QR16(1024, 2, 8);
      QR16(512, 4, 16); QR16(512, 2, 32);
    }
#undef QR16
    return hipErrorInvalidValue;  // a configuration without an instance
  }
  const int t1 = qr_tpc(n, 1024);
  const int need1 = (s + t1 - 1) / t1;
  if (need1 <= 1) return launch_qr_rb<T, 1, 1024>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  if (need1 <= 2) return launch_qr_rb<T, 2, 1024>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  if (need1 <= 4) return launch_qr_rb<T, 4, 1024>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  if (need1 <= 8) return launch_qr_rb<T, 8, 1024>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  if (need1 <= 16) return launch_qr_rb<T, 16, 1024>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  if constexpr (sizeof(T) == 4)  // float fits 32 rows per thread at 1024 threads without spills
    if (need1 <= 32) return launch_qr_rb<T, 32, 1024>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  const int t5 = qr_tpc(n, 512);
  const int need5 = (s + t5 - 1) / t5;
  if (need5 <= 32) return launch_qr_rb<T, 32, 512>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  if (need5 <= 64) return launch_qr_rb<T, 64, 512>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
  return hipErrorInvalidValue;
}

hipError_t launch_sketch_qr(bool f64, const double* Y, int s, int n, int64_t ldy, double* Rs, int64_t ldr,
                            double* kappa, Ctrl* ctrl, int slot, int phase, hipStream_t st) {
  return f64 ? launch_qr_t<double>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st)
             : launch_qr_t<float>(Y, s, n, ldy, Rs, ldr, kappa, ctrl, slot, phase, st);
}

// Configuration key of the sketch QR of an (s, n) sketch for a grouped
// launch: nt * 10000 + cpt * 100 + rpt, or -1 when the shape needs the
// general kernel (never for s <= 256).
int qr_group_key(bool f64, int s, int n) {
  int nt, cpt, rpt;
  const bool ok = f64 ? qr16_config<double>(s, n, nt, cpt, rpt) : qr16_config<float>(s, n, nt, cpt, rpt);
  return ok ? nt * 10000 + cpt * 100 + rpt : -1;
}

hipError_t launch_sketch_qr_grouped(bool f64, int key, const BatchInst* bi, const int32_t* members, int count,
                                    int max_n, const BatchCall& call, int slot, int phase, hipStream_t st) {
  const int nt = key / 10000, cpt = (key / 100) % 100, rpt = key % 100;
#define QRG(T, N, C, R)                                     \
  if (nt == N && cpt == C && rpt == R)                      \
    return launch_qr16_grouped<T, N, C, R>(bi, members, count, max_n, call, slot, phase, st)
  if (!f64) {
    QRG(float, 1024, 1, 4); QRG(float, 1024, 1, 8); QRG(float, 1024, 1, 16); QRG(float, 1024, 1, 32);
    QRG(float, 1024, 2, 4); QRG(float, 1024, 2, 8); QRG(float, 1024, 2, 16);
  } else {
    QRG(double, 1024, 1, 4); QRG(double, 1024, 1, 8); QRG(double, 1024, 1, 16);
    QRG(double, 1024, 2, 4); QRG(double, 1024, 2, 8);
    QRG(double, 512, 4, 16); QRG(double, 512, 2, 32);
  }
#undef QRG
  return hipErrorInvalidValue;
}

hipError_t launch_condest(const double* R, int n, int64_t ldr, double* kappa, hipStream_t st) {
  allow_dynamic_lds(reinterpret_cast<const void*>(&condest_kernel), (size_t)n * n * 8);
  hipLaunchKernelGGL(condest_kernel, dim3(1), dim3(256), (size_t)n * n * 8, st, R, n, ldr, kappa);
  return hipGetLastError();
}

}  // namespace mrcqr
