// Algorithm 2, Stage 1, first step: draw the row sample S and the signs D.
//
// S is Floyd's uniform s-subset of [0, m): for j = m-s .. m-1 take
// r_j = floor(h(key1, j) * (j + 1) / 2^64) in [0, j]; insert r_j unless it is
// already present, else insert j. If all r_j are distinct no insertion ever
// collides and S = {r_j}; that case is detected after sorting (no two equal
// neighbours) and needs no sequential pass. Otherwise one wave replays the
// insertions in order, keeping the set in registers (membership by ballot).
#include "batch.hpp"

namespace mrcqr {

constexpr int DRAW_THREADS = 1024;
constexpr int DRAW_SMAX = 2048;           // largest supported s

__device__ __forceinline__ uint32_t floyd_r(uint64_t key1, uint64_t j) {
  return (uint32_t)__umul64hi(hash_at(key1, j), j + 1);
}

// Ascending bitonic sort of keys[0..P) (P a power of two). With one key per
// thread (P <= blockDim.x) the exchanges inside a wave are shuffles and
// only distances >= 64 go through LDS (3 of 36 stages at P = 256).
__device__ void bitonic_sort(uint32_t* keys, int P) {
  if (P <= (int)blockDim.x) {
    const int i = threadIdx.x;
    uint32_t v = (i < P) ? keys[i] : 0xFFFFFFFFu;
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        uint32_t o;
        if (j >= 64) {
          __syncthreads();
          if (i < P) keys[i] = v;
          __syncthreads();
          o = (i < P) ? keys[i ^ j] : v;
        } else {
          o = (uint32_t)__shfl_xor((int)v, j);
        }
        const bool up = (i & k) == 0, lower = (i & j) == 0;
        v = (lower == up) ? min(v, o) : max(v, o);
      }
    }
    __syncthreads();
    if (i < P) keys[i] = v;
    __syncthreads();
    return;
  }
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        int ixj = i ^ j;
        if (ixj > i) {
          uint32_t a = keys[i], b = keys[ixj];
          bool up = (i & k) == 0;
          if ((a > b) == up) { keys[i] = b; keys[ixj] = a; }
        }
      }
      __syncthreads();
    }
  }
}

// With a control block, thread 0 also resets it for a new factorization
// (the first launch of the call).
__device__ __forceinline__ void draw_body(uint64_t seed, int m, int s, int32_t* S_out, Ctrl* ctrl, int prec,
                                          int auto_mode) {
  if (ctrl && threadIdx.x == 0) ctrl_reset(ctrl, prec, auto_mode);
  __shared__ uint32_t keys[DRAW_SMAX];
  __shared__ int dup;
  const uint64_t key1 = stream_key(seed, 1);
  int P = 1;
  while (P < s) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x)
    keys[i] = (i < s) ? floyd_r(key1, (uint64_t)(m - s + i)) : 0xFFFFFFFFu;
  if (threadIdx.x == 0) dup = 0;
  __syncthreads();
  bitonic_sort(keys, P);
  for (int i = threadIdx.x; i + 1 < s; i += blockDim.x)
    if (keys[i] == keys[i + 1]) dup = 1;
  __syncthreads();
  if (dup) {
    // Floyd's insertion it (j = m - s + it, r = r_it <= j) keeps r unless an
    // earlier insertion already holds r, and then takes j. Every earlier
    // value is below j, so j itself never repeats one, and whether r_it is a
    // repeat depends only on the decisions of insertions before it. Jacobi
    // rounds over all insertions at once therefore reach the sequential
    // decisions exactly: after round k the first k are final, and the rounds
    // stop at the first one that changes nothing (at most s + 1 rounds;
    // about one more than the longest chain of repeats in practice).
    __shared__ uint32_t rv[DRAW_SMAX];
    __shared__ uint8_t took_j[DRAW_SMAX];
    __shared__ int changed;
    for (int i = threadIdx.x; i < s; i += blockDim.x) {
      rv[i] = floyd_r(key1, (uint64_t)(m - s + i));
      took_j[i] = 0;
    }
    __syncthreads();
    for (int round = 0; round <= s; ++round) {
      if (threadIdx.x == 0) changed = 0;
      // a thread has at most two insertions: the launches give s <= 2 blockDim
      uint8_t next[2] = {0, 0};
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = threadIdx.x + u * (int)blockDim.x;
        if (i < s) {
          const uint32_t r = rv[i];
          bool rep = false;
#pragma unroll 8
          for (int k = 0; k < i; ++k) {
            const uint32_t vk = took_j[k] ? (uint32_t)(m - s + k) : rv[k];
            rep |= (vk == r);
          }
          next[u] = rep ? 1 : 0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = threadIdx.x + u * (int)blockDim.x;
        if (i < s && next[u] != took_j[i]) {
          took_j[i] = next[u];
          changed = 1;
        }
      }
      __syncthreads();
      if (!changed) break;
      __syncthreads();
    }
    for (int i = threadIdx.x; i < P; i += blockDim.x)
      keys[i] = (i < s) ? (took_j[i] ? (uint32_t)(m - s + i) : rv[i]) : 0xFFFFFFFFu;
    __syncthreads();
    bitonic_sort(keys, P);
  }
  for (int i = threadIdx.x; i < s; i += blockDim.x) S_out[i] = (int32_t)keys[i];
}

__global__ __launch_bounds__(DRAW_THREADS) void draw_kernel(uint64_t seed, int m, int s, int32_t* S_out,
                                                            Ctrl* ctrl, int prec, int auto_mode) {
  draw_body(seed, m, s, S_out, ctrl, prec, auto_mode);
}

// Grouped: one workgroup per instance; the instance's policy gives the
// starting precision and the AUTO mode.
__global__ __launch_bounds__(DRAW_THREADS) void draw_grouped(const BatchInst* __restrict__ bi,
                                                             const int32_t* __restrict__ members, BatchCall call) {
  const int i = bat_index(members);
  const BatchInst& d = bi[i];
  const int p = call.prec[i];
  const bool am = p == P_AUTO || p == P_AUTO_CARRY;
  Ctrl* ctrl = bat_ptr<Ctrl>(call, d, d.off_ctrl);
  draw_body(call.seed[i], d.m, d.s, bat_ptr<int32_t>(call, d, d.off_S), ctrl, am ? P_FP16 : p,
            p == P_AUTO_CARRY ? AM_CARRY : am ? AM_AUTO : AM_FIXED);
  // the per-call arguments live in device memory: checked here, and a
  // member that fails is skipped by every later kernel of the batch
  if (threadIdx.x == 0) {
    const bool ok = call.A[i] != nullptr && call.Q[i] != nullptr && call.R[i] != nullptr &&
                    call.A[i] != call.Q[i] && call.lda[i] >= d.m && call.ldq[i] >= d.m && call.ldr[i] >= d.n &&
                    p >= P_AUTO && p <= P_AUTO_CARRY;
    if (!ok) ctrl->status = ST_ARG;
  }
}

__global__ void signs_kernel(uint64_t seed, int m, int8_t* D) {
  const uint64_t key0 = stream_key(seed, 0);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x)
    D[t] = (hash_at(key0, (uint64_t)t) >> 63) ? (int8_t)-1 : (int8_t)1;
}

// Forgets the carry record of a control block.
__global__ void regime_reset_kernel(Ctrl* ctrl) {
  if (threadIdx.x == 0) {
    ctrl->carry_tag = 0;
    ctrl->carry_prec = 0;
  }
}

hipError_t launch_regime_reset(Ctrl* ctrl, hipStream_t st) {
  hipLaunchKernelGGL(regime_reset_kernel, dim3(1), dim3(64), 0, st, ctrl);
  return hipGetLastError();
}

hipError_t launch_draw_grouped(const BatchInst* bi, const int32_t* members, int count, int max_s,
                               const BatchCall& call, hipStream_t st) {
  int P = 1;
  while (P < max_s) P <<= 1;
  const int threads = P <= DRAW_THREADS ? (P < 64 ? 64 : P) : DRAW_THREADS;
  hipLaunchKernelGGL(draw_grouped, dim3(1, count), dim3(threads), 0, st, bi, members, call);
  return hipGetLastError();
}

hipError_t launch_draw(uint64_t seed, int m, int s, int32_t* S, int8_t* D, hipStream_t st, Ctrl* ctrl, int prec,
                       int auto_mode) {
  int P = 1;
  while (P < s) P <<= 1;
  const int threads = P <= DRAW_THREADS ? (P < 64 ? 64 : P) : DRAW_THREADS;
  hipLaunchKernelGGL(draw_kernel, dim3(1), dim3(threads), 0, st, seed, m, s, S, ctrl, prec, auto_mode);
  if (D) {
    int blocks = (m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(signs_kernel, dim3(blocks), dim3(256), 0, st, seed, m, D);
  }
  return hipGetLastError();
}

}  // namespace mrcqr
