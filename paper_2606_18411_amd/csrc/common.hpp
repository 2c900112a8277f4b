// Shared device definitions for the MRCQR gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace mrcqr {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

enum Prec : int { P_AUTO = 0, P_FP64 = 1, P_FP32 = 2, P_FP16 = 3, P_BF16 = 4, P_AUTO_CARRY = 5 };

// MFMA lane layouts on gfx950 (16x16xK, wave64), checked on the device:
//   A operand (16 x K): lane l holds A[l % 16][(l / 16) * (K / 4) + j], j < K/4
//   B operand (K x 16): lane l holds B[(l / 16) * (K / 4) + j][l % 16]
//   D for the f32-accumulating 16x16x4f32 / 16x16x32 f16 / bf16 forms:
//       lane l, register r holds D[4 * (l / 16) + r][l % 16]
//   D for 16x16x4f64: lane l, register r holds D[4 * r + l / 16][l % 16]
__device__ __forceinline__ int d_row_f32(int lane, int r) { return 4 * (lane >> 4) + r; }
__device__ __forceinline__ int d_row_f64(int lane, int r) { return 4 * r + (lane >> 4); }

__device__ __forceinline__ f32x4 mfma_f16(half8 a, half8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// f(integral_constant<0>), ..., f(integral_constant<N-1>), in this order
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

// Counter-based generator (SplitMix64 of Steele, Lea and Flood, 2014).
//   key(seed, stream) = mix64(seed ^ stream * 0xD1B54A32D192ED03)
//   h(key, i)         = mix64(key + (i + 1) * 0x9E3779B97F4A7C15)
// stream 0: Rademacher sign of row t is -1 iff bit 63 of h(key0, t) is set;
// stream 1: Floyd sampling of S; stream 2: per-instance seeds of a batch.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ (stream * 0xD1B54A32D192ED03ull));
}
__host__ __device__ __forceinline__ uint64_t hash_at(uint64_t key, uint64_t i) {
  return mix64(key + (i + 1) * 0x9E3779B97F4A7C15ull);
}

// Per-call device state (lives in the workspace).
struct Ctrl {
  int32_t cur_prec;     // precision of the Stage-1 attempt that is current
  int32_t status;       // mrcqr_status so far
  int32_t chol_fail;    // first failing Cholesky pivot of the accepted pass or -1
  int32_t escalations;  // AUTO escalations
  int32_t auto_mode;    // AutoMode: how the precision is chosen
  int32_t retry;        // reruns the posterior check asked for (0, 1 or 2)
  int32_t carry_prec;   // precision the last carrying call accepted
  int32_t pad0;
  uint64_t carry_tag;   // CARRY_TAG while carry_prec holds a record
  double kappa_rs;
  double kappa_rc;
  int32_t pass_fail;    // Cholesky breakdown index of the current pass or -1
  int32_t pad1;
};

// Precision choice of a call: fixed; AUTO from FP16; AUTO from the
// precision the previous carrying call on this workspace accepted (repeated
// calls on similar matrices, Section "Adaptive Precision Selection").
enum AutoMode : int32_t { AM_FIXED = 0, AM_AUTO = 1, AM_CARRY = 2 };
constexpr uint64_t CARRY_TAG = 0x4D52435152454731ull;

// Status values (mirror of mrcqr_status in mrcqr.h).
enum : int32_t {
  ST_OK = 0, ST_ARG = 1, ST_NONFINITE = 2, ST_CHOL = 3, ST_SINGULAR = 4, ST_POSTERIOR = 7
};

// Regime bounds on the condition estimate of Rs (Section "Adaptive
// Precision Selection": half below 1e4, single below 1e8) and the posterior
// bound on kappa(Rc) = kappa(A Rs^{-1}): Cholesky-QR loses orthogonality
// like kappa^2 u, so 20 keeps it near 4e-14.
constexpr double TAU_FP16 = 1e4;
constexpr double TAU_FP32 = 1e8;
constexpr double TAU_POSTERIOR = 20.0;
// Power steps of the posterior estimate of kappa(Rc) (see posterior.hip).
constexpr int POSTERIOR_STEPS = 12;

// Start-of-call state of the control block (one thread writes it). The
// carry record survives; a carrying call starts from it when it is valid.
__device__ __forceinline__ void ctrl_reset(Ctrl* ctrl, int prec, int auto_mode) {
  int start = prec;
  if (auto_mode == AM_CARRY && ctrl->carry_tag == CARRY_TAG &&
      (ctrl->carry_prec == P_FP32 || ctrl->carry_prec == P_FP64))
    start = ctrl->carry_prec;
  ctrl->cur_prec = start;
  ctrl->status = ST_OK;
  ctrl->chol_fail = -1;
  ctrl->escalations = 0;
  ctrl->auto_mode = auto_mode;
  ctrl->retry = 0;
  ctrl->kappa_rs = 0.0;
  ctrl->kappa_rc = 0.0;
  ctrl->pass_fail = -1;
}

// Called once the call's precision is final: a carrying call leaves it as
// the start of the next one.
__device__ __forceinline__ void ctrl_carry_record(Ctrl* ctrl) {
  if (ctrl->auto_mode == AM_CARRY) {
    ctrl->carry_prec = ctrl->cur_prec;
    ctrl->carry_tag = CARRY_TAG;
  }
}

// Launch gating of the static launch sequence (no host round trip). The
// posterior check may ask for up to two reruns (FP16 -> FP32 -> FP64):
//   phase 0: first pass, always runs;
//   phase 1: first rerun pass, runs when at least one rerun was asked for;
//   phase 2: tail of the first pass (Q), skipped when a rerun follows;
//   phase 3: second rerun pass (with its tail), runs when two were asked for;
//   phase 4: tail of the first rerun pass, skipped when a second follows.
// A Stage-1 kernel for precision slot_prec runs only while that precision
// is the current one (P_AUTO = any).
enum Phase : int { PH_FIRST = 0, PH_RERUN = 1, PH_FIRST_TAIL = 2, PH_RERUN2 = 3, PH_RERUN_TAIL = 4 };

__device__ __forceinline__ bool skip_launch(const Ctrl* ctrl, int slot_prec, int phase) {
  if (ctrl == nullptr) return false;
  if (ctrl->status == ST_ARG) return true;  // a batch member with invalid arguments
  const int retry = ctrl->retry;
  if (phase == PH_RERUN && retry < 1) return true;
  if (phase == PH_FIRST_TAIL && retry != 0) return true;
  if (phase == PH_RERUN2 && retry < 2) return true;
  if (phase == PH_RERUN_TAIL && retry != 1) return true;
  return slot_prec != P_AUTO && ctrl->cur_prec != slot_prec;
}

// An element of a matrix, or zero where the element lies outside it, by an
// unconditional global load from either the element or a zero word: with
// no branch around the load and no select on its value, the compiler keeps
// counting the loads in flight across loop iterations (loads read several
// steps ahead of a serial chain stay in flight) instead of waiting for all
// of them at a branch.
typedef const __attribute__((address_space(1))) double gdouble;
static __device__ const double k_zero_word[1] = {0.0};
__device__ __forceinline__ double load_or_zero(const double* p, bool in) {
  return *(in ? (gdouble*)p : (gdouble*)k_zero_word);
}

// Raise a kernel's dynamic LDS limit to `bytes` when above the default
// 64 KiB; the call's own error state is cleared so that a later
// hipGetLastError() reports only launch failures.
inline void allow_dynamic_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipGetLastError();
  }
}

// ---- wave-level reductions on DPP (no LDS crossbar round trips) ---------
// DPP controls (GFX9 encoding): quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140. After the four stages every
// lane holds the sum over its aligned group of 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <typename T>
__device__ __forceinline__ T dpp_t(T v, int stage) {
  if constexpr (sizeof(T) == 4) {
    switch (stage) { case 0: return dpp_f32<0xB1>(v); case 1: return dpp_f32<0x4E>(v);
                     case 2: return dpp_f32<0x141>(v); default: return dpp_f32<0x140>(v); }
  } else {
    switch (stage) { case 0: return dpp_f64<0xB1>(v); case 1: return dpp_f64<0x4E>(v);
                     case 2: return dpp_f64<0x141>(v); default: return dpp_f64<0x140>(v); }
  }
}
template <typename T>
__device__ __forceinline__ T readlane_t(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  } else {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
  }
}
// Sum over aligned groups of g lanes (g a power of two, 1..64); every lane
// of a group receives the group's sum. Summation order is fixed.
template <typename T>
__device__ __forceinline__ T group_sum_dpp(T v, int g) {
  if (g >= 2) v += dpp_t(v, 0);
  if (g >= 4) v += dpp_t(v, 1);
  if (g >= 8) v += dpp_t(v, 2);
  if (g >= 16) v += dpp_t(v, 3);
  if (g >= 32) {
    const T r0 = readlane_t(v, 0), r1 = readlane_t(v, 16), r2 = readlane_t(v, 32), r3 = readlane_t(v, 48);
    if (g == 32) v = ((threadIdx.x & 63) < 32) ? (r0 + r1) : (r2 + r3);
    else v = (r0 + r1) + (r2 + r3);
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v) { return group_sum_dpp(v, 64); }
// Max over aligned groups of 8 lanes.
__device__ __forceinline__ double group8_max_dpp(double v) {
  v = fmax(v, dpp_t(v, 0));
  v = fmax(v, dpp_t(v, 1));
  v = fmax(v, dpp_t(v, 2));
  return v;
}

}  // namespace mrcqr
