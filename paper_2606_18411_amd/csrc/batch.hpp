// Grouped launches for a batch of independent factorizations: one launch
// per step covers every instance of the batch (or of one kernel
// configuration), grid (blocks per instance, instances). blockIdx.y picks
// the instance from a member list; blockIdx.x is the block's index inside
// that instance's own launch, and blocks past the instance's own count
// return at once. The step kernels run the same bodies as for a single
// factorization, so every instance's result is bitwise that of a single
// call with the same inputs and seed.
#pragma once
#include "common.hpp"

namespace mrcqr {

// Fixed per instance for the life of a batch plan (device array).
struct BatchInst {
  int32_t m, n, s;
  int32_t sk_chunks, sk_rows;   // sketch row chunks and rows per chunk
  int32_t gram_chunks;          // Gram partial sums
  int32_t trsm_blocks;          // blocks of the solve (grid-stride over row panels)
  int32_t qform_blocks;         // blocks of Q = B X (grid-stride over row passes)
  uint64_t ws;                  // byte offset of the instance's workspace region
  uint64_t off_ctrl, off_S, off_Ypart, off_Y, off_Rs, off_Gpart, off_G, off_Rc, off_Rci, off_Tw, off_B;
};

// Per call: device arrays indexed by instance, and the workspace base.
struct BatchCall {
  char* ws;
  const double* const* A;
  const int64_t* lda;
  double* const* Q;
  const int64_t* ldq;
  double* const* R;
  const int64_t* ldr;
  const int32_t* prec;
  const uint64_t* seed;
  void* info;  // batch of 32-byte mrcqr_info records, or null
};

template <typename T>
__device__ __forceinline__ T* bat_ptr(const BatchCall& c, const BatchInst& d, uint64_t off) {
  return reinterpret_cast<T*>(c.ws + d.ws + off);
}

// The instance a block of a grouped launch works for.
__device__ __forceinline__ int bat_index(const int32_t* __restrict__ members) { return members[blockIdx.y]; }

}  // namespace mrcqr
