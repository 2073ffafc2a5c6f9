// sparrow_ring_dev.h -- the experience buffer's device layout and storage
// conversions, shared by the ring's own kernels and the collecting rollout.
//
// Structure of arrays over the slots (every array indexed by slot):
//   rs, rsn   uint8 [cap][n_rays]  range levels of s and s'
//   cs, csn   uint16 [cap][4]      binary16 scalars of s and s'
//   act       int8 [cap], rew float [cap], done one bit per slot (uint32 words)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sparrow.h"

namespace sp {

constexpr int kRingScalars = 4;

struct RingDev {
  uint8_t* rs;
  uint8_t* rsn;
  uint16_t* cs;
  uint16_t* csn;
  int8_t* act;
  float* rew;
  uint32_t* done;
  int32_t cap, nr;
};

// nearest level of 255 * clamp(o, 0, 1): the product rounds to binary32,
// v_rndne_f32 rounds it to the nearest integer, ties to even; NaN -> 0
__device__ __forceinline__ uint8_t quant_u8(float o) {
  const float c = fminf(fmaxf(o, 0.0f), 1.0f);
  return (uint8_t)__builtin_rintf(c * 255.0f);
}
__device__ __forceinline__ float dequant_u8(uint8_t q) { return (float)q / 255.0f; }
// binary32 -> binary16 with v_cvt_f16_f32 (round to nearest even)
__device__ __forceinline__ uint16_t f16_bits(float f) {
  return __builtin_bit_cast(uint16_t, (_Float16)f);
}
__device__ __forceinline__ float f16_value(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);
}

// set the done bit of a slot whose bit was cleared beforehand (writers of
// one word may race)
__device__ __forceinline__ void ring_set_done(const RingDev& R, int64_t slot) {
  atomicOr(&R.done[slot >> 5], 1u << (uint32_t)(slot & 31));
}

}  // namespace sp

namespace sp {
// Host side (library-internal): the device view of a ring and its next slot,
// and advancing its head and size after another kernel wrote n transitions.
int ring_view(const sparrow_ring* ring, RingDev* view, int64_t* head);
void ring_advance(sparrow_ring* ring, int64_t n);
// Clear the done bits of slots head .. head + n - 1 (mod capacity), on stream.
int ring_clear_done(const RingDev& ring, int64_t head, int64_t n, hipStream_t stream);
}  // namespace sp
