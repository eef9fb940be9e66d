// Wavefront-level building blocks shared by the kernels (wave64, gfx950).
#pragma once

#include "common.h"

namespace systec {
namespace dev {

constexpr int kV = 8;                 // entries per lane
constexpr int kTile = kWave * kV;     // entries per wavefront tile

// ---- wave-level primitives (DPP; wave64) ----------------------------------
// DPP controls: row_shr:n = 0x110+n, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_i32(int old, int src) {
  return __builtin_amdgcn_update_dpp(old, src, kCtrl, kRowMask, 0xf, false);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_f32(float old, float src) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), kCtrl, kRowMask, 0xf,
                                  false));
}

// The value of the next lane (lane 63 gets `last`), by the DPP whole-wave
// shift (wave_shl:1), which, unlike a shuffle through ds_bpermute, does not
// wait for the LDS operations still in flight.
__device__ __forceinline__ int next_lane_i32(int v, int last) {
  return dpp_i32<0x130, 0xf>(last, v);
}

// Inclusive max-scan over the 64 lanes.
__device__ __forceinline__ int wave_incl_max(int v) {
  v = max(v, dpp_i32<0x111, 0xf>(INT_MIN, v));
  v = max(v, dpp_i32<0x112, 0xf>(INT_MIN, v));
  v = max(v, dpp_i32<0x114, 0xf>(INT_MIN, v));
  v = max(v, dpp_i32<0x118, 0xf>(INT_MIN, v));
  v = max(v, dpp_i32<0x142, 0xa>(INT_MIN, v));
  v = max(v, dpp_i32<0x143, 0xc>(INT_MIN, v));
  return v;
}

// Inclusive segmented sum over the 64 lanes; segments are runs of equal keys
// (keys are nondecreasing across lanes).
__device__ __forceinline__ float wave_seg_sum(int key, float v) {
#define SYSTEC_SEG_STEP(CTRL, MASK)                         \
  {                                                         \
    const int k2 = dpp_i32<CTRL, MASK>(-2, key);            \
    const float v2 = dpp_f32<CTRL, MASK>(0.0f, v);          \
    v += (k2 == key) ? v2 : 0.0f;                           \
  }
  SYSTEC_SEG_STEP(0x111, 0xf)
  SYSTEC_SEG_STEP(0x112, 0xf)
  SYSTEC_SEG_STEP(0x114, 0xf)
  SYSTEC_SEG_STEP(0x118, 0xf)
  SYSTEC_SEG_STEP(0x142, 0xa)
  SYSTEC_SEG_STEP(0x143, 0xc)
#undef SYSTEC_SEG_STEP
  return v;
}

// Inclusive segmented minimum over the 64 lanes (segments as for
// wave_seg_sum; +inf is the identity).
__device__ __forceinline__ float wave_seg_min(int key, float v) {
#define SYSTEC_SEGMIN_STEP(CTRL, MASK)                      \
  {                                                         \
    const int k2 = dpp_i32<CTRL, MASK>(-2, key);            \
    const float v2 = dpp_f32<CTRL, MASK>(INFINITY, v);      \
    v = (k2 == key) ? fminf(v, v2) : v;                     \
  }
  SYSTEC_SEGMIN_STEP(0x111, 0xf)
  SYSTEC_SEGMIN_STEP(0x112, 0xf)
  SYSTEC_SEGMIN_STEP(0x114, 0xf)
  SYSTEC_SEGMIN_STEP(0x118, 0xf)
  SYSTEC_SEGMIN_STEP(0x142, 0xa)
  SYSTEC_SEGMIN_STEP(0x143, 0xc)
#undef SYSTEC_SEGMIN_STEP
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Finishes a wave's segmented sums. Each lane has summed its own entries by
// key (keys nondecreasing across lanes): segments strictly inside the lane are
// already written; `first_key`/`head_val` is its first segment when the lane
// holds more than one (nseg >= 2) and `tail_key`/`tail` its last one. The
// last segments are combined across lanes with a segmented scan; a segment
// that continues into the next lane is written by the lane where it ends.
__device__ __forceinline__ void flush_lane_segments(int lane, int first_key, int tail_key,
                                                    float tail_part, float head_val, int nseg,
                                                    float* __restrict__ y) {
  const float tail = wave_seg_sum(tail_key, tail_part);
  const int prev_key = __shfl_up(tail_key, 1);
  const float prev_tail = __shfl_up(tail, 1);
  const int next_first = __shfl_down(first_key, 1);
  if (nseg >= 2) {
    const float c = (lane > 0 && prev_key == first_key) ? prev_tail : 0.0f;
    atomic_add_noret(y + first_key, head_val + c);
  }
  if (lane == kWave - 1 || next_first != tail_key) atomic_add_noret(y + tail_key, tail);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void read8(const int* p, int (&o)[kV]) {
  const int4 a = reinterpret_cast<const int4*>(p)[0], b = reinterpret_cast<const int4*>(p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
  o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}

}  // namespace dev
}  // namespace systec
