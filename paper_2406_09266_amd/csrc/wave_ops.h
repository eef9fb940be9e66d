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

// DPP move whose lanes without a source read zero (bound_ctrl), so that the
// compiler can fold it into the consuming add.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_f32_zero(float src) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(src), kCtrl, kRowMask, 0xf, true));
}

// The lanes b, b + 1, ... that continue the run of lane b - 1 (at most w of
// them), as a lane mask: the run of set bits of `same` from bit b.
__device__ __forceinline__ uint64_t run_from(uint64_t same, int b, int w) {
  const uint64_t x = ~(same >> b);  // nonzero for b >= 1
  const int len = min(__builtin_ctzll(x), w);
  return ((uint64_t(1) << len) - 1) << b;
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

// Whether this lane belongs to a wave-uniform 64-bit lane mask; the compiler
// uses the mask's scalar registers as the lane condition directly.
__device__ __forceinline__ bool lane_in(uint64_t m) {
  return __builtin_amdgcn_inverse_ballot_w64(m);
}

// The run structure of keys that are nondecreasing across the wave: bit l is
// set when lane l holds the same key as lane l - 1 (bit 0 is clear).
__device__ __forceinline__ uint64_t wave_same_as_prev(int key) {
  const int prev = dpp_i32<0x138, 0xf>(~key, key);  // wave_shr:1; lane 0 keeps ~key
  return __ballot(prev == key);
}

// Inclusive segmented sum over the 64 lanes for nondecreasing keys whose run
// structure is `same` (wave_same_as_prev): the same result as wave_seg_sum,
// with the key comparisons made once, on the scalar unit. At distance d a
// lane hands its partial sum to the lane d above it only when the two hold
// one key (bit s of m: lanes s and s + d share a key), so each level is one
// select and one DPP add with zero fill; distances that no run within a row
// of 16 lanes needs are skipped, and so are the two cross-row steps when no
// run crosses the boundary they serve.
__device__ __forceinline__ float wave_seg_sum_runs(float v, uint64_t same) {
  constexpr uint64_t kIn1 = 0x7fff7fff7fff7fffull;  // lanes s with s % 16 + d < 16
  constexpr uint64_t kIn2 = 0x3fff3fff3fff3fffull;
  constexpr uint64_t kIn4 = 0x0fff0fff0fff0fffull;
  constexpr uint64_t kIn8 = 0x00ff00ff00ff00ffull;
  uint64_t m = same >> 1;
  if (m == 0) return v;  // no two lanes share a key
  if (m & kIn1) {
    v += dpp_f32_zero<0x111, 0xf>(lane_in(m) ? v : 0.0f);
    m &= m >> 1;
    if (m & kIn2) {
      v += dpp_f32_zero<0x112, 0xf>(lane_in(m) ? v : 0.0f);
      m &= m >> 2;
      if (m & kIn4) {
        v += dpp_f32_zero<0x114, 0xf>(lane_in(m) ? v : 0.0f);
        m &= m >> 4;
        if (m & kIn8) v += dpp_f32_zero<0x118, 0xf>(lane_in(m) ? v : 0.0f);
      }
    }
  }
  // runs that cross a row boundary: the lanes of rows 1 and 3 that continue
  // the run of lane 15 (47) take its partial (row_bcast:15), then the lanes of
  // rows 2 and 3 that continue the run of lane 31 take its partial
  // (row_bcast:31)
  const uint64_t b15 = run_from(same, 16, 16) | run_from(same, 48, 16);
  if (b15) {
    const float t = dpp_f32<0x142, 0xa>(0.0f, v);
    v += lane_in(b15) ? t : 0.0f;
  }
  const uint64_t b31 = run_from(same, 32, 32);
  if (b31) {
    const float t = dpp_f32<0x143, 0xc>(0.0f, v);
    v += lane_in(b31) ? t : 0.0f;
  }
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
