// SSYMV over the panel format, as a workgroup-level device function shared
// by the standalone kernel and the serving step kernel.
#pragma once

#include "common.h"
#include "wave_ops.h"

namespace systec {
namespace dev {

// SSYMV over one chunk (tiles [tb, te) of panel p) of a matrix in the panel
// format (see plan.hip), by the whole workgroup, which it synchronizes. The
// panel's row sums live in LDS as FP32 (s_rows, H of them) and are flushed
// to y once per chunk. A row-side update is a compare-and-swap on the LDS
// word (read, add, ds_cmpst), which runs at the integer LDS atomic rate;
// gfx950 runs the LDS FP32 add (ds_add_f32) at about a tenth of that rate.
// A tile's attempts go out back to back before its column-side work and are
// checked after it, so their LDS round trip overlaps that work; an attempt
// that lost a race (another lane or wave changed the word in between, which
// happens on the hub rows) is finished with one ds_add_f32, so contended
// rows take the FP32 add and the rest take the integer pipeline.
// The entries arrive sorted
// by column and are taken lane-strided (step k of a wave holds 64 consecutive
// entries), so the column-side updates y[j] += a x[i] reduce across the wave
// by a segmented scan per step, and the segment totals leave in one atomic
// instruction whose lanes hold consecutive columns (coalesced into few cache
// lines). A segment running past the step carries into the next step; the
// carry is wave-uniform and moves through scalar registers (readlane), not
// through LDS.
// With kStageX the panel's slice of x (H elements) is copied to s_x first and
// the row-side gathers x[i] read LDS: their rows are scattered over the
// panel, so from global memory each such wave load touches up to 64 cache
// lines and the L1 tag lookups, not HBM, set the pace.
// With kTwoPhase a segment total is not added to y: segment k of tile t (the
// k-th run of equal columns in the tile, in entry order) is stored to
// seg_out[seg_tile0[t] + k], and a second pass adds each column's segments.
// The stores of one step go to consecutive words, where the atomics went to
// scattered cache lines, each resolved at the memory side.
template <typename XT, bool kStageX = false, bool kTwoPhase = false>
__device__ __forceinline__ void ssymv_panel_chunk(int n, int H, int p, int tb, int te,
                                                  const int32_t* __restrict__ pcol,
                                                  const uint16_t* __restrict__ prow,
                                                  const float* __restrict__ pval,
                                                  const XT* __restrict__ x, float* __restrict__ y,
                                                  float* s_rows, XT* s_x = nullptr,
                                                  const int32_t* __restrict__ seg_tile0 = nullptr,
                                                  float* __restrict__ seg_out = nullptr) {
  const int r0 = p * H;
  for (int i = threadIdx.x; i < H; i += blockDim.x) s_rows[i] = 0.0f;
  if constexpr (kStageX) {
    for (int i = threadIdx.x; i < H; i += blockDim.x)
      s_x[i] = r0 + i < n ? x[r0 + i] : XT(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int tile = tb + w; tile < te; tile += nw) {
    const int64_t base = static_cast<int64_t>(tile) * kTile + lane;
    int c[kV];
    int ro[kV];
    float a[kV];
#pragma unroll
    for (int k = 0; k < kV; ++k) {  // coalesced: a step reads 64 consecutive entries
      c[k] = pcol[base + k * kWave];
      ro[k] = prow[base + k * kWave];
      a[k] = pval[base + k * kWave];
    }
    // every gather of the tile is issued before the first update (a gather
    // behind a branch waits for all earlier memory operations, the atomics
    // included); padding entries point at a valid diagonal position, so no
    // gather needs a guard
    float xc[kV];
    float xr[kV];
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      xc[k] = load_f32(x, c[k]);
      xr[k] = kStageX ? load_f32(s_x, ro[k]) : load_f32(x, r0 + ro[k]);
    }
    // row side, y[i] += a x[j]: first compare-and-swap attempts, issued
    // without a branch so that they leave back to back (a zero product
    // swaps a word for itself)
    unsigned* const s_bits = reinterpret_cast<unsigned*>(s_rows);
    float rv[kV];
    unsigned seen[kV];
    unsigned got[kV];
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      rv[k] = a[k] * xc[k];
      seen[k] = s_bits[ro[k]];
    }
#pragma unroll
    for (int k = 0; k < kV; ++k)
      got[k] = atomicCAS(s_bits + ro[k], seen[k],
                         __float_as_uint(__uint_as_float(seen[k]) + rv[k]));
    int carry_key = -1;
    float carry = 0.0f;
    // two-phase: the tile's first segment slot and the segments written so
    // far (wave-uniform)
    const int seg0 = kTwoPhase ? __builtin_amdgcn_readfirstlane(seg_tile0[tile]) : 0;
    int nseg = 0;
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const int r = r0 + ro[k];
      const float v = (c[k] != r) ? a[k] * xr[k] : 0.0f;  // y[j] += a x[i]
      // the previous step's last segment either continues in lane 0 here or
      // is complete and must be written now
      if (__builtin_amdgcn_readlane(c[k], 0) != carry_key) {
        if constexpr (kTwoPhase) {
          if (carry_key != -1) {
            if (lane == 0) seg_out[seg0 + nseg] = carry;
            ++nseg;
          }
        } else {
          if (lane == 0 && carry != 0.0f) atomic_add_noret(y + carry_key, carry);
        }
        carry_key = -1;
        carry = 0.0f;
      }
      float seg = wave_seg_sum(c[k], v);
      if (c[k] == carry_key) seg += carry;  // only lanes of the first segment match
      const int next_key = next_lane_i32(c[k], -1);
      const bool ends = lane != kWave - 1 && next_key != c[k];
      if constexpr (kTwoPhase) {
        const uint64_t m = __ballot(ends);
        const int below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
        if (ends) seg_out[seg0 + nseg + below] = seg;
        nseg += __popcll(m);
      } else {
        if (ends && seg != 0.0f) atomic_add_noret(y + c[k], seg);
      }
      carry_key = __builtin_amdgcn_readlane(c[k], kWave - 1);
      carry = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(seg), kWave - 1));
    }
    // row side: an attempt that lost a race (another lane or wave changed the
    // word in between; mostly the hub rows) is finished with the LDS FP32 add
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      // the empty asm pins the check (and its wait for the attempt's result)
      // here, after the column side, instead of between the attempts
      asm volatile("" : "+v"(got[k])::"memory");
      if (got[k] != seen[k]) atomicAdd(s_rows + ro[k], rv[k]);
    }
    if constexpr (kTwoPhase) {
      if (lane == 0) seg_out[seg0 + nseg] = carry;  // the tile's last segment
    } else {
      if (lane == 0 && carry != 0.0f) atomic_add_noret(y + carry_key, carry);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    const float v = s_rows[i];
    if (v != 0.0f && r0 + i < n) atomic_add_noret(y + r0 + i, v);
  }
}

}  // namespace dev
}  // namespace systec
