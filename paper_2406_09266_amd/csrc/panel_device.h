// SSYMV over the panel format, as a workgroup-level device function shared
// by the standalone kernel and the serving step kernel.
#pragma once

#include "common.h"
#include "wave_ops.h"

namespace systec {
namespace dev {

// SSYMV over one chunk (tiles [tb, te) of panel p) of a matrix in the panel
// format (see plan.hip), by the whole workgroup, which it synchronizes. The
// panel's row sums live in LDS (s_rows, H floats); the entries arrive sorted
// by column, so the column-side updates reduce by segments across each lane
// and wave before their atomic.
template <typename XT>
__device__ __forceinline__ void ssymv_panel_chunk(int n, int H, int p, int tb, int te,
                                                  const int32_t* __restrict__ pcol,
                                                  const uint16_t* __restrict__ prow,
                                                  const float* __restrict__ pval,
                                                  const XT* __restrict__ x, float* __restrict__ y,
                                                  float* s_rows) {
  const int r0 = p * H;
  for (int i = threadIdx.x; i < H; i += blockDim.x) s_rows[i] = 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int tile = tb + w; tile < te; tile += nw) {
    const int64_t base = static_cast<int64_t>(tile) * kTile + lane * kV;
    int c[kV];
    read8(pcol + base, c);
    const int4 rr = *reinterpret_cast<const int4*>(prow + base);
    const uint16_t ro[kV] = {
        static_cast<uint16_t>(rr.x & 0xffff), static_cast<uint16_t>(static_cast<uint32_t>(rr.x) >> 16),
        static_cast<uint16_t>(rr.y & 0xffff), static_cast<uint16_t>(static_cast<uint32_t>(rr.y) >> 16),
        static_cast<uint16_t>(rr.z & 0xffff), static_cast<uint16_t>(static_cast<uint32_t>(rr.z) >> 16),
        static_cast<uint16_t>(rr.w & 0xffff), static_cast<uint16_t>(static_cast<uint32_t>(rr.w) >> 16)};
    const float4 va = reinterpret_cast<const float4*>(pval + base)[0];
    const float4 vb = reinterpret_cast<const float4*>(pval + base)[1];
    const float a[kV] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};

    const int first_key = c[0];
    int cur = c[0];
    float acc = 0.0f, head_val = 0.0f;
    int nseg = 1;
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const int r = r0 + ro[k];
      if (a[k] != 0.0f) atomicAdd(s_rows + ro[k], a[k] * load_f32(x, c[k]));  // y[i] += a x[j]
      if (c[k] != cur) {
        if (nseg == 1) head_val = acc;
        else atomic_add_noret(y + cur, acc);
        ++nseg;
        cur = c[k];
        acc = 0.0f;
      }
      if (c[k] != r) acc += a[k] * load_f32(x, r);  // y[j] += a x[i], j > i
    }
    flush_lane_segments(lane, first_key, cur, acc, head_val, nseg, y);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    const float v = s_rows[i];
    if (v != 0.0f && r0 + i < n) atomic_add_noret(y + r0 + i, v);
  }
}

}  // namespace dev
}  // namespace systec
