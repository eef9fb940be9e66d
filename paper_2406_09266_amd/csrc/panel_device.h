// SSYMV over the panel format, as a workgroup-level device function shared
// by the standalone kernel and the serving step kernel.
#pragma once

#include "common.h"
#include "wave_ops.h"

namespace systec {
namespace dev {

// Copies src[0, count) to dst[0, H) in LDS, zero-filled past count, by the
// whole workgroup (the caller synchronizes). Each thread issues all its
// loads of a round before any of its LDS writes, so the copy pays about one
// memory round trip per round, where a load-then-write loop would pay one per
// element. A whole 16-byte-aligned slice moves in 16-byte pieces (H is a
// multiple of the elements per piece); a partial or unaligned one (the last
// panel) element by element.
template <typename XT>
__device__ __forceinline__ void stage_slice(const XT* __restrict__ src, int count, int H,
                                            XT* dst) {
  const int bd = static_cast<int>(blockDim.x);
  if (count >= H && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    constexpr int kPer = 16 / sizeof(XT);
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    const int pieces = H / kPer;
    for (int q = threadIdx.x; q < pieces; q += 2 * bd) {
      const bool two = q + bd < pieces;
      const uint4 a = s4[q];
      const uint4 b = two ? s4[q + bd] : uint4{};
      d4[q] = a;
      if (two) d4[q + bd] = b;
    }
    return;
  }
  constexpr int kU = 8;
  for (int i0 = threadIdx.x; i0 < H; i0 += kU * bd) {
    XT t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * bd;
      t[u] = i < count ? src[i] : XT(0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * bd;
      if (i < H) dst[i] = t[u];
    }
  }
}

// S steps of a tile's packed index and value streams from entry base (this
// lane's first entry), lane-strided: a step reads 64 consecutive entries
// (coalesced); the steps' base columns (from step0, wave-uniform) are
// scalar loads. Decoding waits for the loads, so it is left to
// decode_panel_steps, which the caller runs when the unit starts.
template <int S>
__device__ __forceinline__ void load_panel_steps(int64_t base, int64_t step0,
                                                 const uint32_t* __restrict__ ppack,
                                                 const int32_t* __restrict__ pbase,
                                                 const float* __restrict__ pval, uint32_t (&pk)[S],
                                                 int (&pb)[S], float (&a)[S]) {
#pragma unroll
  for (int k = 0; k < S; ++k) {
    pk[k] = __builtin_nontemporal_load(ppack + base + k * kWave);
    a[k] = __builtin_nontemporal_load(pval + base + k * kWave);
    pb[k] = pbase[step0 + k];
  }
}

// The column and panel row of each step's entry: base column plus offset
// and the low bits; a step whose base has bit 31 set (columns spanning more
// than the offsets hold, rare) reads them from pcol and prow instead.
template <int S>
__device__ __forceinline__ void decode_panel_steps(int64_t base, int hbits,
                                                   const int32_t* __restrict__ pcol,
                                                   const uint16_t* __restrict__ prow,
                                                   const uint32_t (&pk)[S], const int (&pb)[S],
                                                   int (&c)[S], int (&ro)[S]) {
  const uint32_t rmask = (1u << hbits) - 1;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    if (pb[k] >= 0) {
      c[k] = pb[k] + static_cast<int>(pk[k] >> hbits);
      ro[k] = static_cast<int>(pk[k] & rmask);
    } else {
      c[k] = pcol[base + k * kWave];
      ro[k] = prow[base + k * kWave];
    }
  }
}

// SSYMV over one chunk (tiles [tb, te) of panel p) of a matrix in the panel
// format (see plan.hip), by the whole workgroup, which it synchronizes. The
// panel's row sums live in LDS as FP32 (s_rows, H of them) and are flushed
// to y once per chunk. A row-side update is a compare-and-swap on the LDS
// word (read, add, ds_cmpst), which runs at the integer LDS atomic rate;
// gfx950 runs the LDS FP32 add (ds_add_f32) at about a tenth of that rate.
// A unit's attempts go out back to back before its column-side work and are
// checked after it, so their LDS round trip overlaps that work; an attempt
// that lost a race (another lane or wave changed the word in between, which
// happens on the hub rows) is finished with one ds_add_f32, so contended
// rows take the FP32 add and the rest take the integer pipeline.
// The entries arrive sorted
// by column and are taken lane-strided (step k of a wave holds 64 consecutive
// entries), so the column-side updates y[j] += a x[i] reduce across the wave
// by a segmented scan per step (its run structure is one ballot, and the
// scalar unit derives the scan's lane masks from it), and the segment totals
// leave in one atomic instruction whose lanes hold consecutive columns
// (coalesced into few cache lines). A segment running past the step carries
// into the next step; the carry is wave-uniform and moves through scalar
// registers (readlane), not through LDS, and enters the next step's scan at
// lane 0.
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
                                                  const uint32_t* __restrict__ ppack,
                                                  const int32_t* __restrict__ pbase,
                                                  const XT* __restrict__ x, float* __restrict__ y,
                                                  float* s_rows, XT* s_x = nullptr,
                                                  const int32_t* __restrict__ seg_tile0 = nullptr,
                                                  float* __restrict__ seg_out = nullptr) {
  const int r0 = p * H;
  // H is a power of two of at least 64 rows, so 16-byte pieces tile it
  for (int i = 4 * threadIdx.x; i < H; i += 4 * blockDim.x)
    *reinterpret_cast<float4*>(s_rows + i) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if constexpr (kStageX) stage_slice(x + r0, min(H, n - r0), H, s_x);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nw = blockDim.x / kWave;
  const int hbits = __builtin_ctz(static_cast<unsigned>(H));
  // the wave walks its tiles (tb + w, tb + w + nw, ...) in units of kSub
  // steps (half a tile, which keeps the registers of a unit, its prefetched
  // successor included, within 64 per lane); a unit's index and value
  // streams are loaded one unit ahead, behind the current unit's gathers, so
  // that waiting for the gathers does not wait for them and their latency
  // overlaps the unit's work
  constexpr int kSub = kV / 2;
  constexpr int kUnits = kV / kSub;
  const int first = tb + w;
  const int nunits = first < te ? (te - first + nw - 1) / nw * kUnits : 0;
  const auto unit_step = [&](int u) {  // the unit's first step
    return static_cast<int64_t>(first + (u / kUnits) * nw) * kV + (u % kUnits) * kSub;
  };
  uint32_t pk[kSub];
  int pb[kSub];
  float a[kSub];
  if (nunits > 0) load_panel_steps(unit_step(0) * kWave + lane, unit_step(0), ppack, pbase, pval, pk, pb, a);
  unsigned* const s_bits = reinterpret_cast<unsigned*>(s_rows);
  int carry_key = -1;
  float carry = 0.0f;
  // two-phase: the tile's first segment slot and the segments written so far
  // (wave-uniform)
  int seg0 = 0;
  int nseg = 0;
  for (int u = 0; u < nunits; ++u) {
    const int tile = first + (u / kUnits) * nw;
    const int part = u % kUnits;
    int c[kSub];
    int ro[kSub];
    decode_panel_steps(unit_step(u) * kWave + lane, hbits, pcol, prow, pk, pb, c, ro);
    // every gather of the unit is issued before the first update (a gather
    // behind a branch waits for all earlier memory operations, the atomics
    // included); padding entries point at a valid column of the panel, so
    // no gather needs a guard
    float xc[kSub];
    float xr[kSub];
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      xc[k] = load_f32(x, c[k]);
      xr[k] = kStageX ? load_f32(s_x, ro[k]) : load_f32(x, r0 + ro[k]);
    }
    // the next unit's streams (the last unit reloads itself: no branch)
    uint32_t pkn[kSub];
    int pbn[kSub];
    float an[kSub];
    const int un = u + 1 < nunits ? u + 1 : u;
    load_panel_steps(unit_step(un) * kWave + lane, unit_step(un), ppack, pbase, pval, pkn, pbn, an);
    if (part == 0) {  // a tile starts: no segment carried in
      carry_key = -1;
      carry = 0.0f;
      seg0 = kTwoPhase ? __builtin_amdgcn_readfirstlane(seg_tile0[tile]) : 0;
      nseg = 0;
    }
    // row side, y[i] += a x[j]: first compare-and-swap attempts, issued
    // without a branch so that they leave back to back (a zero product
    // swaps a word for itself)
    float rv[kSub];
    unsigned seen[kSub];
    unsigned got[kSub];
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      rv[k] = a[k] * xc[k];
      seen[k] = s_bits[ro[k]];
    }
#pragma unroll
    for (int k = 0; k < kSub; ++k)
      got[k] = atomicCAS(s_bits + ro[k], seen[k],
                         __float_as_uint(__uint_as_float(seen[k]) + rv[k]));
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      const int r = r0 + ro[k];
      float v = (c[k] != r) ? a[k] * xr[k] : 0.0f;  // y[j] += a x[i]
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
      // a continued segment's partial enters the scan at lane 0 (zero if none)
      v += lane == 0 ? carry : 0.0f;
      const uint64_t same = wave_same_as_prev(c[k]);
      const float seg = wave_seg_sum_runs(v, same);
      // lanes that end their segment inside the step (lane 63's is carried)
      const uint64_t ends = ~(same >> 1) & ~(uint64_t(1) << (kWave - 1));
      if constexpr (kTwoPhase) {
        const int below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(ends >> 32),
                                                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(ends), 0));
        if (lane_in(ends)) seg_out[seg0 + nseg + below] = seg;
        nseg += __popcll(ends);
      } else {
        if (lane_in(ends) && seg != 0.0f) atomic_add_noret(y + c[k], seg);
      }
      carry_key = __builtin_amdgcn_readlane(c[k], kWave - 1);
      carry = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(seg), kWave - 1));
    }
    // row side: an attempt that lost a race (another lane or wave changed the
    // word in between; mostly the hub rows) is finished with the LDS FP32 add
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      // the empty asm pins the check (and its wait for the attempt's result)
      // here, after the column side, instead of between the attempts
      asm volatile("" : "+v"(got[k])::"memory");
      if (got[k] != seen[k]) atomicAdd(s_rows + ro[k], rv[k]);
    }
    if (part == kUnits - 1) {  // the tile's last segment
      if constexpr (kTwoPhase) {
        if (lane == 0) seg_out[seg0 + nseg] = carry;
      } else {
        if (lane == 0 && carry != 0.0f) atomic_add_noret(y + carry_key, carry);
      }
    }
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      pk[k] = pkn[k];
      pb[k] = pbn[k];
      a[k] = an[k];
    }
  }
  __syncthreads();
  // the row sums, four LDS reads ahead of their atomics
  for (int i0 = threadIdx.x; i0 < H; i0 += 4 * blockDim.x) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * static_cast<int>(blockDim.x);
      v[u] = i < H ? s_rows[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * static_cast<int>(blockDim.x);
      if (v[u] != 0.0f && r0 + i < n) atomic_add_noret(y + r0 + i, v[u]);
    }
  }
}

}  // namespace dev
}  // namespace systec
