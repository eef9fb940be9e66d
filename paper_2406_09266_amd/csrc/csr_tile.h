// Merge-path tiles over a CSR matrix, shared by the one-shot kernels over
// the stored triangle (SSYMV, SYPRD, the Bellman-Ford update) and the plain
// CSR SpMV used as the comparison.
//
// The matrix is cut along its merge path (the row end offsets and the entry
// indices as one sequence of n + nnz items) into tiles of kTile = 512 items,
// so a wavefront's tile holds at most 512 entries and at most 512 rows
// whatever the row lengths. The tile's entries are read with coalesced loads
// and staged in LDS; lane l then takes entries 8l .. 8l+7. The row of each
// entry comes from row-start markers placed in LDS followed by a max-scan.
#pragma once

#include "common.h"
#include "wave_ops.h"

namespace systec {
namespace dev {

// Merge-path split (Merrill & Garland's merge-based CSR decomposition): the
// rows' end offsets and the entry indices form one sorted sequence of n + nnz
// items; diagonal d of it splits at the largest row i in [0, n] with
// rowptr[i] + i <= d. The wave searches cooperatively, 64 probes per step.
__device__ __forceinline__ int merge_split(const int32_t* __restrict__ rowptr, int n,
                                           int64_t d, int lane) {
  int lo = 0, hi = n + 1;  // f(lo) <= d; hi == n+1 or f(hi) > d
  while (hi - lo > 1) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int probe = lo + (lane + 1) * step;
    const bool le = probe < hi && static_cast<int64_t>(rowptr[probe]) + probe <= d;
    const int c = __popcll(__ballot(le));
    const int nlo = lo + c * step;
    hi = min(hi, lo + (c + 1) * step);
    lo = nlo;
  }
  return lo;
}

// The entries of one merge-path tile, lane-contiguous: lane l holds tile
// entries 8l .. 8l+7 (entries past the tile's end get val = 0 and the last
// row).
struct LaneEntries {
  int row[kV];
  int col[kV];
  float val[kV];
  int valid;  // number of valid entries of this lane (0..8)
  int count;  // entries of the tile (wave-uniform)
};

// Per-wave LDS staging: row-start markers and the tile's columns and values.
struct TileLds {
  int head[kTile];
  int col[kTile];
  float val[kTile];
};

// Loads merge-path tile `tile` (items [tile*kTile, (tile+1)*kTile) of the
// n + nnz sequence): at most kTile rows and kTile entries. Returns false if
// the tile holds no entry.
__device__ __forceinline__ bool load_tile_split(const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const float* __restrict__ val, int n, int nnz,
                                                int64_t tile, int i0, int i1, int lane,
                                                TileLds& S, LaneEntries& L);

__device__ __forceinline__ bool load_tile(const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ col,
                                          const float* __restrict__ val, int n, int nnz,
                                          int64_t tile, int lane, TileLds& S, LaneEntries& L) {
  const int64_t total = static_cast<int64_t>(n) + nnz;
  const int64_t d0 = tile * kTile;
  const int64_t d1 = min(d0 + kTile, total);
  return load_tile_split(rowptr, col, val, n, nnz, tile, merge_split(rowptr, n, d0, lane),
                         merge_split(rowptr, n, d1, lane), lane, S, L);
}

// load_tile with the tile's merge-path split rows given: i0 = the split of
// diagonal tile * kTile, i1 = that of the tile's end.
__device__ __forceinline__ bool load_tile_split(const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ col,
                                                const float* __restrict__ val, int n, int nnz,
                                                int64_t tile, int i0, int i1, int lane,
                                                TileLds& S, LaneEntries& L) {
  const int64_t total = static_cast<int64_t>(n) + nnz;
  const int64_t d0 = tile * kTile;
  const int64_t d1 = min(d0 + kTile, total);
  const int j0 = static_cast<int>(d0 - i0);
  const int j1 = static_cast<int>(d1 - i1);
  const int cnt = j1 - j0;  // 0..kTile
  if (cnt <= 0) return false;

  // row-start markers: head[p] = largest row whose first entry is j0 + p
  {
    int4* h4 = reinterpret_cast<int4*>(S.head + lane * kV);
    const int4 none = make_int4(-1, -1, -1, -1);
    h4[0] = none;
    h4[1] = none;
  }
  wave_sync();
  if (lane == 0) S.head[0] = i0;
  wave_sync();
  // rows (i0, i1] start at or after j0; at most kTile of them
  for (int r = i0 + 1 + lane; r <= i1; r += kWave) {
    const int s = rowptr[r];
    if (s < j1) atomicMax(S.head + (s - j0), r);
  }
  // coalesced loads of the tile's entries into LDS
#pragma unroll
  for (int q = 0; q < kV; ++q) {
    const int p = q * kWave + lane;
    if (p < cnt) {
      S.col[p] = __builtin_nontemporal_load(col + j0 + p);  // read once
      S.val[p] = __builtin_nontemporal_load(val + j0 + p);
    }
  }
  wave_sync();

  int h[kV];
  read8(S.head + lane * kV, h);
#pragma unroll
  for (int k = 1; k < kV; ++k) h[k] = max(h[k], h[k - 1]);
  // carry-in: the largest marker of all earlier lanes
  const int incl = wave_incl_max(h[kV - 1]);
  int carry = __shfl_up(incl, 1);
  if (lane == 0) carry = INT_MIN;
#pragma unroll
  for (int k = 0; k < kV; ++k) L.row[k] = max(h[k], carry);

  L.valid = max(0, min(kV, cnt - lane * kV));
  L.count = cnt;
  int c[kV];
  read8(S.col + lane * kV, c);
  const float* vp = S.val + lane * kV;
  const float4 va = reinterpret_cast<const float4*>(vp)[0];
  const float4 vb = reinterpret_cast<const float4*>(vp)[1];
  const float v[kV] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
#pragma unroll
  for (int k = 0; k < kV; ++k) {
    const bool ok = k < L.valid;
    L.col[k] = ok ? c[k] : L.row[k];
    L.val[k] = ok ? v[k] : 0.0f;
  }
  return true;
}

}  // namespace dev
}  // namespace systec
