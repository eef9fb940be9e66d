// Bellman-Ford update over a symmetric sparse matrix stored by its upper
// triangle: y[i] = min over the stored coordinates (i, j) of the full matrix
// of A[i,j] + d[j] (Sec. 5.2.2, the (min, +) form of SSYMV). A stored entry
// a = A[i,j], i <= j, is read once and serves both of its coordinates:
// y[i] min= a + d[j] and, when i < j, y[j] min= a + d[i] (Sec. 3.1, reusing
// canonical reads, with min in place of + and + in place of *). An index
// with no stored coordinate gets +inf, the identity of min.
//
// The minimum of FP32 values is resolved with integer atomics on an
// order-preserving map of the values to unsigned keys: the output is
// filled with the key of +inf, the kernels take atomic minima of keys, and a
// last pass turns the keys back into values in place. The keys make the
// result exact: it is the FP32 sum a + d of the minimizing coordinate,
// whatever the order of the updates.
//
// Two forms, as for SSYMV: one-shot over the canonical CSR (merge-path
// tiles, the row side as segmented minima in registers, the column side by
// one atomic per off-diagonal entry) and over a prepared matrix (panel
// format: the row side in LDS with integer LDS minima, which run at the full
// integer LDS atomic rate, the column side by segmented minima across the
// wave and one atomic per run of equal columns).
#include "common.h"
#include "csr_tile.h"
#include "panel_device.h"
#include "wave_ops.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kWaves = 4;
constexpr int kBlock = kWave * kWaves;
constexpr unsigned kKeyInf = 0xff800000u;  // the key of +inf

// Unsigned keys in the numeric order of the FP32 values: a non-negative
// value gets its bits with the top bit set, a negative one its bits
// inverted (so larger magnitudes sort lower).
__device__ __forceinline__ unsigned f2key(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key2f(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ __forceinline__ void atomic_min_key(unsigned* p, float v) {
  if (v != INFINITY) __hip_atomic_fetch_min(p, f2key(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void fill_key_inf_kernel(unsigned* __restrict__ y, int n) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = kKeyInf;
}

// y[i] = value of key[i], in place
__global__ void decode_keys_kernel(unsigned* __restrict__ y, int n) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    reinterpret_cast<float*>(y)[i] = key2f(y[i]);
}

// The segmented minima of the lanes' last segments, combined across the
// wave (the min form of flush_lane_segments).
__device__ __forceinline__ void flush_lane_minima(int lane, int first_key, int tail_key,
                                                  float tail_part, float head_val, int nseg,
                                                  unsigned* __restrict__ y) {
  const float tail = wave_seg_min(tail_key, tail_part);
  const int prev_key = __shfl_up(tail_key, 1);
  const float prev_tail = __shfl_up(tail, 1);
  const int next_first = __shfl_down(first_key, 1);
  if (nseg >= 2) {
    const float c = (lane > 0 && prev_key == first_key) ? prev_tail : INFINITY;
    atomic_min_key(y + first_key, fminf(head_val, c));
  }
  if (lane == kWave - 1 || next_first != tail_key) atomic_min_key(y + tail_key, tail);
}

// One merge-path tile of the canonical CSR.
__global__ __launch_bounds__(kBlock) void bf_tiles_kernel(int n, int nnz,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const float* __restrict__ val,
                                                        const float* __restrict__ d,
                                                        unsigned* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) TileLds s_tile[kWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + w;
  if (tile * kTile >= static_cast<int64_t>(n) + nnz) return;  // wave-local sync only below
  LaneEntries L;
  if (!load_tile(rowptr, col, val, n, nnz, tile, lane, s_tile[w], L)) return;
  // lane-sequential segment minima of the row side; interior segments are
  // written here
  const int first_key = L.row[0];
  int cur = L.row[0];
  float acc = INFINITY, head_val = INFINITY;
  int nseg = 1;
  float dr = d[cur];
#pragma unroll
  for (int k = 0; k < kV; ++k) {
    const int r = L.row[k];
    if (r != cur) {
      if (nseg == 1) head_val = acc;
      else atomic_min_key(y + cur, acc);
      ++nseg;
      cur = r;
      acc = INFINITY;
      dr = d[cur];
    }
    if (k < L.valid) {
      const int c = L.col[k];
      const float a = L.val[k];
      acc = fminf(acc, a + d[c]);                     // y[i] min= a + d[j]
      if (c != r) atomic_min_key(y + c, a + dr);      // y[j] min= a + d[i]
    }
  }
  flush_lane_minima(lane, first_key, cur, acc, head_val, nseg, y);
}

// One chunk of a prepared matrix (tiles [tb, te) of panel p; entries from
// vend on are padding). The panel's row minima are LDS keys (s_min, H of
// them); the panel's slice of d is staged beside them (s_d).
__global__ __launch_bounds__(kPanelThreads) void bf_panel_kernel(
    int n, int H, const int32_t* __restrict__ chunk_panel,
    const int32_t* __restrict__ chunk_tile_begin, const int32_t* __restrict__ chunk_tile_end,
    const int32_t* __restrict__ chunk_valid_end, const int32_t* __restrict__ pcol,
    const uint16_t* __restrict__ prow, const float* __restrict__ pval, const float* __restrict__ d,
    unsigned* __restrict__ y) {
  extern __shared__ unsigned s_min[];
  float* s_d = reinterpret_cast<float*>(s_min + H);
  const int chunk = blockIdx.x;
  const int r0 = chunk_panel[chunk] * H;
  const int tb = chunk_tile_begin[chunk], te = chunk_tile_end[chunk];
  const int64_t vend = chunk_valid_end[chunk];
  for (int i = threadIdx.x; i < H; i += blockDim.x) s_min[i] = kKeyInf;
  // the slice of d with every load of a thread issued before its LDS writes
  // (rows at or past n, zero-filled, hold no entries)
  stage_slice(d + r0, min(H, n - r0), H, s_d);
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
    float dc[kV];
#pragma unroll
    for (int k = 0; k < kV; ++k) dc[k] = d[c[k]];  // padding points at a valid position
    // row side, y[i] min= a + d[j]
#pragma unroll
    for (int k = 0; k < kV; ++k)
      if (base + k * kWave < vend) atomicMin(s_min + ro[k], f2key(a[k] + dc[k]));
    // column side, y[j] min= a + d[i]: segmented minima across the wave per
    // step, the last segment carried into the next step through readlane
    int carry_key = -1;
    float carry = INFINITY;
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const bool valid = base + k * kWave < vend;
      const float v = (valid && c[k] != r0 + ro[k]) ? a[k] + s_d[ro[k]] : INFINITY;
      if (__builtin_amdgcn_readlane(c[k], 0) != carry_key) {
        if (lane == 0) atomic_min_key(y + carry_key, carry);
        carry_key = -1;
        carry = INFINITY;
      }
      float seg = wave_seg_min(c[k], v);
      if (c[k] == carry_key) seg = fminf(seg, carry);  // only lanes of the first segment match
      const int next_key = next_lane_i32(c[k], -1);
      if (lane != kWave - 1 && next_key != c[k]) atomic_min_key(y + c[k], seg);
      carry_key = __builtin_amdgcn_readlane(c[k], kWave - 1);
      carry = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(seg), kWave - 1));
    }
    if (lane == 0) atomic_min_key(y + carry_key, carry);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H; i += blockDim.x)
    if (s_min[i] != kKeyInf && r0 + i < n)
      __hip_atomic_fetch_min(y + r0 + i, s_min[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// d'[i] = d[perm[i]] (distances in the stored vertex order), y' filled with
// the key of +inf
__global__ void bf_permute_in_kernel(int n, const int32_t* __restrict__ perm,
                                     const float* __restrict__ d, float* __restrict__ dp,
                                     unsigned* __restrict__ yp) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    dp[i] = d[perm[i]];
    yp[i] = kKeyInf;
  }
}

// y[j] = value of the key y'[inv[j]] (back in the caller's vertex order)
__global__ void bf_permute_out_kernel(int n, const int32_t* __restrict__ inv,
                                      const unsigned* __restrict__ yp, float* __restrict__ y) {
  const int stride = gridDim.x * blockDim.x;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) y[j] = key2f(yp[inv[j]]);
}

int grid_of(int64_t n) { return static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192)); }

int panel_minima(const Tensor* t, const float* d, unsigned* ykey, hipStream_t s) {
  if (t->nchunks == 0) return SYSTEC_OK;
  const size_t lds = static_cast<size_t>(t->panel_rows) * (sizeof(unsigned) + sizeof(float));
  int rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(bf_panel_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds)),
                     "hipFuncSetAttribute(dynamic LDS)");
  if (rc) return rc;
  LaunchTimer timer(s);
  bf_panel_kernel<<<dim3(t->nchunks), dim3(kPanelThreads), lds, s>>>(
      static_cast<int>(t->dim), t->panel_rows, t->chunk_panel, t->chunk_tile_begin,
      t->chunk_tile_end, t->chunk_valid_end, t->pcol, t->prow, t->pval, d, ykey);
  return check_launch("bellman-ford panel kernel");
}

}  // namespace

int launch_bellman_ford(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                        const float* val, const float* d, float* y, hipStream_t s) {
  unsigned* ykey = reinterpret_cast<unsigned*>(y);
  const int ni = static_cast<int>(n), nz = static_cast<int>(nnz);
  fill_key_inf_kernel<<<grid_of(n), 256, 0, s>>>(ykey, ni);
  int rc = check_launch("bellman-ford fill");
  if (!rc && nnz > 0) {
    const int64_t tiles = (n + nnz + kTile - 1) / kTile;
    const int64_t blocks = (tiles + kWaves - 1) / kWaves;
    LaunchTimer timer(s);
    bf_tiles_kernel<<<dim3(blocks), dim3(kBlock), 0, s>>>(ni, nz, rowptr, col, val, d, ykey);
    rc = check_launch("bellman-ford kernel");
  }
  if (!rc) {
    decode_keys_kernel<<<grid_of(n), 256, 0, s>>>(ykey, ni);
    rc = check_launch("bellman-ford decode");
  }
  return rc;
}

int launch_bellman_ford_panel(const Tensor* t, const float* d, float* y, hipStream_t s) {
  const int n = static_cast<int>(t->dim);
  if (!t->relabeled) {
    unsigned* ykey = reinterpret_cast<unsigned*>(y);
    fill_key_inf_kernel<<<grid_of(n), 256, 0, s>>>(ykey, n);
    int rc = check_launch("bellman-ford fill");
    if (!rc) rc = panel_minima(t, d, ykey, s);
    if (!rc) {
      decode_keys_kernel<<<grid_of(n), 256, 0, s>>>(ykey, n);
      rc = check_launch("bellman-ford decode");
    }
    return rc;
  }
  // relabeled matrix: d into the stored order, the panels, y back
  WorkLease lease(t, s);
  int rc = lease.status();
  float* dp = static_cast<float*>(t->work_x);
  unsigned* yp = reinterpret_cast<unsigned*>(t->work_y);
  if (!rc) {
    bf_permute_in_kernel<<<grid_of(n), 256, 0, s>>>(n, t->perm, d, dp, yp);
    rc = check_launch("bellman-ford input permutation");
  }
  if (!rc) rc = panel_minima(t, dp, yp, s);
  if (!rc) {
    bf_permute_out_kernel<<<grid_of(n), 256, 0, s>>>(n, t->inv, yp, y);
    rc = check_launch("bellman-ford output permutation");
  }
  return rc;
}

}  // namespace systec
