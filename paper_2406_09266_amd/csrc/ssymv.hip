// SSYMV (y = A x) and SYPRD (s = x^T A x) over the stored upper triangle of a
// symmetric sparse matrix, and the plain CSR SpMV used as the comparison.
//
// Method (SySTeC, arXiv 2406.09266): a stored entry a = A[i,j], i <= j, is
// read once and serves both of its permutations: y[i] += a x[j] and, when
// i < j, y[j] += a x[i] (Sec. 3.1, "reusing canonical reads"). The row-side
// sums are accumulated in registers per row segment and written once per
// segment (the workspace transformation of Sec. 4.2.8); the column-side
// updates are scattered with FP32 atomics, which a parallel traversal of the
// canonical triangle needs (Sec. 7, parallelization). SYPRD gives an
// off-diagonal entry the factor 2 (Sec. 3.2.2, invisible output symmetry).
//
// GPU decomposition. The matrix is cut along its merge path (the row end
// offsets and the entry indices as one sequence of n + nnz items) into tiles
// of kTile = 512 items, so a wavefront's tile holds at most 512 entries and at
// most 512 rows whatever the row lengths (long hub rows and long runs of
// empty rows cost the same). The tile's entries are read with coalesced loads
// (the index and value streams are read exactly once) and staged in LDS; lane
// l then takes entries 8l .. 8l+7. The row of each entry comes from row-start
// markers placed in LDS followed by a max-scan. Each lane sums its entries
// sequentially by row; the wave combines the segments that cross lanes with a
// DPP segmented scan, so a row spanning a whole tile costs one atomic.
#include "common.h"
#include "csr_tile.h"
#include "panel_device.h"
#include "wave_ops.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kWaves = 4;             // wavefronts per workgroup
constexpr int kBlock = kWave * kWaves;

// y (+)= A x over one tile. kSym: the stored entries are the upper triangle
// and each off-diagonal entry also updates y[col].
template <typename XT, bool kSym>
__global__ __launch_bounds__(kBlock) void csr_tiles_kernel(int n, int nnz,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const float* __restrict__ val,
                                                         const XT* __restrict__ x,
                                                         float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) TileLds s_tile[kWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + w;
  if (tile * kTile >= static_cast<int64_t>(n) + nnz) return;  // wave-local sync only below
  LaneEntries L;
  if (!load_tile(rowptr, col, val, n, nnz, tile, lane, s_tile[w], L)) return;

  // lane-sequential segmented sums; interior segments are flushed here
  int first_key = L.row[0];
  int cur = L.row[0];
  float acc = 0.0f, head_val = 0.0f;
  int nseg = 1;
  float xr = load_f32(x, cur);
#pragma unroll
  for (int k = 0; k < kV; ++k) {
    const int r = L.row[k];
    if (r != cur) {
      if (nseg == 1) head_val = acc;
      else atomic_add_noret(y + cur, acc);
      ++nseg;
      cur = r;
      acc = 0.0f;
      if (kSym) xr = load_f32(x, cur);
    }
    if (k < L.valid) {
      const int c = L.col[k];
      const float a = L.val[k];
      acc += a * load_f32(x, c);
      if (kSym && c != r) atomic_add_noret(y + c, a * xr);
    }
  }
  flush_lane_segments(lane, first_key, cur, acc, head_val, nseg, y);
}

// SYPRD partial sums: one FP32 partial per workgroup.
template <typename XT>
__global__ __launch_bounds__(kBlock) void syprd_tiles_kernel(int n, int nnz,
                                                           const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ val,
                                                           const XT* __restrict__ x,
                                                           float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) TileLds s_tile[kWaves];
  __shared__ float s_part[kWaves];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t tile = static_cast<int64_t>(blockIdx.x) * kWaves + w;
  float sum = 0.0f;
  LaneEntries L;
  if (tile * kTile < static_cast<int64_t>(n) + nnz &&
      load_tile(rowptr, col, val, n, nnz, tile, lane, s_tile[w], L)) {
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      if (k < L.valid) {
        const int r = L.row[k], c = L.col[k];
        const float f = (r == c) ? 1.0f : 2.0f;
        sum += f * L.val[k] * load_f32(x, r) * load_f32(x, c);
      }
    }
  }
  sum = wave_sum(sum);
  if (lane == 0) s_part[w] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < kWaves; ++i) t += s_part[i];
    partial[blockIdx.x] = t;
  }
}

// Final reduction of the per-workgroup partials in FP64.
__global__ __launch_bounds__(1024) void reduce_partials_f64(const float* __restrict__ partial,
                                                          int count, double* __restrict__ out) {
  __shared__ double s[1024 / kWave];
  double t = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) t += static_cast<double>(partial[i]);
  for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x / kWave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int i = 0; i < static_cast<int>(blockDim.x) / kWave; ++i) u += s[i];
    out[0] = u;
  }
}

// kStageX: the panel's slice of x follows the row sums in LDS (H floats,
// then H elements of x).
template <typename XT, bool kStageX>
__global__ __launch_bounds__(kPanelThreads) void ssymv_panel_kernel(
    int n, int H, const int32_t* __restrict__ chunk_panel,
    const int32_t* __restrict__ chunk_tile_begin, const int32_t* __restrict__ chunk_tile_end,
    const int32_t* __restrict__ pcol, const uint16_t* __restrict__ prow,
    const float* __restrict__ pval, const uint32_t* __restrict__ ppack,
    const int32_t* __restrict__ pbase, const XT* __restrict__ x, float* __restrict__ y,
    const int32_t* __restrict__ seg_tile0, float* __restrict__ seg_out) {
  extern __shared__ float s_rows[];  // the panel's row sums
  const int chunk = blockIdx.x;
  ssymv_panel_chunk<XT, kStageX, true>(n, H, chunk_panel[chunk], chunk_tile_begin[chunk],
                                       chunk_tile_end[chunk], pcol, prow, pval, ppack, pbase, x,
                                       y, s_rows,
                                       reinterpret_cast<XT*>(s_rows + H), seg_tile0, seg_out);
}

// The second pass of the panel SSYMV, over the stored vertex order c:
// y[c] += the sums of column c's segments, in segment order, so the column
// side of the result does not depend on the schedule. (For a relabeled
// matrix the output permutation follows as its own gather: scattering y
// through the permutation here was slower, 0.252 against 0.248 ms per call
// at R-MAT scale 22.)
__global__ __launch_bounds__(256) void panel_colsum_kernel(int n, const int32_t* __restrict__ colptr,
                                                          const int32_t* __restrict__ seg_ids,
                                                          const float* __restrict__ seg_val,
                                                          float* __restrict__ y) {
  // one thread per column; its loads go out in groups (the slot ids of four
  // segments, then their sums, y beside the first ids) so that a column pays
  // about three memory round trips, not one per segment; the sums are still
  // added in slot order
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int k0 = colptr[c], k1 = colptr[c + 1];
  if (k1 == k0) return;
  const float y0 = y[c];
  float v = 0.0f;
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    const int i0 = seg_ids[k], i1 = seg_ids[k + 1], i2 = seg_ids[k + 2], i3 = seg_ids[k + 3];
    const float a0 = seg_val[i0], a1 = seg_val[i1], a2 = seg_val[i2], a3 = seg_val[i3];
    v = (((v + a0) + a1) + a2) + a3;
  }
  for (; k < k1; ++k) v += seg_val[seg_ids[k]];
  y[c] = y0 + v;
}

// SYPRD over the panel format: each stored entry gives a x[i] x[j], twice
// off the diagonal (the scalar of the symmetric product, Sec. 3.2.2), summed
// in FP32 per lane and wave, one FP32 partial per chunk (no scattered
// writes at all); the panel's slice of x is staged in LDS (H elements) for
// the row-side reads, as in the panel SSYMV.
template <typename XT>
__global__ __launch_bounds__(kPanelThreads) void syprd_panel_kernel(
    int n, int H, const int32_t* __restrict__ chunk_panel,
    const int32_t* __restrict__ chunk_tile_begin, const int32_t* __restrict__ chunk_tile_end,
    const int32_t* __restrict__ pcol, const uint16_t* __restrict__ prow,
    const float* __restrict__ pval, const uint32_t* __restrict__ ppack,
    const int32_t* __restrict__ pbase, const XT* __restrict__ x, float* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  XT* s_x = reinterpret_cast<XT*>(s_dyn);
  __shared__ float s_part[kPanelThreads / kWave];
  const int chunk = blockIdx.x;
  const int r0 = chunk_panel[chunk] * H;
  const int tb = chunk_tile_begin[chunk], te = chunk_tile_end[chunk];
  stage_slice(x + r0, min(H, n - r0), H, s_x);
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int nw = blockDim.x / kWave;
  const int hbits = __builtin_ctz(static_cast<unsigned>(H));
  // the wave's tiles in halves, the next half's streams loaded behind the
  // current half's gathers (as in the panel SSYMV)
  constexpr int kSub = kV / 2;
  constexpr int kUnits = kV / kSub;
  const int first = tb + w;
  const int nunits = first < te ? (te - first + nw - 1) / nw * kUnits : 0;
  const auto unit_step = [&](int u) {
    return static_cast<int64_t>(first + (u / kUnits) * nw) * kV + (u % kUnits) * kSub;
  };
  uint32_t pk[kSub];
  int pb[kSub];
  float a[kSub];
  if (nunits > 0)
    load_panel_steps(unit_step(0) * kWave + lane, unit_step(0), ppack, pbase, pval, pk, pb, a);
  float sum = 0.0f;
  for (int u = 0; u < nunits; ++u) {
    int c[kSub];
    int ro[kSub];
    decode_panel_steps(unit_step(u) * kWave + lane, hbits, pcol, prow, pk, pb, c, ro);
    float xc[kSub];
#pragma unroll
    for (int k = 0; k < kSub; ++k) xc[k] = load_f32(x, c[k]);  // padding: a valid position
    uint32_t pkn[kSub];
    int pbn[kSub];
    float an[kSub];
    const int un = u + 1 < nunits ? u + 1 : u;
    load_panel_steps(unit_step(un) * kWave + lane, unit_step(un), ppack, pbase, pval, pkn, pbn,
                     an);
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      const float f = c[k] != r0 + ro[k] ? 2.0f : 1.0f;
      sum += f * a[k] * load_f32(s_x, ro[k]) * xc[k];
    }
#pragma unroll
    for (int k = 0; k < kSub; ++k) {
      pk[k] = pkn[k];
      pb[k] = pbn[k];
      a[k] = an[k];
    }
  }
  sum = wave_sum(sum);
  if (lane == 0) s_part[w] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int i = 0; i < nw; ++i) t += s_part[i];
    partial[chunk] = t;
  }
}

// xp[i] = x[perm[i]] (the input in the prepared matrix's vertex order), and
// yp cleared unless it is null
template <typename XT>
__global__ void permute_in_kernel(int n, const int32_t* __restrict__ perm, const XT* __restrict__ x,
                                  XT* __restrict__ xp, float* __restrict__ yp) {
  // two elements per thread: both gathers in flight, and the index loads,
  // stores and clears of a wave 8 bytes a lane (n odd: the last one alone)
  const int stride = gridDim.x * blockDim.x;
  const int pairs = n / 2;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < pairs; k += stride) {
    const int2 p = reinterpret_cast<const int2*>(perm)[k];
    const XT a = x[p.x], b = x[p.y];
    xp[2 * k] = a;
    xp[2 * k + 1] = b;
    if (yp) reinterpret_cast<float2*>(yp)[k] = make_float2(0.0f, 0.0f);  // the panels accumulate
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    xp[n - 1] = x[perm[n - 1]];
    if (yp) yp[n - 1] = 0.0f;
  }
}

// y[j] = yp[inv[j]] (the output back in the caller's vertex order)
__global__ void permute_out_kernel(int n, const int32_t* __restrict__ inv,
                                   const float* __restrict__ yp, float* __restrict__ y) {
  const int stride = gridDim.x * blockDim.x;
  const int pairs = n / 2;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < pairs; k += stride) {
    const int2 q = reinterpret_cast<const int2*>(inv)[k];
    const float a = yp[q.x], b = yp[q.y];
    y[2 * k] = a;  // y is the caller's: 4-byte aligned only
    y[2 * k + 1] = b;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) y[n - 1] = yp[inv[n - 1]];
}

__global__ void fill_f32_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t k = i; k < n; k += stride) p[k] = 0.0f;
}

template <typename XT, bool kSym>
int launch_csr_typed(int n, int nnz, const int32_t* rowptr, const int32_t* col,
                     const float* val, const XT* x, float* y, hipStream_t s) {
  const int64_t tiles = (static_cast<int64_t>(n) + nnz + kTile - 1) / kTile;
  const int64_t blocks = (tiles + kWaves - 1) / kWaves;
  if (blocks == 0) return SYSTEC_OK;
  LaunchTimer timer(s);
  csr_tiles_kernel<XT, kSym><<<dim3(blocks), dim3(kBlock), 0, s>>>(n, nnz, rowptr, col, val, x, y);
  return check_launch(kSym ? "ssymv kernel" : "spmv kernel");
}

}  // namespace

int launch_fill_f32(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return SYSTEC_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  fill_f32_kernel<<<dim3(blocks), dim3(256), 0, s>>>(p, n);
  return check_launch("fill kernel");
}

int launch_ssymv(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, float* y, bool symmetric,
                 hipStream_t s) {
  int rc = launch_fill_f32(y, n, s);
  if (rc != SYSTEC_OK || nnz == 0) return rc;
  if (symmetric) {
    rc = launch_ssymv_bucketed(n, nnz, rowptr, col, val, x, xdt, y, s);
    if (rc != -1) return rc;
  }
  const int ni = static_cast<int>(n), nz = static_cast<int>(nnz);
  if (xdt == SYSTEC_F32) {
    const float* xf = static_cast<const float*>(x);
    return symmetric ? launch_csr_typed<float, true>(ni, nz, rowptr, col, val, xf, y, s)
                     : launch_csr_typed<float, false>(ni, nz, rowptr, col, val, xf, y, s);
  }
  const uint16_t* xb = static_cast<const uint16_t*>(x);
  return symmetric ? launch_csr_typed<uint16_t, true>(ni, nz, rowptr, col, val, xb, y, s)
                   : launch_csr_typed<uint16_t, false>(ni, nz, rowptr, col, val, xb, y, s);
}

namespace {

int64_t syprd_blocks(int64_t n, int64_t nnz) {
  const int64_t tiles = (n + nnz + kTile - 1) / kTile;
  return std::max<int64_t>(1, (tiles + kWaves - 1) / kWaves);
}

// The one-shot SYPRD into `partial` (one FP32 partial per workgroup, every
// one written) and its FP64 final sum.
int syprd_into(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
               const float* val, const void* x, systec_dtype xdt, double* out, float* partial,
               hipStream_t s) {
  const int64_t blocks = syprd_blocks(n, nnz);
  const int ni = static_cast<int>(n), nz = static_cast<int>(nnz);
  if (xdt == SYSTEC_F32)
    syprd_tiles_kernel<float><<<dim3(blocks), dim3(kBlock), 0, s>>>(
        ni, nz, rowptr, col, val, static_cast<const float*>(x), partial);
  else
    syprd_tiles_kernel<uint16_t><<<dim3(blocks), dim3(kBlock), 0, s>>>(
        ni, nz, rowptr, col, val, static_cast<const uint16_t*>(x), partial);
  int rc = check_launch("syprd kernel");
  if (rc == SYSTEC_OK) {
    reduce_partials_f64<<<dim3(1), dim3(1024), 0, s>>>(partial, static_cast<int>(blocks), out);
    rc = check_launch("syprd final reduction");
  }
  return rc;
}

// The scratch of the allocation-free SYPRD (systec_syprd_noalloc): room for
// the per-workgroup partials of n + nnz <= kNoAllocItems. Each device holds
// its own copy for the life of the process; in host code its name is only a
// stand-in, so kernels get the address from hipGetSymbolAddress.
constexpr int64_t kNoAllocPartials = int64_t(1) << 18;  // 1 MiB of FP32
constexpr int64_t kNoAllocItems = kNoAllocPartials * kTile * kWaves;
__device__ __align__(256) float scratch[kNoAllocPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The address of the current device's copy of `scratch`, looked up once
// per device with that device current.
int scratch_address(float** out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(SYSTEC_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return SYSTEC_OK;
}

}  // namespace

int launch_syprd(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, double* out,
                 hipStream_t s) {
  const int64_t blocks = syprd_blocks(n, nnz);
  float* partial = nullptr;
  int rc = check_hip(hipMallocAsync(reinterpret_cast<void**>(&partial), blocks * sizeof(float), s),
                     "hipMallocAsync(syprd partials)");
  if (rc != SYSTEC_OK) return rc;
  {
    LaunchTimer timer(s);
    rc = syprd_into(n, nnz, rowptr, col, val, x, xdt, out, partial, s);
  }
  const int rc2 = check_hip(hipFreeAsync(partial, s), "hipFreeAsync(syprd partials)");
  return rc != SYSTEC_OK ? rc : rc2;
}

int launch_syprd_noalloc(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                         const float* val, const void* x, systec_dtype xdt, double* out,
                         hipStream_t s) {
  if (n + nnz > kNoAllocItems)
    return fail(SYSTEC_EINVAL, "systec_syprd_noalloc: n + nnz exceeds the fixed scratch (" +
                                   std::to_string(kNoAllocItems) + ")");
  float* partial = nullptr;
  const int rc = scratch_address(&partial);
  return rc ? rc : syprd_into(n, nnz, rowptr, col, val, x, xdt, out, partial, s);
}

namespace {

// The two passes of the panel SSYMV over a prepared matrix in its own
// vertex order: the panel kernel (row sums into y, column segments into
// the handle's work_seg), then the column pass (see panel_colsum_kernel).
// The caller holds the work lease.
template <typename XT, bool kStageX>
int panel_launch(const Tensor* t, const XT* x, float* y, hipStream_t s) {
  const size_t H = static_cast<size_t>(t->panel_rows);
  const size_t lds = H * sizeof(float) + (kStageX ? H * sizeof(XT) : 0);
  const void* kern = reinterpret_cast<const void*>(ssymv_panel_kernel<XT, kStageX>);
  // more than the default 64 KiB of dynamic LDS
  const int rc = check_hip(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               static_cast<int>(lds)),
                           "hipFuncSetAttribute(dynamic LDS)");
  if (rc) return rc;
  if (t->nchunks == 0) return SYSTEC_OK;
  LaunchTimer timer(s);
  const int n = static_cast<int>(t->dim);
  ssymv_panel_kernel<XT, kStageX><<<dim3(t->nchunks), dim3(kPanelThreads), lds, s>>>(
      n, t->panel_rows, t->chunk_panel, t->chunk_tile_begin, t->chunk_tile_end, t->pcol,
      t->prow, t->pval, t->ppack, t->pbase, x, y, t->seg_tile0, t->work_seg);
  if (const int lrc = check_launch("ssymv panel kernel")) return lrc;
  panel_colsum_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, t->seg_colptr, t->seg_ids, t->work_seg,
                                                       y);
  return check_launch("ssymv panel column pass");
}

// y is cleared first unless the caller has done so (y_clear).
int panel_call(const Tensor* t, const void* x, systec_dtype xdt, float* y, bool y_clear,
               hipStream_t s) {
  int rc = y_clear ? SYSTEC_OK : launch_fill_f32(y, t->dim, s);
  if (rc != SYSTEC_OK) return rc;
  // the panel's slice of x goes to LDS beside the row sums when the device
  // allows that much per workgroup (8192 rows: 48 KiB with BF16 x, 64 KiB
  // with FP32 x)
  int dev = 0;
  int limit = 0;
  rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc)
    rc = check_hip(hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                   "hipDeviceGetAttribute(max shared memory)");
  if (rc) return rc;
  const size_t rows = static_cast<size_t>(t->panel_rows) * sizeof(float);
  if (xdt == SYSTEC_F32) {
    const float* xf = static_cast<const float*>(x);
    return rows + static_cast<size_t>(t->panel_rows) * sizeof(float) <= static_cast<size_t>(limit)
               ? panel_launch<float, true>(t, xf, y, s)
               : panel_launch<float, false>(t, xf, y, s);
  }
  const uint16_t* xb = static_cast<const uint16_t*>(x);
  return rows + static_cast<size_t>(t->panel_rows) * sizeof(uint16_t) <= static_cast<size_t>(limit)
             ? panel_launch<uint16_t, true>(t, xb, y, s)
             : panel_launch<uint16_t, false>(t, xb, y, s);
}

}  // namespace

int launch_permute_in(int n, const int32_t* perm, const void* x, systec_dtype xdt, void* xp,
                      float* yp, hipStream_t s) {
  if (n == 0) return SYSTEC_OK;
  const int grid = static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192));
  if (xdt == SYSTEC_F32)
    permute_in_kernel<float><<<grid, 256, 0, s>>>(n, perm, static_cast<const float*>(x),
                                                 static_cast<float*>(xp), yp);
  else
    permute_in_kernel<uint16_t><<<grid, 256, 0, s>>>(n, perm, static_cast<const uint16_t*>(x),
                                                    static_cast<uint16_t*>(xp), yp);
  return check_launch("ssymv input permutation");
}

int launch_permute_out(int n, const int32_t* inv, const float* yp, float* y, hipStream_t s) {
  if (n == 0) return SYSTEC_OK;
  const int grid = static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192));
  permute_out_kernel<<<grid, 256, 0, s>>>(n, inv, yp, y);
  return check_launch("ssymv output permutation");
}

namespace {

// The prepared SYPRD over a matrix in its own vertex order (x already in
// that order); the caller holds the work lease (per-chunk partials).
int syprd_panel_call(const Tensor* t, const void* x, systec_dtype xdt, double* out,
                     hipStream_t s) {
  const int nch = std::max(1, t->nchunks);
  float* partial = t->work_partial;
  int rc = SYSTEC_OK;
  if (t->nchunks == 0) {
    fill_f32_kernel<<<1, 64, 0, s>>>(partial, 1);
    rc = check_launch("syprd partial clear");
  } else {
    const size_t lds = static_cast<size_t>(t->panel_rows) * (xdt == SYSTEC_F32 ? 4 : 2);
    const void* kern = xdt == SYSTEC_F32
                           ? reinterpret_cast<const void*>(syprd_panel_kernel<float>)
                           : reinterpret_cast<const void*>(syprd_panel_kernel<uint16_t>);
    rc = check_hip(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds)),
                   "hipFuncSetAttribute(dynamic LDS)");
    if (!rc) {
      LaunchTimer timer(s);
      const int n = static_cast<int>(t->dim);
      if (xdt == SYSTEC_F32)
        syprd_panel_kernel<float><<<dim3(t->nchunks), dim3(kPanelThreads), lds, s>>>(
            n, t->panel_rows, t->chunk_panel, t->chunk_tile_begin, t->chunk_tile_end, t->pcol,
            t->prow, t->pval, t->ppack, t->pbase, static_cast<const float*>(x), partial);
      else
        syprd_panel_kernel<uint16_t><<<dim3(t->nchunks), dim3(kPanelThreads), lds, s>>>(
            n, t->panel_rows, t->chunk_panel, t->chunk_tile_begin, t->chunk_tile_end, t->pcol,
            t->prow, t->pval, t->ppack, t->pbase, static_cast<const uint16_t*>(x), partial);
      rc = check_launch("syprd panel kernel");
    }
  }
  if (!rc) {
    reduce_partials_f64<<<dim3(1), dim3(1024), 0, s>>>(partial, nch, out);
    rc = check_launch("syprd final reduction");
  }
  return rc;
}

}  // namespace

int launch_syprd_panel(const Tensor* t, const void* x, systec_dtype xdt, double* out,
                       hipStream_t s) {
  WorkLease lease(t, s);
  if (lease.status()) return lease.status();
  if (!t->relabeled || t->dim == 0) return syprd_panel_call(t, x, xdt, out, s);
  // relabeled matrix: s = x_p^T (P A P^T) x_p with x_p[i] = x[perm[i]]
  const int rc = launch_permute_in(static_cast<int>(t->dim), t->perm, x, xdt, t->work_x, nullptr, s);
  return rc ? rc : syprd_panel_call(t, t->work_x, xdt, out, s);
}

int launch_ssymv_panel_stored(const Tensor* t, const void* x, systec_dtype xdt, float* y,
                              hipStream_t s) {
  WorkLease lease(t, s);  // the column segments' buffer
  if (lease.status()) return lease.status();
  return panel_call(t, x, xdt, y, false, s);
}

int launch_syprd_panel_stored(const Tensor* t, const void* x, systec_dtype xdt, double* out,
                              hipStream_t s) {
  WorkLease lease(t, s);
  if (lease.status()) return lease.status();
  return syprd_panel_call(t, x, xdt, out, s);
}

int launch_ssymv_panel(const Tensor* t, const void* x, systec_dtype xdt, float* y,
                       hipStream_t s) {
  WorkLease lease(t, s);  // the column segments' buffer (and, relabeled, x and y)
  if (lease.status()) return lease.status();
  if (!t->relabeled) return panel_call(t, x, xdt, y, false, s);
  // relabeled matrix: x into the stored order (clearing the stored-order
  // output), the two passes, y back into the caller's order
  const int n = static_cast<int>(t->dim);
  if (n == 0) return SYSTEC_OK;
  int rc = launch_permute_in(n, t->perm, x, xdt, t->work_x, t->work_y, s);
  if (!rc) rc = panel_call(t, t->work_x, xdt, t->work_y, true, s);
  if (!rc) rc = launch_permute_out(n, t->inv, t->work_y, y, s);
  return rc;
}

}  // namespace systec
