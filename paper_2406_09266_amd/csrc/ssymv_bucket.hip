// One-shot SSYMV over the stored upper triangle (canonical CSR) with the
// column side binned by column range instead of scattered with atomics.
//
// Method (SySTeC, arXiv 2406.09266): a stored entry a = A[i,j], i <= j,
// serves y[i] += a x[j] and, when i < j, y[j] += a x[i] (Sec. 3.1, reusing
// canonical reads). The row side is summed per row segment as in the
// merge-path kernel (Sec. 4.2.8). The column side y[j] += a x[i] is what a
// parallel traversal of the triangle has to scatter (Sec. 7); here it goes
// through a bucket pass instead of one device atomic per entry:
//
//   count    each workgroup counts its entries per bucket of 2^14 columns;
//   offsets  one exclusive scan over the (bucket, workgroup) counts gives
//            every workgroup a private range of each bucket;
//   bin      the merge-path kernel's row side as before, and each entry's
//            column update (its column within the bucket and a x[i] as
//            FP32, 8 bytes) written into its workgroup's range of its
//            bucket, the position from an LDS counter (one update per run
//            of consecutive entries in one bucket);
//   work     a list of (bucket, slice) items of at most kSlice entries;
//   sum      one workgroup per item adds its slice into 2^14 FP32 words of
//            LDS and adds the non-zero words to y (coalesced atomics).
//
// The scattered device atomics (one per off-diagonal entry, 34 M at R-MAT
// scale 22, each resolved at the memory side) become streaming writes and
// reads of 8 bytes per entry and LDS accumulation. The diagonal entries
// are binned with a zero update, so the count pass needs no row structure.
#include <hipcub/hipcub.hpp>

#include "common.h"
#include "csr_tile.h"
#include "wave_ops.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kBucketBits = 14;                 // columns per bucket: 16,384
constexpr int kBucketCols = 1 << kBucketBits;
constexpr int kMaxBuckets = 4096;               // n <= 2^26
constexpr int kBinWaves = 4;
constexpr int kBinThreads = kBinWaves * kWave;
constexpr int kTilesPerBlock = 8;               // merge-path tiles of 512 items per workgroup
constexpr int kSlice = 1 << 18;                 // entries per summing workgroup
constexpr int kSumThreads = 1024;

// Adds to counters[key] for the active lanes of a wave, one LDS atomic per
// run of lanes with equal keys (consecutive entries of one row fall in one
// bucket, so most instructions of a row touch one or two counters); returns
// each active lane's slot: the run's base plus its rank in the run.
__device__ __forceinline__ uint32_t run_atomic_add(uint32_t* counters, int key, bool active,
                                                   int lane) {
  const int prev = __shfl_up(key, 1);
  const bool head = active && (lane == 0 || prev != key);
  const uint64_t breaks = __ballot(head || !active);  // a run ends before the next break
  const uint64_t upto = (lane == kWave - 1) ? ~uint64_t(0) : ((uint64_t(2) << lane) - 1);
  const int head_lane = 63 - __clzll(breaks & upto);  // the lane's run head (itself if a head)
  const uint64_t after = breaks & ~upto;
  const int next = after ? __ffsll(static_cast<long long>(after)) - 1 : kWave;
  uint32_t base = 0;
  if (head) base = atomicAdd(counters + key, static_cast<uint32_t>(next - lane));
  base = __shfl(base, head_lane);
  return base + static_cast<uint32_t>(lane - head_lane);
}

// Per-workgroup bucket counts of the entries of its merge-path tiles,
// stored bucket-major: count[b * G + g].
// Also stores each tile's merge-path split row, split[t] for t <= tiles
// (split[tiles] = n), for the binning pass.
__global__ __launch_bounds__(kBinThreads) void bucket_count_kernel(
    int n, int nnz, int nbuckets, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, uint32_t* __restrict__ count, int32_t* __restrict__ split) {
  extern __shared__ uint32_t s_cnt[];  // nbuckets counters
  for (int b = threadIdx.x; b < nbuckets; b += kBinThreads) s_cnt[b] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t total = static_cast<int64_t>(n) + nnz;
  for (int k = w; k < kTilesPerBlock; k += kBinWaves) {
    const int64_t tile = static_cast<int64_t>(blockIdx.x) * kTilesPerBlock + k;
    const int64_t d0 = tile * kTile;
    if (d0 >= total) break;  // wave-uniform
    const int64_t d1 = min(d0 + kTile, total);
    const int i0 = merge_split(rowptr, n, d0, lane);
    const int i1 = merge_split(rowptr, n, d1, lane);
    if (lane == 0) {
      split[tile] = i0;
      if (d1 == total) split[tile + 1] = i1;  // the last tile
    }
    const int j0 = static_cast<int>(d0 - i0);
    const int cnt = static_cast<int>(d1 - i1) - j0;  // at most kTile entries
    // all of the tile's column loads first, then the counter updates (a
    // load behind each update would wait for it)
    int cc[kV];
#pragma unroll
    for (int q = 0; q < kV; ++q) {
      const int p = q * kWave + lane;
      cc[q] = p < cnt ? col[j0 + p] : -1;
    }
#pragma unroll
    for (int q = 0; q < kV; ++q) {
      if (q * kWave >= cnt) break;  // wave-uniform
      // columns outside [0, n) are left out, as in the binning pass
      const bool ok = static_cast<unsigned>(cc[q]) < static_cast<unsigned>(n);
      run_atomic_add(s_cnt, ok ? (cc[q] >> kBucketBits) : -1, ok, lane);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbuckets; b += kBinThreads)
    count[static_cast<int64_t>(b) * gridDim.x + blockIdx.x] = s_cnt[b];
}

// The merge-path SSYMV tiles of one workgroup: row side as in the
// one-shot kernel, column side binned (see the file comment).
template <typename XT>
__global__ __launch_bounds__(kBinThreads) void bucket_bin_kernel(
    int n, int nnz, int nbuckets, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const float* __restrict__ val, const XT* __restrict__ x,
    const uint32_t* __restrict__ offset, const int32_t* __restrict__ split,
    uint2* __restrict__ out, float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) TileLds s_tile[kBinWaves];
  extern __shared__ uint32_t s_pos[];  // nbuckets counters
  for (int b = threadIdx.x; b < nbuckets; b += kBinThreads)
    s_pos[b] = offset[static_cast<int64_t>(b) * gridDim.x + blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t total = static_cast<int64_t>(n) + nnz;
  for (int k = w; k < kTilesPerBlock; k += kBinWaves) {
    const int64_t tile = static_cast<int64_t>(blockIdx.x) * kTilesPerBlock + k;
    if (tile * kTile >= total) break;  // wave-uniform
    LaneEntries L;
    const int i0 = __builtin_amdgcn_readfirstlane(split[tile]);
    const int i1 = __builtin_amdgcn_readfirstlane(split[tile + 1]);
    if (!load_tile_split(rowptr, col, val, n, nnz, tile, i0, i1, lane, s_tile[w], L)) continue;
    int first_key = L.row[0];
    int cur = L.row[0];
    float acc = 0.0f, head_val = 0.0f;
    int nseg = 1;
    float xr = load_f32(x, cur);
    float u[kV];  // the entries' column updates
#pragma unroll
    for (int q = 0; q < kV; ++q) {
      const int r = L.row[q];
      if (r != cur) {
        if (nseg == 1) head_val = acc;
        else atomic_add_noret(y + cur, acc);
        ++nseg;
        cur = r;
        acc = 0.0f;
        xr = load_f32(x, cur);
      }
      const int c = L.col[q];
      const float a = L.val[q];  // 0 past the tile's end
      acc += a * load_f32(x, c);
      u[q] = c != r ? a * xr : 0.0f;
    }
    flush_lane_segments(lane, first_key, cur, acc, head_val, nseg, y);
    // the updates replace the entries' values in the tile's LDS (the lane's
    // own eight words, two 16-byte writes)
    {
      float4* v4 = reinterpret_cast<float4*>(s_tile[w].val + lane * kV);
      v4[0] = make_float4(u[0], u[1], u[2], u[3]);
      v4[1] = make_float4(u[4], u[5], u[6], u[7]);
    }
    wave_sync();
    // column side in entry order, 64 consecutive entries per step: runs of
    // one row fall in one bucket, so a run takes one counter update and its
    // lanes write consecutive slots
    const int cnt = __builtin_amdgcn_readfirstlane(L.count);
    for (int p0 = 0; p0 < cnt; p0 += kWave) {  // wave-uniform
      const int p = p0 + lane;
      const int c = p < cnt ? s_tile[w].col[p] : -1;
      // a column outside [0, n) (input that was not validated) is left out
      // here and in the count, so no write leaves its range
      const bool ok = static_cast<unsigned>(c) < static_cast<unsigned>(n);
      const uint32_t pos = run_atomic_add(s_pos, ok ? (c >> kBucketBits) : -1, ok, lane);
      if (ok)
        out[pos] = make_uint2(static_cast<uint32_t>(c & (kBucketCols - 1)),
                              __float_as_uint(s_tile[w].val[p]));
    }
    wave_sync();  // the tile's LDS is reused by the next tile
  }
}

// The (bucket, slice) work items: bucket b's entries are [offset[b * G],
// offset[(b + 1) * G]); item i = (b, begin, end). One workgroup.
__global__ __launch_bounds__(1024) void bucket_work_kernel(int nbuckets, int G,
                                                           const uint32_t* __restrict__ count,
                                                           const uint32_t* __restrict__ offset,
                                                           int4* __restrict__ items,
                                                           int* __restrict__ nitems) {
  __shared__ int s_first[kMaxBuckets + 1];
  // entries binned in all (the stored entries whose column is in range)
  const int64_t last = static_cast<int64_t>(nbuckets) * G - 1;
  const int64_t nnz = static_cast<int64_t>(offset[last]) + count[last];
  // slices per bucket, then an exclusive scan over the buckets in LDS
  for (int b = threadIdx.x; b < nbuckets; b += blockDim.x) {
    const int64_t lo = offset[static_cast<int64_t>(b) * G];
    const int64_t hi = b + 1 < nbuckets ? offset[static_cast<int64_t>(b + 1) * G] : nnz;
    s_first[b + 1] = static_cast<int>((hi - lo + kSlice - 1) / kSlice);
  }
  if (threadIdx.x == 0) s_first[0] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int b = 1; b <= nbuckets; ++b) s_first[b] += s_first[b - 1];  // LDS only
    *nitems = s_first[nbuckets];
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbuckets; b += blockDim.x) {
    const int64_t lo = offset[static_cast<int64_t>(b) * G];
    const int64_t hi = b + 1 < nbuckets ? offset[static_cast<int64_t>(b + 1) * G] : nnz;
    for (int i = s_first[b]; i < s_first[b + 1]; ++i) {
      const int64_t s0 = lo + static_cast<int64_t>(i - s_first[b]) * kSlice;
      items[i] = make_int4(b, static_cast<int>(s0), static_cast<int>(min(hi, s0 + kSlice)), 0);
    }
  }
}

// Adds one slice of a bucket into LDS (one compare-and-swap attempt per
// update, the FP32 LDS add when it loses a race) and its non-zero words to y.
__global__ __launch_bounds__(kSumThreads) void bucket_sum_kernel(int n,
                                                                const int4* __restrict__ items,
                                                                const int* __restrict__ nitems,
                                                                const uint2* __restrict__ binned,
                                                                float* __restrict__ y) {
  __shared__ float s_sum[kBucketCols];
  if (static_cast<int>(blockIdx.x) >= *nitems) return;  // whole workgroup
  const int4 it = items[blockIdx.x];
  for (int i = threadIdx.x; i < kBucketCols; i += kSumThreads) s_sum[i] = 0.0f;
  __syncthreads();
  unsigned* const s_bits = reinterpret_cast<unsigned*>(s_sum);
  // four entries per thread in flight: their loads first, then the updates
  constexpr int kU = 4;
  for (int e0 = it.y; e0 < it.z; e0 += kU * kSumThreads) {
    uint2 u[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      const int e = e0 + q * kSumThreads + static_cast<int>(threadIdx.x);
      u[q] = e < it.z ? binned[e] : make_uint2(0u, 0u);  // a zero update of word 0
    }
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      const int c = static_cast<int>(u[q].x);
      const float v = __uint_as_float(u[q].y);
      const unsigned seen = s_bits[c];
      const unsigned got = atomicCAS(s_bits + c, seen, __float_as_uint(__uint_as_float(seen) + v));
      if (got != seen) atomicAdd(s_sum + c, v);
    }
  }
  __syncthreads();
  const int base = it.x << kBucketBits;
  for (int i = threadIdx.x; i < kBucketCols; i += kSumThreads) {
    const float v = s_sum[i];
    if (v != 0.0f && base + i < n) atomic_add_noret(y + base + i, v);
  }
}

int exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count, void* tmp, size_t& tmp_bytes,
                       hipStream_t s) {
  return check_hip(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out,
                                                     static_cast<int>(count), s),
                   "bucket offsets scan");
}

template <typename XT>
int bucketed(int n, int nnz, const int32_t* rowptr, const int32_t* col, const float* val,
             const XT* x, float* y, hipStream_t s) {
  const int nbuckets = (n + kBucketCols - 1) / kBucketCols;
  const int64_t tiles = (static_cast<int64_t>(n) + nnz + kTile - 1) / kTile;
  const int G = static_cast<int>((tiles + kTilesPerBlock - 1) / kTilesPerBlock);
  const int64_t ncount = static_cast<int64_t>(nbuckets) * G;
  const int max_items = static_cast<int>(nnz / kSlice) + nbuckets + 1;
  size_t scan_bytes = 0;
  int rc = exclusive_scan_u32(nullptr, nullptr, ncount, nullptr, scan_bytes, s);
  if (rc) return rc;
  // one stream-ordered scratch block: counts, offsets, items, the item
  // count, the scan's temporary and the binned updates
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t b_count = up(ncount * 4), b_items = up(static_cast<size_t>(max_items) * 16),
               b_n = up(4), b_scan = up(scan_bytes), b_bin = up(static_cast<size_t>(nnz) * 8);
  const size_t b_split = up(static_cast<size_t>(tiles + 1) * 4);
  const size_t bytes = 2 * b_count + b_items + b_n + b_scan + b_bin + b_split;
  unsigned char* scratch = nullptr;
  const hipError_t ae = hipMallocAsync(reinterpret_cast<void**>(&scratch), bytes, s);
  if (ae != hipSuccess)
    return fail(SYSTEC_ENOMEM, std::string("hipMallocAsync(ssymv bucket scratch): ") +
                                   hipGetErrorString(ae));
  auto* count = reinterpret_cast<uint32_t*>(scratch);
  auto* offset = reinterpret_cast<uint32_t*>(scratch + b_count);
  auto* items = reinterpret_cast<int4*>(scratch + 2 * b_count);
  auto* nitems = reinterpret_cast<int*>(scratch + 2 * b_count + b_items);
  void* scan_tmp = scratch + 2 * b_count + b_items + b_n;
  auto* binned = reinterpret_cast<uint2*>(scratch + 2 * b_count + b_items + b_n + b_scan);
  auto* split = reinterpret_cast<int32_t*>(scratch + 2 * b_count + b_items + b_n + b_scan + b_bin);
  {
    LaunchTimer timer(s);
    const size_t lds = static_cast<size_t>(nbuckets) * sizeof(uint32_t);
    bucket_count_kernel<<<G, kBinThreads, lds, s>>>(n, nnz, nbuckets, rowptr, col, count, split);
    rc = check_launch("ssymv bucket count");
    if (!rc) rc = exclusive_scan_u32(count, offset, ncount, scan_tmp, scan_bytes, s);
    if (!rc) {
      bucket_bin_kernel<XT><<<G, kBinThreads, lds, s>>>(n, nnz, nbuckets, rowptr, col, val, x,
                                                      offset, split, binned, y);
      rc = check_launch("ssymv bucket bin");
    }
    if (!rc) {
      bucket_work_kernel<<<1, 1024, 0, s>>>(nbuckets, G, count, offset, items, nitems);
      rc = check_launch("ssymv bucket work list");
    }
    if (!rc) {
      bucket_sum_kernel<<<max_items, kSumThreads, 0, s>>>(n, items, nitems, binned, y);
      rc = check_launch("ssymv bucket sum");
    }
  }
  const int frc = check_hip(hipFreeAsync(scratch, s), "hipFreeAsync(ssymv bucket scratch)");
  return rc ? rc : frc;
}

}  // namespace

int launch_ssymv_bucketed(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                          const float* val, const void* x, systec_dtype xdt, float* y,
                          hipStream_t s) {
  // above 2^26 rows the buckets' counters outgrow the workgroup's LDS; small
  // matrices keep the single-kernel form
  if (n > static_cast<int64_t>(kMaxBuckets) * kBucketCols || nnz < kBucketNnzMin) return -1;
  const int ni = static_cast<int>(n), nz = static_cast<int>(nnz);
  return xdt == SYSTEC_F32
             ? bucketed<float>(ni, nz, rowptr, col, val, static_cast<const float*>(x), y, s)
             : bucketed<uint16_t>(ni, nz, rowptr, col, val, static_cast<const uint16_t*>(x), y, s);
}

}  // namespace systec
