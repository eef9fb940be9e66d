// Symmetric MTTKRP over the slot views of a prepared tensor with the factor
// rows staged in LDS, for index spaces small enough that a column slice of B
// fits one workgroup's LDS (the 5-D workload, I = 5,000: all 16 BF16 columns
// are 160,000 bytes).
//
// Same updates as the view kernel (Sec. 4.3; per-run coefficients of the
// simplicial lookup table, Sec. 4.2.5; distributive grouping, Sec. 4.2.7):
// view t lists the entries whose slot t starts a run, sorted by c_t, and each
// adds coef[mask][t] * v * prod_{s != t} B[c_s, :] to C[c_t, :]. Here every
// factor-row read is an LDS read, and the sums over a run of equal c_t stay
// in registers (the workspace transformation, Sec. 4.2.8): a wave writes to C
// with atomics once per run it covers, so there are no scattered updates.
//
// Decomposition. The columns are cut into slices of W columns; each lane
// reads 16 bytes of a row (8 BF16 or 4 FP32 columns), so a group of W*2/16
// (BF16) or W*4/16 (FP32) lanes covers one entry. The concatenated views are
// cut into one contiguous range per workgroup and per wave; the lane groups
// of a wave take consecutive entries, so index loads are coalesced. Workgroup
// (slice, chunk): the slices of one chunk get block indices equal modulo 8,
// so they run on one XCD (blocks are dispatched round-robin over the 8 XCDs)
// and share the chunk's index stream in that XCD's L2.
#include <type_traits>

#include "common.h"
#include "mttkrp_device.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kLdsThreads = 1024;
constexpr int kLdsWaves = kLdsThreads / kWave;
constexpr int kLdsUnroll = 4;  // entries in flight per lane group

struct LdsViews {
  IdxPtrs idx[5];
  const float* val[5];
  int64_t off[6];  // first entry of each view in the concatenation; off[N] = total
};

// Elements of one 16-byte LDS read.
template <typename BT>
constexpr int vec_of() {
  return 16 / static_cast<int>(sizeof(BT));
}

template <typename BT>
__device__ __forceinline__ void unpack16(const uint4& u, float (&out)[vec_of<BT>()]) {
  if constexpr (std::is_same_v<BT, uint16_t>) {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      out[2 * q] = __uint_as_float(w[q] << 16);              // element 2q (low half)
      out[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);  // element 2q+1 (high half)
    }
  } else {
    out[0] = __uint_as_float(u.x);
    out[1] = __uint_as_float(u.y);
    out[2] = __uint_as_float(u.z);
    out[3] = __uint_as_float(u.w);
  }
}

// Sum of v over the lanes that hold the same columns (lanes equal modulo
// Lg), left in every lane.
template <int Lg>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int d = Lg; d < kWave; d *= 2) v += __shfl_xor(v, d);
  return v;
}

// A wave runs entries [e0, e1) of view T. Lane group g (Lg lanes) takes entry
// base + u*G + g of each iteration (u < kLdsUnroll), so index loads are
// coalesced; lane `sub` of the group owns columns col .. col + V-1.
//
// The view is sorted by c_T, so an iteration's entries carry nondecreasing
// output rows. Each lane sums the entries of the wave's current row `cur`;
// when an iteration reaches a later row, the lanes' sums for `cur` are added
// across the groups and one group writes them with atomics (once per run of
// equal rows per wave), the entries of the iteration's last row start the
// next sum, and rows strictly between (runs shorter than an iteration) are
// written directly.
template <int N, typename BT, int T, int Lg>
__device__ __forceinline__ void lds_view_range(int e0, int e1, const IdxPtrs& ip,
                                               const float* __restrict__ val,
                                               const unsigned char* sB, int row_bytes, int g,
                                               int sub, const float* sCoef,
                                               float* __restrict__ C, int R, int col) {
  constexpr int V = vec_of<BT>();
  constexpr int G = kWave / Lg;
  if (e0 >= e1) return;
  const int32_t* __restrict__ out_idx = ip.p[T];
  int cur = out_idx[e0];  // same address in every lane
  float acc[V], nxt[V];
#pragma unroll
  for (int j = 0; j < V; ++j) acc[j] = nxt[j] = 0.0f;
  auto emit = [&](int row, const float (&x)[V], bool lane_writes) {
    if (!lane_writes) return;
    float* out = C + static_cast<int64_t>(row) * R + col;
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (col + j < R) atomic_add_noret(out + j, x[j]);
  };
  for (int base = e0; base < e1; base += G * kLdsUnroll) {
    int c[kLdsUnroll][N];
    float v[kLdsUnroll];
    bool ok[kLdsUnroll];
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
      const int e = base + u * G + g;
      ok[u] = e < e1;
#pragma unroll
      for (int s = 0; s < N; ++s) c[u][s] = ok[u] ? ip.p[s][e] : 0;
      v[u] = ok[u] ? val[e] : 0.0f;
    }
    const int last = out_idx[min(e1, base + G * kLdsUnroll) - 1];  // uniform
    float p[kLdsUnroll][V];
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
#pragma unroll
      for (int j = 0; j < V; ++j) p[u][j] = 0.0f;
      if (!ok[u]) continue;
      const float kv = sCoef[5 * equality_mask_of(c[u], N) + T] * v[u];
#pragma unroll
      for (int j = 0; j < V; ++j) p[u][j] = kv;
#pragma unroll
      for (int s = 0; s < N; ++s) {
        if (s == T) continue;
        const uint4 raw = *reinterpret_cast<const uint4*>(
            sB + static_cast<int64_t>(c[u][s]) * row_bytes + sub * 16);
        float b[V];
        unpack16<BT>(raw, b);
#pragma unroll
        for (int j = 0; j < V; ++j) p[u][j] *= b[j];
      }
    }
    if (last == cur) {  // the whole iteration continues the current run
#pragma unroll
      for (int u = 0; u < kLdsUnroll; ++u)
#pragma unroll
        for (int j = 0; j < V; ++j) acc[j] += p[u][j];
      continue;
    }
#pragma unroll
    for (int u = 0; u < kLdsUnroll; ++u) {
      const int row = c[u][T];
      if (!ok[u]) continue;
      if (row == cur) {
#pragma unroll
        for (int j = 0; j < V; ++j) acc[j] += p[u][j];
      } else if (row == last) {
#pragma unroll
        for (int j = 0; j < V; ++j) nxt[j] += p[u][j];
      } else {
        emit(row, p[u], true);  // a run shorter than an iteration
      }
    }
    // close the current run: one write per wave
#pragma unroll
    for (int j = 0; j < V; ++j) acc[j] = group_sum<Lg>(acc[j]);
    emit(cur, acc, g == 0);
    cur = last;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      acc[j] = nxt[j];
      nxt[j] = 0.0f;
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) acc[j] = group_sum<Lg>(acc[j]);
  emit(cur, acc, g == 0);
}

template <int N, typename BT, int Lg>
__device__ __forceinline__ void lds_view_slot(int t, int e0, int e1, const LdsViews& vs,
                                              const unsigned char* sB, int row_bytes, int g,
                                              int sub, const float* sCoef, float* C, int R,
                                              int col) {
  switch (t) {
    case 0:
      lds_view_range<N, BT, 0, Lg>(e0, e1, vs.idx[0], vs.val[0], sB, row_bytes, g, sub, sCoef, C,
                                   R, col);
      break;
    case 1:
      lds_view_range<N, BT, 1, Lg>(e0, e1, vs.idx[1], vs.val[1], sB, row_bytes, g, sub, sCoef, C,
                                   R, col);
      break;
    case 2:
      lds_view_range<N, BT, 2, Lg>(e0, e1, vs.idx[2], vs.val[2], sB, row_bytes, g, sub, sCoef, C,
                                   R, col);
      break;
    case 3:
      if constexpr (N > 3)
        lds_view_range<N, BT, 3, Lg>(e0, e1, vs.idx[3], vs.val[3], sB, row_bytes, g, sub, sCoef,
                                     C, R, col);
      break;
    default:
      if constexpr (N > 4)
        lds_view_range<N, BT, 4, Lg>(e0, e1, vs.idx[4], vs.val[4], sB, row_bytes, g, sub, sCoef,
                                     C, R, col);
      break;
  }
}

// W: slice width in columns (a multiple of the 16-byte vector, at most 64).
// vec_rows: R is a multiple of the 16-byte vector and B is 16-byte aligned,
// so the slice is staged in 16-byte pieces.
template <int N, typename BT, int W>
__global__ __launch_bounds__(kLdsThreads) void mttkrp_views_lds_kernel(
    LdsViews vs, const BT* __restrict__ B, int R, int I, int nslices, int nchunks, int vec_rows,
    float* __restrict__ C) {
  constexpr int V = vec_of<BT>();
  constexpr int Lg = W / V;          // lanes per entry
  constexpr int kRowBytes = W * static_cast<int>(sizeof(BT));
  extern __shared__ __align__(16) unsigned char lds[];
  const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
  const int slice = j % nslices;
  const int chunk = xcd + 8 * (j / nslices);
  const int col0 = slice * W;

  unsigned char* sB = lds;
  float* sCoef = reinterpret_cast<float*>(lds + static_cast<int64_t>(I) * kRowBytes);
  if (vec_rows) {
    constexpr int kPieces = kRowBytes / 16;  // 16-byte pieces per staged row
    uint4* s4 = reinterpret_cast<uint4*>(sB);
    const int n = I * kPieces;
#pragma unroll 4
    for (int q = threadIdx.x; q < n; q += kLdsThreads) {
      const int i = q / kPieces, c = col0 + (q - i * kPieces) * V;
      s4[q] = (c < R) ? *reinterpret_cast<const uint4*>(B + static_cast<int64_t>(i) * R + c)
                      : make_uint4(0u, 0u, 0u, 0u);
    }
  } else {
    BT* sBt = reinterpret_cast<BT*>(sB);
    for (int q = threadIdx.x; q < I * W; q += kLdsThreads) {
      const int i = q / W, c = col0 + (q - (q / W) * W);
      sBt[q] = (c < R) ? B[static_cast<int64_t>(i) * R + c] : BT(0);
    }
  }
  if (threadIdx.x < 80) sCoef[threadIdx.x] = coef_table<N>().coef[threadIdx.x / 5][threadIdx.x % 5];
  __syncthreads();

  // contiguous ranges: chunk of the concatenated views, then wave, then group
  const int64_t total = vs.off[N];
  const int64_t per = (total + nchunks - 1) / nchunks;
  const int64_t c_lo = min<int64_t>(total, chunk * per), c_hi = min<int64_t>(total, c_lo + per);
  const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int g = lane / Lg, sub = lane - g * Lg;
  const int64_t wper = (c_hi - c_lo + kLdsWaves - 1) / kLdsWaves;
  const int64_t w_lo = min<int64_t>(c_hi, c_lo + wv * wper), w_hi = min<int64_t>(c_hi, w_lo + wper);
  const int col = col0 + sub * V;
  int64_t e = w_lo;
  while (e < w_hi) {  // the wave's range, one view at a time
    int t = 0;
#pragma unroll
    for (int q = 1; q < N; ++q) t += (e >= vs.off[q]) ? 1 : 0;
    const int64_t seg_hi = min<int64_t>(w_hi, vs.off[t + 1]);
    lds_view_slot<N, BT, Lg>(t, static_cast<int>(e - vs.off[t]), static_cast<int>(seg_hi - vs.off[t]),
                             vs, sB, kRowBytes, g, sub, sCoef, C, R, col);
    e = seg_hi;
  }
}

int device_limits(int* lds_bytes, int* cus) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc)
    rc = check_hip(hipDeviceGetAttribute(lds_bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                   "hipDeviceGetAttribute(max shared memory)");
  if (!rc)
    rc = check_hip(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev),
                   "hipDeviceGetAttribute(CU count)");
  return rc;
}

constexpr size_t kCoefBytes = 80 * sizeof(float);

template <typename BT>
size_t lds_bytes_for(int64_t I, int W) {
  return static_cast<size_t>(I) * W * sizeof(BT) + kCoefBytes;
}

// Widest slice (a power of two from one 16-byte vector up to 64 columns, no
// wider than R needs) whose B slice fits the LDS limit; 0 if none does.
template <typename BT>
int lds_width(int64_t I, int64_t R, int limit) {
  constexpr int V = vec_of<BT>();
  int want = V;
  while (want < R && want < 64) want *= 2;
  for (int w = want; w >= V; w /= 2)
    if (lds_bytes_for<BT>(I, w) <= static_cast<size_t>(limit)) return w;
  return 0;
}

template <int N, typename BT, int W>
int launch_lds_w(const LdsViews& vs, const BT* B, int R, int I, float* C, int cus,
                 hipStream_t s) {
  const int nslices = (R + W - 1) / W;
  // one workgroup per CU in total (LDS-bound), at least 16384 entries each
  const int64_t total = vs.off[N];
  const int64_t k = std::min<int64_t>((cus + nslices - 1) / nslices, (total + 16383) / 16384);
  const int nchunks = static_cast<int>((std::max<int64_t>(k, 1) + 7) / 8 * 8);
  const size_t lds = lds_bytes_for<BT>(I, W);
  auto kern = mttkrp_views_lds_kernel<N, BT, W>;
  int rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds)),
                     "hipFuncSetAttribute(dynamic LDS)");
  if (rc) return rc;
  const int vec_rows = (R % vec_of<BT>() == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0) ? 1 : 0;
  kern<<<dim3(nchunks * nslices), dim3(kLdsThreads), lds, s>>>(vs, B, R, I, nslices, nchunks,
                                                               vec_rows, C);
  return check_launch("mttkrp LDS view kernel");
}

template <int N, typename BT>
int launch_lds_typed(const Tensor* tn, const BT* B, int R, float* C, hipStream_t s) {
  int limit = 0, cus = 0;
  int rc = device_limits(&limit, &cus);
  if (rc) return rc;
  LdsViews vs{};
  int64_t off = 0;
  for (int t = 0; t < N; ++t) {
    for (int q = 0; q < N; ++q) vs.idx[t].p[q] = tn->vidx[t][q];
    vs.val[t] = tn->vval[t];
    vs.off[t] = off;
    off += tn->vnnz[t];
  }
  for (int t = N; t <= 5; ++t) vs.off[t] = off;
  const int I = static_cast<int>(tn->dim);
  switch (lds_width<BT>(I, R, limit)) {
    case 64: return launch_lds_w<N, BT, 64>(vs, B, R, I, C, cus, s);
    case 32: return launch_lds_w<N, BT, 32>(vs, B, R, I, C, cus, s);
    case 16: return launch_lds_w<N, BT, 16>(vs, B, R, I, C, cus, s);
    case 8: return launch_lds_w<N, BT, 8>(vs, B, R, I, C, cus, s);
    case 4:
      if constexpr (vec_of<BT>() == 4) return launch_lds_w<N, BT, 4>(vs, B, R, I, C, cus, s);
      [[fallthrough]];
    default:
      return fail(SYSTEC_EINVAL, "mttkrp: the index space is too large to stage B in LDS");
  }
}

}  // namespace

int mttkrp_lds_width(int64_t I, systec_dtype bdt, int64_t R) {
  int limit = 0, cus = 0;
  if (I > (1 << 20) || device_limits(&limit, &cus) != SYSTEC_OK) return 0;
  return bdt == SYSTEC_F32 ? lds_width<float>(I, R, limit) : lds_width<uint16_t>(I, R, limit);
}

int launch_mttkrp_views_lds(const Tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                            hipStream_t s) {
  // all of B in LDS with one lane per view entry where it fits, else
  // column slices of B
  const int lrc = launch_mttkrp_views_lane(t, B, bdt, R, C, s);
  if (lrc != -1) return lrc;
  int rc = launch_fill_f32(C, t->dim * R, s);
  if (rc != SYSTEC_OK || t->nnz == 0) return rc;
  const int r = static_cast<int>(R);
  const bool f32 = bdt == SYSTEC_F32;
  const auto* bf = static_cast<const float*>(B);
  const auto* bh = static_cast<const uint16_t*>(B);
  LaunchTimer timer(s);
  switch (t->order) {
    case 3:
      return f32 ? launch_lds_typed<3, float>(t, bf, r, C, s) : launch_lds_typed<3, uint16_t>(t, bh, r, C, s);
    case 4:
      return f32 ? launch_lds_typed<4, float>(t, bf, r, C, s) : launch_lds_typed<4, uint16_t>(t, bh, r, C, s);
    default:
      return f32 ? launch_lds_typed<5, float>(t, bf, r, C, s) : launch_lds_typed<5, uint16_t>(t, bh, r, C, s);
  }
}

}  // namespace systec
