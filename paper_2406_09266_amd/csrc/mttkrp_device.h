// Symmetric MTTKRP tile processing, as wave-level device functions shared by
// the standalone kernels and the serving step kernel.
//
// A wave processes the entries [e0, e1) of a tile. It is split into groups of
// L lanes (one lane per output column); group g takes every G-th entry. The
// loop is unrolled U entries deep per group: the indices of U entries are
// loaded, then all their factor-row gathers are issued, and only then are
// they consumed, so each wave keeps U*(N-1) gathers in flight instead of
// waiting on one dependent chain at a time.
#pragma once

#include "common.h"

namespace systec {
namespace dev {

constexpr int kTileE = 256;  // entries per wavefront tile
constexpr int kUnroll = 4;   // entries in flight per lane group

// coefficient tables (see make_coef_table): one copy per translation unit
static __constant__ CoefTable kCoef3 = make_coef_table(3);
static __constant__ CoefTable kCoef4 = make_coef_table(4);
static __constant__ CoefTable kCoef5 = make_coef_table(5);

template <int N>
__device__ __forceinline__ const CoefTable& coef_table();
template <>
__device__ __forceinline__ const CoefTable& coef_table<3>() { return kCoef3; }
template <>
__device__ __forceinline__ const CoefTable& coef_table<4>() { return kCoef4; }
template <>
__device__ __forceinline__ const CoefTable& coef_table<5>() { return kCoef5; }

struct IdxPtrs {
  const int32_t* p[5];
};

// The coefficients of one output slot T, coef[mask][T] for every equality
// mask of order N, packed 8 bits per mask into two 64-bit constants (masks
// 0..7 and 8..15). They are integers from 0 to 24 (the largest is 5!/5 for
// five distinct indices), so a view kernel, whose slot is a template
// parameter, reads its coefficient with a shift instead of a memory load.
template <int N, int T>
constexpr uint64_t packed_slot_coef(int half) {
  const CoefTable t = make_coef_table(N);
  uint64_t w = 0;
  for (int k = 0; k < 8; ++k) {
    const float c = t.coef[half * 8 + k][T];
    w |= static_cast<uint64_t>(static_cast<uint32_t>(c)) << (8 * k);
  }
  return w;
}

template <int N, int T>
constexpr bool slot_coef_packable() {
  const CoefTable t = make_coef_table(N);
  for (int m = 0; m < 16; ++m) {
    const float c = t.coef[m][T];
    if (c < 0.0f || c > 255.0f || c != static_cast<float>(static_cast<uint32_t>(c))) return false;
  }
  return true;
}

template <int N, int T>
__device__ __forceinline__ float slot_coef(int mask) {
  static_assert(slot_coef_packable<N, T>(), "slot coefficients must be integers in 0..255");
  constexpr uint64_t lo = packed_slot_coef<N, T>(0);
  constexpr uint64_t hi = packed_slot_coef<N, T>(1);
  const uint64_t w = (N < 5 || mask < 8) ? lo : hi;
  return static_cast<float>(static_cast<uint32_t>(w >> (8 * (mask & 7))) & 0xffu);
}

// Leave-one-out products: loo[t] = prod_{s != t} b[s].
template <int N>
__device__ __forceinline__ void leave_one_out(const float (&b)[N], float (&loo)[N]) {
  float pre[N], suf[N];
  pre[0] = 1.0f;
#pragma unroll
  for (int t = 1; t < N; ++t) pre[t] = (t == 1) ? b[0] : pre[t - 1] * b[t - 1];
  suf[N - 1] = 1.0f;
#pragma unroll
  for (int t = N - 2; t >= 0; --t) suf[t] = (t == N - 2) ? b[N - 1] : suf[t + 1] * b[t + 1];
#pragma unroll
  for (int t = 0; t < N; ++t)
    loo[t] = (t == 0) ? suf[0] : (t == N - 1) ? pre[N - 1] : pre[t] * suf[t];
}

__device__ __forceinline__ int equality_mask_of(const int* c, int n) {
  int mask = 0;
  for (int s = 0; s + 1 < n; ++s) mask |= (c[s] == c[s + 1]) ? (1 << s) : 0;
  return mask;
}

// Lane geometry of a wave: group g of L lanes, lane cl of the group handles
// output column col0 + cl (if cl < ncols).
template <int L>
struct LaneCols {
  int g, cl, col;
  bool col_ok;
  __device__ __forceinline__ LaneCols(int col0, int ncols) {
    const int lane = threadIdx.x & (kWave - 1);
    g = lane / L;
    cl = lane - g * L;
    col_ok = cl < ncols;
    col = col0 + (col_ok ? cl : 0);
  }
};

// Canonical entries (kSym) or plain entries (!kSym: only slot 1 is output,
// the comparison kernel over an expanded tensor). Output slot 1 is summed in
// registers across a run of equal c1; the other run-start slots (kSym) are
// scattered with atomics.
template <int N, typename BT, int L, bool kSym>
__device__ __forceinline__ void mttkrp_canonical_tile(int e0, int e1, const IdxPtrs& idx,
                                                      const float* __restrict__ val,
                                                      const BT* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int col0,
                                                      int ncols) {
  constexpr int G = kWave / L;
  const LaneCols<L> lc(col0, ncols);
  int cur = -1;
  float acc = 0.0f;
  for (int base = e0 + lc.g; base < e1; base += G * kUnroll) {
    int c[kUnroll][N];
    float v[kUnroll];
    bool ok[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = base + u * G;
      ok[u] = e < e1;
#pragma unroll
      for (int s = 0; s < N; ++s) c[u][s] = ok[u] ? idx.p[s][e] : 0;
      v[u] = ok[u] ? val[e] : 0.0f;
    }
    float b[kUnroll][N];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int s = 0; s < N; ++s) b[u][s] = load_f32(B, static_cast<int64_t>(c[u][s]) * ldb + lc.col);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (!ok[u]) continue;
      float loo[N];
      leave_one_out<N>(b[u], loo);
      if (c[u][0] != cur) {
        if (cur >= 0 && lc.col_ok)
          atomic_add_noret(C + static_cast<int64_t>(cur) * ldc + lc.col, acc);
        cur = c[u][0];
        acc = 0.0f;
      }
      if constexpr (kSym) {
        const float* coef = coef_table<N>().coef[equality_mask_of(c[u], N)];
        acc += coef[0] * v[u] * loo[0];
#pragma unroll
        for (int t = 1; t < N; ++t) {
          const float k = coef[t];
          if (k != 0.0f && lc.col_ok)
            atomic_add_noret(C + static_cast<int64_t>(c[u][t]) * ldc + lc.col, k * v[u] * loo[t]);
        }
      } else {
        acc += v[u] * loo[0];
      }
    }
  }
  if (cur >= 0 && lc.col_ok) atomic_add_noret(C + static_cast<int64_t>(cur) * ldc + lc.col, acc);
}

// One tile of slot view T (see plan.hip): every entry updates C[c_T] with its
// slot-T coefficient; the view is sorted by c_T, so the updates are register
// sums written once per run of equal c_T. T is a template parameter so that
// only the N-1 factor rows of the product are gathered and the loop stays
// straight-line code (callers switch on the slot once per tile).
template <int N, typename BT, int L, int T>
__device__ __forceinline__ void mttkrp_view_tile(int e0, int e1, const IdxPtrs& idx,
                                                 const float* __restrict__ val,
                                                 const BT* __restrict__ B, int ldb,
                                                 float* __restrict__ C, int ldc, int col0,
                                                 int ncols) {
  constexpr int G = kWave / L;
  const LaneCols<L> lc(col0, ncols);
  int cur = -1;
  float acc = 0.0f;
  for (int base = e0 + lc.g; base < e1; base += G * kUnroll) {
    int c[kUnroll][N];
    float v[kUnroll];
    bool ok[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = base + u * G;
      ok[u] = e < e1;
#pragma unroll
      for (int s = 0; s < N; ++s) c[u][s] = ok[u] ? idx.p[s][e] : 0;
      v[u] = ok[u] ? val[e] : 0.0f;
    }
    float b[kUnroll][N];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int s = 0; s < N; ++s)
        b[u][s] = (s == T) ? 1.0f : load_f32(B, static_cast<int64_t>(c[u][s]) * ldb + lc.col);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (!ok[u]) continue;
      float p = 1.0f;
#pragma unroll
      for (int s = 0; s < N; ++s)
        if (s != T) p *= b[u][s];
      const float k = slot_coef<N, T>(equality_mask_of(c[u], N));
      const int out = c[u][T];
      if (out != cur) {
        if (cur >= 0 && lc.col_ok)
          atomic_add_noret(C + static_cast<int64_t>(cur) * ldc + lc.col, acc);
        cur = out;
        acc = 0.0f;
      }
      acc += k * v[u] * p;
    }
  }
  if (cur >= 0 && lc.col_ok) atomic_add_noret(C + static_cast<int64_t>(cur) * ldc + lc.col, acc);
}

// Runs the view tile of slot t (a value uniform across the wave).
template <int N, typename BT, int L>
__device__ __forceinline__ void mttkrp_view_tile_slot(int t, int e0, int e1, const IdxPtrs& idx,
                                                      const float* __restrict__ val,
                                                      const BT* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int col0,
                                                      int ncols) {
  switch (t) {
    case 0: mttkrp_view_tile<N, BT, L, 0>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols); break;
    case 1: mttkrp_view_tile<N, BT, L, 1>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols); break;
    case 2: mttkrp_view_tile<N, BT, L, 2>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols); break;
    case 3:
      if constexpr (N > 3) mttkrp_view_tile<N, BT, L, 3>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols);
      break;
    default:
      if constexpr (N > 4) mttkrp_view_tile<N, BT, L, 4>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols);
      break;
  }
}

// ---- vector lanes -------------------------------------------------------------
// The view kernels above give every output column its own lane, so a lane
// loads 2 (BF16) or 4 (FP32) bytes of a factor row and a wave instruction
// covers only 64/L rows: at R = 32 the kernels issue a load instruction for
// every two rows, and their time goes to issuing loads, not to moving bytes.
// Here each lane loads V consecutive columns of a row (4 to 16 bytes), so a
// group of Lg = R/V lanes covers a row. V is chosen so that a row takes four
// lanes where it can (lane_vec_width): with fewer lanes per row each lane
// carries more columns and an iteration spans more entries, and measured
// kernels ran up to 3x slower with one or two lanes per row. Requires R to be
// a multiple of V and B aligned to V elements (rows stay aligned).

// entries in flight per lane group (a group already covers a whole row)
constexpr int kUnrollVec = 4;

// Words (4 bytes) per lane for V elements of BT.
template <typename BT, int V>
constexpr int vec_words() {
  return V * static_cast<int>(sizeof(BT)) / 4;
}

// Loads V elements of BT at p (aligned to their size) as raw words.
template <typename BT, int V>
__device__ __forceinline__ void load_vec_words(const BT* p, uint32_t (&w)[vec_words<BT, V>()]) {
  constexpr int W = vec_words<BT, V>();
  if constexpr (W == 1) {
    w[0] = *reinterpret_cast<const uint32_t*>(p);
  } else if constexpr (W == 2) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);
    w[0] = t.x;
    w[1] = t.y;
  } else {
#pragma unroll
    for (int k = 0; k < W / 4; ++k) {
      const uint4 t = reinterpret_cast<const uint4*>(p)[k];
      w[4 * k] = t.x;
      w[4 * k + 1] = t.y;
      w[4 * k + 2] = t.z;
      w[4 * k + 3] = t.w;
    }
  }
}

// Raw words -> V FP32 values (BF16: the 16 bits become the top half).
template <typename BT, int V>
__device__ __forceinline__ void unpack_vec(const uint32_t (&w)[vec_words<BT, V>()], float (&out)[V]) {
  if constexpr (sizeof(BT) == 2) {
#pragma unroll
    for (int q = 0; q < V / 2; ++q) {
      out[2 * q] = __uint_as_float(w[q] << 16);              // element 2q (low half)
      out[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);  // element 2q+1 (high half)
    }
  } else {
#pragma unroll
    for (int q = 0; q < V; ++q) out[q] = __uint_as_float(w[q]);
  }
}

// Sum over the lanes that hold the same columns (lanes equal modulo Lg).
template <int Lg>
__device__ __forceinline__ float lane_group_sum(float v) {
#pragma unroll
  for (int d = Lg; d < kWave; d *= 2) v += __shfl_xor(v, d);
  return v;
}

// Writes the wave's sum for output row `row` with one atomic per column: the
// sums of group 0 (lane sub holds columns sub*V .. sub*V+V-1) are spread so
// that lane l adds column l, and consecutive lanes hit consecutive addresses.
template <int V, int Lg>
__device__ __forceinline__ void emit_row_spread(float* __restrict__ C, int ldc, int row, int col0,
                                                int ncols, const float (&acc)[V]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int src = lane / V, j = lane - src * V;
  float x = 0.0f;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const float t = __shfl(acc[q], src);
    x = (j == q) ? t : x;
  }
  if (lane < ncols && lane < V * Lg)
    atomic_add_noret(C + static_cast<int64_t>(row) * ldc + col0 + lane, x);
}

// Rows of one unroll slot that lie strictly between the iteration's first
// and last rows (runs shorter than an iteration). The slot's entries are
// sorted, so a row's entries sit in consecutive lane groups: a segmented sum
// across the groups leaves each row's total in its last group, which writes
// it with one atomic per column (spread as in emit_row_spread). key < 0 marks
// entries of no such row; v holds the lane's V columns of its entry.
template <int V, int Lg>
__device__ __forceinline__ void emit_short_rows(float* __restrict__ C, int ldc, int col0,
                                                int ncols, int key, float (&v)[V]) {
  constexpr int G = kWave / Lg;
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane / Lg;
  // (every shuffle runs in all lanes: a lane that reads from a lane left out
  // of a divergent shuffle gets 0, not that lane's value)
#pragma unroll
  for (int d = 1; d < G; d *= 2) {
    const int earlier = __shfl_up(key, d * Lg);
    const bool same = g >= d && earlier == key;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const float t = __shfl_up(v[j], d * Lg);
      v[j] += same ? t : 0.0f;
    }
  }
  const int next = __shfl_down(key, Lg);
  const bool ends = key >= 0 && (g == G - 1 || next != key);
  uint64_t heads = __ballot(ends && lane % Lg == 0);  // the first lane of each ending group
  const int j = lane % V;
  while (heads != 0) {
    const int first = __ffsll(static_cast<unsigned long long>(heads)) - 1;
    heads &= heads - 1;
    const int row = __shfl(key, first);
    const int src = first + lane / V;  // the lane holding column `lane` (lanes < V * Lg)
    float x = 0.0f;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const float t = __shfl(v[q], src);
      x = (j == q) ? t : x;
    }
    if (lane < ncols && lane < V * Lg)
      atomic_add_noret(C + static_cast<int64_t>(row) * ldc + col0 + lane, x);
  }
}

// A wave runs entries [e0, e1) of view T (sorted by c_T). Lane group g takes
// entry base + u*G + g of each iteration, so index loads are coalesced. Each
// lane sums the entries of the wave's current output row `cur`; when an
// iteration reaches a later row, the sums for `cur` are added across the
// groups and written once, the entries of the iteration's last row start the
// next sum, and rows strictly between (runs shorter than an iteration) are
// summed across the groups and written once per row (emit_short_rows).
template <int N, typename BT, int V, int Lg, int T>
__device__ __forceinline__ void mttkrp_view_range_vec(int e0, int e1, const IdxPtrs& ip,
                                                      const float* __restrict__ val,
                                                      const BT* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int col0,
                                                      int ncols) {
  constexpr int W = vec_words<BT, V>();
  constexpr int G = kWave / Lg;
  if (e0 >= e1) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int g = lane / Lg, sub = lane - g * Lg;
  const bool lane_cols = sub * V < ncols;
  const int col = col0 + sub * V;
  const int32_t* __restrict__ out_idx = ip.p[T];
  int cur = out_idx[e0];  // same address in every lane
  float acc[V], nxt[V];
#pragma unroll
  for (int j = 0; j < V; ++j) acc[j] = nxt[j] = 0.0f;
  for (int base = e0; base < e1; base += G * kUnrollVec) {
    int c[kUnrollVec][N];
    float v[kUnrollVec];
    bool ok[kUnrollVec];
#pragma unroll
    for (int u = 0; u < kUnrollVec; ++u) {
      const int e = base + u * G + g;
      ok[u] = e < e1;
#pragma unroll
      for (int s = 0; s < N; ++s) c[u][s] = ok[u] ? ip.p[s][e] : 0;
      v[u] = ok[u] ? val[e] : 0.0f;
    }
    uint32_t raw[kUnrollVec][N][W];
#pragma unroll
    for (int u = 0; u < kUnrollVec; ++u)
#pragma unroll
      for (int s = 0; s < N; ++s) {
        if (s == T) continue;
        if (ok[u] && lane_cols) {
          load_vec_words<BT, V>(B + static_cast<int64_t>(c[u][s]) * ldb + col, raw[u][s]);
        } else {
#pragma unroll
          for (int k = 0; k < W; ++k) raw[u][s][k] = 0u;
        }
      }
    const int last = out_idx[min(e1, base + G * kUnrollVec) - 1];  // uniform
    float p[kUnrollVec][V];
#pragma unroll
    for (int u = 0; u < kUnrollVec; ++u) {
      const float kv = ok[u] ? slot_coef<N, T>(equality_mask_of(c[u], N)) * v[u] : 0.0f;
#pragma unroll
      for (int j = 0; j < V; ++j) p[u][j] = kv;
#pragma unroll
      for (int s = 0; s < N; ++s) {
        if (s == T) continue;
        float b[V];
        unpack_vec<BT, V>(raw[u][s], b);
#pragma unroll
        for (int j = 0; j < V; ++j) p[u][j] *= b[j];
      }
    }
    if (last == cur) {  // the whole iteration continues the current run
#pragma unroll
      for (int u = 0; u < kUnrollVec; ++u)
#pragma unroll
        for (int j = 0; j < V; ++j) acc[j] += p[u][j];
      continue;
    }
#pragma unroll
    for (int u = 0; u < kUnrollVec; ++u) {
      const int row = c[u][T];
      const bool between = ok[u] && row != cur && row != last;
      if (ok[u] && row == cur) {
#pragma unroll
        for (int j = 0; j < V; ++j) acc[j] += p[u][j];
      } else if (ok[u] && row == last) {
#pragma unroll
        for (int j = 0; j < V; ++j) nxt[j] += p[u][j];
      }
      if (__ballot(between) != 0) {  // runs shorter than an iteration
        float v[V];
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = between ? p[u][j] : 0.0f;
        emit_short_rows<V, Lg>(C, ldc, col0, ncols, between ? row : -1, v);
      }
    }
#pragma unroll
    for (int j = 0; j < V; ++j) acc[j] = lane_group_sum<Lg>(acc[j]);
    emit_row_spread<V, Lg>(C, ldc, cur, col0, ncols, acc);
    cur = last;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      acc[j] = nxt[j];
      nxt[j] = 0.0f;
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) acc[j] = lane_group_sum<Lg>(acc[j]);
  emit_row_spread<V, Lg>(C, ldc, cur, col0, ncols, acc);
}

// Runs view slot t (a value uniform across the wave) with vector lanes.
template <int N, typename BT, int V, int Lg>
__device__ __forceinline__ void mttkrp_view_range_vec_slot(int t, int e0, int e1,
                                                           const IdxPtrs& idx,
                                                           const float* __restrict__ val,
                                                           const BT* __restrict__ B, int ldb,
                                                           float* __restrict__ C, int ldc,
                                                           int col0, int ncols) {
  switch (t) {
    case 0: mttkrp_view_range_vec<N, BT, V, Lg, 0>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols); break;
    case 1: mttkrp_view_range_vec<N, BT, V, Lg, 1>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols); break;
    case 2: mttkrp_view_range_vec<N, BT, V, Lg, 2>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols); break;
    case 3:
      if constexpr (N > 3)
        mttkrp_view_range_vec<N, BT, V, Lg, 3>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols);
      break;
    default:
      if constexpr (N > 4)
        mttkrp_view_range_vec<N, BT, V, Lg, 4>(e0, e1, idx, val, B, ldb, C, ldc, col0, ncols);
      break;
  }
}

}  // namespace dev
}  // namespace systec
