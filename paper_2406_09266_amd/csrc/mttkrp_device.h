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
      const float k = coef_table<N>().coef[equality_mask_of(c[u], N)][T];
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

}  // namespace dev
}  // namespace systec
