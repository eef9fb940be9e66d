// Symmetric MTTKRP of order N = 3, 4, 5 over canonical COO, and the plain
// MTTKRP over an expanded (non-symmetric) COO used as the comparison.
//
// Method (SySTeC, arXiv 2406.09266, Sec. 4.3 and 5.2.6): a stored entry
// (c1 <= ... <= cN, v) stands for v at every distinct permutation of its
// indices. For MTTKRP the permutations that put the same index value in the
// output slot produce identical updates (invisible output symmetry,
// Sec. 3.2.2), so they are merged into one update scaled by their count
// (distributive grouping, Sec. 4.2.7). The count depends only on the
// equality pattern of the sorted tuple, so it comes from a small table
// indexed by that pattern (the simplicial lookup table, Sec. 4.2.5):
//   C[c_t, :] += coef[pattern][t] * v * prod_{s != t} B[c_s, :]
// for each slot t that starts a run of equal indices. Each factor row is
// read once per entry (common tensor access elimination, Sec. 4.2.1).
//
// GPU decomposition (mttkrp_device.h). A wavefront owns a tile of consecutive
// entries. It is split into groups of L lanes (L = 8/16/32/64, the smallest
// power of two >= R, or 64 with column blocks for R > 64); each group walks
// every (64/L)-th entry of the tile with one lane per output column, so
// factor-row gathers and output-row updates are contiguous L-wide accesses.
// Entries are sorted by c1, so slot 1 accumulates in registers across a run
// of equal c1 and is written once per run (the workspace transformation,
// Sec. 4.2.8); the other run-start slots scatter with FP32 atomics. The
// prepared form (slot views) has no scattered slot at all.
#include "common.h"
#include "mttkrp_device.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kWaves = 4;
constexpr int kBlock = kWave * kWaves;

// One wave per tile of kTileE consecutive canonical entries.
template <int N, typename BT, int L, bool kSym>
__global__ __launch_bounds__(kBlock) void mttkrp_tiles_kernel(int nnz, IdxPtrs idx,
                                                            const float* __restrict__ val,
                                                            const BT* __restrict__ B, int ldb,
                                                            float* __restrict__ C, int ldc,
                                                            int col0, int ncols) {
  const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWaves + threadIdx.x / kWave;
  const int64_t e0 = wave * kTileE;
  if (e0 >= nnz) return;
  const int e1 = static_cast<int>(min<int64_t>(nnz, e0 + kTileE));
  mttkrp_canonical_tile<N, BT, L, kSym>(static_cast<int>(e0), e1, idx, val, B, ldb, C, ldc, col0,
                                        ncols);
}

// The N slot views of a prepared tensor, processed by one launch: blocks
// [block0[t], block0[t+1]) take view t, one wave per tile of kTileE entries.
struct ViewSet {
  IdxPtrs idx[5];
  const float* val[5];
  int nnz[5];
  int block0[6];
};

template <int N, typename BT, int L, int T>
__device__ __forceinline__ void view_block(const ViewSet& vs, int b, const BT* __restrict__ B,
                                           int ldb, float* __restrict__ C, int ldc, int col0,
                                           int ncols) {
  const int64_t wave = static_cast<int64_t>(b - vs.block0[T]) * kWaves + threadIdx.x / kWave;
  const int64_t e0 = wave * kTileE;
  if (e0 >= vs.nnz[T]) return;
  const int e1 = static_cast<int>(min<int64_t>(vs.nnz[T], e0 + kTileE));
  mttkrp_view_tile<N, BT, L, T>(static_cast<int>(e0), e1, vs.idx[T], vs.val[T], B, ldb, C, ldc,
                                col0, ncols);
}

template <int N, typename BT, int L>
__global__ __launch_bounds__(kBlock) void mttkrp_views_kernel(ViewSet vs,
                                                            const BT* __restrict__ B, int ldb,
                                                            float* __restrict__ C, int ldc,
                                                            int col0, int ncols) {
  const int b = blockIdx.x;
  if (b < vs.block0[1]) {
    view_block<N, BT, L, 0>(vs, b, B, ldb, C, ldc, col0, ncols);
  } else if (b < vs.block0[2]) {
    view_block<N, BT, L, 1>(vs, b, B, ldb, C, ldc, col0, ncols);
  } else if (N == 3 || b < vs.block0[3]) {
    view_block<N, BT, L, 2>(vs, b, B, ldb, C, ldc, col0, ncols);
  } else if constexpr (N > 3) {
    if (N == 4 || b < vs.block0[4]) view_block<N, BT, L, 3>(vs, b, B, ldb, C, ldc, col0, ncols);
    else if constexpr (N > 4) view_block<N, BT, L, 4>(vs, b, B, ldb, C, ldc, col0, ncols);
  }
}

// The same launch with vector lanes (mttkrp_device.h): one wave per range
// of kTileVec entries of a view; V columns per lane, Lg lanes per row.
constexpr int kTileVec = 1024;

template <int N, typename BT, int V, int Lg, int T>
__device__ __forceinline__ void vec_block(const ViewSet& vs, int b, const BT* __restrict__ B,
                                          int ldb, float* __restrict__ C, int ldc, int col0,
                                          int ncols) {
  const int64_t wave = static_cast<int64_t>(b - vs.block0[T]) * kWaves + threadIdx.x / kWave;
  const int64_t e0 = wave * kTileVec;
  if (e0 >= vs.nnz[T]) return;
  const int e1 = static_cast<int>(min<int64_t>(vs.nnz[T], e0 + kTileVec));
  mttkrp_view_range_vec<N, BT, V, Lg, T>(static_cast<int>(e0), e1, vs.idx[T], vs.val[T], B, ldb,
                                         C, ldc, col0, ncols);
}

template <int N, typename BT, int V, int Lg>
__global__ __launch_bounds__(kBlock) void mttkrp_views_vec_kernel(ViewSet vs,
                                                                const BT* __restrict__ B, int ldb,
                                                                float* __restrict__ C, int ldc,
                                                                int col0, int ncols) {
  const int b = blockIdx.x;
  if (b < vs.block0[1]) {
    vec_block<N, BT, V, Lg, 0>(vs, b, B, ldb, C, ldc, col0, ncols);
  } else if (b < vs.block0[2]) {
    vec_block<N, BT, V, Lg, 1>(vs, b, B, ldb, C, ldc, col0, ncols);
  } else if (N == 3 || b < vs.block0[3]) {
    vec_block<N, BT, V, Lg, 2>(vs, b, B, ldb, C, ldc, col0, ncols);
  } else if constexpr (N > 3) {
    if (N == 4 || b < vs.block0[4]) vec_block<N, BT, V, Lg, 3>(vs, b, B, ldb, C, ldc, col0, ncols);
    else if constexpr (N > 4) vec_block<N, BT, V, Lg, 4>(vs, b, B, ldb, C, ldc, col0, ncols);
  }
}

template <int N, typename BT, int L, bool kSym>
void launch_one(int nnz, const IdxPtrs& ip, const float* val, const BT* B, int ldb, float* C,
                int ldc, int col0, int ncols, hipStream_t s) {
  const int64_t tiles = (static_cast<int64_t>(nnz) + kTileE - 1) / kTileE;
  const int64_t blocks = (tiles + kWaves - 1) / kWaves;
  mttkrp_tiles_kernel<N, BT, L, kSym>
      <<<dim3(blocks), dim3(kBlock), 0, s>>>(nnz, ip, val, B, ldb, C, ldc, col0, ncols);
}

template <int N, typename BT, bool kSym>
void launch_cols(int nnz, const IdxPtrs& ip, const float* val, const BT* B, int R, float* C,
                 hipStream_t s) {
  if (R <= 8) {
    launch_one<N, BT, 8, kSym>(nnz, ip, val, B, R, C, R, 0, R, s);
  } else if (R <= 16) {
    launch_one<N, BT, 16, kSym>(nnz, ip, val, B, R, C, R, 0, R, s);
  } else if (R <= 32) {
    launch_one<N, BT, 32, kSym>(nnz, ip, val, B, R, C, R, 0, R, s);
  } else {
    for (int c0 = 0; c0 < R; c0 += 64)
      launch_one<N, BT, 64, kSym>(nnz, ip, val, B, R, C, R, c0, std::min(64, R - c0), s);
  }
}

template <int N, bool kSym>
void launch_order(int nnz, const IdxPtrs& ip, const float* val, const void* B, systec_dtype bdt,
                  int R, float* C, hipStream_t s) {
  if (bdt == SYSTEC_F32)
    launch_cols<N, float, kSym>(nnz, ip, val, static_cast<const float*>(B), R, C, s);
  else
    launch_cols<N, uint16_t, kSym>(nnz, ip, val, static_cast<const uint16_t*>(B), R, C, s);
}

}  // namespace

int launch_mttkrp(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                  const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                  bool symmetric, hipStream_t s) {
  int rc = launch_fill_f32(C, I * R, s);
  if (rc != SYSTEC_OK || nnz == 0) return rc;
  IdxPtrs ip{};
  for (int t = 0; t < order; ++t) ip.p[t] = idx[t];
  const int nz = static_cast<int>(nnz), r = static_cast<int>(R);
  LaunchTimer timer(s);
  switch (order) {
    case 2:
      if (!symmetric) launch_order<2, false>(nz, ip, val, B, bdt, r, C, s);
      break;
    case 3:
      symmetric ? launch_order<3, true>(nz, ip, val, B, bdt, r, C, s)
                : launch_order<3, false>(nz, ip, val, B, bdt, r, C, s);
      break;
    case 4:
      symmetric ? launch_order<4, true>(nz, ip, val, B, bdt, r, C, s)
                : launch_order<4, false>(nz, ip, val, B, bdt, r, C, s);
      break;
    default:
      symmetric ? launch_order<5, true>(nz, ip, val, B, bdt, r, C, s)
                : launch_order<5, false>(nz, ip, val, B, bdt, r, C, s);
      break;
  }
  return check_launch(symmetric ? "mttkrp kernel" : "mttkrp (full) kernel");
}

namespace {

template <int N, typename BT, int L>
void launch_views_cols(const ViewSet& vs, const BT* B, int ldb, float* C, int ldc, int col0,
                       int ncols, hipStream_t s) {
  mttkrp_views_kernel<N, BT, L>
      <<<dim3(vs.block0[N]), dim3(kBlock), 0, s>>>(vs, B, ldb, C, ldc, col0, ncols);
}

template <int N, typename BT>
ViewSet view_set(const Tensor* tn, int tile) {
  ViewSet vs{};
  int64_t blocks = 0;
  for (int t = 0; t < N; ++t) {
    for (int q = 0; q < N; ++q) vs.idx[t].p[q] = tn->vidx[t][q];
    vs.val[t] = tn->vval[t];
    vs.nnz[t] = static_cast<int>(tn->vnnz[t]);
    vs.block0[t] = static_cast<int>(blocks);
    const int64_t tiles = (tn->vnnz[t] + tile - 1) / tile;
    blocks += (tiles + kWaves - 1) / kWaves;
  }
  for (int t = N; t <= 5; ++t) vs.block0[t] = static_cast<int>(blocks);
  return vs;
}

template <int N, typename BT, int V, int Lg>
void launch_vec_cols(const ViewSet& vs, const BT* B, int R, float* C, int col0, int ncols,
                     hipStream_t s) {
  mttkrp_views_vec_kernel<N, BT, V, Lg>
      <<<dim3(vs.block0[N]), dim3(kBlock), 0, s>>>(vs, B, R, C, R, col0, ncols);
}

// One column block with V columns per lane; false if its lane count has no
// kernel (the caller then takes the lane-per-column kernel).
template <int N, typename BT, int V>
bool launch_vec_block(const ViewSet& vs, const BT* B, int R, float* C, int c0, int w,
                      hipStream_t s) {
  int lanes = 1;
  while (lanes * V < w) lanes *= 2;
  switch (lanes) {
    case 1: launch_vec_cols<N, BT, V, 1>(vs, B, R, C, c0, w, s); return true;
    case 2: launch_vec_cols<N, BT, V, 2>(vs, B, R, C, c0, w, s); return true;
    case 4: launch_vec_cols<N, BT, V, 4>(vs, B, R, C, c0, w, s); return true;
    case 8: launch_vec_cols<N, BT, V, 8>(vs, B, R, C, c0, w, s); return true;
    default:
      if constexpr (V == 4) {
        launch_vec_cols<N, BT, V, 16>(vs, B, R, C, c0, w, s);
        return true;
      }
      return false;
  }
}

// Vector lanes (lane_vec_width: four lanes per row where R allows) when
// use_vector_lanes allows, every column block has a kernel and B is aligned
// to the lane width, else one lane per column.
template <int N, typename BT>
void launch_views_typed(const Tensor* tn, const BT* B, int R, float* C, hipStream_t s) {
  bool vec = use_vector_lanes(tn->short_runs, R);
  for (int c0 = 0; c0 < R && vec; c0 += 64) {
    const int w = std::min(64, R - c0);
    const int V = lane_vec_width(w, R, sizeof(BT));
    const int lanes = V ? (w + V - 1) / V : 0;
    vec = V != 0 && lanes <= (V == 4 ? 16 : 8) &&
          (reinterpret_cast<uintptr_t>(B) % (static_cast<size_t>(V) * sizeof(BT))) == 0;
  }
  if (vec) {
    const ViewSet vs = view_set<N, BT>(tn, kTileVec);
    if (vs.block0[N] == 0) return;
    for (int c0 = 0; c0 < R; c0 += 64) {
      const int w = std::min(64, R - c0);  // a multiple of V
      switch (lane_vec_width(w, R, sizeof(BT))) {
        case 2: launch_vec_block<N, BT, 2>(vs, B, R, C, c0, w, s); break;
        case 4: launch_vec_block<N, BT, 4>(vs, B, R, C, c0, w, s); break;
        default:
          if constexpr (sizeof(BT) == 2) launch_vec_block<N, BT, 8>(vs, B, R, C, c0, w, s);
          break;
      }
    }
    return;
  }
  const ViewSet vs = view_set<N, BT>(tn, kTileE);
  if (vs.block0[N] == 0) return;
  if (R <= 8) launch_views_cols<N, BT, 8>(vs, B, R, C, R, 0, R, s);
  else if (R <= 16) launch_views_cols<N, BT, 16>(vs, B, R, C, R, 0, R, s);
  else if (R <= 32) launch_views_cols<N, BT, 32>(vs, B, R, C, R, 0, R, s);
  else
    for (int c0 = 0; c0 < R; c0 += 64)
      launch_views_cols<N, BT, 64>(vs, B, R, C, R, c0, std::min(64, R - c0), s);
}

template <int N>
void launch_views_order(const Tensor* tn, const void* B, systec_dtype bdt, int R, float* C,
                        hipStream_t s) {
  if (bdt == SYSTEC_F32)
    launch_views_typed<N, float>(tn, static_cast<const float*>(B), R, C, s);
  else
    launch_views_typed<N, uint16_t>(tn, static_cast<const uint16_t*>(B), R, C, s);
}

}  // namespace

int launch_mttkrp_views(const Tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                        hipStream_t s) {
  int rc = launch_fill_f32(C, t->dim * R, s);
  if (rc != SYSTEC_OK || t->nnz == 0) return rc;
  const int r = static_cast<int>(R);
  LaunchTimer timer(s);
  switch (t->order) {
    case 3: launch_views_order<3>(t, B, bdt, r, C, s); break;
    case 4: launch_views_order<4>(t, B, bdt, r, C, s); break;
    default: launch_views_order<5>(t, B, bdt, r, C, s); break;
  }
  return check_launch("mttkrp view kernels");
}

}  // namespace systec
