// Symmetric MTTKRP over packed slot views with one lane per view entry and
// the whole factor B staged in LDS: the form for tensors whose index space is
// small enough for B to fit one workgroup's LDS (the 5-D workload, I =
// 5,000 and R = 16 in BF16: 160,000 bytes) and whose runs of equal output
// rows are long (each view's entries sorted by output row, about a thousand
// entries per row at that shape).
//
// Same updates as the other view kernels (Sec. 4.3; per-run coefficients,
// Sec. 4.2.5 and 4.2.7): view t lists the entries whose slot t starts a run,
// sorted by c_t, and each adds coef[mask][t] * v * prod_{s != t} B[c_s, :] to
// C[c_t, :], the sum over a run of equal c_t kept in registers (Sec. 4.2.8).
//
// Why this layout. Lane l of a wave takes record base + l, so one load of
// 8 or 12 bytes per lane brings the wave 64 whole records (the N - 1 indices
// other than the output's as 16-bit halves and the weight coef * v,
// computed once when the tensor is prepared; the output index is not
// stored: each view's records are grouped by it through a row pointer, the
// leading-index level of a compressed fiber layout, Sec. 2.2), and the loads
// of the next kDepth iterations are in flight while one is consumed; the
// N - 1 factor rows of the record are read from LDS. The lane keeps the R
// partial sums of the wave's current output row; an iteration that stays
// in that row (known from the row pointer) just accumulates. When the row
// changes inside an iteration, each lane finds its record's row from the
// row pointer, the lanes' sums are added across the wave by a transposing
// butterfly (each exchange halves the columns a lane holds, so R = 16
// columns take 15 exchanges instead of 16 full reductions), and rows that
// begin and end inside one iteration are summed by a segmented scan across
// the lanes. The views are padded to whole iterations with records of
// weight 0 on the view's last row, so the loop has no bounds checks.
#include "common.h"
#include "mttkrp_device.h"
#include "wave_ops.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kLaneThreads = 1024;
constexpr int kLaneWaves = kLaneThreads / kWave;
constexpr int kLaneTile = 512;  // records per wave tile (a multiple of 64)
// iterations of record loads in flight (fewer at 32 columns, whose sums
// take most of the registers)
constexpr int depth_of(int R) { return R >= 32 ? 2 : 4; }

// record words: the N - 1 indices other than the view's slot, two 16-bit
// halves to a word, then the weight
constexpr int lane_words_of(int N) { return N / 2 + 1; }

// LDS after the factor: the workgroup's tile counter and the flag of an
// inexact FP16 conversion (the kernel declares no static LDS, so B starts
// at LDS address 0; the launch checks that)
constexpr int kLaneExtraLds = 16;

struct LaneViews {
  const uint32_t* rec[5];
  const int32_t* rowptr[5];    // per view: first record of each output row (I + 1)
  const int32_t* tile_row[5];  // per view: output row of each tile's first record
  int nrec[5];   // padded record counts (multiples of 64)
  int tile0[6];  // first tile of each view; tile0[N] = total
};

template <int K>
__device__ __forceinline__ void load_record(const uint32_t* __restrict__ rec, int e,
                                            uint32_t (&w)[K]) {
  const uint32_t* p = rec + static_cast<int64_t>(e) * K;
  if constexpr (K == 4) {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    w[0] = u.x; w[1] = u.y; w[2] = u.z; w[3] = u.w;
  } else {
#pragma unroll
    for (int q = 0; q < K; ++q) w[q] = p[q];
  }
}

// A window of a view's row pointer: lane j holds rowptr[wbase + j] (INT_MAX
// past row I), the starts of rows wbase .. wbase + 63.
struct RowWindow {
  int wbase;
  int start;
};

__device__ __forceinline__ RowWindow load_row_window(const int32_t* __restrict__ rowptr, int I,
                                                     int wbase, int lane) {
  const int r = wbase + lane;
  return RowWindow{wbase, r <= I ? rowptr[r] : INT_MAX};
}

// The output row of record e, for each lane of the wave, given that the
// wave's records lie in rows cur and above (rows up to cur start at or before
// e - lane): cur plus the starts of rows above cur at or below e. The starts come from the window when it
// covers them (it is reloaded from row cur + 1 otherwise); with few starts
// inside the wave's records (long rows) each is compared directly, else each
// lane binary-searches the 64 starts held across the lanes.
__device__ __forceinline__ int lane_row(const int32_t* __restrict__ rowptr, int I, int cur, int e,
                                        int lane, RowWindow& win) {
  const int e_max = __builtin_amdgcn_readlane(e, kWave - 1);
  int off = cur + 1 - win.wbase;  // window lanes below off hold rows up to cur
  if (off < 0 || off >= kWave) {
    win = load_row_window(rowptr, I, cur + 1, lane);
    off = 0;
  }
  // rows wbase .. cur start at or before every lane's record and are counted
  // below with the rest; they are not above cur
  int count = -off;
  for (;;) {  // wave-uniform
    const int b = win.start;
    uint64_t reach = __ballot(b <= e_max);  // the starts inside the wave's records
    const int b_last = __builtin_amdgcn_readlane(b, kWave - 1);
    if (__popcll(reach) <= 4) {
      while (reach) {
        const int j = __ffsll(static_cast<long long>(reach)) - 1;
        count += e >= __builtin_amdgcn_readlane(b, j) ? 1 : 0;
        reach &= reach - 1;
      }
    } else {
      int pos = 0;  // starts b_0 .. b_{pos-1} are <= e (b ascends across lanes)
#pragma unroll
      for (int k = kWave / 2; k >= 1; k /= 2)
        if (__shfl(b, pos + k - 1) <= e) pos += k;
      if (pos == kWave - 1 && b_last <= e) pos = kWave;
      count += pos;
    }
    if (b_last > e_max) break;  // no later start is at or below any lane's record
    win = load_row_window(rowptr, I, win.wbase + kWave, lane);
  }
  return cur + count;
}

// The start of row cur + 1 (the first record past row cur), from the window
// when it holds it.
__device__ __forceinline__ int next_row_start(const int32_t* __restrict__ rowptr, int I, int cur,
                                              int lane, RowWindow& win) {
  const int j = cur + 1 - win.wbase;
  if (j < 0 || j >= kWave) win = load_row_window(rowptr, I, cur + 1, lane);
  return __builtin_amdgcn_readlane(win.start, cur + 1 - win.wbase);
}

template <typename BT, int R>
constexpr int pieces_of() { return R * static_cast<int>(sizeof(BT)) / 16; }

// B in LDS piece-major: the q-th 16-byte piece of row r at byte r * 16 + q *
// plane, plane = I * 16. The LDS has 64 four-byte banks, 16 groups of four
// for a 16-byte read, and a read's bank group is r mod 16, so the random
// rows of a wave's read spread over all 16 groups. (Rows stored whole, 32
// bytes apart at R = 16 in BF16, put piece q of every row in one of 8 groups
// and doubled the collisions.)
// (B is the first thing in the workgroup's LDS, at LDS address 0: the
// kernel declares no static LDS, which the launch checks, so a row's byte
// offset is its LDS address.)
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const u32x4_t lds_piece_t;

template <typename BT, int R>
__device__ __forceinline__ void lds_row_raw(const BT*, int plane, int row,
                                            uint4 (&u)[pieces_of<BT, R>()]) {
  const uint32_t first = static_cast<uint32_t>(row) << 4;
#pragma unroll
  for (int q = 0; q < pieces_of<BT, R>(); ++q)
  {
    const u32x4_t v = *reinterpret_cast<lds_piece_t*>(static_cast<uintptr_t>(first + q * plane));
    u[q] = make_uint4(v.x, v.y, v.z, v.w);
  }
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// Element j of a row held as FP16 pieces, as FP32 (the conversion folds into
// the mixed-precision FMA that consumes it).
template <int R>
__device__ __forceinline__ float half_at(const uint4 (&raw)[R / 8], int j) {
  const uint4 u = raw[j / 8];
  const int k = (j % 8) / 2;
  const uint32_t word = k == 0 ? u.x : k == 1 ? u.y : k == 2 ? u.z : u.w;
  const half2_t h = __builtin_bit_cast(half2_t, word);
  return (j & 1) ? static_cast<float>(h.y) : static_cast<float>(h.x);
}

// Eight BF16 values (a 16-byte piece) as FP16; inexact is set unless every
// value converts exactly (BF16 values of magnitude 2^-14 to 65,504, and
// zeros, do; FP16 has the wider significand).
__device__ __forceinline__ uint4 bf16_piece_to_half(uint4 u, bool& inexact) {
  uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float lo = __uint_as_float(w[k] << 16), hi = __uint_as_float(w[k] & 0xffff0000u);
    const _Float16 hlo = static_cast<_Float16>(lo), hhi = static_cast<_Float16>(hi);
    inexact |= static_cast<float>(hlo) != lo || static_cast<float>(hhi) != hi;
    half2_t h;
    h.x = hlo;
    h.y = hhi;
    w[k] = __builtin_bit_cast(uint32_t, h);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// The R elements of a row's pieces as FP32.
template <typename BT, int R>
__device__ __forceinline__ void unpack_row(const uint4 (&raw)[pieces_of<BT, R>()], float (&b)[R]) {
  constexpr int kPieces = pieces_of<BT, R>();
  constexpr int kPer = 16 / static_cast<int>(sizeof(BT));  // elements per 16-byte piece
#pragma unroll
  for (int q = 0; q < kPieces; ++q) {
    const uint4 u = raw[q];
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
    if constexpr (sizeof(BT) == 2) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        b[q * kPer + 2 * k] = __uint_as_float(w[k] << 16);
        b[q * kPer + 2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) b[q * kPer + k] = __uint_as_float(w[k]);
    }
  }
}

// ---- the transposing wave sum ------------------------------------------------
// Level L pairs lane l with a partner that differs from it in lane bit
// kBit[L] (and possibly in lower bits): l ^ 32 and l ^ 16 by the permlane
// swaps, l ^ 15 and l ^ 7 by the DPP row mirrors, l ^ 2 and l ^ 1 by DPP
// quad permutations. Partners agree in every bit above kBit[L], so after
// levels 0..L-1 they hold the same columns; the pair's columns j and j + M/2
// are summed, the lane with the bit clear keeping column j. The partner sets
// generate all 64 lanes, so a value folded through every level (and summed
// over the levels left) is the sum over the wave.
constexpr int kBit[6] = {32, 16, 8, 4, 2, 1};

template <int L>
__device__ __forceinline__ float dpp_partner(float v) {
  static_assert(L >= 2 && L <= 5, "DPP levels");
  constexpr int kCtrl = L == 2 ? 0x140 : L == 3 ? 0x141 : L == 4 ? 0x4e : 0xb1;
  return dpp_f32<kCtrl, 0xf>(0.0f, v);
}

template <int L, int M>
__device__ __forceinline__ void fold_level(const float (&v)[M], float (&o)[M / 2], int lane) {
  constexpr int H = M / 2;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    if constexpr (L == 0) {
      const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]),
                                                      __float_as_uint(v[j + H]), false, false);
      o[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else if constexpr (L == 1) {
      const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[j]),
                                                      __float_as_uint(v[j + H]), false, false);
      o[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
      const bool hi = (lane & kBit[L]) != 0;
      const float keep = hi ? v[j + H] : v[j];
      const float send = hi ? v[j] : v[j + H];
      o[j] = keep + dpp_partner<L>(send);
    }
  }
}

// Folds M columns through levels L, L+1, ... until one is left, then sums
// over the remaining levels. Returns the wave's sum of the lane's column.
template <int L, int M>
__device__ __forceinline__ float fold_all(const float (&v)[M], int lane) {
  if constexpr (M == 1) {
    float s = v[0];
    if constexpr (L <= 2) s += dpp_partner<2>(s);
    if constexpr (L <= 3) s += dpp_partner<3>(s);
    if constexpr (L <= 4) s += dpp_partner<4>(s);
    if constexpr (L <= 5) s += dpp_partner<5>(s);
    return s;
  } else {
    float o[M / 2];
    fold_level<L, M>(v, o, lane);
    return fold_all<L + 1, M / 2>(o, lane);
  }
}

// Column of the sum that lane `lane` holds after folding R columns.
template <int R>
__device__ __forceinline__ int folded_column(int lane) {
  int col = 0, m = R;
#pragma unroll
  for (int L = 0; L < 6 && m > 1; ++L) {
    m /= 2;
    if (lane & kBit[L]) col += m;
  }
  return col;
}

// Adds the lanes' sums for `row` across the wave and writes them once per
// column (the lane of each column whose unfolded bits are zero).
template <int R>
__device__ __forceinline__ void flush_row(float* __restrict__ C, int row, const float (&acc)[R],
                                          int lane) {
  static_assert(R == 8 || R == 16 || R == 32, "lane form columns");
  constexpr int kFolds = R == 8 ? 3 : R == 16 ? 4 : 5;
  constexpr int kLowMask = (1 << (6 - kFolds)) - 1;
  const float s = fold_all<0, R>(acc, lane);
  if ((lane & kLowMask) == 0)
    atomic_add_noret(C + static_cast<int64_t>(row) * R + folded_column<R>(lane), s);
}

// The N - 1 factor rows of the lane's record (the slots other than T).
template <int N, typename BT, int R, int T, int K>
__device__ __forceinline__ void lds_rows(const uint32_t (&w)[K], const BT* sB, int plane,
                                         uint4 (&raw)[N - 1][pieces_of<BT, R>()]) {
#pragma unroll
  for (int r = 0; r < N - 1; ++r) {  // record position r holds the r-th slot other than T
    const int c = (r & 1) ? static_cast<int>(w[r / 2] >> 16) : static_cast<int>(w[r / 2] & 0xffffu);
    lds_row_raw<BT, R>(sB, plane, c, raw[r]);
  }
}

// One iteration of a wave: the 64 records in w (one per lane) added to the
// running row `cur` (wave-uniform) and its partial sums acc. With kHalf the
// factor sits in LDS as FP16 (the exact re-encoding of BF16 values in range)
// and every product is one mixed-precision FMA: kv * b_1, times b_2, ...,
// the last row fused with the accumulation (4 operations per column for
// N = 5, against 8 with BF16 rows widened to FP32 first).
// The wave's iteration covers records [it, it + 64); `bound` is the first
// record of row cur + 1, so the iteration stays in row cur when it + 64 <=
// bound (the rows' starts come from the view's row pointer, not from the
// records).
template <int N, typename BT, int R, int T, int K, bool kHalf>
__device__ __forceinline__ void lane_step(const uint32_t (&w)[K], float (&acc)[R], int& cur,
                                          int& bound, RowWindow& win, int it,
                                          const int32_t* __restrict__ rowptr, int I, int lane,
                                          const BT* sB, int plane, float* __restrict__ C) {
  constexpr int kP = pieces_of<BT, R>();
  const float kv = __uint_as_float(w[K - 1]);
  const bool whole = it + kWave <= bound;  // wave-uniform
  float p[R];  // the lane's product coef * v * prod_{s != T} B[c_s, :]
  if constexpr (kHalf) {
    static_assert(sizeof(BT) == 2 && (N - 1) * kP <= 8, "FP16 rows in registers");
    uint4 raw[N - 1][kP];
    lds_rows<N, BT, R, T, K>(w, sB, plane, raw);
#pragma unroll
    for (int j = 0; j < R; ++j) p[j] = fmaf(kv, half_at<R>(raw[0], j), 0.0f);
#pragma unroll
    for (int r = 1; r + 1 < N - 1; ++r) {
#pragma unroll
      for (int j = 0; j < R; ++j) p[j] = fmaf(p[j], half_at<R>(raw[r], j), 0.0f);
    }
    // the last row whole in registers before the branch, so that its pieces
    // stay single 16-byte reads (the compiler otherwise splits one into
    // 4-byte reads, which collide in the LDS banks)
#pragma unroll
    for (int q = 0; q < kP; ++q)
      asm volatile("" ::"v"(raw[N - 2][q].x), "v"(raw[N - 2][q].y), "v"(raw[N - 2][q].z),
                   "v"(raw[N - 2][q].w));
    if (whole) {  // the whole iteration continues the current row
#pragma unroll
      for (int j = 0; j < R; ++j) acc[j] = fmaf(p[j], half_at<R>(raw[N - 2], j), acc[j]);
      return;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) p[j] = fmaf(p[j], half_at<R>(raw[N - 2], j), 0.0f);
  } else {
    if constexpr ((N - 1) * kP <= 8) {
      // all N - 1 rows (at most 32 registers) requested from LDS before the
      // first is used
      uint4 raw[N - 1][kP];
      lds_rows<N, BT, R, T, K>(w, sB, plane, raw);
      unpack_row<BT, R>(raw[0], p);
#pragma unroll
      for (int r = 1; r < N - 1; ++r) {
        float b[R];
        unpack_row<BT, R>(raw[r], b);
#pragma unroll
        for (int j = 0; j < R; ++j) p[j] *= b[j];
      }
    } else {
      // wider rows one at a time (register budget of 1,024-thread workgroups)
      bool first = true;
#pragma unroll
      for (int s = 0; s < N; ++s) {
        if (s == T) continue;
        const int q = s < T ? s : s - 1;  // its record position
        const int c = (q & 1) ? static_cast<int>(w[q / 2] >> 16) : static_cast<int>(w[q / 2] & 0xffffu);
        uint4 raw[kP];
        lds_row_raw<BT, R>(sB, plane, c, raw);
        float b[R];
        unpack_row<BT, R>(raw, b);
#pragma unroll
        for (int j = 0; j < R; ++j) p[j] = first ? b[j] : p[j] * b[j];
        first = false;
      }
    }
    if (whole) {  // the weight applied last, fused with the accumulation
#pragma unroll
      for (int j = 0; j < R; ++j) acc[j] = fmaf(p[j], kv, acc[j]);
      return;
    }
#pragma unroll
    for (int j = 0; j < R; ++j) p[j] *= kv;
  }
  // the row changes inside this iteration
  const int row = lane_row(rowptr, I, cur, it + lane, lane, win);
  const int last = __builtin_amdgcn_readlane(row, kWave - 1);
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j] += (row == cur) ? p[j] : 0.0f;
  flush_row<R>(C, cur, acc, lane);
  const bool between = row != cur && row != last;
  if (__ballot(between) != 0) {  // rows that begin and end in this iteration
    const int key = between ? row : INT_MAX;
    const int next_key = next_lane_i32(key, INT_MAX);
    const bool ends = between && next_key != key;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const float sj = wave_seg_sum(key, between ? p[j] : 0.0f);
      if (ends) atomic_add_noret(C + static_cast<int64_t>(row) * R + j, sj);
    }
  }
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j] = (row == last) ? p[j] : 0.0f;
  cur = last;
  bound = next_row_start(rowptr, I, cur, lane, win);
}

// A wave runs records [e0, e1) of view T (wave-uniform, both multiples of
// 64, e0 < e1). The record loads run kDepth iterations ahead through a ring
// of registers; near the end of the range they re-read its last iteration
// (in bounds, never consumed), so that no load sits under a branch.
template <int N, typename BT, int R, int T, bool kHalf>
__device__ __forceinline__ void lane_view_range(int e0, int e1, int row0,
                                                const uint32_t* __restrict__ rec,
                                                const int32_t* __restrict__ rowptr, int I,
                                                const BT* sB, int plane, float* __restrict__ C) {
  constexpr int K = lane_words_of(N);
  constexpr int kDepth = depth_of(R);
  const int lane = threadIdx.x & (kWave - 1);
  const int e_last = e1 - kWave;  // first record of the range's last iteration
  uint32_t ring[kDepth][K];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) load_record<K>(rec, min(e0 + d * kWave, e_last) + lane, ring[d]);
  int cur = row0;  // the row of record e0
  RowWindow win = load_row_window(rowptr, I, cur + 1, lane);  // the starts of the next rows
  int bound = __builtin_amdgcn_readlane(win.start, 0);
  float acc[R];
#pragma unroll
  for (int j = 0; j < R; ++j) acc[j] = 0.0f;
  int it = e0;
  // whole groups of kDepth iterations: slot d holds iteration it + d * 64
  for (; it + kDepth * kWave <= e1; it += kDepth * kWave) {
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      uint32_t w[K];
#pragma unroll
      for (int q = 0; q < K; ++q) w[q] = ring[d][q];
      load_record<K>(rec, min(it + (kDepth + d) * kWave, e_last) + lane, ring[d]);
      lane_step<N, BT, R, T, K, kHalf>(w, acc, cur, bound, win, it + d * kWave, rowptr, I, lane,
                                       sB, plane, C);
    }
  }
  // the last iterations (fewer than kDepth), already in the ring
#pragma unroll
  for (int d = 0; d + 1 < kDepth; ++d)
    if (it + d * kWave < e1)
      lane_step<N, BT, R, T, K, kHalf>(ring[d], acc, cur, bound, win, it + d * kWave, rowptr, I,
                                       lane, sB, plane, C);
  flush_row<R>(C, cur, acc, lane);
}

template <int N, typename BT, int R, bool kHalf>
__device__ __forceinline__ void lane_view_slot(int t, int e0, int e1, int row0, const LaneViews& vs,
                                               int I, const BT* sB, int plane, float* C) {
  switch (t) {
    case 0: lane_view_range<N, BT, R, 0, kHalf>(e0, e1, row0, vs.rec[0], vs.rowptr[0], I, sB, plane, C); break;
    case 1: lane_view_range<N, BT, R, 1, kHalf>(e0, e1, row0, vs.rec[1], vs.rowptr[1], I, sB, plane, C); break;
    case 2: lane_view_range<N, BT, R, 2, kHalf>(e0, e1, row0, vs.rec[2], vs.rowptr[2], I, sB, plane, C); break;
    case 3:
      if constexpr (N > 3)
        lane_view_range<N, BT, R, 3, kHalf>(e0, e1, row0, vs.rec[3], vs.rowptr[3], I, sB, plane, C);
      break;
    default:
      if constexpr (N > 4)
        lane_view_range<N, BT, R, 4, kHalf>(e0, e1, row0, vs.rec[4], vs.rowptr[4], I, sB, plane, C);
      break;
  }
}

// The waves' walk over the tiles of the concatenated views. Workgroup b owns
// tiles b, b + G, b + 2G, ... (G workgroups), a sample of every view and
// region; its waves take them one at a time from a counter in LDS, so a wave
// that drew cheap tiles (long runs of one row) takes more of them and the
// workgroup ends with its last tile, not with its slowest wave. `next` holds
// kLaneWaves (the first tiles go to the waves in order) when this begins.
template <int N, typename BT, int R, bool kHalf>
__device__ __forceinline__ void lane_tiles(const LaneViews& vs, int I, const BT* sB, int plane,
                                           float* C, int* next) {
  const int lane = threadIdx.x & (kWave - 1);
  int k = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (;;) {
    const int tile = blockIdx.x + k * static_cast<int>(gridDim.x);
    if (tile >= vs.tile0[N]) break;
    int claim = 0;
    if (lane == 0) claim = atomicAdd(next, 1);  // the wave's next slot, claimed early
    int t = 0;
#pragma unroll
    for (int q = 1; q < N; ++q) t += (tile >= vs.tile0[q]) ? 1 : 0;
    // wave-uniform: scalar registers and branches
    t = __builtin_amdgcn_readfirstlane(t);
    const int local = tile - vs.tile0[t];
    const int e0 = __builtin_amdgcn_readfirstlane(local * kLaneTile);
    const int e1 = __builtin_amdgcn_readfirstlane(min(vs.nrec[t], e0 + kLaneTile));
    const int row0 = __builtin_amdgcn_readfirstlane(vs.tile_row[t][local]);
    lane_view_slot<N, BT, R, kHalf>(t, e0, e1, row0, vs, I, sB, plane, C);
    k = __builtin_amdgcn_readfirstlane(claim);
  }
}

// One 1,024-thread workgroup per CU stages B (I x R, row-major, a multiple
// of 16 bytes per row) in LDS piece-major, then walks its share of the
// tiles. A BF16 factor is staged as FP16 when every value converts exactly
// (the workgroups all see the same B, so all decide alike), else as BF16.
template <int N, typename BT, int R>
__global__ __launch_bounds__(kLaneThreads) void mttkrp_views_lane_kernel(LaneViews vs,
                                                                       const BT* __restrict__ B,
                                                                       int I,
                                                                       float* __restrict__ C) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int kP = pieces_of<BT, R>();
  const int plane = I * 16;
  const int pieces = I * kP;
  const BT* sB = reinterpret_cast<const BT*>(lds_raw);
  int* next = reinterpret_cast<int*>(lds_raw + static_cast<size_t>(plane) * kP);  // tile slot
  int* inexact_flag = next + 1;
  if (threadIdx.x == 0) {
    *next = kLaneWaves;  // the first tiles go to the waves in order
    *inexact_flag = 0;
  }
  const uint4* src = reinterpret_cast<const uint4*>(B);
  uint4* dst = reinterpret_cast<uint4*>(lds_raw);
  if constexpr (sizeof(BT) == 2 && (N - 1) * kP <= 8) {
    __syncthreads();  // the flag cleared before any thread sets it
    bool inexact = false;
    for (int q = threadIdx.x; q < pieces; q += kLaneThreads)
      dst[(q % kP) * I + q / kP] = bf16_piece_to_half(src[q], inexact);
    if (inexact) atomicOr(inexact_flag, 1);
    __syncthreads();
    if (*inexact_flag == 0) {
      lane_tiles<N, BT, R, true>(vs, I, sB, plane, C, next);
      return;
    }
  }
  for (int q = threadIdx.x; q < pieces; q += kLaneThreads) dst[(q % kP) * I + q / kP] = src[q];
  __syncthreads();
  lane_tiles<N, BT, R, false>(vs, I, sB, plane, C, next);
}

template <int N, typename BT, int R>
int launch_lane(const Tensor* tn, const BT* B, float* C, size_t lds, int cus, hipStream_t s) {
  LaneViews vs{};
  int tiles = 0;
  for (int t = 0; t < N; ++t) {
    vs.rec[t] = tn->lview[t];
    vs.rowptr[t] = tn->lrowptr[t];
    vs.tile_row[t] = tn->ltile_row[t];
    vs.nrec[t] = static_cast<int>(tn->lnnz[t]);
    vs.tile0[t] = tiles;
    tiles += static_cast<int>((tn->lnnz[t] + kLaneTile - 1) / kLaneTile);
  }
  for (int t = N; t <= 5; ++t) vs.tile0[t] = tiles;
  if (tiles == 0) return SYSTEC_OK;
  auto kern = mttkrp_views_lane_kernel<N, BT, R>;
  hipFuncAttributes attr{};
  int rc = check_hip(hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kern)),
                     "hipFuncGetAttributes");
  if (rc) return rc;
  if (attr.sharedSizeBytes != 0)
    return fail(SYSTEC_EDEVICE, "mttkrp lane view kernel: unexpected static LDS");
  rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds)),
                     "hipFuncSetAttribute(dynamic LDS)");
  if (rc) return rc;
  const int grid = std::max(1, std::min(cus, (tiles + kLaneWaves - 1) / kLaneWaves));
  kern<<<dim3(grid), dim3(kLaneThreads), lds, s>>>(vs, B, static_cast<int>(tn->dim), C);
  return check_launch("mttkrp lane view kernel");
}

template <int N, typename BT>
int launch_lane_r(const Tensor* tn, const BT* B, int R, float* C, size_t lds, int cus,
                  hipStream_t s) {
  switch (R) {
    case 8:
      if constexpr (sizeof(BT) == 2) return launch_lane<N, BT, 8>(tn, B, C, lds, cus, s);
      return -1;
    case 16: return launch_lane<N, BT, 16>(tn, B, C, lds, cus, s);
    case 32: return launch_lane<N, BT, 32>(tn, B, C, lds, cus, s);
    default: return -1;
  }
}

// ---- packed views ------------------------------------------------------------

// Record e of packed view T from the view's entry e (weight coef * v, the
// product the kernels over the unpacked views form), or a padding record of
// weight 0 (it belongs to the view's last output row). The record holds
// the indices of the slots other than T; the output row is the view's
// row pointer's business.
template <int N, int T>
__global__ void lane_pack_kernel(IdxPtrs ip, const float* __restrict__ val, int m, int padded,
                                 uint32_t* __restrict__ out) {
  constexpr int K = lane_words_of(N);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= padded) return;
  int c[N];
  float kv = 0.0f;
  if (e < m) {
#pragma unroll
    for (int q = 0; q < N; ++q) c[q] = ip.p[q][e];
    kv = slot_coef<N, T>(equality_mask_of(c, N)) * val[e];
  } else {
#pragma unroll
    for (int q = 0; q < N; ++q) c[q] = 0;
  }
  int o[N - 1];
#pragma unroll
  for (int s = 0, r = 0; s < N; ++s)
    if (s != T) o[r++] = c[s];
  uint32_t* dst = out + static_cast<int64_t>(e) * K;
#pragma unroll
  for (int q = 0; q + 1 < K; ++q) {
    const uint32_t lo = static_cast<uint32_t>(o[2 * q]);
    const uint32_t hi = 2 * q + 1 < N - 1 ? static_cast<uint32_t>(o[2 * q + 1]) : 0u;
    dst[q] = lo | (hi << 16);
  }
  dst[K - 1] = __float_as_uint(kv);
}

// The row pointer of a packed view: rowptr[r] = the first record whose row
// is r or more (records [m, padded) belong to the last row), for r in [0, I];
// and the row of each tile's first record.
__global__ void lane_rowptr_kernel(const int32_t* __restrict__ rows, int m, int padded, int I,
                                   int32_t* __restrict__ rowptr, int32_t* __restrict__ tile_row) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= padded) return;
  const int last_row = rows[m - 1];
  const int row = e < m ? rows[e] : last_row;
  const int prev = e == 0 ? -1 : (e - 1 < m ? rows[e - 1] : last_row);
  for (int r = prev + 1; r <= row; ++r) rowptr[r] = e;  // rows starting here (empty ones too)
  if (e == padded - 1)
    for (int r = row + 1; r <= I; ++r) rowptr[r] = padded;
  if (e % kLaneTile == 0) tile_row[e / kLaneTile] = row;
}

template <int N, int T>
int pack_view(const Tensor* t, uint32_t* out, hipStream_t s) {
  IdxPtrs ip{};
  for (int q = 0; q < N; ++q) ip.p[q] = t->vidx[T][q];
  const int m = static_cast<int>(t->vnnz[T]);
  const int padded = static_cast<int>(t->lnnz[T]);
  lane_pack_kernel<N, T><<<(padded + 255) / 256, 256, 0, s>>>(ip, t->vval[T], m, padded, out);
  if (const int rc = check_launch("mttkrp lane pack kernel")) return rc;
  lane_rowptr_kernel<<<(padded + 255) / 256, 256, 0, s>>>(t->vidx[T][T], m, padded,
                                                          static_cast<int>(t->dim), t->lrowptr[T],
                                                          t->ltile_row[T]);
  return check_launch("mttkrp lane row pointer kernel");
}

template <int N>
int pack_view_slot(const Tensor* t, int v, uint32_t* out, hipStream_t s) {
  switch (v) {
    case 0: return pack_view<N, 0>(t, out, s);
    case 1: return pack_view<N, 1>(t, out, s);
    case 2: return pack_view<N, 2>(t, out, s);
    case 3:
      if constexpr (N > 3) return pack_view<N, 3>(t, out, s);
      return fail(SYSTEC_EINVAL, "mttkrp lane pack: slot out of range");
    default:
      if constexpr (N > 4) return pack_view<N, 4>(t, out, s);
      return fail(SYSTEC_EINVAL, "mttkrp lane pack: slot out of range");
  }
}

int lane_limits(int* lds_limit, int* cus) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc) rc = check_hip(hipDeviceGetAttribute(lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                          "hipDeviceGetAttribute(max shared memory)");
  if (!rc) rc = check_hip(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev),
                          "hipDeviceGetAttribute(CU count)");
  return rc;
}

bool lane_shape(int64_t I, size_t es, int64_t R, int lds_limit) {
  // B in one workgroup's LDS in whole 16-byte pieces per row
  return I * R * static_cast<int64_t>(es) + kLaneExtraLds <= lds_limit &&
         (R * static_cast<int64_t>(es)) % 16 == 0 &&
         (R == 16 || R == 32 || (R == 8 && es == 2));
}

}  // namespace

int build_lane_views(Tensor* t, hipStream_t s) {
  int limit = 0, cus = 0;
  int rc = lane_limits(&limit, &cus);
  if (rc) return rc;
  // the smallest factor the form takes (8 BF16 columns, 16 bytes a row)
  // must fit; the indices must fit 16 bits
  if (t->kind != 1 || t->short_runs || t->nnz == 0 || t->dim * 16 + kLaneExtraLds > limit ||
      t->dim > 65535)
    return SYSTEC_OK;
  const int N = t->order;
  const int K = lane_words_of(N);
  for (int v = 0; v < N && !rc; ++v) {
    t->lnnz[v] = (t->vnnz[v] + kWave - 1) / kWave * kWave;
    if (t->lnnz[v] == 0) continue;
    rc = tensor_alloc(t, &t->lview[v], static_cast<size_t>(t->lnnz[v]) * K);
    if (!rc) rc = tensor_alloc(t, &t->lrowptr[v], static_cast<size_t>(t->dim) + 1);
    if (!rc)
      rc = tensor_alloc(t, &t->ltile_row[v], static_cast<size_t>((t->lnnz[v] + kLaneTile - 1) / kLaneTile));
    if (rc) break;
    rc = N == 3   ? pack_view_slot<3>(t, v, t->lview[v], s)
         : N == 4 ? pack_view_slot<4>(t, v, t->lview[v], s)
                  : pack_view_slot<5>(t, v, t->lview[v], s);
  }
  if (!rc) t->lane_words = K;
  return rc;
}

bool mttkrp_lane_shape_fits(int64_t I, systec_dtype bdt, int64_t R) {
  int limit = 0, cus = 0;
  if (I < 1 || I > 65535 || lane_limits(&limit, &cus) != SYSTEC_OK) return false;
  return lane_shape(I, bdt == SYSTEC_F32 ? 4 : 2, R, limit);
}

int launch_mttkrp_views_lane(const Tensor* t, const void* B, systec_dtype bdt, int64_t R,
                             float* C, hipStream_t s) {
  const size_t es = bdt == SYSTEC_F32 ? 4 : 2;
  const size_t lds = static_cast<size_t>(t->dim) * R * es + kLaneExtraLds;  // B, then counter and flag
  int limit = 0, cus = 0;
  int rc = lane_limits(&limit, &cus);
  if (rc) return rc;
  // packed views exist for tensors with long runs of output rows (short runs
  // would flush rows in almost every iteration) and small index spaces
  const bool fits = t->lane_words > 0 && lane_shape(t->dim, es, R, limit) &&
                    (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  if (!fits) return -1;
  rc = launch_fill_f32(C, t->dim * R, s);
  if (rc != SYSTEC_OK) return rc;
  const int r = static_cast<int>(R);
  LaunchTimer timer(s);
  if (bdt == SYSTEC_F32) {
    const auto* b = static_cast<const float*>(B);
    switch (t->order) {
      case 3: return launch_lane_r<3, float>(t, b, r, C, lds, cus, s);
      case 4: return launch_lane_r<4, float>(t, b, r, C, lds, cus, s);
      default: return launch_lane_r<5, float>(t, b, r, C, lds, cus, s);
    }
  }
  const auto* b = static_cast<const uint16_t*>(B);
  switch (t->order) {
    case 3: return launch_lane_r<3, uint16_t>(t, b, r, C, lds, cus, s);
    case 4: return launch_lane_r<4, uint16_t>(t, b, r, C, lds, cus, s);
    default: return launch_lane_r<5, uint16_t>(t, b, r, C, lds, cus, s);
  }
}

}  // namespace systec
