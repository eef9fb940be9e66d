// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "systec.h"

namespace systec {

// ---- error reporting (abi.cpp) -------------------------------------------
int fail(int status, const std::string& msg);
int check_hip(hipError_t e, const char* what);
// Checks the launch that was just issued; records an error message on failure.
int check_launch(const char* what);

// ---- kernel timing (abi.cpp) ---------------------------------------------
// Brackets one hot-kernel launch with events when timing is enabled.
struct LaunchTimer {
  explicit LaunchTimer(hipStream_t s);
  ~LaunchTimer();
  hipStream_t stream;
  hipEvent_t start = nullptr;
};

// ---- device helpers --------------------------------------------------------
constexpr int kWave = 64;

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);  // exact widening
}

template <typename T>
__device__ __forceinline__ float load_f32(const T* p, int64_t i);
template <>
__device__ __forceinline__ float load_f32<float>(const float* p, int64_t i) {
  return p[i];
}
template <>
__device__ __forceinline__ float load_f32<uint16_t>(const uint16_t* p, int64_t i) {
  return bf16_to_f32(p[i]);
}

// FP32 atomic add whose result is unused (hardware global_atomic_add_f32).
__device__ __forceinline__ void atomic_add_noret(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- launchers (one per hot kernel family) ---------------------------------
// All sizes are validated by the caller (abi.cpp).
int launch_fill_f32(float* p, int64_t n, hipStream_t s);
int launch_ssymv(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, float* y, bool symmetric,
                 hipStream_t s);
int launch_syprd(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, double* out,
                 hipStream_t s);
// launch_syprd with its partials in the library's fixed per-device scratch
// (allocates nothing; EINVAL when n + nnz exceeds what the scratch holds).
int launch_syprd_noalloc(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                         const float* val, const void* x, systec_dtype xdt, double* out,
                         hipStream_t s);
int launch_mttkrp(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                  const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                  bool symmetric, hipStream_t s);
// MTTKRP over the slot views with B staged in LDS by column slices; usable
// when mttkrp_lds_width(I, bdt, R) > 0 (the slice width in columns).
int mttkrp_lds_width(int64_t I, systec_dtype bdt, int64_t R);
int launch_quantize_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s);
int launch_expansion_stats(int order, int64_t nnz, const int32_t* const* idx,
                           unsigned long long* d_counts /* 17 */, hipStream_t s);
int launch_validate_csr_upper(int64_t n, int64_t nnz, const int32_t* rowptr,
                              const int32_t* col, unsigned int* d_flags, hipStream_t s);
int launch_validate_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                        unsigned int* d_flags, hipStream_t s);
int expand_csr_size(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                    int64_t* full_nnz, hipStream_t s);
int expand_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
               const float* val, int32_t* full_rowptr, int32_t* full_col, float* full_val,
               hipStream_t s);
int expand_coo_size(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                    int64_t* full_nnz, hipStream_t s);
int expand_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx, const float* val,
               int32_t* const* out_idx, float* out_val, hipStream_t s);

// ---- prepared operands (plan.hip) -------------------------------------------
// A matrix in the symmetric panel format: the stored upper triangle cut into
// panels of H consecutive rows; inside a panel the entries are sorted by
// (column, row) and padded to a multiple of kPanelTile entries (padding:
// value 0 at the panel's first row and last column, so the columns stay
// sorted). The kernel keeps the
// panel's row sums in LDS and reduces the column side by segments.
// A tensor as slot views: for each slot t, the canonical entries whose slot t
// starts a run of equal indices, sorted by their slot-t index (stable), so
// that every output update of view t is a segmented reduction.
constexpr int kPanelTile = 512;
constexpr int64_t kShortRun = 64;
struct ServeTensor;
struct ServeUnit;
struct Tensor {
  int kind = 0;  // 0: matrix (panel format), 1: tensor (slot views)
  int order = 0;
  int64_t dim = 0;
  int64_t nnz = 0;
  int64_t effective_nnz = 0;
  uint64_t bytes = 0;
  // matrix
  int panel_rows = 0;
  int npanels = 0;
  int64_t padded = 0;
  int32_t* pcol = nullptr;
  uint16_t* prow = nullptr;
  float* pval = nullptr;
  // The SSYMV kernels' index stream: per entry one word holding the column's
  // offset from its step's base column (the high 32 - log2(H) bits) and the
  // row in the panel (the low log2(H) bits); per step of 64 entries the base
  // column, with bit 31 set where the step's columns span too much for the
  // offsets (those steps read pcol and prow instead).
  uint32_t* ppack = nullptr;
  int32_t* pbase = nullptr;
  int nchunks = 0;
  int32_t* chunk_panel = nullptr;
  int32_t* chunk_tile_begin = nullptr;
  int32_t* chunk_tile_end = nullptr;
  // entry index where the chunk's padding starts (padding entries hold
  // value 0, which is no contribution to a sum but is one to a minimum)
  int32_t* chunk_valid_end = nullptr;
  std::vector<int32_t> h_chunk_panel, h_chunk_tile_begin, h_chunk_tile_end;  // host copies
  // Column segments of the panel SSYMV: the maximal runs of equal column
  // inside each 512-entry tile, numbered in entry order (tile t's segments
  // are [seg_tile0[t], seg_tile0[t + 1])). The kernel writes one FP32 sum per
  // segment to work_seg instead of adding it to y with an atomic, and a
  // second pass adds each column's segments, listed by column in
  // seg_ids[seg_colptr[c] .. seg_colptr[c + 1]) (in segment order).
  int64_t nsegs = 0;
  int32_t* seg_tile0 = nullptr;
  int32_t* seg_colptr = nullptr;
  int32_t* seg_ids = nullptr;
  float* work_seg = nullptr;
  // vertex relabeling (matrix prepared with its vertices ordered by degree):
  // the panels hold P A P^T; perm[new] = old, inv[old] = new
  bool relabeled = false;
  int32_t* perm = nullptr;
  int32_t* inv = nullptr;
  // work buffers of a prepared matrix, allocated with it so that a call
  // allocates nothing: the input and output in the stored vertex order (a
  // relabeled matrix: n elements each) and SYPRD's per-chunk partials. Calls
  // that use them hold work_mu while they enqueue and wait on the device for
  // the previous user (work_done), so calls on different streams that share
  // the handle run one after another on the device.
  void* work_x = nullptr;
  float* work_y = nullptr;
  float* work_partial = nullptr;
  mutable std::mutex work_mu;
  mutable hipEvent_t work_done = nullptr;
  mutable bool work_recorded = false;
  // tensor
  int64_t vnnz[5] = {0, 0, 0, 0, 0};
  // Fewer than kShortRun stored entries per index on average: the views' runs
  // of equal output rows are short. Above 16 columns the view kernels then
  // take one lane per column (each entry one contiguous row update), which
  // measured faster there than the vector lanes' per-iteration sums of short
  // rows (use_vector_lanes).
  bool short_runs = false;
  int32_t* vidx[5][5] = {};
  float* vval[5] = {};
  // Packed views for the one-lane-per-entry MTTKRP with B in LDS, built
  // when that form can apply (I * 16 bytes fits one workgroup's LDS, so I <
  // 65,536, and the runs are long): view t as records of lane_words 32-bit
  // words, the N - 1 indices other than slot t as 16-bit halves (two to a
  // word, in slot order) and then coef[mask][t] * v in FP32, grouped by the
  // output index c_t through a row pointer (the leading-index level of a
  // compressed fiber layout); each view padded to a multiple of 64 records
  // of weight 0 that belong to its last output row.
  uint32_t* lview[5] = {};
  int32_t* lrowptr[5] = {};    // per view: first record of each output row (I + 1)
  int32_t* ltile_row[5] = {};  // per view: output row of each 512-record tile's first record
  int64_t lnnz[5] = {0, 0, 0, 0, 0};  // padded record counts
  int lane_words = 0;
  // serving (built at registration)
  ServeTensor* d_serve = nullptr;
  ServeUnit* d_units = nullptr;
  std::vector<void*> allocations;
};
// Device memory owned by a prepared operand (freed with it, counted in its
// bytes).
template <typename T>
int tensor_alloc(Tensor* t, T** p, size_t count) {
  void* q = nullptr;
  const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess)
    return fail(SYSTEC_ENOMEM, std::string("hipMalloc (prepared operand): ") + hipGetErrorString(e));
  t->allocations.push_back(q);
  t->bytes += bytes;
  *p = static_cast<T*>(q);
  return SYSTEC_OK;
}

// Holds a prepared matrix's work buffers for one call: the host lock while
// the call enqueues, and on the device the call's stream waits for the
// previous holder's work (any stream) and marks the end of its own.
class WorkLease {
 public:
  WorkLease(const Tensor* t, hipStream_t s) : t_(t), s_(s), lock_(t->work_mu) {
    if (t_->work_recorded) rc_ = check_hip(hipStreamWaitEvent(s_, t_->work_done, 0),
                                           "hipStreamWaitEvent");
  }
  ~WorkLease() {
    if (hipEventRecord(t_->work_done, s_) == hipSuccess) t_->work_recorded = true;
  }
  int status() const { return rc_; }

 private:
  const Tensor* t_;
  hipStream_t s_;
  std::lock_guard<std::mutex> lock_;
  int rc_ = SYSTEC_OK;
};

// relabel: 1 orders the vertices by degree, 0 keeps them, -1 decides from the
// degree skew.
int tensor_create_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                      const float* val, int panel_rows, int relabel, hipStream_t s,
                      Tensor** out);
int tensor_create_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                      const float* val, hipStream_t s, Tensor** out);
void tensor_free(Tensor* t);
// The same with x and y (or x alone) already in the matrix's stored vertex
// order: no permutations.
int launch_ssymv_panel_stored(const Tensor* t, const void* x, systec_dtype xdt, float* y,
                              hipStream_t s);
int launch_syprd_panel_stored(const Tensor* t, const void* x, systec_dtype xdt, double* out,
                              hipStream_t s);
// s = x^T A x for a prepared matrix (out: device double[1]).
int launch_syprd_panel(const Tensor* t, const void* x, systec_dtype xdt, double* out,
                       hipStream_t s);
// Vertex permutations of a relabeled matrix (n elements): xp[i] = x[perm[i]]
// with yp cleared (if not null), and y[j] = yp[inv[j]].
int launch_permute_in(int n, const int32_t* perm, const void* x, systec_dtype xdt, void* xp,
                      float* yp, hipStream_t s);
int launch_permute_out(int n, const int32_t* inv, const float* yp, float* y, hipStream_t s);
int launch_ssymv_panel(const Tensor* t, const void* x, systec_dtype xdt, float* y,
                       hipStream_t s);
int launch_mttkrp_views(const Tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                        hipStream_t s);
// Bellman-Ford update y[i] = min_j (A[i,j] + d[j]) over the stored
// coordinates of the symmetric matrix (bellman.hip): over the canonical CSR,
// and over a prepared matrix (panel format).
int launch_bellman_ford(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                        const float* val, const float* d, float* y, hipStream_t s);
int launch_bellman_ford_panel(const Tensor* t, const float* d, float* y, hipStream_t s);
// TTM with visible output symmetry (ttm.hip): C[j,l,r] = sum_k T[k,j,l]
// B[k,r] over canonical 3-index COO; the canonical half j <= l is computed,
// then copied to the other half if mirror.
int launch_ttm(int64_t I, int64_t nnz, const int32_t* const* idx, const float* val,
               const void* B, systec_dtype bdt, int64_t R, float* C, bool mirror,
               hipStream_t s);
// MTTKRP of a tensor symmetric within consecutive parts of its slots
// (mttkrp_partial.hip), one factor matrix per part, output mode 1.
int launch_mttkrp_partial(int order, int nparts, const int32_t* part_sizes, int64_t I,
                          int64_t nnz, const int32_t* const* idx, const float* val,
                          const void* const* F, systec_dtype fdt, int64_t R, float* C,
                          hipStream_t s);
// One symmetric CP-ALS step around the prepared tensor's MTTKRP (cp.hip):
// C = MTTKRP(T, B), G = B^T B, B_new = C (G^(N-1))^-1, fit = {||T||^2,
// <T,[[B]]>, ||[[B]]||^2, ||T - [[B]]||^2}. R <= 64.
int launch_cp_step(const Tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                   float* B_new, float* G, double* fit, hipStream_t s);
int launch_mttkrp_views_lds(const Tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                            hipStream_t s);
// One lane per view entry with all of B staged in LDS (mttkrp_lane.hip);
// -1 (nothing launched) unless B fits one workgroup's LDS, R is 8 (BF16), 16
// or 32 and the tensor's runs are long.
int launch_mttkrp_views_lane(const Tensor* t, const void* B, systec_dtype bdt, int64_t R,
                             float* C, hipStream_t s);
// Builds the packed views (Tensor::lview) of a tensor whose views exist, if
// the one-lane-per-entry form can apply to it; else leaves them empty.
int build_lane_views(Tensor* t, hipStream_t s);
// One-shot SSYMV with the column side binned by column range
// (ssymv_bucket.hip) for matrices of at least kBucketNnzMin stored entries
// and at most 2^26 rows; -1 (nothing launched) otherwise. y must be zeroed.
constexpr int64_t kBucketNnzMin = int64_t(1) << 18;
int launch_ssymv_bucketed(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                          const float* val, const void* x, systec_dtype xdt, float* y,
                          hipStream_t s);
// Whether the one-lane-per-entry form applies to this shape (B fits one
// workgroup's LDS, R is 8 in BF16, 16 or 32); the tensor's runs decide the
// rest.
bool mttkrp_lane_shape_fits(int64_t I, systec_dtype bdt, int64_t R);

// ---- serving step (serve_kernel.hip) ----------------------------------------
// A prepared operand as the serving kernels see it (device memory, built when
// the operand is registered), with its work units: SSYMV {panel, first tile,
// end tile}, MTTKRP {view, first entry, end entry}.
struct ServeUnit {
  int32_t a, b, c, d;
};
struct ServeTensor {
  int32_t kind;   // 0: matrix (panel format), 1: tensor (slot views)
  int32_t order;
  int32_t dim;    // n or I
  int32_t H;      // panel rows (matrix)
  const void* p[5][5];  // matrix: p[0] = {pcol, prow, pval, ppack, pbase}; tensor: p[v] = view v's indices
  const float* val[5];  // tensor: view values
  const ServeUnit* units;
};
// One request's share of a step: units [unit0, unit0 + count) of its
// operand run as items [item0, item0 + count) of the launch.
struct StepReq {
  const ServeTensor* t;
  const void* in;  // x or B
  float* out;      // y or C
  int32_t unit0, item0, R, dtype;
};
// Everything a step launch needs travels in its kernel arguments (1.3 KB),
// so a step costs no host-to-device copy.
constexpr int kStepReqs = 32;
struct StepArgs {
  int32_t nreq, nitems;
  StepReq req[kStepReqs];  // ascending item0
};
struct ZeroArgs {
  int32_t n, pad;
  float* ptr[kStepReqs];
  int64_t count[kStepReqs];
};
// Prepared SSYMV panels: 8,192 rows (32 KiB of FP32 row sums in LDS, 48 KiB
// with the staged BF16 x slice, so three workgroups share a CU), run by
// 512-thread workgroups.
constexpr int kPanelRows = 8192;
constexpr int kPanelThreads = 512;
constexpr int kServeBlock = kPanelThreads;  // SSYMV step kernel
constexpr int kServeMttkrpBlock = 256; // MTTKRP step kernel
constexpr int kServeLds = kPanelRows * 4;  // bytes: the FP32 row sums of one panel
constexpr int kServeLdsStaged = kPanelRows * (4 + 2);  // and the panel's BF16 x slice
// Zeroes the outputs of newly admitted requests; runs on a stream before
// its step launches.
int launch_serve_prologue(const ZeroArgs& z, hipStream_t s);
// Step kernel variants: kind 0 is SSYMV (one variant); kinds 3, 4, 5 are
// MTTKRP of that order, variant = 8 * (input is BF16) + 4 * (vector lanes:
// use_vector_lanes, R a multiple of the class's lane width and the input
// aligned to it) + lane class (R <= 8, 16, 32, 64).
constexpr int kStepVariants = 16;
// Lane width (columns per lane) of the MTTKRP vector-lane kernels for a block
// of `cols` columns of a factor with R columns of `elem_bytes`-byte elements:
// the widest of 8, 4, 2 columns that fits 16 bytes, divides R and leaves at
// least four lanes per row (two for blocks narrower than eight columns); 0 if
// R is odd (no vector lanes).
constexpr int lane_vec_width(int cols, int64_t R, int elem_bytes) {
  for (int v = 8; v >= 2; v /= 2)
    if (v * elem_bytes <= 16 && R % v == 0 && (v * 4 <= cols || v == 2)) return v;
  return 0;
}
// Whether the view kernels use vector lanes for R columns of a tensor.
inline bool use_vector_lanes(bool short_runs, int64_t R) { return !(short_runs && R > 16); }
inline int step_variant(int dtype, int64_t R, const void* in, bool short_runs) {
  const int lane_class = R <= 8 ? 0 : R <= 16 ? 1 : R <= 32 ? 2 : 3;
  const int esize = dtype == SYSTEC_BF16 ? 2 : 4;
  const int L = 8 << lane_class;
  const int V = lane_vec_width(L, L, esize);  // the lane width of the class's kernel
  const bool vec_lanes = use_vector_lanes(short_runs, R) && V != 0 && R % V == 0 &&
                         reinterpret_cast<uintptr_t>(in) % static_cast<uintptr_t>(V * esize) == 0;
  return (dtype == SYSTEC_BF16 ? 8 : 0) + (vec_lanes ? 4 : 0) + lane_class;
}
// Runs the step kernel of one (kind, variant): one workgroup per item.
int launch_serve_step(int kind, int variant, const StepArgs& a, hipStream_t s);
// Once per device before the first step: the SSYMV step kernel's LDS limit.
int serve_init_kernels();

// ---- multiplicity rule (host and device) ----------------------------------
// For a sorted tuple of `order` indices whose equality pattern is `mask`
// (bit t set when c[t] == c[t+1]) the number of distinct permutations is
// order! / prod(run length!). Slot t that starts a run of length m gets the
// coefficient (distinct permutations) * m / order, the number of permutations
// that put that run's value in the output slot; other slots get 0.
struct CoefTable {
  float coef[16][5];
  int32_t mult[16];
};

constexpr int64_t cfact(int n) { return n <= 1 ? 1 : n * cfact(n - 1); }

constexpr CoefTable make_coef_table(int order) {
  CoefTable t{};
  for (int mask = 0; mask < 16; ++mask) {
    for (int s = 0; s < 5; ++s) t.coef[mask][s] = 0.0f;
    t.mult[mask] = 0;
    if (mask >= (1 << (order - 1))) continue;
    int run_len[5] = {0, 0, 0, 0, 0};
    int run_start[5] = {0, 0, 0, 0, 0};
    int runs = 0;
    for (int s = 0; s < order; ++s) {
      bool continues = s > 0 && ((mask >> (s - 1)) & 1);
      if (!continues) {
        run_start[runs] = s;
        run_len[runs] = 0;
        ++runs;
      }
      ++run_len[runs - 1];
    }
    int64_t denom = 1;
    for (int r = 0; r < runs; ++r) denom *= cfact(run_len[r]);
    int64_t mult = cfact(order) / denom;
    t.mult[mask] = static_cast<int32_t>(mult);
    for (int r = 0; r < runs; ++r)
      t.coef[mask][run_start[r]] = static_cast<float>(mult * run_len[r] / order);
  }
  return t;
}

}  // namespace systec

// The opaque handle of the C ABI.
struct systec_tensor {
  systec::Tensor* impl;
};
