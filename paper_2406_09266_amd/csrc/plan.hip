// Prepared operands: the canonical entries rearranged once into a layout
// that lets every output update become a register or LDS reduction.
//
// This is the data rearrangement the paper keeps outside its timings
// (Sec. 5.2: rearranging data before or after a kernel is not timed) and the
// symmetry-aware format it names as future work (Sec. 7). Both layouts keep
// only canonical entries; they change their order, not their meaning.
//
// Matrix panel format. Rows are cut into panels of H rows. Inside a panel the
// stored entries (i <= j) are sorted by (j, i). The SSYMV kernel then keeps
// the panel's row sums y[i] in LDS, and the column-side updates y[j] += a x[i]
// arrive sorted by j, so they reduce by segments and leave the workgroup as
// one atomic per (panel, column) instead of one per entry.
//
// Tensor slot views. For MTTKRP, view t holds the canonical entries whose
// slot t starts a run of equal indices (the slots that receive an update,
// Sec. 4.3), stably sorted by their slot-t index. Every update of view t goes
// to C[c_t], so a view is reduced by segments like a CSR row, without
// scattered atomics.
#include "common.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

namespace systec {
namespace {

constexpr int kChunkTiles = 96;  // panel tiles per workgroup work item

int grid_for(int64_t n, int block) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 8192)));
}

// entry -> row by binary search over rowptr
__global__ void entry_rows_kernel(int n, int nnz, const int32_t* __restrict__ rowptr,
                                  int32_t* __restrict__ rows) {
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    int lo = 0, hi = n;  // rowptr[lo] <= e < rowptr[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (rowptr[mid] <= e) lo = mid;
      else hi = mid;
    }
    rows[e] = lo;
  }
}

// ---- vertex relabeling by degree ----
// deg[v]: stored entries in row v plus off-diagonal stored entries in column
// v (the vertex's degree in the symmetric matrix).
// The stored entries of row v, then (col_degree_kernel) one more for each
// off-diagonal entry in column v: the rows are sorted, so counting them by
// atomics would put a whole wave on one address.
__global__ void row_degree_kernel(int n, const int32_t* __restrict__ rowptr,
                                  int32_t* __restrict__ deg) {
  const int stride = gridDim.x * blockDim.x;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    deg[v] = rowptr[v + 1] - rowptr[v];
}

__global__ void col_degree_kernel(int nnz, const int32_t* __restrict__ rows,
                                  const int32_t* __restrict__ col, int32_t* __restrict__ deg) {
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride)
    if (col[e] != rows[e]) atomicAdd(deg + col[e], 1);
}

// Largest degree (one atomic per workgroup) and the sort keys: descending
// degree, ties in vertex order (the radix sort is stable).
__global__ void degree_keys_kernel(int n, const int32_t* __restrict__ deg,
                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                   int* __restrict__ max_deg) {
  __shared__ int s_max;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  int m = 0;
  const int stride = gridDim.x * blockDim.x;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int d = deg[v];
    m = max(m, d);
    keys[v] = 0xffffffffu - static_cast<uint32_t>(d);
    ids[v] = static_cast<uint32_t>(v);
  }
  atomicMax(&s_max, m);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(max_deg, s_max);
}

// inv[perm[i]] = i
__global__ void invert_perm_kernel(int n, const uint32_t* __restrict__ perm,
                                   int32_t* __restrict__ inv) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    inv[perm[i]] = i;
}

// The stored entry (r, c), r <= c, in the new labels: (min, max) of
// (inv[r], inv[c]), so it stays in the upper triangle.
__global__ void relabel_entries_kernel(int nnz, const int32_t* __restrict__ inv,
                                       int32_t* __restrict__ rows, const int32_t* __restrict__ col,
                                       int32_t* __restrict__ col_out) {
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int a = inv[rows[e]], b = inv[col[e]];
    rows[e] = min(a, b);
    col_out[e] = max(a, b);
  }
}

// sort key of a stored entry: (panel, column, row within panel)
__global__ void panel_keys_kernel(int nnz, int hbits, const int32_t* __restrict__ rows,
                                  const int32_t* __restrict__ col,
                                  unsigned long long* __restrict__ keys,
                                  uint32_t* __restrict__ ids) {
  const int stride = gridDim.x * blockDim.x;
  const unsigned long long hmask = (1ull << hbits) - 1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const unsigned long long r = static_cast<uint32_t>(rows[e]);
    const unsigned long long c = static_cast<uint32_t>(col[e]);
    keys[e] = ((r >> hbits) << (31 + hbits)) | (c << hbits) | (r & hmask);
    ids[e] = static_cast<uint32_t>(e);
  }
}

// First sorted key of every panel: entry e starts panels (panel(e-1),
// panel(e)] (empty panels start where the next non-empty one does), and the
// last entry closes the remaining panels with nnz.
__global__ void panel_starts_kernel(int nnz, int hbits, int npanels,
                                    const unsigned long long* __restrict__ keys,
                                    int32_t* __restrict__ start) {
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int pe = static_cast<int>(keys[e] >> (31 + hbits));
    const int pp = e == 0 ? -1 : static_cast<int>(keys[e - 1] >> (31 + hbits));
    for (int p = pp + 1; p <= pe && p < npanels; ++p) start[p] = e;
    if (e == nnz - 1)
      for (int p = pe + 1; p <= npanels; ++p) start[p] = nnz;
  }
}

__global__ void panel_scatter_kernel(int nnz, int hbits, const unsigned long long* __restrict__ keys,
                                     const uint32_t* __restrict__ ids,
                                     const float* __restrict__ val,
                                     const int32_t* __restrict__ start,
                                     const int32_t* __restrict__ pstart,
                                     int32_t* __restrict__ pcol, uint16_t* __restrict__ prow,
                                     float* __restrict__ pval) {
  const int stride = gridDim.x * blockDim.x;
  const unsigned long long hmask = (1ull << hbits) - 1;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nnz; s += stride) {
    const unsigned long long k = keys[s];
    const int p = static_cast<int>(k >> (31 + hbits));
    const int64_t dst = static_cast<int64_t>(pstart[p]) + (s - start[p]);
    pcol[dst] = static_cast<int32_t>((k >> hbits) & 0x7fffffffull);
    prow[dst] = static_cast<uint16_t>(k & hmask);
    pval[dst] = val[ids[s]];
  }
}

// padding of panel p: positions [pstart[p] + count[p], pstart[p+1])
__global__ void panel_pad_kernel(int npanels, int H, const int32_t* __restrict__ counts,
                                 const int32_t* __restrict__ pstart, int32_t* __restrict__ pcol,
                                 uint16_t* __restrict__ prow, float* __restrict__ pval) {
  for (int p = blockIdx.x; p < npanels; p += gridDim.x) {
    const int64_t b = static_cast<int64_t>(pstart[p]) + counts[p];
    const int64_t e = pstart[p + 1];
    // value 0 at row 0 of the panel and the panel's last column, so the
    // entries stay sorted by column (a zero contribution to both sides)
    for (int64_t q = b + threadIdx.x; q < e; q += blockDim.x) {
      pcol[q] = pcol[b - 1];
      prow[q] = 0;
      pval[q] = 0.0f;
    }
  }
}

// The packed index stream of the panel SSYMV (see Tensor::ppack): one thread
// per entry; a step's columns are sorted, so its first is its base and its
// last sets its span.
__global__ void panel_pack_kernel(int64_t padded, int hbits, const int32_t* __restrict__ pcol,
                                  const uint16_t* __restrict__ prow, uint32_t* __restrict__ ppack,
                                  int32_t* __restrict__ pbase) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < padded;
       e += stride) {
    const int64_t s0 = e / kWave * kWave;
    const int32_t base = pcol[s0];
    const bool wide = static_cast<uint32_t>(pcol[s0 + kWave - 1] - base) >> (32 - hbits) != 0;
    ppack[e] = wide ? 0u : (static_cast<uint32_t>(pcol[e] - base) << hbits) | prow[e];
    if (e == s0) pbase[e / kWave] = wide ? static_cast<int32_t>(static_cast<uint32_t>(base) | 0x80000000u) : base;
  }
}

__global__ void iota_kernel(int64_t n, uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<uint32_t>(i);
}

// ---- column segments of the panel SSYMV ----
// flag[e] = 1 where a segment starts: at a tile's first entry or where the
// column changes.
__global__ void seg_flag_kernel(int64_t ppos, const int32_t* __restrict__ pcol,
                                uint32_t* __restrict__ flag) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < ppos;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    flag[e] = (e % kPanelTile == 0 || pcol[e] != pcol[e - 1]) ? 1u : 0u;
}

// Segment s's column and each tile's first segment; counts segments per
// column.
__global__ void seg_fill_kernel(int64_t ppos, const int32_t* __restrict__ pcol,
                                const uint32_t* __restrict__ flag,
                                const uint32_t* __restrict__ first, uint32_t* __restrict__ seg_col,
                                int32_t* __restrict__ tile0, uint32_t* __restrict__ col_count) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < ppos;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (flag[e]) {
      seg_col[first[e]] = static_cast<uint32_t>(pcol[e]);
      atomicAdd(col_count + pcol[e], 1u);
    }
    if (e % kPanelTile == 0) tile0[e / kPanelTile] = static_cast<int32_t>(first[e]);
  }
}

// ---- slot views ----
__global__ void view_keys_kernel(int order, int t, int nnz, const int32_t* i0, const int32_t* i1,
                                 const int32_t* i2, const int32_t* i3, const int32_t* i4,
                                 uint32_t* __restrict__ keys, uint32_t* __restrict__ ids,
                                 int* __restrict__ count) {
  const int32_t* ip[5] = {i0, i1, i2, i3, i4};
  const int stride = gridDim.x * blockDim.x;
  int c = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int v = ip[t][e];
    const bool starts = (t == 0) || (ip[t - 1][e] != v);
    keys[e] = starts ? static_cast<uint32_t>(v) : 0xffffffffu;  // non-starts sort last
    ids[e] = static_cast<uint32_t>(e);
    c += starts;
  }
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void view_gather_kernel(int order, int m, const uint32_t* __restrict__ ids,
                                   const int32_t* i0, const int32_t* i1, const int32_t* i2,
                                   const int32_t* i3, const int32_t* i4,
                                   const float* __restrict__ val, int32_t* o0, int32_t* o1,
                                   int32_t* o2, int32_t* o3, int32_t* o4,
                                   float* __restrict__ oval) {
  const int32_t* ip[5] = {i0, i1, i2, i3, i4};
  int32_t* op[5] = {o0, o1, o2, o3, o4};
  const int stride = gridDim.x * blockDim.x;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < m; s += stride) {
    const uint32_t e = ids[s];
    for (int t = 0; t < order; ++t) op[t][s] = ip[t][e];
    oval[s] = val[e];
  }
}

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int alloc(T** p, size_t count) {
    void* q = nullptr;
    int rc = check_hip(hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T)), "hipMalloc");
    if (rc) return rc;
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return SYSTEC_OK;
  }
};

template <typename K>
int radix_sort_pairs(const K* kin, K* kout, const uint32_t* vin, uint32_t* vout, int n,
                     int end_bit, hipStream_t s) {
  size_t tmp_bytes = 0;
  int rc = check_hip(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, kin, kout, vin, vout,
                                                        n, 0, end_bit, s),
                     "radix sort (size)");
  if (rc) return rc;
  Scratch sc;
  unsigned char* tmp = nullptr;
  if ((rc = sc.alloc(&tmp, tmp_bytes))) return rc;
  rc = check_hip(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0,
                                                    end_bit, s),
                 "radix sort");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  return rc;
}

int exclusive_sum(const uint32_t* in, uint32_t* out, int n, hipStream_t s) {
  size_t tmp_bytes = 0;
  int rc = check_hip(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, in, out, n, s),
                     "exclusive scan (size)");
  if (rc) return rc;
  Scratch sc;
  unsigned char* tmp = nullptr;
  if ((rc = sc.alloc(&tmp, tmp_bytes))) return rc;
  rc = check_hip(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, n, s), "exclusive scan");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  return rc;
}

int bits_for(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return std::max(b, 1);
}

}  // namespace

void tensor_free(Tensor* t) {
  if (!t) return;
  if (t->work_done) (void)hipEventDestroy(t->work_done);
  for (void* p : t->allocations) (void)hipFree(p);
  delete t;
}

// Relabels the vertices by descending degree (relabel > 0 always, < 0 when
// the largest degree exceeds kRelabelSkew times the mean): a symmetric
// permutation P A P^T that puts the high-degree vertices together, so that
// a panel's entries share columns and the column-side updates of the SSYMV
// merge into fewer cache lines (at R-MAT scale 22, 2.4 M instead of 5.3 M
// 64-byte lines). rows is rewritten in place; *keycol points to the
// relabeled columns (scratch owned by sc). Stores perm (new -> old) and inv
// (old -> new) on the tensor.
constexpr int kRelabelSkew = 8;

static int relabel_by_degree(Tensor* t, int n, int nnz, const int32_t* rowptr, int32_t* rows,
                             const int32_t* col, int relabel, Scratch& sc, hipStream_t s,
                             const int32_t** keycol) {
  int32_t *deg = nullptr, *col2 = nullptr;
  uint32_t *kin = nullptr, *kout = nullptr, *vin = nullptr;
  int* d_max = nullptr;
  int rc = sc.alloc(&deg, n);
  if (!rc) rc = sc.alloc(&kin, n);
  if (!rc) rc = sc.alloc(&kout, n);
  if (!rc) rc = sc.alloc(&vin, n);
  if (!rc) rc = sc.alloc(&d_max, 1);
  if (!rc) rc = check_hip(hipMemsetAsync(d_max, 0, sizeof(int), s), "hipMemsetAsync");
  if (rc) return rc;
  row_degree_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rowptr, deg);
  col_degree_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, rows, col, deg);
  degree_keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, deg, kin, vin, d_max);
  if ((rc = check_launch("degree kernels"))) return rc;
  if (relabel < 0) {
    int h_max = 0;
    rc = check_hip(hipMemcpyAsync(&h_max, d_max, sizeof(int), hipMemcpyDeviceToHost, s),
                   "hipMemcpyAsync");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (rc) return rc;
    // the mean degree is at most 2 nnz / n
    if (static_cast<int64_t>(h_max) * n <= static_cast<int64_t>(kRelabelSkew) * 2 * nnz)
      return SYSTEC_OK;
  }
  if ((rc = tensor_alloc(t, &t->perm, n))) return rc;
  if ((rc = tensor_alloc(t, &t->inv, n))) return rc;
  if ((rc = sc.alloc(&col2, nnz))) return rc;
  if ((rc = radix_sort_pairs(kin, kout, vin, reinterpret_cast<uint32_t*>(t->perm), n, 32, s)))
    return rc;
  invert_perm_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, reinterpret_cast<const uint32_t*>(t->perm),
                                                     t->inv);
  relabel_entries_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, t->inv, rows, col, col2);
  if ((rc = check_launch("relabel kernels"))) return rc;
  t->relabeled = true;
  *keycol = col2;
  return SYSTEC_OK;
}

namespace {

// The column segments (Tensor::nsegs and the seg_* arrays) of a matrix whose
// panels are built, and the per-call buffer of their sums.
int build_column_segments(Tensor* t, hipStream_t s) {
  const int64_t ppos = t->padded;
  const int n = static_cast<int>(t->dim);
  const int64_t ntiles = ppos / kPanelTile;
  Scratch sc;
  uint32_t *flag = nullptr, *first = nullptr, *count = nullptr, *ptr = nullptr;
  int rc = sc.alloc(&flag, ppos);
  if (!rc) rc = sc.alloc(&first, ppos);
  if (!rc) rc = sc.alloc(&count, n + 1);
  if (!rc) rc = sc.alloc(&ptr, n + 1);
  if (rc) return rc;
  const int grid = static_cast<int>(std::min<int64_t>((ppos + 255) / 256, 65536));
  seg_flag_kernel<<<grid, 256, 0, s>>>(ppos, t->pcol, flag);
  if ((rc = check_launch("segment flag kernel"))) return rc;
  if ((rc = exclusive_sum(flag, first, static_cast<int>(ppos), s))) return rc;
  uint32_t last_first = 0, last_flag = 0;
  rc = check_hip(hipMemcpyAsync(&last_first, first + ppos - 1, 4, hipMemcpyDeviceToHost, s), "memcpy");
  if (!rc)
    rc = check_hip(hipMemcpyAsync(&last_flag, flag + ppos - 1, 4, hipMemcpyDeviceToHost, s), "memcpy");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) return rc;
  const int64_t S = static_cast<int64_t>(last_first) + last_flag;
  t->nsegs = S;
  uint32_t *seg_col = nullptr, *seg_col_sorted = nullptr, *ids_in = nullptr;
  if ((rc = sc.alloc(&seg_col, S)) || (rc = sc.alloc(&seg_col_sorted, S)) ||
      (rc = sc.alloc(&ids_in, S)))
    return rc;
  if ((rc = tensor_alloc(t, &t->seg_tile0, ntiles + 1))) return rc;
  if ((rc = tensor_alloc(t, &t->seg_colptr, n + 1))) return rc;
  if ((rc = tensor_alloc(t, &t->seg_ids, S))) return rc;
  if ((rc = tensor_alloc(t, &t->work_seg, S))) return rc;
  rc = check_hip(hipMemsetAsync(count, 0, (n + 1) * sizeof(uint32_t), s), "hipMemsetAsync");
  if (rc) return rc;
  seg_fill_kernel<<<grid, 256, 0, s>>>(ppos, t->pcol, flag, first, seg_col, t->seg_tile0, count);
  if ((rc = check_launch("segment fill kernel"))) return rc;
  const int32_t s32 = static_cast<int32_t>(S);
  rc = check_hip(hipMemcpyAsync(t->seg_tile0 + ntiles, &s32, 4, hipMemcpyHostToDevice, s), "memcpy");
  // column pointer: exclusive sum of the counts (n + 1 of them, the last 0)
  if (!rc) rc = exclusive_sum(count, ptr, n + 1, s);
  if (!rc)
    rc = check_hip(hipMemcpyAsync(t->seg_colptr, ptr, (n + 1) * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s), "memcpy");
  // segment ids grouped by column, in segment order within a column (the
  // sort is stable)
  if (!rc) {
    iota_kernel<<<static_cast<int>(std::min<int64_t>((S + 255) / 256, 65536)), 256, 0, s>>>(
        S, ids_in);
    rc = check_launch("iota kernel");
  }
  if (!rc)
    rc = radix_sort_pairs(seg_col, seg_col_sorted, ids_in,
                          reinterpret_cast<uint32_t*>(t->seg_ids), static_cast<int>(S),
                          bits_for(n + 1), s);
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  return rc;
}

}  // namespace

int tensor_create_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                      const float* val, int panel_rows, int relabel, hipStream_t s,
                      Tensor** out) {
  const int hbits = bits_for(panel_rows);
  const int H = 1 << hbits;
  auto* t = new Tensor();
  t->kind = 0;
  t->order = 2;
  t->dim = n;
  t->nnz = nnz;
  t->panel_rows = H;
  t->npanels = static_cast<int>((n + H - 1) / H);
  const int P = t->npanels;
  const int nz = static_cast<int>(nnz), ni = static_cast<int>(n);
  Scratch sc;
  int32_t* rows = nullptr;
  unsigned long long *kin = nullptr, *kout = nullptr;
  uint32_t *vin = nullptr, *vout = nullptr;
  int32_t *counts = nullptr, *d_start = nullptr, *d_pstart = nullptr;
  int rc = sc.alloc(&rows, nnz);
  if (!rc) rc = sc.alloc(&kin, nnz);
  if (!rc) rc = sc.alloc(&kout, nnz);
  if (!rc) rc = sc.alloc(&vin, nnz);
  if (!rc) rc = sc.alloc(&vout, nnz);
  if (!rc) rc = sc.alloc(&counts, P);
  if (!rc) rc = sc.alloc(&d_start, P + 1);
  if (!rc) rc = sc.alloc(&d_pstart, P + 1);
  if (rc) {
    tensor_free(t);
    return rc;
  }
  std::vector<int32_t> h_counts(P, 0);
  // counts must be zero even without entries: the padding kernel reads them
  rc = check_hip(hipMemsetAsync(counts, 0, P * sizeof(int32_t), s), "hipMemsetAsync");
  if (rc) {
    tensor_free(t);
    return rc;
  }
  if (nnz > 0) {
    entry_rows_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(ni, nz, rowptr, rows);
    rc = check_launch("entry row kernel");
    const int32_t* keycol = col;
    if (!rc && relabel != 0)
      rc = relabel_by_degree(t, ni, nz, rowptr, rows, col, relabel, sc, s, &keycol);
    if (!rc) {
      panel_keys_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(nz, hbits, rows, keycol, kin, vin);
      rc = check_launch("panel key kernels");
    }
    if (!rc) rc = radix_sort_pairs(kin, kout, vin, vout, nz, 31 + hbits + bits_for(P + 1), s);
    if (!rc) {
      panel_starts_kernel<<<grid_for(nz, 256), 256, 0, s>>>(nz, hbits, P, kout, d_start);
      rc = check_launch("panel start kernel");
    }
    std::vector<int32_t> h_first(P + 1, 0);
    if (!rc)
      rc = check_hip(hipMemcpyAsync(h_first.data(), d_start, (P + 1) * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int p = 0; p < P && !rc; ++p) h_counts[p] = h_first[p + 1] - h_first[p];
    if (!rc)
      rc = check_hip(hipMemcpyAsync(counts, h_counts.data(), P * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (rc) {
      tensor_free(t);
      return rc;
    }
  }
  // padded panel offsets and the chunk table (host, P is small)
  std::vector<int32_t> h_start(P + 1, 0), h_pstart(P + 1, 0);
  std::vector<int32_t> ch_panel, ch_begin, ch_end, ch_valid;
  int64_t pos = 0, ppos = 0;
  for (int p = 0; p < P; ++p) {
    h_start[p] = static_cast<int32_t>(pos);
    h_pstart[p] = static_cast<int32_t>(ppos);
    const int64_t tiles = (h_counts[p] + kPanelTile - 1) / kPanelTile;
    const int64_t tile0 = ppos / kPanelTile;
    for (int64_t c = 0; c < tiles; c += kChunkTiles) {
      ch_panel.push_back(p);
      ch_begin.push_back(static_cast<int32_t>(tile0 + c));
      ch_end.push_back(static_cast<int32_t>(tile0 + std::min<int64_t>(tiles, c + kChunkTiles)));
      ch_valid.push_back(static_cast<int32_t>(
          std::min<int64_t>((tile0 + std::min<int64_t>(tiles, c + kChunkTiles)) * kPanelTile,
                            ppos + h_counts[p])));
    }
    pos += h_counts[p];
    ppos += tiles * kPanelTile;
  }
  h_start[P] = static_cast<int32_t>(pos);
  h_pstart[P] = static_cast<int32_t>(ppos);
  if (ppos > (int64_t(1) << 31) - 1) {
    tensor_free(t);
    return fail(SYSTEC_EINVAL, "prepared matrix too large for int32 offsets");
  }
  t->padded = ppos;
  t->nchunks = static_cast<int>(ch_panel.size());
  t->h_chunk_panel = ch_panel;
  t->h_chunk_tile_begin = ch_begin;
  t->h_chunk_tile_end = ch_end;
  rc = tensor_alloc(t, &t->pcol, ppos);
  if (!rc) rc = tensor_alloc(t, &t->prow, ppos);
  if (!rc) rc = tensor_alloc(t, &t->pval, ppos);
  if (!rc) rc = tensor_alloc(t, &t->chunk_panel, t->nchunks);
  if (!rc) rc = tensor_alloc(t, &t->chunk_tile_begin, t->nchunks);
  if (!rc) rc = tensor_alloc(t, &t->chunk_tile_end, t->nchunks);
  if (!rc) rc = tensor_alloc(t, &t->chunk_valid_end, t->nchunks);
  const size_t pb = (P + 1) * sizeof(int32_t);
  if (!rc) rc = check_hip(hipMemcpyAsync(d_start, h_start.data(), pb, hipMemcpyHostToDevice, s), "memcpy");
  if (!rc) rc = check_hip(hipMemcpyAsync(d_pstart, h_pstart.data(), pb, hipMemcpyHostToDevice, s), "memcpy");
  const size_t cb = t->nchunks * sizeof(int32_t);
  if (!rc && t->nchunks) {
    rc = check_hip(hipMemcpyAsync(t->chunk_panel, ch_panel.data(), cb, hipMemcpyHostToDevice, s), "memcpy");
    if (!rc) rc = check_hip(hipMemcpyAsync(t->chunk_tile_begin, ch_begin.data(), cb, hipMemcpyHostToDevice, s), "memcpy");
    if (!rc) rc = check_hip(hipMemcpyAsync(t->chunk_tile_end, ch_end.data(), cb, hipMemcpyHostToDevice, s), "memcpy");
    if (!rc) rc = check_hip(hipMemcpyAsync(t->chunk_valid_end, ch_valid.data(), cb, hipMemcpyHostToDevice, s), "memcpy");
  }
  if (!rc && nnz > 0) {
    panel_scatter_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(nz, hbits, kout, vout, val, d_start,
                                                            d_pstart, t->pcol, t->prow, t->pval);
    rc = check_launch("panel scatter kernel");
  }
  if (!rc && P > 0) {
    panel_pad_kernel<<<std::min(P, 4096), 256, 0, s>>>(P, H, counts, d_pstart, t->pcol, t->prow,
                                                      t->pval);
    rc = check_launch("panel pad kernel");
  }
  if (!rc) rc = tensor_alloc(t, &t->ppack, ppos);
  if (!rc) rc = tensor_alloc(t, &t->pbase, ppos / kWave);
  if (!rc && ppos > 0) {
    panel_pack_kernel<<<grid_for(ppos, 256), 256, 0, s>>>(ppos, hbits, t->pcol, t->prow, t->ppack,
                                                          t->pbase);
    rc = check_launch("panel pack kernel");
  }
  if (!rc && ppos > 0) rc = build_column_segments(t, s);
  // the calls' work buffers (see Tensor)
  if (!rc) rc = tensor_alloc(t, &t->work_partial, std::max(1, t->nchunks));
  if (!rc && t->relabeled) {
    float* wx = nullptr;
    rc = tensor_alloc(t, &wx, n);  // x in the stored order, FP32 or BF16
    t->work_x = wx;
    if (!rc) rc = tensor_alloc(t, &t->work_y, n);
  }
  if (!rc)
    rc = check_hip(hipEventCreateWithFlags(&t->work_done, hipEventDisableTiming), "hipEventCreate");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) {
    tensor_free(t);
    return rc;
  }
  *out = t;
  return SYSTEC_OK;
}

int tensor_create_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                      const float* val, hipStream_t s, Tensor** out) {
  auto* t = new Tensor();
  t->kind = 1;
  t->order = order;
  t->dim = I;
  t->nnz = nnz;
  t->short_runs = nnz < kShortRun * I;
  const int nz = static_cast<int>(nnz);
  const int32_t* ip[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int q = 0; q < order; ++q) ip[q] = idx[q];
  Scratch sc;
  uint32_t *kin = nullptr, *kout = nullptr, *vin = nullptr, *vout = nullptr;
  int* d_count = nullptr;
  int rc = sc.alloc(&kin, nnz);
  if (!rc) rc = sc.alloc(&kout, nnz);
  if (!rc) rc = sc.alloc(&vin, nnz);
  if (!rc) rc = sc.alloc(&vout, nnz);
  if (!rc) rc = sc.alloc(&d_count, 1);
  for (int v = 0; v < order && !rc; ++v) {
    int m = 0;
    if (nnz > 0) {
      rc = check_hip(hipMemsetAsync(d_count, 0, sizeof(int), s), "hipMemsetAsync");
      if (rc) break;
      view_keys_kernel<<<grid_for(nnz, 256), 256, 0, s>>>(order, v, nz, ip[0], ip[1], ip[2],
                                                          ip[3], ip[4], kin, vin, d_count);
      if ((rc = check_launch("view key kernel"))) break;
      if ((rc = radix_sort_pairs(kin, kout, vin, vout, nz, 32, s))) break;
      if ((rc = check_hip(hipMemcpyAsync(&m, d_count, sizeof(int), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync")))
        break;
      if ((rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
    }
    t->vnnz[v] = m;
    for (int q = 0; q < order && !rc; ++q) rc = tensor_alloc(t, &t->vidx[v][q], m);
    if (!rc) rc = tensor_alloc(t, &t->vval[v], m);
    if (rc) break;
    if (m > 0) {
      int32_t* op[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
      for (int q = 0; q < order; ++q) op[q] = t->vidx[v][q];
      view_gather_kernel<<<grid_for(m, 256), 256, 0, s>>>(order, m, vout, ip[0], ip[1], ip[2],
                                                          ip[3], ip[4], val, op[0], op[1], op[2],
                                                          op[3], op[4], t->vval[v]);
      if ((rc = check_launch("view gather kernel"))) break;
      if ((rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"))) break;
    }
  }
  if (!rc) rc = build_lane_views(t, s);
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) {
    tensor_free(t);
    return rc;
  }
  *out = t;
  return SYSTEC_OK;
}

}  // namespace systec
