// Support kernels: BF16 quantization, expansion statistics, canonical-form
// validation, and the expansion of a symmetric operand into its full
// (non-symmetric) form for the comparison kernels.
#include "common.h"

#include <vector>

namespace systec {

namespace {

// ---- BF16 quantization (round to nearest, ties to even) --------------------
__global__ void quantize_bf16_kernel(const float* __restrict__ in, uint16_t* __restrict__ out,
                                     int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const uint32_t u = __float_as_uint(in[i]);
    uint16_t r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
      r = static_cast<uint16_t>((u >> 16) | 0x0040u);  // quiet NaN
    } else {
      // add half an ulp of the 16-bit result, plus one if the kept part is
      // odd (ties go to the even neighbour), then truncate
      const uint32_t lsb = (u >> 16) & 1u;
      r = static_cast<uint16_t>((u + 0x7fffu + lsb) >> 16);
    }
    out[i] = r;
  }
}

// ---- expansion statistics ---------------------------------------------------
template <int N>
struct MultTable {
  int32_t mult[16];
};

__device__ __forceinline__ int64_t dev_fact(int n) {
  int64_t f = 1;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

// counts[0..15]: entries per equality pattern; counts[16]: sum of distinct
// permutation counts.
__global__ void expansion_stats_kernel(int order, int nnz, const int32_t* i0, const int32_t* i1,
                                       const int32_t* i2, const int32_t* i3, const int32_t* i4,
                                       unsigned long long* __restrict__ counts) {
  __shared__ unsigned long long s[17];
  if (threadIdx.x < 17) s[threadIdx.x] = 0;
  __syncthreads();
  const int32_t* ip[5] = {i0, i1, i2, i3, i4};
  const int stride = gridDim.x * blockDim.x;
  unsigned long long eff = 0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    int c[5];
    for (int t = 0; t < order; ++t) c[t] = ip[t][e];
    int mask = 0;
    int64_t denom = 1;
    int run = 1;
    for (int t = 1; t <= order; ++t) {
      if (t < order && c[t] == c[t - 1]) {
        mask |= 1 << (t - 1);
        ++run;
      } else {
        denom *= dev_fact(run);
        run = 1;
      }
    }
    eff += static_cast<unsigned long long>(dev_fact(order) / denom);
    atomicAdd(&s[mask], 1ull);
  }
  atomicAdd(&s[16], eff);
  __syncthreads();
  if (threadIdx.x < 17 && s[threadIdx.x]) atomicAdd(&counts[threadIdx.x], s[threadIdx.x]);
}

// ---- validation -------------------------------------------------------------
enum : unsigned int {
  kBadRowptr = 1u,
  kColRange = 2u,
  kBelowDiag = 4u,
  kRowOrder = 8u,
  kIdxRange = 16u,
  kTupleOrder = 32u,
  kListOrder = 64u,
};

// Row of entry q: the last r in [0, n) with rowptr[r] <= q. Reads rowptr
// only within [0, n], so it stays in bounds whatever rowptr holds.
__device__ __forceinline__ int row_of(const int32_t* __restrict__ rowptr, int n, int q) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rowptr[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Moves r forward to the row of entry q (a few steps, else a search).
__device__ __forceinline__ int advance_row(const int32_t* __restrict__ rowptr, int n, int r, int q) {
  for (int k = 0; k < 4; ++k) {
    if (r + 1 >= n || rowptr[r + 1] > q) return r;
    ++r;
  }
  return (r + 1 >= n || rowptr[r + 1] > q) ? r : row_of(rowptr, n, q);
}

// Entries are checked in chunks of kChunk consecutive entries per thread, so
// a long row is spread over many threads (rows of 10^5 entries occur in
// graph matrices).
constexpr int kChunk = 16;

__global__ void validate_rowptr_kernel(int n, int nnz, const int32_t* __restrict__ rowptr,
                                       unsigned int* flags) {
  const int stride = gridDim.x * blockDim.x;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int a = rowptr[r], b = rowptr[r + 1];
    if ((r == 0 && a != 0) || (r == n - 1 && b != nnz) || a > b || a < 0 || b > nnz)
      atomicOr(flags, kBadRowptr);
  }
}

__global__ void validate_csr_entries_kernel(int n, int nnz, const int32_t* __restrict__ rowptr,
                                            const int32_t* __restrict__ col, unsigned int* flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t chunks = (static_cast<int64_t>(nnz) + kChunk - 1) / kChunk;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < chunks;
       k += stride) {
    const int q0 = static_cast<int>(k * kChunk);
    const int q1 = min(nnz, q0 + kChunk);
    int r = row_of(rowptr, n, q0);
    unsigned int f = 0;
    for (int q = q0; q < q1; ++q) {
      r = advance_row(rowptr, n, r, q);
      const int c = col[q];
      if (c < 0 || c >= n) f |= kColRange;
      if (c < r) f |= kBelowDiag;
      if (q > 0 && q > rowptr[r] && col[q - 1] >= c) f |= kRowOrder;
    }
    if (f) atomicOr(flags, f);
  }
}

__global__ void validate_coo_kernel(int order, int dim, int nnz, const int32_t* i0,
                                    const int32_t* i1, const int32_t* i2, const int32_t* i3,
                                    const int32_t* i4, unsigned int* flags) {
  const int32_t* ip[5] = {i0, i1, i2, i3, i4};
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    unsigned int f = 0;
    int c[5], p[5];
    for (int t = 0; t < order; ++t) {
      c[t] = ip[t][e];
      if (c[t] < 0 || c[t] >= dim) f |= kIdxRange;
      if (t > 0 && c[t - 1] > c[t]) f |= kTupleOrder;
    }
    if (e > 0) {
      int cmp = 0;  // previous tuple vs this one, lexicographically
      for (int t = 0; t < order; ++t) {
        p[t] = ip[t][e - 1];
        if (cmp == 0 && p[t] != c[t]) cmp = p[t] < c[t] ? -1 : 1;
      }
      if (cmp >= 0) f |= kListOrder;
    }
    if (f) atomicOr(flags, f);
  }
}

std::string describe_flags(unsigned int f) {
  std::string m;
  if (f & kBadRowptr) m += "rowptr not a valid row pointer; ";
  if (f & kColRange) m += "column index out of range; ";
  if (f & kBelowDiag) m += "entry below the diagonal (col < row); ";
  if (f & kRowOrder) m += "columns not strictly ascending within a row; ";
  if (f & kIdxRange) m += "index out of range; ";
  if (f & kTupleOrder) m += "tuple not ascending; ";
  if (f & kListOrder) m += "list not strictly increasing (unsorted or duplicate tuple); ";
  return m;
}

// ---- expansion to the full operand ------------------------------------------
__global__ void csr_count_diag_kernel(int n, int nnz, const int32_t* __restrict__ rowptr,
                                      const int32_t* __restrict__ col,
                                      unsigned long long* __restrict__ diag) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t chunks = (static_cast<int64_t>(nnz) + kChunk - 1) / kChunk;
  unsigned long long d = 0;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < chunks;
       k += stride) {
    const int q0 = static_cast<int>(k * kChunk);
    const int q1 = min(nnz, q0 + kChunk);
    int r = row_of(rowptr, n, q0);
    for (int q = q0; q < q1; ++q) {
      r = advance_row(rowptr, n, r, q);
      d += (col[q] == r);
    }
  }
  if (d) atomicAdd(diag, d);
}

// full row lengths: stored row length plus the transposed off-diagonal entries
__global__ void csr_full_counts_kernel(int n, const int32_t* __restrict__ rowptr,
                                       const int32_t* __restrict__ col,
                                       int32_t* __restrict__ cnt) {
  const int stride = gridDim.x * blockDim.x;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    atomicAdd(&cnt[r], rowptr[r + 1] - rowptr[r]);
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q)
      if (col[q] != r) atomicAdd(&cnt[col[q]], 1);
  }
}

__global__ void csr_full_fill_kernel(int n, const int32_t* __restrict__ rowptr,
                                     const int32_t* __restrict__ col,
                                     const float* __restrict__ val, int32_t* __restrict__ cursor,
                                     int32_t* __restrict__ fcol, float* __restrict__ fval) {
  const int stride = gridDim.x * blockDim.x;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) {
      const int c = col[q];
      const float a = val[q];
      int pos = atomicAdd(&cursor[r], 1);
      fcol[pos] = c;
      fval[pos] = a;
      if (c != r) {
        pos = atomicAdd(&cursor[c], 1);
        fcol[pos] = r;
        fval[pos] = a;
      }
    }
  }
}

// Exclusive scan of cnt[0..n) into out[0..n], out[n] = total; one workgroup.
__global__ __launch_bounds__(1024) void scan_single_block_kernel(const int32_t* __restrict__ cnt,
                                                                 int n,
                                                                 int32_t* __restrict__ out) {
  __shared__ long long s[1024];
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int lo = min(n, static_cast<int>(threadIdx.x) * per);
  const int hi = min(n, lo + per);
  long long t = 0;
  for (int i = lo; i < hi; ++i) t += cnt[i];
  s[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = 0;
    for (int i = 0; i < static_cast<int>(blockDim.x); ++i) {
      const long long v = s[i];
      s[i] = run;
      run += v;
    }
    out[n] = static_cast<int32_t>(run);
  }
  __syncthreads();
  long long run = s[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    out[i] = static_cast<int32_t>(run);
    run += cnt[i];
  }
}

// Next lexicographic permutation of a small array; false after the last one.
template <int N>
__device__ __forceinline__ bool next_perm(int (&a)[N]) {
  int k = N - 2;
  while (k >= 0 && a[k] >= a[k + 1]) --k;
  if (k < 0) return false;
  int l = N - 1;
  while (a[k] >= a[l]) --l;
  int t = a[k];
  a[k] = a[l];
  a[l] = t;
  for (int i = k + 1, j = N - 1; i < j; ++i, --j) {
    t = a[i];
    a[i] = a[j];
    a[j] = t;
  }
  return true;
}

// kWrite=false: count expanded entries per leading index into cursor;
// kWrite=true: write them at positions taken from cursor.
template <int N, bool kWrite>
__global__ void coo_expand_kernel(int nnz, const int32_t* i0, const int32_t* i1,
                                  const int32_t* i2, const int32_t* i3, const int32_t* i4,
                                  const float* __restrict__ val, int32_t* __restrict__ cursor,
                                  int32_t* o0, int32_t* o1, int32_t* o2, int32_t* o3,
                                  int32_t* o4, float* __restrict__ oval) {
  const int32_t* ip[5] = {i0, i1, i2, i3, i4};
  int32_t* op[5] = {o0, o1, o2, o3, o4};
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    int p[N];
    for (int t = 0; t < N; ++t) p[t] = ip[t][e];
    const float v = kWrite ? val[e] : 0.0f;
    do {
      const int pos = atomicAdd(&cursor[p[0]], 1);
      if (kWrite) {
        for (int t = 0; t < N; ++t) op[t][pos] = p[t];
        oval[pos] = v;
      }
    } while (next_perm<N>(p));
  }
}

int grid_for(int64_t n, int block) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 4096)));
}

template <bool kWrite>
void launch_coo_expand(int order, int nnz, const int32_t* const* idx, const float* val,
                       int32_t* cursor, int32_t* const* out, float* oval, hipStream_t s) {
  const int32_t* ip[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t* op[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int t = 0; t < order; ++t) {
    ip[t] = idx[t];
    if (kWrite) op[t] = out[t];
  }
  const int g = grid_for(nnz, 256);
#define SYSTEC_EXPAND(N)                                                                    \
  coo_expand_kernel<N, kWrite><<<dim3(g), dim3(256), 0, s>>>(nnz, ip[0], ip[1], ip[2], ip[3], \
                                                             ip[4], val, cursor, op[0], op[1], \
                                                             op[2], op[3], op[4], oval)
  switch (order) {
    case 2: SYSTEC_EXPAND(2); break;
    case 3: SYSTEC_EXPAND(3); break;
    case 4: SYSTEC_EXPAND(4); break;
    default: SYSTEC_EXPAND(5); break;
  }
#undef SYSTEC_EXPAND
}

// RAII device buffer for setup work.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int launch_quantize_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return SYSTEC_OK;
  quantize_bf16_kernel<<<dim3(grid_for(n, 256)), dim3(256), 0, s>>>(in, out, n);
  return check_launch("quantize kernel");
}

int launch_expansion_stats(int order, int64_t nnz, const int32_t* const* idx,
                           unsigned long long* d_counts, hipStream_t s) {
  const int32_t* ip[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int t = 0; t < order; ++t) ip[t] = idx[t];
  if (nnz == 0) return SYSTEC_OK;
  expansion_stats_kernel<<<dim3(grid_for(nnz, 256)), dim3(256), 0, s>>>(
      order, static_cast<int>(nnz), ip[0], ip[1], ip[2], ip[3], ip[4], d_counts);
  return check_launch("expansion stats kernel");
}

int launch_validate_csr_upper(int64_t n, int64_t nnz, const int32_t* rowptr,
                              const int32_t* col, unsigned int* d_flags, hipStream_t s) {
  validate_rowptr_kernel<<<dim3(grid_for(n, 256)), dim3(256), 0, s>>>(
      static_cast<int>(n), static_cast<int>(nnz), rowptr, d_flags);
  int rc = check_launch("validate rowptr kernel");
  if (rc || nnz == 0) return rc;
  validate_csr_entries_kernel<<<dim3(grid_for((nnz + kChunk - 1) / kChunk, 256)), dim3(256), 0, s>>>(
      static_cast<int>(n), static_cast<int>(nnz), rowptr, col, d_flags);
  return check_launch("validate csr kernel");
}

int launch_validate_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                        unsigned int* d_flags, hipStream_t s) {
  const int32_t* ip[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int t = 0; t < order; ++t) ip[t] = idx[t];
  if (nnz == 0) return SYSTEC_OK;
  validate_coo_kernel<<<dim3(grid_for(nnz, 256)), dim3(256), 0, s>>>(
      order, static_cast<int>(I), static_cast<int>(nnz), ip[0], ip[1], ip[2], ip[3], ip[4],
      d_flags);
  return check_launch("validate coo kernel");
}

std::string validation_message(unsigned int flags) { return describe_flags(flags); }

int expand_csr_size(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                    int64_t* full_nnz, hipStream_t s) {
  DevBuf d;
  int rc = check_hip(hipMalloc(&d.p, sizeof(unsigned long long)), "hipMalloc");
  if (rc) return rc;
  if ((rc = check_hip(hipMemsetAsync(d.p, 0, sizeof(unsigned long long), s), "hipMemsetAsync")))
    return rc;
  csr_count_diag_kernel<<<dim3(grid_for((nnz + kChunk - 1) / kChunk, 256)), dim3(256), 0, s>>>(
      static_cast<int>(n), static_cast<int>(nnz), rowptr, col,
      static_cast<unsigned long long*>(d.p));
  if ((rc = check_launch("count diagonal kernel"))) return rc;
  unsigned long long diag = 0;
  if ((rc = check_hip(hipMemcpyAsync(&diag, d.p, sizeof(diag), hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync")))
    return rc;
  if ((rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
  *full_nnz = 2 * nnz - static_cast<int64_t>(diag);
  return SYSTEC_OK;
}

int expand_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
               const float* val, int32_t* full_rowptr, int32_t* full_col, float* full_val,
               hipStream_t s) {
  DevBuf cnt, cursor;
  const size_t bytes = static_cast<size_t>(n) * sizeof(int32_t);
  int rc = check_hip(hipMalloc(&cnt.p, bytes), "hipMalloc");
  if (!rc) rc = check_hip(hipMalloc(&cursor.p, bytes + sizeof(int32_t)), "hipMalloc");
  if (!rc) rc = check_hip(hipMemsetAsync(cnt.p, 0, bytes, s), "hipMemsetAsync");
  if (rc) return rc;
  const int ni = static_cast<int>(n);
  auto* c = static_cast<int32_t*>(cnt.p);
  auto* cur = static_cast<int32_t*>(cursor.p);
  csr_full_counts_kernel<<<dim3(grid_for(n, 256)), dim3(256), 0, s>>>(ni, rowptr, col, c);
  if ((rc = check_launch("full counts kernel"))) return rc;
  scan_single_block_kernel<<<dim3(1), dim3(1024), 0, s>>>(c, ni, full_rowptr);
  if ((rc = check_launch("scan kernel"))) return rc;
  if ((rc = check_hip(hipMemcpyAsync(cur, full_rowptr, bytes, hipMemcpyDeviceToDevice, s),
                      "hipMemcpyAsync")))
    return rc;
  csr_full_fill_kernel<<<dim3(grid_for(n, 256)), dim3(256), 0, s>>>(ni, rowptr, col, val, cur,
                                                                    full_col, full_val);
  if ((rc = check_launch("full fill kernel"))) return rc;
  (void)nnz;
  return check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

int expand_coo_size(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                    int64_t* full_nnz, hipStream_t s) {
  DevBuf d;
  int rc = check_hip(hipMalloc(&d.p, 17 * sizeof(unsigned long long)), "hipMalloc");
  if (!rc) rc = check_hip(hipMemsetAsync(d.p, 0, 17 * sizeof(unsigned long long), s), "memset");
  if (!rc) rc = launch_expansion_stats(order, nnz, idx, static_cast<unsigned long long*>(d.p), s);
  unsigned long long h[17] = {0};
  if (!rc)
    rc = check_hip(hipMemcpyAsync(h, d.p, sizeof(h), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) return rc;
  (void)I;
  *full_nnz = static_cast<int64_t>(h[16]);
  return SYSTEC_OK;
}

int expand_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx, const float* val,
               int32_t* const* out_idx, float* out_val, hipStream_t s) {
  DevBuf cnt, cursor;
  const size_t bytes = static_cast<size_t>(I) * sizeof(int32_t);
  int rc = check_hip(hipMalloc(&cnt.p, bytes), "hipMalloc");
  if (!rc) rc = check_hip(hipMalloc(&cursor.p, bytes + sizeof(int32_t)), "hipMalloc");
  if (!rc) rc = check_hip(hipMemsetAsync(cnt.p, 0, bytes, s), "hipMemsetAsync");
  if (rc) return rc;
  auto* c = static_cast<int32_t*>(cnt.p);
  auto* cur = static_cast<int32_t*>(cursor.p);
  const int nz = static_cast<int>(nnz);
  launch_coo_expand<false>(order, nz, idx, val, c, nullptr, nullptr, s);
  if ((rc = check_launch("expand count kernel"))) return rc;
  scan_single_block_kernel<<<dim3(1), dim3(1024), 0, s>>>(c, static_cast<int>(I), cur);
  if ((rc = check_launch("scan kernel"))) return rc;
  launch_coo_expand<true>(order, nz, idx, val, cur, out_idx, out_val, s);
  if ((rc = check_launch("expand write kernel"))) return rc;
  return check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

}  // namespace systec
