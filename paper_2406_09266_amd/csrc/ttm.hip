// TTM with visible output symmetry (Sec. 5.2.5; Sec. 3.2.1): for a fully
// symmetric 3-index tensor T,
//   C[j, l, r] = sum_k T[k, j, l] B[k, r]
// and C is symmetric in (j, l). Only the canonical half of C (j <= l) is
// computed from the canonical entries, then copied to the other half in a
// separate pass (the paper's post-processing loop for visible output
// symmetry).
//
// A stored (a <= b <= c, v) stands for every distinct arrangement (k, j, l)
// of its tuple. Those with j <= l are one per distinct value k of the tuple:
// k takes that value and (j, l) the other two indices in ascending order, so
// C[j, l, :] += v B[k, :] once per distinct value (3, 2, 2 or 1 updates for
// the patterns a<b<c, a=b<c, a<b=c, a=b=c; Sec. 3.1, the TTM listing and
// its output-symmetry rewrite). Every update is a contiguous row of R
// columns, added with FP32 atomics (different entries share output rows).
#include "common.h"

namespace systec {
namespace {

// Zeroes C[j, l, :] for l >= j (the canonical half, one row j per block
// iteration: a contiguous run of (I - j) R floats).
__global__ void ttm_zero_half_kernel(int I, int R, float* __restrict__ C) {
  for (int j = blockIdx.x; j < I; j += gridDim.x) {
    float* row = C + (static_cast<int64_t>(j) * I + j) * R;
    const int64_t len = static_cast<int64_t>(I - j) * R;
    for (int64_t q = threadIdx.x; q < len; q += blockDim.x) row[q] = 0.0f;
  }
}

// Canonical-half updates: thread (e, r) over the entries and the R columns
// (consecutive threads take consecutive columns of one entry, so the factor
// gathers and the output atomics are contiguous rows).
template <typename BT>
__global__ __launch_bounds__(256) void ttm_canonical_kernel(int I, int64_t nnz,
                                                          const int32_t* __restrict__ i0,
                                                          const int32_t* __restrict__ i1,
                                                          const int32_t* __restrict__ i2,
                                                          const float* __restrict__ val,
                                                          const BT* __restrict__ B, int R,
                                                          float* __restrict__ C) {
  const int64_t total = nnz * R;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < total;
       w += stride) {
    const int64_t e = w / R;
    const int r = static_cast<int>(w - e * R);
    const int a = i0[e], b = i1[e], c = i2[e];
    const float v = val[e];
    auto out = [&](int j, int l) -> float* {
      return C + (static_cast<int64_t>(j) * I + l) * R + r;
    };
    // k = a: (j, l) = (b, c)
    atomic_add_noret(out(b, c), v * load_f32(B, static_cast<int64_t>(a) * R + r));
    // k = b, a distinct value (b != a): (j, l) = (a, c)
    if (b != a) atomic_add_noret(out(a, c), v * load_f32(B, static_cast<int64_t>(b) * R + r));
    // k = c, a distinct value (c != b): (j, l) = (a, b)
    if (c != b) atomic_add_noret(out(a, b), v * load_f32(B, static_cast<int64_t>(c) * R + r));
  }
}

// C[j, l, :] = C[l, j, :] for l < j: row j of the lower half is written
// contiguously, each source is a contiguous run of R floats.
__global__ void ttm_mirror_kernel(int I, int R, float* __restrict__ C) {
  for (int j = blockIdx.x; j < I; j += gridDim.x) {
    float* dst = C + static_cast<int64_t>(j) * I * R;
    const int64_t len = static_cast<int64_t>(j) * R;  // l < j
    for (int64_t q = threadIdx.x; q < len; q += blockDim.x) {
      const int64_t l = q / R;
      const int r = static_cast<int>(q - l * R);
      dst[q] = C[(l * I + j) * R + r];
    }
  }
}

}  // namespace

int launch_ttm(int64_t I, int64_t nnz, const int32_t* const* idx, const float* val,
               const void* B, systec_dtype bdt, int64_t R, float* C, bool mirror,
               hipStream_t s) {
  const int Ii = static_cast<int>(I), Ri = static_cast<int>(R);
  const int rows_grid = static_cast<int>(std::min<int64_t>(I, 8192));
  ttm_zero_half_kernel<<<rows_grid, 256, 0, s>>>(Ii, Ri, C);
  int rc = check_launch("ttm zero kernel");
  if (!rc && nnz > 0) {
    const int64_t blocks = std::min<int64_t>((nnz * R + 255) / 256, 65536);
    LaunchTimer timer(s);
    if (bdt == SYSTEC_F32)
      ttm_canonical_kernel<float><<<dim3(blocks), 256, 0, s>>>(
          Ii, nnz, idx[0], idx[1], idx[2], val, static_cast<const float*>(B), Ri, C);
    else
      ttm_canonical_kernel<uint16_t><<<dim3(blocks), 256, 0, s>>>(
          Ii, nnz, idx[0], idx[1], idx[2], val, static_cast<const uint16_t*>(B), Ri, C);
    rc = check_launch("ttm kernel");
  }
  if (!rc && mirror) {
    ttm_mirror_kernel<<<rows_grid, 256, 0, s>>>(Ii, Ri, C);
    rc = check_launch("ttm mirror kernel");
  }
  return rc;
}

}  // namespace systec
