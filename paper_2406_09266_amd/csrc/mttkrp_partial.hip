// MTTKRP of a partially symmetric tensor (Sec. 2.1, partial symmetry; the
// general case of the symmetrization of Sec. 3.1 and 4.1). The slots of the
// order-N tensor form consecutive parts; the tensor is invariant under
// permutations of the indices inside each part, and only coordinates whose
// indices ascend inside every part are stored (canonical). Each part q has
// its own factor matrix F_q (I x R), and
//   C[i, r] = sum T[i, k2, ..., kN] prod_{t >= 2} F_{part(t)}[k_t, r]
// (output mode 1, in part 0).
//
// A stored (c, v) stands for every arrangement obtained by permuting each
// part on its own. Grouped by the value placed in slot 1 (a value of part 0),
// the arrangements that put the run of part 0 starting at slot t there number
// coef0(t) * prod_{q >= 1} mult_q, where mult_q = N_q! / prod(m!) counts the
// distinct arrangements of part q and coef0(t) = mult_0 m / N_0 those of part
// 0 with that run's value first (the per-run form of the multiplicity rule,
// applied to part 0, times the other parts' counts); their products are all
// equal, because a factor row depends on the part and the index only. So
//   C[c_t, :] += coef0(t) prod_{q>=1} mult_q * v * prod_{s != t} F_{part(s)}[c_s, :]
// for every slot t of part 0 that starts a run. With one part this is the
// fully symmetric MTTKRP.
#include "common.h"

namespace systec {
namespace {

struct IdxPtrsArg {
  const int32_t* p[5];
};

struct PartDesc {
  int32_t order, nparts;
  int32_t part_of[5];   // part of each slot
  int32_t start[5], size[5];
  const void* F[5];     // factor matrix of each part
};

__device__ __forceinline__ int64_t fact(int n) {
  int64_t f = 1;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

// Thread (e, r) over the entries and the R columns: consecutive threads take
// consecutive columns of one entry.
template <int N, typename FT>
__global__ __launch_bounds__(256) void mttkrp_partial_kernel(int64_t nnz, IdxPtrsArg idx,
                                                           const float* __restrict__ val,
                                                           PartDesc pd, int R,
                                                           float* __restrict__ C) {
  const int64_t total = nnz * R;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < total;
       w += stride) {
    const int64_t e = w / R;
    const int r = static_cast<int>(w - e * R);
    int c[N];
#pragma unroll
    for (int t = 0; t < N; ++t) c[t] = idx.p[t][e];
    const float v = val[e];
    // the factor entry of every slot, and the product over the slots outside
    // part 0 times those parts' arrangement counts
    float f[N];
#pragma unroll
    for (int t = 0; t < N; ++t)
      f[t] = load_f32(static_cast<const FT*>(pd.F[pd.part_of[t]]), static_cast<int64_t>(c[t]) * R + r);
    float other = 1.0f;
    int64_t mult_other = 1;
    for (int q = 1; q < pd.nparts; ++q) {
      int64_t denom = 1;
      int run = 1;
      for (int t = pd.start[q]; t < pd.start[q] + pd.size[q]; ++t) {
        other *= f[t];
        if (t > pd.start[q] && c[t] == c[t - 1]) denom *= ++run;
        else run = 1;
      }
      mult_other *= fact(pd.size[q]) / denom;
    }
    // part 0: runs of equal indices in slots [0, N0)
    const int N0 = pd.size[0];
    int64_t denom0 = 1;
    int run = 1;
    for (int t = 1; t < N0; ++t) {
      if (c[t] == c[t - 1]) denom0 *= ++run;
      else run = 1;
    }
    const int64_t mult0 = fact(N0) / denom0;
    const float base = v * other * static_cast<float>(mult_other);
#pragma unroll
    for (int t = 0; t < N; ++t) {
      if (t >= N0) break;
      if (t > 0 && c[t] == c[t - 1]) continue;  // not the start of a run
      int m = 1;
      while (t + m < N0 && c[t + m] == c[t]) ++m;
      float p = base * static_cast<float>(mult0 * m / N0);
      for (int s = 0; s < N0; ++s)
        if (s != t) p *= f[s];
      atomic_add_noret(C + static_cast<int64_t>(c[t]) * R + r, p);
    }
  }
}

template <int N>
int launch_partial_n(int64_t nnz, const IdxPtrsArg& ip, const float* val, const PartDesc& pd,
                     systec_dtype fdt, int R, float* C, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((nnz * R + 255) / 256, 65536);
  if (fdt == SYSTEC_F32)
    mttkrp_partial_kernel<N, float><<<dim3(blocks), 256, 0, s>>>(nnz, ip, val, pd, R, C);
  else
    mttkrp_partial_kernel<N, uint16_t><<<dim3(blocks), 256, 0, s>>>(nnz, ip, val, pd, R, C);
  return check_launch("partially symmetric mttkrp kernel");
}

}  // namespace

int launch_mttkrp_partial(int order, int nparts, const int32_t* part_sizes, int64_t I,
                          int64_t nnz, const int32_t* const* idx, const float* val,
                          const void* const* F, systec_dtype fdt, int64_t R, float* C,
                          hipStream_t s) {
  int rc = launch_fill_f32(C, I * R, s);
  if (rc || nnz == 0) return rc;
  PartDesc pd{};
  pd.order = order;
  pd.nparts = nparts;
  int slot = 0;
  for (int q = 0; q < nparts; ++q) {
    pd.start[q] = slot;
    pd.size[q] = part_sizes[q];
    pd.F[q] = F[q];
    for (int k = 0; k < part_sizes[q]; ++k) pd.part_of[slot++] = q;
  }
  IdxPtrsArg ip{};
  for (int t = 0; t < order; ++t) ip.p[t] = idx[t];
  const int Ri = static_cast<int>(R);
  LaunchTimer timer(s);
  switch (order) {
    case 2: return launch_partial_n<2>(nnz, ip, val, pd, fdt, Ri, C, s);
    case 3: return launch_partial_n<3>(nnz, ip, val, pd, fdt, Ri, C, s);
    case 4: return launch_partial_n<4>(nnz, ip, val, pd, fdt, Ri, C, s);
    default: return launch_partial_n<5>(nnz, ip, val, pd, fdt, Ri, C, s);
  }
}

}  // namespace systec
