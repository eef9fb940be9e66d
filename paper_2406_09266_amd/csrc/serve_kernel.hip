// The serving step: one persistent launch runs the work items of every
// request admitted to the step (continuous batching). Workgroups pull items
// through an atomic counter until the list is exhausted, so a step of small
// items from many requests fills the device as well as one large request.
// Each item runs the same device code as the standalone kernels.
#include "common.h"
#include "mttkrp_device.h"
#include "panel_device.h"

namespace systec {
namespace {

using namespace dev;

// Zeroes the outputs of newly admitted requests: block (s, k) of the grid
// clears part k of segment s. Block 0 also resets the step's work counter.
__global__ void serve_zero_kernel(const ZeroSeg* __restrict__ segs, int nseg, int parts,
                                  int* __restrict__ counter) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  for (int b = blockIdx.x; b < nseg * parts; b += gridDim.x) {
    const ZeroSeg z = segs[b / parts];
    const int k = b % parts;
    const int64_t per = (z.count + parts - 1) / parts;
    const int64_t lo = k * per;
    const int64_t hi = min(z.count, lo + per);
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) z.ptr[i] = 0.0f;
  }
}

template <int N, typename BT>
__device__ __forceinline__ void view_range(const ServeItem& it) {
  IdxPtrs ip{};
#pragma unroll
  for (int q = 0; q < N; ++q) ip.p[q] = static_cast<const int32_t*>(it.p[q]);
  const BT* B = static_cast<const BT*>(it.in);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int e0 = it.begin + w * kTileE; e0 < it.end; e0 += nw * kTileE) {
    const int e1 = min(it.end, e0 + kTileE);
    if (it.R <= 8)
      mttkrp_view_tile<N, BT, 8>(it.slot, e0, e1, ip, it.val, B, it.R, it.out, it.R, 0, it.R);
    else if (it.R <= 16)
      mttkrp_view_tile<N, BT, 16>(it.slot, e0, e1, ip, it.val, B, it.R, it.out, it.R, 0, it.R);
    else if (it.R <= 32)
      mttkrp_view_tile<N, BT, 32>(it.slot, e0, e1, ip, it.val, B, it.R, it.out, it.R, 0, it.R);
    else
      mttkrp_view_tile<N, BT, 64>(it.slot, e0, e1, ip, it.val, B, it.R, it.out, it.R, 0, it.R);
  }
}

template <typename BT>
__device__ __forceinline__ void mttkrp_item(const ServeItem& it) {
  switch (it.order) {
    case 3: view_range<3, BT>(it); break;
    case 4: view_range<4, BT>(it); break;
    default: view_range<5, BT>(it); break;
  }
}

__global__ __launch_bounds__(kServeBlock) void serve_step_kernel(const ServeItem* __restrict__ items,
                                                               int nitems,
                                                               int* __restrict__ counter) {
  extern __shared__ float s_lds[];
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
    __syncthreads();
    const int i = s_next;
    __syncthreads();
    if (i >= nitems) return;  // uniform across the workgroup
    const ServeItem it = items[i];
    if (it.kind == 0) {
      const auto* pcol = static_cast<const int32_t*>(it.p[0]);
      const auto* prow = static_cast<const uint16_t*>(it.p[1]);
      const auto* pval = static_cast<const float*>(it.p[2]);
      if (it.dtype == SYSTEC_F32)
        ssymv_panel_chunk<float>(it.dim, it.H, it.panel, it.begin, it.end, pcol, prow, pval,
                                 static_cast<const float*>(it.in), it.out, s_lds);
      else
        ssymv_panel_chunk<uint16_t>(it.dim, it.H, it.panel, it.begin, it.end, pcol, prow, pval,
                                    static_cast<const uint16_t*>(it.in), it.out, s_lds);
    } else {
      if (it.dtype == SYSTEC_F32) mttkrp_item<float>(it);
      else mttkrp_item<uint16_t>(it);
    }
    __syncthreads();
  }
}

}  // namespace

int launch_serve_step(const ZeroSeg* d_zero, int nzero, const ServeItem* d_items, int nitems,
                      int* d_counter, int grid, hipStream_t s) {
  const int parts = 64;
  const int zgrid = std::max(1, std::min(nzero * parts, 4096));
  serve_zero_kernel<<<dim3(zgrid), dim3(256), 0, s>>>(d_zero, nzero, parts, d_counter);
  int rc = check_launch("serve zero kernel");
  if (rc || nitems == 0) return rc;
  serve_step_kernel<<<dim3(std::max(1, grid)), dim3(kServeBlock), kServeLds, s>>>(d_items, nitems,
                                                                               d_counter);
  return check_launch("serve step kernel");
}

}  // namespace systec
