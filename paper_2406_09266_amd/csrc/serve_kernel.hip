// The serving step: persistent launches run the work items of every request
// admitted to the step (continuous batching): one for the SSYMV items and one
// for the MTTKRP items, on two streams so that they overlap. Workgroups pull
// items through an atomic counter until the list is exhausted, so a step of
// small items from many requests fills the device as well as one large
// request. Each item runs the same device code as the standalone kernels.
#include "common.h"
#include "mttkrp_device.h"
#include "panel_device.h"

namespace systec {
namespace {

using namespace dev;

// Zeroes the outputs of newly admitted requests, cut into pieces of at most
// 16384 floats (one piece per workgroup iteration). Block 0 also resets the
// step's four work counters (SSYMV items, MTTKRP items of order 3, 4, 5).
__global__ void serve_zero_kernel(const ZeroSeg* __restrict__ segs, int nseg,
                                  int* __restrict__ counters) {
  if (blockIdx.x == 0 && threadIdx.x < 4) counters[threadIdx.x] = 0;
  for (int b = blockIdx.x; b < nseg; b += gridDim.x) {
    const ZeroSeg z = segs[b];
    for (int64_t i = threadIdx.x; i < z.count; i += blockDim.x) z.ptr[i] = 0.0f;
  }
}

template <int N, typename BT, int L>
__device__ __forceinline__ void view_range(const ServeItem& it) {
  IdxPtrs ip{};
#pragma unroll
  for (int q = 0; q < N; ++q) ip.p[q] = static_cast<const int32_t*>(it.p[q]);
  const BT* B = static_cast<const BT*>(it.in);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int e0 = it.begin + w * kTileE; e0 < it.end; e0 += nw * kTileE)
    mttkrp_view_tile<N, BT, L>(it.slot, e0, min(it.end, e0 + kTileE), ip, it.val, B, it.R, it.out,
                               it.R, 0, it.R);
}

template <int N, typename BT>
__device__ __forceinline__ void view_item(const ServeItem& it) {
  if (it.R <= 8) view_range<N, BT, 8>(it);
  else if (it.R <= 16) view_range<N, BT, 16>(it);
  else if (it.R <= 32) view_range<N, BT, 32>(it);
  else view_range<N, BT, 64>(it);
}

// Persistent step kernels: workgroups pull items through an atomic counter
// until the list is exhausted (every workgroup reaches the same exit).
// SSYMV panel chunks need the panel's row sums in LDS (512 threads, 64 KiB);
// MTTKRP view ranges need no LDS and run at full occupancy (256 threads, one
// kernel per tensor order so that each keeps the registers of its own order).
__device__ __forceinline__ int next_item(int* counter, int* s_next) {
  if (threadIdx.x == 0) *s_next = atomicAdd(counter, 1);
  __syncthreads();
  // the same for every lane: make that visible so the item is read with
  // scalar loads into SGPRs instead of occupying vector registers
  const int i = __builtin_amdgcn_readfirstlane(*s_next);
  __syncthreads();
  return i;
}

__global__ __launch_bounds__(kServeBlock) void serve_ssymv_kernel(const ServeItem* __restrict__ items,
                                                                int nitems,
                                                                int* __restrict__ counter) {
  extern __shared__ float s_lds[];
  __shared__ int s_next;
  for (;;) {
    const int i = next_item(counter, &s_next);
    if (i >= nitems) return;  // uniform across the workgroup
    const ServeItem it = items[i];
    const auto* pcol = static_cast<const int32_t*>(it.p[0]);
    const auto* prow = static_cast<const uint16_t*>(it.p[1]);
    const auto* pval = static_cast<const float*>(it.p[2]);
    if (it.dtype == SYSTEC_F32)
      ssymv_panel_chunk<float>(it.dim, it.H, it.panel, it.begin, it.end, pcol, prow, pval,
                               static_cast<const float*>(it.in), it.out, s_lds);
    else
      ssymv_panel_chunk<uint16_t>(it.dim, it.H, it.panel, it.begin, it.end, pcol, prow, pval,
                                  static_cast<const uint16_t*>(it.in), it.out, s_lds);
    __syncthreads();
  }
}

template <int N>
__global__ __launch_bounds__(kServeMttkrpBlock, 7) void serve_mttkrp_kernel(
    const ServeItem* __restrict__ items, int nitems, int* __restrict__ counter) {
  __shared__ int s_next;
  for (;;) {
    const int i = next_item(counter, &s_next);
    if (i >= nitems) return;
    const ServeItem it = items[i];
    if (it.dtype == SYSTEC_F32) view_item<N, float>(it);
    else view_item<N, uint16_t>(it);
  }
}

}  // namespace

int launch_serve_zero(const ZeroSeg* d_zero, int nzero, int* d_counters, hipStream_t s) {
  const int zgrid = std::max(1, std::min(nzero, 8192));
  serve_zero_kernel<<<dim3(zgrid), dim3(256), 0, s>>>(d_zero, nzero, d_counters);
  return check_launch("serve zero kernel");
}

int launch_serve_items(int kind, const ServeItem* d_items, int nitems, int* d_counter, int grid,
                       hipStream_t s) {
  if (nitems == 0) return SYSTEC_OK;
  const dim3 g(std::max(1, grid));
  switch (kind) {
    case 0:
      serve_ssymv_kernel<<<g, dim3(kServeBlock), kServeLds, s>>>(d_items, nitems, d_counter);
      break;
    case 3:
      serve_mttkrp_kernel<3><<<g, dim3(kServeMttkrpBlock), 0, s>>>(d_items, nitems, d_counter);
      break;
    case 4:
      serve_mttkrp_kernel<4><<<g, dim3(kServeMttkrpBlock), 0, s>>>(d_items, nitems, d_counter);
      break;
    default:
      serve_mttkrp_kernel<5><<<g, dim3(kServeMttkrpBlock), 0, s>>>(d_items, nitems, d_counter);
      break;
  }
  return check_launch(kind == 0 ? "serve ssymv kernel" : "serve mttkrp kernel");
}

}  // namespace systec
