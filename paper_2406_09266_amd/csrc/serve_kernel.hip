// The serving step: one launch per kernel kind runs the work of every request
// admitted to the step (continuous batching): one for SSYMV and one per
// MTTKRP order, on separate streams so that they overlap. The step's
// requests and their unit ranges arrive as kernel arguments. The launches
// are persistent: as many workgroups as fit on the device at once take items
// from eight work queues until all are empty, and each item runs the same
// device code as the standalone kernels.
//
// Work queues. Item i belongs to queue i mod 8; a queue is a counter that
// hands out its items in order. Workgroup b starts on queue b mod 8 (blocks
// are dispatched round-robin over the 8 XCDs, so a queue's items tend to stay
// on one XCD) and moves on to the other queues when its own is empty. A
// single counter serializes every workgroup of the chip on one address
// (about 80 M atomics/s); eight counters on separate cache lines spread that
// over eight. A prologue kernel on the same stream resets the counters
// before every step launch, and zeroes the outputs of newly admitted
// requests.
#include "common.h"
#include "mttkrp_device.h"
#include "panel_device.h"

namespace systec {
namespace {

using namespace dev;

__global__ void serve_prologue_kernel(ZeroArgs z, StepCounter* ctr, int nsets) {
  if (blockIdx.x == 0 && threadIdx.x < kStepQueues * nsets)
    ctr[threadIdx.x / kStepQueues].next[(threadIdx.x % kStepQueues) * kQueueStride] = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int s = 0; s < z.n; ++s) {
    float* p = z.ptr[s];
    const int64_t n = z.count[s];
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      float4* q = reinterpret_cast<float4*>(p);
      const int64_t n4 = n / 4;
      for (int64_t i = t0; i < n4; i += stride) q[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int64_t i = n4 * 4 + t0; i < n; i += stride) p[i] = 0.0f;
    } else {
      for (int64_t i = t0; i < n; i += stride) p[i] = 0.0f;
    }
  }
}

// Values that are the same in every lane, moved to scalar registers (the
// compiler cannot prove that loads through the step's descriptors are
// uniform, and would otherwise keep every pointer in vector registers).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return reinterpret_cast<T*>((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ ServeUnit load_unit(const ServeTensor* t, int k) {
  const ServeUnit u = uni_ptr(t->units)[k];
  return ServeUnit{uni(u.a), uni(u.b), uni(u.c), 0};
}

// The request that item i belongs to (item0 ascends; uniform across the
// workgroup, so this runs on scalar registers).
__device__ __forceinline__ int find_req(const StepArgs& a, int i) {
  int r = 0;
  for (int k = 1; k < a.nreq; ++k) r = (a.req[k].item0 <= i) ? k : r;
  return r;
}

// One MTTKRP item is a range of a few tiles of one view; the waves of the
// workgroup take every fourth tile (one lane per column) or a quarter of the
// range each (16-byte lanes, which sum runs across the wave).
template <int N, typename BT, int L>
__device__ __forceinline__ void view_range_vec(const ServeTensor* t, const ServeUnit& u,
                                               const StepReq& q) {
  constexpr int V = vec_cols<BT>();
  constexpr int Lg = (L / V) < 1 ? 1 : (L / V);  // lanes per row at R <= L
  IdxPtrs ip{};
#pragma unroll
  for (int s = 0; s < N; ++s) ip.p[s] = uni_ptr(static_cast<const int32_t*>(t->p[u.a][s]));
  const float* val = uni_ptr(t->val[u.a]);
  const BT* B = static_cast<const BT*>(q.in);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int per = (u.c - u.b + nw - 1) / nw;
  const int e0 = min(u.c, u.b + w * per), e1 = min(u.c, e0 + per);
  mttkrp_view_range_vec_slot<N, BT, Lg>(u.a, e0, e1, ip, val, B, q.R, q.out, q.R, 0, q.R);
}

template <int N, typename BT, int L>
__device__ __forceinline__ void view_range(const ServeTensor* t, const ServeUnit& u,
                                           const StepReq& q) {
  IdxPtrs ip{};
#pragma unroll
  for (int s = 0; s < N; ++s) ip.p[s] = uni_ptr(static_cast<const int32_t*>(t->p[u.a][s]));
  const float* val = uni_ptr(t->val[u.a]);
  const BT* B = static_cast<const BT*>(q.in);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (int e0 = u.b + w * kTileE; e0 < u.c; e0 += nw * kTileE)
    mttkrp_view_tile_slot<N, BT, L>(u.a, e0, min(u.c, e0 + kTileE), ip, val, B, q.R, q.out, q.R,
                                    0, q.R);
}

// Takes this workgroup's next item (uniform across the workgroup), or
// returns n when every queue is empty. `q` is the queue being drained.
__device__ __forceinline__ int take_item(StepCounter* c, int n, int* q, int* s_item) {
  if (threadIdx.x == 0) {
    int item = n;
    for (int k = 0; k < kStepQueues; ++k) {
      const int qq = (*q + k) & (kStepQueues - 1);
      int* ctr = c->next + qq * kQueueStride;
      // skip a drained queue without contending for its counter
      if (k > 0 && __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) * kStepQueues +
                           qq >= n)
        continue;
      const int i = atomicAdd(ctr, 1) * kStepQueues + qq;
      if (i < n) {
        item = i;
        *q = qq;
        break;
      }
    }
    *s_item = item;
  }
  __syncthreads();
  const int i = uni(*s_item);
  __syncthreads();
  return i;
}

// SSYMV items need the panel's row sums in LDS (1,024 threads, 128 KiB); MTTKRP
// items need no LDS and run at full occupancy (256 threads, one kernel per
// tensor order so that each keeps the registers of its own order); the four
// waves of an MTTKRP workgroup share an item of a few tiles each.
__global__ __launch_bounds__(kServeBlock) void serve_ssymv_kernel(StepArgs a, StepCounter* ctr) {
  extern __shared__ float s_lds[];
  __shared__ int s_item;
  int q = blockIdx.x & (kStepQueues - 1);
  for (int i = take_item(ctr, a.nitems, &q, &s_item); i < a.nitems;
       i = take_item(ctr, a.nitems, &q, &s_item)) {
    const StepReq& r = a.req[find_req(a, i)];
    const ServeTensor* t = r.t;
    const ServeUnit u = load_unit(t, r.unit0 + (i - r.item0));
    const auto* pcol = uni_ptr(static_cast<const int32_t*>(t->p[0][0]));
    const auto* prow = uni_ptr(static_cast<const uint16_t*>(t->p[0][1]));
    const auto* pval = uni_ptr(static_cast<const float*>(t->p[0][2]));
    const int dim = uni(t->dim), H = uni(t->H);
    if (r.dtype == SYSTEC_F32)
      ssymv_panel_chunk<float>(dim, H, u.a, u.b, u.c, pcol, prow, pval,
                               static_cast<const float*>(r.in), r.out, s_lds);
    else
      ssymv_panel_chunk<uint16_t>(dim, H, u.a, u.b, u.c, pcol, prow, pval,
                                  static_cast<const uint16_t*>(r.in), r.out, s_lds);
  }
}

// One MTTKRP step kernel per (order, input dtype, lane layout, lane class),
// so that each keeps only the registers of its own variant.
template <int N, typename BT, int L, bool kVec>
__global__ __launch_bounds__(kServeMttkrpBlock) void serve_mttkrp_kernel(StepArgs a,
                                                                         StepCounter* ctr) {
  __shared__ int s_item;
  int q = blockIdx.x & (kStepQueues - 1);
  for (int i = take_item(ctr, a.nitems, &q, &s_item); i < a.nitems;
       i = take_item(ctr, a.nitems, &q, &s_item)) {
    const StepReq& r = a.req[find_req(a, i)];
    const ServeTensor* t = r.t;
    const ServeUnit u = load_unit(t, r.unit0 + (i - r.item0));
    if constexpr (kVec) view_range_vec<N, BT, L>(t, u, r);
    else view_range<N, BT, L>(t, u, r);
  }
}

template <int N, typename BT, bool kVec>
const void* mttkrp_kernel_lanes(int lane_class) {
  switch (lane_class) {
    case 0: return reinterpret_cast<const void*>(serve_mttkrp_kernel<N, BT, 8, kVec>);
    case 1: return reinterpret_cast<const void*>(serve_mttkrp_kernel<N, BT, 16, kVec>);
    case 2: return reinterpret_cast<const void*>(serve_mttkrp_kernel<N, BT, 32, kVec>);
    default: return reinterpret_cast<const void*>(serve_mttkrp_kernel<N, BT, 64, kVec>);
  }
}

// The kernel of an MTTKRP variant (see step_variant).
template <int N>
const void* mttkrp_kernel_of(int variant) {
  const int lane_class = variant & 3;
  const bool vec = (variant & 4) != 0;
  if (variant & 8)
    return vec ? mttkrp_kernel_lanes<N, uint16_t, true>(lane_class)
               : mttkrp_kernel_lanes<N, uint16_t, false>(lane_class);
  return vec ? mttkrp_kernel_lanes<N, float, true>(lane_class)
             : mttkrp_kernel_lanes<N, float, false>(lane_class);
}

template <int N>
hipError_t launch_mttkrp_variant(int variant, const StepArgs& a, dim3 g, StepCounter* ctr,
                                 hipStream_t s) {
  const void* k = mttkrp_kernel_of<N>(variant);
  void* args[] = {const_cast<StepArgs*>(&a), &ctr};
  return hipLaunchKernel(k, g, dim3(kServeMttkrpBlock), args, 0, s);
}

}  // namespace

int launch_serve_prologue(const ZeroArgs& z, StepCounter* ctr, int nsets, hipStream_t s) {
  int64_t total = 0;
  for (int k = 0; k < z.n; ++k) total += z.count[k];
  const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((total / 4 + 255) / 256, 2048)));
  serve_prologue_kernel<<<dim3(grid), dim3(256), 0, s>>>(z, ctr, nsets);
  return check_launch("serve prologue kernel");
}

int launch_serve_step(int kind, int variant, const StepArgs& a, int grid, StepCounter* ctr,
                      hipStream_t s) {
  if (a.nitems == 0) return SYSTEC_OK;
  const dim3 g(std::max(1, std::min(grid, a.nitems)));
  hipError_t e = hipSuccess;
  switch (kind) {
    case 0: serve_ssymv_kernel<<<g, dim3(kServeBlock), kServeLds, s>>>(a, ctr); break;  // LDS limit set by serve_blocks_per_cu
    case 3: e = launch_mttkrp_variant<3>(variant, a, g, ctr, s); break;
    case 4: e = launch_mttkrp_variant<4>(variant, a, g, ctr, s); break;
    default: e = launch_mttkrp_variant<5>(variant, a, g, ctr, s); break;
  }
  if (e != hipSuccess) return check_hip(e, "serve mttkrp kernel launch");
  return check_launch(kind == 0 ? "serve ssymv kernel" : "serve mttkrp kernel");
}

int serve_blocks_per_cu(int kind, int variant, int* blocks) {
  hipError_t e;
  if (kind == 0) {
    // more than the default 64 KiB of dynamic LDS (set once, before any launch)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(serve_ssymv_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kServeLds);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, serve_ssymv_kernel, kServeBlock,
                                                       kServeLds);
  } else {
    const void* k = kind == 3 ? mttkrp_kernel_of<3>(variant)
                    : kind == 4 ? mttkrp_kernel_of<4>(variant)
                                : mttkrp_kernel_of<5>(variant);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, kServeMttkrpBlock, 0);
  }
  return check_hip(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
}

}  // namespace systec
