// The serving step: one launch per kernel kind and variant runs the work of
// every request admitted to the step (continuous batching). SSYMV and the
// MTTKRP orders run on separate streams so that they overlap. The step's
// requests and their unit ranges arrive as kernel arguments; workgroup b runs
// item b (one work unit of one request) with the same device code as the
// standalone kernels. Work units are short (a few microseconds), so the
// hardware dispatcher balances the items and interleaves the workgroups of
// the kinds that run at the same time; a prologue kernel on each stream
// zeroes the outputs of newly admitted requests first.
#include <atomic>

#include "common.h"
#include "mttkrp_device.h"
#include "panel_device.h"

namespace systec {
namespace {

using namespace dev;

__global__ void serve_prologue_kernel(ZeroArgs z) {
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
// range each (vector lanes, which sum runs across the wave).
template <int N, typename BT, int L>
__device__ __forceinline__ void view_range_vec(const ServeTensor* t, const ServeUnit& u,
                                               const StepReq& q) {
  constexpr int V = lane_vec_width(L, L, sizeof(BT));  // step_variant checked R % V
  static_assert(V > 0, "vector lanes need an even lane class");
  constexpr int Lg = L / V;  // lanes per row at R <= L
  IdxPtrs ip{};
#pragma unroll
  for (int s = 0; s < N; ++s) ip.p[s] = uni_ptr(static_cast<const int32_t*>(t->p[u.a][s]));
  const float* val = uni_ptr(t->val[u.a]);
  const BT* B = static_cast<const BT*>(q.in);
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int per = (u.c - u.b + nw - 1) / nw;
  const int e0 = min(u.c, u.b + w * per), e1 = min(u.c, e0 + per);
  mttkrp_view_range_vec_slot<N, BT, V, Lg>(u.a, e0, e1, ip, val, B, q.R, q.out, q.R, 0, q.R);
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

// SSYMV items need the panel's row sums in LDS (512 threads, 32 KiB, and
// 16 KiB more for a BF16 request's staged x slice); MTTKRP
// items need no LDS and run at full occupancy (256 threads, one kernel per
// tensor order so that each keeps the registers of its own order); the four
// waves of an MTTKRP workgroup share an item of a few tiles each.
template <bool kStageX>
__global__ __launch_bounds__(kServeBlock) void serve_ssymv_kernel(StepArgs a) {
  extern __shared__ float s_lds[];
  const int i = blockIdx.x;
  const StepReq& r = a.req[find_req(a, i)];
  const ServeTensor* t = r.t;
  const ServeUnit u = load_unit(t, r.unit0 + (i - r.item0));
  const auto* pcol = uni_ptr(static_cast<const int32_t*>(t->p[0][0]));
  const auto* prow = uni_ptr(static_cast<const uint16_t*>(t->p[0][1]));
  const auto* pval = uni_ptr(static_cast<const float*>(t->p[0][2]));
  const auto* ppack = uni_ptr(static_cast<const uint32_t*>(t->p[0][3]));
  const auto* pbase = uni_ptr(static_cast<const int32_t*>(t->p[0][4]));
  const int dim = uni(t->dim), H = uni(t->H);
  if (r.dtype == SYSTEC_F32)
    ssymv_panel_chunk<float>(dim, H, u.a, u.b, u.c, pcol, prow, pval, ppack, pbase,
                             static_cast<const float*>(r.in), r.out, s_lds);
  else  // BF16 x: with kStageX the panel's x slice follows the row sums in LDS
    ssymv_panel_chunk<uint16_t, kStageX>(dim, H, u.a, u.b, u.c, pcol, prow, pval, ppack, pbase,
                                         static_cast<const uint16_t*>(r.in), r.out, s_lds,
                                         reinterpret_cast<uint16_t*>(s_lds + H));
}

// Whether the device gives a workgroup room for the staged x slice (set by
// serve_init_kernels).
std::atomic<bool> g_serve_stage_x{false};

// One MTTKRP step kernel per (order, input dtype, lane layout, lane class),
// so that each keeps only the registers of its own variant.
template <int N, typename BT, int L, bool kVec>
__global__ __launch_bounds__(kServeMttkrpBlock) void serve_mttkrp_kernel(StepArgs a) {
  const int i = blockIdx.x;
  const StepReq& r = a.req[find_req(a, i)];
  const ServeTensor* t = r.t;
  const ServeUnit u = load_unit(t, r.unit0 + (i - r.item0));
  if constexpr (kVec) view_range_vec<N, BT, L>(t, u, r);
  else view_range<N, BT, L>(t, u, r);
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
hipError_t launch_mttkrp_variant(int variant, const StepArgs& a, dim3 g, hipStream_t s) {
  const void* k = mttkrp_kernel_of<N>(variant);
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipLaunchKernel(k, g, dim3(kServeMttkrpBlock), args, 0, s);
}

}  // namespace

int launch_serve_prologue(const ZeroArgs& z, hipStream_t s) {
  int64_t total = 0;
  for (int k = 0; k < z.n; ++k) total += z.count[k];
  if (total == 0) return SYSTEC_OK;
  const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((total / 4 + 255) / 256, 2048)));
  serve_prologue_kernel<<<dim3(grid), dim3(256), 0, s>>>(z);
  return check_launch("serve prologue kernel");
}

int launch_serve_step(int kind, int variant, const StepArgs& a, hipStream_t s) {
  if (a.nitems == 0) return SYSTEC_OK;
  const dim3 g(a.nitems);
  hipError_t e = hipSuccess;
  switch (kind) {
    case 0:  // LDS limits set by serve_init_kernels
      if (g_serve_stage_x.load(std::memory_order_relaxed))
        serve_ssymv_kernel<true><<<g, dim3(kServeBlock), kServeLdsStaged, s>>>(a);
      else
        serve_ssymv_kernel<false><<<g, dim3(kServeBlock), kServeLds, s>>>(a);
      break;
    case 3: e = launch_mttkrp_variant<3>(variant, a, g, s); break;
    case 4: e = launch_mttkrp_variant<4>(variant, a, g, s); break;
    default: e = launch_mttkrp_variant<5>(variant, a, g, s); break;
  }
  if (e != hipSuccess) return check_hip(e, "serve mttkrp kernel launch");
  return check_launch(kind == 0 ? "serve ssymv kernel" : "serve mttkrp kernel");
}

int serve_init_kernels() {
  // more than the default 64 KiB of dynamic LDS (set before any launch)
  int dev = 0, limit = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (!rc)
    rc = check_hip(hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                   "hipDeviceGetAttribute(max shared memory)");
  if (!rc)
    rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(serve_ssymv_kernel<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kServeLds),
                   "hipFuncSetAttribute(dynamic LDS)");
  const bool stage = !rc && limit >= kServeLdsStaged;
  if (stage)
    rc = check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(serve_ssymv_kernel<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kServeLdsStaged),
                   "hipFuncSetAttribute(dynamic LDS)");
  g_serve_stage_x.store(stage && !rc, std::memory_order_relaxed);
  return rc;
}

}  // namespace systec
