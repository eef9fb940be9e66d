// One step of symmetric CP-ALS around MTTKRP. A symmetric CP decomposition
// models a symmetric tensor T of order N by one factor matrix B (I x R):
// T ~ [[B]] = sum_r b_r (x) ... (x) b_r, so the least-squares update of B is
// the same in every mode (Sec. 5.2.6: the symmetric CPD that MTTKRP serves).
// A step computes
//   C      = MTTKRP(T, B)                          (the symmetric kernel)
//   G      = B^T B                                 (R x R)
//   H      = G^(N-1), elementwise                  (the Gram matrix of the
//                                                   Khatri-Rao product of
//                                                   N-1 copies of B)
//   B_new  = C H^-1                                (the normal equations)
// and the terms of the fit of the model [[B]]:
//   ||T||^2      = sum over stored entries of (distinct permutations) v^2
//   <T, [[B]]>   = sum_{i,r} C[i,r] B[i,r]
//   ||[[B]]||^2  = sum_{r,s} G[r,s]^N
//   ||T - [[B]]||^2 = ||T||^2 - 2 <T, [[B]]> + ||[[B]]||^2.
//
// The small dense steps are HBM-bound (each reads B or C once; at I =
// 100,000 and R = 32 the Gram matrix is 0.2 GFLOP against 6.4-12.8 MB of
// reads), so they run on the vector ALUs, not on MFMA. Products and sums are
// FP32; the scalars are reduced from FP32 partials in FP64 at the end.
#include "common.h"
#include "mttkrp_device.h"

namespace systec {
namespace {

using namespace dev;

constexpr int kGramThreads = 256;
constexpr int kGramRows = 64;          // rows of B staged in LDS at a time
constexpr int kMaxPairs = 64 * 64 / kGramThreads;  // pairs (r, s) per thread, R <= 64
constexpr int kGramBlocks = 512;

// Partial Gram matrices: block b sums B[i,r] B[i,s] over its rows; thread
// tid owns the pairs q = tid + k * 256 of the R x R matrix.
template <typename BT>
__global__ __launch_bounds__(kGramThreads) void gram_partial_kernel(int I, int R,
                                                                  const BT* __restrict__ B,
                                                                  int rows_per_block,
                                                                  float* __restrict__ partial) {
  __shared__ float sB[kGramRows * 64];
  const int i0 = blockIdx.x * rows_per_block;
  const int i1 = min(I, i0 + rows_per_block);
  const int RR = R * R;
  float acc[kMaxPairs];
#pragma unroll
  for (int k = 0; k < kMaxPairs; ++k) acc[k] = 0.0f;
  for (int t0 = i0; t0 < i1; t0 += kGramRows) {
    const int nrows = min(kGramRows, i1 - t0);
    for (int q = threadIdx.x; q < nrows * R; q += blockDim.x)
      sB[q] = load_f32(B, static_cast<int64_t>(t0) * R + q);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxPairs; ++k) {
      const int q = threadIdx.x + k * kGramThreads;
      if (q < RR) {
        const int r = q / R, s = q - r * R;
        float a = acc[k];
        for (int i = 0; i < nrows; ++i) a += sB[i * R + r] * sB[i * R + s];
        acc[k] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kMaxPairs; ++k) {
    const int q = threadIdx.x + k * kGramThreads;
    if (q < RR) partial[static_cast<int64_t>(blockIdx.x) * RR + q] = acc[k];
  }
}

// G = sum of the partials, block by block in order (deterministic).
__global__ void gram_reduce_kernel(int RR, int nblk, const float* __restrict__ partial,
                                   float* __restrict__ G) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= RR) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += partial[static_cast<int64_t>(b) * RR + q];
  G[q] = g;
}

// One workgroup: H = G^(N-1) (elementwise), its Cholesky factor L (H = L
// L^T) and H^-1 = L^-T L^-1, all in LDS; ||[[B]]||^2 = sum G^N with FP32
// terms summed in FP64 at the end. If H is not positive definite (B does not
// have full column rank) H^-1 is filled with NaN.
__global__ __launch_bounds__(256) void cp_solve_kernel(int R, int order,
                                                      const float* __restrict__ G,
                                                      float* __restrict__ Hinv,
                                                      double* __restrict__ norm_model) {
  __shared__ float L[64 * 64];
  __shared__ float Li[64 * 64];
  __shared__ double s_part[256 / kWave];
  __shared__ int s_bad;
  const int RR = R * R;
  double part = 0.0;
  for (int q = threadIdx.x; q < RR; q += blockDim.x) {
    const float g = G[q];
    float h = 1.0f;
    for (int k = 1; k < order; ++k) h *= g;  // G^(N-1)
    L[q] = h;
    part += static_cast<double>(h * g);     // G^N
  }
  if (threadIdx.x == 0) s_bad = 0;
  for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d);
  if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x) / kWave; ++w) u += s_part[w];
    norm_model[0] = u;
  }
  // right-looking Cholesky in place (lower triangle of L)
  for (int k = 0; k < R; ++k) {
    if (threadIdx.x == 0) {
      const float p = L[k * R + k];
      if (!(p > 0.0f) || !isfinite(p)) s_bad = 1;
      L[k * R + k] = sqrtf(fmaxf(p, 0.0f));
    }
    __syncthreads();
    const float lkk = L[k * R + k];
    for (int i = k + 1 + threadIdx.x; i < R; i += blockDim.x) L[i * R + k] /= lkk;
    __syncthreads();
    for (int q = threadIdx.x; q < (R - k - 1) * (R - k - 1); q += blockDim.x) {
      const int i = k + 1 + q / (R - k - 1), j = k + 1 + q % (R - k - 1);
      if (j <= i) L[i * R + j] -= L[i * R + k] * L[j * R + k];
    }
    __syncthreads();
  }
  // L^-1 by forward substitution, one column per thread
  for (int j = threadIdx.x; j < R; j += blockDim.x) {
    for (int i = 0; i < R; ++i) Li[i * R + j] = 0.0f;
    for (int i = j; i < R; ++i) {
      float s = (i == j) ? 1.0f : 0.0f;
      for (int k = j; k < i; ++k) s -= L[i * R + k] * Li[k * R + j];
      Li[i * R + j] = s / L[i * R + i];
    }
  }
  __syncthreads();
  // H^-1 = L^-T L^-1: (i, j) = sum_{k >= max(i,j)} Li[k][i] Li[k][j]
  const bool bad = s_bad != 0;
  for (int q = threadIdx.x; q < RR; q += blockDim.x) {
    const int i = q / R, j = q - (q / R) * R;
    float s = 0.0f;
    for (int k = max(i, j); k < R; ++k) s += Li[k * R + i] * Li[k * R + j];
    Hinv[q] = bad ? __int_as_float(0x7fc00000) : s;
  }
}

// B_new = C H^-1 row by row (H^-1 staged in LDS), and the partial sums of
// <T, [[B]]> = sum C * B, one FP32 partial per block.
template <typename BT>
__global__ __launch_bounds__(256) void cp_update_kernel(int I, int R, const float* __restrict__ C,
                                                      const BT* __restrict__ B,
                                                      const float* __restrict__ Hinv,
                                                      float* __restrict__ B_new,
                                                      float* __restrict__ inner_partial) {
  __shared__ float sH[64 * 64];
  __shared__ float s_part[256 / kWave];
  const int RR = R * R;
  for (int q = threadIdx.x; q < RR; q += blockDim.x) sH[q] = Hinv[q];
  __syncthreads();
  float inner = 0.0f;
  const int64_t total = static_cast<int64_t>(I) * R;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += stride) {
    const int64_t i = e / R;
    const int r = static_cast<int>(e - i * R);
    const float* ci = C + i * R;
    float s = 0.0f;
    for (int k = 0; k < R; ++k) s += ci[k] * sH[k * R + r];
    B_new[e] = s;
    inner += ci[r] * load_f32(B, e);
  }
  for (int d = 32; d >= 1; d >>= 1) inner += __shfl_xor(inner, d);
  if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = inner;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < static_cast<int>(blockDim.x) / kWave; ++w) t += s_part[w];
    inner_partial[blockIdx.x] = t;
  }
}

// ||T||^2 partials: each stored entry stands for (distinct permutations)
// coordinates of value v.
template <int N>
__global__ __launch_bounds__(256) void norm2_partial_kernel(int nnz, IdxPtrs idx,
                                                          const float* __restrict__ val,
                                                          float* __restrict__ partial) {
  __shared__ float s_part[256 / kWave];
  float acc = 0.0f;
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    int c[N];
#pragma unroll
    for (int t = 0; t < N; ++t) c[t] = idx.p[t][e];
    const float v = val[e];
    acc += static_cast<float>(coef_table<N>().mult[equality_mask_of(c, N)]) * v * v;
  }
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
  if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < static_cast<int>(blockDim.x) / kWave; ++w) t += s_part[w];
    partial[blockIdx.x] = t;
  }
}

// fit = {||T||^2, <T,[[B]]>, ||[[B]]||^2, ||T - [[B]]||^2}: the FP32
// partials of the norm and the inner product summed in FP64.
__global__ __launch_bounds__(256) void cp_fit_kernel(const float* __restrict__ norm_partial,
                                                    int nnorm,
                                                    const float* __restrict__ inner_partial,
                                                    int ninner, const double* __restrict__ model,
                                                    double* __restrict__ fit) {
  __shared__ double s_a[256 / kWave], s_b[256 / kWave];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nnorm; k += blockDim.x) a += static_cast<double>(norm_partial[k]);
  for (int k = threadIdx.x; k < ninner; k += blockDim.x) b += static_cast<double>(inner_partial[k]);
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d);
    b += __shfl_xor(b, d);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_a[threadIdx.x / kWave] = a;
    s_b[threadIdx.x / kWave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x) / kWave; ++w) {
      ta += s_a[w];
      tb += s_b[w];
    }
    fit[0] = ta;
    fit[1] = tb;
    fit[2] = model[0];
    fit[3] = ta - 2.0 * tb + model[0];
  }
}

constexpr int kUpdateBlocks = 1024;
constexpr int kNormBlocks = 1024;

}  // namespace

int cp_workspace_floats(int64_t R) {
  return static_cast<int>(kGramBlocks * R * R + R * R + kUpdateBlocks + kNormBlocks + 2);
}

int launch_cp_step(const Tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                   float* B_new, float* G, double* fit, hipStream_t s) {
  const int I = static_cast<int>(t->dim);
  const int Ri = static_cast<int>(R);
  const int RR = Ri * Ri;
  // the MTTKRP as the automatic choice runs it: the one-lane-per-entry form
  // with B in LDS where it applies, else the slot views
  int rc = mttkrp_lane_shape_fits(I, bdt, R) ? launch_mttkrp_views_lane(t, B, bdt, R, C, s) : -1;
  if (rc == -1) rc = launch_mttkrp_views(t, B, bdt, R, C, s);
  if (rc) return rc;
  // workspace: Gram partials, H^-1, the inner-product and norm partials and
  // ||[[B]]||^2 (one double), stream-ordered
  float* ws = nullptr;
  const size_t ws_bytes = static_cast<size_t>(cp_workspace_floats(R)) * sizeof(float) + 16;
  rc = check_hip(hipMallocAsync(reinterpret_cast<void**>(&ws), ws_bytes, s),
                 "hipMallocAsync(cp step workspace)");
  if (rc) return rc;
  float* gpart = ws;
  float* hinv = gpart + static_cast<size_t>(kGramBlocks) * RR;
  float* ipart = hinv + RR;
  float* npart = ipart + kUpdateBlocks;
  double* model = reinterpret_cast<double*>(
      (reinterpret_cast<uintptr_t>(npart + kNormBlocks) + 7) & ~uintptr_t(7));
  const int nblk = std::max(1, std::min(kGramBlocks, (I + kGramRows - 1) / kGramRows));
  const int rows_per = (I + nblk - 1) / nblk;
  {
    LaunchTimer timer(s);
    if (bdt == SYSTEC_F32)
      gram_partial_kernel<float><<<nblk, kGramThreads, 0, s>>>(
          I, Ri, static_cast<const float*>(B), rows_per, gpart);
    else
      gram_partial_kernel<uint16_t><<<nblk, kGramThreads, 0, s>>>(
          I, Ri, static_cast<const uint16_t*>(B), rows_per, gpart);
    rc = check_launch("gram kernel");
  }
  if (!rc) {
    gram_reduce_kernel<<<(RR + 255) / 256, 256, 0, s>>>(RR, nblk, gpart, G);
    rc = check_launch("gram reduction");
  }
  if (!rc) {
    cp_solve_kernel<<<1, 256, 0, s>>>(Ri, t->order, G, hinv, model);
    rc = check_launch("cp solve kernel");
  }
  if (!rc) {
    LaunchTimer timer(s);
    if (bdt == SYSTEC_F32)
      cp_update_kernel<float><<<kUpdateBlocks, 256, 0, s>>>(
          I, Ri, C, static_cast<const float*>(B), hinv, B_new, ipart);
    else
      cp_update_kernel<uint16_t><<<kUpdateBlocks, 256, 0, s>>>(
          I, Ri, C, static_cast<const uint16_t*>(B), hinv, B_new, ipart);
    rc = check_launch("cp update kernel");
  }
  if (!rc) {
    IdxPtrs ip{};
    for (int q = 0; q < t->order; ++q) ip.p[q] = t->vidx[0][q];
    const int nz = static_cast<int>(t->nnz);
    switch (t->order) {
      case 3: norm2_partial_kernel<3><<<kNormBlocks, 256, 0, s>>>(nz, ip, t->vval[0], npart); break;
      case 4: norm2_partial_kernel<4><<<kNormBlocks, 256, 0, s>>>(nz, ip, t->vval[0], npart); break;
      default: norm2_partial_kernel<5><<<kNormBlocks, 256, 0, s>>>(nz, ip, t->vval[0], npart); break;
    }
    rc = check_launch("tensor norm kernel");
  }
  if (!rc) {
    cp_fit_kernel<<<1, 256, 0, s>>>(npart, kNormBlocks, ipart, kUpdateBlocks, model, fit);
    rc = check_launch("cp fit kernel");
  }
  const int rc2 = check_hip(hipFreeAsync(ws, s), "hipFreeAsync(cp step workspace)");
  return rc ? rc : rc2;
}

}  // namespace systec
