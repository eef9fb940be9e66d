// The C ABI of libsystec: argument checking, dispatch, error reporting and
// kernel timing. Every step of the computation runs in the HIP kernels of
// ssymv.hip, mttkrp.hip and aux.hip; this file only checks and routes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"

namespace systec {

std::string validation_message(unsigned int flags);

namespace {
thread_local std::string g_last_error;

constexpr int64_t kMaxIndex = (int64_t(1) << 31) - 1;

// kernel timing state
std::mutex g_timing_mu;
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;

bool valid_dtype(systec_dtype d) { return d == SYSTEC_F32 || d == SYSTEC_BF16; }

int check_csr_args(const char* fn, int64_t n, int64_t nnz, const int32_t* rowptr,
                   const int32_t* col, const float* val, const void* x, systec_dtype xdt,
                   const void* out) {
  if (n < 1 || n > kMaxIndex - 1) return fail(SYSTEC_EINVAL, std::string(fn) + ": n out of range");
  if (nnz < 0 || nnz > kMaxIndex) return fail(SYSTEC_EINVAL, std::string(fn) + ": nnz out of range");
  if (!valid_dtype(xdt)) return fail(SYSTEC_EINVAL, std::string(fn) + ": unsupported dtype");
  if (!rowptr || !x || !out) return fail(SYSTEC_EINVAL, std::string(fn) + ": NULL pointer");
  if (nnz > 0 && (!col || !val)) return fail(SYSTEC_EINVAL, std::string(fn) + ": NULL pointer");
  return SYSTEC_OK;
}

int check_coo_args(const char* fn, int order, int min_order, int64_t I, int64_t nnz,
                   const int32_t* const* idx, const float* val) {
  if (order < min_order || order > 5)
    return fail(SYSTEC_EINVAL, std::string(fn) + ": order out of range");
  if (I < 1 || I > kMaxIndex) return fail(SYSTEC_EINVAL, std::string(fn) + ": I out of range");
  if (nnz < 0 || nnz > kMaxIndex) return fail(SYSTEC_EINVAL, std::string(fn) + ": nnz out of range");
  if (nnz > 0) {
    if (!idx) return fail(SYSTEC_EINVAL, std::string(fn) + ": NULL index array");
    for (int t = 0; t < order; ++t)
      if (!idx[t]) return fail(SYSTEC_EINVAL, std::string(fn) + ": NULL index pointer");
    if (!val) return fail(SYSTEC_EINVAL, std::string(fn) + ": NULL value pointer");
  }
  return SYSTEC_OK;
}

int check_factor_args(const char* fn, int64_t I, const void* B, systec_dtype bdt, int64_t R,
                      const float* C) {
  if (R < 1 || R > kMaxIndex) return fail(SYSTEC_EINVAL, std::string(fn) + ": R out of range");
  if (I * R > kMaxIndex) return fail(SYSTEC_EINVAL, std::string(fn) + ": I*R too large");
  if (!valid_dtype(bdt)) return fail(SYSTEC_EINVAL, std::string(fn) + ": unsupported dtype");
  if (!B || !C) return fail(SYSTEC_EINVAL, std::string(fn) + ": NULL pointer");
  return SYSTEC_OK;
}

// Optional device validation before every one-shot call (SYSTEC_VALIDATE=1).
bool validate_always() {
  static const bool on = [] {
    const char* v = std::getenv("SYSTEC_VALIDATE");
    return v && v[0] == '1';
  }();
  return on;
}

}  // namespace

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return SYSTEC_OK;
  return fail(SYSTEC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

LaunchTimer::LaunchTimer(hipStream_t s) : stream(s) {
  std::lock_guard<std::mutex> lock(g_timing_mu);
  if (!g_timing) return;
  if (hipEventCreate(&start) != hipSuccess) {
    start = nullptr;
    return;
  }
  (void)hipEventRecord(start, s);
}

LaunchTimer::~LaunchTimer() {
  if (!start) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess) {
    (void)hipEventDestroy(start);
    return;
  }
  (void)hipEventRecord(stop, stream);
  std::lock_guard<std::mutex> lock(g_timing_mu);
  g_events.emplace_back(start, stop);
}

}  // namespace systec

using namespace systec;

extern "C" {

const char* systec_last_error(void) { return g_last_error.c_str(); }

const char* systec_version(void) { return "systec-gfx950 0.1"; }

int systec_ssymv(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, float* y,
                 systec_stream stream) {
  int rc = check_csr_args("systec_ssymv", n, nnz, rowptr, col, val, x, xdt, y);
  if (rc) return rc;
  auto s = static_cast<hipStream_t>(stream);
  if (validate_always() && (rc = systec_validate_csr_upper(n, nnz, rowptr, col, stream)))
    return rc;
  return launch_ssymv(n, nnz, rowptr, col, val, x, xdt, y, true, s);
}

int systec_spmv_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                    const float* val, const void* x, systec_dtype xdt, float* y,
                    systec_stream stream) {
  int rc = check_csr_args("systec_spmv_csr", n, nnz, rowptr, col, val, x, xdt, y);
  if (rc) return rc;
  return launch_ssymv(n, nnz, rowptr, col, val, x, xdt, y, false, static_cast<hipStream_t>(stream));
}

int systec_syprd(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                 const float* val, const void* x, systec_dtype xdt, double* out,
                 systec_stream stream) {
  int rc = check_csr_args("systec_syprd", n, nnz, rowptr, col, val, x, xdt, out);
  if (rc) return rc;
  if (validate_always() && (rc = systec_validate_csr_upper(n, nnz, rowptr, col, stream)))
    return rc;
  return launch_syprd(n, nnz, rowptr, col, val, x, xdt, out, static_cast<hipStream_t>(stream));
}

int systec_syprd_noalloc(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                         const float* val, const void* x, systec_dtype xdt, double* out,
                         systec_stream stream) {
  const int rc = check_csr_args("systec_syprd_noalloc", n, nnz, rowptr, col, val, x, xdt, out);
  if (rc) return rc;
  return launch_syprd_noalloc(n, nnz, rowptr, col, val, x, xdt, out,
                              static_cast<hipStream_t>(stream));
}

namespace {

// A prepared tensor whose whole factor fits one workgroup's LDS takes the
// one-lane-per-entry form with B in LDS: on the 5-D workload (I = 5,000,
// R = 16, BF16) it runs in 0.26 ms against 0.48 ms for the views, whose
// lane groups gather the factor rows through the L1.
bool lds_preferred(int64_t I, systec_dtype bdt, int64_t R) {
  return mttkrp_lane_shape_fits(I, bdt, R);
}

}  // namespace

int systec_mttkrp_choose(int64_t I, systec_dtype bdt, int64_t R, int prepared,
                         systec_mttkrp_algo* algo) {
  if (!algo) return fail(SYSTEC_EINVAL, "systec_mttkrp_choose: NULL pointer");
  if (I < 1 || I > kMaxIndex || R < 1 || R > kMaxIndex || !valid_dtype(bdt))
    return fail(SYSTEC_EINVAL, "systec_mttkrp_choose: argument out of range");
  if (!prepared) *algo = SYSTEC_MTTKRP_ATOMIC;
  else *algo = lds_preferred(I, bdt, R) ? SYSTEC_MTTKRP_LDS : SYSTEC_MTTKRP_VIEWS;
  return SYSTEC_OK;
}

int systec_mttkrp_ex(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                     const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                     systec_mttkrp_algo algo, systec_stream stream) {
  int rc = check_coo_args("systec_mttkrp", order, 3, I, nnz, idx, val);
  if (!rc) rc = check_factor_args("systec_mttkrp", I, B, bdt, R, C);
  if (rc) return rc;
  if (algo != SYSTEC_MTTKRP_AUTO && algo != SYSTEC_MTTKRP_ATOMIC)
    return fail(SYSTEC_EINVAL, "systec_mttkrp: algorithm needs a prepared tensor");
  if (validate_always() && (rc = systec_validate_coo(order, I, nnz, idx, stream))) return rc;
  return launch_mttkrp(order, I, nnz, idx, val, B, bdt, R, C, true,
                       static_cast<hipStream_t>(stream));
}

int systec_mttkrp(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                  const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                  systec_stream stream) {
  return systec_mttkrp_ex(order, I, nnz, idx, val, B, bdt, R, C, SYSTEC_MTTKRP_AUTO, stream);
}

int systec_mttkrp_full(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                       const float* val, const void* B, systec_dtype bdt, int64_t R, float* C,
                       systec_stream stream) {
  int rc = check_coo_args("systec_mttkrp_full", order, 2, I, nnz, idx, val);
  if (!rc) rc = check_factor_args("systec_mttkrp_full", I, B, bdt, R, C);
  if (rc) return rc;
  return launch_mttkrp(order, I, nnz, idx, val, B, bdt, R, C, false,
                       static_cast<hipStream_t>(stream));
}

int systec_expand_csr_size(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                           int64_t* full_nnz, systec_stream stream) {
  if (n < 1 || n > kMaxIndex - 1 || nnz < 0 || nnz > kMaxIndex)
    return fail(SYSTEC_EINVAL, "systec_expand_csr_size: size out of range");
  if (!rowptr || (nnz > 0 && !col) || !full_nnz)
    return fail(SYSTEC_EINVAL, "systec_expand_csr_size: NULL pointer");
  return expand_csr_size(n, nnz, rowptr, col, full_nnz, static_cast<hipStream_t>(stream));
}

int systec_expand_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                      const float* val, int32_t* full_rowptr, int32_t* full_col,
                      float* full_val, systec_stream stream) {
  int rc = check_csr_args("systec_expand_csr", n, nnz, rowptr, col, val, rowptr, SYSTEC_F32,
                          full_rowptr);
  if (rc) return rc;
  if (nnz > 0 && (!full_col || !full_val))
    return fail(SYSTEC_EINVAL, "systec_expand_csr: NULL output");
  return expand_csr(n, nnz, rowptr, col, val, full_rowptr, full_col, full_val,
                    static_cast<hipStream_t>(stream));
}

int systec_expand_coo_size(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                           int64_t* full_nnz, systec_stream stream) {
  int rc = check_coo_args("systec_expand_coo_size", order, 2, I, nnz, idx, nullptr);
  if (rc && nnz > 0 && idx) {
    // val is not needed here; re-check without it
    bool ok = order >= 2 && order <= 5 && I >= 1;
    for (int t = 0; ok && t < order; ++t) ok = idx[t] != nullptr;
    if (ok) rc = SYSTEC_OK;
  }
  if (rc) return rc;
  if (!full_nnz) return fail(SYSTEC_EINVAL, "systec_expand_coo_size: NULL output");
  *full_nnz = 0;
  if (nnz == 0) return SYSTEC_OK;
  return expand_coo_size(order, I, nnz, idx, full_nnz, static_cast<hipStream_t>(stream));
}

int systec_expand_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                      const float* val, int32_t* const* out_idx, float* out_val,
                      systec_stream stream) {
  int rc = check_coo_args("systec_expand_coo", order, 2, I, nnz, idx, val);
  if (rc) return rc;
  if (nnz == 0) return SYSTEC_OK;
  if (!out_idx || !out_val) return fail(SYSTEC_EINVAL, "systec_expand_coo: NULL output");
  for (int t = 0; t < order; ++t)
    if (!out_idx[t]) return fail(SYSTEC_EINVAL, "systec_expand_coo: NULL output");
  return expand_coo(order, I, nnz, idx, val, out_idx, out_val, static_cast<hipStream_t>(stream));
}

int systec_expansion_stats(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                           int64_t* hist, int64_t* effective_nnz, systec_stream stream) {
  if (order < 2 || order > 5) return fail(SYSTEC_EINVAL, "systec_expansion_stats: order");
  if (I < 1 || nnz < 0 || nnz > kMaxIndex)
    return fail(SYSTEC_EINVAL, "systec_expansion_stats: size");
  if (!hist || !effective_nnz) return fail(SYSTEC_EINVAL, "systec_expansion_stats: NULL output");
  if (nnz > 0) {
    if (!idx) return fail(SYSTEC_EINVAL, "systec_expansion_stats: NULL index array");
    for (int t = 0; t < order; ++t)
      if (!idx[t]) return fail(SYSTEC_EINVAL, "systec_expansion_stats: NULL index pointer");
  }
  auto s = static_cast<hipStream_t>(stream);
  unsigned long long* d = nullptr;
  int rc = check_hip(hipMalloc(&d, 17 * sizeof(unsigned long long)), "hipMalloc");
  if (rc) return rc;
  unsigned long long h[17] = {0};
  rc = check_hip(hipMemsetAsync(d, 0, sizeof(h), s), "hipMemsetAsync");
  if (!rc) rc = launch_expansion_stats(order, nnz, idx, d, s);
  if (!rc) rc = check_hip(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  (void)hipFree(d);
  if (rc) return rc;
  for (int m = 0; m < 16; ++m) hist[m] = static_cast<int64_t>(h[m]);
  *effective_nnz = static_cast<int64_t>(h[16]);
  return SYSTEC_OK;
}

static int finish_validation(unsigned int* d, hipStream_t s, int rc) {
  unsigned int flags = 0;
  if (!rc) rc = check_hip(hipMemcpyAsync(&flags, d, sizeof(flags), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync");
  if (!rc) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  (void)hipFree(d);
  if (rc) return rc;
  if (flags) return fail(SYSTEC_ENONCANON, "not canonical: " + validation_message(flags));
  return SYSTEC_OK;
}

int systec_validate_csr_upper(int64_t n, int64_t nnz, const int32_t* rowptr,
                              const int32_t* col, systec_stream stream) {
  if (n < 1 || n > kMaxIndex - 1 || nnz < 0 || nnz > kMaxIndex)
    return fail(SYSTEC_EINVAL, "systec_validate_csr_upper: size");
  if (!rowptr || (nnz > 0 && !col)) return fail(SYSTEC_EINVAL, "systec_validate_csr_upper: NULL");
  auto s = static_cast<hipStream_t>(stream);
  unsigned int* d = nullptr;
  int rc = check_hip(hipMalloc(&d, sizeof(unsigned int)), "hipMalloc");
  if (rc) return rc;
  rc = check_hip(hipMemsetAsync(d, 0, sizeof(unsigned int), s), "hipMemsetAsync");
  if (!rc) rc = launch_validate_csr_upper(n, nnz, rowptr, col, d, s);
  return finish_validation(d, s, rc);
}

int systec_validate_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                        systec_stream stream) {
  if (order < 2 || order > 5 || I < 1 || I > kMaxIndex || nnz < 0 || nnz > kMaxIndex)
    return fail(SYSTEC_EINVAL, "systec_validate_coo: size or order");
  if (nnz > 0) {
    if (!idx) return fail(SYSTEC_EINVAL, "systec_validate_coo: NULL index array");
    for (int t = 0; t < order; ++t)
      if (!idx[t]) return fail(SYSTEC_EINVAL, "systec_validate_coo: NULL index pointer");
  }
  auto s = static_cast<hipStream_t>(stream);
  unsigned int* d = nullptr;
  int rc = check_hip(hipMalloc(&d, sizeof(unsigned int)), "hipMalloc");
  if (rc) return rc;
  rc = check_hip(hipMemsetAsync(d, 0, sizeof(unsigned int), s), "hipMemsetAsync");
  if (!rc) rc = launch_validate_coo(order, I, nnz, idx, d, s);
  return finish_validation(d, s, rc);
}

int systec_canonicalize_coo(int order, int64_t nnz, int32_t* const* idx, double* val,
                            int64_t* nnz_out) {
  if (order < 1 || order > 5 || nnz < 0 || nnz > kMaxIndex || !nnz_out)
    return fail(SYSTEC_EINVAL, "systec_canonicalize_coo: argument");
  if (nnz > 0) {
    if (!idx || !val) return fail(SYSTEC_EINVAL, "systec_canonicalize_coo: NULL pointer");
    for (int t = 0; t < order; ++t)
      if (!idx[t]) return fail(SYSTEC_EINVAL, "systec_canonicalize_coo: NULL pointer");
  }
  struct Entry {
    int32_t c[5];
    double v;
  };
  std::vector<Entry> e(static_cast<size_t>(nnz));
  for (int64_t q = 0; q < nnz; ++q) {
    for (int t = 0; t < 5; ++t) e[q].c[t] = t < order ? idx[t][q] : 0;
    std::sort(e[q].c, e[q].c + order);
    e[q].v = val[q];
  }
  std::stable_sort(e.begin(), e.end(), [order](const Entry& a, const Entry& b) {
    return std::lexicographical_compare(a.c, a.c + order, b.c, b.c + order);
  });
  int64_t m = 0;
  for (int64_t q = 0; q < nnz; ++q) {
    if (m > 0 && std::equal(e[q].c, e[q].c + order, e[m - 1].c)) {
      e[m - 1].v += e[q].v;
    } else {
      e[m++] = e[q];
    }
  }
  for (int64_t q = 0; q < m; ++q) {
    for (int t = 0; t < order; ++t) idx[t][q] = e[q].c[t];
    val[q] = e[q].v;
  }
  *nnz_out = m;
  return SYSTEC_OK;
}

int systec_quantize_bf16(const float* in, uint16_t* out, int64_t n, systec_stream stream) {
  if (n < 0) return fail(SYSTEC_EINVAL, "systec_quantize_bf16: n < 0");
  if (n > 0 && (!in || !out)) return fail(SYSTEC_EINVAL, "systec_quantize_bf16: NULL pointer");
  return launch_quantize_bf16(in, out, n, static_cast<hipStream_t>(stream));
}

int systec_tensor_create_csr(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                             const float* val, systec_stream stream, systec_tensor** out) {
  return systec_tensor_create_csr_ex(n, nnz, rowptr, col, val, 0, stream, out);
}

int systec_tensor_create_csr_ex(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                                const float* val, int relabel, systec_stream stream,
                                systec_tensor** out) {
  int rc = check_csr_args("systec_tensor_create_csr", n, nnz, rowptr, col, val, rowptr,
                          SYSTEC_F32, out);
  if (rc) return rc;
  if (relabel < -1 || relabel > 1)
    return fail(SYSTEC_EINVAL, "systec_tensor_create_csr_ex: relabel must be -1, 0 or 1");
  if ((rc = systec_validate_csr_upper(n, nnz, rowptr, col, stream))) return rc;
  auto s = static_cast<hipStream_t>(stream);
  int64_t full = 0;
  if (nnz > 0 && (rc = expand_csr_size(n, nnz, rowptr, col, &full, s))) return rc;
  Tensor* t = nullptr;
  if ((rc = tensor_create_csr(n, nnz, rowptr, col, val, kPanelRows, relabel, s, &t))) return rc;
  t->effective_nnz = full;
  *out = new systec_tensor{t};
  return SYSTEC_OK;
}

int systec_tensor_create_coo(int order, int64_t I, int64_t nnz, const int32_t* const* idx,
                             const float* val, systec_stream stream, systec_tensor** out) {
  int rc = check_coo_args("systec_tensor_create_coo", order, 3, I, nnz, idx, val);
  if (rc) return rc;
  if (!out) return fail(SYSTEC_EINVAL, "systec_tensor_create_coo: NULL output");
  if ((rc = systec_validate_coo(order, I, nnz, idx, stream))) return rc;
  auto s = static_cast<hipStream_t>(stream);
  int64_t hist[16], eff = 0;
  if (nnz > 0 && (rc = systec_expansion_stats(order, I, nnz, idx, hist, &eff, stream))) return rc;
  Tensor* t = nullptr;
  if ((rc = tensor_create_coo(order, I, nnz, idx, val, s, &t))) return rc;
  t->effective_nnz = eff;
  *out = new systec_tensor{t};
  return SYSTEC_OK;
}

int systec_tensor_info(const systec_tensor* t, int* order, int64_t* dim, int64_t* nnz,
                       int64_t* effective_nnz, uint64_t* bytes) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_tensor_info: NULL handle");
  if (order) *order = t->impl->order;
  if (dim) *dim = t->impl->dim;
  if (nnz) *nnz = t->impl->nnz;
  if (effective_nnz) *effective_nnz = t->impl->effective_nnz;
  if (bytes) *bytes = t->impl->bytes;
  return SYSTEC_OK;
}

int systec_ssymv_t_ex(const systec_tensor* t, const void* x, systec_dtype xdt, float* y,
                      int vertex_order, systec_stream stream) {
  if (vertex_order != SYSTEC_ORDER_CALLER && vertex_order != SYSTEC_ORDER_STORED)
    return fail(SYSTEC_EINVAL, "systec_ssymv_t_ex: vertex_order must be 0 or 1");
  if (vertex_order == SYSTEC_ORDER_CALLER) return systec_ssymv_t(t, x, xdt, y, stream);
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_ssymv_t_ex: NULL handle");
  if (t->impl->kind != 0) return fail(SYSTEC_EINVAL, "systec_ssymv_t_ex: not a matrix");
  if (!valid_dtype(xdt)) return fail(SYSTEC_EINVAL, "systec_ssymv_t_ex: unsupported dtype");
  if (!x || !y) return fail(SYSTEC_EINVAL, "systec_ssymv_t_ex: NULL pointer");
  return launch_ssymv_panel_stored(t->impl, x, xdt, y, static_cast<hipStream_t>(stream));
}

int systec_syprd_t_ex(const systec_tensor* t, const void* x, systec_dtype xdt, double* out,
                      int vertex_order, systec_stream stream) {
  if (vertex_order != SYSTEC_ORDER_CALLER && vertex_order != SYSTEC_ORDER_STORED)
    return fail(SYSTEC_EINVAL, "systec_syprd_t_ex: vertex_order must be 0 or 1");
  if (vertex_order == SYSTEC_ORDER_CALLER) return systec_syprd_t(t, x, xdt, out, stream);
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_syprd_t_ex: NULL handle");
  if (t->impl->kind != 0) return fail(SYSTEC_EINVAL, "systec_syprd_t_ex: not a matrix");
  if (!valid_dtype(xdt)) return fail(SYSTEC_EINVAL, "systec_syprd_t_ex: unsupported dtype");
  if (!x || !out) return fail(SYSTEC_EINVAL, "systec_syprd_t_ex: NULL pointer");
  return launch_syprd_panel_stored(t->impl, x, xdt, out, static_cast<hipStream_t>(stream));
}

int systec_syprd_t(const systec_tensor* t, const void* x, systec_dtype xdt, double* out,
                   systec_stream stream) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_syprd_t: NULL handle");
  if (t->impl->kind != 0) return fail(SYSTEC_EINVAL, "systec_syprd_t: not a matrix");
  if (!valid_dtype(xdt)) return fail(SYSTEC_EINVAL, "systec_syprd_t: unsupported dtype");
  if (!x || !out) return fail(SYSTEC_EINVAL, "systec_syprd_t: NULL pointer");
  return launch_syprd_panel(t->impl, x, xdt, out, static_cast<hipStream_t>(stream));
}

int systec_tensor_vertex_order(const systec_tensor* t, int* relabeled, int32_t* perm,
                               systec_stream stream) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_tensor_vertex_order: NULL handle");
  if (t->impl->kind != 0) return fail(SYSTEC_EINVAL, "systec_tensor_vertex_order: not a matrix");
  const bool r = t->impl->relabeled;
  if (relabeled) *relabeled = r ? 1 : 0;
  if (!perm || !r || t->impl->dim == 0) return SYSTEC_OK;
  return check_hip(hipMemcpyAsync(perm, t->impl->perm, static_cast<size_t>(t->impl->dim) * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                   "hipMemcpyAsync(vertex order)");
}

int systec_tensor_destroy(systec_tensor* t) {
  if (!t) return SYSTEC_OK;
  tensor_free(t->impl);
  delete t;
  return SYSTEC_OK;
}

int systec_bellman_ford(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                        const float* val, const float* d, float* y, systec_stream stream) {
  int rc = check_csr_args("systec_bellman_ford", n, nnz, rowptr, col, val, d, SYSTEC_F32, y);
  if (rc) return rc;
  auto s = static_cast<hipStream_t>(stream);
  if (validate_always() && (rc = systec_validate_csr_upper(n, nnz, rowptr, col, stream))) return rc;
  return launch_bellman_ford(n, nnz, rowptr, col, val, d, y, s);
}

int systec_bellman_ford_t(const systec_tensor* t, const float* d, float* y,
                          systec_stream stream) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_bellman_ford_t: NULL handle");
  if (t->impl->kind != 0) return fail(SYSTEC_EINVAL, "systec_bellman_ford_t: not a matrix");
  if (!d || !y) return fail(SYSTEC_EINVAL, "systec_bellman_ford_t: NULL pointer");
  return launch_bellman_ford_panel(t->impl, d, y, static_cast<hipStream_t>(stream));
}

int systec_ttm(int64_t I, int64_t nnz, const int32_t* const* idx, const float* val,
               const void* B, systec_dtype bdt, int64_t R, float* C, int mirror,
               systec_stream stream) {
  int rc = check_coo_args("systec_ttm", 3, 3, I, nnz, idx, val);
  if (rc) return rc;
  if (R < 1 || R > kMaxIndex) return fail(SYSTEC_EINVAL, "systec_ttm: R out of range");
  if (I * R > kMaxIndex) return fail(SYSTEC_EINVAL, "systec_ttm: I*R too large");
  if (I > (int64_t(1) << 40) / (I * R)) return fail(SYSTEC_EINVAL, "systec_ttm: I*I*R too large");
  if (!valid_dtype(bdt)) return fail(SYSTEC_EINVAL, "systec_ttm: unsupported dtype");
  if (!B || !C) return fail(SYSTEC_EINVAL, "systec_ttm: NULL pointer");
  if (mirror != 0 && mirror != 1) return fail(SYSTEC_EINVAL, "systec_ttm: mirror must be 0 or 1");
  auto s = static_cast<hipStream_t>(stream);
  if (validate_always() && (rc = systec_validate_coo(3, I, nnz, idx, stream))) return rc;
  return launch_ttm(I, nnz, idx, val, B, bdt, R, C, mirror == 1, s);
}

int systec_mttkrp_partial(int order, int nparts, const int32_t* part_sizes, int64_t I,
                          int64_t nnz, const int32_t* const* idx, const float* val,
                          const void* const* F, systec_dtype fdt, int64_t R, float* C,
                          systec_stream stream) {
  int rc = check_coo_args("systec_mttkrp_partial", order, 2, I, nnz, idx, val);
  if (rc) return rc;
  if (!part_sizes || nparts < 1 || nparts > order)
    return fail(SYSTEC_EINVAL, "systec_mttkrp_partial: bad partition");
  int sum = 0;
  for (int q = 0; q < nparts; ++q) {
    if (part_sizes[q] < 1) return fail(SYSTEC_EINVAL, "systec_mttkrp_partial: empty part");
    sum += part_sizes[q];
  }
  if (sum != order) return fail(SYSTEC_EINVAL, "systec_mttkrp_partial: parts must sum to order");
  if (!F) return fail(SYSTEC_EINVAL, "systec_mttkrp_partial: NULL factor array");
  for (int q = 0; q < nparts; ++q)
    if (!F[q]) return fail(SYSTEC_EINVAL, "systec_mttkrp_partial: NULL factor");
  if ((rc = check_factor_args("systec_mttkrp_partial", I, F[0], fdt, R, C))) return rc;
  return launch_mttkrp_partial(order, nparts, part_sizes, I, nnz, idx, val, F, fdt, R, C,
                               static_cast<hipStream_t>(stream));
}

int systec_cp_step(const systec_tensor* t, const void* B, systec_dtype bdt, int64_t R, float* C,
                   float* B_new, float* G, double* fit, systec_stream stream) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_cp_step: NULL handle");
  const Tensor* tn = t->impl;
  if (tn->kind != 1) return fail(SYSTEC_EINVAL, "systec_cp_step: not an order-3..5 tensor");
  int rc = check_factor_args("systec_cp_step", tn->dim, B, bdt, R, C);
  if (rc) return rc;
  if (R > 64) return fail(SYSTEC_EINVAL, "systec_cp_step: R must be at most 64");
  if (!B_new || !G || !fit) return fail(SYSTEC_EINVAL, "systec_cp_step: NULL pointer");
  return launch_cp_step(tn, B, bdt, R, C, B_new, G, fit, static_cast<hipStream_t>(stream));
}

int systec_ssymv_t(const systec_tensor* t, const void* x, systec_dtype xdt, float* y,
                   systec_stream stream) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_ssymv_t: NULL handle");
  if (t->impl->kind != 0) return fail(SYSTEC_EINVAL, "systec_ssymv_t: not a matrix");
  if (!valid_dtype(xdt)) return fail(SYSTEC_EINVAL, "systec_ssymv_t: unsupported dtype");
  if (!x || !y) return fail(SYSTEC_EINVAL, "systec_ssymv_t: NULL pointer");
  return launch_ssymv_panel(t->impl, x, xdt, y, static_cast<hipStream_t>(stream));
}

int systec_mttkrp_t_ex(const systec_tensor* t, const void* B, systec_dtype bdt, int64_t R,
                       float* C, systec_mttkrp_algo algo, systec_stream stream) {
  if (!t || !t->impl) return fail(SYSTEC_EINVAL, "systec_mttkrp_t: NULL handle");
  const Tensor* tn = t->impl;
  if (tn->kind != 1) return fail(SYSTEC_EINVAL, "systec_mttkrp_t: not an order-3..5 tensor");
  int rc = check_factor_args("systec_mttkrp_t", tn->dim, B, bdt, R, C);
  if (rc) return rc;
  if (algo < SYSTEC_MTTKRP_AUTO || algo > SYSTEC_MTTKRP_VIEWS)
    return fail(SYSTEC_EINVAL, "systec_mttkrp_t: unknown algorithm");
  auto s = static_cast<hipStream_t>(stream);
  if (algo == SYSTEC_MTTKRP_AUTO) {
    if (lds_preferred(tn->dim, bdt, R)) {
      rc = launch_mttkrp_views_lane(tn, B, bdt, R, C, s);
      if (rc != -1) return rc;  // else the tensor's runs are short: the views
    }
    algo = SYSTEC_MTTKRP_VIEWS;
  }
  if (algo == SYSTEC_MTTKRP_VIEWS) return launch_mttkrp_views(tn, B, bdt, R, C, s);
  if (algo == SYSTEC_MTTKRP_LDS) return launch_mttkrp_views_lds(tn, B, bdt, R, C, s);
  // the first view holds every entry in canonical order
  const int32_t* idx[5];
  for (int q = 0; q < tn->order; ++q) idx[q] = tn->vidx[0][q];
  return launch_mttkrp(tn->order, tn->dim, tn->nnz, idx, tn->vval[0], B, bdt, R, C, true, s);
}

int systec_mttkrp_t(const systec_tensor* t, const void* B, systec_dtype bdt, int64_t R,
                    float* C, systec_stream stream) {
  return systec_mttkrp_t_ex(t, B, bdt, R, C, SYSTEC_MTTKRP_AUTO, stream);
}

int systec_kernel_timing(int enable) {
  std::lock_guard<std::mutex> lock(g_timing_mu);
  g_timing = enable != 0;
  return SYSTEC_OK;
}

int systec_kernel_timing_read(double* total_ms, int64_t* launches) {
  if (!total_ms || !launches) return fail(SYSTEC_EINVAL, "systec_kernel_timing_read: NULL");
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    ev.swap(g_events);
  }
  double total = 0.0;
  int rc = SYSTEC_OK;
  for (auto& p : ev) {
    if (!rc) rc = check_hip(hipEventSynchronize(p.second), "hipEventSynchronize");
    float ms = 0.0f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, p.first, p.second), "hipEventElapsedTime");
    total += ms;
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  *total_ms = total;
  *launches = static_cast<int64_t>(ev.size());
  return rc;
}

}  // extern "C"
