// Serving runtime: the GPU executor behind the scheduler core (serve_core.h)
// and the systec_serve_* entry points.
//
// Each step copies its work items from a ring of pinned host buffers to the
// device, then issues one zero kernel for the outputs of newly admitted
// requests and the persistent step kernels (SSYMV items with the panel row
// sums in LDS on the first stream; MTTKRP items, one kernel per tensor
// order, each on a stream of its own), every stream closed by an event. Up to
// three steps are in flight, so the host builds the next step while others
// run.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "serve_core.h"

namespace systec {
namespace {

constexpr int kRing = 4;                   // step buffers (> steps in flight)
constexpr int kMaxItems = 1 << 16;         // work items per step
constexpr int kMaxZero = 1 << 16;          // output pieces to zero per step
constexpr int64_t kZeroPiece = 16384;      // floats per zeroed piece
constexpr int64_t kViewUnit = 64 * 256;    // entries per MTTKRP work unit
constexpr int kSsymvUnitTiles = 64;        // panel tiles per SSYMV work unit

class GpuExecutor {
 public:
  int init(int device, std::string* err) {
    device_ = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
      e = hipStreamCreateWithFlags(&mstream_[k], hipStreamNonBlocking);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    grid_ = std::max(1, cus) * 2;   // SSYMV: two 512-thread workgroups (64 KiB LDS each) per CU
    grid2_ = std::max(1, cus) * 8;  // MTTKRP: eight 256-thread workgroups per CU
    for (int i = 0; i < kRing && e == hipSuccess; ++i) {
      e = hipHostMalloc(reinterpret_cast<void**>(&h_items_[i]), kMaxItems * sizeof(ServeItem));
      if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&h_zero_[i]), kMaxZero * sizeof(ZeroSeg));
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_items_[i]), kMaxItems * sizeof(ServeItem));
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_zero_[i]), kMaxZero * sizeof(ZeroSeg));
      if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_counter_[i]), 4 * sizeof(int));
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming);
      for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&mev_[i][k], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&evz_[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      *err = std::string("serving executor init: ") + hipGetErrorString(e);
      return serve::kEdevice;
    }
    return serve::kOk;
  }

  ~GpuExecutor() {
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (hipStream_t ms : mstream_)
      if (ms) (void)hipStreamSynchronize(ms);
    for (int i = 0; i < kRing; ++i) {
      if (h_items_[i]) (void)hipHostFree(h_items_[i]);
      if (h_zero_[i]) (void)hipHostFree(h_zero_[i]);
      if (d_items_[i]) (void)hipFree(d_items_[i]);
      if (d_zero_[i]) (void)hipFree(d_zero_[i]);
      if (d_counter_[i]) (void)hipFree(d_counter_[i]);
      if (ev_[i]) (void)hipEventDestroy(ev_[i]);
      for (hipEvent_t me : mev_[i])
        if (me) (void)hipEventDestroy(me);
      if (evz_[i]) (void)hipEventDestroy(evz_[i]);
    }
    if (stream_) (void)hipStreamDestroy(stream_);
    for (hipStream_t ms : mstream_)
      if (ms) (void)hipStreamDestroy(ms);
  }

  uint64_t request_bytes(const serve::TensorEntry& t, int dtype, int64_t R) const {
    const uint64_t es = dtype == SYSTEC_BF16 ? 2 : 4;
    const uint64_t cols = t.kind == 0 ? 1 : static_cast<uint64_t>(R);
    return static_cast<uint64_t>(t.dim) * cols * (es + 4);  // input + FP32 output
  }

  int launch(const serve::Plan& plan, std::string* err) {
    size_t pieces = 0;
    for (const serve::Request* r : plan.zero)
      pieces += (r->tensor->dim * (r->tensor->kind == 0 ? 1 : r->R) + kZeroPiece - 1) / kZeroPiece;
    if (plan.items.size() > static_cast<size_t>(kMaxItems) || pieces > static_cast<size_t>(kMaxZero)) {
      *err = "serving step too large for the executor's buffers";
      return serve::kEinval;
    }
    (void)hipSetDevice(device_);
    const int slot = static_cast<int>(plan.step_id % kRing);
    // the slot's previous step has completed (fewer than kRing steps in flight)
    // items grouped by kernel: SSYMV, then MTTKRP of order 3, 4, 5
    std::vector<ServeItem> groups[4];
    for (size_t k = 0; k < plan.items.size(); ++k) {
      const serve::PlanItem& pi = plan.items[k];
      const Tensor* t = static_cast<const Tensor*>(pi.tensor->payload);
      const serve::Unit& u = *pi.unit;
      ServeItem it{};
      it.dtype = pi.req->dtype;
      it.order = t->order;
      it.dim = static_cast<int32_t>(t->dim);
      it.in = pi.req->in;
      it.out = pi.req->out;
      if (t->kind == 0) {
        it.kind = 0;
        it.H = t->panel_rows;
        it.panel = u.a;
        it.begin = u.b;
        it.end = u.c;
        it.p[0] = t->pcol;
        it.p[1] = t->prow;
        it.p[2] = t->pval;
        groups[0].push_back(it);
      } else {
        it.kind = 1;
        it.R = static_cast<int32_t>(pi.req->R);
        it.slot = u.a;
        it.begin = u.b;
        it.end = u.c;
        for (int q = 0; q < t->order; ++q) it.p[q] = t->vidx[u.a][q];
        it.val = t->vval[u.a];
        groups[t->order - 2].push_back(it);
      }
    }
    ServeItem* hi = h_items_[slot];
    int offs[4], cnt[4], total = 0;
    for (int g = 0; g < 4; ++g) {
      offs[g] = total;
      cnt[g] = static_cast<int>(groups[g].size());
      std::copy(groups[g].begin(), groups[g].end(), hi + total);
      total += cnt[g];
    }
    ZeroSeg* hz = h_zero_[slot];
    int nz = 0;
    for (const serve::Request* r : plan.zero) {
      const int64_t count = r->tensor->dim * (r->tensor->kind == 0 ? 1 : r->R);
      for (int64_t o = 0; o < count; o += kZeroPiece)
        hz[nz++] = ZeroSeg{r->out + o, std::min(kZeroPiece, count - o)};
    }
    hipError_t e = hipSuccess;
    if (total)
      e = hipMemcpyAsync(d_items_[slot], hi, total * sizeof(ServeItem), hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess && nz)
      e = hipMemcpyAsync(d_zero_[slot], hz, nz * sizeof(ZeroSeg), hipMemcpyHostToDevice, stream_);
    if (e != hipSuccess) {
      *err = std::string("serving step copy: ") + hipGetErrorString(e);
      return serve::kEdevice;
    }
    int rc;
    {
      LaunchTimer timer(stream_);
      // copies and zeroing on the first stream; everything else after them
      rc = launch_serve_zero(d_zero_[slot], nz, d_counter_[slot], stream_);
      if (!rc) rc = check_hip(hipEventRecord(evz_[slot], stream_), "hipEventRecord");
      // MTTKRP items of order 3, 4, 5 on their own streams, so that the
      // persistent kernels of a step overlap instead of draining one by one
      for (int g = 1; g < 4 && !rc; ++g) {
        hipStream_t ms = mstream_[g - 1];
        rc = check_hip(hipStreamWaitEvent(ms, evz_[slot], 0), "hipStreamWaitEvent");
        if (!rc)
          rc = launch_serve_items(g + 2, d_items_[slot] + offs[g], cnt[g], d_counter_[slot] + g,
                                  std::min(grid2_, std::max(1, cnt[g])), ms);
        if (!rc) rc = check_hip(hipEventRecord(mev_[slot][g - 1], ms), "hipEventRecord");
      }
      if (!rc)
        rc = launch_serve_items(0, d_items_[slot], cnt[0], d_counter_[slot],
                                std::min(grid_, std::max(1, cnt[0])), stream_);
    }
    if (rc) {
      *err = systec_last_error();
      return rc;
    }
    e = hipEventRecord(ev_[slot], stream_);
    if (e != hipSuccess) {
      *err = std::string("serving step event: ") + hipGetErrorString(e);
      return serve::kEdevice;
    }
    slot_step_[slot] = plan.step_id;
    return serve::kOk;
  }

  int query(int64_t step_id, std::string* err) {
    const int slot = static_cast<int>(step_id % kRing);
    for (hipEvent_t ev : {ev_[slot], mev_[slot][0], mev_[slot][1], mev_[slot][2]}) {
      const hipError_t e = hipEventQuery(ev);
      if (e == hipErrorNotReady) return 0;
      if (e != hipSuccess) {
        *err = std::string("serving step failed: ") + hipGetErrorString(e);
        return -1;
      }
    }
    return 1;
  }

  void release(serve::TensorEntry& t) {
    tensor_free(static_cast<Tensor*>(t.payload));
    t.payload = nullptr;
  }

  hipStream_t stream() const { return stream_; }

 private:
  int device_ = 0;
  int grid_ = 512, grid2_ = 2048;
  hipStream_t stream_ = nullptr;
  hipStream_t mstream_[3] = {nullptr, nullptr, nullptr};
  ServeItem* h_items_[kRing] = {};
  ZeroSeg* h_zero_[kRing] = {};
  ServeItem* d_items_[kRing] = {};
  ZeroSeg* d_zero_[kRing] = {};
  int* d_counter_[kRing] = {};
  hipEvent_t ev_[kRing] = {}, evz_[kRing] = {};
  hipEvent_t mev_[kRing][3] = {};
  int64_t slot_step_[kRing] = {-1, -1, -1, -1};
};

// Work units of a prepared operand: SSYMV chunks, MTTKRP view ranges.
void make_units(const Tensor* t, std::vector<serve::Unit>* units) {
  if (t->kind == 0) {
    // the prepared chunks, cut into pieces of at most kSsymvUnitTiles tiles
    for (int c = 0; c < t->nchunks; ++c)
      for (int b = t->h_chunk_tile_begin[c]; b < t->h_chunk_tile_end[c]; b += kSsymvUnitTiles) {
        serve::Unit u;
        u.a = t->h_chunk_panel[c];
        u.b = b;
        u.c = std::min(t->h_chunk_tile_end[c], b + kSsymvUnitTiles);
        u.cost = static_cast<int64_t>(u.c - u.b) * kPanelTile;
        units->push_back(u);
      }
  } else {
    for (int v = 0; v < t->order; ++v)
      for (int64_t e = 0; e < t->vnnz[v]; e += kViewUnit) {
        serve::Unit u;
        u.a = v;
        u.b = static_cast<int32_t>(e);
        u.c = static_cast<int32_t>(std::min<int64_t>(t->vnnz[v], e + kViewUnit));
        u.cost = u.c - u.b;
        units->push_back(u);
      }
  }
}

}  // namespace
}  // namespace systec

using namespace systec;

struct systec_server {
  std::unique_ptr<GpuExecutor> exec;
  std::unique_ptr<serve::Scheduler<GpuExecutor>> sched;
};

namespace {
int serve_fail(int rc, const std::string& msg) { return systec::fail(rc, msg); }
}  // namespace

extern "C" {

int systec_serve_create(const systec_serve_config* cfg, systec_server** out) {
  if (!cfg || !out) return serve_fail(SYSTEC_EINVAL, "systec_serve_create: NULL argument");
  if (cfg->budget_bytes == 0 || cfg->max_slots < 1 || cfg->step_work_nnz < 1)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_create: budget, slots and step work must be positive");
  auto* s = new systec_server();
  s->exec.reset(new GpuExecutor());
  std::string err;
  int rc = s->exec->init(cfg->device, &err);
  if (rc) {
    delete s;
    return serve_fail(rc, err);
  }
  serve::Config c;
  c.budget_bytes = cfg->budget_bytes;
  c.max_slots = cfg->max_slots;
  c.step_work = cfg->step_work_nnz;
  c.max_queue = cfg->max_queue > 0 ? cfg->max_queue : (1 << 20);
  c.max_inflight = 3;
  s->sched.reset(new serve::Scheduler<GpuExecutor>(c, *s->exec));
  *out = s;
  return SYSTEC_OK;
}

int systec_serve_register(systec_server* s, systec_tensor* t, int64_t* tensor_id) {
  if (!s || !t || !t->impl || !tensor_id)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_register: NULL argument");
  auto e = std::make_shared<serve::TensorEntry>();
  e->kind = t->impl->kind;
  e->order = t->impl->order;
  e->dim = t->impl->dim;
  e->effective_nnz = t->impl->effective_nnz;
  e->bytes = t->impl->bytes;
  e->payload = t->impl;
  make_units(t->impl, &e->units);
  std::string err;
  const int rc = s->sched->register_tensor(e, tensor_id, &err);
  if (rc) return serve_fail(rc, err);
  t->impl = nullptr;  // ownership moved to the server
  delete t;
  return SYSTEC_OK;
}

int systec_serve_unregister(systec_server* s, int64_t tensor_id) {
  if (!s) return serve_fail(SYSTEC_EINVAL, "systec_serve_unregister: NULL server");
  std::string err;
  const int rc = s->sched->unregister_tensor(tensor_id, &err);
  return rc ? serve_fail(rc, err) : SYSTEC_OK;
}

int systec_serve_submit(systec_server* s, int64_t tensor_id, const void* in, systec_dtype dt,
                        int64_t R, float* out, int64_t arrival_ns, int64_t* req_id) {
  if (!s || !in || !out || !req_id) return serve_fail(SYSTEC_EINVAL, "systec_serve_submit: NULL argument");
  if (dt != SYSTEC_F32 && dt != SYSTEC_BF16)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_submit: unsupported dtype");
  if (R < 1 || R > 64) return serve_fail(SYSTEC_EINVAL, "systec_serve_submit: R must be in 1..64");
  std::string err;
  const int rc = s->sched->submit(tensor_id, in, dt, R, out, arrival_ns, req_id, &err);
  return rc ? serve_fail(rc, err) : SYSTEC_OK;
}

int systec_serve_poll(systec_server* s, int64_t req_id, int* state) {
  if (!s || !state) return serve_fail(SYSTEC_EINVAL, "systec_serve_poll: NULL argument");
  const int rc = s->sched->poll(req_id, state);
  return rc ? serve_fail(rc, "systec_serve_poll: unknown request id") : SYSTEC_OK;
}

int systec_serve_wait(systec_server* s, int64_t req_id, int64_t timeout_us) {
  if (!s) return serve_fail(SYSTEC_EINVAL, "systec_serve_wait: NULL server");
  std::string err;
  const int rc = s->sched->wait(req_id, timeout_us, &err);
  return rc ? serve_fail(rc, err) : SYSTEC_OK;
}

int systec_serve_get_stats(systec_server* s, systec_serve_stats* out) {
  if (!s || !out) return serve_fail(SYSTEC_EINVAL, "systec_serve_get_stats: NULL argument");
  const serve::Stats st = s->sched->stats();
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->failed = st.failed;
  out->rejected = st.rejected;
  out->steps = st.steps;
  out->queued = st.queued;
  out->running = st.running;
  out->p50_us = st.p50_us;
  out->p99_us = st.p99_us;
  out->mean_us = st.mean_us;
  out->max_us = st.max_us;
  out->req_per_s = st.req_per_s;
  out->eff_nnz_per_s = st.eff_nnz_per_s;
  out->bytes_in_use = st.bytes_in_use;
  return SYSTEC_OK;
}

int systec_serve_reset_stats(systec_server* s) {
  if (!s) return serve_fail(SYSTEC_EINVAL, "systec_serve_reset_stats: NULL server");
  s->sched->reset_stats();
  return SYSTEC_OK;
}

int64_t systec_serve_now_ns(void) { return serve::now_ns(); }

int systec_serve_destroy(systec_server* s) {
  if (!s) return SYSTEC_OK;
  s->sched->shutdown();
  s->sched.reset();
  s->exec.reset();
  delete s;
  return SYSTEC_OK;
}

}  // extern "C"
