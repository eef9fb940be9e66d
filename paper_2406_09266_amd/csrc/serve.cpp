// Serving runtime: the GPU executor behind the scheduler core (serve_core.h)
// and the systec_serve_* entry points.
//
// A step issues, on one stream per kernel kind (SSYMV; MTTKRP of order 3,
// 4, 5), a zero kernel for the outputs of the kind's newly admitted requests
// and then its step kernels (one per variant, one workgroup per work item;
// the requests and their unit ranges travel as kernel arguments), each
// stream closed by an event. A few steps are in flight (max_inflight), so
// the host builds the next step while others run. A request on a matrix
// stored with its vertices relabeled gets two stream-ordered scratch vectors
// at admission (its input in the stored order, and the output there, both
// filled by one permutation kernel in place of the zero kernel); the step
// that runs its last unit permutes the output back and frees them, before
// the step's event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "serve_core.h"

namespace systec {
namespace {

constexpr int kRing = 4;                   // step events (> steps in flight)
constexpr int64_t kViewUnit = 16 * 256;    // entries per MTTKRP work unit (4 tiles per wave)
constexpr int kSsymvUnitTiles = 64;        // panel tiles per SSYMV work unit

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

class GpuExecutor {
 public:
  int init(int device, bool one_stream, std::string* err) {
    device_ = device;
    hipError_t e = hipSetDevice(device);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      if (one_stream && k > 0) streams_[k] = streams_[0];
      else e = hipStreamCreateWithFlags(&streams_[k], hipStreamNonBlocking);
    }
    one_stream_ = one_stream;
    stream_ = streams_[0];
    if (e == hipSuccess && serve_init_kernels() != SYSTEC_OK) e = hipErrorInvalidValue;
    for (int i = 0; i < kRing && e == hipSuccess; ++i)
      for (int k = 0; k < 4 && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&ev_[i][k], hipEventDisableTiming);
    if (e != hipSuccess) {
      *err = std::string("serving executor init: ") + hipGetErrorString(e);
      return serve::kEdevice;
    }
    return serve::kOk;
  }

  ~GpuExecutor() {
    for (hipStream_t st : streams_)
      if (st) (void)hipStreamSynchronize(st);
    for (auto& kv : scratch_) {  // requests that failed before their last unit
      (void)hipFree(kv.second.xp);
      (void)hipFree(kv.second.yp);
    }
    for (auto& evs : ev_)
      for (hipEvent_t ev : evs)
        if (ev) (void)hipEventDestroy(ev);
    for (int k = 0; k < 4; ++k)
      if (streams_[k] && !(one_stream_ && k > 0)) (void)hipStreamDestroy(streams_[k]);
  }

  // Builds the device descriptor and the unit table of an operand being
  // registered (owned by the operand, freed with it).
  int prepare(Tensor* t, std::vector<serve::Unit>* units, std::string* err) {
    make_units(t, units);
    std::vector<ServeUnit> hu(std::max<size_t>(1, units->size()));
    for (size_t k = 0; k < units->size(); ++k)
      hu[k] = ServeUnit{(*units)[k].a, (*units)[k].b, (*units)[k].c, 0};
    ServeTensor d{};
    d.kind = t->kind;
    d.order = t->order;
    d.dim = static_cast<int32_t>(t->dim);
    d.H = t->panel_rows;
    if (t->kind == 0) {
      d.p[0][0] = t->pcol;
      d.p[0][1] = t->prow;
      d.p[0][2] = t->pval;
      d.p[0][3] = t->ppack;
      d.p[0][4] = t->pbase;
    } else {
      for (int v = 0; v < t->order; ++v) {
        for (int q = 0; q < t->order; ++q) d.p[v][q] = t->vidx[v][q];
        d.val[v] = t->vval[v];
      }
    }
    (void)hipSetDevice(device_);
    void *pu = nullptr, *pd = nullptr;
    hipError_t e = hipMalloc(&pu, hu.size() * sizeof(ServeUnit));
    if (e == hipSuccess) {
      t->allocations.push_back(pu);
      t->bytes += hu.size() * sizeof(ServeUnit);
      e = hipMalloc(&pd, sizeof(ServeTensor));
    }
    if (e == hipSuccess) {
      t->allocations.push_back(pd);
      t->bytes += sizeof(ServeTensor);
      d.units = static_cast<const ServeUnit*>(pu);
      e = hipMemcpy(pu, hu.data(), hu.size() * sizeof(ServeUnit), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(pd, &d, sizeof(ServeTensor), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      *err = std::string("serving registration: ") + hipGetErrorString(e);
      return serve::kEdevice;
    }
    t->d_units = static_cast<ServeUnit*>(pu);
    t->d_serve = static_cast<ServeTensor*>(pd);
    return serve::kOk;
  }

  uint64_t request_bytes(const serve::TensorEntry& t, int dtype, int64_t R) const {
    const uint64_t es = dtype == SYSTEC_BF16 ? 2 : 4;
    const uint64_t cols = t.kind == 0 ? 1 : static_cast<uint64_t>(R);
    const uint64_t b = static_cast<uint64_t>(t.dim) * cols * (es + 4);  // input + FP32 output
    return permuted(t) ? 2 * b : b;  // and their copies in the stored vertex order
  }

  int launch(const serve::Plan& plan, std::string* err) {
    (void)hipSetDevice(device_);
    const int slot = static_cast<int>(plan.step_id % kRing);
    // the slot's previous step has completed (fewer than kRing steps in flight)

    // each request's share of the step: a contiguous range of its units
    struct Share {
      const serve::Request* req;
      const Tensor* t;
      int32_t unit0, count;
    };
    // (a request taken in both passes of the fill has two adjacent ranges)
    std::vector<Share> shares;
    for (const serve::PlanItem& pi : plan.items) {
      const auto u0 = static_cast<int32_t>(pi.unit0);
      const auto n = static_cast<int32_t>(pi.count);
      auto it = std::find_if(shares.begin(), shares.end(),
                             [&](const Share& sh) { return sh.req == pi.req; });
      if (it == shares.end()) {
        shares.push_back(Share{pi.req, static_cast<const Tensor*>(pi.tensor->payload), u0, n});
      } else {
        it->unit0 = std::min(it->unit0, u0);
        it->count += n;
      }
    }

    int rc = SYSTEC_OK;
    {
      LaunchTimer timer(stream_);
      // one stream per kernel kind (SSYMV; MTTKRP of order 3, 4, 5): the
      // outputs of the kind's newly admitted requests are zeroed on that
      // stream, then its step kernel runs; the kinds overlap
      for (int g = 0; g < 4 && !rc; ++g) {
        hipStream_t st = streams_[g];
        auto kind_of = [](const Tensor* t) { return t->kind == 0 ? 0 : t->order - 2; };
        // outputs to zero, in batches of kStepReqs, before the kind's step
        // launches (the step kernels add into them)
        int launched = 0;
        ZeroArgs z{};
        for (size_t k = 0; k < plan.zero.size() && !rc; ++k) {
          const serve::Request* r = plan.zero[k];
          if (kind_of(static_cast<const Tensor*>(r->tensor->payload)) != g) continue;
          if (r->ready) {  // the caller's work on the request's buffers comes first
            rc = check_hip(hipStreamWaitEvent(st, static_cast<hipEvent_t>(r->ready.get()), 0),
                           "hipStreamWaitEvent(request ready)");
            r->ready.reset();
            if (rc) break;
          }
          if (permuted(*r->tensor)) {
            rc = begin_permuted(*r, st);
            ++launched;
            continue;
          }
          z.ptr[z.n] = r->out;
          z.count[z.n] = r->tensor->dim * (r->tensor->kind == 0 ? 1 : r->R);
          if (++z.n == kStepReqs) {
            rc = launch_serve_prologue(z, st);
            z = ZeroArgs{};
            ++launched;
          }
        }
        if (!rc && z.n) {
          rc = launch_serve_prologue(z, st);
          ++launched;
        }
        for (int v = 0; v < kStepVariants && !rc; ++v) {
          StepArgs a{};
          for (size_t k = 0; k < shares.size() && !rc; ++k) {
            const Share& sh = shares[k];
            if (kind_of(sh.t) != g) continue;
            if (g > 0 && step_variant(sh.req->dtype, sh.req->R, sh.req->in, sh.t->short_runs) != v)
              continue;
            if (g == 0 && v != 0) continue;
            StepReq& q = a.req[a.nreq++];
            q.t = sh.t->d_serve;
            q.in = sh.req->in;
            q.out = sh.req->out;
            const auto sc = scratch_.find(sh.req->id);
            if (sc != scratch_.end()) {  // relabeled matrix: the stored vertex order
              q.in = sc->second.xp;
              q.out = sc->second.yp;
            }
            q.unit0 = sh.unit0;
            q.item0 = a.nitems;
            q.R = static_cast<int32_t>(sh.req->R);
            q.dtype = sh.req->dtype;
            a.nitems += sh.count;
            if (a.nreq == kStepReqs) {
              rc = launch_serve_step(g == 0 ? 0 : g + 2, v, a, st);
              a = StepArgs{};
              ++launched;
            }
          }
          if (!rc && a.nreq) {
            rc = launch_serve_step(g == 0 ? 0 : g + 2, v, a, st);
            ++launched;
          }
        }
        // relabeled matrices whose last unit ran in this step: output back
        // in the caller's vertex order, scratch released (stream-ordered)
        for (size_t k = 0; g == 0 && k < shares.size() && !rc; ++k) {
          const Share& sh = shares[k];
          if (kind_of(sh.t) != 0) continue;
          const auto sc = scratch_.find(sh.req->id);
          if (sc == scratch_.end()) continue;
          if (static_cast<size_t>(sh.unit0) + sh.count != sh.req->tensor->units.size()) continue;
          rc = launch_permute_out(static_cast<int>(sh.t->dim), sh.t->inv, sc->second.yp,
                                  sh.req->out, st);
          const int rc2 = check_hip(hipFreeAsync(sc->second.xp, st), "hipFreeAsync");
          const int rc3 = check_hip(hipFreeAsync(sc->second.yp, st), "hipFreeAsync");
          scratch_.erase(sc);
          if (!rc) rc = rc2 ? rc2 : rc3;
          ++launched;
        }
        // a stream with no work this step records no event (queries of it
        // report done)
        used_[slot][g] = launched != 0;
        if (!rc && used_[slot][g]) rc = check_hip(hipEventRecord(ev_[slot][g], st), "hipEventRecord");
      }
    }
    if (rc) {
      *err = systec_last_error();
      return rc;
    }
    return serve::kOk;
  }

  // The stream (kernel kind) that runs an operand's work.
  int part_of(const serve::TensorEntry& t) const { return t.kind == 0 ? 0 : t.order - 2; }

  int query_part(int64_t step_id, int part, std::string* err) {
    if (!used_[step_id % kRing][part]) return 1;
    const hipError_t e = hipEventQuery(ev_[step_id % kRing][part]);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) {
      *err = std::string("serving step failed: ") + hipGetErrorString(e);
      return -1;
    }
    return 1;
  }

  int query(int64_t step_id, std::string* err) {
    const int slot = static_cast<int>(step_id % kRing);
    for (int g = 0; g < 4; ++g) {
      if (!used_[slot][g]) continue;
      const hipError_t e = hipEventQuery(ev_[slot][g]);
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
  // A matrix stored with its vertices relabeled and with work to run: its
  // requests compute in the stored order.
  static bool permuted(const serve::TensorEntry& t) {
    const Tensor* tt = static_cast<const Tensor*>(t.payload);
    return t.kind == 0 && tt && tt->relabeled && !t.units.empty();
  }

  // Scratch of a newly admitted request on a relabeled matrix, filled on st.
  int begin_permuted(const serve::Request& r, hipStream_t st) {
    const Tensor* t = static_cast<const Tensor*>(r.tensor->payload);
    const auto n = static_cast<size_t>(t->dim);
    const systec_dtype dt = r.dtype == SYSTEC_BF16 ? SYSTEC_BF16 : SYSTEC_F32;
    Scratch sc;
    int rc = check_hip(hipMallocAsync(&sc.xp, n * (dt == SYSTEC_BF16 ? 2 : 4), st),
                       "hipMallocAsync(serving scratch)");
    if (rc) return rc;
    rc = check_hip(hipMallocAsync(reinterpret_cast<void**>(&sc.yp), n * sizeof(float), st),
                   "hipMallocAsync(serving scratch)");
    if (rc) {
      (void)hipFreeAsync(sc.xp, st);
      return rc;
    }
    scratch_[r.id] = sc;
    return launch_permute_in(static_cast<int>(n), t->perm, r.in, dt, sc.xp, sc.yp, st);
  }

  struct Scratch {
    void* xp = nullptr;   // the input in the stored vertex order
    float* yp = nullptr;  // the output in the stored vertex order
  };
  std::unordered_map<int64_t, Scratch> scratch_;  // by request id

  int device_ = 0;
  hipStream_t streams_[4] = {nullptr, nullptr, nullptr, nullptr};  // per kernel kind
  hipStream_t stream_ = nullptr;                                   // streams_[0]
  bool one_stream_ = false;  // every kind on streams_[0], in order
  hipEvent_t ev_[kRing][4] = {};                                   // step done, per stream
  bool used_[kRing][4] = {};  // the step slot's stream had work (recorded its event)
};

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
  int rc = s->exec->init(cfg->device, cfg->streams == 1, &err);
  if (rc) {
    delete s;
    return serve_fail(rc, err);
  }
  serve::Config c;
  c.budget_bytes = cfg->budget_bytes;
  c.max_slots = cfg->max_slots;
  c.step_work = cfg->step_work_nnz;
  c.min_step_work = cfg->min_step_work_nnz;
  c.max_queue = cfg->max_queue > 0 ? cfg->max_queue : (1 << 20);
  c.max_inflight = std::min(kRing, cfg->max_inflight > 0 ? cfg->max_inflight : 2);
  s->sched.reset(new serve::Scheduler<GpuExecutor>(c, *s->exec));
  *out = s;
  return SYSTEC_OK;
}

int systec_serve_register(systec_server* s, systec_tensor* t, int64_t* tensor_id) {
  if (!s || !t || !t->impl || !tensor_id)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_register: NULL argument");
  auto e = std::make_shared<serve::TensorEntry>();
  std::string err;
  if (!t->impl->d_serve) {
    const int prc = s->exec->prepare(t->impl, &e->units, &err);
    if (prc) return serve_fail(prc, err);
  } else {
    make_units(t->impl, &e->units);
  }
  e->kind = t->impl->kind;
  e->order = t->impl->order;
  e->dim = t->impl->dim;
  e->effective_nnz = t->impl->effective_nnz;
  e->bytes = t->impl->bytes;
  e->payload = t->impl;
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

int systec_serve_submit_after(systec_server* s, int64_t tensor_id, const void* in,
                              systec_dtype dt, int64_t R, float* out, int64_t arrival_ns,
                              systec_stream after, int64_t* req_id) {
  if (!s || !in || !out || !req_id)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_submit_after: NULL argument");
  if (dt != SYSTEC_F32 && dt != SYSTEC_BF16)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_submit_after: unsupported dtype");
  if (R < 1 || R > 64)
    return serve_fail(SYSTEC_EINVAL, "systec_serve_submit_after: R must be in 1..64");
  // a marker after the work enqueued on `after` so far; the server's stream
  // waits for it before the request's first kernel
  hipEvent_t ev = nullptr;
  int rc = check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
  if (rc) return rc;
  std::shared_ptr<void> ready(ev, [](void* e) { (void)hipEventDestroy(static_cast<hipEvent_t>(e)); });
  rc = check_hip(hipEventRecord(ev, static_cast<hipStream_t>(after)), "hipEventRecord");
  if (rc) return rc;
  std::string err;
  rc = s->sched->submit(tensor_id, in, dt, R, out, arrival_ns, req_id, &err, std::move(ready));
  return rc ? serve_fail(rc, err) : SYSTEC_OK;
}

int systec_tensor_bytes(const systec_tensor* t, uint64_t* bytes) {
  if (!t || !t->impl || !bytes) return fail(SYSTEC_EINVAL, "systec_tensor_bytes: NULL argument");
  *bytes = t->impl->bytes;
  return SYSTEC_OK;
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
