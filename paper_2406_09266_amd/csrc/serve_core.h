// Serving core: admission, continuous batching into steps, retirement and
// latency accounting. Free of HIP so that it can be driven by a fake
// executor in CPU tests; the GPU executor lives in serve.cpp.
//
// Model. Tensors are registered once and stay resident; their bytes count
// against the memory budget for as long as they are registered. A request
// names a tensor, an input (x or B) and an output (y or C); its input and
// output bytes are charged when it is admitted and released when it retires.
// Requests are admitted in arrival order (FIFO, no overtaking) while a slot
// is free and the budget allows; a request that could never fit returns
// SYSTEC_EBUDGET at submit. Each step takes work units (chunks of the
// prepared operand) from the admitted requests, up to a work budget in
// entries (every running request gets at least one unit, then half of the
// budget is shared round-robin and the rest goes in admission order), and
// hands them to the executor as one launch; requests admitted while a step
// runs join the next one (continuous batching). The executor runs a step in
// parts (the GPU executor: one stream per kernel kind), each in order across
// steps; a request retires as soon as the part that runs its work has
// completed the step holding its last unit, and its latency runs from its
// arrival to that moment, queueing included.
//
// Executor interface: request_bytes(tensor, dtype, R), part_of(tensor) in
// [0, 8), launch(plan, err), query(step, err) and query_part(step, part, err)
// (1 done, 0 running, -1 failed), release(tensor).
#pragma once

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include <sys/prctl.h>

namespace systec {
namespace serve {

enum Status { kOk = 0, kEinval = 1, kEnomem = 3, kEbudget = 4, kEbusy = 5, kEtimeout = 6,
              kEnotfound = 7, kEdevice = 8 };
enum State { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Nearest-rank percentile of an ascending, nonempty sample: the smallest
// value with at least p percent of the sample at or below it.
inline double percentile_sorted(const std::vector<double>& v, double p) {
  size_t k = static_cast<size_t>(std::ceil(p / 100.0 * static_cast<double>(v.size())));
  k = std::max<size_t>(1, std::min(k, v.size()));
  return v[k - 1];
}

struct Config {
  uint64_t budget_bytes = 0;
  int max_slots = 16;
  int64_t step_work = 1 << 24;  // entries per step (at most)
  // Entries per step with few running requests: the budget grows linearly
  // from min_step_work (one running request) to step_work (max_slots
  // running). Short steps while the device has room keep a newly arrived
  // request from waiting behind a long step; full steps under load keep the
  // per-step costs small. <= 0: always step_work.
  int64_t min_step_work = 0;
  int max_queue = 1 << 20;
  int max_inflight = 3;         // steps in flight (build step s+1 while s runs)
};

// One schedulable piece of a registered tensor (opaque to the core).
struct Unit {
  int64_t cost = 0;  // entries
  int32_t a = 0, b = 0, c = 0, d = 0;
};

struct TensorEntry {
  int64_t id = 0;
  int kind = 0;  // 0 matrix, 1 tensor
  int order = 0;
  int64_t dim = 0;
  int64_t effective_nnz = 0;
  uint64_t bytes = 0;
  std::vector<Unit> units;
  std::vector<int64_t> unit_prefix;  // unit_prefix[k] = cost of units [0, k)
  void* payload = nullptr;           // executor-owned
};

struct Request {
  int64_t id = 0;
  std::shared_ptr<TensorEntry> tensor;
  const void* in = nullptr;
  float* out = nullptr;
  int dtype = 0;
  int64_t R = 1;
  uint64_t bytes = 0;
  int state = kQueued;
  int64_t arrival_ns = 0, admit_ns = 0, done_ns = 0;
  size_t next_unit = 0;
  int64_t last_step = -1;
  int part = 0;  // the executor part (stream) that runs this request's work
  std::string error;
  // Executor-owned marker of the caller's work that must finish before the
  // request's own work starts (its input written, its output free); the
  // executor takes it when it first schedules the request's work.
  mutable std::shared_ptr<void> ready;
};

// Units [unit0, unit0 + count) of a request's operand, run in one step.
struct PlanItem {
  const TensorEntry* tensor;
  const Request* req;
  int64_t unit0, count;
};

struct Plan {
  int64_t step_id = 0;
  std::vector<const Request*> zero;  // newly admitted: zero their outputs first
  std::vector<PlanItem> items;
};

struct Stats {
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, steps = 0;
  double p50_us = 0, p99_us = 0, mean_us = 0, max_us = 0, req_per_s = 0, eff_nnz_per_s = 0;
  uint64_t bytes_in_use = 0;
  int64_t queued = 0, running = 0;
};

// Exec provides:
//   uint64_t request_bytes(const TensorEntry&, int dtype, int64_t R)
//   int launch(const Plan&, std::string* err)        0 or a Status
//   int query(int64_t step_id, std::string* err)     0 running, 1 done, <0 failed
//   void release(TensorEntry&)                        frees the payload
template <class Exec>
class Scheduler {
 public:
  Scheduler(const Config& cfg, Exec& exec) : cfg_(cfg), exec_(exec) {
    thread_ = std::thread([this] {
      // The loop's timed waits are short; the default 50 us timer slack of a
      // Linux thread would stretch each of them.
      prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
      loop();
    });
  }
  ~Scheduler() { shutdown(); }

  int register_tensor(std::shared_ptr<TensorEntry> t, int64_t* id, std::string* err) {
    std::lock_guard<std::mutex> lk(mu_);
    if (bytes_in_use_ + t->bytes > cfg_.budget_bytes) {
      *err = "registering the tensor would exceed the memory budget";
      return kEbudget;
    }
    t->unit_prefix.assign(t->units.size() + 1, 0);
    for (size_t k = 0; k < t->units.size(); ++k)
      t->unit_prefix[k + 1] = t->unit_prefix[k] + std::max<int64_t>(1, t->units[k].cost);
    t->id = next_tensor_id_++;
    bytes_in_use_ += t->bytes;
    tensors_[t->id] = t;
    *id = t->id;
    return kOk;
  }

  int unregister_tensor(int64_t id, std::string* err) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tensors_.find(id);
    if (it == tensors_.end()) {
      *err = "unknown tensor id";
      return kEnotfound;
    }
    if (it->second.use_count() > 1) {
      *err = "tensor has requests in flight";
      return kEbusy;
    }
    bytes_in_use_ -= it->second->bytes;
    exec_.release(*it->second);
    tensors_.erase(it);
    return kOk;
  }

  int submit(int64_t tensor_id, const void* in, int dtype, int64_t R, float* out,
             int64_t arrival_ns, int64_t* req_id, std::string* err,
             std::shared_ptr<void> ready = nullptr) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tensors_.find(tensor_id);
    if (it == tensors_.end()) {
      *err = "unknown tensor id";
      return kEnotfound;
    }
    if (stop_) {
      *err = "server is shutting down";
      return kEinval;
    }
    const uint64_t b = exec_.request_bytes(*it->second, dtype, R);
    if (registered_bytes_locked() + b > cfg_.budget_bytes) {
      ++rejected_;
      *err = "request can never fit the memory budget";
      return kEbudget;
    }
    if (static_cast<int>(queue_.size()) >= cfg_.max_queue) {
      *err = "queue full";
      return kEbusy;
    }
    auto r = std::make_shared<Request>();
    r->id = next_req_id_++;
    r->tensor = it->second;
    r->in = in;
    r->out = out;
    r->dtype = dtype;
    r->R = R;
    r->bytes = b;
    r->arrival_ns = arrival_ns > 0 ? arrival_ns : now_ns();
    r->ready = std::move(ready);
    requests_[r->id] = r;
    queue_.push_back(r);
    ++submitted_;
    if (first_arrival_ns_ == 0 || r->arrival_ns < first_arrival_ns_) first_arrival_ns_ = r->arrival_ns;
    *req_id = r->id;
    lk.unlock();
    wake_.notify_all();
    return kOk;
  }

  int poll(int64_t req_id, int* state) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = requests_.find(req_id);
    if (it == requests_.end()) return kEnotfound;
    *state = it->second->state;
    return kOk;
  }

  // Waits until the request is done or failed; timeout_us < 0 waits forever.
  int wait(int64_t req_id, int64_t timeout_us, std::string* err) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = requests_.find(req_id);
    if (it == requests_.end()) {
      *err = "unknown request id";
      return kEnotfound;
    }
    auto r = it->second;
    auto done = [&] { return r->state == kDone || r->state == kFailed; };
    if (timeout_us < 0) {
      done_cv_.wait(lk, done);
    } else if (!done_cv_.wait_until(lk, deadline(std::chrono::microseconds(timeout_us)), done)) {
      *err = "timed out";
      return kEtimeout;
    }
    if (r->state == kFailed) {
      *err = r->error;
      return kEdevice;
    }
    return kOk;
  }

  Stats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    Stats s;
    s.submitted = submitted_;
    s.completed = static_cast<int64_t>(latencies_us_.size());
    s.failed = failed_;
    s.rejected = rejected_;
    s.steps = steps_;
    s.bytes_in_use = bytes_in_use_;
    s.queued = static_cast<int64_t>(queue_.size());
    s.running = static_cast<int64_t>(active_.size());
    if (!latencies_us_.empty()) {
      std::vector<double> v = latencies_us_;
      std::sort(v.begin(), v.end());
      s.p50_us = percentile_sorted(v, 50);
      s.p99_us = percentile_sorted(v, 99);
      s.max_us = v.back();
      double sum = 0;
      for (double x : v) sum += x;
      s.mean_us = sum / v.size();
      const double span_s = (last_done_ns_ - first_arrival_ns_) * 1e-9;
      if (span_s > 0) {
        s.req_per_s = v.size() / span_s;
        s.eff_nnz_per_s = static_cast<double>(done_eff_nnz_) / span_s;
      }
    }
    return s;
  }

  void reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    latencies_us_.clear();
    failed_ = rejected_ = 0;
    submitted_ = static_cast<int64_t>(queue_.size() + active_.size());
    done_eff_nnz_ = 0;
    first_arrival_ns_ = 0;
    last_done_ns_ = 0;
    for (auto& r : queue_) first_arrival_ns_ = first_arrival_ns_ ? std::min(first_arrival_ns_, r->arrival_ns) : r->arrival_ns;
  }

  // Stops admitting, fails queued requests, drains running ones.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_ && !thread_.joinable()) return;
      stop_ = true;
      for (auto& r : queue_) {
        r->state = kFailed;
        r->error = "cancelled: server destroyed";
        ++failed_;
      }
      queue_.clear();
    }
    wake_.notify_all();
    done_cv_.notify_all();
    if (thread_.joinable()) thread_.join();
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : tensors_) exec_.release(*kv.second);
    tensors_.clear();
  }

 private:
  // Timed waits use system_clock deadlines (pthread_cond_timedwait), which
  // thread sanitizers understand; the latency clock stays steady_clock.
  template <class D>
  static std::chrono::system_clock::time_point deadline(D d) {
    return std::chrono::system_clock::now() + d;
  }

  static constexpr int kParts = 8;  // executor parts (Exec::part_of returns 0..7)

  struct InFlight {
    int64_t step_id;
    std::vector<std::shared_ptr<Request>> reqs;  // every request with an item in the step
  };

  uint64_t registered_bytes_locked() const {
    uint64_t b = 0;
    for (auto& kv : tensors_) b += kv.second->bytes;
    return b;
  }

  void admit_locked(Plan& plan) {
    while (!queue_.empty() && static_cast<int>(active_.size()) < cfg_.max_slots) {
      auto& r = queue_.front();
      if (bytes_in_use_ + r->bytes > cfg_.budget_bytes) break;  // FIFO: the head waits
      bytes_in_use_ += r->bytes;
      r->part = exec_.part_of(*r->tensor);
      r->state = kRunning;
      r->admit_ns = now_ns();
      plan.zero.push_back(r.get());
      active_.push_back(r);
      queue_.pop_front();
    }
  }

  // Fills a step. Half of the work budget is shared round-robin among the
  // running requests (a small request finishes within its share, so it is
  // not stuck behind large ones); the rest goes to the running requests in
  // admission order (a large request keeps most of the device, as it would
  // alone). Every running request with work left gets at least one unit.
  int64_t step_budget_locked() const {
    if (cfg_.min_step_work <= 0 || cfg_.min_step_work >= cfg_.step_work) return cfg_.step_work;
    const int64_t live = static_cast<int64_t>(active_.size());
    const int64_t slots = std::max(1, cfg_.max_slots);
    const int64_t span = cfg_.step_work - cfg_.min_step_work;
    return cfg_.min_step_work + span * std::min<int64_t>(std::max<int64_t>(live - 1, 0), slots - 1) /
                                    std::max<int64_t>(slots - 1, 1);
  }

  void fill_locked(Plan& plan, std::vector<std::shared_ptr<Request>>& touched) {
    const int64_t step_work = step_budget_locked();
    int64_t budget = step_work;
    // Takes the request's next units up to `limit` entries (and the step's
    // remaining budget), the unit that crosses the limit included; with
    // at_least_one, one unit even when the budget is spent.
    auto take = [&](const std::shared_ptr<Request>& r, int64_t limit, bool at_least_one) {
      const auto& pre = r->tensor->unit_prefix;
      const size_t n = r->tensor->units.size();
      const size_t first = r->next_unit;
      if (first < n) {
        const int64_t lim = std::min(limit, budget);
        size_t end = first;
        if (lim > 0)
          end = static_cast<size_t>(
              std::lower_bound(pre.begin() + first + 1, pre.end(), pre[first] + lim) - pre.begin());
        if (at_least_one) end = std::max(end, first + 1);
        end = std::min(end, n);
        if (end > first) {
          plan.items.push_back(PlanItem{r->tensor.get(), r.get(), static_cast<int64_t>(first),
                                        static_cast<int64_t>(end - first)});
          budget -= pre[end] - pre[first];
          r->next_unit = end;
          if (std::find(touched.begin(), touched.end(), r) == touched.end()) touched.push_back(r);
        }
      }
      if (r->next_unit == n && r->last_step < 0) {
        r->last_step = plan.step_id;
        if (std::find(touched.begin(), touched.end(), r) == touched.end()) touched.push_back(r);
      }
    };
    const int64_t live = std::max<int64_t>(1, static_cast<int64_t>(active_.size()));
    const int64_t share = std::max<int64_t>(1, step_work / (2 * live));
    for (auto& r : active_) take(r, share, true);
    for (auto& r : active_) {
      if (budget <= 0) break;
      take(r, budget, false);
    }
    // requests whose operand has no units at all finish with this step
    for (auto& r : active_)
      if (r->tensor->units.empty() && r->last_step < 0) {
        r->last_step = plan.step_id;
        if (std::find(touched.begin(), touched.end(), r) == touched.end()) touched.push_back(r);
      }
  }

  void retire_one_locked(const std::shared_ptr<Request>& r, bool ok, const std::string& err,
                         int64_t t) {
    if (!ok) {
      r->state = kFailed;
      r->error = err;
      ++failed_;
    } else {
      r->state = kDone;
      r->done_ns = t;
      latencies_us_.push_back((t - r->arrival_ns) * 1e-3);
      done_eff_nnz_ += r->tensor->effective_nnz;
      last_done_ns_ = std::max(last_done_ns_, t);
    }
    bytes_in_use_ -= r->bytes;
    r->tensor.reset();  // drop the reference: the request no longer pins the tensor
    active_.erase(std::remove(active_.begin(), active_.end(), r), active_.end());
  }

  void retire_locked(const InFlight& f, bool ok, const std::string& err) {
    const int64_t t = now_ns();
    for (auto& r : f.reqs) {
      if (r->state != kRunning) continue;
      if (ok && r->last_step != f.step_id) continue;
      retire_one_locked(r, ok, err, t);
    }
  }

  // Retires the requests whose last step has completed on their own part of
  // the executor (a request does not wait for the other parts' work of its
  // step, nor for earlier steps of other parts). Returns whether any retired.
  bool retire_parts_locked(std::unique_lock<std::mutex>& lk) {
    bool retired = false;
    for (auto& f : inflight_) {
      int state[kParts];
      std::string errs[kParts];
      std::fill(state, state + kParts, -2);  // not queried yet
      for (auto& r : f.reqs) {
        if (r->state != kRunning || r->last_step != f.step_id) continue;
        const int part = r->part;
        if (state[part] == -2) {
          lk.unlock();
          state[part] = exec_.query_part(f.step_id, part, &errs[part]);
          lk.lock();
        }
        if (state[part] != 0) {
          retire_one_locked(r, state[part] > 0, errs[part], now_ns());
          retired = true;
        }
      }
    }
    return retired;
  }

  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    int64_t step_id = 0;
    while (true) {
      if (stop_ && queue_.empty() && active_.empty() && inflight_.empty()) break;
      // 1. build and launch a step if a slot in the pipeline is free
      if (static_cast<int>(inflight_.size()) < cfg_.max_inflight) {
        Plan plan;
        plan.step_id = step_id;
        admit_locked(plan);
        std::vector<std::shared_ptr<Request>> touched;
        fill_locked(plan, touched);
        if (!plan.items.empty() || !plan.zero.empty() || !touched.empty()) {
          ++step_id;
          ++steps_;
          std::string err;
          lk.unlock();
          const int rc = exec_.launch(plan, &err);
          lk.lock();
          InFlight f{plan.step_id, touched};
          for (const Request* z : plan.zero) {
            auto it = requests_.find(z->id);
            if (it != requests_.end() &&
                std::find(f.reqs.begin(), f.reqs.end(), it->second) == f.reqs.end())
              f.reqs.push_back(it->second);
          }
          if (rc != 0) {
            retire_locked(f, false, err);
            done_cv_.notify_all();
          } else {
            inflight_.push_back(std::move(f));
          }
          continue;
        }
      }
      // 2. retire requests done on their own part, then completed steps in order
      bool retired = retire_parts_locked(lk);
      while (!inflight_.empty()) {
        std::string err;
        lk.unlock();
        const int q = exec_.query(inflight_.front().step_id, &err);
        lk.lock();
        if (q == 0) break;
        retire_locked(inflight_.front(), q > 0, err);
        inflight_.pop_front();
        retired = true;
      }
      if (retired) {
        done_cv_.notify_all();
        continue;
      }
      // 3. nothing to do right now. With steps in flight the loop polls
      // their events without sleeping (a completed request is noticed within
      // microseconds; this thread occupies one host core while the device
      // works); idle, it sleeps until a submit wakes it.
      if (!inflight_.empty()) {
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else if (queue_.empty() || static_cast<int>(active_.size()) >= cfg_.max_slots ||
                 bytes_in_use_ + queue_.front()->bytes > cfg_.budget_bytes) {
        if (stop_ && queue_.empty() && active_.empty()) continue;
        wake_.wait_until(lk, deadline(std::chrono::milliseconds(5)));
      }
    }
  }

  Config cfg_;
  Exec& exec_;
  std::mutex mu_;
  std::condition_variable wake_, done_cv_;
  std::thread thread_;
  bool stop_ = false;
  int64_t next_tensor_id_ = 1, next_req_id_ = 1;
  std::map<int64_t, std::shared_ptr<TensorEntry>> tensors_;
  std::map<int64_t, std::shared_ptr<Request>> requests_;
  std::deque<std::shared_ptr<Request>> queue_;
  std::vector<std::shared_ptr<Request>> active_;
  std::deque<InFlight> inflight_;
  uint64_t bytes_in_use_ = 0;
  int64_t submitted_ = 0, failed_ = 0, rejected_ = 0, steps_ = 0;
  std::vector<double> latencies_us_;
  int64_t done_eff_nnz_ = 0, first_arrival_ns_ = 0, last_done_ns_ = 0;
};

}  // namespace serve
}  // namespace systec
