// CPU tests of the serving scheduler core with a fake executor: admission by
// budget and slots, FIFO order, continuous batching, failure propagation,
// timeouts, shutdown, and the percentile arithmetic. Built with g++ (and
// with -fsanitize=thread) by tests/test_serve_cpu.py.
#include <atomic>
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "serve_core.h"

using namespace systec::serve;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// Completes steps in launch order, each `delay_us` after the previous one
// started; can fail one chosen step.
struct FakeExec {
  std::mutex mu;
  int64_t delay_us = 200;
  int64_t fail_step = -1;
  std::map<int64_t, int64_t> started;   // step -> start time (ns)
  std::vector<Plan> plans;              // copies for inspection
  std::set<std::pair<int64_t, size_t>> done_units;  // (request id, unit index)
  std::vector<std::vector<int64_t>> step_reqs;      // request ids with items per step
  uint64_t max_running_bytes = 0;
  int max_running = 0;
  std::map<int64_t, uint64_t> running_bytes;  // request id -> bytes (while running)

  uint64_t request_bytes(const TensorEntry& t, int, int64_t R) const {
    return static_cast<uint64_t>(t.dim) * (t.kind == 0 ? 1 : R) * 8;
  }
  int launch(const Plan& p, std::string* err) {
    std::lock_guard<std::mutex> lk(mu);
    plans.push_back(p);
    std::vector<int64_t> ids;
    for (auto& it : p.items) {
      CHECK(it.count >= 1);
      for (int64_t k = 0; k < it.count; ++k) {
        auto key = std::make_pair(it.req->id, static_cast<size_t>(it.unit0 + k));
        CHECK(done_units.insert(key).second);  // every unit runs exactly once
        ids.push_back(it.req->id);
      }
      running_bytes[it.req->id] = it.req->bytes;
    }
    for (auto* z : p.zero) running_bytes[z->id] = z->bytes;
    uint64_t b = 0;
    for (auto& kv : running_bytes) b += kv.second;
    max_running_bytes = std::max(max_running_bytes, b);
    max_running = std::max<int>(max_running, static_cast<int>(running_bytes.size()));
    step_reqs.push_back(ids);
    int64_t start = now_ns();
    if (!started.empty()) start = std::max(start, started.rbegin()->second + delay_us * 1000);
    started[p.step_id] = start;
    (void)err;
    return 0;
  }
  int query(int64_t step, std::string* err) {
    std::lock_guard<std::mutex> lk(mu);
    if (now_ns() < started[step] + delay_us * 1000) return 0;
    if (step == fail_step) {
      *err = "injected failure";
      return -1;
    }
    return 1;
  }
  int part_of(const TensorEntry& t) const { return t.kind; }
  int query_part(int64_t step, int, std::string* err) { return query(step, err); }
  void finished(int64_t req) {
    std::lock_guard<std::mutex> lk(mu);
    running_bytes.erase(req);
  }
  void release(TensorEntry&) {}
};

std::shared_ptr<TensorEntry> tensor(int kind, int64_t dim, int units, int64_t cost) {
  auto t = std::make_shared<TensorEntry>();
  t->kind = kind;
  t->order = kind == 0 ? 2 : 3;
  t->dim = dim;
  t->effective_nnz = units * cost;
  t->bytes = 1000;
  for (int u = 0; u < units; ++u) {
    Unit x;
    x.cost = cost;
    x.a = u;
    t->units.push_back(x);
  }
  return t;
}

void test_basic_all_units_once() {
  FakeExec ex;
  ex.delay_us = 100;
  Config c;
  c.budget_bytes = 1 << 30;
  c.step_work = 1000;
  Scheduler<FakeExec> s(c, ex);
  int64_t tid;
  std::string err;
  CHECK(s.register_tensor(tensor(1, 100, 25, 100), &tid, &err) == kOk);
  std::vector<int64_t> ids;
  for (int i = 0; i < 5; ++i) {
    int64_t r;
    CHECK(s.submit(tid, &ex, 0, 4, reinterpret_cast<float*>(&ex), 0, &r, &err) == kOk);
    ids.push_back(r);
  }
  for (auto r : ids) CHECK(s.wait(r, 5000000, &err) == kOk);
  Stats st = s.stats();
  CHECK(st.completed == 5 && st.failed == 0);
  CHECK(ex.done_units.size() == 5 * 25);
  CHECK(st.p50_us > 0 && st.p99_us >= st.p50_us && st.max_us >= st.p99_us);
  std::printf("PASS basic_all_units_once steps=%lld p50=%.0fus\n", (long long)st.steps, st.p50_us);
}

void test_budget_and_slots() {
  FakeExec ex;
  ex.delay_us = 300;
  Config c;
  c.budget_bytes = 1000 + 3 * 800;  // tensor + three requests of 800 bytes
  c.max_slots = 2;
  c.step_work = 300;
  Scheduler<FakeExec> s(c, ex);
  int64_t tid;
  std::string err;
  CHECK(s.register_tensor(tensor(0, 100, 6, 100), &tid, &err) == kOk);  // request: 100*8 = 800 B
  // a tensor whose single request can never fit
  int64_t big;
  auto tb = tensor(0, 100000, 1, 10);
  tb->bytes = 0;
  CHECK(s.register_tensor(tb, &big, &err) == kOk);
  int64_t r;
  CHECK(s.submit(big, &ex, 0, 1, nullptr, 0, &r, &err) == kEbudget);
  std::vector<int64_t> ids;
  std::atomic<bool> stop{false};
  int64_t max_running = 0;
  uint64_t max_bytes = 0;
  std::thread monitor([&] {
    while (!stop) {
      Stats st = s.stats();
      max_running = std::max(max_running, st.running);
      max_bytes = std::max(max_bytes, st.bytes_in_use);
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  });
  for (int i = 0; i < 8; ++i) {
    CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &r, &err) == kOk);
    ids.push_back(r);
  }
  for (auto q : ids) CHECK(s.wait(q, 10000000, &err) == kOk);
  stop = true;
  monitor.join();
  CHECK(max_running >= 1 && max_running <= 2);
  CHECK(max_bytes <= c.budget_bytes);
  Stats st = s.stats();
  CHECK(st.completed == 8 && st.rejected == 1);
  CHECK(st.bytes_in_use == 1000);
  std::printf("PASS budget_and_slots max_running=%lld\n", (long long)max_running);
}

void test_budget_blocks_then_resumes() {
  FakeExec ex;
  ex.delay_us = 500;
  Config c;
  c.budget_bytes = 1000 + 800;  // room for exactly one request at a time
  c.max_slots = 8;
  c.step_work = 1 << 20;
  Scheduler<FakeExec> s(c, ex);
  int64_t tid, r1, r2;
  std::string err;
  CHECK(s.register_tensor(tensor(0, 100, 4, 100), &tid, &err) == kOk);
  CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &r1, &err) == kOk);
  CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &r2, &err) == kOk);
  std::this_thread::sleep_for(std::chrono::microseconds(150));
  int st1, st2;
  CHECK(s.poll(r1, &st1) == kOk && s.poll(r2, &st2) == kOk);
  CHECK(st2 == kQueued);  // blocked by the budget while r1 runs
  CHECK(s.wait(r2, 10000000, &err) == kOk);
  CHECK(s.poll(r1, &st1) == kOk && st1 == kDone);
  std::printf("PASS budget_blocks_then_resumes\n");
}

void test_fifo_and_continuous_batching() {
  FakeExec ex;
  ex.delay_us = 2000;
  Config c;
  c.budget_bytes = 1 << 30;
  c.max_slots = 4;
  c.step_work = 200;  // two units per step in total
  Scheduler<FakeExec> s(c, ex);
  int64_t tid, a, b;
  std::string err;
  CHECK(s.register_tensor(tensor(1, 10, 10, 100), &tid, &err) == kOk);
  CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &a, &err) == kOk);
  std::this_thread::sleep_for(std::chrono::milliseconds(1));  // first step is running
  CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &b, &err) == kOk);
  CHECK(s.wait(a, 20000000, &err) == kOk && s.wait(b, 20000000, &err) == kOk);
  // b joined while a was still running: some step holds items of both
  bool shared = false;
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    for (auto& ids : ex.step_reqs) {
      bool ha = false, hb = false;
      for (auto q : ids) ha |= q == a, hb |= q == b;
      shared |= ha && hb;
    }
    // FIFO: a's first item precedes b's
    int first_a = -1, first_b = -1;
    for (size_t k = 0; k < ex.step_reqs.size(); ++k)
      for (auto q : ex.step_reqs[k]) {
        if (q == a && first_a < 0) first_a = static_cast<int>(k);
        if (q == b && first_b < 0) first_b = static_cast<int>(k);
      }
    CHECK(first_a >= 0 && first_b >= 0 && first_a <= first_b);
  }
  CHECK(shared);
  std::printf("PASS fifo_and_continuous_batching\n");
}

void test_failure_and_timeout() {
  FakeExec ex;
  ex.delay_us = 1000;
  ex.fail_step = 1;
  Config c;
  c.budget_bytes = 1 << 30;
  c.step_work = 100;  // one unit per step
  Scheduler<FakeExec> s(c, ex);
  int64_t tid, r;
  std::string err;
  CHECK(s.register_tensor(tensor(1, 10, 3, 100), &tid, &err) == kOk);
  CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &r, &err) == kOk);
  CHECK(s.wait(r, 10, &err) == kEtimeout);
  CHECK(s.wait(r, 20000000, &err) == kEdevice);
  CHECK(err.find("injected") != std::string::npos);
  int st;
  CHECK(s.poll(r, &st) == kOk && st == kFailed);
  // a later request still completes
  int64_t r2;
  CHECK(s.submit(tid, &ex, 0, 1, nullptr, 0, &r2, &err) == kOk);
  CHECK(s.wait(r2, 20000000, &err) == kOk);
  Stats stt = s.stats();
  CHECK(stt.failed == 1 && stt.completed == 1);
  CHECK(s.unregister_tensor(999, &err) == kEnotfound);
  std::printf("PASS failure_and_timeout\n");
}

void test_shutdown_cancels_queue() {
  FakeExec ex;
  ex.delay_us = 5000;
  Config c;
  c.budget_bytes = 1 << 30;
  c.max_slots = 1;
  c.step_work = 100;
  auto* s = new Scheduler<FakeExec>(c, ex);
  int64_t tid, r1, r2;
  std::string err;
  CHECK(s->register_tensor(tensor(1, 10, 2, 100), &tid, &err) == kOk);
  CHECK(s->submit(tid, &ex, 0, 1, nullptr, 0, &r1, &err) == kOk);
  CHECK(s->submit(tid, &ex, 0, 1, nullptr, 0, &r2, &err) == kOk);
  std::this_thread::sleep_for(std::chrono::milliseconds(1));
  CHECK(s->unregister_tensor(tid, &err) == kEbusy);
  s->shutdown();
  int st1, st2;
  CHECK(s->poll(r1, &st1) == kOk && s->poll(r2, &st2) == kOk);
  CHECK(st1 == kDone);    // running work is drained
  CHECK(st2 == kFailed);  // queued work is cancelled
  delete s;
  std::printf("PASS shutdown_cancels_queue\n");
}

void test_percentiles() {
  std::vector<double> v;
  for (int i = 1; i <= 100; ++i) v.push_back(i);
  CHECK(percentile_sorted(v, 50) == 50 && percentile_sorted(v, 99) == 99);
  CHECK(percentile_sorted(v, 100) == 100 && percentile_sorted(v, 0) == 1);
  std::vector<double> w = {3, 7, 9};
  CHECK(percentile_sorted(w, 50) == 7 && percentile_sorted(w, 99) == 9);
  std::printf("PASS percentiles\n");
}

void test_concurrent_submitters() {
  FakeExec ex;
  ex.delay_us = 50;
  Config c;
  c.budget_bytes = 1 << 30;
  c.max_slots = 8;
  c.step_work = 500;
  Scheduler<FakeExec> s(c, ex);
  int64_t tid;
  std::string err;
  CHECK(s.register_tensor(tensor(1, 10, 7, 100), &tid, &err) == kOk);
  std::atomic<int> ok{0};
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t)
    th.emplace_back([&] {
      for (int i = 0; i < 25; ++i) {
        int64_t r;
        std::string e;
        if (s.submit(tid, &ex, 0, 1, nullptr, 0, &r, &e) == kOk && s.wait(r, 20000000, &e) == kOk) ++ok;
      }
    });
  for (auto& t : th) t.join();
  CHECK(ok == 100);
  CHECK(ex.done_units.size() == 100 * 7);
  std::printf("PASS concurrent_submitters\n");
}


void test_every_running_request_progresses() {
  // a step budget smaller than one unit: each running request still gets a
  // unit in every step, so a small request that joins a long one finishes
  // first instead of waiting for the long one to drain
  FakeExec ex;
  ex.delay_us = 200;
  Config c;
  c.budget_bytes = 1 << 30;
  c.max_slots = 4;
  c.step_work = 1;
  Scheduler<FakeExec> s(c, ex);
  int64_t big_t, small_t, big, small;
  std::string err;
  CHECK(s.register_tensor(tensor(1, 10, 200, 100), &big_t, &err) == kOk);
  CHECK(s.register_tensor(tensor(1, 10, 3, 100), &small_t, &err) == kOk);
  CHECK(s.submit(big_t, &ex, 0, 1, nullptr, 0, &big, &err) == kOk);
  std::this_thread::sleep_for(std::chrono::milliseconds(2));
  CHECK(s.submit(small_t, &ex, 0, 1, nullptr, 0, &small, &err) == kOk);
  CHECK(s.wait(small, 20000000, &err) == kOk);
  int state = -1;
  CHECK(s.poll(big, &state) == kOk && state == kRunning);
  CHECK(s.wait(big, 20000000, &err) == kOk);
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    for (auto& ids : ex.step_reqs) {
      bool hb = false, hs = false;
      for (auto q : ids) hb |= q == big, hs |= q == small;
      CHECK(!hs || hb);  // the small request shared its steps with the big one
      CHECK(ids.size() <= 2);
    }
  }
  std::printf("PASS every_running_request_progresses\n");
}

// With min_step_work set, a lone request runs in short steps, and the step
// budget grows with the number of running requests up to step_work.
void test_step_budget_grows_with_load() {
  FakeExec ex;
  ex.delay_us = 50;
  Config c;
  c.budget_bytes = 1 << 30;
  c.max_slots = 5;
  c.step_work = 1000;
  c.min_step_work = 200;
  Scheduler<FakeExec> s(c, ex);
  int64_t tid;
  std::string err;
  CHECK(s.register_tensor(tensor(1, 100, 100, 10), &tid, &err) == kOk);
  int64_t r;
  CHECK(s.submit(tid, &ex, 0, 4, reinterpret_cast<float*>(&ex), 0, &r, &err) == kOk);
  CHECK(s.wait(r, 5000000, &err) == kOk);
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    // one running request: 200 entries (20 units) per step
    for (size_t k = 0; k + 1 < ex.step_reqs.size(); ++k) CHECK(ex.step_reqs[k].size() == 20);
    CHECK(ex.step_reqs.size() == 5);
    ex.step_reqs.clear();
  }
  // five at once: the first step has all five running, so its budget is
  // the full 1000 entries
  std::vector<int64_t> ids;
  for (int i = 0; i < 5; ++i) {
    CHECK(s.submit(tid, &ex, 0, 4, reinterpret_cast<float*>(&ex), 0, &r, &err) == kOk);
    ids.push_back(r);
  }
  for (auto q : ids) CHECK(s.wait(q, 5000000, &err) == kOk);
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    size_t most = 0;
    for (auto& v : ex.step_reqs) most = std::max(most, v.size());
    CHECK(most == 100);  // 1000 entries of 10-entry units
  }
  std::printf("PASS step_budget_grows_with_load\n");
}

int main() {
  test_percentiles();
  test_basic_all_units_once();
  test_budget_and_slots();
  test_budget_blocks_then_resumes();
  test_fifo_and_continuous_batching();
  test_every_running_request_progresses();
  test_failure_and_timeout();
  test_shutdown_cancels_queue();
  test_concurrent_submitters();
  test_step_budget_grows_with_load();
  std::printf("ALL PASS\n");
  return 0;
}
