// Host-only checks of the continuous-batching scheduler with a mock executor
// (no device): admission never exceeds the budget, FIFO start order, slots
// overlap, BUSY / NOMEM / NOTFOUND, failure propagation, drain on shutdown.
#include <atomic>
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "serve_core.hpp"

using namespace litho;
using namespace litho::serve;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

struct MockReq {
  double duration_us;
  bool fail_launch = false;
  bool fail_device = false;
  int value = 0;
  int result = -1;
};

class MockExecutor : public Executor {
 public:
  explicit MockExecutor(int n) : start_(size_t(n), 0.0), dur_(size_t(n), 0.0), req_(size_t(n), nullptr) {}
  int slots() const override { return int(start_.size()); }
  int launch(Job &job, int s) override {
    auto *r = static_cast<MockReq *>(job.payload.get());
    std::lock_guard<std::mutex> lk(mu);
    starts.push_back(job.ticket);
    size_t live = 0;
    for (auto *q : req_) live += q ? 1 : 0;
    max_concurrent = std::max(max_concurrent, live + 1);
    if (r->fail_launch) {
      job.error = "injected launch failure";
      return LITHO_E_HIP;
    }
    start_[size_t(s)] = now_us();
    dur_[size_t(s)] = r->duration_us;
    req_[size_t(s)] = r;
    return LITHO_OK;
  }
  bool ready(int s) override {
    std::lock_guard<std::mutex> lk(mu);
    return now_us() >= start_[size_t(s)] + dur_[size_t(s)];
  }
  int collect(Job &job, int s) override {
    std::lock_guard<std::mutex> lk(mu);
    MockReq *r = req_[size_t(s)];
    req_[size_t(s)] = nullptr;
    if (r->fail_device) {
      job.error = "injected device failure";
      return LITHO_E_HIP;
    }
    r->result = r->value * 2;
    return LITHO_OK;
  }
  mutable std::mutex mu;
  std::vector<uint64_t> starts;
  size_t max_concurrent = 0;

 private:
  std::vector<double> start_, dur_;
  std::vector<MockReq *> req_;
};

// An executor whose slots keep buffers sized for the largest request they
// ran (like device arenas) until the scheduler trims them.
class KeepingExecutor : public MockExecutor {
 public:
  explicit KeepingExecutor(int n) : MockExecutor(n), kept_(size_t(n), 0) {}
  int launch(Job &job, int s) override {
    {
      std::lock_guard<std::mutex> lk(mu);
      if (kept_[size_t(s)] < job.footprint) kept_[size_t(s)] = job.footprint;
      size_t total = 0;
      for (size_t k : kept_) total += k;
      max_kept_total = std::max(max_kept_total, total);
    }
    return MockExecutor::launch(job, s);
  }
  size_t held(int s) const override {
    std::lock_guard<std::mutex> lk(mu);
    return kept_[size_t(s)];
  }
  void trim(int s) override {
    std::lock_guard<std::mutex> lk(mu);
    kept_[size_t(s)] = 0;
    ++trims;
  }
  size_t max_kept_total = 0;
  int trims = 0;

 private:
  std::vector<size_t> kept_;
};

static std::shared_ptr<Job> make_job(size_t fp, double dur, int value, bool fl = false, bool fd = false) {
  auto j = std::make_shared<Job>();
  j->footprint = fp;
  auto r = std::make_shared<MockReq>();
  r->duration_us = dur;
  r->value = value;
  r->fail_launch = fl;
  r->fail_device = fd;
  j->payload = r;
  return j;
}

int main() {
  // 1. budget, FIFO, overlap
  {
    MockExecutor ex(4);
    const size_t budget = 100;
    std::map<uint64_t, std::shared_ptr<Job>> sent;
    size_t peak = 0;
    {
      Scheduler sch(&ex, budget, 1000);
      for (int i = 0; i < 60; ++i) {
        const size_t fp = 10 + size_t((i * 37) % 50);  // 10..59
        auto j = make_job(fp, 200 + (i % 7) * 100, i);
        uint64_t t = 0;
        CHECK(sch.submit(j, &t) == LITHO_OK);
        sent[t] = j;
      }
      for (auto &kv : sent) {
        std::shared_ptr<Job> out;
        CHECK(sch.wait(kv.first, -1, &out) == LITHO_OK);
        CHECK(out->status == LITHO_OK);
        auto *r = static_cast<MockReq *>(out->payload.get());
        CHECK(r->result == r->value * 2);
        CHECK(out->t_submit <= out->t_start && out->t_start <= out->t_done);
        std::shared_ptr<Job> again;
        CHECK(sch.wait(kv.first, 0, &again) == LITHO_E_NOTFOUND);
      }
      peak = sch.peak_in_use();
      CHECK(sch.in_use() == 0);
    }
    CHECK(peak <= budget);
    CHECK(ex.max_concurrent >= 2);  // requests overlapped
    for (size_t i = 1; i < ex.starts.size(); ++i) CHECK(ex.starts[i] > ex.starts[i - 1]);  // FIFO
    std::printf("budget/fifo ok: peak %zu of %zu, max concurrent %zu\n", peak, budget, ex.max_concurrent);
  }
  // 2. oversize, queue full, unknown ticket, pending poll
  {
    MockExecutor ex(1);
    Scheduler sch(&ex, 50, 3);
    uint64_t t;
    CHECK(sch.submit(make_job(51, 10, 0), &t) == LITHO_E_NOMEM);
    std::vector<uint64_t> ts;
    int busy = 0;
    for (int i = 0; i < 8; ++i) {
      const int rc = sch.submit(make_job(40, 20000, i), &t);
      if (rc == LITHO_OK)
        ts.push_back(t);
      else {
        CHECK(rc == LITHO_E_BUSY);
        ++busy;
      }
    }
    CHECK(busy > 0);
    std::shared_ptr<Job> out;
    CHECK(sch.wait(ts.back(), 0, &out) == LITHO_PENDING);
    CHECK(sch.wait(123456789, 0, &out) == LITHO_E_NOTFOUND);
    for (auto x : ts) CHECK(sch.wait(x, -1, &out) == LITHO_OK);
    std::printf("nomem/busy/notfound ok (%d busy)\n", busy);
  }
  // 3. injected failures surface on poll; the server keeps running
  {
    MockExecutor ex(2);
    Scheduler sch(&ex, 100, 100);
    uint64_t a, b, c;
    CHECK(sch.submit(make_job(10, 100, 1, true, false), &a) == LITHO_OK);
    CHECK(sch.submit(make_job(10, 100, 2, false, true), &b) == LITHO_OK);
    CHECK(sch.submit(make_job(10, 100, 3), &c) == LITHO_OK);
    std::shared_ptr<Job> out;
    CHECK(sch.wait(a, -1, &out) == LITHO_OK && out->status == LITHO_E_HIP && out->error.find("launch") != std::string::npos);
    CHECK(sch.wait(b, -1, &out) == LITHO_OK && out->status == LITHO_E_HIP && out->error.find("device") != std::string::npos);
    CHECK(sch.wait(c, -1, &out) == LITHO_OK && out->status == LITHO_OK);
    CHECK(sch.in_use() == 0);
    std::printf("failure propagation ok\n");
  }
  // 4. shutdown drains queued work
  {
    MockExecutor ex(2);
    std::vector<std::shared_ptr<Job>> jobs;
    {
      Scheduler sch(&ex, 100, 100);
      for (int i = 0; i < 10; ++i) {
        auto j = make_job(30, 300, i);
        uint64_t t;
        CHECK(sch.submit(j, &t) == LITHO_OK);
        jobs.push_back(j);
      }
    }
    for (auto &j : jobs) CHECK(j->state == State::Done && j->status == LITHO_OK);
    std::printf("drain ok\n");
  }
  // 5. kept slot buffers count against the budget: their total never exceeds
  //    it, idle slots are trimmed to admit a request, and everything finishes
  {
    KeepingExecutor ex(4);
    const size_t budget = 100;
    std::vector<std::shared_ptr<Job>> jobs;
    {
      Scheduler sch(&ex, budget, 1000);
      for (int i = 0; i < 40; ++i) {
        // runs of small requests fill every slot's buffers, then a large one
        // needs the buffers of idle slots released
        const size_t fp = (i % 10 == 9) ? 90 : 20 + size_t(i % 6);
        auto j = make_job(fp, 100 + (i % 3) * 50, i);
        uint64_t t;
        CHECK(sch.submit(j, &t) == LITHO_OK);
        jobs.push_back(j);
      }
      for (auto &j : jobs) {
        std::shared_ptr<Job> out;
        CHECK(sch.wait(j->ticket, -1, &out) == LITHO_OK);
        CHECK(out->status == LITHO_OK);
      }
      CHECK(sch.peak_in_use() <= budget);
    }
    CHECK(ex.max_kept_total <= budget);
    CHECK(ex.trims > 0);
    std::printf("kept buffers ok: max kept %zu of %zu, %d trims\n", ex.max_kept_total, budget, ex.trims);
  }
  std::printf("ALL OK\n");
  return 0;
}
