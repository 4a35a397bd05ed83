// Continuous-batching request scheduler (host only, no HIP).
//
// Requests wait in a FIFO queue.  A scheduler thread admits the head request
// as soon as a slot is free and its device footprint fits the remaining
// budget, starts it on that slot (asynchronously), and keeps polling running
// slots so that finished requests release their slot and footprint at once;
// requests that arrive while others run are admitted as soon as room appears,
// so work from different requests overlaps on the device.  Admission is strict
// FIFO, which bounds waiting: no request is overtaken.
//
// The executor (device work) is an interface, so the policy can be exercised
// with a host-only mock.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "litho.h"

namespace litho {
namespace serve {

inline double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// Timed condition-variable wait.  Builds with LITHO_SERVE_SYSTEM_CLOCK_WAITS
// wait on the system clock: older ThreadSanitizer runtimes do not intercept
// the steady-clock wait primitive and then report false lock errors.
template <typename Pred>
inline bool timed_wait(std::condition_variable &cv, std::unique_lock<std::mutex> &lk, int64_t us, Pred pred) {
#ifdef LITHO_SERVE_SYSTEM_CLOCK_WAITS
  return cv.wait_until(lk, std::chrono::system_clock::now() + std::chrono::microseconds(us), pred);
#else
  return cv.wait_for(lk, std::chrono::microseconds(us), pred);
#endif
}

enum class State { Queued, Running, Done };

struct Job {
  uint64_t ticket = 0;
  size_t footprint = 0;     // device bytes held while running
  State state = State::Queued;
  int status = LITHO_OK;    // result of the request
  std::string error;
  int slot = -1;
  double t_submit = 0, t_start = 0, t_done = 0;
  std::shared_ptr<void> payload;  // executor-specific request and result data
};

class Executor {
 public:
  virtual ~Executor() = default;
  virtual int slots() const = 0;
  // Starts the job on a free slot, asynchronously.  A non-OK return finishes
  // the job with that status (job.error may carry the reason).
  virtual int launch(Job &job, int slot) = 0;
  // True once the work started on the slot has finished.
  virtual bool ready(int slot) = 0;
  // Moves the finished job's results to host memory; returns its status.
  virtual int collect(Job &job, int slot) = 0;
  // Called once on the scheduler thread before anything else.
  virtual void thread_init() {}
  // Device bytes the slot keeps between requests (buffers sized for the
  // largest request it has run), and their release while the slot is idle.
  // Admission counts these against the budget.
  virtual size_t held(int /*slot*/) const { return 0; }
  virtual void trim(int /*slot*/) {}
};

class Scheduler {
 public:
  Scheduler(Executor *ex, size_t budget, int max_queue, int poll_us = 20)
      : ex_(ex), budget_(budget), max_queue_(max_queue), poll_us_(poll_us),
        running_(size_t(ex->slots())) {
    th_ = std::thread([this] { loop(); });
  }

  ~Scheduler() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    if (th_.joinable()) th_.join();
  }

  Scheduler(const Scheduler &) = delete;
  Scheduler &operator=(const Scheduler &) = delete;

  // Queues a job.  LITHO_E_NOMEM if it can never fit the budget,
  // LITHO_E_BUSY if the queue is full.
  int submit(std::shared_ptr<Job> job, uint64_t *ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return LITHO_E_INVALID;
    if (job->footprint > budget_) return LITHO_E_NOMEM;
    if (int(queue_.size()) >= max_queue_) return LITHO_E_BUSY;
    job->ticket = next_ticket_++;
    job->state = State::Queued;
    job->t_submit = now_us();
    jobs_[job->ticket] = job;
    queue_.push_back(job);
    *ticket = job->ticket;
    cv_work_.notify_one();
    return LITHO_OK;
  }

  // Waits up to timeout_us (< 0: forever, 0: no wait) for a ticket.  On
  // completion returns LITHO_OK, hands the job over in *out and forgets the
  // ticket; LITHO_PENDING if not done yet; LITHO_E_NOTFOUND if unknown.
  int wait(uint64_t ticket, int64_t timeout_us, std::shared_ptr<Job> *out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return LITHO_E_NOTFOUND;
    std::shared_ptr<Job> job = it->second;
    auto done = [&] { return job->state == State::Done; };
    if (!done()) {
      if (timeout_us < 0)
        cv_done_.wait(lk, done);
      else if (timeout_us > 0)
        timed_wait(cv_done_, lk, timeout_us, done);
    }
    if (!done()) return LITHO_PENDING;
    jobs_.erase(ticket);
    *out = job;
    return LITHO_OK;
  }

  size_t in_use() const {
    std::lock_guard<std::mutex> lk(mu_);
    return in_use_;
  }
  size_t peak_in_use() const {
    std::lock_guard<std::mutex> lk(mu_);
    return peak_;
  }
  size_t queued() const {
    std::lock_guard<std::mutex> lk(mu_);
    return queue_.size();
  }

 private:
  void finish(const std::shared_ptr<Job> &job, int slot, int status) {
    std::lock_guard<std::mutex> lk(mu_);
    job->status = status;
    job->t_done = now_us();
    job->state = State::Done;
    in_use_ -= job->footprint;
    running_[size_t(slot)].reset();
    cv_done_.notify_all();
  }

  void loop() {
    ex_->thread_init();
    for (;;) {
      // 1. completions (executor calls outside the lock)
      std::vector<std::pair<int, std::shared_ptr<Job>>> active;
      {
        std::lock_guard<std::mutex> lk(mu_);
        for (size_t s = 0; s < running_.size(); ++s)
          if (running_[s]) active.emplace_back(int(s), running_[s]);
      }
      for (auto &a : active)
        if (ex_->ready(a.first)) finish(a.second, a.first, ex_->collect(*a.second, a.first));
      // 2. admission, strict FIFO.  A slot commits max(kept bytes, footprint
      // of its running request); the head request is admitted on a free slot
      // when the total commitment stays within the budget, releasing the kept
      // buffers of other idle slots (largest first) if that makes it fit.
      for (;;) {
        std::shared_ptr<Job> job;
        int slot = -1;
        {
          std::lock_guard<std::mutex> lk(mu_);
          if (queue_.empty()) break;
          const size_t need = queue_.front()->footprint;
          // free slot: one already holding enough, else the one holding most
          for (size_t s = 0; s < running_.size(); ++s) {
            if (running_[s]) continue;
            const size_t h = ex_->held(int(s));
            if (slot < 0) {
              slot = int(s);
              continue;
            }
            const size_t hb = ex_->held(slot);
            if ((h >= need && (hb < need || h < hb)) || (hb < need && h > hb)) slot = int(s);
          }
          if (slot < 0) break;
          auto committed = [&] {
            size_t c = 0;
            for (size_t s = 0; s < running_.size(); ++s) {
              const size_t h = ex_->held(int(s));
              const size_t f = running_[s] ? running_[s]->footprint : 0;
              c += h > f ? h : f;
            }
            return c;
          };
          auto with_job = [&] {
            const size_t h = ex_->held(slot);
            return committed() - h + (h > need ? h : need);
          };
          while (with_job() > budget_) {
            int victim = -1;
            for (size_t s = 0; s < running_.size(); ++s)
              if (!running_[s] && int(s) != slot && ex_->held(int(s)) > 0 &&
                  (victim < 0 || ex_->held(int(s)) > ex_->held(victim)))
                victim = int(s);
            if (victim < 0) break;
            ex_->trim(victim);
          }
          if (with_job() > budget_) break;
          job = queue_.front();
          queue_.pop_front();
          running_[size_t(slot)] = job;
          in_use_ += job->footprint;
          const size_t c = committed();
          if (c > peak_) peak_ = c;
          job->slot = slot;
          job->state = State::Running;
          job->t_start = now_us();
        }
        const int rc = ex_->launch(*job, slot);
        if (rc != LITHO_OK) finish(job, slot, rc);
      }
      // 3. idle or poll
      std::unique_lock<std::mutex> lk(mu_);
      bool any_running = false;
      for (auto &r : running_) any_running = any_running || bool(r);
      if (stop_ && queue_.empty() && !any_running) break;
      if (!any_running && queue_.empty())
        cv_work_.wait(lk, [&] { return stop_ || !queue_.empty(); });
      else
        // requests are running (or queued behind a full device): check again
        // after the poll interval; a stop does not cut the wait short, so
        // draining does not spin
        timed_wait(cv_work_, lk, poll_us_, [] { return false; });
    }
  }

  Executor *ex_;
  size_t budget_;
  int max_queue_;
  int poll_us_;
  mutable std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<std::shared_ptr<Job>> queue_;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs_;
  std::vector<std::shared_ptr<Job>> running_;
  size_t in_use_ = 0, peak_ = 0;
  uint64_t next_ticket_ = 1;
  bool stop_ = false;
  std::thread th_;
};

}  // namespace serve
}  // namespace litho
