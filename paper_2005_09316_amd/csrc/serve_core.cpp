// serve_core.cpp -- the serving scheduler's policy (see serve_core.h).
#include "serve_core.h"

#include <time.h>

#include <chrono>

#include "../../include/vp.h"

namespace vp {

static uint64_t monotonic_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

ServeCore::ServeCore(ServeExecutor *ex, uint64_t budget, uint64_t (*clock_ns)())
    : ex_(ex), budget_(budget), clock_(clock_ns ? clock_ns : monotonic_ns) {
  th_ = std::thread([this]() { loop(); });
}

ServeCore::~ServeCore() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    quit_ = true;
  }
  cv_.notify_all();
  if (th_.joinable()) th_.join();
  for (auto &kv : jobs_) delete kv.second;
}

int ServeCore::submit(CoreJob *j, uint64_t *ticket) {
  if (j->footprint > budget_) return VP_ECAPACITY;
  {
    std::lock_guard<std::mutex> lk(mu_);
    j->state = kQueued;
    j->t_submit = clock_();
    j->ticket = next_ticket_++;
    jobs_[j->ticket] = j;
    queue_.push_back(j);
    *ticket = j->ticket;
  }
  cv_.notify_all();
  return VP_OK;
}

int ServeCore::poll(uint64_t ticket, CoreJob *out) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = jobs_.find(ticket);
  if (it == jobs_.end()) return VP_ENOTFOUND;
  CoreJob *j = it->second;
  if (j->state != kDone) return VP_EAGAIN;
  *out = *j;
  out->payload = nullptr;
  jobs_.erase(it);
  delete j;
  return VP_OK;
}

bool ServeCore::pending() {
  std::lock_guard<std::mutex> lk(mu_);
  return !queue_.empty() || !running_.empty();
}

uint64_t ServeCore::in_use() {
  std::lock_guard<std::mutex> lk(mu_);
  return in_use_;
}

void ServeCore::end_job(CoreJob *j, int status) {
  j->status = status;
  j->state = kDone;
  j->t_done = clock_();
  if (j->t_start == 0) j->t_start = j->t_done;
  ex_->retired(*j);
}

void ServeCore::loop() {
  ex_->thread_start();
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    // completions
    for (size_t i = 0; i < running_.size();) {
      CoreJob *j = running_[i];
      if (ex_->poll(*j)) {
        in_use_ -= j->footprint;
        ex_->finished(*j);
        end_job(j, j->status);
        running_[i] = running_.back();
        running_.pop_back();
      } else {
        ++i;
      }
    }
    // admissions, strictly first come first served: the head of the queue
    // waits for room and budget, and nothing overtakes it.  The budget
    // covers running jobs and the leftovers of finished ones (the executor's
    // evictable bytes), which are released when they stand in the way.
    while (!queue_.empty()) {
      CoreJob *j = queue_.front();
      if (!ex_->has_room(*j)) break;
      if (in_use_ + j->footprint > budget_) break;
      if (in_use_ + ex_->evictable_bytes() + j->footprint > budget_) {
        ex_->evict();
        if (in_use_ + ex_->evictable_bytes() + j->footprint > budget_) break;
      }
      queue_.pop_front();
      j->t_admit = clock_();
      j->state = kRunning;
      const int rc = ex_->admit(*j);
      if (rc != VP_OK) {
        end_job(j, rc);
      } else {
        in_use_ += j->footprint;
        running_.push_back(j);
      }
    }
    if (!running_.empty()) {
      const int rc = ex_->kick();
      if (rc != VP_OK) {
        ex_->abandon(running_, rc);
        for (CoreJob *j : running_) {
          in_use_ -= j->footprint;
          end_job(j, rc);
        }
        running_.clear();
      }
    } else {
      ex_->idle();
    }
    if (quit_ && queue_.empty() && running_.empty()) break;
    if (queue_.empty() && running_.empty()) {
      // a poll period for idle(); submit() and the destructor notify.  The
      // deadline is on the system clock, whose timed wait ThreadSanitizer
      // follows (a clock step only stretches one idle period)
      cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(2));
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

}  // namespace vp
