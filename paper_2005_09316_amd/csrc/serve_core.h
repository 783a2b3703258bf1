// serve_core.h -- the serving scheduler's policy, free of any device code:
// FIFO admission by HBM footprint, tickets, completion bookkeeping and the
// scheduler thread.  What a job does on the device (publishing its work,
// launching the persistent kernel, reading completion flags) sits behind
// ServeExecutor; libvp's executor lives in vp_serve.cpp, and the tests drive
// the core with a mock executor on the CPU (also under ThreadSanitizer).
#ifndef VP_SERVE_CORE_H
#define VP_SERVE_CORE_H

#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace vp {

enum CoreJobState { kQueued = 0, kRunning = 1, kDone = 2 };

// One job as the core sees it.  Times are CLOCK_MONOTONIC ns; dev_start and
// dev_done are the executor's device timestamps (0 when it has none).
struct CoreJob {
  uint64_t ticket = 0;
  uint64_t footprint = 0;  // bytes charged against the budget while the job runs
  int state = kQueued;
  int status = 0;          // VP_OK or the job's error code, once done
  uint64_t t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  uint64_t dev_start = 0, dev_done = 0;
  void *payload = nullptr;  // the executor's per-job state
};

// Device side of the scheduler.  Every call comes from the core's thread with
// the core's lock held, so an executor needs no locking of its own for state
// that only these calls touch.
class ServeExecutor {
 public:
  virtual ~ServeExecutor() = default;
  // First call on the core's thread, before any other (e.g. to select a device).
  virtual void thread_start() {}
  // Room for the job beyond the HBM budget (job slots, queue space).
  virtual bool has_room(const CoreJob &j) = 0;
  // Bytes held by finished jobs' leftovers that evict() would free.
  virtual uint64_t evictable_bytes() = 0;
  virtual void evict() = 0;
  // Starts the job: VP_OK (it runs), or an error code that ends this job
  // alone (the executor has undone whatever it started).
  virtual int admit(CoreJob &j) = 0;
  // Advances a running job; true once it is done (status, t_start and the
  // device timestamps filled in).
  virtual bool poll(CoreJob &j) = 0;
  // Makes the device consume the running jobs' work; an error means the work
  // of every running job is lost.
  virtual int kick() = 0;
  // Called while no job runs.
  virtual void idle() = 0;
  // After kick() failed: the running jobs end with rc; the executor drops
  // their device work and resources (finished() is not called for them).
  virtual void abandon(const std::vector<CoreJob *> &running, int rc) = 0;
  // A job is done or failed after admission: release its resources.
  virtual void finished(CoreJob &j) = 0;
  // A job leaves the core (done, failed or refused at admission): drop the
  // caller-side references it holds.  Once per job.
  virtual void retired(CoreJob &j) = 0;
};

class ServeCore {
 public:
  // The budget bounds the footprint of running jobs; the thread starts here.
  ServeCore(ServeExecutor *ex, uint64_t budget, uint64_t (*clock_ns)() = nullptr);
  // Drains: waits until every submitted job is done, then stops the thread.
  ~ServeCore();
  ServeCore(const ServeCore &) = delete;
  ServeCore &operator=(const ServeCore &) = delete;

  // Takes the job (allocated with new; the core deletes it) and returns its
  // ticket.  VP_ECAPACITY when its footprint exceeds the whole budget.
  int submit(CoreJob *j, uint64_t *ticket);
  // VP_OK with *out filled once the job is done (the ticket is then
  // forgotten), VP_EAGAIN while it is queued or running, VP_ENOTFOUND for an
  // unknown ticket.
  int poll(uint64_t ticket, CoreJob *out);
  // Jobs queued or running.
  bool pending();
  uint64_t in_use();

 private:
  void loop();
  void end_job(CoreJob *j, int status);  // lock held

  ServeExecutor *ex_;
  const uint64_t budget_;
  uint64_t (*clock_)();
  std::mutex mu_;
  std::condition_variable cv_;
  bool quit_ = false;
  std::deque<CoreJob *> queue_;
  std::vector<CoreJob *> running_;
  std::unordered_map<uint64_t, CoreJob *> jobs_;
  uint64_t next_ticket_ = 1;
  uint64_t in_use_ = 0;
  std::thread th_;
};

}  // namespace vp

#endif  // VP_SERVE_CORE_H
