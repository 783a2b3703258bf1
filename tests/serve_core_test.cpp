// serve_core_test.cpp -- the serving scheduler's policy (ServeCore) driven by
// a mock executor on the CPU: admission by budget, strict FIFO order, slot
// limits, VP_ECAPACITY, ticket release, the VP_EBUSY protocol (a job holds its
// sky until it retires), eviction of leftovers, a per-job admission failure, a
// device failure that ends every running job, draining on destruction, and a
// multi-threaded stress run.  Built with g++ (also with -fsanitize=thread) by
// test_serve_core.py; prints one line per case and exits non-zero on failure.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "serve_core.h"
#include "vp.h"

using namespace vp;

static int g_fail = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
      ++g_fail;                                                      \
    }                                                                \
  } while (0)

template <class F>
static bool wait_until(F pred, int ms = 5000) {
  auto t0 = std::chrono::steady_clock::now();
  while (!pred()) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(ms)) return false;
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  return true;
}

// A caller-side object that jobs hold while pending (a sky or an observation).
struct MockSky {
  std::atomic<int> jobs{0};
  int destroy() { return jobs.load() > 0 ? VP_EBUSY : VP_OK; }
};

struct MockJob {
  uint64_t ticket = 0;
  int fail_admit = VP_OK;             // admit() returns this
  std::atomic<bool> complete{false};  // the test completes the job
  int auto_polls = -1;                // or: the job completes after this many polls
  int polls = 0;
  MockSky *sky = nullptr;
  std::atomic<int> retired{0};
  std::atomic<int> finished{0};
  std::atomic<int> abandoned{0};
};

static MockJob &mj(CoreJob &j) { return *(MockJob *)j.payload; }

class MockExec : public ServeExecutor {
 public:
  std::mutex mu;  // guards what the test thread reads while the core runs
  int slots = 1 << 30;
  int running = 0, max_running = 0;
  uint64_t running_bytes = 0, max_running_bytes = 0;
  uint64_t evictable = 0;
  bool evict_frees = true;
  int evicts = 0;
  std::vector<uint64_t> admit_order;
  int kick_fail = 0;        // the next kick_fail kicks fail
  int kick_fail_every = 0;  // and, if > 0, every kick_fail_every-th kick
  uint64_t kicks = 0, idles = 0;
  int kick_rc = VP_EDEVICE;
  std::vector<std::vector<uint64_t>> abandon_sets;
  std::thread::id core_thread;
  bool wrong_thread = false;

  void on_core() {
    if (core_thread == std::thread::id()) core_thread = std::this_thread::get_id();
    if (core_thread != std::this_thread::get_id()) wrong_thread = true;
  }
  void thread_start() override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
  }
  bool has_room(const CoreJob &) override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    return running < slots;
  }
  uint64_t evictable_bytes() override {
    std::lock_guard<std::mutex> lk(mu);
    return evictable;
  }
  void evict() override {
    std::lock_guard<std::mutex> lk(mu);
    ++evicts;
    if (evict_frees) evictable = 0;
  }
  int admit(CoreJob &j) override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    MockJob &m = mj(j);
    if (m.fail_admit != VP_OK) return m.fail_admit;
    admit_order.push_back(j.ticket);
    ++running;
    max_running = std::max(max_running, running);
    running_bytes += j.footprint;
    max_running_bytes = std::max(max_running_bytes, running_bytes);
    return VP_OK;
  }
  bool poll(CoreJob &j) override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    MockJob &m = mj(j);
    ++m.polls;
    if (j.t_start == 0) j.t_start = j.t_admit;
    const bool done = m.auto_polls >= 0 ? m.polls >= m.auto_polls : m.complete.load();
    if (done) j.status = VP_OK;
    return done;
  }
  int kick() override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    ++kicks;
    if (kick_fail > 0) {
      --kick_fail;
      return kick_rc;
    }
    if (kick_fail_every > 0 && kicks % (uint64_t)kick_fail_every == 0) return kick_rc;
    return VP_OK;
  }
  void idle() override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    ++idles;
  }
  void abandon(const std::vector<CoreJob *> &run, int) override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    std::vector<uint64_t> t;
    for (CoreJob *j : run) {
      t.push_back(j->ticket);
      mj(*j).abandoned += 1;
      --running;
      running_bytes -= j->footprint;
    }
    std::sort(t.begin(), t.end());
    abandon_sets.push_back(t);
  }
  void finished(CoreJob &j) override {
    std::lock_guard<std::mutex> lk(mu);
    on_core();
    mj(j).finished += 1;
    --running;
    running_bytes -= j.footprint;
  }
  void retired(CoreJob &j) override {
    MockJob &m = mj(j);
    m.retired += 1;
    if (m.sky) m.sky->jobs -= 1;
  }
  std::vector<uint64_t> admitted() {
    std::lock_guard<std::mutex> lk(mu);
    return admit_order;
  }
};

// Submits a job as vp_submit does: the sky is held from here until retired().
static int submit(ServeCore &core, MockJob &m, uint64_t footprint, uint64_t *ticket) {
  if (m.sky) m.sky->jobs += 1;
  CoreJob *j = new CoreJob();
  j->footprint = footprint;
  j->payload = &m;
  const int rc = core.submit(j, ticket);
  if (rc != VP_OK) {
    if (m.sky) m.sky->jobs -= 1;
    delete j;
  } else {
    m.ticket = *ticket;
  }
  return rc;
}

static bool admitted(MockExec &ex, uint64_t t) {
  auto a = ex.admitted();
  return std::find(a.begin(), a.end(), t) != a.end();
}

static int poll_done(ServeCore &core, uint64_t t, CoreJob *out, int ms = 5000) {
  int rc = VP_EAGAIN;
  wait_until([&]() { return (rc = core.poll(t, out)) != VP_EAGAIN; }, ms);
  return rc;
}

static void t_capacity() {
  MockExec ex;
  ServeCore core(&ex, 100);
  MockJob a, b;
  uint64_t t = 0;
  CHECK(submit(core, a, 101, &t) == VP_ECAPACITY);
  CHECK(t == 0);
  CHECK(submit(core, b, 100, &t) == VP_OK);  // exactly the budget is admissible
  CHECK(t == 1);                             // the refused job took no ticket
  b.complete = true;
  CoreJob out;
  CHECK(poll_done(core, t, &out) == VP_OK);
  CHECK(out.status == VP_OK);
}

static void t_budget_fifo() {
  MockExec ex;
  ServeCore core(&ex, 100);
  MockJob a, b, c;
  uint64_t ta, tb, tc;
  CHECK(submit(core, a, 60, &ta) == VP_OK);
  CHECK(wait_until([&]() { return admitted(ex, ta); }));
  CHECK(submit(core, b, 60, &tb) == VP_OK);  // does not fit beside a
  CHECK(submit(core, c, 10, &tc) == VP_OK);  // fits, but b is ahead of it
  std::this_thread::sleep_for(std::chrono::milliseconds(30));
  CHECK(!admitted(ex, tb));
  CHECK(!admitted(ex, tc));
  CHECK(core.in_use() == 60);
  CoreJob out;
  CHECK(core.poll(tb, &out) == VP_EAGAIN);
  a.complete = true;
  CHECK(wait_until([&]() { return admitted(ex, tb) && admitted(ex, tc); }));
  CHECK(core.in_use() == 70);
  b.complete = c.complete = true;
  CHECK(poll_done(core, ta, &out) == VP_OK);
  CHECK(poll_done(core, tb, &out) == VP_OK);
  CHECK(poll_done(core, tc, &out) == VP_OK);
  CHECK((ex.admitted() == std::vector<uint64_t>{ta, tb, tc}));
  CHECK(ex.max_running_bytes <= 100);
  CHECK(core.in_use() == 0);
}

static void t_slots() {
  MockExec ex;
  ex.slots = 2;
  ServeCore core(&ex, 1000);
  std::vector<MockJob> m(5);
  std::vector<uint64_t> t(5);
  for (int i = 0; i < 5; ++i) CHECK(submit(core, m[i], 1, &t[i]) == VP_OK);
  CHECK(wait_until([&]() { return admitted(ex, t[1]); }));
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  CHECK(!admitted(ex, t[2]));  // only two slots, although the budget has room
  for (int i = 0; i < 5; ++i) m[i].complete = true;
  CoreJob out;
  for (int i = 0; i < 5; ++i) CHECK(poll_done(core, t[i], &out) == VP_OK);
  std::lock_guard<std::mutex> lk(ex.mu);
  CHECK(ex.max_running == 2);
}

static void t_tickets() {
  MockExec ex;
  ServeCore core(&ex, 100);
  MockJob a;
  uint64_t t;
  CHECK(submit(core, a, 10, &t) == VP_OK);
  CoreJob out;
  CHECK(core.poll(t, &out) == VP_EAGAIN);
  CHECK(core.pending());
  a.complete = true;
  CHECK(poll_done(core, t, &out) == VP_OK);
  CHECK(out.ticket == t);
  CHECK(out.status == VP_OK);
  CHECK(out.payload == nullptr);
  CHECK(out.t_submit > 0 && out.t_submit <= out.t_admit && out.t_admit <= out.t_start &&
        out.t_start <= out.t_done);
  CHECK(core.poll(t, &out) == VP_ENOTFOUND);  // released by the first VP_OK poll
  CHECK(core.poll(987654, &out) == VP_ENOTFOUND);
  CHECK(!core.pending());
  CHECK(a.retired == 1 && a.finished == 1);
}

static void t_busy() {
  MockExec ex;
  ServeCore core(&ex, 100);
  MockSky sky;
  MockJob a, b;
  a.sky = b.sky = &sky;
  uint64_t ta, tb;
  CHECK(submit(core, a, 10, &ta) == VP_OK);
  CHECK(submit(core, b, 10, &tb) == VP_OK);
  CHECK(sky.destroy() == VP_EBUSY);
  CHECK(core.pending());  // a context with pending jobs refuses to go (VP_EBUSY)
  a.complete = true;
  CoreJob out;
  CHECK(poll_done(core, ta, &out) == VP_OK);
  CHECK(sky.destroy() == VP_EBUSY);  // b still holds it
  b.complete = true;
  CHECK(wait_until([&]() { return !core.pending(); }));
  CHECK(sky.destroy() == VP_OK);  // b retired, though its ticket is not yet collected
  CHECK(poll_done(core, tb, &out) == VP_OK);
}

static void t_evict() {
  MockExec ex;
  ex.evictable = 50;
  ServeCore core(&ex, 100);
  MockJob a;
  uint64_t ta;
  CHECK(submit(core, a, 60, &ta) == VP_OK);
  CHECK(wait_until([&]() { return admitted(ex, ta); }));
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    CHECK(ex.evicts >= 1);
    CHECK(ex.evictable == 0);
  }
  a.complete = true;
  CoreJob out;
  CHECK(poll_done(core, ta, &out) == VP_OK);
  // leftovers that eviction cannot free hold the next job back
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    ex.evictable = 50;
    ex.evict_frees = false;
  }
  MockJob b;
  uint64_t tb;
  CHECK(submit(core, b, 60, &tb) == VP_OK);
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  CHECK(!admitted(ex, tb));
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    ex.evictable = 40;  // 40 + 60 fits
  }
  CHECK(wait_until([&]() { return admitted(ex, tb); }));
  b.complete = true;
  CHECK(poll_done(core, tb, &out) == VP_OK);
}

static void t_admit_failure() {
  MockExec ex;
  ServeCore core(&ex, 100);
  MockSky sky;
  MockJob a, b, c;
  a.sky = b.sky = c.sky = &sky;
  b.fail_admit = VP_ENOMEM;
  uint64_t ta, tb, tc;
  CHECK(submit(core, a, 30, &ta) == VP_OK);
  CHECK(submit(core, b, 30, &tb) == VP_OK);
  CHECK(submit(core, c, 30, &tc) == VP_OK);
  CoreJob out;
  CHECK(poll_done(core, tb, &out) == VP_OK);  // b ends alone, with its error
  CHECK(out.status == VP_ENOMEM);
  CHECK(b.retired == 1 && b.finished == 0);
  CHECK(wait_until([&]() { return admitted(ex, tc); }));
  CHECK(core.in_use() == 60);  // b was never charged
  CHECK(core.poll(ta, &out) == VP_EAGAIN);
  a.complete = c.complete = true;
  CHECK(poll_done(core, ta, &out) == VP_OK && out.status == VP_OK);
  CHECK(poll_done(core, tc, &out) == VP_OK && out.status == VP_OK);
  CHECK(core.in_use() == 0);
  CHECK(sky.destroy() == VP_OK);
}

static void t_kick_failure() {
  MockExec ex;
  ServeCore core(&ex, 100);
  MockJob a, b;
  uint64_t ta, tb;
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    ex.kick_fail = 0;
  }
  CHECK(submit(core, a, 30, &ta) == VP_OK);
  CHECK(submit(core, b, 30, &tb) == VP_OK);
  CHECK(wait_until([&]() { return admitted(ex, ta) && admitted(ex, tb); }));
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    ex.kick_fail = 1;  // the device fails under both
  }
  CoreJob out;
  CHECK(poll_done(core, ta, &out) == VP_OK && out.status == VP_EDEVICE);
  CHECK(poll_done(core, tb, &out) == VP_OK && out.status == VP_EDEVICE);
  CHECK(a.abandoned == 1 && b.abandoned == 1);
  CHECK(a.finished == 0 && b.finished == 0);
  CHECK(a.retired == 1 && b.retired == 1);
  {
    std::lock_guard<std::mutex> lk(ex.mu);
    CHECK(ex.abandon_sets.size() == 1);
    if (!ex.abandon_sets.empty()) CHECK((ex.abandon_sets[0] == std::vector<uint64_t>{ta, tb}));
    CHECK(ex.running == 0);
  }
  CHECK(core.in_use() == 0);
  MockJob c;  // the scheduler goes on
  uint64_t tc;
  CHECK(submit(core, c, 30, &tc) == VP_OK);
  c.complete = true;
  CHECK(poll_done(core, tc, &out) == VP_OK && out.status == VP_OK);
}

static void t_drain() {
  MockExec ex;
  std::vector<MockJob> m(20);
  {
    ServeCore core(&ex, 50);
    for (int i = 0; i < 20; ++i) {
      m[i].auto_polls = 1 + i % 4;
      uint64_t t;
      CHECK(submit(core, m[i], 10 + i, &t) == VP_OK);
    }
  }  // the destructor waits for every job
  for (int i = 0; i < 20; ++i) CHECK(m[i].retired == 1 && m[i].finished == 1);
  CHECK(ex.running == 0 && ex.max_running_bytes <= 50);
  CHECK(!ex.wrong_thread);
}

static void t_stress() {
  MockExec ex;
  ex.slots = 6;
  ex.kick_fail_every = 101;
  const uint64_t budget = 100;
  const int nthreads = 8, per = 250;
  std::vector<MockJob> m(nthreads * per);
  MockSky sky;
  std::atomic<int> bad{0}, failed{0}, ok{0};
  std::mutex tmu;
  std::set<uint64_t> tickets;
  {
    ServeCore core(&ex, budget);
    std::vector<std::thread> th;
    for (int w = 0; w < nthreads; ++w) {
      th.emplace_back([&, w]() {
        std::mt19937 rng(1234 + w);
        std::vector<std::pair<uint64_t, MockJob *>> mine;
        for (int i = 0; i < per; ++i) {
          MockJob &j = m[w * per + i];
          j.sky = &sky;
          j.auto_polls = 1 + (int)(rng() % 5);
          if (rng() % 50 == 0) j.fail_admit = VP_ENOMEM;
          uint64_t t;
          if (submit(core, j, 1 + rng() % 40, &t) != VP_OK) {
            ++bad;
            continue;
          }
          {
            std::lock_guard<std::mutex> lk(tmu);
            if (!tickets.insert(t).second) ++bad;
          }
          mine.push_back({t, &j});
          if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
        }
        for (auto &p : mine) {
          CoreJob out;
          const int rc = poll_done(core, p.first, &out, 60000);
          if (rc != VP_OK) {
            ++bad;
            continue;
          }
          if (out.status == VP_OK) {
            ++ok;
          } else if (out.status == VP_ENOMEM && p.second->fail_admit == VP_ENOMEM) {
            ++failed;
          } else if (out.status == VP_EDEVICE && p.second->abandoned == 1) {
            ++failed;
          } else {
            ++bad;
          }
          if (core.poll(p.first, &out) != VP_ENOTFOUND) ++bad;
        }
      });
    }
    for (auto &t : th) t.join();
    CHECK(!core.pending());
    CHECK(core.in_use() == 0);
  }
  CHECK(bad == 0);
  CHECK(ok + failed == nthreads * per);
  CHECK(sky.destroy() == VP_OK);
  for (auto &j : m) CHECK(j.retired == 1);
  CHECK(ex.max_running_bytes <= budget);
  CHECK(ex.max_running <= ex.slots);
  CHECK(ex.running == 0);
  CHECK(!ex.wrong_thread);
  // strict FIFO: admissions in ticket order
  CHECK(std::is_sorted(ex.admit_order.begin(), ex.admit_order.end()));
  printf("  stress: %d ok, %d failed by injection, %zu abandon events, %llu kicks\n", ok.load(), failed.load(),
         ex.abandon_sets.size(), (unsigned long long)ex.kicks);
}

int main() {
  struct {
    const char *name;
    void (*f)();
  } cases[] = {{"capacity", t_capacity},         {"budget_fifo", t_budget_fifo}, {"slots", t_slots},
               {"tickets", t_tickets},           {"busy", t_busy},               {"evict", t_evict},
               {"admit_failure", t_admit_failure}, {"kick_failure", t_kick_failure}, {"drain", t_drain},
               {"stress", t_stress}};
  for (auto &c : cases) {
    const int before = g_fail;
    c.f();
    printf("%s %s\n", g_fail == before ? "PASS" : "FAIL", c.name);
    fflush(stdout);
  }
  return g_fail ? 1 : 0;
}
