// CPU tests of the serving scheduler with a fake executor: no GPU, no HIP.
// Admission by footprint (first come first served), queue bounds, whole-
// budget refusal, cancellation of queued and running jobs, levels of 0
// steps, launch groups by window / metric / K, failure isolation of a
// non-finite job, device errors, and the threaded serving loop with stop.
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "scheduler.h"

using namespace muster;

static int g_failed = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::printf("  FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);            \
      ++g_failed;                                                             \
    }                                                                         \
  } while (0)

static double fake_clock() {
  static double t = 0.0;
  return t += 0.001;
}

struct FakeJob : JobHandle {
  struct Fake* ex = nullptr;
  int tag = 0;             // dims[1] of the job: identifies it in the log
  uint64_t bytes = 0;
  int level = 0;
  bool nonfinite = false;
  int steps = 0;
  ~FakeJob() override;
};

struct Fake : Executor {
  uint64_t budget_ = 0, used = 0;
  std::map<int, std::vector<int>> steps_at;   // tag -> level of each step taken
  std::vector<std::vector<int>> ticks;        // per step() call: the tags stepped
  int nonfinite_tag = -1, nonfinite_after = 0;  // this job's loss turns non-finite
  bool throw_on_step = false;
  bool poisoned = false;
  int admits = 0;
  uint64_t footprint(const muster_job& j) override { return (uint64_t)j.dims[0]; }
  uint64_t budget() override { return budget_; }
  bool fits(uint64_t b) override { return budget_ == 0 || used + b <= budget_; }
  std::unique_ptr<JobHandle> admit(const muster_job& j) override {
    if (j.N == 99) throw Error{MUSTER_E_NOMEM, "fake: no memory"};
    auto h = std::make_unique<FakeJob>();
    h->ex = this;
    h->tag = j.dims[1];
    h->bytes = footprint(j);
    used += h->bytes;
    ++admits;
    return h;
  }
  void step(const GroupKey& key, const std::vector<JobHandle*>& group,
            const std::vector<std::pair<uint64_t, int>>& sig) override {
    (void)key;
    if (throw_on_step) throw Error{MUSTER_E_DEVICE, "fake: device lost"};
    std::vector<int> tags;
    CHECK(sig.size() == group.size());
    for (JobHandle* g : group) {
      auto* f = static_cast<FakeJob*>(g);
      steps_at[f->tag].push_back(f->level);
      tags.push_back(f->tag);
      ++f->steps;
      if (f->tag == nonfinite_tag && f->steps >= nonfinite_after) f->nonfinite = true;
    }
    ticks.push_back(tags);
  }
  void forget_groups_except(const std::vector<GroupKey>&) override {}
  void sync(const std::vector<JobHandle*>&) override {}
  int level(JobHandle& h) override { return static_cast<FakeJob&>(h).level; }
  bool nonfinite(JobHandle& h) override { return static_cast<FakeJob&>(h).nonfinite; }
  void begin_level(JobHandle& h, int level) override { static_cast<FakeJob&>(h).level = level; }
  void finish(JobHandle& h, double t_submit, muster_report* rep) override {
    (void)t_submit;
    rep->loss_first = 1.0;
    rep->loss_last = 0.5;
    (void)h;
  }
  uint64_t held_bytes(JobHandle& h) override { return static_cast<FakeJob&>(h).bytes; }
  void on_device_error() override { poisoned = true; }
};

FakeJob::~FakeJob() {
  if (ex) ex->used -= bytes;
}

static muster_job job(uint64_t bytes, int tag, std::vector<int> iters, int window = 3,
                      int metric = MUSTER_METRIC_SILNCC, int K = 5) {
  muster_job j;
  std::memset(&j, 0, sizeof j);
  j.N = 3;
  j.dims[0] = (int)bytes;
  j.dims[1] = tag;
  j.dims[2] = 8;
  j.params.levels = (int)iters.size();
  for (size_t l = 0; l < iters.size(); ++l) j.params.iters[l] = iters[l];
  j.params.window = window;
  j.params.metric = metric;
  j.params.K = K;
  return j;
}

static muster_status status_of(Scheduler& s, uint64_t id, muster_report* rep = nullptr) {
  muster_report r{};
  std::string err;
  const muster_status st = s.wait(id, rep ? rep : &r, &err);
  return st;
}

static void test_fifo_admission_by_footprint() {
  std::printf("fifo admission by footprint\n");
  Fake ex;
  ex.budget_ = 100;
  Scheduler s(ex, 16, fake_clock);
  const uint64_t a = s.submit(job(60, 1, {2}));
  const uint64_t b = s.submit(job(60, 2, {1}));
  const uint64_t c = s.submit(job(30, 3, {1}));  // fits beside a, but waits behind b
  s.tick();
  int res = 0, q = 0;
  s.stats(&res, &q);
  CHECK(res == 1 && q == 2);
  CHECK(s.poll(a) == 1 && s.poll(b) == 0 && s.poll(c) == 0);
  s.tick();  // a's second step: a finishes and leaves
  CHECK(s.poll(a) == 2);
  CHECK(ex.used == 0);
  s.tick();  // b and c fit together now
  CHECK(s.poll(b) == 2 && s.poll(c) == 2);
  muster_report rb{};
  CHECK(status_of(s, a) == MUSTER_OK);
  CHECK(status_of(s, b, &rb) == MUSTER_OK);
  CHECK(rb.iterations == 1 && rb.footprint_bytes == 60 && rb.queue_seconds > 0);
  CHECK(status_of(s, c) == MUSTER_OK);
  CHECK(ex.steps_at[1].size() == 2 && ex.steps_at[2].size() == 1 && ex.steps_at[3].size() == 1);
}

static void test_refusals() {
  std::printf("whole-budget refusal and full queue\n");
  Fake ex;
  ex.budget_ = 100;
  Scheduler s(ex, 2, fake_clock);
  bool nomem = false, busy = false;
  try {
    s.submit(job(101, 1, {1}));
  } catch (const Error& e) {
    nomem = e.st == MUSTER_E_NOMEM;
  }
  CHECK(nomem);
  s.submit(job(10, 2, {1}));
  s.submit(job(10, 3, {1}));
  try {
    s.submit(job(10, 4, {1}));
  } catch (const Error& e) {
    busy = e.st == MUSTER_E_BUSY;
  }
  CHECK(busy);
  bool unknown = false;
  try {
    s.poll(12345);
  } catch (const Error& e) {
    unknown = e.st == MUSTER_E_INVALID;
  }
  CHECK(unknown);
}

static void test_cancellation() {
  std::printf("cancellation of queued and running jobs\n");
  Fake ex;
  ex.budget_ = 100;
  Scheduler s(ex, 16, fake_clock);
  const uint64_t run = s.submit(job(80, 1, {1000}));
  const uint64_t queued = s.submit(job(80, 2, {3}));
  s.tick();
  CHECK(s.poll(run) == 1 && s.poll(queued) == 0);
  s.cancel(queued);
  s.cancel(run);
  s.tick();
  muster_report r{};
  CHECK(status_of(s, run, &r) == MUSTER_E_CANCELLED);
  CHECK(r.iterations == 1);
  CHECK(status_of(s, queued) == MUSTER_E_CANCELLED);
  CHECK(ex.used == 0 && ex.admits == 1);
  const uint64_t next = s.submit(job(80, 3, {2}));
  s.tick();
  s.tick();
  CHECK(status_of(s, next) == MUSTER_OK);
}

static void test_levels_without_steps_are_passed_over() {
  std::printf("levels of 0 steps\n");
  Fake ex;
  Scheduler s(ex, 16, fake_clock);
  const uint64_t a = s.submit(job(1, 1, {0, 3}));
  const uint64_t b = s.submit(job(1, 2, {2, 0, 1}));
  for (int k = 0; k < 6; ++k) s.tick();
  muster_report ra{}, rb{};
  CHECK(status_of(s, a, &ra) == MUSTER_OK && ra.iterations == 3);
  CHECK(status_of(s, b, &rb) == MUSTER_OK && rb.iterations == 3);
  CHECK((ex.steps_at[1] == std::vector<int>{1, 1, 1}));
  CHECK((ex.steps_at[2] == std::vector<int>{0, 0, 2}));
}

static void test_groups_share_ticks() {
  std::printf("launch groups by window, metric and K\n");
  Fake ex;
  Scheduler s(ex, 16, fake_clock);
  const uint64_t a = s.submit(job(1, 1, {3}, 3, MUSTER_METRIC_SILNCC, 5));
  const uint64_t b = s.submit(job(1, 2, {3}, 5, MUSTER_METRIC_SILNCC, 5));
  const uint64_t c = s.submit(job(1, 3, {3}, 3, MUSTER_METRIC_LNCC, 5));
  const uint64_t d = s.submit(job(1, 4, {3}, 3, MUSTER_METRIC_SILNCC, 7));
  const uint64_t e = s.submit(job(1, 5, {3}, 3, MUSTER_METRIC_SILNCC, 5));
  s.tick();
  // one step() per group, every job stepped in the first tick (no job waits
  // behind one it cannot share launches with); a and e share a group
  CHECK(ex.ticks.size() == 4);
  int stepped = 0;
  for (auto& t : ex.ticks) stepped += (int)t.size();
  CHECK(stepped == 5);
  bool ae = false;
  for (auto& t : ex.ticks)
    if (t.size() == 2) ae = (t[0] == 1 && t[1] == 5);
  CHECK(ae);
  s.tick();
  s.tick();
  for (uint64_t id : {a, b, c, d, e}) CHECK(status_of(s, id) == MUSTER_OK);
}

static void test_nonfinite_job_fails_alone() {
  std::printf("failure isolation\n");
  Fake ex;
  ex.nonfinite_tag = 2;
  ex.nonfinite_after = 2;
  Scheduler s(ex, 16, fake_clock);
  const uint64_t a = s.submit(job(1, 1, {4}));
  const uint64_t b = s.submit(job(1, 2, {4}));
  for (int k = 0; k < 4; ++k) s.tick();
  muster_report rb{};
  CHECK(status_of(s, b, &rb) == MUSTER_E_NONFINITE && rb.iterations == 2);
  CHECK(status_of(s, a) == MUSTER_OK);
  CHECK(ex.steps_at[1].size() == 4 && ex.steps_at[2].size() == 2);
}

static void test_admission_and_device_errors() {
  std::printf("admission failure and device error\n");
  Fake ex;
  Scheduler s(ex, 16, fake_clock);
  muster_job bad = job(1, 9, {2});
  bad.N = 99;  // the fake refuses it at admission
  const uint64_t x = s.submit(bad);
  const uint64_t a = s.submit(job(1, 1, {5}));
  s.tick();
  CHECK(status_of(s, x) == MUSTER_E_NOMEM);
  CHECK(s.poll(a) == 1);
  ex.throw_on_step = true;
  s.tick();
  CHECK(status_of(s, a) == MUSTER_E_DEVICE);
  CHECK(ex.poisoned && ex.used == 0);
}

static void test_threaded_loop_and_stop() {
  std::printf("threaded serving loop\n");
  Fake ex;
  Scheduler s(ex, 64, fake_clock);
  std::thread th([&] {
    while (s.wait_for_work()) s.tick();
    s.shutdown();
  });
  std::vector<uint64_t> ids;
  for (int k = 0; k < 8; ++k) ids.push_back(s.submit(job(1, k, {3, 2})));
  for (uint64_t id : ids) {
    muster_report r{};
    CHECK(status_of(s, id, &r) == MUSTER_OK && r.iterations == 5);
  }
  const uint64_t longjob = s.submit(job(1, 100, {1000000}));
  while (s.poll(longjob) == 0) std::this_thread::yield();
  s.stop();
  th.join();
  CHECK(status_of(s, longjob) == MUSTER_E_CANCELLED);
}

int main() {
  test_fifo_admission_by_footprint();
  test_refusals();
  test_cancellation();
  test_levels_without_steps_are_passed_over();
  test_groups_share_ticks();
  test_nonfinite_job_fails_alone();
  test_admission_and_device_errors();
  test_threaded_loop_and_stop();
  std::printf(g_failed ? "%d checks failed\n" : "all passed\n", g_failed);
  return g_failed ? 1 : 0;
}
