// Continuous-batching scheduler of the registration server: the queue,
// admission by device-memory footprint, cancellation, one iteration of every
// resident job per tick, level changes and retirement.  It holds no device
// code: everything that touches the GPU goes through an Executor, which the
// runtime implements with HIP (jobs, launch plans, kernels) and the CPU tests
// implement with a fake that simulates jobs.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/muster.h"

namespace muster {

// The executor's device-side state of one admitted job.
struct JobHandle {
  virtual ~JobHandle() = default;
};

// Failure inside the library (thrown, converted to a status at the ABI).
struct Error {
  muster_status st;
  std::string msg;
};

// Launch group of resident jobs: {window, metric, K}.
using GroupKey = std::vector<int>;

// What the scheduler needs from the device side.  Every call comes from the
// serving thread, except footprint and budget (also from submitting
// threads).  Failures are thrown as Error.
struct Executor {
  virtual ~Executor() = default;
  // Device bytes the job will hold (admission size).
  virtual uint64_t footprint(const muster_job& j) = 0;
  // The whole budget (0 = unbounded): a job larger than this can never run.
  virtual uint64_t budget() = 0;
  // Whether `bytes` more fit the budget now.
  virtual bool fits(uint64_t bytes) = 0;
  // Create the job's device state and start its first level.
  virtual std::unique_ptr<JobHandle> admit(const muster_job& j) = 0;
  // One iteration of every job of a group: jobs that share window, metric
  // and K, all at a level with steps.  `sig` identifies the group's members
  // and their levels (the executor may keep a launch plan per group).
  virtual void step(const GroupKey& key, const std::vector<JobHandle*>& group,
                    const std::vector<std::pair<uint64_t, int>>& sig) = 0;
  // Groups that no longer exist (their plans may be dropped).
  virtual void forget_groups_except(const std::vector<GroupKey>& live) = 0;
  // After the tick's steps: make every resident job's state readable.
  virtual void sync(const std::vector<JobHandle*>& resident) = 0;
  virtual int level(JobHandle& h) = 0;
  virtual bool nonfinite(JobHandle& h) = 0;
  virtual void begin_level(JobHandle& h, int level) = 0;
  // The job's outputs and report after its last level.
  virtual void finish(JobHandle& h, double t_submit, muster_report* rep) = 0;
  virtual uint64_t held_bytes(JobHandle& h) = 0;
  // A device error ended the tick: every resident job fails with it.
  virtual void on_device_error() = 0;
};

struct Ticket {
  uint64_t id = 0;
  muster_job job{};
  std::unique_ptr<JobHandle> rt;
  int state = 0;                      // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
  muster_status status = MUSTER_OK;
  std::string err;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int level_iter = 0;                 // steps done at the current level
  int total_iter = 0;
  bool cancel = false;
  muster_report report{};
};

class Scheduler {
 public:
  Scheduler(Executor& ex, int max_queue, double (*clock)());
  // ---- client side (any thread); failures throw Error ----
  uint64_t submit(const muster_job& j);
  int poll(uint64_t id);
  // Blocks until the job is terminal; returns its status and releases it.
  muster_status wait(uint64_t id, muster_report* rep, std::string* err);
  void cancel(uint64_t id);
  void stats(int* resident, int* queued);
  // ---- serving side (one thread) ----
  // Blocks until there is work; false once stop() was called.
  bool wait_for_work();
  // One round: cancellations, admission, one iteration of every resident
  // job whose level has steps, level changes and retirement.
  void tick();
  // Stop serving: waiting and resident jobs end with E_CANCELLED.
  void stop();
  void shutdown();  // after the serving thread has left: fail what is left

 private:
  void finish_ticket(Ticket& t, int state, muster_status st, const std::string& err);
  Executor& ex_;
  int max_queue_;
  double (*clock_)();
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  bool stop_ = false;
  uint64_t next_id_ = 1;
  std::deque<std::shared_ptr<Ticket>> queue_;
  std::vector<std::shared_ptr<Ticket>> resident_;
  std::map<uint64_t, std::shared_ptr<Ticket>> all_;
};

}  // namespace muster
