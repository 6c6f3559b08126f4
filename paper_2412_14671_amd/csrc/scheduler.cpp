// Continuous-batching scheduler (see scheduler.h).
#include "scheduler.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>

namespace muster {

namespace {
[[noreturn]] void sched_fail(muster_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error{st, buf};
}
}  // namespace

Scheduler::Scheduler(Executor& ex, int max_queue, double (*clock)())
    : ex_(ex), max_queue_(max_queue), clock_(clock) {}

uint64_t Scheduler::submit(const muster_job& j) {
  const uint64_t fp = ex_.footprint(j);
  const uint64_t budget = ex_.budget();
  if (budget != 0 && fp > budget)
    sched_fail(MUSTER_E_NOMEM, "job footprint %llu exceeds the context budget %llu",
               (unsigned long long)fp, (unsigned long long)budget);
  std::lock_guard<std::mutex> lk(mu_);
  if (stop_) sched_fail(MUSTER_E_CANCELLED, "server stopped");
  if ((int)queue_.size() >= max_queue_) sched_fail(MUSTER_E_BUSY, "serving queue is full");
  auto t = std::make_shared<Ticket>();
  t->id = next_id_++;
  t->job = j;
  t->t_submit = clock_();
  queue_.push_back(t);
  all_[t->id] = t;
  cv_.notify_all();
  return t->id;
}

int Scheduler::poll(uint64_t id) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) sched_fail(MUSTER_E_INVALID, "unknown ticket %llu", (unsigned long long)id);
  return it->second->state;
}

muster_status Scheduler::wait(uint64_t id, muster_report* rep, std::string* err) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) sched_fail(MUSTER_E_INVALID, "unknown ticket %llu", (unsigned long long)id);
  auto t = it->second;
  done_cv_.wait(lk, [&] { return t->state >= 2; });
  if (rep) *rep = t->report;
  if (err) *err = t->err;
  all_.erase(id);
  return t->status;
}

void Scheduler::cancel(uint64_t id) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = all_.find(id);
  if (it == all_.end()) sched_fail(MUSTER_E_INVALID, "unknown ticket %llu", (unsigned long long)id);
  it->second->cancel = true;
  cv_.notify_all();
}

void Scheduler::stats(int* resident, int* queued) {
  std::lock_guard<std::mutex> lk(mu_);
  if (resident) *resident = (int)resident_.size();
  if (queued) *queued = (int)queue_.size();
}

bool Scheduler::wait_for_work() {
  std::unique_lock<std::mutex> lk(mu_);
  cv_.wait(lk, [&] { return stop_ || !queue_.empty() || !resident_.empty(); });
  return !stop_;
}

void Scheduler::stop() {
  std::lock_guard<std::mutex> lk(mu_);
  stop_ = true;
  cv_.notify_all();
}

// Caller holds mu_.
void Scheduler::finish_ticket(Ticket& t, int state, muster_status st, const std::string& err) {
  if (t.rt) {
    t.report.footprint_bytes = ex_.held_bytes(*t.rt);
    t.rt.reset();
  }
  t.state = state;
  t.status = st;
  t.err = err;
  t.t_done = clock_();
  t.report.status = st;
  t.report.seconds = t.t_done - t.t_submit;
  t.report.queue_seconds = (t.t_admit > 0 ? t.t_admit : t.t_done) - t.t_submit;
  t.report.iterations = t.total_iter;
}

void Scheduler::tick() {
  std::vector<std::shared_ptr<Ticket>> admit;
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return;
    for (auto it = queue_.begin(); it != queue_.end();) {
      if ((*it)->cancel) {
        finish_ticket(**it, 4, MUSTER_E_CANCELLED, "cancelled");
        it = queue_.erase(it);
      } else {
        ++it;
      }
    }
    for (auto it = resident_.begin(); it != resident_.end();) {
      if ((*it)->cancel) {
        finish_ticket(**it, 4, MUSTER_E_CANCELLED, "cancelled");
        it = resident_.erase(it);
      } else {
        ++it;
      }
    }
    // admission by footprint, first come first served; a job that cannot
    // share launches with the residents (another window, metric or K) runs
    // in a group of its own in the same ticks
    uint64_t pending = 0;
    while (!queue_.empty()) {
      auto& t = queue_.front();
      const uint64_t fp = ex_.footprint(t->job);
      if (!ex_.fits(pending + fp)) break;
      pending += fp;
      admit.push_back(t);
      queue_.pop_front();
    }
    done_cv_.notify_all();
  }
  for (auto& t : admit) {
    try {
      auto h = ex_.admit(t->job);
      std::lock_guard<std::mutex> lk(mu_);
      t->rt = std::move(h);
      t->t_admit = clock_();
      t->state = 1;
      resident_.push_back(t);
    } catch (const Error& e) {
      std::lock_guard<std::mutex> lk(mu_);
      finish_ticket(*t, 3, e.st, e.msg);
      if (e.st == MUSTER_E_DEVICE) ex_.on_device_error();
      done_cv_.notify_all();
    }
  }
  std::vector<std::shared_ptr<Ticket>> res;
  {
    std::lock_guard<std::mutex> lk(mu_);
    res = resident_;
  }
  if (res.empty()) return;
  try {
    // one iteration of every resident job whose current level has steps (a
    // level of 0 steps is passed over below without touching the job)
    std::map<GroupKey, std::vector<JobHandle*>> groups;
    std::map<GroupKey, std::vector<std::pair<uint64_t, int>>> sigs;
    std::vector<JobHandle*> all;
    for (auto& t : res) {
      all.push_back(t->rt.get());
      const int lv = ex_.level(*t->rt);
      if (t->job.params.iters[lv] <= 0) continue;
      const GroupKey k{t->job.params.window, t->job.params.metric, t->job.params.K};
      groups[k].push_back(t->rt.get());
      sigs[k].push_back({t->id, lv});
    }
    std::vector<GroupKey> live;
    for (auto& g : groups) live.push_back(g.first);
    ex_.forget_groups_except(live);
    for (auto& g : groups) ex_.step(g.first, g.second, sigs[g.first]);
    ex_.sync(all);
    std::vector<std::shared_ptr<Ticket>> done;
    for (auto& t : res) {
      JobHandle& h = *t->rt;
      const int lv = ex_.level(h);
      const int T = t->job.params.iters[lv];
      if (T > 0) {
        t->level_iter++;
        t->total_iter++;
      }
      if (ex_.nonfinite(h)) {
        done.push_back(t);
        continue;
      }
      if (t->level_iter >= T) {
        if (lv + 1 < t->job.params.levels) {
          ex_.begin_level(h, lv + 1);
          t->level_iter = 0;
        } else {
          ex_.finish(h, t->t_submit, &t->report);
          done.push_back(t);
        }
      }
    }
    if (!done.empty()) {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& t : done) {
        const bool nf = t->rt && ex_.nonfinite(*t->rt);
        finish_ticket(*t, nf ? 3 : 2, nf ? MUSTER_E_NONFINITE : MUSTER_OK,
                      nf ? "the loss became non-finite" : "");
        resident_.erase(std::remove(resident_.begin(), resident_.end(), t), resident_.end());
      }
      done_cv_.notify_all();
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> lk(mu_);
    if (e.st == MUSTER_E_DEVICE) ex_.on_device_error();
    for (auto& t : resident_) finish_ticket(*t, 3, e.st, e.msg);
    resident_.clear();
    ex_.forget_groups_except({});
    done_cv_.notify_all();
  }
}

void Scheduler::shutdown() {
  std::lock_guard<std::mutex> lk(mu_);
  stop_ = true;
  for (auto& t : queue_) finish_ticket(*t, 4, MUSTER_E_CANCELLED, "server stopped");
  for (auto& t : resident_) finish_ticket(*t, 4, MUSTER_E_CANCELLED, "server stopped");
  queue_.clear();
  resident_.clear();
  done_cv_.notify_all();
}

}  // namespace muster
