// Admission and bookkeeping of the serving loop: which simulation requests are resident on
// the GPU, which wait, how much device memory they hold, and their timestamps.  Plain C++
// (no HIP), so the policy is tested on the CPU with a fake executor.
//
// Policy.  A request asks for `bytes` of device memory (its footprint) and `n_steps` time
// layers.  Requests are admitted in arrival order while they fit the memory budget and the
// resident-slot limit.  A later request may bypass a waiting head that does not fit, but the
// head can be bypassed at most `max_bypass` times; after that nothing behind it is admitted
// until it is.  A request larger than the whole budget is refused at submission.  Every
// resident request advances by one layer per server step; it leaves when its last layer is
// done or its solve fails, freeing its bytes.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <map>
#include <vector>

namespace mc {

enum ReqState { REQ_QUEUED = 0, REQ_RUNNING = 1, REQ_DONE = 2, REQ_FAILED = 3 };

struct ReqMeta {
  uint64_t id = 0;
  int64_t bytes = 0;
  int n_steps = 0;
  int steps_done = 0;
  int state = REQ_QUEUED;
  int status = 0;          // library status of a failed request
  int bypassed = 0;        // times a later request was admitted while this one waited
  double t_submit = 0, t_admit = -1, t_finish = -1;
};

class Scheduler {
 public:
  Scheduler(int64_t budget, int max_resident, int max_bypass = 8);

  // Queue a request; false if it can never fit (bytes > budget or bytes < 0).
  bool submit(uint64_t id, int64_t bytes, int n_steps, double t);

  // Admit queued requests under the policy; returns the admitted ids in admission order.
  std::vector<uint64_t> admit(double t);

  // The resident requests `ids` completed one layer between t0 and t1; returns the ids that
  // finished with it (they leave the resident set and free their bytes).
  std::vector<uint64_t> stepped(const std::vector<uint64_t>& ids, double t0, double t1);

  // A resident (or admitted) request failed: it leaves with its bytes freed.
  void fail(uint64_t id, int status, double t);

  // Correct the bytes charged for a resident request (e.g. the measured footprint).
  void recharge(uint64_t id, int64_t bytes);

  std::vector<uint64_t> resident() const;
  const ReqMeta* find(uint64_t id) const;
  bool forget(uint64_t id);   // drop a finished or failed request's record

  int64_t budget() const { return budget_; }
  int64_t in_use() const { return in_use_; }
  size_t queued() const { return queue_.size(); }
  size_t n_resident() const { return resident_.size(); }
  const std::vector<double>& step_seconds() const { return step_s_; }

 private:
  int64_t budget_, in_use_ = 0;
  int max_resident_, max_bypass_;
  std::deque<uint64_t> queue_;
  std::vector<uint64_t> resident_;   // admission order
  std::map<uint64_t, ReqMeta> reqs_;
  std::vector<double> step_s_;       // duration of every server step
};

}  // namespace mc
