#include "scheduler.hpp"

#include <algorithm>

namespace mc {

Scheduler::Scheduler(int64_t budget, int max_resident, int max_bypass)
    : budget_(budget), max_resident_(std::max(1, max_resident)),
      max_bypass_(std::max(0, max_bypass)) {}

bool Scheduler::submit(uint64_t id, int64_t bytes, int n_steps, double t) {
  if (bytes < 0 || bytes > budget_ || n_steps < 1 || reqs_.count(id)) return false;
  ReqMeta m;
  m.id = id;
  m.bytes = bytes;
  m.n_steps = n_steps;
  m.t_submit = t;
  reqs_[id] = m;
  queue_.push_back(id);
  return true;
}

std::vector<uint64_t> Scheduler::admit(double t) {
  std::vector<uint64_t> out;
  auto it = queue_.begin();
  while (it != queue_.end() && (int)resident_.size() < max_resident_) {
    ReqMeta& m = reqs_[*it];
    const bool fits = in_use_ + m.bytes <= budget_;
    if (fits) {
      // a request behind the head only if the head may still be bypassed
      if (it != queue_.begin()) {
        ReqMeta& head = reqs_[queue_.front()];
        if (head.bypassed >= max_bypass_) break;
        head.bypassed += 1;
      }
      m.state = REQ_RUNNING;
      m.t_admit = t;
      in_use_ += m.bytes;
      resident_.push_back(m.id);
      out.push_back(m.id);
      it = queue_.erase(it);
      continue;
    }
    if (it == queue_.begin() && m.bypassed >= max_bypass_) break;   // head reserved
    ++it;
  }
  return out;
}

std::vector<uint64_t> Scheduler::stepped(const std::vector<uint64_t>& ids, double t0,
                                         double t1) {
  step_s_.push_back(t1 - t0);
  std::vector<uint64_t> done;
  for (uint64_t id : ids) {
    auto f = reqs_.find(id);
    if (f == reqs_.end() || f->second.state != REQ_RUNNING) continue;
    ReqMeta& m = f->second;
    m.steps_done += 1;
    if (m.steps_done >= m.n_steps) {
      m.state = REQ_DONE;
      m.t_finish = t1;
      in_use_ -= m.bytes;
      resident_.erase(std::find(resident_.begin(), resident_.end(), id));
      done.push_back(id);
    }
  }
  return done;
}

void Scheduler::fail(uint64_t id, int status, double t) {
  auto f = reqs_.find(id);
  if (f == reqs_.end()) return;
  ReqMeta& m = f->second;
  if (m.state == REQ_RUNNING) {
    in_use_ -= m.bytes;
    resident_.erase(std::find(resident_.begin(), resident_.end(), id));
  } else if (m.state == REQ_QUEUED) {
    queue_.erase(std::find(queue_.begin(), queue_.end(), id));
  }
  m.state = REQ_FAILED;
  m.status = status;
  m.t_finish = t;
}

void Scheduler::recharge(uint64_t id, int64_t bytes) {
  auto f = reqs_.find(id);
  if (f == reqs_.end() || f->second.state != REQ_RUNNING) return;
  in_use_ += bytes - f->second.bytes;
  f->second.bytes = bytes;
}

std::vector<uint64_t> Scheduler::resident() const { return resident_; }

const ReqMeta* Scheduler::find(uint64_t id) const {
  auto f = reqs_.find(id);
  return f == reqs_.end() ? nullptr : &f->second;
}

bool Scheduler::forget(uint64_t id) {
  auto f = reqs_.find(id);
  if (f == reqs_.end()) return false;
  if (f->second.state == REQ_QUEUED || f->second.state == REQ_RUNNING) return false;
  reqs_.erase(f);
  return true;
}

}  // namespace mc
