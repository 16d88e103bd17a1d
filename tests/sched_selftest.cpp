// CPU self-test of the serving scheduler (admission by footprint, bounded bypass, resident
// slots, completion and failure).  Built and run by tests/test_scheduler.py with g++; the
// GPU executor is replaced by a fake that finishes one layer per step.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "../paper_2209_01158_amd/csrc/scheduler.hpp"

using mc::Scheduler;

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);          \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static bool has(const std::vector<uint64_t>& v, uint64_t x) {
  for (auto y : v)
    if (y == x) return true;
  return false;
}

static void fixed_scenarios() {
  {  // first fit behind a head that does not fit, then the head once memory frees up
    Scheduler s(100, 10, 8);
    CHECK(s.submit(1, 60, 2, 0.0));
    CHECK(s.submit(2, 50, 1, 0.1));
    CHECK(s.submit(3, 30, 1, 0.2));
    CHECK(s.submit(4, 20, 1, 0.3));
    auto a = s.admit(1.0);
    CHECK(a.size() == 2 && a[0] == 1 && a[1] == 3);
    CHECK(s.in_use() == 90 && s.queued() == 2);
    CHECK(s.find(2)->bypassed == 1);
    auto d = s.stepped({1, 3}, 1.0, 2.0);   // 3 finishes (1 layer), 1 has one more
    CHECK(d.size() == 1 && d[0] == 3);
    CHECK(s.in_use() == 60);
    a = s.admit(2.0);                        // 2 (50) still does not fit; 4 (20) does
    CHECK(a.size() == 1 && a[0] == 4);
    d = s.stepped({1, 4}, 2.0, 3.0);
    CHECK(d.size() == 2);
    a = s.admit(3.0);
    CHECK(a.size() == 1 && a[0] == 2);
    CHECK(s.find(2)->t_admit == 3.0 && s.find(2)->t_submit == 0.1);
    CHECK(s.find(1)->t_finish == 3.0 && s.find(1)->steps_done == 2);
  }
  {  // bounded bypass: after max_bypass admissions past it, the head blocks the queue
    Scheduler s(100, 10, 1);
    s.submit(1, 70, 5, 0);
    s.submit(2, 50, 1, 0);
    s.submit(3, 10, 1, 0);
    s.submit(4, 10, 1, 0);
    auto a = s.admit(0);
    CHECK(a.size() == 2 && a[0] == 1 && a[1] == 3);   // one bypass of head 2, then it blocks
    CHECK(!has(a, 4));
  }
  {  // never fits / invalid
    Scheduler s(100, 4, 8);
    CHECK(!s.submit(1, 101, 1, 0));
    CHECK(!s.submit(2, -1, 1, 0));
    CHECK(!s.submit(3, 10, 0, 0));
    CHECK(s.submit(4, 100, 1, 0));
    CHECK(!s.submit(4, 10, 1, 0));            // duplicate id
  }
  {  // resident-slot limit
    Scheduler s(1000, 2, 8);
    for (int i = 1; i <= 5; ++i) s.submit(i, 10, 1, 0);
    auto a = s.admit(0);
    CHECK(a.size() == 2 && s.n_resident() == 2 && s.queued() == 3);
  }
  {  // failure frees memory; forget only finished or failed requests
    Scheduler s(100, 10, 8);
    s.submit(1, 80, 3, 0);
    s.submit(2, 80, 1, 0);
    s.admit(0);
    CHECK(!s.forget(1) && !s.forget(2));
    s.fail(1, -3, 0.5);
    CHECK(s.in_use() == 0 && s.find(1)->state == mc::REQ_FAILED && s.find(1)->status == -3);
    auto a = s.admit(0.5);
    CHECK(a.size() == 1 && a[0] == 2);
    CHECK(s.forget(1));
    CHECK(s.find(1) == nullptr);
    s.fail(2, -4, 0.6);
    CHECK(s.in_use() == 0 && s.n_resident() == 0);
  }
}

// Random arrivals of random sizes and lengths against a fake executor: memory and slot
// limits hold at every step, the charged bytes match the resident set, every request ends
// (done or failed), each head is bypassed at most max_bypass times, and timestamps are
// ordered.
static void random_simulation(unsigned seed) {
  std::mt19937_64 rng(seed);
  const int64_t budget = 1000;
  const int max_res = 6, max_bypass = 3;
  Scheduler s(budget, max_res, max_bypass);
  std::uniform_int_distribution<int> size(1, 600), len(1, 12), arrivals(0, 7);
  uint64_t next = 1;
  int submitted = 0;
  std::vector<uint64_t> admit_order;
  double t = 0;
  // arrivals (about one every 8 steps, below the capacity on average but in bursts) for
  // 3000 steps, then the queue drains
  for (int step = 0; step < 100000; ++step, t += 1.0) {
    if (step >= 3000 && s.queued() == 0 && s.n_resident() == 0) break;
    if (step < 3000 && arrivals(rng) == 0)
      for (int k = 1 + (int)(rng() % 3); k > 0; --k) {
        CHECK(s.submit(next++, size(rng), len(rng), t));
        ++submitted;
      }
    for (auto id : s.admit(t)) admit_order.push_back(id);
    CHECK(s.in_use() <= budget);
    CHECK((int)s.n_resident() <= max_res);
    int64_t sum = 0;
    for (auto id : s.resident()) sum += s.find(id)->bytes;
    CHECK(sum == s.in_use());
    auto res = s.resident();
    if (!res.empty() && (rng() % 97) == 0) s.fail(res[rng() % res.size()], -3, t);
    s.stepped(s.resident(), t, t + 1.0);
  }
  CHECK(s.queued() == 0 && s.n_resident() == 0 && s.in_use() == 0);
  int done = 0;
  for (uint64_t id = 1; id < next; ++id) {
    const mc::ReqMeta* m = s.find(id);
    CHECK(m && (m->state == mc::REQ_DONE || m->state == mc::REQ_FAILED));
    CHECK(m->bypassed <= max_bypass);
    if (m->state == mc::REQ_DONE) {
      ++done;
      CHECK(m->steps_done == m->n_steps);
      CHECK(m->t_admit >= m->t_submit && m->t_finish > m->t_admit);
    }
  }
  CHECK((int)admit_order.size() <= submitted);
  if (done == 0) CHECK(false);
}

int main() {
  fixed_scenarios();
  for (unsigned seed = 1; seed <= 20; ++seed) random_simulation(seed);
  if (failures) {
    std::printf("%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
