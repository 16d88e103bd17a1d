// Serving loop: simulation requests of different sizes arrive at any time; a stepping
// thread admits them by device-memory footprint (Scheduler), keeps their state resident on
// the device, and advances every ready resident request by one time layer per batched step
// (all of their continua in the same PCG launches through the batch executor).  A setup
// thread creates each admitted problem (device allocation, coefficients, factors, optional
// autotuning) on the problem's own stream, so admission never stalls the resident requests'
// steps; a request joins the batch once its problem is ready.  Finished requests hand their
// final state to host memory and free their device memory, which admits the next ones.
// Only the library's C ABI is used here.
#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mcdec.h"
#include "scheduler.hpp"

namespace {

// Owned copy of a descriptor's arrays (the caller's arrays are valid only during submit).
struct HostDesc {
  mc_problem_desc d{};
  std::vector<double> k[2], src[2], p0[2], flen, edge_d, sigma_f, src_f, p0_f, well_q, well_p;
  std::vector<int32_t> host, edges;

  void take(const mc_problem_desc& in) {
    d = in;
    const size_t nc = (size_t)in.nx * in.ny * (in.nz > 1 ? in.nz : 1);
    auto cp = [](std::vector<double>& v, const double* a, size_t n) -> const double* {
      if (!a) return nullptr;
      v.assign(a, a + n);
      return v.data();
    };
    for (int a = 0; a < in.n_omega && a < 2; ++a) {
      d.omega[a].k = cp(k[a], in.omega[a].k, nc);
      d.omega[a].src = cp(src[a], in.omega[a].src, nc);
      d.omega[a].p0 = cp(p0[a], in.omega[a].p0, nc);
    }
    const size_t nf = in.nf > 0 ? in.nf : 0, ne = in.ne > 0 ? in.ne : 0;
    if (in.host && nf) {
      host.assign(in.host, in.host + nf);
      d.host = host.data();
    }
    if (in.edges && ne) {
      edges.assign(in.edges, in.edges + 2 * ne);
      d.edges = edges.data();
    }
    d.flen = cp(flen, in.flen, nf);
    d.edge_d = cp(edge_d, in.edge_d, ne);
    d.sigma_f = cp(sigma_f, in.sigma_f, (size_t)(in.n_omega > 0 ? in.n_omega : 0) * nf);
    d.src_f = cp(src_f, in.src_f, nf);
    d.p0_f = cp(p0_f, in.p0_f, nf);
    d.well_q = cp(well_q, in.well_q, nf);
    d.well_p = cp(well_p, in.well_p, nf);
  }
};

struct Request {
  uint64_t id = 0;
  std::unique_ptr<HostDesc> desc;       // until the problem is created
  mc_problem* prob = nullptr;
  int ncont = 0;
  int64_t dof = 0;
  std::vector<std::vector<double>> result;   // final state of a finished request
};

double now_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct mc_server {
  mc_server_config cfg{};
  mc_options opt{};
  mc_batch* batch = nullptr;
  std::unique_ptr<mc::Scheduler> sched;
  std::map<uint64_t, Request> reqs;
  std::mutex mu;
  std::condition_variable cv_work, cv_idle, cv_setup;
  std::thread worker, setup;
  bool stop = false;
  std::vector<uint64_t> pending;   // admitted, problem not created yet (setup thread's queue)
  int64_t setting_up = 0;          // problems being created right now
  uint64_t events = 0;             // submissions and finished setups (wakes the stepper)
  uint64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  // statistics (under mu)
  int64_t submitted = 0, finished = 0, failed = 0, steps = 0;
  int64_t finalizing = 0;   // finished, state still being copied to host memory
  double cell_updates = 0, busy = 0;
  std::string err, worker_err;
};

static thread_local std::string g_server_error;

namespace {

// Creates the admitted problems, oldest admission first; a failed creation fails the
// request and frees its bytes.
void run_setup(mc_server* S) {
  for (;;) {
    uint64_t id;
    Request* R;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_setup.wait(lk, [&] { return S->stop || !S->pending.empty(); });
      if (S->stop) return;
      id = S->pending.front();
      S->pending.erase(S->pending.begin());
      S->setting_up += 1;
      R = &S->reqs[id];
    }
    mc_problem* P = nullptr;
    mc_status st = mc_create_problem(&R->desc->d, &S->opt, &P);
    if (st == MC_OK && S->cfg.autotune) st = mc_autotune(&P, 1, 10);
    std::string why = st != MC_OK ? std::string(P ? mc_last_error(P) : mc_last_error(nullptr))
                                  : std::string();
    mc_info inf;
    if (st == MC_OK) mc_get_info(P, &inf);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (st != MC_OK) {
        if (P) mc_destroy(P);
        S->sched->fail(id, st, now_since(S->t0));
        S->failed += 1;
        S->worker_err = why;
      } else {
        R->ncont = inf.n_cont;
        for (int c = 0; c < inf.n_cont; ++c) R->dof += inf.sizes[c];
        R->prob = P;
      }
      R->desc.reset();
      S->setting_up -= 1;
      S->events += 1;
    }
    S->cv_work.notify_all();
    S->cv_idle.notify_all();
  }
}

void run_worker(mc_server* S) {
  std::vector<uint64_t> ids;
  std::vector<mc_problem*> probs;
  std::vector<mc_report> reps;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop) return;
      const std::vector<uint64_t> admitted = S->sched->admit(now_since(S->t0));
      if (!admitted.empty()) {
        S->pending.insert(S->pending.end(), admitted.begin(), admitted.end());
        S->cv_setup.notify_all();
      }
      // step the resident requests whose problems are ready
      ids.clear();
      probs.clear();
      for (uint64_t id : S->sched->resident()) {
        mc_problem* P = S->reqs[id].prob;
        if (P) {
          ids.push_back(id);
          probs.push_back(P);
        }
      }
      if (ids.empty()) {
        if (S->sched->n_resident() == 0 && S->sched->queued() == 0) S->cv_idle.notify_all();
        // wait for a submission or a finished setup
        const uint64_t seen = S->events;
        S->cv_work.wait(lk, [&] { return S->stop || S->events != seen; });
        continue;
      }
    }
    reps.assign(ids.size(), mc_report{});
    const double ta = now_since(S->t0);
    mc_status st = mc_batch_step(S->batch, probs.data(), (int32_t)probs.size(), 1, reps.data());
    const double tb = now_since(S->t0);
    std::vector<uint64_t> ok, bad;
    if (st == MC_OK || st == MC_ENOCONV || st == MC_EBREAKDOWN) {
      for (size_t i = 0; i < ids.size(); ++i) (reps[i].failed < 0 ? ok : bad).push_back(ids[i]);
    } else {
      bad = ids;   // a device or argument error: every stepped request fails
    }
    std::vector<uint64_t> done;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      done = S->sched->stepped(ok, ta, tb);
      S->finalizing += (int64_t)done.size();
      S->steps += 1;
      S->busy += tb - ta;
      for (uint64_t id : ok) S->cell_updates += (double)S->reqs[id].dof;
      for (uint64_t id : bad) {
        S->sched->fail(id, st == MC_OK ? MC_ENOCONV : st, tb);
        S->failed += 1;
        S->worker_err = mc_batch_last_error(S->batch);
      }
    }
    // finished or failed requests: final state to host memory, device memory released
    for (uint64_t id : done) {
      Request* R;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        R = &S->reqs[id];
      }
      mc_info inf;
      mc_get_info(R->prob, &inf);
      std::vector<std::vector<double>> res(inf.n_cont);
      for (int c = 0; c < inf.n_cont; ++c) {
        res[c].resize(inf.sizes[c]);
        mc_get_state(R->prob, c, res[c].data());
      }
      mc_destroy(R->prob);
      std::lock_guard<std::mutex> lk(S->mu);
      R->result = std::move(res);
      R->prob = nullptr;
      S->finished += 1;
      S->finalizing -= 1;
    }
    for (uint64_t id : bad) {
      std::lock_guard<std::mutex> lk(S->mu);
      Request& R = S->reqs[id];
      if (R.prob) mc_destroy(R.prob);
      R.prob = nullptr;
    }
    S->cv_idle.notify_all();
  }
}

}  // namespace

extern "C" {

mc_status mc_server_create(const mc_server_config* cfg, const mc_options* opt,
                           mc_server** out) {
  if (!out || !cfg) {
    g_server_error = "cfg and out are required";
    return MC_EINVAL;
  }
  *out = nullptr;
  if (cfg->hbm_budget <= 0 || cfg->max_resident < 0 || cfg->max_bypass < 0) {
    g_server_error = "hbm_budget must be > 0, max_resident and max_bypass >= 0";
    return MC_EINVAL;
  }
  mc_options o;
  mc_options_default(&o);
  if (opt) o = *opt;
  if (o.scheme == MC_SCHEME_L || o.scheme == MC_SCHEME_U || o.scheme == MC_SCHEME_COUPLED) {
    g_server_error = "the server runs the D or EX scheme";
    return MC_EINVAL;
  }
  mc_server* S = new mc_server();
  S->cfg = *cfg;
  if (S->cfg.max_resident == 0) S->cfg.max_resident = 256;
  mc_status st = mc_batch_create(&o, &S->batch);
  if (st != MC_OK) {
    g_server_error = mc_batch_last_error(nullptr);
    delete S;
    return st;
  }
  // each problem orders its setup on its own stream (the options' stream, or a stream of
  // its own when none is given); the batched steps run on the batch's stream
  S->opt = o;
  S->sched.reset(new mc::Scheduler(S->cfg.hbm_budget, S->cfg.max_resident, S->cfg.max_bypass));
  S->t0 = std::chrono::steady_clock::now();
  S->worker = std::thread(run_worker, S);
  S->setup = std::thread(run_setup, S);
  *out = S;
  return MC_OK;
}

mc_status mc_server_destroy(mc_server* S) {
  if (!S) return MC_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_setup.notify_all();
  if (S->worker.joinable()) S->worker.join();
  if (S->setup.joinable()) S->setup.join();
  for (auto& kv : S->reqs)
    if (kv.second.prob) mc_destroy(kv.second.prob);
  mc_batch_destroy(S->batch);
  delete S;
  return MC_OK;
}

mc_status mc_server_submit(mc_server* S, const mc_problem_desc* d, int32_t n_steps,
                           uint64_t* id) {
  if (!S) return MC_EINVAL;
  if (!d || !id || n_steps < 1) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = "desc, id and n_steps >= 1 are required";
    return MC_EINVAL;
  }
  int64_t bytes = 0;
  mc_footprint(d, &S->opt, &bytes);
  std::unique_ptr<HostDesc> hd(new HostDesc());
  hd->take(*d);
  std::lock_guard<std::mutex> lk(S->mu);
  const uint64_t rid = S->next_id++;
  if (!S->sched->submit(rid, bytes, n_steps, now_since(S->t0))) {
    S->err = "request needs " + std::to_string(bytes) + " device bytes, more than the budget " +
             std::to_string(S->cfg.hbm_budget);
    return MC_ENOMEM;
  }
  Request& R = S->reqs[rid];
  R.id = rid;
  R.desc = std::move(hd);
  S->submitted += 1;
  S->events += 1;
  *id = rid;
  S->cv_work.notify_all();
  return MC_OK;
}

mc_status mc_server_poll(mc_server* S, uint64_t id, mc_request_info* info) {
  if (!S || !info) return MC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  const mc::ReqMeta* m = S->sched->find(id);
  if (!m) {
    S->err = "unknown request " + std::to_string(id);
    return MC_ENOTFOUND;
  }
  auto f = S->reqs.find(id);
  // a finished request reports done once its state has reached host memory
  const bool finalizing = f != S->reqs.end() && f->second.prob && m->state == mc::REQ_DONE;
  info->state = finalizing ? mc::REQ_RUNNING : m->state;
  info->status = m->status;
  info->steps_done = m->steps_done;
  info->n_steps = m->n_steps;
  info->bytes = m->bytes;
  info->t_submit = m->t_submit;
  info->t_admit = m->t_admit;
  info->t_finish = m->t_finish;
  return MC_OK;
}

mc_status mc_server_fetch(mc_server* S, uint64_t id, int32_t alpha, double* out) {
  if (!S || !out) return MC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto f = S->reqs.find(id);
  const mc::ReqMeta* m = S->sched->find(id);
  if (f == S->reqs.end() || !m) {
    S->err = "unknown request " + std::to_string(id);
    return MC_ENOTFOUND;
  }
  if (m->state != mc::REQ_DONE || f->second.prob) {
    S->err = "request " + std::to_string(id) + " has not finished";
    return MC_EINVAL;
  }
  if (alpha < 0 || alpha >= (int)f->second.result.size()) {
    S->err = "alpha out of range";
    return MC_EINVAL;
  }
  const auto& v = f->second.result[alpha];
  std::memcpy(out, v.data(), v.size() * sizeof(double));
  return MC_OK;
}

mc_status mc_server_release(mc_server* S, uint64_t id) {
  if (!S) return MC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto f = S->reqs.find(id);
  if (f == S->reqs.end() || f->second.prob || !S->sched->forget(id)) {
    S->err = "request " + std::to_string(id) + " is unknown or still queued / running";
    return MC_EINVAL;
  }
  S->reqs.erase(id);
  return MC_OK;
}

mc_status mc_server_wait(mc_server* S, double timeout_s) {
  if (!S) return MC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto idle = [&] {
    return S->sched->queued() == 0 && S->sched->n_resident() == 0 && S->finalizing == 0 &&
           S->pending.empty() && S->setting_up == 0;
  };
  if (timeout_s < 0) {
    S->cv_idle.wait(lk, idle);
    return MC_OK;
  }
  if (!S->cv_idle.wait_for(lk, std::chrono::duration<double>(timeout_s), idle)) {
    S->err = "requests still queued or running after the timeout";
    return MC_ETIMEOUT;
  }
  return MC_OK;
}

mc_status mc_server_get_stats(mc_server* S, mc_server_stats* st) {
  if (!S || !st) return MC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(st, 0, sizeof(*st));
  st->submitted = S->submitted;
  st->finished = S->finished;
  st->failed = S->failed;
  st->queued = (int64_t)S->sched->queued();
  st->resident = (int64_t)S->sched->n_resident();
  st->bytes_in_use = S->sched->in_use();
  st->budget = S->sched->budget();
  st->steps = S->steps;
  st->cell_updates = S->cell_updates;
  st->busy_seconds = S->busy;
  st->elapsed_seconds = now_since(S->t0);
  return MC_OK;
}

mc_status mc_server_step_seconds(mc_server* S, double* out, int64_t cap, int64_t* n) {
  if (!S || !n) return MC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  const auto& v = S->sched->step_seconds();
  *n = (int64_t)v.size();
  if (out)
    for (int64_t i = 0; i < cap && i < (int64_t)v.size(); ++i) out[i] = v[i];
  return MC_OK;
}

const char* mc_server_last_error(const mc_server* S) {
  if (!S) return g_server_error.c_str();
  mc_server* M = const_cast<mc_server*>(S);
  std::lock_guard<std::mutex> lk(M->mu);
  g_server_error = S->err.empty() ? S->worker_err : S->err;
  return g_server_error.c_str();
}

}  // extern "C"
