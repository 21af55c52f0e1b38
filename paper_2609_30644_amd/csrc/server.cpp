// Serving planning requests with continuous batching (mrpop_server_*).
//
// One scheduling thread owns a JobEngine.  Between merged launches it retires
// finished requests (freeing their device memory), admits queued requests in
// arrival order while a slot is free and the memory budget holds, and starts
// them; their work joins the next merged launch.  Submitters only touch the
// queue; results are kept per ticket until released.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"

using namespace mrpop;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t ticket;
  const mrpop_scene *scene;
  std::vector<float> qs, qg;
  mrpop_plan_params params;
  double t_submit;
};

struct Result {
  mrpop_server_result r;
  std::vector<float> path;
};

}  // namespace

struct mrpop_server {
  mrpop_ctx *ctx = nullptr;
  mrpop_server_config cfg{};
  double t0 = 0.0;
  std::unique_ptr<JobEngine> eng;
  std::thread loop;

  // queue and results (qmu)
  std::mutex qmu;
  std::condition_variable cv_done;
  std::deque<Request> queue;
  std::unordered_map<int64_t, Result> results;
  int64_t next_ticket = 1;
  mrpop_server_stats st{};

  // scheduling thread only (slot table), plus what on_done writes under the
  // engine's lock
  struct Slot {
    std::unique_ptr<PlanJob> job;
    int64_t ticket = 0;
    size_t bytes = 0;
    mrpop_status status = MRPOP_PENDING;
    double t_admit = 0.0, t_done = 0.0, t_submit = 0.0;
  };
  std::vector<Slot> slots;
  size_t reserved = 0;

  std::atomic<int> queued{0};
  std::atomic<bool> stop{false};

  double clock() const { return now_s() - t0; }
  void run();
  void retire();  // records finished requests and frees their memory
  void finish(int64_t ticket, const Result &res);
};

void mrpop_server::finish(int64_t ticket, const Result &res) {
  std::lock_guard<std::mutex> lk(qmu);
  results[ticket] = res;
  ++st.completed;
  cv_done.notify_all();
}

void mrpop_server::retire() {
  for (int k : eng->reap()) {
    Slot &sl = slots[k];
    Result res;
    std::memset(&res.r, 0, sizeof(res.r));
    res.r.status = sl.status;
    res.r.stats = sl.job->stats();
    res.r.t_submit = sl.t_submit;
    res.r.t_admit = sl.t_admit;
    res.r.t_done = sl.t_done;
    res.r.device_bytes = (int64_t)sl.bytes;
    res.r.cost = INFINITY;
    if (sl.status == MRPOP_OK) {
      res.path = sl.job->path();
      res.r.path_len = (int32_t)(res.path.size() / sl.job->dof());
      res.r.cost = sl.job->cost();
    }
    sl.job.reset();  // frees its device memory (the stream is idle here)
    reserved -= sl.bytes;
    sl.bytes = 0;
    finish(sl.ticket, res);
  }
}

void mrpop_server::run() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    retire();
    // admit in arrival order while a slot is free and the budget holds
    for (;;) {
      Request rq;
      size_t need = 0;
      {
        std::lock_guard<std::mutex> lk(qmu);
        if (queue.empty()) break;
        const Request &f = queue.front();
        need = PlanJob::device_bytes_for(f.scene, f.params);
        const size_t budget = (size_t)cfg.mem_budget_bytes;
        if (budget && need > budget) {  // can never fit
          Result res;
          std::memset(&res.r, 0, sizeof(res.r));
          res.r.status = MRPOP_E_NOMEM;
          res.r.cost = INFINITY;
          res.r.t_submit = f.t_submit;
          res.r.t_admit = res.r.t_done = clock();
          results[f.ticket] = res;
          ++st.rejected;
          ++st.completed;
          queue.pop_front();
          --queued;
          cv_done.notify_all();
          continue;
        }
        if (eng->free_slots() == 0) break;
        if (budget && reserved + need > budget) break;
        rq = std::move(queue.front());
        queue.pop_front();
        --queued;
        ++st.admitted;
      }
      std::unique_ptr<PlanJob> job(new PlanJob());
      const double t_admit = clock();
      mrpop_status ps = job->prepare(ctx, rq.scene, rq.qs.data(), rq.qg.data(), rq.params);
      if (ps != MRPOP_OK) {
        Result res;
        std::memset(&res.r, 0, sizeof(res.r));
        res.r.status = ps;
        res.r.cost = INFINITY;
        res.r.t_submit = rq.t_submit;
        res.r.t_admit = t_admit;
        res.r.t_done = clock();
        finish(rq.ticket, res);
        continue;
      }
      PlanJob *jp = job.get();
      mrpop_server *self = this;
      // The slot record below is filled before the job can end: a job ends
      // only after a merged launch, which this thread makes.
      const int k = eng->start(jp, [self](int slot, mrpop_status s) {
        self->slots[slot].status = s;
        self->slots[slot].t_done = self->clock();
      });
      if (k < 0) {  // no free slot after all (only this thread takes slots): queue it again
        std::lock_guard<std::mutex> lk(qmu);
        --st.admitted;
        queue.push_front(std::move(rq));
        ++queued;
        break;
      }
      Slot &sl = slots[k];
      sl.job = std::move(job);
      sl.ticket = rq.ticket;
      sl.bytes = need;
      sl.t_submit = rq.t_submit;
      sl.t_admit = t_admit;
      reserved += need;
      {
        std::lock_guard<std::mutex> lk(qmu);
        st.reserved_bytes = (int64_t)reserved;
        st.peak_reserved_bytes = std::max<int64_t>(st.peak_reserved_bytes, (int64_t)reserved);
        st.running = eng->running();
        st.max_running = std::max(st.max_running, st.running);
      }
    }
    if (stop && queued == 0 && eng->running() == 0) {
      retire();
      break;
    }
    // one merged launch (or wait for arrivals / finished requests)
    eng->step([this] { return stop.load() || queued.load() > 0; });
    {
      std::lock_guard<std::mutex> lk(qmu);
      st.flushes = eng->flushes();
      st.launches = eng->launches();
      st.running = eng->running();
      st.queue_len = (int32_t)queue.size();
    }
  }
}

extern "C" {

mrpop_status mrpop_server_create(mrpop_ctx *ctx, const mrpop_server_config *cfg, mrpop_server **out) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "server_create: ctx is NULL");
  if (!cfg || !out || cfg->max_slots < 1 || cfg->max_slots > 4096 || cfg->mem_budget_bytes < 0)
    return fail(ctx, MRPOP_E_INVALID_ARG, "server_create: bad config");
  mrpop_server *s = new mrpop_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  s->t0 = now_s();
  s->eng.reset(new JobEngine(ctx, nullptr, cfg->max_slots));
  s->slots.resize(cfg->max_slots);
  s->loop = std::thread([s] { s->run(); });
  *out = s;
  return MRPOP_OK;
}

void mrpop_server_destroy(mrpop_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->qmu);
    srv->queued -= (int)srv->queue.size();
    srv->queue.clear();
  }
  srv->stop = true;
  srv->eng->notify();
  if (srv->loop.joinable()) srv->loop.join();
  delete srv;
}

mrpop_status mrpop_server_submit(mrpop_server *srv, const mrpop_scene *scene, const float *q_start,
                                 const float *q_goal, const mrpop_plan_params *params, int64_t *ticket) {
  if (!srv) return fail(nullptr, MRPOP_E_INVALID_ARG, "server_submit: server is NULL");
  if (!scene || scene->ctx != srv->ctx || !q_start || !q_goal || !params || !ticket)
    return fail(srv->ctx, MRPOP_E_INVALID_ARG, "server_submit: bad argument");
  Request rq;
  rq.scene = scene;
  rq.qs.assign(q_start, q_start + scene->dof);
  rq.qg.assign(q_goal, q_goal + scene->dof);
  rq.params = *params;
  {
    std::lock_guard<std::mutex> lk(srv->qmu);
    rq.ticket = srv->next_ticket++;
    rq.t_submit = srv->clock();
    Result pend;
    std::memset(&pend.r, 0, sizeof(pend.r));
    pend.r.status = MRPOP_PENDING;
    pend.r.cost = INFINITY;
    pend.r.t_submit = rq.t_submit;
    srv->results[rq.ticket] = pend;
    *ticket = rq.ticket;
    srv->queue.push_back(std::move(rq));
    ++srv->queued;
    ++srv->st.submitted;
    srv->st.queue_len = (int32_t)srv->queue.size();
    srv->st.max_queue_len = std::max(srv->st.max_queue_len, srv->st.queue_len);
  }
  srv->eng->notify();
  return MRPOP_OK;
}

mrpop_status mrpop_server_poll(mrpop_server *srv, int64_t ticket, mrpop_server_result *out) {
  if (!srv || !out) return MRPOP_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->qmu);
  auto it = srv->results.find(ticket);
  if (it == srv->results.end()) return MRPOP_E_INVALID_ARG;
  *out = it->second.r;
  return MRPOP_OK;
}

mrpop_status mrpop_server_wait(mrpop_server *srv, int64_t ticket, double timeout_s, mrpop_server_result *out) {
  if (!srv || !out) return MRPOP_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(srv->qmu);
  auto done = [&] {
    auto it = srv->results.find(ticket);
    return it == srv->results.end() || it->second.r.status != MRPOP_PENDING;
  };
  srv->cv_done.wait_for(lk, std::chrono::duration<double>(std::max(0.0, timeout_s)), done);
  auto it = srv->results.find(ticket);
  if (it == srv->results.end()) return MRPOP_E_INVALID_ARG;
  *out = it->second.r;
  return MRPOP_OK;
}

mrpop_status mrpop_server_path(mrpop_server *srv, int64_t ticket, float *path_out, int32_t cap) {
  if (!srv) return MRPOP_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->qmu);
  auto it = srv->results.find(ticket);
  if (it == srv->results.end() || it->second.r.status != MRPOP_OK) return MRPOP_E_INVALID_ARG;
  if (it->second.r.path_len > cap || !path_out) return MRPOP_E_BUFFER;
  std::memcpy(path_out, it->second.path.data(), sizeof(float) * it->second.path.size());
  return MRPOP_OK;
}

mrpop_status mrpop_server_release(mrpop_server *srv, int64_t ticket) {
  if (!srv) return MRPOP_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->qmu);
  auto it = srv->results.find(ticket);
  if (it == srv->results.end() || it->second.r.status == MRPOP_PENDING) return MRPOP_E_INVALID_ARG;
  srv->results.erase(it);
  return MRPOP_OK;
}

mrpop_status mrpop_server_get_stats(mrpop_server *srv, mrpop_server_stats *out) {
  if (!srv || !out) return MRPOP_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(srv->qmu);
  *out = srv->st;
  return MRPOP_OK;
}

double mrpop_server_clock(const mrpop_server *srv) { return srv ? srv->clock() : 0.0; }

}  // extern "C"
