// Many independent planning instances at once (mrpop_plan_batch).
//
// Every instance is a PlanJob coroutine driven by one host thread: its
// device work goes to a queue of its own instead of a stream, and at each
// synchronisation point it is parked.  Once every running instance is
// parked, the work of all of them is merged and launched on one stream:
// layer by layer (the next command of every instance), commands of one kind
// in one launch over all instances' argument records (a device-resident
// table of records), and the validations of a layer in one many-scene
// launch.  Then every parked instance is resumed.  An instance's commands
// keep their order, and each instance computes exactly what it computes
// alone: the batch changes when work runs, never what it computes.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "batch.h"

namespace mrpop {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Grow-only buffers.
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    const size_t want = std::max(bytes, n * 2);
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) n = want;
    return e;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct HostBuf {
  unsigned char *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    const size_t want = std::max(bytes, n * 2);
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipHostMalloc((void **)&p, want);
    if (e == hipSuccess) n = want;
    return e;
  }
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
};

}  // namespace

class QueuedExec;

struct JobEngine::Impl {
  mrpop_ctx *ctx;
  hipStream_t s;
  std::mutex mu;  // guards only the wake-up of an idle step() (notify from other threads)
  std::condition_variable cv_main;
  struct Slot {
    std::vector<Cmd> pending;
    bool used = false, running = false, parked = false, finished = false;
    PlanJob *job = nullptr;
    std::function<void(int, mrpop_status)> on_done;
    std::unique_ptr<QueuedExec> ex;
    Task<mrpop_status> task;
    std::coroutine_handle<> resume_at;  // where the job continues (innermost parked coroutine)
  };
  std::vector<Slot> slots;  // fixed capacity
  int n_running = 0, n_finished = 0;  // finished: ended, not yet reaped
  hipError_t last_err = hipSuccess;
  // merge buffers
  HostBuf h_args;
  DevBuf d_args, seg_scratch;
  int64_t flushes = 0, launches = 0;
  static constexpr int kMaxPerLaunch = 65535;

  Impl(mrpop_ctx *c, hipStream_t st, int cap) : ctx(c), s(st), slots(cap) {}
  hipError_t flush();
};

// Device work of one slot, queued for the next merged launch; a
// synchronisation parks the slot's coroutine until that launch has completed.
class QueuedExec : public Exec {
 public:
  QueuedExec(JobEngine::Impl *e, int k) : e_(e), k_(k) {}
  hipError_t submit(const Cmd &c) override {
    e_->slots[k_].pending.push_back(c);
    return hipSuccess;
  }
  hipError_t sync() override { return hipErrorNotSupported; }  // (deferred: never called)
  bool deferred() const override { return true; }
  void park(std::coroutine_handle<> h) override {
    JobEngine::Impl::Slot &sl = e_->slots[k_];
    sl.resume_at = h;
    sl.parked = true;
  }
  hipError_t resumed_status() override { return e_->last_err; }

 private:
  JobEngine::Impl *e_;
  int k_;
};

hipError_t JobEngine::Impl::flush() {
  const int K = (int)slots.size();
  std::vector<size_t> head(K, 0);
  last_err = hipSuccess;
  // plan every layer: (op, records), packing argument records into h_args
  struct Launch {
    Op op;
    size_t off;   // byte offset of the records in the argument buffer
    int count;    // records
    int grid_x;   // blocks (Validate: flat edges)
    int r_max;
  };
  std::vector<Launch> plan;
  std::vector<unsigned char> packed;
  auto put = [&](const void *p, size_t n) -> size_t {
    const size_t off = (packed.size() + 255) & ~size_t(255);
    packed.resize(off + n);
    std::memcpy(packed.data() + off, p, n);
    return off;
  };
  for (;;) {
    // next command of every slot, grouped by kind (kinds in enum order); a
    // slot whose next command is a validation contributes its whole run of
    // consecutive validations (independent by contract)
    bool any = false;
    std::vector<std::vector<int>> by_op(kNumOps);
    std::vector<int> vals;  // (slot, command index) pairs of this layer's validations
    for (int k = 0; k < K; ++k)
      if (head[k] < slots[k].pending.size()) {
        const Op op = slots[k].pending[head[k]].op;
        if (op == Op::Validate) {
          size_t h = head[k];
          while (h < slots[k].pending.size() && slots[k].pending[h].op == Op::Validate) {
            vals.push_back(k);
            vals.push_back((int)h);
            ++h;
          }
          head[k] = h - 1;  // advanced past the run below
          by_op[(int)op].push_back(k);
        } else {
          by_op[(int)op].push_back(k);
        }
        any = true;
      }
    if (!any) break;
    for (int o = 0; o < kNumOps; ++o) {
      const std::vector<int> &ks = by_op[o];
      for (size_t c0 = 0; c0 < ks.size(); c0 += kMaxPerLaunch) {
        const size_t c1 = std::min(ks.size(), c0 + (size_t)kMaxPerLaunch);
        const Op op = (Op)o;
        if (op == Op::Validate) {
          if (c0 > 0) break;  // all of the layer's validations go into one launch below
          std::vector<const ValidateReq *> reqs;
          for (size_t i = 0; i < vals.size(); i += 2) {
            const ValidateReq &v = slots[vals[i]].pending[vals[i + 1]].val;
            if (v.n > 0) reqs.push_back(&v);
          }
          std::vector<ValSeg> segs;
          int64_t flat = 0;
          int r_max = 1;
          for (const ValidateReq *v : reqs) {
            r_max = std::max(r_max, (int)v->scene->n_robots);
            flat += v->n;
          }
          if (reqs.empty()) continue;
          if ((int64_t)reqs.size() > kMaxPerLaunch) return hipErrorInvalidValue;
          int W = 0, cache = 0;
          seg_shape(r_max, flat, &W, &cache);
          flat = 0;
          for (const ValidateReq *vp : reqs) {
            const ValidateReq &v = *vp;
            ValSeg g;
            std::memset(&g, 0, sizeof(g));
            g.sc = *v.scene;
            g.qa = v.qa;
            g.qb = v.qb;
            g.edge0 = flat;
            g.n_edges = v.n;
            g.tile0 = 0;
            g.res = v.res;
            g.S = seg_link_split(v.scene->n_robots, W);
            g.out = v.out;
            g.counters = v.counters;
            flat += v.n;
            segs.push_back(g);
          }
          const size_t off = put(segs.data(), sizeof(ValSeg) * segs.size());
          plan.push_back({op, off, (int)segs.size(), (int)std::min<int64_t>(flat, 0x7fffffff), r_max});
          if (flat > 0x7fffffff) return hipErrorInvalidValue;
        } else {
          const size_t rec = op_args_bytes(op);
          const size_t off = (packed.size() + 255) & ~size_t(255);
          packed.resize(off + rec * (c1 - c0));
          int gx = 0;
          for (size_t i = c0; i < c1; ++i) {
            const Cmd &c = slots[ks[i]].pending[head[ks[i]]];
            std::memcpy(packed.data() + off + rec * (i - c0), c.args(), rec);
            gx = std::max(gx, op_blocks(op, c.args()));
          }
          if (gx > 0) plan.push_back({op, off, (int)(c1 - c0), gx, 0});
        }
      }
      for (int k : ks) ++head[k];
    }
  }
  if (plan.empty()) return hipSuccess;
  hipError_t e;
  if ((e = h_args.ensure(packed.size())) != hipSuccess) return e;
  if ((e = d_args.ensure(packed.size())) != hipSuccess) return e;
  std::memcpy(h_args.p, packed.data(), packed.size());
  int64_t flat_max = 0;
  for (const Launch &L : plan)
    if (L.op == Op::Validate) flat_max = std::max<int64_t>(flat_max, L.grid_x);
  if (flat_max > 0 && (e = seg_scratch.ensure(seg_scratch_bytes(flat_max))) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_args.p, h_args.p, packed.size(), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  for (const Launch &L : plan) {
    unsigned char *rec = (unsigned char *)d_args.p + L.off;
    if (L.op == Op::Validate) {
      const SegScratch ws = seg_scratch_layout(seg_scratch.p, L.grid_x);
      e = launch_validate_segments((ValSeg *)rec, L.count, L.r_max, L.grid_x, ws, s, profile_slot(ctx),
                                   ctx->profiling ? ctx->prof_totals : nullptr, &ctx->last_grid, &ctx->last_block);
    } else {
      e = launch_op_batch(L.op, rec, L.count, L.grid_x, s);
    }
    if (e != hipSuccess) return e;
    ++launches;
  }
  ++flushes;
  return hipStreamSynchronize(s);
}

JobEngine::JobEngine(mrpop_ctx *ctx, hipStream_t s, int capacity) : impl_(new Impl(ctx, s, std::max(1, capacity))) {}

JobEngine::~JobEngine() { delete impl_; }  // (the slots' coroutine frames go with them)

int JobEngine::start(PlanJob *job, std::function<void(int, mrpop_status)> on_done) {
  Impl &I = *impl_;
  int k = -1;
  for (int i = 0; i < (int)I.slots.size(); ++i)
    if (!I.slots[i].used) {
      k = i;
      break;
    }
  if (k < 0) return -1;
  Impl::Slot &sl = I.slots[k];
  sl.used = true;
  sl.running = true;
  sl.finished = false;
  sl.parked = false;
  sl.pending.clear();
  sl.job = job;
  sl.on_done = std::move(on_done);
  sl.ex.reset(new QueuedExec(&I, k));
  sl.task = job->run(*sl.ex);
  sl.resume_at = sl.task.handle();  // first resume starts it
  ++I.n_running;
  return k;
}

bool JobEngine::step(const std::function<bool()> &wake) {
  Impl &I = *impl_;
  // every running job that is not parked runs until it parks or ends
  for (int k = 0; k < (int)I.slots.size(); ++k) {
    Impl::Slot &sl = I.slots[k];
    if (!sl.running || sl.parked) continue;
    const std::coroutine_handle<> h = sl.resume_at;
    sl.resume_at = nullptr;
    h.resume();
    if (sl.task.done()) {
      sl.running = false;
      sl.finished = true;
      sl.pending.clear();
      --I.n_running;
      ++I.n_finished;
      if (sl.on_done) sl.on_done(k, sl.task.result());
    }
  }
  if (I.n_finished > 0) return false;  // jobs to reap first
  if (I.n_running == 0) {              // nothing runs: wait for wake()
    std::unique_lock<std::mutex> lk(I.mu);
    I.cv_main.wait(lk, [&] { return wake(); });
    return false;
  }
  // every running job is parked on its device work: merge and launch it
  const hipError_t e = I.flush();
  I.last_err = e;
  for (auto &sl : I.slots) {
    sl.pending.clear();
    sl.parked = false;
  }
  return true;
}

void JobEngine::notify() {
  std::lock_guard<std::mutex> lk(impl_->mu);
  impl_->cv_main.notify_all();
}

std::vector<int> JobEngine::reap() {
  Impl &I = *impl_;
  std::vector<int> done;
  for (int k = 0; k < (int)I.slots.size(); ++k)
    if (I.slots[k].used && I.slots[k].finished) {
      Impl::Slot &sl = I.slots[k];
      sl.task = Task<mrpop_status>();
      sl.ex.reset();
      sl.used = false;
      sl.finished = false;
      sl.job = nullptr;
      --I.n_finished;
      done.push_back(k);
    }
  return done;
}

int JobEngine::running() const { return impl_->n_running; }
int JobEngine::capacity() const { return (int)impl_->slots.size(); }
int JobEngine::free_slots() const {
  int n = 0;
  for (const auto &sl : impl_->slots) n += sl.used ? 0 : 1;
  return n;
}
int64_t JobEngine::flushes() const { return impl_->flushes; }
int64_t JobEngine::launches() const { return impl_->launches; }

}  // namespace mrpop

using namespace mrpop;

extern "C" {

mrpop_status mrpop_plan_batch(mrpop_ctx *ctx, mrpop_plan_request *reqs, int32_t n, mrpop_batch_stats *stats_opt) {
  if (!ctx) return fail(nullptr, MRPOP_E_INVALID_ARG, "plan_batch: ctx is NULL");
  if (n < 0 || (n > 0 && !reqs)) return fail(ctx, MRPOP_E_INVALID_ARG, "plan_batch: bad request array");
  const double t0 = now_s();
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MRPOP_E_DEVICE, "plan_batch: hipSetDevice");
  std::vector<std::unique_ptr<PlanJob>> jobs(n);
  std::vector<PlanJob *> run_jobs(n, nullptr);
  for (int i = 0; i < n; ++i) {
    mrpop_plan_request &q = reqs[i];
    q.status = MRPOP_OK;
    q.path_len = 0;
    q.cost = INFINITY;
    std::memset(&q.stats, 0, sizeof(q.stats));
    if (!q.scene || q.scene->ctx != ctx || !q.q_start || !q.q_goal || (q.path_cap > 0 && !q.path_out)) {
      q.status = MRPOP_E_INVALID_ARG;
      continue;
    }
    jobs[i].reset(new PlanJob());
    q.status = jobs[i]->prepare(ctx, q.scene, q.q_start, q.q_goal, q.params);
    if (q.status == MRPOP_OK) run_jobs[i] = jobs[i].get();
  }
  std::vector<mrpop_status> st(n, MRPOP_OK);
  JobEngine eng(ctx, nullptr, std::max(1, n));
  for (int i = 0; i < n; ++i)
    if (run_jobs[i]) eng.start(run_jobs[i], [&st, i](int, mrpop_status s) { st[i] = s; });
  for (;;) {
    eng.reap();
    if (eng.running() == 0) break;
    eng.step([] { return false; });
  }
  int solved = 0;
  for (int i = 0; i < n; ++i) {
    if (!run_jobs[i]) continue;
    mrpop_plan_request &q = reqs[i];
    PlanJob &j = *jobs[i];
    q.stats = j.stats();
    q.status = st[i];
    if (st[i] != MRPOP_OK) continue;
    const int len = (int)(j.path().size() / j.dof());
    q.path_len = len;
    q.cost = j.cost();
    ++solved;
    if (len > q.path_cap) {
      q.status = MRPOP_E_BUFFER;
      continue;
    }
    std::memcpy(q.path_out, j.path().data(), sizeof(float) * j.path().size());
  }
  if (stats_opt) {
    stats_opt->wall_s = now_s() - t0;
    stats_opt->instances = n;
    stats_opt->solved = solved;
    stats_opt->flushes = eng.flushes();
    stats_opt->launches = eng.launches();
  }
  return MRPOP_OK;
}

}  // extern "C"
