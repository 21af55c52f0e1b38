// Planning instances sharing merged launches (see batch.cpp).
#pragma once

#include <functional>
#include <mutex>
#include <vector>

#include "plan_job.h"

namespace mrpop {

// Runs PlanJobs on host threads of their own, with their device work merged:
// whenever every running job waits for its queued work, the queued work of
// all of them is launched together on one stream.  Jobs can start while
// others run (continuous batching): a started job's work joins the next merge.
class JobEngine {
 public:
  JobEngine(mrpop_ctx *ctx, hipStream_t s, int capacity);
  ~JobEngine();
  JobEngine(const JobEngine &) = delete;
  JobEngine &operator=(const JobEngine &) = delete;

  // Starts `job` (prepared on this context) in a free slot; returns the slot,
  // or -1 when every slot is taken.  on_done(slot, status) runs on the job's
  // thread, under the engine's lock, once the job has returned.
  int start(PlanJob *job, std::function<void(int, mrpop_status)> on_done);
  // Blocks until every running job waits for its device work.  Then, if a
  // job has ended and awaits reap(), or nothing runs, returns false at once
  // (with nothing running it first waits for an ended job or for wake(),
  // checked under the engine's lock); otherwise merges and launches the
  // waiting work, lets the jobs continue and returns true.  Call from one
  // thread only.
  bool step(const std::function<bool()> &wake);
  // Wakes a step() waiting with no running job (after changing what wake() reads).
  void notify();
  // Joins the threads of jobs that have finished; returns their slots.
  std::vector<int> reap();
  int running() const;
  int capacity() const;
  int free_slots() const;  // slots neither running nor holding an unreaped job
  int64_t flushes() const;   // merged submissions so far
  int64_t launches() const;  // kernel launches they made
  // The engine's lock, for state shared with on_done callbacks.
  std::mutex &mutex();
  struct Impl;

 private:
  Impl *impl_;
};

}  // namespace mrpop
