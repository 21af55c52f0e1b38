// Planning instances sharing merged launches (see batch.cpp).
#pragma once

#include <functional>
#include <vector>

#include "plan_job.h"

namespace mrpop {

// Runs PlanJobs as coroutines on the calling thread, with their device work
// merged: whenever every running job is parked on its queued work, the queued
// work of all of them is launched together on one stream, then they resume.
// Jobs can start while others run (continuous batching): a started job's
// work joins the next merge.  start, step, reap and the queries are called
// from one thread; notify may be called from any.
class JobEngine {
 public:
  JobEngine(mrpop_ctx *ctx, hipStream_t s, int capacity);
  ~JobEngine();
  JobEngine(const JobEngine &) = delete;
  JobEngine &operator=(const JobEngine &) = delete;

  // Starts `job` (prepared on this context) in a free slot; returns the slot,
  // or -1 when every slot is taken.  The job first runs at the next step();
  // on_done(slot, status) runs on the engine's thread once it has returned.
  int start(PlanJob *job, std::function<void(int, mrpop_status)> on_done);
  // Runs every job that is not parked until it parks or ends.  Then, if a
  // job has ended and awaits reap(), returns false; if nothing runs, waits
  // for wake() (checked whenever notify() is called) and returns false;
  // otherwise merges and launches the parked jobs' work, waits for it,
  // unparks them and returns true.
  bool step(const std::function<bool()> &wake);
  // Wakes a step() waiting with no running job (after changing what wake() reads).
  void notify();
  // Releases jobs that have ended; returns their slots.
  std::vector<int> reap();
  int running() const;
  int capacity() const;
  int free_slots() const;  // slots neither running nor holding an unreaped job
  int64_t flushes() const;   // merged submissions so far
  int64_t launches() const;  // kernel launches they made
  struct Impl;

 private:
  Impl *impl_;
};

}  // namespace mrpop
