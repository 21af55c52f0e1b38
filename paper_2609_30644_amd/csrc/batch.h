// Many planning instances sharing merged launches (see batch.cpp).
#pragma once

#include <vector>

#include "plan_job.h"

namespace mrpop {

class BatchEngine {
 public:
  BatchEngine(mrpop_ctx *ctx, hipStream_t s);
  ~BatchEngine();
  BatchEngine(const BatchEngine &) = delete;
  BatchEngine &operator=(const BatchEngine &) = delete;
  // Runs every non-null job (each prepared on this context) to completion;
  // status[k] is job k's result.
  void run(std::vector<PlanJob *> &jobs, std::vector<mrpop_status> &status);
  int64_t flushes() const;   // merged submissions so far
  int64_t launches() const;  // kernel launches they made
  struct Impl;

 private:
  Impl *impl_;
};

}  // namespace mrpop
